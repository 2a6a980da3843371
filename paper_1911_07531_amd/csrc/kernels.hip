// Device kernels of the H-LU library (gfx950).
//
// Every task of the traced DAG runs in one 256-thread workgroup:
//   GETRF    dense LU of a diagonal leaf with leaf-local partial pivoting
//            (Algorithm 2, non-recursive branch)
//   TRSM_*   triangular solves of a panel with a diagonal leaf
//            (Algorithm 3, non-recursive branch, and its mirror)
//   GEMM     dense products of leaves and panels (Algorithm 1 leaf cases)
//   LRGEMM   product with a low-rank leaf, y += alpha U (V^T x)
//   TRUNC    truncated low-rank addition C <- T_eps(C + alpha A B) (Sec. 2.3)
// plus the executors that replay the DAG (one launch per level, or one
// persistent dataflow launch), the assembly kernels and the H-matvec.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hm_internal.h"

namespace hm {

// ---------------------------------------------------------------------------
// views
// ---------------------------------------------------------------------------
struct RV {  // a view with its run-time extents resolved
  int64_t off;
  int rows, cols, rs, cs, type;
};

__device__ __forceinline__ RV resolve(const ExecArgs& a, const View& v) {
  RV r;
  r.off = v.off;
  r.rows = (v.dyn & DYN_ROWS) ? a.ranks[v.rank_id] : v.rows;
  r.cols = (v.dyn & DYN_COLS2) ? a.ranks[v.rank_id2] : (v.dyn & DYN_COLS) ? a.ranks[v.rank_id] : v.cols;
  r.rs = v.rs;
  r.cs = v.cs;
  r.type = v.type;
  return r;
}

__device__ __forceinline__ double vld(const ExecArgs& a, const RV& v, int i, int j) {
  if (v.type == VT_F64) return a.f64[v.off + (int64_t)i * v.rs + (int64_t)j * v.cs];
  if (v.type == VT_F32) return (double)a.f32[v.off + (int64_t)i * v.rs + (int64_t)j * v.cs];
  if (v.type == VT_IDENT) return i == j ? 1.0 : 0.0;
  return 0.0;
}

__device__ __forceinline__ void vst(const ExecArgs& a, const RV& v, int i, int j, double x) {
  if (v.type == VT_F64)
    a.f64[v.off + (int64_t)i * v.rs + (int64_t)j * v.cs] = x;
  else if (v.type == VT_F32)
    a.f32[v.off + (int64_t)i * v.rs + (int64_t)j * v.cs] = (float)x;
}

__device__ __forceinline__ int64_t vbytes(const RV& v) {
  if (v.type == VT_F64) return (int64_t)v.rows * v.cols * 8;
  if (v.type == VT_F32) return (int64_t)v.rows * v.cols * 4;
  return 0;
}

// ---------------------------------------------------------------------------
// Matrix-core (MFMA) steps: one wavefront multiplies a 16 x 4 by a 4 x 16
// block into a 16 x 16 accumulator.  Operand lanes: lane l supplies
// A(l mod 16, l / 16) and B(l / 16, l mod 16).  Entry r of the accumulator in
// lane l is column l mod 16 and row row(l / 16, r): rows 4 (l / 16) + r for
// the FP32 MFMA, rows 4 r + l / 16 for the FP64 MFMA (both measured with an
// in-bounds probe on gfx950).  FP64 operands use the FP64 MFMA; FP32
// operands the FP32 MFMA with FP32 accumulation.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename CT>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = v4d;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * r + lk; }
};
template <>
struct Mfma<float> {
  using acc_t = v4f;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// C = A B for operands staged in LDS (A m x k column-major with leading
// dimension lda, B k x n column-major with leading dimension ldb, both
// double), on the matrix cores: each wavefront takes 16 x 16 output tiles in
// turn and sweeps k in steps of 4; st(i, j, value) receives every entry of C.
template <typename CT, class ST>
__device__ void mfma_lds_gemm(int m, int n, int k, const double* lA, int lda, const double* lB, int ldb, ST st) {
  using M = Mfma<CT>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
  for (int tile = wave; tile < tm * tn; tile += nw) {
    const int i0 = (tile % tm) << 4, j0 = (tile / tm) << 4;
    const int ia = i0 + li, jb = j0 + li;
    typename M::acc_t acc = M::zero();
    for (int k0 = 0; k0 < k; k0 += 4) {
      const int kk = k0 + lk;
      const CT av = (ia < m && kk < k) ? (CT)lA[(int64_t)kk * lda + ia] : CT(0);
      const CT bv = (jb < n && kk < k) ? (CT)lB[(int64_t)jb * ldb + kk] : CT(0);
      acc = M::step(av, bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + M::row(lk, r);
      if (i < m && jb < n) st(i, jb, (double)acc[r]);
    }
  }
}

// ---------------------------------------------------------------------------
// tiled GEMM core: C(m x n) = sum_k A(i, k) B(k, j), 64x64 output tiles,
// 16-deep k slices staged in LDS, 4x4 outputs per thread.
// a_kcontig / b_kcontig choose which tile index consecutive threads walk so
// that global loads are coalesced for the operand's storage order.  (Scalar
// FMA: these serve the products too large to stage whole, and an MFMA
// version's accumulators pushed the persistent executors past the register
// budget of two workgroups per compute unit.)
// ---------------------------------------------------------------------------
constexpr int TM = 64, TN = 64, TK = 16, TP = 4;

template <typename CT, class LA, class LB, class ST>
__device__ void gemm_tiles(int m, int n, int k, LA la, LB lb, ST st, bool a_kcontig, bool b_kcontig, CT* sA,
                           CT* sB) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  for (int i0 = 0; i0 < m; i0 += TM)
    for (int j0 = 0; j0 < n; j0 += TN) {
      CT acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = CT(0);
      for (int k0 = 0; k0 < k; k0 += TK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int l = tid + 256 * q;
          int ii, kk;
          if (a_kcontig) {
            kk = l & 15;
            ii = l >> 4;
          } else {
            ii = l & 63;
            kk = l >> 6;
          }
          int gi = i0 + ii, gk = k0 + kk;
          sA[kk * (TM + TP) + ii] = (gi < m && gk < k) ? (CT)la(gi, gk) : CT(0);
          int jj;
          if (b_kcontig) {
            kk = l & 15;
            jj = l >> 4;
          } else {
            jj = l & 63;
            kk = l >> 6;
          }
          int gj = j0 + jj;
          gk = k0 + kk;
          sB[kk * (TN + TP) + jj] = (gj < n && gk < k) ? (CT)lb(gk, gj) : CT(0);
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < TK; ++kk) {
          CT av[4], bv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) av[r] = sA[kk * (TM + TP) + tx * 4 + r];
#pragma unroll
          for (int c = 0; c < 4; ++c) bv[c] = sB[kk * (TN + TP) + ty * 4 + c];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += av[r] * bv[c];
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          int gi = i0 + tx * 4 + r, gj = j0 + ty * 4 + c;
          if (gi < m && gj < n) st(gi, gj, (double)acc[r][c]);
        }
      __syncthreads();
    }
}

constexpr int kTileBytes = 2 * TK * (TM + TP) * 8;  // both tiles in double

// ---------------------------------------------------------------------------
// block copies with several loads in flight per thread (a plain strided loop
// waits for every load before its store)
// ---------------------------------------------------------------------------
template <class Dst>
__device__ __forceinline__ void copy_batched(Dst dst, const double* src, int n) {
  for (int base = 0; base < n; base += 8 * kThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      v[u] = e < n ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      if (e < n) dst(e, v[u]);
    }
  }
}
__device__ __forceinline__ void copy_batched(double* dst, const double* src, int n) {
  copy_batched([&](int e, double x) { dst[e] = x; }, src, n);
}

// ---------------------------------------------------------------------------
// Jacobi rotation: for the column pair with squared norms al, be and inner
// product ga (ga != 0), cs and sn of the rotation that makes the pair
// orthogonal (Hestenes; t the smaller root of t^2 + 2 zeta t - 1 = 0).  The
// square roots come from the hardware reciprocal square root with two Newton
// steps (relative error near the rounding level).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double& cs, double& sn) {
  const double zeta = (be - al) / (2.0 * ga);
  const double h = 1.0 + zeta * zeta;
  const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + h * rsqrt_nr(h));
  cs = rsqrt_nr(1.0 + tt * tt);
  sn = cs * tt;
}

// ---------------------------------------------------------------------------
// cross-lane reductions
// ---------------------------------------------------------------------------
// A double moved between lanes by a DPP pattern (both 32-bit halves).
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of g lanes (g a power of two <= 64); every lane of
// a group gets the group's total.  Within a row of 16 lanes the partners come
// from DPP mirror and quad patterns (each step joins two disjoint lane sets),
// across rows from a shuffle.
__device__ __forceinline__ double group_sum(double x, int g) {
  if (g >= 64) x += __shfl_xor(x, 32);
  if (g >= 32) x += __shfl_xor(x, 16);
  if (g >= 16) x += dpp_f64<0x140>(x);  // row_mirror: i <-> 15 - i
  if (g >= 8) x += dpp_f64<0x141>(x);   // row_half_mirror: i <-> 7 - i
  if (g >= 4) x += dpp_f64<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  if (g >= 2) x += dpp_f64<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  return x;
}

// Largest value (smallest index among ties) over the whole wavefront; every
// lane gets the winner.
template <int kCtrl>
__device__ __forceinline__ void argmax_step(double& v, int& i) {
  const double ov = dpp_f64<kCtrl>(v);
  const int oi = __builtin_amdgcn_update_dpp(0, i, kCtrl, 0xF, 0xF, false);
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int off = 32; off >= 16; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(i, off);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  argmax_step<0x140>(v, i);
  argmax_step<0x141>(v, i);
  argmax_step<0x4E>(v, i);
  argmax_step<0xB1>(v, i);
}

// ---------------------------------------------------------------------------
// simple element-wise ops
// ---------------------------------------------------------------------------
__device__ void op_zero(const ExecArgs& a, const Task& t) {
  RV y = resolve(a, t.y);
  int total = y.rows * y.cols;
  for (int e = threadIdx.x; e < total; e += blockDim.x) vst(a, y, e % y.rows, e / y.rows, 0.0);
}

__device__ void op_copy(const ExecArgs& a, const Task& t) {
  RV y = resolve(a, t.y), x = resolve(a, t.a);
  int total = y.rows * y.cols;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int i = e % y.rows, j = e / y.rows;
    vst(a, y, i, j, vld(a, x, i, j));
  }
}

// ---------------------------------------------------------------------------
// small operands: every operand of a task staged into LDS in one batched
// load phase (up to 16 loads per thread in flight), so that the task pays one
// global round trip before its arithmetic instead of one per k slice
// ---------------------------------------------------------------------------
struct StageSrc {
  RV v;
  double* dst;           // column-major, leading dimension = v.rows
  const int32_t* rows;   // optional row gather: element (i, j) <- v(rows[i], j)
};

__device__ __forceinline__ double stage_ld(const ExecArgs& a, const StageSrc& s, int e) {
  const int r = s.v.rows, i = e % r, j = e / r;
  return vld(a, s.v, s.rows ? s.rows[i] : i, j);
}

// Up to four sources (unused ones with zero rows); element e of the joint
// index space belongs to the first source whose prefix holds it.
__device__ __forceinline__ void stage_views(const ExecArgs& a, const StageSrc& s0, const StageSrc& s1,
                                            const StageSrc& s2, const StageSrc& s3) {
  const int c0 = s0.v.rows * s0.v.cols, c1 = c0 + s1.v.rows * s1.v.cols, c2 = c1 + s2.v.rows * s2.v.cols,
            total = c2 + s3.v.rows * s3.v.cols;
  for (int base = 0; base < total; base += 16 * kThreads) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      v[u] = 0.0;
      if (e < c0)
        v[u] = stage_ld(a, s0, e);
      else if (e < c1)
        v[u] = stage_ld(a, s1, e - c0);
      else if (e < c2)
        v[u] = stage_ld(a, s2, e - c1);
      else if (e < total)
        v[u] = stage_ld(a, s3, e - c2);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      if (e < c0)
        s0.dst[e] = v[u];
      else if (e < c1)
        s1.dst[e - c0] = v[u];
      else if (e < c2)
        s2.dst[e - c1] = v[u];
      else if (e < total)
        s3.dst[e - c2] = v[u];
    }
  }
}

constexpr int kLdsDoubles = kLdsBytes / 8;

// Debug timeline: ticks of a task's phases, added to the running task's six
// phase slots (thread 0, only while a timeline is recorded).
struct PhaseClock {
  unsigned long long* s;
  uint64_t t;
  __device__ PhaseClock(const ExecArgs& a, char* lds)
      : s(a.trace && threadIdx.x == 0 ? (unsigned long long*)(lds + kLdsBytes) + kCtrSize : nullptr),
        t(s ? wall_clock64() : 0) {}
  __device__ __forceinline__ void mark(int k) {
    if (s) {
      const uint64_t n = wall_clock64();
      s[k] += n - t;
      t = n;
    }
  }
};

// y <- beta y + alpha a b
template <typename CT>
__device__ void op_gemm_ct(const ExecArgs& a, const Task& t, char* lds) {
  RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b);
  int m = y.rows, n = y.cols, k = A.cols;
  if (m == 0 || n == 0) return;
  const double alpha = t.alpha, beta = t.beta;
  if (k == 0) {
    for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
      int i = e % m, j = e / m;
      vst(a, y, i, j, beta == 0.0 ? 0.0 : beta * vld(a, y, i, j));
    }
    return;
  }
  if ((int64_t)m * k + (int64_t)k * n + (int64_t)m * n <= kLdsDoubles) {
    double* lA = (double*)lds;
    double* lB = lA + m * k;
    double* lY = lB + k * n;
    const StageSrc none{RV{0, 0, 0, 1, 1, VT_NONE}, nullptr, nullptr};
    stage_views(a, {A, lA, nullptr}, {B, lB, nullptr}, beta != 0.0 ? StageSrc{y, lY, nullptr} : none, none);
    __syncthreads();
    mfma_lds_gemm<CT>(m, n, k, lA, m, lB, k, [&](int i, int j, double v) {
      vst(a, y, i, j, (beta == 0.0 ? 0.0 : beta * lY[i + j * m]) + alpha * v);
    });
    __syncthreads();
    return;
  }
  CT* sA = (CT*)lds;
  CT* sB = sA + TK * (TM + TP);
  gemm_tiles<CT>(
      m, n, k, [&](int i, int kk) { return vld(a, A, i, kk); }, [&](int kk, int j) { return vld(a, B, kk, j); },
      [&](int i, int j, double v) {
        double o = beta == 0.0 ? 0.0 : beta * vld(a, y, i, j);
        vst(a, y, i, j, o + alpha * v);
      },
      A.rs != 1, B.rs == 1, sA, sB);
}

// y <- beta y + alpha a (b x); a: m x k, b: k x n2, x: n2 x c, k <= 64
template <typename CT>
__device__ void op_lrgemm_ct(const ExecArgs& a, const Task& t, char* lds) {
  RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b), X = resolve(a, t.x);
  int m = y.rows, c = y.cols, k = A.cols, n2 = B.cols;
  if (m == 0 || c == 0) return;
  const double alpha = t.alpha, beta = t.beta;
  if (k == 0 || n2 == 0) {
    for (int e = threadIdx.x; e < m * c; e += blockDim.x) {
      int i = e % m, j = e / m;
      vst(a, y, i, j, beta == 0.0 ? 0.0 : beta * vld(a, y, i, j));
    }
    return;
  }
  if ((int64_t)m * k + (int64_t)k * n2 + (int64_t)n2 * c + (int64_t)m * c + (int64_t)k * c <= kLdsDoubles) {
    double* lA = (double*)lds;
    double* lB = lA + m * k;
    double* lX = lB + k * n2;
    double* lY = lX + n2 * c;
    double* lT = lY + m * c;
    const StageSrc none{RV{0, 0, 0, 1, 1, VT_NONE}, nullptr, nullptr};
    PhaseClock pc(a, lds);
    stage_views(a, {A, lA, nullptr}, {B, lB, nullptr}, {X, lX, nullptr},
                beta != 0.0 ? StageSrc{y, lY, nullptr} : none);
    __syncthreads();
    pc.mark(0);
    // T = b x (k x c), then y = beta y + alpha a T, both on the matrix cores
    mfma_lds_gemm<CT>(k, c, n2, lB, k, lX, n2, [&](int i, int j, double v) { lT[i + j * k] = v; });
    __syncthreads();
    pc.mark(1);
    mfma_lds_gemm<CT>(m, c, k, lA, m, lT, k, [&](int i, int j, double v) {
      vst(a, y, i, j, (beta == 0.0 ? 0.0 : beta * lY[i + j * m]) + alpha * v);
    });
    __syncthreads();
    pc.mark(2);
    return;
  }
  CT* sA = (CT*)lds;
  CT* sB = sA + TK * (TM + TP);
  CT* sT = (CT*)(lds + kTileBytes);  // k x 64 chunk of T = b x
  for (int j0 = 0; j0 < c; j0 += 64) {
    int cc = min(64, c - j0);
    gemm_tiles<CT>(
        k, cc, n2, [&](int i, int kk) { return vld(a, B, i, kk); },
        [&](int kk, int j) { return vld(a, X, kk, j0 + j); }, [&](int i, int j, double v) { sT[j * 64 + i] = (CT)v; },
        B.rs != 1, X.rs == 1, sA, sB);
    __syncthreads();
    gemm_tiles<CT>(
        m, cc, k, [&](int i, int kk) { return vld(a, A, i, kk); },
        [&](int kk, int j) { return (double)sT[j * 64 + kk]; },
        [&](int i, int j, double v) {
          double o = beta == 0.0 ? 0.0 : beta * vld(a, y, i, j0 + j);
          vst(a, y, i, j0 + j, o + alpha * v);
        },
        A.rs != 1, true, sA, sB);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Products of the forward / backward substitution (solve executors only).
// A solve applies each low-rank block as y += alpha U (V^T x) with c <= 64
// panel columns: a tall-skinny reduction over the block's columns followed by
// a row-wise update.  Both stream their operands through LDS in chunks, 32
// loads per thread in flight, and compute with 4 x 4 register tiles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stage_pair(const ExecArgs& a, const RV& v0, double* d0, const RV& v1, double* d1) {
  const int c0 = v0.rows * v0.cols, total = c0 + v1.rows * v1.cols;
  for (int base = 0; base < total; base += 32 * kThreads) {
    double v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      v[u] = 0.0;
      if (e < c0)
        v[u] = vld(a, v0, e % v0.rows, e / v0.rows);
      else if (e < total)
        v[u] = vld(a, v1, (e - c0) % v1.rows, (e - c0) / v1.rows);
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      if (e < c0)
        d0[e] = v[u];
      else if (e < total)
        d1[e - c0] = v[u];
    }
  }
}

// Result tiles of an m x n (<= 64 x 64) product: thread t owns rows
// 4*tx .. 4*tx+3 and columns 4*ty .. 4*ty+3 of tile t mod NT, and works on
// every G-th row of each staged chunk (G groups split the reduction).
struct SkinnyMap {
  int mt, nt, g, tx, ty, grp;
  __device__ SkinnyMap(int m, int n) {
    mt = (m + 3) >> 2;
    nt = mt * ((n + 3) >> 2);
    g = max(1, kThreads / nt);
    const int t = (int)threadIdx.x;
    grp = t / nt;
    tx = (t % nt) % mt;
    ty = (t % nt) / mt;
  }
  __device__ bool active() const { return grp < g; }
};

// acc = A B for A m x K, B K x n (m, n <= 64), K streamed through `work`
// (nwork doubles).  A chunk is staged transposed (rows of B's reduction
// index contiguous), so that A = V^T and B = x read columns of V and x.
// Threads of group grp > 0 leave partial sums; reduce_groups adds them.
__device__ void skinny_ab(const ExecArgs& a, const RV& A, const RV& B, double* work, int nwork, const SkinnyMap& mp,
                          double (&acc)[4][4]) {
  const int m = A.rows, n = B.cols, K = A.cols;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  int kc = min(K, nwork / (m + n));
  if (kc > 1 && !(kc & 1)) --kc;  // odd: the staged columns start in different LDS banks
  double* lA = work;
  const int i0 = min(4 * mp.tx, m - 1), j0 = min(4 * mp.ty, n - 1);
  for (int k0 = 0; k0 < K; k0 += kc) {
    const int kk = min(kc, K - k0);
    double* lB = lA + kk * m;
    const RV At{A.off + (int64_t)k0 * A.cs, kk, m, A.cs, A.rs, A.type};
    const RV Bc{B.off + (int64_t)k0 * B.rs, kk, n, B.rs, B.cs, B.type};
    __syncthreads();
    stage_pair(a, At, lA, Bc, lB);
    __syncthreads();
    if (mp.active()) {
      const double* pa[4];
      const double* pb[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) pa[r] = lA + min(i0 + r, m - 1) * kk;
#pragma unroll
      for (int c = 0; c < 4; ++c) pb[c] = lB + min(j0 + c, n - 1) * kk;
      for (int l = mp.grp; l < kk; l += mp.g) {
        double av[4], bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) av[r] = pa[r][l];
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = pb[c][l];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] += av[r] * bv[c];
      }
    }
  }
  __syncthreads();
}

// Adds the groups' partial sums into group 0's registers (through `work`,
// which must hold g * 16 * nt doubles).
__device__ void reduce_groups(double* work, const SkinnyMap& mp, double (&acc)[4][4]) {
  if (mp.g == 1) return;
  const int slot = (int)threadIdx.x % mp.nt;
  if (mp.active() && mp.grp > 0)
#pragma unroll
    for (int e = 0; e < 16; ++e) work[((mp.grp - 1) * mp.nt + slot) * 16 + e] = acc[e >> 2][e & 3];
  __syncthreads();
  if (mp.grp == 0)
    for (int q = 1; q < mp.g; ++q)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e >> 2][e & 3] += work[((q - 1) * mp.nt + slot) * 16 + e];
  __syncthreads();
}

// y (m x c) <- beta y + alpha U T: U m x k from the arenas, T k x c in LDS
// (column-major, leading dimension k); rows streamed through `work`.
// Thread t owns rows rg, rg + RG, rg + 2 RG, rg + 3 RG of a chunk of 4 RG rows
// (consecutive threads on consecutive rows) and columns 4 cg .. 4 cg + 3.
__device__ void rows_update(const ExecArgs& a, const RV& y, const RV& U, const double* lT, double alpha, double beta,
                            double* work, int nwork) {
  const int m = y.rows, c = y.cols, k = U.cols;
  const int cg_n = (c + 3) >> 2;
  int rg_n = kThreads / cg_n;
  rg_n = min(rg_n, max(1, (nwork / (k + c)) >> 2));
  const int R = 4 * rg_n;
  const int t = (int)threadIdx.x, rg = t % rg_n, cg = t / rg_n;
  const bool act = cg < cg_n;
  const int j0 = 4 * cg;
  const RV none{0, 0, 0, 1, 1, VT_NONE};
  for (int r0 = 0; r0 < m; r0 += R) {
    const int rr = min(R, m - r0);
    double* lU = work;
    double* lY = work + rr * k;
    const RV Ur{U.off + (int64_t)r0 * U.rs, rr, k, U.rs, U.cs, U.type};
    const RV Yr{y.off + (int64_t)r0 * y.rs, rr, c, y.rs, y.cs, y.type};
    __syncthreads();
    stage_pair(a, Ur, lU, beta != 0.0 ? Yr : none, lY);
    __syncthreads();
    if (act) {
      double acc[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) acc[q][cc] = 0.0;
      int ri[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) ri[q] = min(rg + q * rg_n, rr - 1);
      const double* pt[4];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) pt[cc] = lT + min(j0 + cc, c - 1) * k;
      for (int l = 0; l < k; ++l) {
        double uv[4], tv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) uv[q] = lU[ri[q] + l * rr];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) tv[cc] = pt[cc][l];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) acc[q][cc] += uv[q] * tv[cc];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = rg + q * rg_n;
        if (i >= rr) continue;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int j = j0 + cc;
          if (j < c) vst(a, Yr, i, j, (beta == 0.0 ? 0.0 : beta * lY[i + j * rr]) + alpha * acc[q][cc]);
        }
      }
    }
  }
  __syncthreads();
}

// OP_GEMM in a solve when the result is at most 64 x 64 and the reduction is
// long (the partial products V_p^T x_p of a split low-rank block).
__device__ void op_gemm_skinny(const ExecArgs& a, const Task& t, char* lds) {
  const RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b);
  const int m = y.rows, n = y.cols;
  if (m == 0 || n == 0) return;
  PhaseClock pc(a, lds);
  double* work = (double*)lds;
  const SkinnyMap mp(m, n);
  double acc[4][4];
  skinny_ab(a, A, B, work, kLdsDoubles, mp, acc);
  pc.mark(0);
  reduce_groups(work, mp, acc);
  pc.mark(1);
  if (mp.grp == 0)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = 4 * mp.tx + r, j = 4 * mp.ty + c;
        if (i < m && j < n) vst(a, y, i, j, (t.beta == 0.0 ? 0.0 : t.beta * vld(a, y, i, j)) + t.alpha * acc[r][c]);
      }
  __syncthreads();
  pc.mark(2);
}

// T (k x c, LDS) from registers of group 0
__device__ __forceinline__ void acc_to_lds(double* lT, int m, int n, const SkinnyMap& mp, const double (&acc)[4][4]) {
  if (mp.grp == 0)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = 4 * mp.tx + r, j = 4 * mp.ty + c;
        if (i < m && j < n) lT[i + j * m] = acc[r][c];
      }
  __syncthreads();
}

// OP_LRGEMM in a solve, when its operands do not fit LDS at once:
// T = b x by the streamed reduction, then y <- beta y + alpha a T by rows.
__device__ void op_lrgemm_solve(const ExecArgs& a, const Task& t, char* lds) {
  const RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b), X = resolve(a, t.x);
  const int m = y.rows, c = y.cols, k = A.cols;
  if (m == 0 || c == 0) return;
  double* lT = (double*)lds + (kLdsDoubles - 64 * 64);
  double* work = (double*)lds;
  const int nwork = kLdsDoubles - 64 * 64;
  if (k == 0 || B.cols == 0) {
    for (int e = threadIdx.x; e < k * c; e += blockDim.x) lT[e] = 0.0;
  } else {
    const SkinnyMap mp(k, c);
    double acc[4][4];
    skinny_ab(a, B, X, work, nwork, mp, acc);
    reduce_groups(work, mp, acc);
    acc_to_lds(lT, k, c, mp, acc);
  }
  __syncthreads();
  rows_update(a, y, A, lT, t.alpha, t.beta, work, nwork);
}

// OP_GEMMP: y <- y + alpha a (b_0 + ... + b_{P-1}); b_p (k x c) at offset
// b.off + p * piv, summed in LDS in one batched pass, p in increasing order.
__device__ void op_gemmp(const ExecArgs& a, const Task& t, char* lds) {
  const RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b);
  const int m = y.rows, c = y.cols, k = A.cols, P = t.r0;
  if (k > 64 || c > 64) {
    if (threadIdx.x == 0) atomicOr(&a.status[0], ST_BADOP);
    return;
  }
  if (m == 0 || c == 0) return;
  double* lT = (double*)lds + (kLdsDoubles - 64 * 64);
  double* work = (double*)lds;
  const int nwork = kLdsDoubles - 64 * 64;
  const int kc = k * c;
  // each thread sums its elements over p with up to 32 loads in flight
  for (int e0 = 0; e0 < kc; e0 += kThreads) {
    const int e = e0 + (int)threadIdx.x;
    const int i = e < kc ? e % max(k, 1) : 0, j = e < kc ? e / max(k, 1) : 0;
    double s = 0.0;
    for (int p0 = 0; p0 < P; p0 += 32) {
      double v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        v[u] = 0.0;
        if (e < kc && p0 + u < P) {
          RV bp = B;
          bp.off += (int64_t)(p0 + u) * t.piv;
          v[u] = vld(a, bp, i, j);
        }
      }
#pragma unroll
      for (int u = 0; u < 32; ++u) s += v[u];
    }
    if (e < kc) lT[e] = s;
  }
  __syncthreads();
  rows_update(a, y, A, lT, t.alpha, t.beta, work, nwork);
}

__device__ __forceinline__ bool all_f32(const View& v) { return v.type != VT_F64; }

// a solve GEMM with a result of at most 64 x 64 and a long reduction
__device__ __forceinline__ bool solve_skinny_gemm(const ExecArgs& a, const Task& t) {
  const RV y = resolve(a, t.y), A = resolve(a, t.a);
  return y.rows <= 64 && y.cols <= 64 && A.cols > 64;
}

// op_lrgemm_ct serves the product: its small-operand path applies (every
// operand in LDS), or the rank or panel width exceeds 64
__device__ __forceinline__ bool lrgemm_fits_lds(const ExecArgs& a, const Task& t) {
  const RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b);
  const int64_t m = y.rows, c = y.cols, k = A.cols, n2 = B.cols;
  return m * k + k * n2 + n2 * c + m * c + k * c <= kLdsDoubles || k > 64 || c > 64;
}

// ---------------------------------------------------------------------------
// GETRF: dense LU with partial pivoting (LAPACK getrf convention: first
// maximum |a| wins, full-row interchanges, unit lower L)
// ---------------------------------------------------------------------------
__device__ void op_getrf(const ExecArgs& a, const Task& t, char* lds) {
#pragma clang fp contract(off)
  const int m = t.a.rows;
  double* g = a.f64 + t.a.off;
  const bool in_lds = (int64_t)m * (m + 1) * 8 + 64 + 4 * kMaxLeaf <= kLdsBytes;
  const int ld = in_lds ? m + 1 : m;
  double* A = in_lds ? (double*)lds : g;
  int* s_piv = (int*)(lds + kLdsBytes - 16);
  int* s_perm = (int*)(lds + kLdsBytes - 16 - 4 * kMaxLeaf);
  const int tid = threadIdx.x;
  if (in_lds)
    copy_batched([&](int e, double x) { A[(e / m) * ld + (e % m)] = x; }, g, m * m);
  for (int i = tid; i < m; i += blockDim.x) s_perm[i] = i;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (tid < 64) {
      double best = -1.0;
      int bi = m;
      for (int i = j + tid; i < m; i += 64) {
        double v = fabs(A[j * ld + i]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      wave_argmax(best, bi);
      if (bi >= m) bi = j;  // no comparable entry (NaN column): keep the row
      if (tid == 0) {
        s_piv[0] = bi;
        a.piv[t.piv + j] = bi;
      }
    }
    __syncthreads();
    const int p = s_piv[0];
    if (p != j) {
      for (int c = tid; c < m; c += blockDim.x) {
        double x = A[c * ld + j];
        A[c * ld + j] = A[c * ld + p];
        A[c * ld + p] = x;
      }
      if (tid == 0) {
        int x = s_perm[j];
        s_perm[j] = s_perm[p];
        s_perm[p] = x;
      }
    }
    __syncthreads();
    const double pv = A[j * ld + j];
    if (pv == 0.0) {
      if (tid == 0) {
        atomicOr(&a.status[0], ST_SINGULAR);
        atomicMin(&a.status[1], t.row0 + j);
      }
    } else {
      for (int i = j + 1 + tid; i < m; i += blockDim.x) A[j * ld + i] = A[j * ld + i] / pv;
    }
    __syncthreads();
    const int rem = m - j - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      int i = j + 1 + e % rem, c = j + 1 + e / rem;
      double prod = A[j * ld + i] * A[c * ld + j];
      A[c * ld + i] = A[c * ld + i] - prod;
    }
    __syncthreads();
  }
  if (in_lds)
    for (int e = tid; e < m * m; e += blockDim.x) g[e] = A[(e / m) * ld + (e % m)];
  // row permutation after all interchanges: (P x)[i] = x[perm[i]]
  for (int i = tid; i < m; i += blockDim.x) a.piv[t.piv + m + i] = s_perm[i];
}

// ---------------------------------------------------------------------------
// triangular panel solves with a factored diagonal leaf (f64, m x m packed LU)
// kind 0: x <- L^{-1} P x (unit lower, interchanges first)
// kind 1: x <- U^{-T} x
// kind 2: x <- U^{-1} x
// ---------------------------------------------------------------------------
// A double from one (uniform) lane of the wavefront.
__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// One wavefront per group of CW right-hand sides: lane i keeps rows i (and
// i + 64 when R = 2) of the group in registers; step k broadcasts the finished row k
// (scaled by 1/U_kk for the U solves) and updates the rows it feeds, so the
// steps need no workgroup barrier.  T: the packed LU, column-major.
// ld(i, src, j): the right-hand side entry of row i (source row src after
// the interchanges) in column j; st(i, j, v) stores the solution.
template <int R, int CW, class LD, class ST>
__device__ void trsm_wave_core(const double* T, int m, int kind, const int32_t* perm, int c, const double* rdiag,
                               LD ld, ST st) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j0 = wave * CW; j0 < c; j0 += nw * CW) {
    const int cw = min(CW, c - j0);
    double x[R][CW];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      const int src = i < m ? (kind == 0 ? perm[i] : i) : 0;
#pragma unroll
      for (int q = 0; q < CW; ++q) x[r][q] = (i < m && q < cw) ? ld(i, src, j0 + q) : 0.0;
    }
    const bool fwd = kind != 2;
    for (int s = 0; s < m; ++s) {
      const int k = fwd ? s : m - 1 - s;
      const int kl = k & 63, kr = k >> 6;
      const double sc = kind == 0 ? 1.0 : (rdiag ? rdiag[k] : 1.0 / T[k * m + k]);
      double xk[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        double v = x[0][q];
#pragma unroll
        for (int r = 1; r < R; ++r)
          if (r == kr) v = x[r][q];
        xk[q] = read_lane(v, kl) * sc;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + 64 * r;
        if (i == k) {
#pragma unroll
          for (int q = 0; q < CW; ++q) x[r][q] = xk[q];
        } else if (i < m && (fwd ? i > k : i < k)) {
          // L(i, k) for kind 0, U(k, i) for kind 1, U(i, k) for kind 2
          const double l = kind == 1 ? T[i * m + k] : T[k * m + i];
#pragma unroll
          for (int q = 0; q < CW; ++q) x[r][q] -= l * xk[q];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
#pragma unroll
      for (int q = 0; q < CW; ++q)
        if (i < m && q < cw) st(i, j0 + q, x[r][q]);
    }
  }
}

template <int R, int CW>
__device__ void trsm_wave(const ExecArgs& a, const RV& X, const double* T, int m, int kind, const int32_t* perm,
                          int c, const double* sx, const double* rdiag) {
  trsm_wave_core<R, CW>(
      T, m, kind, perm, c, rdiag,
      [&](int i, int src, int j) { return sx ? sx[j * m + i] : vld(a, X, src, j); },
      [&](int i, int j, double v) { vst(a, X, i, j, v); });
}

__device__ void op_trsm(const ExecArgs& a, const Task& t, char* lds, int kind) {
  PhaseClock pc(a, lds);
  const int m = t.a.rows;
  RV X = resolve(a, t.x);
  const int c = X.cols;
  if (m == 0 || c == 0) return;
  const double* g = a.f64 + t.a.off;
  const int32_t* perm = a.piv + t.piv + m;  // row permutation of the leaf (kind 0)
  if (t.b.type == VT_F64 && (int64_t)m * m + (int64_t)m * c <= kLdsDoubles) {
    // substitution with the inverse of the triangle: x <- T^{-1} (P x), one
    // product on the matrix cores from operands staged in one phase
    double* lI = (double*)lds;
    double* lX = lI + m * m;
    const RV inv{t.b.off, m, m, 1, m, VT_F64};
    const StageSrc none{RV{0, 0, 0, 1, 1, VT_NONE}, nullptr, nullptr};
    stage_views(a, {inv, lI, nullptr}, {X, lX, kind == 0 ? perm : nullptr}, none, none);
    __syncthreads();
    pc.mark(0);
    mfma_lds_gemm<double>(m, c, m, lI, m, lX, m, [&](int i, int j, double v) { vst(a, X, i, j, v); });
    pc.mark(2);
    __syncthreads();
    pc.mark(3);
    return;
  }
  double* sL = (double*)lds;
  const double* sx = nullptr;
  bool tri_lds = false;
  if ((int64_t)m * m + (int64_t)m * c <= kLdsDoubles) {
    // the triangle and the panel (rows gathered for L^{-1} P) in one phase
    double* sX = sL + m * m;
    RV tri{t.a.off, m, m, 1, m, VT_F64};
    const StageSrc none{RV{0, 0, 0, 1, 1, VT_NONE}, nullptr, nullptr};
    stage_views(a, {tri, sL, nullptr}, {X, sX, kind == 0 ? perm : nullptr}, none, none);
    __syncthreads();
    sx = sX;
    tri_lds = true;
  } else if ((int64_t)m * m * 8 <= kLdsBytes) {
    copy_batched(sL, g, m * m);
    __syncthreads();
    tri_lds = true;
  }
  pc.mark(0);
  const double* T = tri_lds ? sL : g;
  // reciprocal diagonal for the U solves, after the staged data when room is left
  double* rdiag = nullptr;
  if (kind != 0 && tri_lds && (int64_t)m * m + (int64_t)(sx ? m * c : 0) + m <= kLdsDoubles) {
    rdiag = sL + m * m + (sx ? m * c : 0);
    for (int i = threadIdx.x; i < m; i += blockDim.x) rdiag[i] = 1.0 / T[i * m + i];
    __syncthreads();
  }
  pc.mark(1);
  // columns per wavefront: spread the panel over all four
  const int per = (c + 3) / 4;
  if (m <= 64) {
    if (per <= 2)
      trsm_wave<1, 2>(a, X, T, m, kind, perm, c, sx, rdiag);
    else if (per <= 4)
      trsm_wave<1, 4>(a, X, T, m, kind, perm, c, sx, rdiag);
    else if (per <= 8)
      trsm_wave<1, 8>(a, X, T, m, kind, perm, c, sx, rdiag);
    else
      trsm_wave<1, 16>(a, X, T, m, kind, perm, c, sx, rdiag);
  } else {
    if (per <= 2)
      trsm_wave<2, 2>(a, X, T, m, kind, perm, c, sx, rdiag);
    else
      trsm_wave<2, 8>(a, X, T, m, kind, perm, c, sx, rdiag);
  }
  pc.mark(2);
  __syncthreads();
  pc.mark(3);
}

// Inverses of the triangles of a factored diagonal leaf (its packed LU, a):
// y = [L^{-1}, U^{-1}], each m x m column-major, column j solving against the
// unit vector e_j.  The substitution applies them as products.
__device__ void op_trtri(const ExecArgs& a, const Task& t, char* lds) {
  const int m = t.a.rows;
  if (m == 0) return;
  const double* g = a.f64 + t.a.off;
  double* Li = a.f64 + t.y.off;
  double* Ui = Li + (int64_t)m * m;
  double* sL = (double*)lds;
  const double* T = g;
  double* rdiag = nullptr;
  if ((int64_t)m * m + m <= kLdsDoubles) {
    copy_batched(sL, g, m * m);
    __syncthreads();
    T = sL;
    rdiag = sL + m * m;
    for (int i = threadIdx.x; i < m; i += blockDim.x) rdiag[i] = 1.0 / sL[i * m + i];
    __syncthreads();
  }
  // the right-hand sides are unit vectors; the interchanges are not applied
  // (kind 0 reads perm, which these sides ignore)
  const int32_t* perm = a.piv + t.piv + m;
  auto unit = [](int i, int, int j) { return i == j ? 1.0 : 0.0; };
  auto stL = [&](int i, int j, double v) { Li[i + (int64_t)j * m] = v; };
  auto stU = [&](int i, int j, double v) { Ui[i + (int64_t)j * m] = v; };
  if (m <= 64) {
    trsm_wave_core<1, 16>(T, m, 0, perm, m, nullptr, unit, stL);
    trsm_wave_core<1, 16>(T, m, 2, perm, m, rdiag, unit, stU);
  } else {
    trsm_wave_core<2, 8>(T, m, 0, perm, m, nullptr, unit, stL);
    trsm_wave_core<2, 8>(T, m, 2, perm, m, rdiag, unit, stU);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Coarsened substitution block (OP_SEQ).  Task refinement may stop at a block
// size (the remark after Algorithm 11): one task then runs the forward (or
// backward) substitution of a diagonal block of at most a few hundred rows,
// in the order of the recursion, with the block's rows of the panel held in
// LDS from its first micro-operation to its last.  The micro-operations (leaf
// triangular solves, dense and low-rank leaf products) read the factors from
// global memory; a product from the neighbouring block (folded into the task
// because it is the last update the block waits for) reads its source rows
// from the global panel.  A panel wider than the LDS copy holds is done in
// column sweeps.
// ---------------------------------------------------------------------------
struct SeqPanel {
  double* p;  // the block's rows of columns [j0, j0 + cw), leading dimension W
  int W, cw, j0;
};

// block rows y += alpha A x; A global (m x k); x block rows or global rows
__device__ void seq_gemm(const ExecArgs& a, const Task& u, const SeqPanel& sp, char* lds) {
  const RV A = resolve(a, u.a);
  const int m = A.rows, k = A.cols, cw = sp.cw;
  if (m == 0 || k == 0) return;
  double* Y = sp.p + u.y.off;
  const bool xl = (u.b.dyn & DYN_LOCAL) != 0;
  const RV B = resolve(a, u.b);
  const double alpha = u.alpha;
  const StageSrc none{RV{0, 0, 0, 1, 1, VT_NONE}, nullptr, nullptr};
  const int kc = min(k, kLdsDoubles / (m + (xl ? 0 : cw)));
  double* lA = (double*)lds;
  for (int k0 = 0; k0 < k; k0 += kc) {
    const int kk = min(kc, k - k0);
    double* lX = lA + m * kk;
    RV As = A;
    As.off += (int64_t)k0 * A.cs;
    As.cols = kk;
    StageSrc sx = none;
    if (!xl) {
      RV Bs = B;
      Bs.off += (int64_t)k0 * B.rs + (int64_t)sp.j0 * B.cs;
      Bs.rows = kk;
      Bs.cols = cw;
      sx = StageSrc{Bs, lX, nullptr};
    }
    stage_views(a, {As, lA, nullptr}, sx, none, none);
    __syncthreads();
    const double* xs = xl ? sp.p + u.b.off + k0 : lX;
    const int ldx = xl ? sp.W : kk;
    mfma_lds_gemm<double>(m, cw, kk, lA, m, xs, ldx, [&](int i, int j, double v) { Y[i + j * sp.W] += alpha * v; });
    __syncthreads();
  }
}

// block rows y += alpha U (V^T x); U (m x k) and V^T (k x n2) global
__device__ void seq_lrgemm(const ExecArgs& a, const Task& u, const SeqPanel& sp, char* lds) {
  const RV U = resolve(a, u.a), Vt = resolve(a, u.b);
  const int m = U.rows, k = U.cols, n2 = Vt.cols, cw = sp.cw;
  if (m == 0 || k == 0 || n2 == 0) return;
  double* Y = sp.p + u.y.off;
  const bool xl = (u.x.dyn & DYN_LOCAL) != 0;
  const RV X = resolve(a, u.x);
  const double alpha = u.alpha;
  const StageSrc none{RV{0, 0, 0, 1, 1, VT_NONE}, nullptr, nullptr};
  const int room = kLdsDoubles - k * cw;
  double* lB = (double*)lds;
  double* lT = lB + room;  // T = V^T x (k x cw)
  const int nc = min(n2, room / (k + (xl ? 0 : cw)));
  for (int c0 = 0; c0 < n2; c0 += nc) {
    const int nn = min(nc, n2 - c0);
    double* lX = lB + k * nn;
    RV Bs = Vt;
    Bs.off += (int64_t)c0 * Vt.cs;
    Bs.cols = nn;
    StageSrc sx = none;
    if (!xl) {
      RV Xs = X;
      Xs.off += (int64_t)c0 * X.rs + (int64_t)sp.j0 * X.cs;
      Xs.rows = nn;
      Xs.cols = cw;
      sx = StageSrc{Xs, lX, nullptr};
    }
    stage_views(a, {Bs, lB, nullptr}, sx, none, none);
    __syncthreads();
    const double* xs = xl ? sp.p + u.x.off + c0 : lX;
    const int ldx = xl ? sp.W : nn;
    const bool first = c0 == 0;
    mfma_lds_gemm<double>(k, cw, nn, lB, k, xs, ldx,
                          [&](int i, int j, double v) { lT[i + j * k] = first ? v : lT[i + j * k] + v; });
    __syncthreads();
  }
  const int mc = min(m, room / k);
  for (int r0 = 0; r0 < m; r0 += mc) {
    const int mm = min(mc, m - r0);
    RV Us = U;
    Us.off += (int64_t)r0 * U.rs;
    Us.rows = mm;
    stage_views(a, {Us, lB, nullptr}, none, none, none);
    __syncthreads();
    mfma_lds_gemm<double>(mm, cw, k, lB, mm, lT, k,
                          [&](int i, int j, double v) { Y[r0 + i + j * sp.W] += alpha * v; });
    __syncthreads();
  }
}

// triangular solve of a diagonal leaf on the block rows (kind 0: L with the
// leaf's interchanges, kind 2: U)
__device__ void seq_trsm(const ExecArgs& a, const Task& u, const SeqPanel& sp, char* lds, int kind) {
  const int m = u.a.rows, c = sp.cw, W = sp.W;
  if (m == 0) return;
  double* X = sp.p + u.x.off;
  const double* g = a.f64 + u.a.off;
  const int32_t* perm = a.piv + u.piv + m;
  if (u.b.type == VT_F64 && (int64_t)m * m + (int64_t)m * c <= kLdsDoubles) {
    // x <- T^{-1} (P x) with the leaf's inverse (see op_trsm)
    double* lI = (double*)lds;
    double* lX = lI + m * m;
    copy_batched(lI, a.f64 + u.b.off, m * m);
    for (int e = threadIdx.x; e < m * c; e += blockDim.x) {
      const int i = e % m, j = e / m;
      lX[e] = X[(kind == 0 ? perm[i] : i) + j * W];
    }
    __syncthreads();
    mfma_lds_gemm<double>(m, c, m, lI, m, lX, m, [&](int i, int j, double v) { X[i + j * W] = v; });
    return;
  }
  double* sL = (double*)lds;
  const double* T = g;
  double* rdiag = nullptr;
  if ((int64_t)m * m + m <= kLdsDoubles) {
    copy_batched(sL, g, m * m);
    __syncthreads();
    T = sL;
    if (kind == 2) {
      rdiag = sL + m * m;
      for (int i = threadIdx.x; i < m; i += blockDim.x) rdiag[i] = 1.0 / sL[i * m + i];
      __syncthreads();
    }
  }
  auto ld = [&](int, int src, int j) { return X[src + j * W]; };
  auto st = [&](int i, int j, double v) { X[i + j * W] = v; };
  const int per = (c + 3) / 4;
  if (m <= 64) {
    if (per <= 2)
      trsm_wave_core<1, 2>(T, m, kind, perm, c, rdiag, ld, st);
    else if (per <= 4)
      trsm_wave_core<1, 4>(T, m, kind, perm, c, rdiag, ld, st);
    else if (per <= 8)
      trsm_wave_core<1, 8>(T, m, kind, perm, c, rdiag, ld, st);
    else
      trsm_wave_core<1, 16>(T, m, kind, perm, c, rdiag, ld, st);
  } else {
    if (per <= 2)
      trsm_wave_core<2, 2>(T, m, kind, perm, c, rdiag, ld, st);
    else
      trsm_wave_core<2, 8>(T, m, kind, perm, c, rdiag, ld, st);
  }
}

__device__ void op_seq(const ExecArgs& a, const Task& t, char* lds) {
  const RV P = resolve(a, t.y);
  const int W = P.rows, c = P.cols, n = t.lr;
  if (W == 0 || c == 0 || n == 0) return;
  const int cmax = a.seq_panel / W;
  if (cmax < 1 || P.rs != 1 || !a.seq) {
    if (threadIdx.x == 0) atomicOr(&a.status[0], ST_BADOP);
    return;
  }
  const int nsw = (c + cmax - 1) / cmax, cwid = (c + nsw - 1) / nsw;
  double* pl = (double*)(lds + kSeqPanelOff);
  Task* rec = (Task*)(lds + kSeqLdsOff);
  constexpr int kWords = (int)(sizeof(Task) / 4);
  const int* src = (const int*)(a.seq + t.piv);
  const int tid = threadIdx.x;
  // timeline (debug): ticks of the triangular solves, dense products,
  // low-rank products and panel copies, and the counts of the first two kinds
  unsigned long long* ph = a.trace ? (unsigned long long*)(lds + kLdsBytes) + kCtrSize : nullptr;
  uint64_t tk0 = 0;
  for (int j0 = 0; j0 < c; j0 += cwid) {
    const int cw = min(cwid, c - j0), tot = W * cw;
    double* g = a.f64 + P.off + (int64_t)j0 * P.cs;
    if (ph && tid == 0) tk0 = wall_clock64();
    for (int base = 0; base < tot; base += 8 * kThreads) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = base + q * kThreads + tid;
        v[q] = e < tot ? g[e % W + (int64_t)(e / W) * P.cs] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = base + q * kThreads + tid;
        if (e < tot) pl[e] = v[q];
      }
    }
    if (tid < kWords) ((int*)rec)[tid] = src[tid];
    __syncthreads();
    if (ph && tid == 0) {
      ph[3] += wall_clock64() - tk0;
      tk0 = wall_clock64();
    }
    const SeqPanel sp{pl, W, cw, j0};
    for (int k = 0; k < n; ++k) {
      const Task& u = rec[k & 1];
      const int uop = u.op;
      // the next record is loaded while this micro-operation runs
      int nxt = 0;
      if (k + 1 < n && tid < kWords) nxt = src[(k + 1) * kWords + tid];
      switch (u.op) {
        case OP_TRSM_L:
          seq_trsm(a, u, sp, lds, 0);
          break;
        case OP_TRSM_U:
          seq_trsm(a, u, sp, lds, 2);
          break;
        case OP_GEMM:
          seq_gemm(a, u, sp, lds);
          break;
        case OP_LRGEMM:
          seq_lrgemm(a, u, sp, lds);
          break;
        default:
          if (tid == 0) atomicOr(&a.status[0], ST_BADOP);
          break;
      }
      if (k + 1 < n && tid < kWords) ((int*)&rec[(k + 1) & 1])[tid] = nxt;
      __syncthreads();
      if (ph && tid == 0) {
        const uint64_t t1 = wall_clock64();
        const int slot = (uop == OP_TRSM_L || uop == OP_TRSM_U) ? 0 : uop == OP_GEMM ? 1 : 2;
        ph[slot] += t1 - tk0;
        ph[slot == 0 ? 4 : 5] += 1;
        tk0 = t1;
      }
    }
    for (int base = 0; base < tot; base += 8 * kThreads) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = base + q * kThreads + tid;
        if (e < tot) g[e % W + (int64_t)(e / W) * P.cs] = pl[e];
      }
    }
    __syncthreads();
    if (ph && tid == 0) ph[3] += wall_clock64() - tk0;
  }
}

// ---------------------------------------------------------------------------
// TRUNC: C <- T_eps(U_C V_C^T + alpha pad(A) pad(B)^T)  (Sec. 2.3)
//
// The stacked factors U_s = [U_C, alpha A], V_s = [V_C, B] (m x K, n x K) are
// never formed.  Each side's R factor comes from the Gram matrix (CholeskyQR
// with column scaling and diagonal pivoting; accumulated in FP64 whatever the
// storage type), the K x K core R_U R_V^T is diagonalised by one-sided Jacobi
// in FP64, and the kept singular triplets are written back as
//   U <- U_s T_U,  V <- V_s T_V   (Sigma folded into U).
// ---------------------------------------------------------------------------
struct Stack {  // one side of the stack: rows [0, m); columns [0, kc) from C, then
  RV c;         // [kc, kc+kp) from term 1 (rows offset by r0, zero outside), then
  RV t;         // [kc+kp, kc+kp+kp2) from term 2 (rows offset by r2)
  RV t2;
  const double* tptr;  // term 1 outside the arenas (column-major, ld t.cs), or null
  int m, kc, kp, r0, kp2, r2;
  double alpha, alpha2;
  __device__ __forceinline__ double operator()(const ExecArgs& a, int r, int i) const {
    if (i < kc) return vld(a, c, r, i);
    i -= kc;
    if (i < kp) {
      int rr = r - r0;
      if (rr < 0 || rr >= t.rows) return 0.0;
      if (tptr) return alpha * tptr[rr + (int64_t)i * t.cs];
      return alpha * vld(a, t, rr, i);
    }
    i -= kp;
    int rr = r - r2;
    if (rr < 0 || rr >= t2.rows) return 0.0;
    return alpha2 * vld(a, t2, rr, i);
  }
};

// scaled, diagonally pivoted Cholesky of the K x K Gram matrix G (row-major, full);
// on exit rows [0, r) of G hold R' (upper trapezoidal, pivoted order), perm[q] =
// original column at pivot position q, dsc[l] = 1/||column l|| (0 for a zero column).
__device__ int pivoted_cholesky(double* G, int K, int* perm, double* dsc, int* s_int) {
  const int tid = threadIdx.x;
  for (int l = tid; l < K; l += blockDim.x) {
    double d = G[l * K + l];
    dsc[l] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    perm[l] = l;
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += blockDim.x) G[e] *= dsc[e / K] * dsc[e % K];
  __syncthreads();
  const double tol = 8.0 * K * 2.220446049250313e-16;
  int r = K;
  for (int s = 0; s < K; ++s) {
    if (tid < 64) {
      double best = -1.0;
      int bi = K;
      for (int i = s + tid; i < K; i += 64) {
        double v = G[i * K + i];
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      wave_argmax(best, bi);
      if (tid == 0) {
        s_int[0] = bi < K ? bi : s;
        s_int[1] = (bi < K && best > tol) ? 1 : 0;
      }
    }
    __syncthreads();
    const int go = s_int[1];
    const int p = s_int[0];
    __syncthreads();
    if (!go) {
      r = s;
      break;
    }
    if (p != s) {
      for (int l = tid; l < K; l += blockDim.x) {  // swap rows s, p
        double x = G[s * K + l];
        G[s * K + l] = G[p * K + l];
        G[p * K + l] = x;
      }
      __syncthreads();
      for (int l = tid; l < K; l += blockDim.x) {  // swap columns s, p
        double x = G[l * K + s];
        G[l * K + s] = G[l * K + p];
        G[l * K + p] = x;
      }
      if (tid == 0) {
        int x = perm[s];
        perm[s] = perm[p];
        perm[p] = x;
      }
      __syncthreads();
    }
    const double d = sqrt(G[s * K + s]);
    __syncthreads();
    for (int l = s + tid; l < K; l += blockDim.x) G[s * K + l] = (l == s) ? d : G[s * K + l] / d;
    __syncthreads();
    const int rem = K - s - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      int i = s + 1 + e / rem, j = s + 1 + e % rem;
      G[i * K + j] -= G[s * K + i] * G[s * K + j];
    }
    __syncthreads();
  }
  return r;
}

// Per-workgroup scratch (doubles) of a truncation with K <= kMaxK, k' <= kMaxCap.
struct TruncScratch {
  double *GU, *GV, *B, *Z, *YU, *YV, *TU, *TV, *dU, *dV, *sig;
  int *pU, *pV, *sel, *posU, *posV;
};


__device__ TruncScratch trunc_scratch(double* p) {
  TruncScratch s;
  s.GU = p;
  p += kMaxK * kMaxK;
  s.GV = p;
  p += kMaxK * kMaxK;
  s.B = p;
  p += kMaxK * kMaxK;
  s.Z = p;
  p += kMaxK * kMaxK;
  s.YU = p;
  p += kMaxK * kMaxCap;
  s.YV = p;
  p += kMaxK * kMaxCap;
  s.TU = p;
  p += kMaxK * kMaxCap;
  s.TV = p;
  p += kMaxK * kMaxCap;
  s.dU = p;
  p += kMaxK;
  s.dV = p;
  p += kMaxK;
  s.sig = p;
  p += kMaxK;
  int* ip = (int*)p;  // 5 * kMaxK ints = 2.5 * kMaxK doubles
  s.pU = ip;
  ip += kMaxK;
  s.pV = ip;
  ip += kMaxK;
  s.sel = ip;
  ip += kMaxK;
  s.posU = ip;
  ip += kMaxK;
  s.posV = ip;
  return s;
}

// One-sided Jacobi (Hestenes) on B (p x q, column-major, ld p): orthogonalise the
// columns; Z (q x q, column-major) accumulates the rotations, or is null when
// the caller needs only B Z.  Round-robin pairing, all pairs of a round in
// parallel.
__device__ int jacobi_svd(double* B, double* Z, int p, int q, int* s_flag, double eps) {
  static_assert(kThreads == 256, "four wavefront partial sums below");
  const int tid = threadIdx.x;
  if (Z)
    for (int e = tid; e < q * q; e += blockDim.x) Z[e] = (e % q == e / q) ? 1.0 : 0.0;
  __syncthreads();
  if (q < 2) return 0;
  const int N = q + (q & 1);
  const int npairs = N / 2;
  int tpp = 1;
  while (tpp * 2 * npairs <= (int)blockDim.x && tpp < 64) tpp *= 2;
  const int pair = tid / tpp, lane = tid % tpp;
  // columns count as orthogonal once |x.y| <= tol ||x|| ||y||, with tol at the
  // rounding level of a length-p dot product (a tighter test never settles);
  // columns below the noise level (u ||B||_F)^2 count as converged
  const double tol = fmax(2.0 * (p > 16 ? p : 16) * 2.220446049250313e-16, 1e-4 * eps);
  if (tid == 0) s_flag[1] = 0;
  __syncthreads();
  double* fro_s = (double*)(s_flag + 2);
  {
    // per-wavefront partial sums added in a fixed order (the slots after
    // fro_s are free once the caller's QR and Cholesky are done)
    double* part = (double*)(s_flag + 4);
    double f = 0.0;
    for (int e = tid; e < p * q; e += blockDim.x) f += B[e] * B[e];
    f = group_sum(f, 64);
    if ((tid & 63) == 0) part[tid >> 6] = f;
    __syncthreads();
    if (tid == 0) *fro_s = part[0] + part[1] + part[2] + part[3];
  }
  __syncthreads();
  const double tiny = *fro_s * fmax(1e-4 * eps * eps, 4.930380657631324e-32 * (p > 16 ? p : 16));
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    if (tid == 0) s_flag[0] = 0;
    __syncthreads();
    for (int rnd = 0; rnd < N - 1; ++rnd) {
      int ci = -1, cj = -1;
      if (pair < npairs) {
        const int mm = N - 1;
        if (pair == 0) {
          ci = mm;
          cj = rnd;
        } else {
          ci = (rnd + pair) % mm;
          cj = (rnd - pair + mm) % mm;
        }
        if (ci >= q || cj >= q) ci = cj = -1;
      }
      double al = 0.0, be = 0.0, ga = 0.0;
      if (ci >= 0)
        for (int r = lane; r < p; r += tpp) {
          double x = B[ci * p + r], y = B[cj * p + r];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
      al = group_sum(al, tpp);
      be = group_sum(be, tpp);
      ga = group_sum(ga, tpp);
      if (ci >= 0 && ga != 0.0 && al > tiny && be > tiny && ga * ga > tol * tol * (al * be)) {
        if (lane == 0) s_flag[0] = 1;
        double cs, sn;
        jacobi_rotation(al, be, ga, cs, sn);
        for (int r = lane; r < p; r += tpp) {
          double x = B[ci * p + r], y = B[cj * p + r];
          B[ci * p + r] = cs * x - sn * y;
          B[cj * p + r] = sn * x + cs * y;
        }
        if (Z)
          for (int r = lane; r < q; r += tpp) {
            double x = Z[ci * q + r], y = Z[cj * q + r];
            Z[ci * q + r] = cs * x - sn * y;
            Z[cj * q + r] = sn * x + cs * y;
          }
      }
      __syncthreads();
    }
    const int again = s_flag[0];
    __syncthreads();
    if (!again) break;
  }
  return sweep + 1;
}

// Solve the r x r upper triangle of R' (rows of G, stride K) against rhs columns
// (r x kk, column-major, ld r) in place; one thread per column (columns j0,
// j0 + stride, ...).
__device__ void upper_solve(const double* R, int K, int r, double* X, int kk, int j0, int stride) {
  for (int j = j0; j < kk; j += stride) {
    double* x = X + (int64_t)j * r;
    for (int i = r - 1; i >= 0; --i) {
      double s = x[i];
      for (int q = i + 1; q < r; ++q) s -= R[i * K + q] * x[q];
      x[i] = s / R[i * K + i];
    }
  }
}

// Statistics counters of the workgroup (after the task work area in LDS);
// only touched when ExecArgs::counters is set, by thread 0.
__device__ __forceinline__ unsigned long long* wg_ctr(char* lds) { return (unsigned long long*)(lds + kLdsBytes); }

// Adds the wall-clock ticks since *t0 to counter slot (thread 0) and restarts *t0.
__device__ __forceinline__ void phase_tick(const ExecArgs& a, char* lds, int slot, uint64_t* t0) {
  if (a.counters && threadIdx.x == 0) {
    uint64_t t1 = wall_clock64();
    wg_ctr(lds)[slot] += t1 - *t0;
    if (a.trace) wg_ctr(lds)[kCtrSize + (slot - kCtrPhase) % 6] += t1 - *t0;
    *t0 = t1;
  }
}

// ---------------------------------------------------------------------------
// Truncation for stacked ranks K <= 32: every K x K work matrix in LDS, the
// two Cholesky factorisations and the Jacobi SVD each run inside one
// wavefront (no workgroup barrier per step), the Gram matrices and the
// rebuild stream the factor panels with many loads in flight.
// ---------------------------------------------------------------------------
constexpr int kSmallK = 32;

// Wavefront-level ordering of LDS accesses (all lanes of a wavefront).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One column of a stacked panel resolved once: stack row r reads element
// (r - lo) of the column at `base` with row stride rs (zero outside
// [lo, hi)), times `scale`; an identity column is `scale` at row `one`.
struct ColRef {
  const double* p64;
  const float* p32;
  int64_t base;
  int rs, lo, hi, one;
  double scale;
  __device__ __forceinline__ double operator()(int r) const {
    if (r < lo || r >= hi) return 0.0;
    if (one >= 0) return r == one ? scale : 0.0;
    const int64_t k = base + (int64_t)(r - lo) * rs;
    return scale * (p64 ? p64[k] : (double)p32[k]);
  }
};

__device__ __forceinline__ ColRef col_of(const RV& v, const ExecArgs& a, int j, int lo, int hi, double scale) {
  ColRef c;
  c.p64 = v.type == VT_F64 ? a.f64 : nullptr;
  c.p32 = v.type == VT_F32 ? a.f32 : nullptr;
  c.base = v.off + (int64_t)j * v.cs;
  c.rs = v.rs;
  c.lo = lo;
  c.hi = (v.type == VT_F64 || v.type == VT_F32 || v.type == VT_IDENT) ? hi : lo;
  c.one = v.type == VT_IDENT ? lo + j : -1;
  c.scale = scale;
  return c;
}

__device__ __forceinline__ ColRef stack_col(const ExecArgs& a, const Stack& st, int i) {
  if (i < st.kc) return col_of(st.c, a, i, 0, st.m, 1.0);
  i -= st.kc;
  if (i < st.kp) {
    ColRef c = col_of(st.t, a, i, st.r0, min(st.m, st.r0 + st.t.rows), st.alpha);
    if (st.tptr) {  // term 1 outside the arenas (column-major, ld t.cs)
      c.p64 = st.tptr;
      c.p32 = nullptr;
      c.base = (int64_t)i * st.t.cs;
      c.rs = 1;
      c.hi = min(st.m, st.r0 + st.t.rows);
      c.one = -1;
    }
    return c;
  }
  i -= st.kp;
  return col_of(st.t2, a, i, st.r2, min(st.m, st.r2 + st.t2.rows), st.alpha2);
}


// A stack column resolved once into LDS for streaming: stack row r reads
// element (r - lo) * rs of `base` (FP32 when is32) times scale inside
// [lo, hi); an identity column holds scale at row `one`.
struct ColDesc {
  const void* base;
  int lo, hi, one, rs, is32, pad_;
  double scale;
};

__device__ __forceinline__ double desc_ld(const ColDesc& d, int r) {
  if (r < d.lo || r >= d.hi) return 0.0;
  if (d.one >= 0) return r == d.one ? d.scale : 0.0;
  const int64_t k = (int64_t)(r - d.lo) * d.rs;
  return d.scale * (d.is32 ? (double)((const float*)d.base)[k] : ((const double*)d.base)[k]);
}

// Descriptors of the K columns of a stack (threads t0 .. t0 + K - 1).
__device__ __forceinline__ void stack_descs(const ExecArgs& a, const Stack& st, int K, ColDesc* out, int t0) {
  const int c = (int)threadIdx.x - t0;
  if (c >= 0 && c < K) {
    const ColRef r = stack_col(a, st, c);
    ColDesc d;
    d.base = r.p64 ? (const void*)(r.p64 + r.base) : r.p32 ? (const void*)(r.p32 + r.base) : nullptr;
    d.lo = r.lo;
    d.hi = (d.base || r.one >= 0) ? r.hi : r.lo;
    d.one = r.one;
    d.rs = r.rs;
    d.is32 = r.p32 != nullptr && r.p64 == nullptr;
    d.pad_ = 0;
    d.scale = r.scale;
    out[c] = d;
  }
}

// Copies rows [r0, r0 + rows) of a stack of K described columns into buf
// (column c at buf + c * ld): element e = c * rows + i, sixteen per thread in
// flight, consecutive threads on consecutive rows.
template <int kBatch = 16>
__device__ __forceinline__ void stage_desc(const ColDesc* desc, int K, int r0, int rows, double* buf, int ld) {
  const int total = rows * K;
  for (int base = 0; base < total; base += kBatch * kThreads) {
    double v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      v[u] = e < total ? desc_ld(desc[e / rows], r0 + e % rows) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = base + u * kThreads + (int)threadIdx.x;
      if (e < total) buf[(e / rows) * ld + e % rows] = v[u];
    }
  }
}


// The three 16 x 16 tiles (00, 01, 11) of a K <= 32 Gram matrix held by one
// wavefront.
struct GramAcc {
  Mfma<double>::acc_t a00, a01, a11;
};

// Adds rows [0, rows) of a staged chunk (column c at buf + c * ld) to the
// calling wavefront's tiles.
__device__ __forceinline__ void gram_rows(const double* buf, int ld, int rows, int K, GramAcc& g) {
  using M = Mfma<double>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (K + 15) >> 4;  // 1 or 2 tiles per side
  const int c0 = li, c1 = 16 + li;
  for (int t0 = 4 * wave; t0 < rows; t0 += 16) {
    const int t = t0 + lk;
    const bool in = t < rows;
    const double x0 = (in && c0 < K) ? buf[c0 * ld + t] : 0.0;
    const double x1 = (in && c1 < K) ? buf[c1 * ld + t] : 0.0;
    g.a00 = M::step(x0, x0, g.a00);
    if (nt > 1) {
      g.a01 = M::step(x0, x1, g.a01);
      g.a11 = M::step(x1, x1, g.a11);
    }
  }
}

// G from the four wavefronts' tiles, summed in a fixed order through `red`
// (4 x 3 x 256 doubles of LDS not otherwise in use); ends with a barrier.
__device__ __forceinline__ void gram_reduce(const GramAcc& g, int K, double* G, double* red) {
  using M = Mfma<double>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = M::row(lk, r) * 16 + li;
    red[(wave * 3 + 0) * 256 + e] = g.a00[r];
    red[(wave * 3 + 1) * 256 + e] = g.a01[r];
    red[(wave * 3 + 2) * 256 + e] = g.a11[r];
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += blockDim.x) {
    const int i = e / K, j = e % K;
    // G(i, j) from tile (ti, tj); the lower tile (1, 0) is the transpose of (0, 1)
    const int ti = i >> 4, tj = j >> 4;
    int tile, ii = i & 15, jj = j & 15;
    if (ti == 0 && tj == 0)
      tile = 0;
    else if (ti == 1 && tj == 1)
      tile = 2;
    else {
      tile = 1;
      if (ti == 1) {  // (1, 0): entry (jj, ii) of tile (0, 1)
        const int x = ii;
        ii = jj;
        jj = x;
      }
    }
    const int idx = tile * 256 + ii * 16 + jj;
    G[e] = (red[idx] + red[3 * 256 + idx]) + (red[6 * 256 + idx] + red[9 * 256 + idx]);
  }
  __syncthreads();
}

// G = X^T X (K x K, row-major, K <= 32) for X = the stacked panel st (m x K),
// staged through LDS in chunks of up to `cap_rows` rows, on the matrix cores
// in FP64: wavefront w takes the rows 4 w + 16 s .. + 3 of every chunk into
// its own 16 x 16 tiles of G (both MFMA operands are columns of X), and the
// four wavefronts' tiles are summed in LDS at the end (the staging buffer,
// free by then, holds them).
__device__ void gram_stream(const ExecArgs& a, const Stack& st, const ColDesc* desc, int K, int m, double* G,
                            double* buf, int cap_rows) {
  using M = Mfma<double>;
  const int ld = cap_rows | 1;  // odd stride: conflict-free column reads
  GramAcc g{M::zero(), M::zero(), M::zero()};
  for (int r0 = 0; r0 < m; r0 += cap_rows) {
    const int rows = min(cap_rows, m - r0);
    // every chunk in batches of sixteen loads per thread over all columns
    stage_desc(desc, K, r0, rows, buf, ld);
    __syncthreads();
    gram_rows(buf, ld, rows, K, g);
    __syncthreads();
  }
  gram_reduce(g, K, G, buf);
}

// G = X^T X (K x K, row-major, K <= 64) for the K described columns of an
// m-row stack, on the FP64 matrix cores.  Rows are staged through `buf`
// (cap doubles) in chunks; the upper 16 x 16 tiles of G (at most ten) are
// dealt to the four wavefronts in turn, and each wavefront sweeps all rows
// of a chunk for its tiles, so no reduction between wavefronts is needed.
// G may overlap buf: it is written after the last chunk has been read.
__device__ void gram_tiles(const ColDesc* desc, int K, int m, double* G, double* buf, int cap) {
  using M = Mfma<double>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (K + 15) >> 4, ntiles = nt * (nt + 1) / 2;
  const int cap_rows = cap / K - 1;
  const int ld = cap_rows | 1;  // odd stride: conflict-free column reads
  int ti[3], tj[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    int idx = wave + 4 * s, a = 0;
    ti[s] = tj[s] = -1;
    if (idx < ntiles) {
      while (idx >= nt - a) {  // row a of the upper triangle holds nt - a tiles
        idx -= nt - a;
        ++a;
      }
      ti[s] = a;
      tj[s] = a + idx;
    }
  }
  M::acc_t acc[3] = {M::zero(), M::zero(), M::zero()};
  for (int r0 = 0; r0 < m; r0 += cap_rows) {
    const int rows = min(cap_rows, m - r0);
    stage_desc(desc, K, r0, rows, buf, ld);
    __syncthreads();
    for (int t0 = 0; t0 < rows; t0 += 4) {
      const int t = t0 + lk;
      const bool in = t < rows;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (ti[s] < 0) continue;
        const int ca = 16 * ti[s] + li, cb = 16 * tj[s] + li;
        const double xa = (in && ca < K) ? buf[ca * ld + t] : 0.0;
        const double xb = (in && cb < K) ? buf[cb * ld + t] : 0.0;
        acc[s] = M::step(xa, xb, acc[s]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if (ti[s] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti[s] + M::row(lk, r), j = 16 * tj[s] + li;
      if (i < K && j < K) {
        G[i * K + j] = acc[s][r];
        if (ti[s] != tj[s]) G[j * K + i] = acc[s][r];
      }
    }
  }
  __syncthreads();
}

// Scaled, diagonally pivoted Cholesky of G (K x K, K <= 128) by the calling
// wavefront alone; same results as pivoted_cholesky.  Returns the rank.
__device__ int pivoted_cholesky_wave(double* G, int K, int* perm, double* dsc) {
  const int lane = threadIdx.x & 63;
  for (int l = lane; l < K; l += 64) {
    double d = G[l * K + l];
    dsc[l] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    perm[l] = l;
  }
  wave_sync();
  for (int e = lane; e < K * K; e += 64) G[e] *= dsc[e / K] * dsc[e % K];
  wave_sync();
  const double tol = 8.0 * K * 2.220446049250313e-16;
  for (int s = 0; s < K; ++s) {
    double best = -1.0;
    int bi = K;
    for (int l = s + lane; l < K; l += 64) {
      double v = G[l * K + l];
      if (v > best) {
        best = v;
        bi = l;
      }
    }
    wave_argmax(best, bi);
    if (bi >= K || !(best > tol)) return s;
    const int p = bi;
    if (p != s) {
      for (int l = lane; l < K; l += 64) {  // swap rows s and p
        double x = G[s * K + l];
        G[s * K + l] = G[p * K + l];
        G[p * K + l] = x;
      }
      wave_sync();
      for (int l = lane; l < K; l += 64) {  // swap columns s and p
        double x = G[l * K + s];
        G[l * K + s] = G[l * K + p];
        G[l * K + p] = x;
      }
      if (lane == 0) {
        int x = perm[s];
        perm[s] = perm[p];
        perm[p] = x;
      }
      wave_sync();
    }
    const double d = sqrt(G[s * K + s]);
    wave_sync();
    for (int l = s + lane; l < K; l += 64) G[s * K + l] = (l == s) ? d : G[s * K + l] / d;
    wave_sync();
    const int rem = K - s - 1;
    for (int e = lane; e < rem * rem; e += 64) {
      int i = s + 1 + e / rem, j = s + 1 + e % rem;
      G[i * K + j] -= G[s * K + i] * G[s * K + j];
    }
    wave_sync();
  }
  return K;
}

// One-sided Jacobi on B (p x q, column-major, q <= 128) by the calling
// wavefront; Z as for jacobi_svd (null: rotations not kept).
__device__ int jacobi_svd_wave(double* B, double* Z, int p, int q, double eps) {
  const int lane = threadIdx.x & 63;
  if (Z)
    for (int e = lane; e < q * q; e += 64) Z[e] = (e % q == e / q) ? 1.0 : 0.0;
  wave_sync();
  if (q < 2) return 0;
  const int N = q + (q & 1);
  const int npairs = N / 2;
  int tpp = 1;
  while (tpp * 2 * npairs <= 64 && tpp < 64) tpp *= 2;
  const int pair = lane / tpp, sub = lane % tpp;
  // Only singular triplets near or above the truncation threshold
  // eps * sigma_1 matter: a pair counts as converged once its cosine is below
  // max(rounding level, 1e-4 eps), and a column whose norm is below
  // 0.01 eps ||B||_F (< 0.1 eps sigma_1 for q <= 64) is discarded anyway and
  // is not rotated.
  const double tol = fmax(2.0 * (p > 16 ? p : 16) * 2.220446049250313e-16, 1e-4 * eps);
  double fro = 0.0;
  for (int e = lane; e < p * q; e += 64) fro += B[e] * B[e];
  for (int off = 32; off >= 1; off >>= 1) fro += __shfl_xor(fro, off);
  const double tiny = fro * fmax(1e-4 * eps * eps, 4.930380657631324e-32 * (p > 16 ? p : 16));
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    int rotated = 0;
    for (int rnd = 0; rnd < N - 1; ++rnd) {
      int ci = -1, cj = -1;
      if (pair < npairs) {
        const int mm = N - 1;
        if (pair == 0) {
          ci = mm;
          cj = rnd;
        } else {
          ci = (rnd + pair) % mm;
          cj = (rnd - pair + mm) % mm;
        }
        if (ci >= q || cj >= q) ci = cj = -1;
      }
      // a pair's columns stay in registers between the products and the
      // rotation when each lane holds at most kRows of their rows (padding
      // rows add exact zeros, so the sums are those of the plain loop)
      constexpr int kRows = 8;
      const bool inreg = p <= kRows * tpp;
      double xs[kRows], ys[kRows];
      double al = 0.0, be = 0.0, ga = 0.0;
      if (ci >= 0) {
        if (inreg) {
#pragma unroll
          for (int k = 0; k < kRows; ++k) {
            const int r = sub + k * tpp;
            xs[k] = r < p ? B[ci * p + r] : 0.0;
            ys[k] = r < p ? B[cj * p + r] : 0.0;
          }
#pragma unroll
          for (int k = 0; k < kRows; ++k) {
            al += xs[k] * xs[k];
            be += ys[k] * ys[k];
            ga += xs[k] * ys[k];
          }
        } else {
          for (int r = sub; r < p; r += tpp) {
            double x = B[ci * p + r], y = B[cj * p + r];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
        }
      }
      al = group_sum(al, tpp);
      be = group_sum(be, tpp);
      ga = group_sum(ga, tpp);
      if (ci >= 0 && ga != 0.0 && al > tiny && be > tiny && ga * ga > tol * tol * (al * be)) {
        rotated = 1;
        double cs, sn;
        jacobi_rotation(al, be, ga, cs, sn);
        if (inreg) {
#pragma unroll
          for (int k = 0; k < kRows; ++k) {
            const int r = sub + k * tpp;
            if (r < p) {
              B[ci * p + r] = cs * xs[k] - sn * ys[k];
              B[cj * p + r] = sn * xs[k] + cs * ys[k];
            }
          }
        } else {
          for (int r = sub; r < p; r += tpp) {
            double x = B[ci * p + r], y = B[cj * p + r];
            B[ci * p + r] = cs * x - sn * y;
            B[cj * p + r] = sn * x + cs * y;
          }
        }
        if (Z)
          for (int r = sub; r < q; r += tpp) {
            double x = Z[ci * q + r], y = Z[cj * q + r];
            Z[ci * q + r] = cs * x - sn * y;
            Z[cj * q + r] = sn * x + cs * y;
          }
      }
      wave_sync();
    }
    // any lane rotated -> another sweep
    unsigned long long anyrot = __ballot(rotated);
    if (anyrot == 0ull) break;
  }
  return sweep + 1;
}

// out (m x kk) = X T for the stacked panel X = st (m x K, K <= 32) and T
// (K x kk, column-major, LDS).  Rows are staged through LDS in chunks; a
// chunk is read completely before any of its rows is written, so out may
// alias the panel's C columns.
__device__ void rebuild_stream(const ExecArgs& a, const Stack& st, const ColDesc* desc, int K, int m, const double* T,
                               int kk, RV out,
                               double* buf, int cap_rows) {
  const int tid = threadIdx.x;
  const int ld = cap_rows | 1;
  for (int r0 = 0; r0 < m; r0 += cap_rows) {
    const int rows = min(cap_rows, m - r0);
    // every chunk in batches of sixteen loads per thread over all columns
    stage_desc(desc, K, r0, rows, buf, ld);
    __syncthreads();
    mfma_lds_gemm<double>(rows, kk, K, buf, ld, T, K, [&](int i, int c, double v) { vst(a, out, r0 + i, c, v); });
    __syncthreads();
  }
}

// Debug note of a truncation for the per-task trace (thread 0, LDS flag
// words 12..14): route (1 small-rank, 2 dense with QR, 3 Gram with QR,
// 4 dense with a full SVD, 5 Gram with a full SVD), SVD operand p x q,
// sweeps, rank.
__device__ __forceinline__ void trunc_note(char* lds, int route, int p, int q, int sweeps, int kk) {
  if (threadIdx.x == 0) {
    int* s_int = (int*)(lds + kLdsBytes - 64);
    s_int[12] = route;
    s_int[13] = (p & 0xffff) | (q << 16);
    s_int[14] = (sweeps & 0xffff) | (kk << 16);
  }
}

__device__ int trunc_core_small(const ExecArgs& a, const LrDesc& d, int lr_index, const Stack& su, const Stack& sv,
                                char* lds, double eps) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const int K = su.kc + su.kp + su.kp2;
  const int m = su.m, n = sv.m;
  int* s_int = (int*)(lds + kLdsBytes - 64);
  uint64_t tph = tid == 0 ? wall_clock64() : 0;
  if (a.counters && tid == 0) {
    wg_ctr(lds)[kCtrK] += K;
    wg_ctr(lds)[kCtrMN] += m + n;
  }
  // LDS: [G_U | G_V | B | Z | T_U | T_V] (K*K each), vectors at the end, the
  // Gram staging buffer over B..T_V and beyond
  double* GU = (double*)lds;
  double* GV = GU + K * K;
  double* B = GV + K * K;
  double* Z = B + K * K;
  double* TU = Z + K * K;
  double* TV = TU + K * K;
  char* vend = lds + kLdsBytes - 64;
  double* dU = (double*)(vend - 4 * kSmallK * 8 - 6 * kSmallK * 4);
  double* dV = dU + kSmallK;
  double* sig = dV + kSmallK;
  double* qa = sig + kSmallK;
  int* pU = (int*)(qa + kSmallK);
  int* pV = pU + kSmallK;
  int* sel = pV + kSmallK;
  int* posU = sel + kSmallK;
  int* posV = posU + kSmallK;
  int* qpos = posV + kSmallK;
  // column descriptors of the two stacks, below the vectors
  ColDesc* descU = (ColDesc*)dU - 2 * kSmallK;
  ColDesc* descV = descU + kSmallK;
  stack_descs(a, su, K, descU, 0);
  stack_descs(a, sv, K, descV, 64);
  __syncthreads();
  double* buf = B;
  const int cap_rows = (int)(((char*)descU - (char*)buf) / 8 / K) - 1;
  // 1. Gram matrices
  gram_stream(a, su, descU, K, m, GU, buf, cap_rows);
  gram_stream(a, sv, descV, K, n, GV, buf, cap_rows);
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 0, &tph);
  // 2. R factors: wavefront 0 factors G_U, wavefront 1 factors G_V
  if (wave == 0) {
    int r = pivoted_cholesky_wave(GU, K, pU, dU);
    if ((tid & 63) == 0) s_int[0] = r;
  } else if (wave == 1) {
    int r = pivoted_cholesky_wave(GV, K, pV, dV);
    if ((tid & 63) == 0) s_int[1] = r;
  }
  __syncthreads();
  const int rU = s_int[0], rV = s_int[1];
  phase_tick(a, lds, kCtrPhase + 1, &tph);
  if (rU == 0 || rV == 0) {
    if (tid == 0) a.ranks[lr_index] = 0;
    __syncthreads();
    return 0;
  }
  for (int q = tid; q < K; q += blockDim.x) {
    posU[pU[q]] = q;
    posV[pV[q]] = q;
  }
  for (int e = tid; e < rU * K; e += blockDim.x)
    if (e % K < e / K) GU[e] = 0.0;
  for (int e = tid; e < rV * K; e += blockDim.x)
    if (e % K < e / K) GV[e] = 0.0;
  for (int l = tid; l < K; l += blockDim.x) sig[l] = (dU[l] == 0.0 || dV[l] == 0.0) ? 0.0 : 1.0 / (dU[l] * dV[l]);
  __syncthreads();
  // 3. core B = Rt_U Rt_V^T (as in trunc_core)
  for (int e = tid; e < rU * rV; e += blockDim.x) {
    const int i = e % rU, j = e / rU;
    const double* ru = GU + i * K;
    const double* rv = GV + j * K;
    double s = 0.0;
    for (int l = 0; l < K; ++l) s += ru[posU[l]] * rv[posV[l]] * sig[l];
    B[j * rU + i] = s;
  }
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 2, &tph);
  // 4. SVD of the core B (p = rU rows, q = rV columns) by wavefront 0:
  //    Householder QR with column pivoting, stopped once the trailing columns
  //    fall below 0.1 eps of the largest column (so B = Q R + E with
  //    ||E||_F <= 0.1 eps sigma_1), then one-sided Jacobi on R^T (q x r):
  //    R^T Z = W Sigma gives the right singular vectors W of B, and B W the
  //    left ones times Sigma.  B itself is kept in Z's place for that product.
  const int qq = rV;
  if (wave == 0) {
    const int lane = tid & 63;
    const int pp = rU, rmax = min(pp, qq);
    double* cn = sig;  // squared norms of the trailing columns
    for (int e = lane; e < pp * qq; e += 64) Z[e] = B[e];
    if (lane < qq) {
      double acc = 0.0;
      for (int i = 0; i < pp; ++i) acc += B[lane * pp + i] * B[lane * pp + i];
      cn[lane] = acc;
      qpos[lane] = kSmallK;
    }
    wave_sync();
    double mx = lane < qq ? cn[lane] : 0.0;
    int mi = lane;
    wave_argmax(mx, mi);
    const double tol2 = 0.01 * eps * eps * mx;
    int r = 0;
    for (int st = 0;; ++st) {
      double best = (lane < qq && qpos[lane] == kSmallK) ? cn[lane] : -1.0;
      double sum = group_sum(best > 0.0 ? best : 0.0, 64);
      int bi = lane < qq ? lane : qq;
      wave_argmax(best, bi);
      if (st == rmax || bi >= qq || sum <= tol2 || !(best > 0.0)) {
        r = st;
        break;
      }
      double* xp = B + bi * pp;
      const double xi = (lane >= st && lane < pp) ? xp[lane] : 0.0;
      const double nrm2 = group_sum(xi * xi, 64);
      const double x0 = xp[st];
      const double nr = sqrt(nrm2);
      const double al = x0 >= 0.0 ? -nr : nr;
      const double v0 = x0 - al;
      const double vtv = nrm2 - x0 * x0 + v0 * v0;
      const double be = vtv > 0.0 ? 2.0 / vtv : 0.0;
      wave_sync();
      if (lane == 0) {
        xp[st] = v0;
        qa[st] = al;
        qpos[bi] = st;
      }
      wave_sync();
      if (lane < qq && qpos[lane] == kSmallK) {
        double* xj = B + lane * pp;
        // rows in batches of eight, every load of a batch issued before its
        // arithmetic (same order of accumulation as a plain loop)
        double w = 0.0;
        int i = st;
        for (; i + 8 <= pp; i += 8) {
          double xv[8], pv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            xv[k] = xj[i + k];
            pv[k] = xp[i + k];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) w += pv[k] * xv[k];
        }
        for (; i < pp; ++i) w += xp[i] * xj[i];
        const double f = be * w;
        double nn = 0.0;
        i = st;
        for (; i + 8 <= pp; i += 8) {
          double xv[8], pv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            xv[k] = xj[i + k];
            pv[k] = xp[i + k];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const double y = xv[k] - f * pv[k];
            xj[i + k] = y;
            if (i + k > st) nn += y * y;
          }
        }
        for (; i < pp; ++i) {
          const double y = xj[i] - f * xp[i];
          xj[i] = y;
          if (i > st) nn += y * y;
        }
        cn[lane] = nn;
      }
      wave_sync();
    }
    // R^T (q x r; column s is row s of R) in TU; its rotations are not kept (only R^T Z is used)
    for (int e = lane; e < qq * r; e += 64) {
      const int j = e % qq, s2 = e / qq, pj = qpos[j];
      TU[e] = pj == s2 ? qa[s2] : (pj > s2 ? B[j * pp + s2] : 0.0);
    }
    wave_sync();
    const int sw = r > 0 ? jacobi_svd_wave(TU, nullptr, qq, r, eps) : 0;
    if (lane == 0) s_int[3] = r;
    trunc_note(lds, 1, qq, r, sw, 0);
  }
  __syncthreads();
  const int rr = s_int[3];
  phase_tick(a, lds, kCtrPhase + 3, &tph);
  // 5. order, truncation rank (singular values: column norms of R^T Z)
  for (int j = tid; j < rr; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < qq; ++r) s += TU[j * qq + r] * TU[j * qq + r];
    sig[j] = sqrt(s);
  }
  if (tid == 0) s_int[2] = 0;
  __syncthreads();
  double smax = 0.0;
  for (int j = 0; j < rr; ++j) smax = fmax(smax, sig[j]);
  for (int j = tid; j < rr; j += blockDim.x) {
    int rk = 0;
    for (int l = 0; l < rr; ++l)
      if (sig[l] > sig[j] || (sig[l] == sig[j] && l < j)) ++rk;
    sel[rk] = j;
    if (smax > 0.0 && sig[j] > eps * smax) atomicAdd(&s_int[2], 1);
  }
  __syncthreads();
  int kk = s_int[2];
  const int limit = min(d.cap, min(d.m, d.n));
  if (kk > limit) {
    if (tid == 0) atomicAdd(&a.status[2], 1);  // the capacity or the cap bound
    kk = limit;
  }
  if (kk == 0) {
    if (tid == 0) a.ranks[lr_index] = 0;
    __syncthreads();
    return 0;
  }
  // 6. T_U = D_U P_U E_r R'_U^{-1} (B Z)_sel, T_V = D_V P_V E_r R'_V^{-1} Z_sel;
  //    the selected columns are solved in T_U / T_V's space, then scattered
  //    into rows by permutation and scale in place of B / Z
  double* yu = TU;
  double* yv = TV;
  {
    double* vc = B;  // right singular vectors (rV x kk), unit columns
    for (int e = tid; e < rV * kk; e += blockDim.x) {
      const int i = e % rV, c = e / rV, j = sel[c];
      vc[e] = TU[j * qq + i] / sig[j];
    }
    __syncthreads();
    for (int e = tid; e < rU * kk; e += blockDim.x) {  // B V (rU x kk), B kept in Z
      const int i = e % rU, c = e / rU;
      double acc = 0.0;
      for (int j = 0; j < rV; ++j) acc += Z[j * rU + i] * vc[c * rV + j];
      yu[e] = acc;
    }
    for (int e = tid; e < rV * kk; e += blockDim.x) yv[e] = vc[e];
  }
  __syncthreads();
  // both triangles at once: the first half of the workgroup solves with R_U,
  // the second with R_V
  if (tid < 128)
    upper_solve(GU, K, rU, yu, kk, tid, 128);
  else
    upper_solve(GV, K, rV, yv, kk, tid - 128, 128);
  __syncthreads();
  double* T_U = B;  // K x kk <= K x K
  double* T_V = Z;
  for (int e = tid; e < K * kk; e += blockDim.x) {
    int l = e % K, c = e / K;
    int qu = posU[l], qv = posV[l];
    T_U[c * K + l] = qu < rU ? dU[l] * yu[c * rU + qu] : 0.0;
    T_V[c * K + l] = qv < rV ? dV[l] * yv[c * rV + qv] : 0.0;
  }
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 4, &tph);
  // 7. rebuild in place (staging buffer after T_U / T_V in the B / Z region)
  {
    double* rbuf = Z + K * K;
    const int rcap = (int)(((char*)descU - (char*)rbuf) / 8 / K) - 1;
    rebuild_stream(a, su, descU, K, m, T_U, kk, RV{d.u_off, m, kk, 1, m, d.type}, rbuf, rcap);
    rebuild_stream(a, sv, descV, K, n, T_V, kk, RV{d.v_off, n, kk, 1, n, d.type}, rbuf, rcap);
  }
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 5, &tph);
  if (tid == 0) a.ranks[lr_index] = kk;
  __syncthreads();
  return kk;
}

// ---------------------------------------------------------------------------
// Truncation with K > kSmallK stacked columns.  LDS: a work area from offset 0
// (GEMM tiles, Gram matrices, the SVD operand and its rotations, a triangle),
// then the per-column vectors, then 64 bytes of flags.
// ---------------------------------------------------------------------------
constexpr int kLargeVecBytes = 7 * kMaxK * 8 + 7 * kMaxK * 4;
constexpr int kLargeWork = (kLdsBytes - 64 - kLargeVecBytes) / 8;  // doubles
constexpr int kTileDoubles = kTileBytes / 8;

struct LargeVecs {
  double *dU, *dV, *eU, *eV, *sig, *qa, *qb;
  int *pU, *pV, *sel, *posU, *posV, *qpos, *qpiv;
};

__device__ LargeVecs large_vecs(char* lds) {
  LargeVecs v;
  double* p = (double*)(lds + kLdsBytes - 64 - kLargeVecBytes);
  v.dU = p;
  v.dV = p + kMaxK;
  v.eU = p + 2 * kMaxK;
  v.eV = p + 3 * kMaxK;
  v.sig = p + 4 * kMaxK;
  v.qa = p + 5 * kMaxK;
  v.qb = p + 6 * kMaxK;
  int* ip = (int*)(p + 7 * kMaxK);
  v.pU = ip;
  v.pV = ip + kMaxK;
  v.sel = ip + 2 * kMaxK;
  v.posU = ip + 3 * kMaxK;
  v.posV = ip + 4 * kMaxK;
  v.qpos = ip + 5 * kMaxK;
  v.qpiv = ip + 6 * kMaxK;
  return v;
}

// Scaled, diagonally pivoted Cholesky of two Gram matrices (K x K, row-major,
// K <= kMaxK), one per half of the workgroup, in left-looking order: step s
// takes the largest remaining diagonal entry of the scaled Schur complement
// (e[]: 1 at the start, -1 once pivoted) and forms row s of the factor from
// that pivot's row of G and the rows found before.  Row s of the factor, in
// the original column order and zero at earlier pivots, overwrites row
// perm[s] of G.  dsc[l] = 1/||column l|| (0 for a zero column).  The ranks go
// to s_int[0] (G_U) and s_int[1] (G_V).
__device__ void pivoted_cholesky_pair(double* GU, double* GV, int K, const LargeVecs& v, int* s_int) {
  const int tid = threadIdx.x, h = tid >> 7, t = tid & 127;
  double* G = h ? GV : GU;
  double* e = h ? v.eV : v.eU;
  double* dsc = h ? v.dV : v.dU;
  int* perm = h ? v.pV : v.pU;
  int* slot = s_int + 4 + 4 * h;  // [0] pivot, [1] go, [2..3] the pivot's Schur entry (double)
  const double tol = 8.0 * K * 2.220446049250313e-16;
  if (t < K) {
    const double g = G[t * K + t];
    dsc[t] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
    e[t] = g > 0.0 ? 1.0 : 0.0;
  }
  if (t == 0) slot[1] = 1;
  __syncthreads();
  int r = 0;
  for (int s = 0; s < K; ++s) {
    if (slot[1] && t < 64) {
      double best = -1.0;
      int bi = K;
      for (int l = t; l < K; l += 64) {
        const double x = e[l];
        if (x > best) {
          best = x;
          bi = l;
        }
      }
      wave_argmax(best, bi);
      if (t == 0) {
        const bool go = bi < K && best > tol;
        slot[0] = bi;
        slot[1] = go ? 1 : 0;
        *(double*)(slot + 2) = best;
        if (go) perm[s] = bi;
      }
    }
    __syncthreads();
    if (!s_int[5] && !s_int[9]) break;
    if (slot[1]) {
      r = s + 1;
      const int p = slot[0];
      const double piv = sqrt(*(const double*)(slot + 2));
      if (t < K) {
        const double et = e[t];
        double val = 0.0;
        if (t == p) {
          val = piv;
        } else if (et >= 0.0) {
          double x = G[p * K + t] * dsc[p] * dsc[t];
          // the earlier rows in batches of eight, every load of a batch
          // issued before its products (same order of subtraction)
          int u = 0;
          for (; u + 8 <= s; u += 8) {
            int pr[8];
            double xa[8], xb[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) pr[k] = perm[u + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const double* ru = G + (int64_t)pr[k] * K;
              xa[k] = ru[p];
              xb[k] = ru[t];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) x -= xa[k] * xb[k];
          }
          for (; u < s; ++u) {
            const double* ru = G + (int64_t)perm[u] * K;
            x -= ru[p] * ru[t];
          }
          val = x / piv;
        }
        G[p * K + t] = val;
        e[t] = t == p ? -1.0 : (et >= 0.0 ? et - val * val : et);
      }
    }
    __syncthreads();
  }
  if (t == 0) s_int[h] = r;
  __syncthreads();
}

// Back substitution y <- R^{-1} y with the r x r upper triangle R(i, j) =
// F[perm[i] * K + perm[j]] of a factor from pivoted_cholesky_pair (copied to
// LDS, column-major, when r * r <= buf_cap), for kk <= kMaxCap right-hand
// sides Y (r x kk, column-major).  Each column is held in registers by a group
// of tpc lanes of one wavefront (row j in lane j % tpc), so no workgroup
// barrier is needed between the steps; groups of columns are taken in passes.
// The solution rows are scattered into T (K x kk, column-major):
// T[perm[j]][c] = dsc[perm[j]] y[j][c]; rows of non-pivot columns are zero.
template <int NR>
__device__ void tri_solve_rows(const double* R, int ldr, bool lds_tri, const double* F, int K, int r,
                               const int* perm, const double* Y, int c, int kk, int tpc, double* T,
                               const double* dsc) {
  const int t = threadIdx.x % tpc;
  const bool on = c < kk;
  double x[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int j = t + k * tpc;
    x[k] = (on && j < r) ? Y[c * r + j] : 0.0;
  }
  for (int i = r - 1; i >= 0; --i) {
    const int owner = i % tpc, sl = i / tpc;
    double xi = 0.0;
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (k == sl) xi = x[k];
    xi = __shfl(xi, owner, tpc);
    const double yi = xi / (lds_tri ? R[i * ldr + i] : F[(int64_t)perm[i] * K + perm[i]]);
    const int pi = perm[i];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int j = t + k * tpc;
      if (k == sl && t == owner)
        x[k] = yi;
      else if (j < i)
        x[k] -= (lds_tri ? R[i * ldr + j] : F[(int64_t)perm[j] * K + pi]) * yi;
    }
  }
  if (on) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int j = t + k * tpc;
      if (j < r) {
        const int l = perm[j];
        T[c * K + l] = dsc[l] * x[k];
      }
    }
  }
}

__device__ void tri_solve_scatter(const double* F, int K, int r, const int* perm, const int* pos, const double* Y,
                                  int kk, double* T, const double* dsc, double* buf, int buf_cap) {
  const int tid = threadIdx.x;
  const bool lds_tri = r * r <= buf_cap;
  if (lds_tri)
    for (int e = tid; e < r * r; e += blockDim.x) {
      const int i = e % r, j = e / r;  // column-major: buf[j * r + i] = R(i, j)
      buf[e] = i <= j ? F[(int64_t)perm[i] * K + perm[j]] : 0.0;
    }
  for (int e = tid; e < K * kk; e += blockDim.x)
    if (pos[e % K] >= r) T[e] = 0.0;
  __syncthreads();
  // lanes per column: enough that each holds at most 8 rows, more when few
  // columns leave lanes idle
  int tpc = 1;
  while (tpc * 8 < r) tpc *= 2;
  while (tpc < 64 && tpc * 2 * kk <= (int)blockDim.x) tpc *= 2;
  const int per_pass = blockDim.x / tpc;
  for (int c0 = 0; c0 < kk; c0 += per_pass) {
    const int c = c0 + tid / tpc;
    if ((r + tpc - 1) / tpc <= 4)
      tri_solve_rows<4>(buf, r, lds_tri, F, K, r, perm, Y, c, kk, tpc, T, dsc);
    else
      tri_solve_rows<8>(buf, r, lds_tri, F, K, r, perm, Y, c, kk, tpc, T, dsc);
  }
  __syncthreads();
}

// Column norms of the rotated operand (p x q) give the singular values; the
// selection sel[] lists the columns by decreasing value; returns the kept
// count (sigma > eps sigma_1, then capped at the leaf's capacity).
__device__ int select_kept(const ExecArgs& a, const LrDesc& d, const double* Bp, int p, int q, double* sig, int* sel,
                           int* s_int, double eps) {
  const int tid = threadIdx.x;
  for (int j = tid; j < q; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < p; ++r) s += Bp[j * p + r] * Bp[j * p + r];
    sig[j] = sqrt(s);
  }
  if (tid == 0) s_int[2] = 0;
  __syncthreads();
  double smax = 0.0;
  for (int j = 0; j < q; ++j) smax = fmax(smax, sig[j]);
  for (int j = tid; j < q; j += blockDim.x) {
    int rk = 0;
    for (int l = 0; l < q; ++l)
      if (sig[l] > sig[j] || (sig[l] == sig[j] && l < j)) ++rk;
    sel[rk] = j;
    if (smax > 0.0 && sig[j] > eps * smax) atomicAdd(&s_int[2], 1);
  }
  __syncthreads();
  int kk = s_int[2];
  const int limit = min(d.cap, min(d.m, d.n));
  if (kk > limit) {
    if (tid == 0) atomicAdd(&a.status[2], 1);  // the capacity or the cap bound
    kk = limit;
  }
  return kk;
}

__device__ int set_rank(const ExecArgs& a, int lr_index, int kk) {
  if (threadIdx.x == 0) a.ranks[lr_index] = kk;
  __syncthreads();
  return kk;
}

// Truncated SVD of an operand B' (p x q, column-major, read-only in global
// memory, q <= kMaxK) through Householder QR with column pivoting stopped
// early: after r steps the trailing columns have Frobenius norm at most
// 0.1 eps times the largest column norm (<= 0.1 eps sigma_1), so B' = Q R + E
// with R r x q (upper triangular up to the column order).  One-sided Jacobi on
// R^T (q x r) then gives R^T Z = W Sigma: the right singular vectors of B' are
// the columns of W, the left ones times Sigma are B' W.  On return Vc (q x kk,
// column-major, global) holds the kept columns of W by decreasing singular
// value; the caller forms B' Vc.  Returns kk, or -1 when r would exceed the
// room left in LDS (the caller then diagonalises B' in full).  gwork (p * q
// doubles of global scratch) holds the work copy when it does not fit in LDS.
__device__ int qr_svd(const ExecArgs& a, const LrDesc& d, const double* Bg, int p, int q, double* Vc, char* lds,
                      double* gwork, const LargeVecs& v, double eps, int* sweeps) {
  const int tid = threadIdx.x;
  int* s_int = (int*)(lds + kLdsBytes - 64);
  double* W = (double*)lds;
  const int rmax = min(p, q);
  constexpr int kReserve = 40;
  const int rres = min(rmax, kReserve);
  const bool x_lds = (int64_t)p * q + (int64_t)q * rres + rres * rres <= kLargeWork;
  double* X = x_lds ? W : gwork;
  double* rest = x_lds ? W + p * q : W;
  const int room = kLargeWork - (x_lds ? p * q : 0);
  int rl = 0;
  while (rl < rmax && q * (rl + 1) + (rl + 1) * (rl + 1) <= room) ++rl;
  copy_batched(X, Bg, p * q);
  __syncthreads();
  // lanes per column: the largest power of two with tpc * q <= 256 (<= 64)
  int tpc = 1;
  while (tpc < 64 && tpc * 2 * q <= (int)blockDim.x) tpc *= 2;
  const int g = tid / tpc, lt = tid % tpc;
  double* cn = v.eU;  // squared norms of the trailing columns
  if (g < q) {
    double acc = 0.0;
    for (int i = lt; i < p; i += tpc) acc += X[g * p + i] * X[g * p + i];
    acc = group_sum(acc, tpc);
    if (lt == 0) {
      cn[g] = acc;
      v.qpos[g] = kMaxK;
    }
  }
  __syncthreads();
  // tolerance from the largest column norm
  if (tid < 64) {
    double mx = 0.0;
    for (int j = tid; j < q; j += 64) mx = fmax(mx, cn[j]);
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (tid == 0) *(double*)(s_int + 4) = 0.01 * eps * eps * mx;
  }
  __syncthreads();
  const double tol2 = *(const double*)(s_int + 4);
  int r = 0;
  for (int st = 0;; ++st) {
    // (a) pivot: the largest trailing column; stop once the trailing block is small
    if (tid < 64) {
      double best = -1.0, sum = 0.0;
      int bi = q;
      for (int j = tid; j < q; j += 64)
        if (v.qpos[j] == kMaxK) {
          const double x = cn[j];
          sum += x;
          if (x > best) {
            best = x;
            bi = j;
          }
        }
      sum = group_sum(sum, 64);
      wave_argmax(best, bi);
      if (tid == 0) {
        int code = 1;                                   // go on
        if (st == rmax || bi >= q || sum <= tol2 || !(best > 0.0)) code = 0;  // done
        else if (st == rl) code = 2;                    // no room for another step
        s_int[8] = code;
        s_int[9] = bi;
        if (code == 1) {
          v.qpos[bi] = st;
          v.qpiv[st] = bi;
        }
      }
    }
    __syncthreads();
    const int code = s_int[8];
    if (code == 2) return -1;
    if (code == 0) {
      r = st;
      break;
    }
    const int jp = s_int[9];
    double* xp = X + jp * p;
    // (b) Householder vector of the pivot column (rows st..p-1), in place
    if (tid < 64) {
      double nrm2 = 0.0;
      for (int i = st + tid; i < p; i += 64) nrm2 += xp[i] * xp[i];
      nrm2 = group_sum(nrm2, 64);
      if (tid == 0) {
        const double x0 = xp[st];
        const double nr = sqrt(nrm2);
        const double al = x0 >= 0.0 ? -nr : nr;
        const double v0 = x0 - al;
        const double vtv = nrm2 - x0 * x0 + v0 * v0;
        xp[st] = v0;
        v.qa[st] = al;
        v.qb[st] = vtv > 0.0 ? 2.0 / vtv : 0.0;
      }
    }
    __syncthreads();
    // (c) apply to every trailing column and refresh its norm below row st
    const double be = v.qb[st];
    if (g < q && v.qpos[g] == kMaxK) {
      double* xj = X + g * p;
      double w = 0.0;
      for (int i = st + lt; i < p; i += tpc) w += xp[i] * xj[i];
      w = group_sum(w, tpc);
      const double f = be * w;
      double nn = 0.0;
      for (int i = st + lt; i < p; i += tpc) {
        const double y = xj[i] - f * xp[i];
        xj[i] = y;
        if (i > st) nn += y * y;
      }
      nn = group_sum(nn, tpc);
      if (lt == 0) cn[g] = nn;
    }
    __syncthreads();
  }
  if (r == 0) {
    *sweeps = 0;
    return 0;
  }
  // R^T (q x r, column-major: column s is row s of R); only R^T Z is used
  double* Rt = rest;
  for (int e = tid; e < q * r; e += blockDim.x) {
    const int j = e % q, s2 = e / q;
    const int pj = v.qpos[j];
    Rt[e] = pj == s2 ? v.qa[s2] : (pj > s2 ? X[j * p + s2] : 0.0);
  }
  __syncthreads();
  *sweeps = jacobi_svd(Rt, nullptr, q, r, s_int, eps);
  const int kk = select_kept(a, d, Rt, q, r, v.sig, v.sel, s_int, eps);
  for (int e = tid; e < q * kk; e += blockDim.x) {
    const int j = e % q, c = e / q, sc = v.sel[c];
    Vc[e] = Rt[sc * q + j] / v.sig[sc];
  }
  __syncthreads();
  return kk;
}

// Dense route for a small leaf (p q <= kMaxK^2 with p = max(m, n), q =
// min(m, n)): M = U_s V_s^T is formed explicitly (as M' = M, or M^T when
// n > m, so that M' has q columns) and truncated by qr_svd: the q-side factor
// is V_c, the p-side factor M' V_c carries the singular values.  When the
// QR route lacks room, M' is diagonalised by one-sided Jacobi in full
// (M' Z = W Sigma; p side (M' Z)_sel, q side Z_sel).
__device__ int trunc_dense(const ExecArgs& a, const LrDesc& d, int lr_index, const Stack& su, const Stack& sv,
                           char* lds, double* scratch, double eps, uint64_t* tph) {
  const int tid = threadIdx.x;
  const int K = su.kc + su.kp + su.kp2;
  const int m = su.m, n = sv.m;
  const bool tr = n > m;
  const int p = tr ? n : m, q = tr ? m : n;
  int* s_int = (int*)(lds + kLdsBytes - 64);
  const LargeVecs v = large_vecs(lds);
  TruncScratch S = trunc_scratch(scratch);
  double* sA = (double*)lds;
  double* sB = sA + TK * (TM + TP);
  double* Mg = S.GU;  // p x q <= kMaxK^2
  // 1. M' (p x q, column-major) = X Y^T with (X, Y) = (U_s, V_s) or (V_s, U_s)
  if (!tr)
    gemm_tiles<double>(
        m, n, K, [&](int i, int l) { return su(a, i, l); }, [&](int l, int j) { return sv(a, j, l); },
        [&](int i, int j, double x) { Mg[j * p + i] = x; }, false, false, sA, sB);
  else
    gemm_tiles<double>(
        n, m, K, [&](int i, int l) { return sv(a, i, l); }, [&](int l, int j) { return su(a, j, l); },
        [&](int i, int j, double x) { Mg[j * p + i] = x; }, false, false, sA, sB);
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 6, tph);
  RV uc{d.u_off, m, 0, 1, m, d.type};
  RV vc{d.v_off, n, 0, 1, n, d.type};
  // 2. QR-preconditioned SVD
  int sw = 0;
  double* Vq = S.YV;  // q x kk
  const int kq = qr_svd(a, d, Mg, p, q, Vq, lds, S.B, v, eps, &sw);
  phase_tick(a, lds, kCtrPhase + 9, tph);
  if (kq >= 0) {
    trunc_note(lds, 2, p, q, sw, kq);
    if (kq == 0) return set_rank(a, lr_index, 0);
    uc.cols = vc.cols = kq;
    const RV qv = tr ? uc : vc, pv = tr ? vc : uc;
    for (int e = tid; e < q * kq; e += blockDim.x) vst(a, qv, e % q, e / q, Vq[e]);
    gemm_tiles<double>(
        p, kq, q, [&](int i, int j) { return Mg[j * p + i]; }, [&](int j, int c) { return Vq[c * q + j]; },
        [&](int i, int c, double x) { vst(a, pv, i, c, x); }, false, true, sA, sB);
    __syncthreads();
    phase_tick(a, lds, kCtrPhase + 11, tph);
    return set_rank(a, lr_index, kq);
  }
  // 3. fallback: one-sided Jacobi on all of M'
  double* Mp = Mg;
  double* Z = S.Z;
  if ((int64_t)p * q + (int64_t)q * q <= kLargeWork) {
    Mp = (double*)lds;
    Z = Mp + p * q;
    copy_batched(Mp, Mg, p * q);
    __syncthreads();
  }
  sw = jacobi_svd(Mp, Z, p, q, s_int, eps);
  phase_tick(a, lds, kCtrPhase + 9, tph);
  const int kk = select_kept(a, d, Mp, p, q, v.sig, v.sel, s_int, eps);
  trunc_note(lds, 4, p, q, sw, kk);
  if (kk == 0) return set_rank(a, lr_index, 0);
  uc.cols = vc.cols = kk;
  for (int e = tid; e < m * kk; e += blockDim.x) {
    const int i = e % m, c = e / m;
    const int j = v.sel[c];
    vst(a, uc, i, c, tr ? Z[j * q + i] : Mp[j * p + i]);
  }
  for (int e = tid; e < n * kk; e += blockDim.x) {
    const int i = e % n, c = e / n;
    const int j = v.sel[c];
    vst(a, vc, i, c, tr ? Mp[j * p + i] : Z[j * q + i]);
  }
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 11, tph);
  return set_rank(a, lr_index, kk);
}

// Gram route: R factors of U_s and V_s from their Gram matrices (pivoted
// Cholesky), the core B = Rt_U W Rt_V^T (rU x rV, W = diag(||u_l|| ||v_l||)),
// oriented as B' = B or B^T so that B' has q = min(rU, rV) columns and
// truncated by qr_svd (or, without room, by one-sided Jacobi on all of B'),
// then U <- U_s D_U P_U R_U11^{-1} Y_U,  V <- V_s D_V P_V R_V11^{-1} Y_V
// with Y the core's kept singular vectors (the side that carries Sigma is
// the p side of B').
__device__ int trunc_gram(const ExecArgs& a, const LrDesc& d, int lr_index, const Stack& su, const Stack& sv,
                          char* lds, double* scratch, double eps, uint64_t* tph) {
  const int tid = threadIdx.x;
  const int K = su.kc + su.kp + su.kp2;
  const int m = su.m, n = sv.m;
  int* s_int = (int*)(lds + kLdsBytes - 64);
  const LargeVecs v = large_vecs(lds);
  TruncScratch S = trunc_scratch(scratch);
  double* sA = (double*)lds;
  double* sB = sA + TK * (TM + TP);
  double* W = (double*)lds;
  // 1. Gram matrices.  K <= 64: on the matrix cores from LDS-staged rows,
  //    the column descriptors parked in the per-column vectors (not in use
  //    before the Cholesky), G_U then G_V in the work area, each staged
  //    through the space after it.  Otherwise by the tiled GEMM, in LDS
  //    after the GEMM tiles when both fit.
  const bool g_mfma = K <= 64;
  const bool g_lds = !g_mfma && kTileDoubles + 2 * K * K <= kLargeWork;
  double* GU = g_mfma ? W : g_lds ? W + kTileDoubles : S.GU;
  double* GV = g_mfma ? W + K * K : g_lds ? GU + K * K : S.GV;
  if (g_mfma) {
    static_assert(2 * 64 * sizeof(ColDesc) <= kLargeVecBytes, "descriptors fit the vector area");
    static_assert(2 * 64 * 64 <= kLargeWork && 64 * 64 + 2 * 64 * 2 <= kLargeWork, "G_U, G_V and a chunk fit");
    ColDesc* du = (ColDesc*)v.dU;
    stack_descs(a, su, K, du, 0);
    stack_descs(a, sv, K, du + K, 64);
    __syncthreads();
    gram_tiles(du, K, m, GU, W, kLargeWork);
    gram_tiles(du + K, K, n, GV, W + K * K, kLargeWork - K * K);
  } else {
    gemm_tiles<double>(
        K, K, m, [&](int i, int r) { return su(a, r, i); }, [&](int r, int j) { return su(a, r, j); },
        [&](int i, int j, double x) { GU[i * K + j] = x; }, true, true, sA, sB);
    gemm_tiles<double>(
        K, K, n, [&](int i, int r) { return sv(a, r, i); }, [&](int r, int j) { return sv(a, r, j); },
        [&](int i, int j, double x) { GV[i * K + j] = x; }, true, true, sA, sB);
  }
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 6, tph);
  // 2. R factors, in LDS whenever both Gram matrices fit there (the GEMM tiles
  //    are free now): the left-looking steps then read earlier rows from LDS
  //    instead of global scratch
  if (!g_mfma && !g_lds && 2 * K * K <= kLargeWork) {
    double* LU = W;
    double* LV = W + K * K;
    copy_batched(LU, S.GU, K * K);
    copy_batched(LV, S.GV, K * K);
    __syncthreads();
    GU = LU;
    GV = LV;
  }
  pivoted_cholesky_pair(GU, GV, K, v, s_int);
  const int rU = s_int[0], rV = s_int[1];
  if (GU != S.GU) {  // the factors move to global scratch to free the work area
    for (int e = tid; e < K * K; e += blockDim.x) {
      S.GU[e] = GU[e];
      S.GV[e] = GV[e];
    }
    GU = S.GU;
    GV = S.GV;
  }
  for (int l = tid; l < K; l += blockDim.x) {
    v.posU[l] = K;
    v.posV[l] = K;
  }
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 7, tph);
  if (rU == 0 || rV == 0) return set_rank(a, lr_index, 0);
  for (int j = tid; j < rU; j += blockDim.x) v.posU[v.pU[j]] = j;
  for (int j = tid; j < rV; j += blockDim.x) v.posV[v.pV[j]] = j;
  for (int l = tid; l < K; l += blockDim.x)
    v.sig[l] = (v.dU[l] == 0.0 || v.dV[l] == 0.0) ? 0.0 : 1.0 / (v.dU[l] * v.dV[l]);
  __syncthreads();
  // 3. core B' (p x q, column-major, global)
  const bool tr = rV > rU;
  const int p = tr ? rV : rU, q = tr ? rU : rV;
  double* Bg = S.B;
  gemm_tiles<double>(
      rU, rV, K, [&](int i, int l) { return GU[(int64_t)v.pU[i] * K + l] * v.sig[l]; },
      [&](int l, int j) { return GV[(int64_t)v.pV[j] * K + l]; },
      [&](int i, int j, double x) {
        if (tr)
          Bg[i * p + j] = x;
        else
          Bg[j * p + i] = x;
      },
      true, true, sA, sB);
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 8, tph);
  // 4. SVD of the core; Y_q (q side) and Y_p (p side, with Sigma)
  double* Yq = tr ? S.YU : S.YV;
  double* Yp = tr ? S.YV : S.YU;
  int sw = 0;
  int kk = qr_svd(a, d, Bg, p, q, Yq, lds, S.Z, v, eps, &sw);
  if (kk >= 0) {
    trunc_note(lds, 3, p, q, sw, kk);
    phase_tick(a, lds, kCtrPhase + 9, tph);
    if (kk == 0) return set_rank(a, lr_index, 0);
    gemm_tiles<double>(
        p, kk, q, [&](int i, int j) { return Bg[j * p + i]; }, [&](int j, int c) { return Yq[c * q + j]; },
        [&](int i, int c, double x) { Yp[c * p + i] = x; }, false, true, sA, sB);
    __syncthreads();
  } else {
    double* Bp = Bg;
    double* Z = S.Z;
    if ((int64_t)p * q + (int64_t)q * q <= kLargeWork) {
      Bp = W;
      Z = W + p * q;
      copy_batched(Bp, Bg, p * q);
      __syncthreads();
    }
    sw = jacobi_svd(Bp, Z, p, q, s_int, eps);
    phase_tick(a, lds, kCtrPhase + 9, tph);
    kk = select_kept(a, d, Bp, p, q, v.sig, v.sel, s_int, eps);
    trunc_note(lds, 5, p, q, sw, kk);
    if (kk == 0) return set_rank(a, lr_index, 0);
    for (int e = tid; e < p * kk; e += blockDim.x) Yp[e] = Bp[v.sel[e / p] * p + e % p];
    for (int e = tid; e < q * kk; e += blockDim.x) Yq[e] = Z[v.sel[e / q] * q + e % q];
    __syncthreads();
  }
  // 5. T_U, T_V (K x kk) by back substitution with the pivoted triangles
  tri_solve_scatter(GU, K, rU, v.pU, v.posU, S.YU, kk, S.TU, v.dU, W, kLargeWork);
  tri_solve_scatter(GV, K, rV, v.pV, v.posV, S.YV, kk, S.TV, v.dV, W, kLargeWork);
  phase_tick(a, lds, kCtrPhase + 10, tph);
  // 6. rebuild in place: U <- U_s T_U, V <- V_s T_V (a single 64-column tile
  //    since kk <= 64, so every row tile is read completely before it is
  //    overwritten)
  RV uc{d.u_off, m, kk, 1, m, d.type};
  RV vc{d.v_off, n, kk, 1, n, d.type};
  gemm_tiles<double>(
      m, kk, K, [&](int r, int l) { return su(a, r, l); }, [&](int l, int c) { return S.TU[c * K + l]; },
      [&](int r, int c, double x) { vst(a, uc, r, c, x); }, false, true, sA, sB);
  gemm_tiles<double>(
      n, kk, K, [&](int r, int l) { return sv(a, r, l); }, [&](int l, int c) { return S.TV[c * K + l]; },
      [&](int r, int c, double x) { vst(a, vc, r, c, x); }, false, true, sA, sB);
  __syncthreads();
  phase_tick(a, lds, kCtrPhase + 11, tph);
  return set_rank(a, lr_index, kk);
}

// Returns the new rank.
__device__ __noinline__ int trunc_core(const ExecArgs& a, const LrDesc& d, int lr_index, const Stack& su, const Stack& sv,
                          char* lds, double* scratch, double eps) {
  const int tid = threadIdx.x;
  const int K = su.kc + su.kp + su.kp2;
  const int m = su.m, n = sv.m;
  trunc_note(lds, 0, 0, 0, 0, 0);
  if (K == 0) return set_rank(a, lr_index, 0);
  if (K <= kSmallK) return trunc_core_small(a, d, lr_index, su, sv, lds, eps);
  uint64_t tph = tid == 0 ? wall_clock64() : 0;
  if (a.counters && tid == 0) {
    wg_ctr(lds)[kCtrK] += K;
    wg_ctr(lds)[kCtrMN] += m + n;
  }
  const int p = max(m, n), q = min(m, n);
  if ((int64_t)p * q <= (int64_t)kMaxK * kMaxK && 4 * K >= 3 * q)
    return trunc_dense(a, d, lr_index, su, sv, lds, scratch, eps, &tph);
  return trunc_gram(a, d, lr_index, su, sv, lds, scratch, eps, &tph);
}

// OP_TRUNC:  C <- T(C + alpha pad(a) pad(b)^T)
// OP_TRUNC2: C <- T(alpha pad(a) pad(b)^T + beta pad(x) pad(y)^T)  (C's old content ignored)
__device__ void op_trunc(const ExecArgs& a, const Task& t, char* lds, double* scratch) {
  const LrDesc d = a.lr[t.lr];
  const bool two = t.op == OP_TRUNC2;
  const int kc = two ? 0 : a.ranks[t.lr];
  RV A = resolve(a, t.a), B = resolve(a, t.b);
  RV X{0, 0, 0, 1, 1, VT_NONE}, Y{0, 0, 0, 1, 1, VT_NONE};
  if (two) {
    X = resolve(a, t.x);
    Y = resolve(a, t.y);
  }
  Stack su, sv;
  su.c = RV{d.u_off, d.m, kc, 1, d.m, d.type};
  sv.c = RV{d.v_off, d.n, kc, 1, d.n, d.type};
  su.t = A;
  sv.t = B;
  su.t2 = X;
  sv.t2 = Y;
  su.tptr = sv.tptr = nullptr;
  su.m = d.m;
  sv.m = d.n;
  su.kc = sv.kc = kc;
  su.kp = sv.kp = A.cols;
  su.kp2 = sv.kp2 = two ? X.cols : 0;
  su.r0 = t.r0;
  sv.r0 = t.c0;
  su.r2 = t.row0;
  sv.r2 = t.c1;
  su.alpha = t.alpha;
  su.alpha2 = t.beta;
  sv.alpha = sv.alpha2 = 1.0;
  __syncthreads();
  const int kn = trunc_core(a, d, t.lr, su, sv, lds, scratch, two ? a.eps * kInnerEps : a.eps);
  if (threadIdx.x == 0 && a.counters) {
    int64_t s = d.type == VT_F64 ? 8 : 4;
    int64_t K = kc + A.cols + su.kp2;
    int64_t bytes = (int64_t)(d.m + d.n) * (kc + kn) * s + vbytes(A) + vbytes(B) + vbytes(X) + vbytes(Y);
    int64_t flops = 4 * (int64_t)(d.m + d.n) * K * K + 2 * (int64_t)(d.m + d.n) * K * kn + 20 * K * K * K;
    wg_ctr(lds)[0] += bytes;
    wg_ctr(lds)[1] += flops;
  }
}

// ---------------------------------------------------------------------------
// task dispatch
// ---------------------------------------------------------------------------
// Algorithmic bytes (every operand read once, every output written once, at
// run-time extents) and flops of one task; the truncation counts itself.
__device__ void count_task(const ExecArgs& a, const Task& t, char* lds) {
  if (!a.counters || t.op == OP_TRUNC || t.op == OP_TRUNC2 || t.op == OP_NOP) return;
  int64_t bytes = 0, flops = 0;
  if (t.op == OP_GETRF) {
    int64_t m = t.a.rows;
    bytes = 2 * m * m * 8;
    flops = 2 * m * m * m / 3;
  } else if (t.op == OP_TRSM_L || t.op == OP_TRSM_UT || t.op == OP_TRSM_U) {
    RV x = resolve(a, t.x);
    int64_t m = t.a.rows;
    bytes = m * m * 8 + 2 * vbytes(x);
    flops = (t.b.type == VT_F64 ? 2 : 1) * m * m * x.cols;
  } else if (t.op == OP_GEMM) {
    RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b);
    bytes = vbytes(A) + vbytes(B) + (t.beta != 0.0 ? 2 : 1) * vbytes(y);
    flops = 2 * (int64_t)y.rows * y.cols * A.cols;
  } else if (t.op == OP_LRGEMM) {
    RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b), X = resolve(a, t.x);
    bytes = vbytes(A) + vbytes(B) + vbytes(X) + (t.beta != 0.0 ? 2 : 1) * vbytes(y);
    flops = 2 * (int64_t)A.cols * B.cols * X.cols + 2 * (int64_t)y.rows * A.cols * y.cols;
  } else if (t.op == OP_GEMMP) {
    RV y = resolve(a, t.y), A = resolve(a, t.a), B = resolve(a, t.b);
    bytes = vbytes(A) + (int64_t)t.r0 * vbytes(B) + 2 * vbytes(y);
    flops = 2 * (int64_t)y.rows * y.cols * A.cols + (int64_t)t.r0 * B.rows * B.cols;
  } else if (t.op == OP_ZERO) {
    bytes = vbytes(resolve(a, t.y));
  } else if (t.op == OP_COPY) {
    RV y = resolve(a, t.y);
    bytes = 2 * vbytes(y);
  } else if (t.op == OP_TRTRI) {
    int64_t m = t.a.rows;
    bytes = 3 * m * m * 8;
    flops = 2 * m * m * m / 3;
  } else if (t.op == OP_SEQ) {
    bytes = 2 * vbytes(resolve(a, t.y));  // the block's panel rows (its micro-operations are not counted)
  }
  wg_ctr(lds)[0] += bytes;
  wg_ctr(lds)[1] += flops;
}

// Task sets of the executors: the H-LU's, the substitution's (TRSM, GEMM,
// LRGEMM, GEMMP, ZERO, COPY with the streamed large-product paths), or both
// (a fused DAG, whose substitution tasks carry c1 = 1).
enum ExecMode { kModeLU = 0, kModeSolve = 1, kModeFused = 2 };

template <int kMode>
__device__ void run_task_body(const ExecArgs& a, const Task& t, char* lds, double* scratch);

// The running task's record and start tick live in LDS after the counters.
__device__ __forceinline__ Task* task_copy(char* lds) { return (Task*)(lds + kLdsBytes + (kCtrSize + 6) * 8); }
__device__ __forceinline__ uint64_t* task_t0(char* lds) {
  return (uint64_t*)(lds + kLdsBytes + (kCtrSize + 6) * 8 + (int)sizeof(Task));
}
// the task's successor range [succ_ptr[id], succ_ptr[id + 1]), loaded with the record
__device__ __forceinline__ int* task_succ(char* lds) {
  return (int*)(lds + kLdsBytes + (kCtrSize + 6) * 8 + (int)sizeof(Task) + 8);
}

// Runs task id: its record is copied into LDS in one load phase (instead of
// dependent global loads as its fields are used), then its body runs.  The
// statistics are taken by account_task after the task, off the hand-off path.
template <int kMode = kModeLU>
__device__ void run_task(const ExecArgs& a, int id, char* lds, double* scratch) {
  Task* lt = task_copy(lds);
  {
    const int* src = (const int*)(a.tasks + id);
    int* dst = (int*)lt;
    for (int i = threadIdx.x; i < (int)(sizeof(Task) / 4); i += blockDim.x) dst[i] = src[i];
    const int w = (int)threadIdx.x - (int)(sizeof(Task) / 4);
    if (w == 0 || w == 1) task_succ(lds)[w] = a.succ_ptr[id + w];
  }
  if (threadIdx.x == 0 && a.counters) {
    if (a.trace)
      for (int k = 0; k < 6; ++k) wg_ctr(lds)[kCtrSize + k] = 0;
    *task_t0(lds) = wall_clock64();
  }
  __syncthreads();
  run_task_body<kMode>(a, *lt, lds, scratch);
}

// Statistics of the task that just ran (one thread, after a barrier that
// follows the task; the record copy is still in LDS).
__device__ void account_task(const ExecArgs& a, int id, char* lds) {
  if (!a.counters) return;
  // the end tick first: the accounting's own loads are not the task's time
  const uint64_t t1 = wall_clock64();
  const Task& t = *task_copy(lds);
  count_task(a, t, lds);
  if (t.op < 0 || t.op >= OP_COUNT) return;
  const uint64_t t0 = *task_t0(lds);
  wg_ctr(lds)[kCtrBusy + t.op] += t1 - t0;
  wg_ctr(lds)[kCtrCount + t.op] += 1;
  if (!a.trace) return;
  uint64_t* tr = a.trace + (int64_t)kTraceWords * id;
  tr[0] = t0;
  tr[1] = t1;
  uint64_t info = blockIdx.x & 0xffff;
  if (t.op == OP_TRUNC || t.op == OP_TRUNC2) {
    const LrDesc d = a.lr[t.lr];
    uint64_t K = (uint64_t)resolve(a, t.a).cols;
    if (t.op == OP_TRUNC2) K += (uint64_t)resolve(a, t.x).cols;
    info |= (K & 0xffff) << 16 | (uint64_t)(d.m & 0xffff) << 32 | (uint64_t)(d.n & 0xffff) << 48;
  } else {
    // output rows / columns and the inner dimension
    const View& o = (t.op == OP_GETRF) ? t.a : (t.op >= OP_TRSM_L && t.op <= OP_TRSM_U) ? t.x : t.y;
    const RV r = resolve(a, o);
    const int kd = (t.op == OP_GEMM || t.op == OP_LRGEMM) ? resolve(a, t.a).cols : t.op == OP_SEQ ? t.lr : t.a.rows;
    info |= (uint64_t)(r.rows & 0xffff) << 16 | (uint64_t)(r.cols & 0xffff) << 32 | (uint64_t)(kd & 0xffff) << 48;
  }
  tr[2] = info;
  uint64_t info2 = 0;
  if (t.op == OP_TRUNC || t.op == OP_TRUNC2) {
    const int* s_int = (const int*)(lds + kLdsBytes - 64);
    info2 = (uint64_t)(s_int[12] & 0xff) | (uint64_t)(s_int[13] & 0xfff) << 8 |
            (uint64_t)((s_int[13] >> 16) & 0xfff) << 20 | (uint64_t)(s_int[14] & 0xff) << 32 |
            (uint64_t)((s_int[14] >> 16) & 0xff) << 40;
  }
  tr[3] = info2;
  for (int k = 0; k < 3; ++k) {
    const uint64_t lo = wg_ctr(lds)[kCtrSize + 2 * k], hi = wg_ctr(lds)[kCtrSize + 2 * k + 1];
    tr[4 + k] = (lo > 0xffffffffull ? 0xffffffffull : lo) | (hi > 0xffffffffull ? 0xffffffffull : hi) << 32;
  }
  // tr[7]: the tick at which the task was pushed to the ready queue
}

template <int kMode>
__device__ void run_task_body(const ExecArgs& a, const Task& t, char* lds, double* scratch) {
  constexpr bool kLU = kMode != kModeSolve, kSub = kMode != kModeLU;
  // streamed paths for the substitution's products only, so that the H-LU
  // part of a fused DAG computes exactly as the H-LU's own DAG
  const bool sub = kSub && (!kLU || t.c1 == 1);
  if ((!kLU && (t.op == OP_GETRF || t.op == OP_TRSM_UT || t.op == OP_TRUNC || t.op == OP_TRUNC2)) ||
      (!kSub && t.op == OP_GEMMP) || (kLU && t.op == OP_SEQ) || (!kLU && t.op == OP_TRTRI)) {
    if (threadIdx.x == 0) atomicOr(&a.status[0], ST_BADOP);
    return;
  }
  switch (t.op) {
    case OP_GETRF:
      if (kLU) op_getrf(a, t, lds);
      break;
    case OP_TRSM_L:
      op_trsm(a, t, lds, 0);
      break;
    case OP_TRSM_UT:
      if (kLU) op_trsm(a, t, lds, 1);
      break;
    case OP_TRSM_U:
      op_trsm(a, t, lds, 2);
      break;
    case OP_GEMM:
      if (sub && solve_skinny_gemm(a, t))
        op_gemm_skinny(a, t, lds);
      else if (all_f32(t.y) && all_f32(t.a) && all_f32(t.b))
        op_gemm_ct<float>(a, t, lds);
      else
        op_gemm_ct<double>(a, t, lds);
      break;
    case OP_LRGEMM:
      if (sub && !lrgemm_fits_lds(a, t))
        op_lrgemm_solve(a, t, lds);
      else if (all_f32(t.y) && all_f32(t.a) && all_f32(t.b) && all_f32(t.x))
        op_lrgemm_ct<float>(a, t, lds);
      else
        op_lrgemm_ct<double>(a, t, lds);
      break;
    case OP_GEMMP:
      if (kSub) op_gemmp(a, t, lds);
      break;
    case OP_SEQ:
      if (!kLU) op_seq(a, t, lds);
      break;
    case OP_TRTRI:
      if (kLU) op_trtri(a, t, lds);
      break;
    case OP_TRUNC:
    case OP_TRUNC2:
      if (kLU) op_trunc(a, t, lds, scratch);
      break;
    case OP_ZERO:
      op_zero(a, t);
      break;
    case OP_COPY:
      op_copy(a, t);
      break;
    default:
      break;
  }
}

__device__ void wg_ctr_init(const ExecArgs& a, char* lds) {
  if (a.counters)
    for (int i = threadIdx.x; i < kCtrSize; i += blockDim.x) wg_ctr(lds)[i] = 0;
  __syncthreads();
}

__device__ void wg_ctr_flush(const ExecArgs& a, char* lds) {
  __syncthreads();
  if (a.counters)
    for (int i = threadIdx.x; i < kCtrSize; i += blockDim.x) {
      const unsigned long long v = wg_ctr(lds)[i];
      if (v) atomicAdd(&a.counters[i], v);
    }
}

// One launch per DAG level: workgroup w runs tasks order[begin + w], order[begin + w + grid], ...
__global__ void __launch_bounds__(kThreads, 2) exec_level_kernel(ExecArgs a, const int32_t* order, int begin, int end) {
  extern __shared__ __align__(16) char lds[];
  double* scratch = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  wg_ctr_init(a, lds);
  for (int i = begin + (int)blockIdx.x; i < end; i += (int)gridDim.x) {
    run_task(a, order[i], lds, scratch);
    __syncthreads();
    if (threadIdx.x == 0) account_task(a, order[i], lds);
    __syncthreads();
  }
  wg_ctr_flush(a, lds);
}

// The level executor for the forward / backward substitution DAGs.
__global__ void __launch_bounds__(kThreads, 2) solve_level_kernel(ExecArgs a, const int32_t* order, int begin,
                                                                  int end) {
  extern __shared__ __align__(16) char lds[];
  double* scratch = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  wg_ctr_init(a, lds);
  for (int i = begin + (int)blockIdx.x; i < end; i += (int)gridDim.x) {
    run_task<kModeSolve>(a, order[i], lds, scratch);
    __syncthreads();
    if (threadIdx.x == 0) account_task(a, order[i], lds);
    __syncthreads();
  }
  wg_ctr_flush(a, lds);
}

__global__ void exec_reset_kernel(ExecArgs a, const int32_t* indeg, const int32_t* roots, int nroots) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int stride = gridDim.x * blockDim.x;
  for (int k = i; k < a.ntasks; k += stride) {
    a.deps[k] = indeg[k];
    a.queue[k] = k < nroots ? roots[k] : -1;
  }
  if (i == 0) {
    a.qctl[0] = 0;
    a.qctl[1] = nroots;
    a.qctl[2] = 0;
    a.qctl[3] = 0;
  }
}

// Persistent dataflow executor: workgroups claim queue slots in order, run the
// task that lands there, and release successors whose predecessor count drops
// to zero.  In the substitution DAGs (narrow chains) a workgroup runs the
// first substitution task it releases itself, with no queue round trip, and
// fills that task's queue slot with a skip marker (-2), so that every slot
// below ntasks is still filled exactly once for an acyclic DAG; a workgroup
// that draws a marker claims the next slot.  A workgroup that waits longer
// than spin_limit wall-clock ticks raises ST_TIMEOUT and every workgroup then
// leaves.
template <int kMode>
__device__ __forceinline__ void dataflow_body(const ExecArgs& a, char* lds, int& s_task) {
  __shared__ int s_next;  // a successor this workgroup released for itself, or -1
  double* scratch = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  const int tid = threadIdx.x;
  if (tid == 0) s_next = -1;
  wg_ctr_init(a, lds);
  for (;;) {
    if (tid == 0) {
      int t = s_next;
      s_next = -1;
      bool stop = false;
      while (t < 0 && !stop) {
        const int slot = atomicAdd(&a.qctl[0], 1);
        if (slot >= a.ntasks) break;
        const uint64_t t0 = wall_clock64();
        int v;
        for (;;) {
          v = __hip_atomic_load(&a.queue[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (v != -1) break;
          if (__hip_atomic_load(&a.qctl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            stop = true;
            break;
          }
          if ((int64_t)(wall_clock64() - t0) > a.spin_limit) {
            atomicOr(&a.status[0], ST_TIMEOUT);
            __hip_atomic_store(&a.qctl[3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            stop = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (!stop && v >= 0) {
          t = v;
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      s_task = t;
    }
    __syncthreads();
    const int t = s_task;
    if (t < 0) {
      wg_ctr_flush(a, lds);
      return;
    }
    run_task<kMode>(a, t, lds, scratch);
    // Publication: every thread's stores precede the workgroup barrier; one
    // agent-scope release fence then makes them visible across XCDs before
    // any successor count drops.  The workgroup that releases a successor
    // (its count reaches zero) puts an acq_rel fence between that decrement
    // and the push: it acquires every other predecessor's release (their
    // fences precede their decrements, which its decrement reads) and
    // releases them with its own data, so the relaxed queue store needs no
    // fence of its own.  The consumer reads the slot relaxed and then takes
    // one agent-scope acquire fence.
    __syncthreads();
    if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid < 64) {
      const int b = task_succ(lds)[0], e = task_succ(lds)[1];
      bool kept = false;
      for (int k0 = b; k0 < e; k0 += 64) {
        const int k = k0 + tid;
        int s = -1;
        bool rel = false, crit = false;
        if (k < e) {
          s = a.succ_idx[k];
          if (a.succ_crit) crit = a.succ_crit[k] != 0;
          rel = __hip_atomic_fetch_add(&a.deps[s], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1;
        }
        if (rel) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        // kept: substitution tasks, and H-LU tasks near the critical path; the
        // other H-LU tasks keep their queue order
        const bool can_keep =
            rel && (kMode == kModeSolve || crit || (kMode == kModeFused && a.tasks[s].c1 == 1));
        const unsigned long long m = __ballot(can_keep);
        int keep = -1;
        if (!kept && m) {
          keep = __ffsll((long long)m) - 1;
          kept = true;
        }
        if (rel) {
          if (a.trace) a.trace[(int64_t)kTraceWords * s + 7] = wall_clock64();
          const int pos = atomicAdd(&a.qctl[1], 1);
          if (tid == keep) s_next = s;
          if (pos < a.ntasks)
            __hip_atomic_store(&a.queue[pos], tid == keep ? -2 : s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    } else if (tid == 64) {
      account_task(a, t, lds);  // beside the hand-off, not before it
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kThreads, 2) exec_dataflow_kernel(ExecArgs a) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_task;
  dataflow_body<kModeLU>(a, lds, s_task);
}

// The same executor for the forward / backward substitution DAGs, built
// with the solve's task set only.
__global__ void __launch_bounds__(kThreads, 2) solve_dataflow_kernel(ExecArgs a) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_task;
  dataflow_body<kModeSolve>(a, lds, s_task);
}

// The persistent executor for a fused DAG (H-LU followed by the substitution).
__global__ void __launch_bounds__(kThreads, 2) fused_dataflow_kernel(ExecArgs a) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_task;
  dataflow_body<kModeFused>(a, lds, s_task);
}

// ---------------------------------------------------------------------------
// assembly: kernel entries and adaptive cross approximation
// ---------------------------------------------------------------------------

__device__ __forceinline__ double kernel_entry(const AsmArgs& s, int64_t i, int64_t j) {
  if (i == j) return s.diag;
  double dx = s.pts[3 * i] - s.pts[3 * j];
  double dy = s.pts[3 * i + 1] - s.pts[3 * j + 1];
  double dz = s.pts[3 * i + 2] - s.pts[3 * j + 2];
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (s.kernel == 0) return 1.0 / (4.0 * 3.14159265358979323846 * r);
  return -log(r) / (2.0 * 3.14159265358979323846);
}


__global__ void __launch_bounds__(kThreads) assemble_dense_kernel(ExecArgs a, AsmArgs s, const DenseAsm* blocks) {
  const DenseAsm b = blocks[blockIdx.x];
  for (int64_t e = threadIdx.x; e < (int64_t)b.m * b.n; e += blockDim.x) {
    int64_t i = e % b.m, j = e / b.m;
    double v = kernel_entry(s, b.r0 + i, b.c0 + j);
    if (b.type == VT_F64)
      a.f64[b.off + e] = v;
    else
      a.f32[b.off + e] = (float)v;
  }
}


// ACA with partial pivoting into scratch factors (capacity kMaxK), then
// recompression through the truncation core with an empty C.
__global__ void __launch_bounds__(kThreads) assemble_aca_kernel(ExecArgs a, AsmArgs s, const LrAsm* blocks,
                                                               double* fac, int64_t fac_stride, double aca_eps) {
  extern __shared__ __align__(16) char lds[];
  const LrAsm blk = blocks[blockIdx.x];
  const LrDesc d = a.lr[blk.lr];
  const int m = d.m, n = d.n, tid = threadIdx.x;
  double* U = fac + (int64_t)blockIdx.x * fac_stride;  // m x kMaxK
  double* V = U + (int64_t)m * kMaxK;                  // n x kMaxK
  char* used = (char*)(V + (int64_t)n * kMaxK);        // m flags
  if ((int64_t)(m + n) * kMaxK * 8 + m > fac_stride * 8) {  // the slot must hold this block
    if (tid == 0) atomicOr(&a.status[0], ST_BADOP);
    return;
  }
  double* red = (double*)(lds + kLdsBytes - 4096);     // reduction scratch
  int* ired = (int*)(lds + kLdsBytes - 2048);
  for (int i = tid; i < m; i += blockDim.x) used[i] = 0;
  const int kmax = min(kMaxK, min(m, n));
  double norm2 = 0.0;  // ||S_k||_F^2
  int k = 0, istar = 0, zero_rows = 0;
  __syncthreads();
  while (k < kmax) {
    // row istar of the residual -> V[:, k]
    for (int j = tid; j < n; j += blockDim.x) {
      double v = kernel_entry(s, blk.r0 + istar, blk.c0 + j);
      for (int l = 0; l < k; ++l) v -= U[(int64_t)l * m + istar] * V[(int64_t)l * n + j];
      V[(int64_t)k * n + j] = v;
    }
    if (tid == 0) used[istar] = 1;
    __syncthreads();
    // pivot column: argmax |v_j|
    double best = -1.0;
    int bj = n;
    for (int j = tid; j < n; j += blockDim.x) {
      double x = fabs(V[(int64_t)k * n + j]);
      if (x > best) {
        best = x;
        bj = j;
      }
    }
    red[tid] = best;
    ired[tid] = bj;
    __syncthreads();
    for (int off = blockDim.x / 2; off >= 1; off >>= 1) {
      if (tid < off) {
        double ob = red[tid + off];
        int oi = ired[tid + off];
        if (ob > red[tid] || (ob == red[tid] && oi < ired[tid])) {
          red[tid] = ob;
          ired[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int jstar = ired[0];
    const double piv = V[(int64_t)k * n + jstar];
    __syncthreads();
    if (piv == 0.0) {
      // zero residual row: try another unused row
      ++zero_rows;
      int next = -1;
      if (tid == 0) {
        for (int i = 0; i < m; ++i)
          if (!used[i]) {
            next = i;
            break;
          }
        ired[0] = next;
      }
      __syncthreads();
      next = ired[0];
      __syncthreads();
      if (next < 0 || zero_rows > 8) break;
      istar = next;
      continue;
    }
    for (int j = tid; j < n; j += blockDim.x) V[(int64_t)k * n + j] /= piv;
    __syncthreads();
    // column jstar of the residual -> U[:, k]
    for (int i = tid; i < m; i += blockDim.x) {
      double v = kernel_entry(s, blk.r0 + i, blk.c0 + jstar);
      for (int l = 0; l < k; ++l) v -= V[(int64_t)l * n + jstar] * U[(int64_t)l * m + i];
      U[(int64_t)k * m + i] = v;
    }
    __syncthreads();
    // norms: ||u||^2 ||v||^2 and cross terms with earlier columns
    double nu = 0, nv = 0;
    for (int i = tid; i < m; i += blockDim.x) nu += U[(int64_t)k * m + i] * U[(int64_t)k * m + i];
    for (int j = tid; j < n; j += blockDim.x) nv += V[(int64_t)k * n + j] * V[(int64_t)k * n + j];
    red[tid] = nu;
    red[blockDim.x + tid] = nv;
    __syncthreads();
    for (int off = blockDim.x / 2; off >= 1; off >>= 1) {
      if (tid < off) {
        red[tid] += red[tid + off];
        red[blockDim.x + tid] += red[blockDim.x + tid + off];
      }
      __syncthreads();
    }
    nu = red[0];
    nv = red[blockDim.x];
    __syncthreads();
    double cross = 0.0;
    for (int l = 0; l < k; ++l) {
      double cu = 0, cv = 0;
      for (int i = tid; i < m; i += blockDim.x) cu += U[(int64_t)l * m + i] * U[(int64_t)k * m + i];
      for (int j = tid; j < n; j += blockDim.x) cv += V[(int64_t)l * n + j] * V[(int64_t)k * n + j];
      red[tid] = cu;
      red[blockDim.x + tid] = cv;
      __syncthreads();
      for (int off = blockDim.x / 2; off >= 1; off >>= 1) {
        if (tid < off) {
          red[tid] += red[tid + off];
          red[blockDim.x + tid] += red[blockDim.x + tid + off];
        }
        __syncthreads();
      }
      cross += red[0] * red[blockDim.x];
      __syncthreads();
    }
    norm2 += nu * nv + 2.0 * cross;
    ++k;
    // next row: argmax |u_i| over unused rows
    best = -1.0;
    int bi = m;
    for (int i = tid; i < m; i += blockDim.x) {
      double x = used[i] ? -1.0 : fabs(U[(int64_t)(k - 1) * m + i]);
      if (x > best) {
        best = x;
        bi = i;
      }
    }
    red[tid] = best;
    ired[tid] = bi;
    __syncthreads();
    for (int off = blockDim.x / 2; off >= 1; off >>= 1) {
      if (tid < off) {
        double ob = red[tid + off];
        int oi = ired[tid + off];
        if (ob > red[tid] || (ob == red[tid] && oi < ired[tid])) {
          red[tid] = ob;
          ired[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int nexti = ired[0];
    const double nb = red[0];
    __syncthreads();
    if (sqrt(nu * nv) <= aca_eps * sqrt(fmax(norm2, 0.0))) break;
    if (nexti >= m || nb < 0.0) break;
    istar = nexti;
  }
  __syncthreads();
  // recompress: C (empty) + U V^T through the truncation core
  if (tid == 0) a.ranks[blk.lr] = 0;
  __syncthreads();
  Stack su, sv;
  su.c = RV{d.u_off, m, 0, 1, m, d.type};
  sv.c = RV{d.v_off, n, 0, 1, n, d.type};
  su.t = RV{0, m, k, 1, m, VT_F64};
  sv.t = RV{0, n, k, 1, n, VT_F64};
  su.tptr = U;
  sv.tptr = V;
  su.t2 = sv.t2 = RV{0, 0, 0, 1, 1, VT_NONE};
  su.m = m;
  sv.m = n;
  su.kc = sv.kc = 0;
  su.kp = sv.kp = k;
  su.kp2 = sv.kp2 = 0;
  su.r0 = sv.r0 = su.r2 = sv.r2 = 0;
  su.alpha = sv.alpha = su.alpha2 = sv.alpha2 = 1.0;
  trunc_core(a, d, blk.lr, su, sv, lds, a.scratch + (int64_t)blockIdx.x * a.scratch_stride, a.eps);
}

// ---------------------------------------------------------------------------
// H-matvec: y = alpha A x + beta y, permuted ordering, nrhs <= 16 per launch
// ---------------------------------------------------------------------------

// phase 1: T_b = V_b^T x_sigma for every low-rank leaf (k x nrhs, ld kMaxCap)
__global__ void __launch_bounds__(kThreads) matvec_phase1_kernel(ExecArgs a, const MvLeaf* leaves,
                                                                 const int32_t* lr_leaves, const double* x,
                                                                 int64_t ldx, int nrhs, double* T) {
  const MvLeaf L = leaves[lr_leaves[blockIdx.x]];
  const int k = a.ranks[L.lr];
  double* out = T + (int64_t)L.lr * kMaxCap * 16;
  const int tid = threadIdx.x;
  // each (l, r) output: sum over n rows
  for (int e = tid / 4; e < k * nrhs; e += blockDim.x / 4) {
    int l = e % k, r = e / k;
    double s = 0.0;
    for (int j = tid % 4; j < L.n; j += 4) {
      double v = L.type == VT_F64 ? a.f64[L.v_off + (int64_t)l * L.n + j] : (double)a.f32[L.v_off + (int64_t)l * L.n + j];
      s += v * x[(L.c0 + j) + (int64_t)r * ldx];
    }
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    if (tid % 4 == 0) out[l + (int64_t)r * kMaxCap] = s;
  }
}

// phase 2: one workgroup per leaf row cluster; y_tau = sum over covering leaves
__global__ void __launch_bounds__(kThreads) matvec_phase2_kernel(ExecArgs a, const MvLeaf* leaves,
                                                                 const int32_t* row_ptr, const MvRow* segs,
                                                                 const int64_t* row_begin, const int32_t* row_size,
                                                                 const double* x, int64_t ldx, int nrhs,
                                                                 const double* T, double* y, int64_t ldy,
                                                                 double alpha, double beta) {
  const int rc = blockIdx.x;
  const int64_t rb = row_begin[rc];
  const int mr = row_size[rc];
  const int tid = threadIdx.x;
  for (int e = tid; e < mr * nrhs; e += blockDim.x) {
    int i = e % mr, r = e / mr;
    double s = 0.0;
    for (int q = row_ptr[rc]; q < row_ptr[rc + 1]; ++q) {
      const MvRow sg = segs[q];
      const MvLeaf L = leaves[sg.leaf];
      const int li = sg.lrow + i;
      if (L.lr < 0) {
        for (int j = 0; j < L.n; ++j) {
          double v = L.type == VT_F64 ? a.f64[L.off + li + (int64_t)j * L.m] : (double)a.f32[L.off + li + (int64_t)j * L.m];
          s += v * x[(L.c0 + j) + (int64_t)r * ldx];
        }
      } else {
        const int k = a.ranks[L.lr];
        const double* t = T + (int64_t)L.lr * kMaxCap * 16 + (int64_t)r * kMaxCap;
        for (int l = 0; l < k; ++l) {
          double u = L.type == VT_F64 ? a.f64[L.u_off + li + (int64_t)l * L.m] : (double)a.f32[L.u_off + li + (int64_t)l * L.m];
          s += u * t[l];
        }
      }
    }
    double* yp = y + (rb + i) + (int64_t)r * ldy;
    *yp = (beta == 0.0 ? 0.0 : beta * *yp) + alpha * s;
  }
}

// ---------------------------------------------------------------------------
// vector helpers for the solve and refinement (all FP64)
// ---------------------------------------------------------------------------
// dst[k + r*ldd] = src[perm[k] + r*lds]   (gather into permuted order)
__global__ void gather_rows_kernel(const double* src, int64_t lds_, const int64_t* perm, int64_t n, int nrhs,
                                   double* dst, int64_t ldd) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t k = i % n, r = i / n;
  dst[k + r * ldd] = src[perm[k] + r * lds_];
}
// dst[perm[k] + r*ldd] = alpha*src[k + r*lds] + beta*dst[...]
__global__ void scatter_rows_kernel(const double* src, int64_t lds_, const int64_t* perm, int64_t n, int nrhs,
                                    double* dst, int64_t ldd, double alpha, double beta) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t k = i % n, r = i / n;
  double* d = dst + perm[k] + r * ldd;
  *d = alpha * src[k + r * lds_] + (beta == 0.0 ? 0.0 : beta * *d);
}
// out[r] = sum_k v[k + r*ld]^2  (one workgroup per column)
__global__ void __launch_bounds__(kThreads) colnorm2_kernel(const double* v, int64_t ld, int64_t n, double* out) {
  __shared__ double red[kThreads];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    double x = v[k + r * ld];
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}
// y += x (n x nrhs, separate leading dimensions), columns with active[r] == 0 skipped
__global__ void axpy_cols_kernel(double* y, int64_t ldy, const double* x, int64_t ldx, int64_t n, int nrhs,
                                 const int32_t* active) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t k = i % n, r = i / n;
  if (active && !active[r]) return;
  y[k + r * ldy] += x[k + r * ldx];
}
// p[i] = v[i] for i < n (small control words written in stream order)
__global__ void set_i32_kernel(int32_t* p, int32_t v0, int32_t v1, int32_t v2, int32_t v3, int n) {
  if (threadIdx.x == 0) {
    if (n > 0) p[0] = v0;
    if (n > 1) p[1] = v1;
    if (n > 2) p[2] = v2;
    if (n > 3) p[3] = v3;
  }
}
// p[0..n) = v (a fill kernel instead of a memset node, so that the clears
// stay kernels when a caller captures the stream)
__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
// The hm_status of a substitution from the executor's status word: 0, or
// HM_EDEVICE (-5) after a timeout or an unexpected task.
__global__ void status_word_kernel(const int32_t* exec_status, int32_t* out) {
  if (threadIdx.x == 0) out[0] = (exec_status[0] & (ST_TIMEOUT | ST_BADOP)) ? -5 : 0;
}
// copy / convert one leaf-block arena region (A layout -> LU layout)
__global__ void convert_blocks_kernel(const double* src, double* d64, float* d32, const CopyDesc* descs) {
  const CopyDesc c = descs[blockIdx.x];
  for (int64_t e = threadIdx.x; e < c.count; e += blockDim.x) {
    double v = src[c.src + e];
    if (c.dst_type == VT_F64)
      d64[c.dst + e] = v;
    else
      d32[c.dst + e] = (float)v;
  }
}

}  // namespace hm
