// Internal structures shared by the host trace (C++) and the device executor (HIP).
//
// The H-LU of Algorithm 2 (with Algorithms 1 and 3 and their leaf branches)
// is traced once on the host into a list of leaf-level tasks.  Each task
// works on strided views of block storage held in one device arena per
// element type.  Data dependencies follow Def. 3.1 / Def. 3.2 (outputs of one
// task intersecting inputs of another on the same storage), extended with
// write-after-read and write-after-write ordering so that any topological
// order reproduces the sequential result.
#pragma once
#include <cstdint>

namespace hm {

constexpr int kThreads = 256;      // threads per workgroup of every block kernel
constexpr int kMaxK = 128;         // widest stacked rank in a truncated addition
constexpr int kMaxCap = 64;        // widest stored rank of a low-rank leaf
constexpr int kMaxLeaf = 128;      // largest diagonal leaf the getrf/trsm kernels take
constexpr int kLdsBytes = 76 * 1024;  // dynamic LDS per workgroup (two workgroups per CU)
// Relative accuracy of the inner truncations that combine collected updates
// (in units of eps): tighter than the final one so that their rounding of the
// partial sums stays below the final truncation threshold.
constexpr double kInnerEps = 0.1;

enum ViewType : int32_t { VT_F64 = 0, VT_F32 = 1, VT_IDENT = 2, VT_NONE = 3 };
enum DynFlags : int32_t { DYN_ROWS = 1, DYN_COLS = 2, DYN_COLS2 = 4, DYN_LOCAL = 8 };

// Strided matrix view: element (i, j) lives at arena[off + i*rs + j*cs].
// With DYN_ROWS / DYN_COLS the extent is ranks[rank_id] (a low-rank leaf's
// current rank, or the nrhs of a solve), bounded by rows / cols; with
// DYN_COLS2 the column count is ranks[rank_id2] instead (a view whose rows
// follow a rank and whose columns follow the nrhs).  DYN_LOCAL marks a view of
// the solve panel inside a coarsened block (OP_SEQ): off is then the first row
// relative to the block, and the rows live in the block's on-chip copy.
struct View {
  int64_t off;
  int32_t rows, cols;
  int32_t rs, cs;
  int32_t type;
  int32_t dyn;
  int32_t rank_id;
  int32_t rank_id2;
};

enum Op : int32_t {
  OP_NOP = 0,
  OP_GETRF = 1,    // a: diagonal leaf (f64, m x m, col-major), piv: int32 offset
  OP_TRSM_L = 2,   // x <- L^{-1} P x     (a: packed LU of a diagonal leaf, piv; in substitutions
                   //                      b: the leaf's L^{-1}, U^{-1} from OP_TRTRI)
  OP_TRSM_UT = 3,  // x <- U^{-T} x
  OP_TRSM_U = 4,   // x <- U^{-1} x
  OP_GEMM = 5,     // y <- beta y + alpha a b
  OP_LRGEMM = 6,   // y <- beta y + alpha a (b x)
  OP_TRUNC = 7,    // low-rank leaf lr <- T_eps(U V^T + alpha pad(a) pad(b)^T)
  OP_ZERO = 8,     // y <- 0
  OP_COPY = 9,     // y <- a (element type conversion allowed)
  OP_TRUNC2 = 10,  // accumulator lr <- T_eps(alpha pad(a) pad(b)^T + beta pad(x) pad(y)^T)
  OP_GEMMP = 11,   // y <- y + alpha a (b_0 + ... + b_{r0-1}), b_p = b shifted by p * piv elements
  OP_SEQ = 12,     // substitution of a coarsened diagonal block: y = its rows of the solve panel,
                   // micro-operations seq[piv .. piv + lr) (TRSM_L / TRSM_U / GEMM / LRGEMM) in order
  OP_TRTRI = 13,   // y (m x 2m, f64) <- [L^{-1}, U^{-1}] of the packed LU a of a factored diagonal leaf
  OP_COUNT = 14,
};
constexpr int kOpSlots = 16;  // per-kind statistics slots of the public structures
static_assert(OP_COUNT <= kOpSlots, "task kinds exceed the statistics slots");

struct Task {
  int32_t op;
  int32_t lr;        // OP_TRUNC / OP_TRUNC2: low-rank leaf or accumulator index
  int32_t r0, c0;    // OP_TRUNC / OP_TRUNC2: offsets of the (first) term inside the target
  int32_t row0;      // OP_GETRF: first permuted row of the leaf; OP_TRUNC2: row offset of the second term
  int32_t c1;        // OP_TRUNC2: column offset of the second term
  int64_t piv;       // OP_GETRF / OP_TRSM_L: offset into the int32 pivot arena
  double alpha, beta;
  View y, a, b, x;
};

// One low-rank leaf: U (m x cap) and V (n x cap), column-major, in the arena of
// element type `type`; its current rank is ranks[index].
struct LrDesc {
  int64_t u_off, v_off;
  int32_t m, n, cap, type;
};

// Device-side arguments of an executor launch.
struct ExecArgs {
  double* f64;
  float* f32;
  int32_t* piv;
  int32_t* ranks;
  const LrDesc* lr;
  const Task* tasks;
  int32_t ntasks;
  int32_t pad0_;
  double eps;
  int32_t max_rank;
  int32_t nwg;
  int32_t* status;     // [0] error code, [1] first singular row, [2] rank overflow count
  double* scratch;     // per-workgroup f64 scratch, scratch_stride doubles each
  int64_t scratch_stride;
  // dataflow executor
  const int32_t* succ_ptr;
  const int32_t* succ_idx;
  int32_t* deps;       // remaining predecessor counts
  int32_t* queue;      // ready queue (ntasks slots, -1 = empty)
  int32_t* qctl;       // [0] head, [1] tail, [2] done, [3] abort
  int64_t spin_limit;  // wall-clock ticks a waiting workgroup polls before giving up
  // [0] algorithmic bytes, [1] algorithmic flops, [kCtrBusy + op] busy
  // wall-clock ticks of each task kind, [kCtrCount + op] task count,
  // [kCtrPhase ..+11] ticks of the truncation phases (+0..5 small-rank path,
  // +6..11 large-rank path), [kCtrK] sum of stacked
  // ranks K, [kCtrMN] sum of m + n (null: off)
  unsigned long long* counters;
  uint64_t* trace;  // optional: per task (start tick, end tick, workgroup)
  // coarsened substitution blocks (OP_SEQ): their micro-operations, and the
  // doubles of on-chip panel storage the launch provides after kSeqLdsOff
  const Task* seq;
  int32_t seq_panel;
  int32_t pad1_;
  // per edge: the successor is near the critical path (null: none flagged)
  const uint8_t* succ_crit;
};


// Assembly, matvec and conversion descriptors (one per workgroup).
struct AsmArgs {
  const double* pts;  // n x 3, permuted order
  int kernel;         // 0: 1/(4 pi r), 1: -log(r)/(2 pi)
  double diag;
};
struct DenseAsm {
  int64_t off;
  int64_t r0, c0;     // permuted row / column start
  int32_t m, n, type, pad;
};
struct LrAsm {
  int64_t r0, c0;
  int32_t lr;         // low-rank leaf index
  int32_t pad;
};
struct MvLeaf {
  int64_t off, u_off, v_off;  // dense data or low-rank factors
  int64_t r0, c0;             // permuted row / column start of the leaf
  int32_t m, n, lr, type;     // lr >= 0: low-rank leaf index
};
struct MvRow {                // one leaf's rows inside a leaf row cluster
  int32_t leaf;
  int32_t lrow;               // first row of the segment inside the leaf
};
struct CopyDesc {
  int64_t src, dst, count;
  int32_t dst_type, pad;
};

constexpr int64_t kScratchDoubles = 4 * kMaxK * kMaxK + 4 * kMaxK * kMaxCap + 6 * kMaxK + 64;

constexpr int kCtrBusy = 2, kCtrCount = 2 + OP_COUNT, kCtrPhase = 2 + 2 * OP_COUNT, kCtrK = kCtrPhase + 12,
              kCtrMN = kCtrK + 1, kCtrSize = kCtrMN + 1;
// dynamic LDS of the executor kernels: the task work area, then the
// workgroup's statistics counters (flushed to ExecArgs::counters at exit),
// then the current task's six truncation-phase tick counts (trace only)
// executor LDS: the task arena, the per-workgroup counters, then a copy of
// the running task's record, its start tick and its successor range
constexpr int kLdsExecBytes = kLdsBytes + (kCtrSize + 6) * 8 + (int)sizeof(Task) + 16;
// substitution executors: two micro-operation records of a coarsened block,
// then its rows of the panel (ExecArgs::seq_panel doubles)
constexpr int kSeqLdsOff = (kLdsExecBytes + 15) / 16 * 16;
constexpr int kSeqPanelOff = kSeqLdsOff + (2 * (int)sizeof(Task) + 15) / 16 * 16;
constexpr int kSeqPanelMax = 10240;  // doubles (80 KiB): 256 rows x 40 columns
constexpr int kMaxCoarsen = 1024;    // largest coarsening block (rows)
// words per task of the debug trace: start, end, info, info2, three words of
// phase ticks (two 32-bit counts each), the tick the task was queued
constexpr int kTraceWords = 8;

enum StatusCode : int32_t { ST_OK = 0, ST_SINGULAR = 1, ST_RANK = 2, ST_TIMEOUT = 4, ST_BADOP = 8 };

}  // namespace hm
