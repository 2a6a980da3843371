// C-ABI of libhm: handles, device memory, executors and the entry points of
// include/hm.h.  Host-only entry points (trees, DAG export) work without a
// device; compute entry points fail with HM_EDEVICE when none is usable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/hm.h"
#include "hm_internal.h"
#include "host.h"

namespace hm {
// kernels.hip
__global__ void exec_level_kernel(ExecArgs a, const int32_t* order, int begin, int end);
__global__ void exec_reset_kernel(ExecArgs a, const int32_t* indeg, const int32_t* roots, int nroots);
__global__ void exec_dataflow_kernel(ExecArgs a);
__global__ void solve_dataflow_kernel(ExecArgs a);
__global__ void solve_level_kernel(ExecArgs a, const int32_t* order, int begin, int end);
__global__ void fused_dataflow_kernel(ExecArgs a);
__global__ void assemble_dense_kernel(ExecArgs a, AsmArgs s, const DenseAsm* blocks);
__global__ void assemble_aca_kernel(ExecArgs a, AsmArgs s, const LrAsm* blocks, double* fac, int64_t fac_stride,
                                    double aca_eps);
__global__ void matvec_phase1_kernel(ExecArgs a, const MvLeaf* leaves, const int32_t* lr_leaves, const double* x,
                                     int64_t ldx, int nrhs, double* T);
__global__ void matvec_phase2_kernel(ExecArgs a, const MvLeaf* leaves, const int32_t* row_ptr, const MvRow* segs,
                                     const int64_t* row_begin, const int32_t* row_size, const double* x, int64_t ldx,
                                     int nrhs, const double* T, double* y, int64_t ldy, double alpha, double beta);
__global__ void gather_rows_kernel(const double* src, int64_t lds_, const int64_t* perm, int64_t n, int nrhs,
                                   double* dst, int64_t ldd);
__global__ void scatter_rows_kernel(const double* src, int64_t lds_, const int64_t* perm, int64_t n, int nrhs,
                                    double* dst, int64_t ldd, double alpha, double beta);
__global__ void colnorm2_kernel(const double* v, int64_t ld, int64_t n, double* out);
__global__ void axpy_cols_kernel(double* y, int64_t ldy, const double* x, int64_t ldx, int64_t n, int nrhs,
                                 const int32_t* active);
__global__ void convert_blocks_kernel(const double* src, double* d64, float* d32, const CopyDesc* descs);
__global__ void set_i32_kernel(int32_t* p, int32_t v0, int32_t v1, int32_t v2, int32_t v3, int n);
__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n);
__global__ void status_word_kernel(const int32_t* exec_status, int32_t* out);
}  // namespace hm

using namespace hm;

// ---------------------------------------------------------------------------
// errors and allocation
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static hm_status fail(hm_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(HM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static void* (*g_alloc)(size_t, void*, void*) = nullptr;
static void (*g_dealloc)(void*, size_t, void*, void*) = nullptr;
static void* g_alloc_ctx = nullptr;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  bool owned = true;  // false: a slice of another allocation (batched factors)
};

// HM_DEBUG_POISON=1 fills every new allocation with all-ones bytes (NaN for
// floating point, -1 for integers) so that a read of unwritten memory shows.
static bool poison_enabled() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("HM_DEBUG_POISON");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

static bool dev_alloc(DevBuf& b, size_t bytes, hipStream_t s) {
  b.bytes = bytes;
  b.stream = s;
  if (bytes == 0) {
    b.p = nullptr;
    return true;
  }
  if (g_alloc) {
    b.p = g_alloc(bytes, (void*)s, g_alloc_ctx);
  } else if (hipMalloc(&b.p, bytes) != hipSuccess) {
    b.p = nullptr;
  }
  if (b.p && poison_enabled()) (void)hipMemsetAsync(b.p, 0xff, bytes, s);
  return b.p != nullptr;
}

static void dev_free(DevBuf& b) {
  if (!b.p) return;
  if (!b.owned) {
    b.p = nullptr;
    b.bytes = 0;
    return;
  }
  if (g_dealloc)
    g_dealloc(b.p, b.bytes, (void*)b.stream, g_alloc_ctx);
  else
    (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

template <class T>
static hm_status upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  if (!dev_alloc(b, v.size() * sizeof(T), s)) return fail(HM_ENOMEM, "device allocation failed");
  if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return HM_OK;
}

static hm_status device_ok() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(HM_EDEVICE, "no HIP device available");
  return HM_OK;
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct DevDag {
  int64_t ntasks = 0, nlevels = 0, nedges = 0;
  DevBuf tasks, indeg, succ_ptr, succ_idx, roots, order;
  DevBuf seq;  // micro-operations of coarsened substitution blocks (OP_SEQ)
  DevBuf succ_crit;  // per edge: successor near the critical path
  int32_t nroots = 0;
  std::vector<int32_t> level_ptr;
  int64_t tasks_by_op[kOpSlots] = {};  // counted once at upload (a pass over the host records is slow)
};

struct PlanEntry {
  Plan plan;
  bool traced = false;
  bool uploaded = false, solve_uploaded = false;
  bool fused_traced = false, fused_uploaded = false;
  DevDag lu, solve, fused;
  DevBuf lr;
  int device = -1;
  // tasks per kind of the H-LU DAG, counted on first use (a pass over the
  // host task records costs tens of milliseconds at a few million tasks)
  int64_t lu_ops[kOpSlots] = {};
  bool lu_ops_done = false;
  // the block copy list from the first assembled matrix's layout into this
  // plan's factor layout (mixed precision), kept on the device for reuse
  const PlanEntry* conv_src = nullptr;
  DevBuf conv;
  int64_t nconv = 0;
};

// (the caller holds the tree's mutex)
static const int64_t* lu_op_counts(PlanEntry* pe) {
  if (!pe->lu_ops_done) {
    for (const Task& tk : pe->plan.lu.tasks)
      if (tk.op >= 0 && tk.op < OP_COUNT) pe->lu_ops[tk.op]++;
    pe->lu_ops_done = true;
  }
  return pe->lu_ops;
}

struct hm_tree_s {
  Tree t;
  hm_opts opts;
  // (prec, max_rank, lazy, span of the temporaries in MiB)
  std::map<std::tuple<int, int, int, int64_t, int>, std::unique_ptr<PlanEntry>> plans;
  std::mutex mu;
  std::vector<int64_t> leaf_begin;  // leaf clusters in order
  std::vector<int32_t> leaf_size;
};

struct hm_matrix_s {
  hm_tree tree;
  PlanEntry* pe;
  int kernel;
  double diag, eps;
  int max_rank;
  DevBuf f64, ranks, pts, perm;
  // matvec tables
  DevBuf mv_leaves, mv_lr, mv_row_ptr, mv_segs, mv_row_begin, mv_row_size, mv_T, mv_x, mv_y;
  int64_t n_lr_leaves = 0, n_rows = 0;
  DevBuf status;
  size_t bytes() const {
    return f64.bytes + ranks.bytes + pts.bytes + perm.bytes + mv_leaves.bytes + mv_lr.bytes + mv_row_ptr.bytes +
           mv_segs.bytes + mv_row_begin.bytes + mv_row_size.bytes + mv_T.bytes + mv_x.bytes + mv_y.bytes;
  }
};

struct ExecState {
  DevBuf deps, queue, qctl, status, counters, trace;
};

struct hm_lu_s {
  hm_tree tree;
  PlanEntry* pe;
  int prec, exec;
  double eps;
  int max_rank;
  int64_t dag_ntasks = 0;  // tasks of the DAG that produced the factors (H-LU, or H-LU + substitution)
  DevBuf f64, f32, piv, ranks, perm;
  ExecState lu_st, solve_st;
  DevBuf work;  // solve/refinement vectors
  size_t work_cols = 0;
  hm_lu_stats stats;
  // factors of h_lu_batched: f64 / f32 / piv / ranks are slices of one
  // allocation shared by the batch, released with its last handle
  std::shared_ptr<void> arena;
};

static int g_nwg = 0;      // executor workgroups at full occupancy (scratch is sized for these)
static int g_seq_panel = 0;  // doubles of on-chip panel storage per substitution workgroup (OP_SEQ)
static int g_cus = 0;
static int64_t g_clock_khz = 0;
// Launch choices that the autotuner sets (hm_set_tuning); environment
// variables give the defaults.
static hm_tuning g_tuning = {0, 64, 0, {0, 0, 0, 0, 0}};

// Workgroups of an H-LU executor launch under the current tuning.
static int exec_workgroups() {
  if (g_tuning.exec_wg_per_cu <= 0 || g_cus <= 0) return g_nwg;
  return std::max(1, std::min(g_nwg, g_cus * g_tuning.exec_wg_per_cu));
}
static void batch_cache_drop(hm_tree t);

// dynamic LDS of a substitution executor launch
static int solve_lds_bytes() { return g_seq_panel > 0 ? kSeqPanelOff + g_seq_panel * 8 : kLdsExecBytes; }

static hm_status device_setup() {
  if (g_nwg > 0) return HM_OK;
  hm_status st = device_ok();
  if (st) return st;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int rate = 0;
  if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate <= 0) rate = 100000;
  g_clock_khz = rate;
  (void)hipFuncSetAttribute((const void*)exec_level_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsExecBytes);
  (void)hipFuncSetAttribute((const void*)exec_dataflow_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kLdsExecBytes);
  // the substitution executors also hold a coarsened block's panel rows
  // (OP_SEQ) after their task area, as much as the workgroup's LDS allows
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds_max = 0;
  hipFuncAttributes fa{};
  const int fixed = hipFuncGetAttributes(&fa, (const void*)solve_dataflow_kernel) == hipSuccess ? (int)fa.sharedSizeBytes : 0;
  g_seq_panel = std::max(0, std::min(kSeqPanelMax, (lds_max - fixed - kSeqPanelOff) / 8));
  (void)hipFuncSetAttribute((const void*)solve_dataflow_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            solve_lds_bytes());
  (void)hipFuncSetAttribute((const void*)solve_level_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            solve_lds_bytes());
  (void)hipFuncSetAttribute((const void*)fused_dataflow_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kLdsExecBytes);
  (void)hipFuncSetAttribute((const void*)assemble_aca_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)exec_dataflow_kernel, kThreads, kLdsExecBytes) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  g_nwg = cus * per_cu;
  g_cus = cus;
  if (const char* e = getenv("HM_SOLVE_NWG")) g_tuning.solve_wg = std::max(1, atoi(e));
  // HM_DEBUG_MAX_WG caps the executor workgroups (1 = one task at a time)
  if (const char* e = getenv("HM_DEBUG_MAX_WG")) {
    int v = atoi(e);
    if (v >= 1 && v < g_nwg) g_nwg = v;
  }
  return HM_OK;
}

static const int64_t kScratchPerWg = kScratchDoubles;

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
// Device bytes the ring of temporaries of one traced DAG may span (per size
// class an eighth); a larger ring means fewer orderings from reuse.
// HM_TEMP_BUDGET_GB overrides it.
static int64_t temp_budget() {
  double gb = 16.0;
  if (const char* e = getenv("HM_TEMP_BUDGET_GB")) gb = std::max(1e-4, atof(e));
  return (int64_t)(gb * (double)(1ll << 30));
}

// Row chunk of the low-rank products that the substitution DAG splits over
// several workgroups (those with a side of at least twice this); 0 = none.
// HM_SOLVE_SPLIT overrides it.
static int32_t solve_split_rows() {
  int v = 1024;
  if (const char* e = getenv("HM_SOLVE_SPLIT")) v = std::max(0, atoi(e));
  return v;
}

static hm_status get_plan(hm_tree t, int prec, int max_rank, int lazy, bool need_trace, PlanEntry** out,
                          int64_t budget = -1, int coarsen = 0) {
  if (budget < 0) budget = temp_budget();
  std::lock_guard<std::mutex> lk(t->mu);
  auto key = std::make_tuple(prec, max_rank, lazy, budget >> 20, coarsen);
  auto it = t->plans.find(key);
  PlanEntry* pe;
  if (it == t->plans.end()) {
    auto up = std::make_unique<PlanEntry>();
    if (!make_layout(t->t, prec, max_rank, 64, up->plan)) return fail(HM_EINVAL, up->plan.err);
    pe = up.get();
    t->plans[key] = std::move(up);
  } else {
    pe = it->second.get();
  }
  if (need_trace && !pe->traced) {
    if (!trace_lu(pe->plan, budget, lazy)) return fail(HM_EINVAL, pe->plan.err);
    if (!trace_solve(pe->plan, solve_split_rows(), coarsen)) return fail(HM_EINVAL, pe->plan.err);
    pe->traced = true;
  }
  *out = pe;
  return HM_OK;
}

// The fused H-LU + substitution DAG of a plan, traced on first use (host only).
static hm_status trace_fused(hm_tree t, PlanEntry* pe, int lazy) {
  std::lock_guard<std::mutex> lk(t->mu);
  if (!pe->fused_traced) {
    if (!trace_lu_solve(pe->plan, temp_budget(), lazy)) return fail(HM_EINVAL, pe->plan.err);
    pe->fused_traced = true;
  }
  return HM_OK;
}

static hm_status upload_dag(const Dag& d, DevDag& dd, hipStream_t s) {
  dd.ntasks = (int64_t)d.tasks.size();
  dd.nedges = d.nedges;
  dd.nlevels = (int64_t)d.level_ptr.size() - 1;
  dd.level_ptr = d.level_ptr;
  dd.nroots = (int32_t)d.roots.size();
  for (int k = 0; k < kOpSlots; ++k) dd.tasks_by_op[k] = 0;
  for (const Task& tk : d.tasks)
    if (tk.op >= 0 && tk.op < OP_COUNT) dd.tasks_by_op[tk.op]++;
  hm_status st;
  if ((st = upload(dd.tasks, d.tasks, s))) return st;
  if ((st = upload(dd.indeg, d.indeg, s))) return st;
  if ((st = upload(dd.succ_ptr, d.succ_ptr, s))) return st;
  if ((st = upload(dd.succ_idx, d.succ_idx, s))) return st;
  if ((st = upload(dd.roots, d.roots, s))) return st;
  if ((st = upload(dd.order, d.level_order, s))) return st;
  if (!d.seq.empty() && (st = upload(dd.seq, d.seq, s))) return st;
  if (!d.succ_crit.empty() && (st = upload(dd.succ_crit, d.succ_crit, s))) return st;
  return HM_OK;
}

// The substitution DAG and the low-rank descriptors of a plan on the device
// (what a solve on its factors needs).
static hm_status ensure_solve_uploaded(PlanEntry* pe, hipStream_t s) {
  if (pe->solve_uploaded) return HM_OK;
  hm_status st;
  if ((st = upload_dag(pe->plan.solve, pe->solve, s))) return st;
  if ((st = upload(pe->lr, pe->plan.lr, s))) return st;
  HIPCHK(hipStreamSynchronize(s));
  pe->solve_uploaded = true;
  return HM_OK;
}

static hm_status ensure_uploaded(PlanEntry* pe, hipStream_t s) {
  hm_status st;
  if ((st = ensure_solve_uploaded(pe, s))) return st;
  if (pe->uploaded) return HM_OK;
  if ((st = upload_dag(pe->plan.lu, pe->lu, s))) return st;
  HIPCHK(hipStreamSynchronize(s));
  pe->uploaded = true;
  return HM_OK;
}

static hm_status exec_state_alloc(ExecState& es, int64_t ntasks, hipStream_t s) {
  if (!dev_alloc(es.deps, std::max<int64_t>(1, ntasks) * 4, s) ||
      !dev_alloc(es.queue, std::max<int64_t>(1, ntasks) * 4, s) || !dev_alloc(es.qctl, 64, s) ||
      !dev_alloc(es.status, 64, s) || !dev_alloc(es.counters, kCtrSize * 8, s))
    return fail(HM_ENOMEM, "device allocation failed (executor state)");
  return HM_OK;
}

static void exec_state_free(ExecState& es) {
  dev_free(es.trace);
  dev_free(es.deps);
  dev_free(es.queue);
  dev_free(es.qctl);
  dev_free(es.status);
  dev_free(es.counters);
}

enum DagKind { DAG_LU = 0, DAG_SOLVE = 1, DAG_FUSED = 2 };

// Wall-clock ticks a waiting executor workgroup polls an empty queue slot
// before it raises ST_TIMEOUT and every workgroup leaves: 30 s.
// HM_DEBUG_SPIN_TICKS overrides it (read at every launch), so that a test can
// make the bounded wait give up from the host while every kernel still exits
// normally.
static int64_t spin_limit_ticks() {
  if (const char* e = getenv("HM_DEBUG_SPIN_TICKS")) return std::max<int64_t>(0, atoll(e));
  return g_clock_khz * 1000 * 30;
}

// Run a DAG on `s`; *ms receives the executor's device time.  The fused DAG
// always runs on the persistent executor.
static hm_status run_dag(const DevDag& dd, ExecArgs a, ExecState& es, int mode, hipStream_t s, float* ms,
                         int kind = DAG_LU, bool reset_status = true) {
  const bool solve = kind == DAG_SOLVE;
  if (kind == DAG_FUSED) mode = HM_EXEC_DATAFLOW;
  if (dd.ntasks == 0) {
    if (ms) *ms = 0.f;
    return HM_OK;
  }
  a.tasks = (const Task*)dd.tasks.p;
  a.ntasks = (int32_t)dd.ntasks;
  a.succ_ptr = (const int32_t*)dd.succ_ptr.p;
  a.succ_idx = (const int32_t*)dd.succ_idx.p;
  a.deps = (int32_t*)es.deps.p;
  a.queue = (int32_t*)es.queue.p;
  a.qctl = (int32_t*)es.qctl.p;
  a.status = (int32_t*)es.status.p;
  // no statistics for substitutions (nothing reads them) unless their
  // timeline is recorded: their tasks skip the per-task accounting
  a.counters = solve && !es.trace.p ? nullptr : (unsigned long long*)es.counters.p;
  a.trace = (uint64_t*)es.trace.p;
  a.seq = (const Task*)dd.seq.p;
  a.succ_crit = (const uint8_t*)dd.succ_crit.p;
  a.seq_panel = g_seq_panel;
  if (dd.seq.p && g_seq_panel < 1) return fail(HM_EDEVICE, "no LDS left for coarsened substitution blocks");
  int nwg = exec_workgroups();
  // The substitution DAG has a few tasks per level: 64 persistent
  // workgroups hold every ready task and leave room for substitutions on
  // other streams (the tuning's solve_wg; HM_SOLVE_NWG sets its default).
  if (solve && mode != HM_EXEC_LEVEL) {
    const int v = g_tuning.solve_wg;
    if (v >= 1 && v < g_nwg) nwg = v;
  }
  a.nwg = nwg;
  a.spin_limit = spin_limit_ticks();
  if (reset_status)
    hipLaunchKernelGGL(set_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)es.status.p, 0, 0x7fffffff, 0, 0, 4);
  if (a.counters)
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(256), 0, s, (int32_t*)es.counters.p, 0, (int64_t)kCtrSize * 2);
  // events only when the caller asks for the device time
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
  }
  if (mode == HM_EXEC_LEVEL) {
    if (ms) HIPCHK(hipEventRecord(e0, s));
    for (int64_t l = 0; l < dd.nlevels; ++l) {
      int b = dd.level_ptr[l], e = dd.level_ptr[l + 1];
      int grid = std::min(e - b, nwg);
      if (solve)
        hipLaunchKernelGGL(solve_level_kernel, dim3(grid), dim3(kThreads), solve_lds_bytes(), s, a,
                           (const int32_t*)dd.order.p, b, e);
      else
        hipLaunchKernelGGL(exec_level_kernel, dim3(grid), dim3(kThreads), kLdsExecBytes, s, a,
                           (const int32_t*)dd.order.p, b, e);
    }
    HIPCHK(hipGetLastError());
    if (ms) HIPCHK(hipEventRecord(e1, s));
  } else {
    int rg = (int)std::min<int64_t>(1024, (dd.ntasks + 255) / 256);
    hipLaunchKernelGGL(exec_reset_kernel, dim3(rg), dim3(256), 0, s, a, (const int32_t*)dd.indeg.p,
                       (const int32_t*)dd.roots.p, dd.nroots);
    HIPCHK(hipGetLastError());
    if (ms) HIPCHK(hipEventRecord(e0, s));
    if (solve)
      hipLaunchKernelGGL(solve_dataflow_kernel, dim3(nwg), dim3(kThreads), solve_lds_bytes(), s, a);
    else if (kind == DAG_FUSED)
      hipLaunchKernelGGL(fused_dataflow_kernel, dim3(nwg), dim3(kThreads), kLdsExecBytes, s, a);
    else
      hipLaunchKernelGGL(exec_dataflow_kernel, dim3(nwg), dim3(kThreads), kLdsExecBytes, s, a);
    HIPCHK(hipGetLastError());
    if (ms) HIPCHK(hipEventRecord(e1, s));
  }
  if (ms) {
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return HM_OK;
}

static ExecArgs base_args(double* f64, float* f32, int32_t* piv, int32_t* ranks, const LrDesc* lr, double eps,
                          int max_rank) {
  ExecArgs a;
  std::memset(&a, 0, sizeof(a));
  a.f64 = f64;
  a.f32 = f32;
  a.piv = piv;
  a.ranks = ranks;
  a.lr = lr;
  a.eps = eps;
  a.max_rank = max_rank;
  return a;
}

// Smallest accepted truncation accuracy.  The truncation's R factors come
// from Cholesky factorizations of FP64 Gram matrices (CholeskyQR), which
// resolve directions down to about sqrt(u) = 1.5e-8 of the largest column;
// a smaller eps (and eps = 0, the exact case) would keep ranks the route
// cannot resolve, so it is rejected.
constexpr double kMinEps = 1e-8;

static bool valid_opts(const hm_opts* o) {
  return o && o->leaf >= 1 && o->eta > 0 && o->eps >= kMinEps && o->max_rank >= 0 && o->max_rank <= kMaxCap &&
         (o->prec == HM_FP64 || o->prec == HM_MIXED) && (o->exec == HM_EXEC_DATAFLOW || o->exec == HM_EXEC_LEVEL) &&
         (o->lazy >= 0 && o->lazy <= 2) && o->coarsen >= 0 && o->coarsen <= kMaxCoarsen;
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
extern "C" {

const char* hm_last_error(void) { return g_err.c_str(); }

hm_status hm_get_tuning(hm_tuning* out) {
  if (!out) return fail(HM_EINVAL, "null pointer");
  *out = g_tuning;
  return HM_OK;
}

hm_status hm_set_tuning(const hm_tuning* t) {
  if (!t) return fail(HM_EINVAL, "null pointer");
  if (t->exec_wg_per_cu < 0 || t->exec_wg_per_cu > 2 || t->solve_wg < 1 || t->solve_wg > 4096 ||
      t->batch_order < 0 || t->batch_order > 1)
    return fail(HM_EINVAL, "tuning out of range (exec_wg_per_cu 0..2, solve_wg 1..4096, batch_order 0..1)");
  g_tuning = *t;
  return HM_OK;
}

hm_status hm_set_allocator(void* (*alloc)(size_t, void*, void*), void (*dealloc)(void*, size_t, void*, void*),
                           void* ctx) {
  if ((alloc == nullptr) != (dealloc == nullptr)) return fail(HM_EINVAL, "allocator and deallocator come in pairs");
  g_alloc = alloc;
  g_dealloc = dealloc;
  g_alloc_ctx = ctx;
  return HM_OK;
}

hm_status build_htree(const double* pts, int64_t n, int dim, const hm_opts* opts, hm_tree* out) {
  if (!pts || !out || !opts) return fail(HM_EINVAL, "null pointer");
  if (n < 1 || opts->leaf < 1 || !(opts->eta > 0) || dim < 1 || dim > 3)
    return fail(HM_EINVAL, "need n >= 1, leaf >= 1, eta > 0, dim in {1,2,3}");
  if (n > (int64_t)1 << 30) return fail(HM_EINVAL, "n too large");
  auto t = new (std::nothrow) hm_tree_s();
  if (!t) return fail(HM_ENOMEM, "host allocation failed");
  t->opts = *opts;
  build_cluster_tree(pts, n, dim, opts->leaf, t->t);
  build_block_tree(t->t, opts->eta);
  for (const Cluster& c : t->t.cl)
    if (c.leaf()) {
      t->leaf_begin.push_back(c.begin);
      t->leaf_size.push_back((int32_t)c.size());
    }
  *out = t;
  return HM_OK;
}

hm_status hm_tree_sizes(hm_tree t, int64_t* n, int64_t* ncl, int64_t* nbl) {
  if (!t) return fail(HM_EINVAL, "null tree");
  if (n) *n = t->t.n;
  if (ncl) *ncl = (int64_t)t->t.cl.size();
  if (nbl) *nbl = (int64_t)t->t.bl.size();
  return HM_OK;
}

hm_status hm_tree_export(hm_tree t, int64_t* perm, int64_t* clusters, double* boxes, int32_t* blocks) {
  if (!t) return fail(HM_EINVAL, "null tree");
  if (perm) std::memcpy(perm, t->t.perm.data(), t->t.n * sizeof(int64_t));
  for (size_t i = 0; i < t->t.cl.size(); ++i) {
    const Cluster& c = t->t.cl[i];
    if (clusters) {
      int64_t* r = clusters + 5 * i;
      r[0] = c.begin;
      r[1] = c.end;
      r[2] = c.son[0];
      r[3] = c.son[1];
      r[4] = c.level;
    }
    if (boxes)
      for (int d = 0; d < 3; ++d) {
        boxes[6 * i + d] = c.lo[d];
        boxes[6 * i + 3 + d] = c.hi[d];
      }
  }
  if (blocks)
    for (size_t i = 0; i < t->t.bl.size(); ++i) {
      const BlockNode& b = t->t.bl[i];
      int32_t* r = blocks + 7 * i;
      r[0] = b.tau;
      r[1] = b.sigma;
      r[2] = b.kind;
      for (int k = 0; k < 4; ++k) r[3 + k] = b.son[k];
    }
  return HM_OK;
}

void hm_tree_free(hm_tree t) {
  if (!t) return;
  batch_cache_drop(t);
  for (auto& kv : t->plans) {
    PlanEntry* pe = kv.second.get();
    for (DevDag* dd : {&pe->lu, &pe->solve, &pe->fused}) {
      dev_free(dd->tasks);
      dev_free(dd->indeg);
      dev_free(dd->succ_ptr);
      dev_free(dd->succ_idx);
      dev_free(dd->roots);
      dev_free(dd->order);
      dev_free(dd->seq);
      dev_free(dd->succ_crit);
    }
    dev_free(pe->lr);
    dev_free(pe->conv);
  }
  delete t;
}

hm_status hm_dag_sizes(hm_tree t, const hm_opts* opts, int which, int64_t* sizes) {
  if (!t || !opts || !sizes || which < 0 || which > 2) return fail(HM_EINVAL, "bad argument");
  if (opts->max_rank < 0 || opts->max_rank > kMaxCap) return fail(HM_EINVAL, "max_rank must be in [0, 64]");
  PlanEntry* pe;
  hm_status st = get_plan(t, opts->prec, opts->max_rank, opts->lazy, true, &pe, -1, opts->coarsen);
  if (st) return st;
  if (which == 2 && (st = trace_fused(t, pe, opts->lazy))) return st;
  const Dag& d = which == 0 ? pe->plan.lu : which == 1 ? pe->plan.solve : pe->plan.fused;
  sizes[0] = (int64_t)d.tasks.size();
  sizes[1] = d.nedges;
  sizes[2] = (int64_t)d.level_ptr.size() - 1;
  sizes[3] = (int64_t)sizeof(Task);
  sizes[4] = pe->plan.n_f64;
  sizes[5] = pe->plan.n_f32;
  sizes[6] = pe->plan.n_piv;
  sizes[7] = (int64_t)pe->plan.lr.size();
  sizes[8] = pe->plan.nranks;
  return HM_OK;
}

hm_status hm_dag_calls(hm_tree t, const hm_opts* opts, int which, int64_t* ncalls, int32_t* calls, int32_t* task_call) {
  if (!t || !opts || which < 0 || which > 2) return fail(HM_EINVAL, "bad argument");
  PlanEntry* pe;
  hm_status st = get_plan(t, opts->prec, opts->max_rank, opts->lazy, true, &pe, -1, opts->coarsen);
  if (st) return st;
  if (which == 2 && (st = trace_fused(t, pe, opts->lazy))) return st;
  const Plan& p = pe->plan;
  const Dag& d = which == 0 ? p.lu : which == 1 ? p.solve : p.fused;
  if (ncalls) *ncalls = (int64_t)(d.calls.size() / 4);
  if (calls && !d.calls.empty()) std::memcpy(calls, d.calls.data(), d.calls.size() * 4);
  if (task_call && !d.task_call.empty()) std::memcpy(task_call, d.task_call.data(), d.task_call.size() * 4);
  return HM_OK;
}

hm_status hm_semiauto_dag(hm_tree t, int sparsify, int max_path, int64_t* ntasks, int64_t* nedges, int32_t* tasks,
                          int32_t* edges) {
  if (!t || max_path < 0) return fail(HM_EINVAL, "bad argument");
  std::vector<int32_t> tv, ev;
  try {
    build_semiauto_dag(t->t, sparsify != 0, max_path, tv, ev);
  } catch (const std::bad_alloc&) {
    return fail(HM_ENOMEM, "host allocation failed");
  }
  if (ntasks) *ntasks = (int64_t)(tv.size() / 4);
  if (nedges) *nedges = (int64_t)(ev.size() / 2);
  if (tasks && !tv.empty()) std::memcpy(tasks, tv.data(), tv.size() * 4);
  if (edges && !ev.empty()) std::memcpy(edges, ev.data(), ev.size() * 4);
  return HM_OK;
}

hm_status hm_dag_export(hm_tree t, const hm_opts* opts, int which, void* tasks, int32_t* succ_ptr, int32_t* succ_idx,
                        int32_t* level, int64_t* block_off, int64_t* lr) {
  if (!t || !opts || which < 0 || which > 2) return fail(HM_EINVAL, "bad argument");
  PlanEntry* pe;
  hm_status st = get_plan(t, opts->prec, opts->max_rank, opts->lazy, true, &pe, -1, opts->coarsen);
  if (st) return st;
  const Plan& p = pe->plan;
  if (which == 2 && (st = trace_fused(t, pe, opts->lazy))) return st;
  const Dag& d = which == 0 ? p.lu : which == 1 ? p.solve : p.fused;
  if (tasks) std::memcpy(tasks, d.tasks.data(), d.tasks.size() * sizeof(Task));
  if (succ_ptr) std::memcpy(succ_ptr, d.succ_ptr.data(), d.succ_ptr.size() * 4);
  if (succ_idx) std::memcpy(succ_idx, d.succ_idx.data(), d.succ_idx.size() * 4);
  if (level) std::memcpy(level, d.level.data(), d.level.size() * 4);
  if (block_off)
    for (size_t b = 0; b < p.data_off.size(); ++b) {
      block_off[4 * b] = p.data_off[b];
      block_off[4 * b + 1] = p.data_type[b];
      block_off[4 * b + 2] = p.lr_index[b];
      block_off[4 * b + 3] = p.piv_off[b];
    }
  if (lr)
    for (size_t i = 0; i < p.lr.size(); ++i) {
      lr[6 * i] = p.lr[i].u_off;
      lr[6 * i + 1] = p.lr[i].v_off;
      lr[6 * i + 2] = p.lr[i].m;
      lr[6 * i + 3] = p.lr[i].n;
      lr[6 * i + 4] = p.lr[i].cap;
      lr[6 * i + 5] = p.lr[i].type;
    }
  return HM_OK;
}

hm_status hm_dag_seq_export(hm_tree t, const hm_opts* opts, int which, int64_t* nseq, void* seq) {
  if (!t || !opts || !nseq || which < 0 || which > 2) return fail(HM_EINVAL, "bad argument");
  if (!valid_opts(opts)) return fail(HM_EINVAL, "invalid options");
  PlanEntry* pe;
  hm_status st = get_plan(t, opts->prec, opts->max_rank, opts->lazy, true, &pe, -1, opts->coarsen);
  if (st) return st;
  if (which == 2 && (st = trace_fused(t, pe, opts->lazy))) return st;
  const Plan& p = pe->plan;
  const Dag& d = which == 0 ? p.lu : which == 1 ? p.solve : p.fused;
  *nseq = (int64_t)d.seq.size();
  if (seq) std::memcpy(seq, d.seq.data(), d.seq.size() * sizeof(Task));
  return HM_OK;
}

// ----------------------------------------------------------------------------
// The H-matvec tables of a matrix (leaf list, row segments per leaf cluster,
// work vectors); used by h_assemble and hm_import.
static hm_status matrix_tables(hm_matrix_s* A, hipStream_t s) {
  hm_tree t = A->tree;
  const Tree& tr = t->t;
  const Plan& p = A->pe->plan;
  hm_status st;
  // matvec tables
  std::vector<MvLeaf> leaves;
  std::vector<int32_t> lr_leaves;
  std::vector<int32_t> leaf_of_block(tr.bl.size(), -1);
  for (size_t b = 0; b < tr.bl.size(); ++b) {
    const BlockNode& bn = tr.bl[b];
    if (bn.kind == BK_STRUCT) continue;
    MvLeaf L;
    L.r0 = tr.cl[bn.tau].begin;
    L.c0 = tr.cl[bn.sigma].begin;
    L.m = (int32_t)tr.cl[bn.tau].size();
    L.n = (int32_t)tr.cl[bn.sigma].size();
    L.type = VT_F64;
    if (bn.kind == BK_DENSE) {
      L.off = p.data_off[b];
      L.u_off = L.v_off = 0;
      L.lr = -1;
    } else {
      const LrDesc& d = p.lr[p.lr_index[b]];
      L.off = 0;
      L.u_off = d.u_off;
      L.v_off = d.v_off;
      L.lr = p.lr_index[b];
      lr_leaves.push_back((int32_t)leaves.size());
    }
    leaf_of_block[b] = (int32_t)leaves.size();
    leaves.push_back(L);
  }
  // row segments per leaf cluster
  const auto& lb = t->leaf_begin;
  std::vector<std::vector<MvRow>> per(lb.size());
  for (size_t i = 0; i < leaves.size(); ++i) {
    const MvLeaf& L = leaves[i];
    auto it = std::lower_bound(lb.begin(), lb.end(), L.r0);
    for (; it != lb.end() && *it < L.r0 + L.m; ++it) {
      size_t rc = it - lb.begin();
      per[rc].push_back(MvRow{(int32_t)i, (int32_t)(*it - L.r0)});
    }
  }
  std::vector<int32_t> row_ptr(1, 0);
  std::vector<MvRow> segs;
  for (auto& v : per) {
    segs.insert(segs.end(), v.begin(), v.end());
    row_ptr.push_back((int32_t)segs.size());
  }
  if ((st = upload(A->mv_leaves, leaves, s))) return st;
  if ((st = upload(A->mv_lr, lr_leaves, s))) return st;
  if ((st = upload(A->mv_row_ptr, row_ptr, s))) return st;
  if ((st = upload(A->mv_segs, segs, s))) return st;
  if ((st = upload(A->mv_row_begin, t->leaf_begin, s))) return st;
  if ((st = upload(A->mv_row_size, t->leaf_size, s))) return st;
  A->n_lr_leaves = (int64_t)lr_leaves.size();
  A->n_rows = (int64_t)lb.size();
  if (!dev_alloc(A->mv_T, std::max<size_t>(1, p.lr.size()) * kMaxCap * 16 * 8, s) ||
      !dev_alloc(A->mv_x, (size_t)tr.n * 16 * 8, s) || !dev_alloc(A->mv_y, (size_t)tr.n * 16 * 8, s))
    return fail(HM_ENOMEM, "device allocation failed (matvec)");
  return HM_OK;
}

hm_status h_assemble(hm_tree t, int kernel, double diag, const hm_opts* opts, void* stream, hm_matrix* out) {
  if (!t || !out) return fail(HM_EINVAL, "null pointer");
  if (!valid_opts(opts)) return fail(HM_EINVAL, "invalid options");
  if (kernel != HM_LAPLACE3D && kernel != HM_LOG2D) return fail(HM_EINVAL, "unknown kernel");
  hm_status st = device_setup();
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  PlanEntry* pe;
  if ((st = get_plan(t, HM_FP64, opts->max_rank, 0, false, &pe))) return st;
  const Plan& p = pe->plan;
  const Tree& tr = t->t;
  auto A = std::make_unique<hm_matrix_s>();
  A->tree = t;
  A->pe = pe;
  A->kernel = kernel;
  A->diag = diag;
  A->eps = opts->eps;
  A->max_rank = opts->max_rank;
  // A's arena: blocks only (no temporaries, no panel)
  if (!dev_alloc(A->f64, p.blocks_f64 * 8, s) || !dev_alloc(A->ranks, ((size_t)p.nlr_leaf + 1) * 4, s) ||
      !dev_alloc(A->status, 64, s))
    return fail(HM_ENOMEM, "device allocation failed (matrix)");
  HIPCHK(hipMemsetAsync(A->ranks.p, 0, ((size_t)p.nlr_leaf + 1) * 4, s));
  HIPCHK(hipMemsetAsync(A->status.p, 0, 64, s));
  if ((st = upload(A->pts, tr.pts_perm, s))) return st;
  if ((st = upload(A->perm, tr.perm, s))) return st;
  DevBuf lrbuf;
  if ((st = upload(lrbuf, p.lr, s))) return st;
  ExecArgs a = base_args((double*)A->f64.p, nullptr, nullptr, (int32_t*)A->ranks.p, (const LrDesc*)lrbuf.p,
                         opts->eps, opts->max_rank);
  a.status = (int32_t*)A->status.p;
  AsmArgs as{(const double*)A->pts.p, kernel, diag};
  // dense leaves
  std::vector<DenseAsm> dense;
  std::vector<LrAsm> lrs;
  for (size_t b = 0; b < tr.bl.size(); ++b) {
    const BlockNode& bn = tr.bl[b];
    if (bn.kind == BK_DENSE)
      dense.push_back(DenseAsm{p.data_off[b], tr.cl[bn.tau].begin, tr.cl[bn.sigma].begin,
                               (int32_t)tr.cl[bn.tau].size(), (int32_t)tr.cl[bn.sigma].size(), VT_F64, 0});
    else if (bn.kind == BK_LOWRANK)
      lrs.push_back(LrAsm{tr.cl[bn.tau].begin, tr.cl[bn.sigma].begin, p.lr_index[b], 0});
  }
  DevBuf dbuf;
  if ((st = upload(dbuf, dense, s))) return st;
  if (!dense.empty()) {
    hipLaunchKernelGGL(assemble_dense_kernel, dim3((unsigned)dense.size()), dim3(kThreads), 0, s, a, as,
                       (const DenseAsm*)dbuf.p);
    HIPCHK(hipGetLastError());
  }
  // low-rank leaves: ACA in batches bounded by scratch memory, largest first
  std::sort(lrs.begin(), lrs.end(), [&](const LrAsm& x, const LrAsm& y) {
    const LrDesc &dx = p.lr[x.lr], &dy = p.lr[y.lr];
    return dx.m + dx.n > dy.m + dy.n;
  });
  DevBuf lbuf;
  if ((st = upload(lbuf, lrs, s))) return st;
  const int64_t fac_budget = int64_t(2) << 30;
  DevBuf scratch, fac;
  const int maxb = std::max(1, g_nwg);
  if (!dev_alloc(scratch, (size_t)maxb * kScratchPerWg * 8, s)) return fail(HM_ENOMEM, "device allocation failed");
  a.scratch = (double*)scratch.p;
  a.scratch_stride = kScratchPerWg;
  size_t i0 = 0;
  size_t fac_bytes = 0;
  while (i0 < lrs.size()) {
    const LrDesc& d0 = p.lr[lrs[i0].lr];
    // one slot per block: U (m x kMaxK), V (n x kMaxK) and m row flags; the
    // batch is sorted by m + n, so (m0 + n0) bounds every block's m + n, and
    // m + n (not m0) bounds its flags
    int64_t stride = ((int64_t)(d0.m + d0.n) * (kMaxK * 8 + 1) + 255) / 256 * 32;  // doubles
    int64_t cnt = std::min<int64_t>({(int64_t)(lrs.size() - i0), maxb, std::max<int64_t>(1, fac_budget / (stride * 8))});
    size_t need = (size_t)(cnt * stride * 8);
    if (need > fac_bytes) {
      HIPCHK(hipStreamSynchronize(s));
      dev_free(fac);
      if (!dev_alloc(fac, need, s)) return fail(HM_ENOMEM, "device allocation failed (ACA)");
      fac_bytes = need;
    }
    double aca_eps = opts->eps > 0 ? opts->eps * 0.1 : 1e-14;
    hipLaunchKernelGGL(assemble_aca_kernel, dim3((unsigned)cnt), dim3(kThreads), kLdsBytes, s, a, as,
                       (const LrAsm*)lbuf.p + i0, (double*)fac.p, stride, aca_eps);
    HIPCHK(hipGetLastError());
    i0 += cnt;
  }
  HIPCHK(hipStreamSynchronize(s));
  dev_free(fac);
  dev_free(scratch);
  dev_free(dbuf);
  dev_free(lbuf);
  dev_free(lrbuf);
  int32_t stv[4];
  HIPCHK(hipMemcpy(stv, A->status.p, 16, hipMemcpyDeviceToHost));
  if ((st = matrix_tables(A.get(), s))) return st;
  HIPCHK(hipStreamSynchronize(s));
  if (stv[0] & ST_BADOP) return fail(HM_EDEVICE, "internal: an ACA scratch slot is too small");
  *out = A.release();
  if (stv[2] > 0 && opts->max_rank == 0) return fail(HM_ERANK, "compression wanted more than 64 columns");
  return HM_OK;
}

hm_status hm_import(hm_tree t, const hm_opts* opts, const int32_t* ranks, const double* data, int64_t ndata,
                    void* stream, hm_matrix* out) {
  if (!t || !out || !ranks || (!data && ndata > 0)) return fail(HM_EINVAL, "null pointer");
  if (!valid_opts(opts)) return fail(HM_EINVAL, "invalid options");
  const Tree& tr = t->t;
  PlanEntry* pe;
  hm_status st = get_plan(t, HM_FP64, opts->max_rank, 0, false, &pe);
  if (st) return st;
  const Plan& p = pe->plan;
  // check the layout of `data` before touching a device
  int64_t need = 0;
  for (size_t b = 0; b < tr.bl.size(); ++b) {
    const BlockNode& bn = tr.bl[b];
    const int64_t m = tr.cl[bn.tau].size(), n = tr.cl[bn.sigma].size();
    if (bn.kind == BK_DENSE) {
      need += m * n;
    } else if (bn.kind == BK_LOWRANK) {
      const int32_t k = ranks[b];
      if (k < 0) return fail(HM_EINVAL, "negative rank at low-rank block " + std::to_string(b));
      if (k > p.lr[p.lr_index[b]].cap)
        return fail(HM_ERANK, "rank " + std::to_string(k) + " above the capacity of block " + std::to_string(b));
      need += (m + n) * k;
    }
  }
  if (need != ndata) return fail(HM_EINVAL, "data holds " + std::to_string(ndata) + " values, the leaves need " +
                                                std::to_string(need));
  if ((st = device_setup())) return st;
  hipStream_t s = (hipStream_t)stream;
  auto A = std::make_unique<hm_matrix_s>();
  A->tree = t;
  A->pe = pe;
  A->kernel = -1;  // imported: no kernel function
  A->diag = 0.0;
  A->eps = opts->eps;
  A->max_rank = opts->max_rank;
  if (!dev_alloc(A->f64, p.blocks_f64 * 8, s) || !dev_alloc(A->ranks, ((size_t)p.nlr_leaf + 1) * 4, s) ||
      !dev_alloc(A->status, 64, s))
    return fail(HM_ENOMEM, "device allocation failed (matrix)");
  HIPCHK(hipMemsetAsync(A->status.p, 0, 64, s));
  if ((st = upload(A->pts, tr.pts_perm, s))) return st;
  if ((st = upload(A->perm, tr.perm, s))) return st;
  std::vector<int32_t> rk((size_t)p.nlr_leaf + 1, 0);
  double* f = (double*)A->f64.p;
  int64_t off = 0;
  for (size_t b = 0; b < tr.bl.size(); ++b) {
    const BlockNode& bn = tr.bl[b];
    const int64_t m = tr.cl[bn.tau].size(), n = tr.cl[bn.sigma].size();
    if (bn.kind == BK_DENSE) {
      HIPCHK(hipMemcpy(f + p.data_off[b], data + off, (size_t)(m * n) * 8, hipMemcpyHostToDevice));
      off += m * n;
    } else if (bn.kind == BK_LOWRANK) {
      const LrDesc& d = p.lr[p.lr_index[b]];
      const int32_t k = ranks[b];
      rk[p.lr_index[b]] = k;
      if (k > 0) {
        HIPCHK(hipMemcpy(f + d.u_off, data + off, (size_t)(m * k) * 8, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(f + d.v_off, data + off + m * k, (size_t)(n * k) * 8, hipMemcpyHostToDevice));
      }
      off += (m + n) * k;
    }
  }
  HIPCHK(hipMemcpy(A->ranks.p, rk.data(), rk.size() * 4, hipMemcpyHostToDevice));
  if ((st = matrix_tables(A.get(), s))) return st;
  HIPCHK(hipStreamSynchronize(s));
  *out = A.release();
  return HM_OK;
}

void hm_matrix_free(hm_matrix A) {
  if (!A) return;
  for (DevBuf* b : {&A->f64, &A->ranks, &A->pts, &A->perm, &A->mv_leaves, &A->mv_lr, &A->mv_row_ptr, &A->mv_segs,
                    &A->mv_row_begin, &A->mv_row_size, &A->mv_T, &A->mv_x, &A->mv_y, &A->status})
    dev_free(*b);
  delete A;
}

// y = alpha A x + beta y, user ordering
static hm_status matvec_impl(hm_matrix A, double alpha, const double* X, int64_t ldx, double beta, double* Y,
                             int64_t ldy, int64_t nrhs, hipStream_t s) {
  const Plan& p = A->pe->plan;
  const int64_t n = A->tree->t.n;
  ExecArgs a = base_args((double*)A->f64.p, nullptr, nullptr, (int32_t*)A->ranks.p, nullptr, A->eps, A->max_rank);
  for (int64_t c0 = 0; c0 < nrhs; c0 += 16) {
    int nc = (int)std::min<int64_t>(16, nrhs - c0);
    int64_t tot = n * nc;
    unsigned g = (unsigned)((tot + 255) / 256);
    hipLaunchKernelGGL(gather_rows_kernel, dim3(g), dim3(256), 0, s, X + c0 * ldx, ldx,
                       (const int64_t*)A->perm.p, n, nc, (double*)A->mv_x.p, n);
    if (A->n_lr_leaves > 0)
      hipLaunchKernelGGL(matvec_phase1_kernel, dim3((unsigned)A->n_lr_leaves), dim3(kThreads), 0, s, a,
                         (const MvLeaf*)A->mv_leaves.p, (const int32_t*)A->mv_lr.p, (const double*)A->mv_x.p, n, nc,
                         (double*)A->mv_T.p);
    hipLaunchKernelGGL(matvec_phase2_kernel, dim3((unsigned)A->n_rows), dim3(kThreads), 0, s, a,
                       (const MvLeaf*)A->mv_leaves.p, (const int32_t*)A->mv_row_ptr.p, (const MvRow*)A->mv_segs.p,
                       (const int64_t*)A->mv_row_begin.p, (const int32_t*)A->mv_row_size.p,
                       (const double*)A->mv_x.p, n, nc, (const double*)A->mv_T.p, (double*)A->mv_y.p, n, 1.0, 0.0);
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(g), dim3(256), 0, s, (const double*)A->mv_y.p, n,
                       (const int64_t*)A->perm.p, n, nc, Y + c0 * ldy, ldy, alpha, beta);
  }
  HIPCHK(hipGetLastError());
  (void)p;
  return HM_OK;
}

hm_status h_matvec(hm_matrix A, double alpha, const double* X, int64_t ldx, double beta, double* Y, int64_t ldy,
                   int64_t nrhs, void* stream) {
  if (!A || !X || !Y) return fail(HM_EINVAL, "null pointer");
  const int64_t n = A->tree->t.n;
  if (nrhs < 0 || ldx < n || ldy < n) return fail(HM_EINVAL, "bad leading dimension or nrhs");
  if (nrhs == 0) return HM_OK;
  hm_status st = device_setup();
  if (st) return st;
  return matvec_impl(A, alpha, X, ldx, beta, Y, ldy, nrhs, (hipStream_t)stream);
}

// ----------------------------------------------------------------------------
// ... and uploaded on first use.
static hm_status get_fused(hm_tree t, PlanEntry* pe, int lazy, hipStream_t s) {
  hm_status st0 = trace_fused(t, pe, lazy);
  if (st0) return st0;
  if (!pe->fused_uploaded) {
    hm_status st = upload_dag(pe->plan.fused, pe->fused, s);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(s));
    pe->fused_uploaded = true;
  }
  return HM_OK;
}

// h_lu, and with B != NULL h_lu_solve: the first min(nrhs, 64) columns of B
// are substituted inside the factorization's DAG.
static hm_status lu_impl(hm_matrix A, const hm_opts* opts, void* stream, hm_lu* out, int64_t* info, double* B,
                         int64_t ldb, int64_t nrhs) {
  if (!A || !out) return fail(HM_EINVAL, "null pointer");
  if (!valid_opts(opts)) return fail(HM_EINVAL, "invalid options");
  if (opts->max_rank != A->max_rank) return fail(HM_EINVAL, "max_rank differs from the assembled matrix");
  const bool fused = B != nullptr && nrhs > 0;
  if (fused && ldb < A->tree->t.n) return fail(HM_EINVAL, "ldb < n");
  hm_status st = device_setup();
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  hm_tree t = A->tree;
  PlanEntry* pe;
  if ((st = get_plan(t, opts->prec, opts->max_rank, opts->lazy, true, &pe, -1, opts->coarsen))) return st;
  if (fused && (st = get_fused(t, pe, opts->lazy, s))) return st;
  if ((st = ensure_uploaded(pe, s))) return st;
  const Plan& p = pe->plan;
  const DevDag& dag = fused ? pe->fused : pe->lu;
  const Plan& pa = A->pe->plan;
  auto F = std::make_unique<hm_lu_s>();
  F->tree = t;
  F->pe = pe;
  F->prec = opts->prec;
  F->exec = opts->exec;
  F->eps = opts->eps;
  F->max_rank = opts->max_rank;
  std::memset(&F->stats, 0, sizeof(F->stats));
  if (!dev_alloc(F->f64, p.n_f64 * 8, s) || !dev_alloc(F->f32, p.n_f32 * 4, s) ||
      !dev_alloc(F->piv, std::max<int64_t>(1, p.n_piv) * 4, s) || !dev_alloc(F->ranks, p.nranks * 4, s))
    return fail(HM_ENOMEM, "device allocation failed (factors)");
  if ((st = upload(F->perm, t->t.perm, s))) return st;
  F->dag_ntasks = dag.ntasks;
  if ((st = exec_state_alloc(F->lu_st, dag.ntasks, s))) return st;
  // HM_DEBUG_TRACE=1 records timing and shape information of every H-LU task
  if (const char* e = getenv("HM_DEBUG_TRACE"))
    if (e[0] == '1') {
      if (!dev_alloc(F->lu_st.trace, (size_t)dag.ntasks * kTraceWords * 8, s))
        return fail(HM_ENOMEM, "device allocation failed (trace)");
      HIPCHK(hipMemsetAsync(F->lu_st.trace.p, 0, (size_t)dag.ntasks * kTraceWords * 8, s));
    }
  if ((st = exec_state_alloc(F->solve_st, pe->solve.ntasks, s))) return st;
  // and of every substitution task (the last pass of h_solve is kept)
  if (const char* e = getenv("HM_DEBUG_TRACE"))
    if (e[0] == '1') {
      if (!dev_alloc(F->solve_st.trace, (size_t)std::max<int64_t>(1, pe->solve.ntasks) * kTraceWords * 8, s))
        return fail(HM_ENOMEM, "device allocation failed (trace)");
      HIPCHK(hipMemsetAsync(F->solve_st.trace.p, 0, (size_t)std::max<int64_t>(1, pe->solve.ntasks) * kTraceWords * 8, s));
    }
  // copy A into the factor layout
  HIPCHK(hipMemsetAsync(F->ranks.p, 0, p.nranks * 4, s));
  HIPCHK(hipMemcpyAsync(F->ranks.p, A->ranks.p, (size_t)p.nlr_leaf * 4, hipMemcpyDeviceToDevice, s));
  if (opts->prec == HM_FP64) {
    HIPCHK(hipMemcpyAsync(F->f64.p, A->f64.p, pa.blocks_f64 * 8, hipMemcpyDeviceToDevice, s));
  } else {
    // The copy list depends only on the two layouts: built and uploaded on
    // the first call, reused while the matrices come from that same
    // assembly layout (another layout gets a list of its own for the call).
    auto build_list = [&](std::vector<CopyDesc>& cd) {
      const Tree& tr = t->t;
      for (size_t b = 0; b < tr.bl.size(); ++b) {
        const BlockNode& bn = tr.bl[b];
        if (bn.kind == BK_DENSE) {
          int64_t cnt = tr.cl[bn.tau].size() * tr.cl[bn.sigma].size();
          cd.push_back(CopyDesc{pa.data_off[b], p.data_off[b], cnt, p.data_type[b], 0});
        } else if (bn.kind == BK_LOWRANK) {
          const LrDesc& da = pa.lr[pa.lr_index[b]];
          const LrDesc& dl = p.lr[p.lr_index[b]];
          cd.push_back(CopyDesc{da.u_off, dl.u_off, (int64_t)da.m * da.cap, dl.type, 0});
          cd.push_back(CopyDesc{da.v_off, dl.v_off, (int64_t)da.n * da.cap, dl.type, 0});
        }
      }
    };
    const CopyDesc* list = nullptr;
    int64_t nlist = 0;
    DevBuf cbuf;
    std::vector<CopyDesc> cd;  // the host source of an upload lives until it is done
    {
      std::lock_guard<std::mutex> lk(t->mu);
      if (!pe->conv_src) {
        build_list(cd);
        if ((st = upload(pe->conv, cd, s))) {
          dev_free(pe->conv);
          return st;
        }
        HIPCHK(hipStreamSynchronize(s));
        pe->nconv = (int64_t)cd.size();
        pe->conv_src = A->pe;
        cd.clear();
      }
      if (pe->conv_src == A->pe) {
        list = (const CopyDesc*)pe->conv.p;
        nlist = pe->nconv;
      }
    }
    if (!list) {
      build_list(cd);
      if ((st = upload(cbuf, cd, s))) return st;
      list = (const CopyDesc*)cbuf.p;
      nlist = (int64_t)cd.size();
    }
    if (nlist > 0)
      hipLaunchKernelGGL(convert_blocks_kernel, dim3((unsigned)nlist), dim3(256), 0, s, (const double*)A->f64.p,
                         (double*)F->f64.p, (float*)F->f32.p, list);
    HIPCHK(hipGetLastError());
    if (cbuf.p) {
      HIPCHK(hipStreamSynchronize(s));
      dev_free(cbuf);
    }
  }
  DevBuf scratch;
  if (!dev_alloc(scratch, (size_t)g_nwg * kScratchPerWg * 8, s)) return fail(HM_ENOMEM, "device allocation failed");
  ExecArgs a = base_args((double*)F->f64.p, (float*)F->f32.p, (int32_t*)F->piv.p, (int32_t*)F->ranks.p,
                         (const LrDesc*)pe->lr.p, opts->eps, opts->max_rank);
  a.scratch = (double*)scratch.p;
  a.scratch_stride = kScratchPerWg;
  const int64_t n = t->t.n;
  const int nc = fused ? (int)std::min<int64_t>(nrhs, p.nrhs_cap) : 0;
  double* panel = (double*)F->f64.p + p.panel_off;
  const unsigned gr = (unsigned)((n * nc + 255) / 256);
  if (fused) {
    hipLaunchKernelGGL(set_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)F->ranks.p + p.nrhs_slot, nc, 0, 0, 0, 1);
    hipLaunchKernelGGL(gather_rows_kernel, dim3(gr), dim3(256), 0, s, (const double*)B, ldb,
                       (const int64_t*)F->perm.p, n, nc, panel, n);
    HIPCHK(hipGetLastError());
  }
  float ms = 0.f;
  st = run_dag(dag, a, F->lu_st, opts->exec, s, &ms, fused ? DAG_FUSED : DAG_LU);
  if (st) return st;
  if (fused) {
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(gr), dim3(256), 0, s, (const double*)panel, n,
                       (const int64_t*)F->perm.p, n, nc, B, ldb, 1.0, 0.0);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(s));
  dev_free(scratch);
  int32_t stv[4];
  unsigned long long ctr[kCtrSize];
  HIPCHK(hipMemcpy(stv, F->lu_st.status.p, 16, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ctr, F->lu_st.counters.p, sizeof(ctr), hipMemcpyDeviceToHost));
  for (int k = 0; k < OP_COUNT; ++k) F->stats.op_busy_ms[k] = (double)ctr[kCtrBusy + k] / (double)g_clock_khz;
  for (int k = 0; k < 12; ++k) F->stats.trunc_phase_ms[k] = (double)ctr[kCtrPhase + k] / (double)g_clock_khz;
  double ntr = (double)std::max<unsigned long long>(1, ctr[kCtrCount + OP_TRUNC] + ctr[kCtrCount + OP_TRUNC2]);
  F->stats.trunc_mean_k = ctr[kCtrK] / ntr;
  F->stats.trunc_mean_mn = ctr[kCtrMN] / ntr;
  F->stats.ntasks = dag.ntasks;
  F->stats.nedges = dag.nedges;
  F->stats.nlevels = dag.nlevels;
  for (int k = 0; k < OP_COUNT; ++k) F->stats.tasks_by_op[k] = dag.tasks_by_op[k];
  F->stats.bytes_alg = (int64_t)ctr[0];
  F->stats.flops_alg = (int64_t)ctr[1];
  F->stats.exec_ms = ms;
  F->stats.temp_bytes = p.temp_bytes;
  F->stats.rank_overflows = stv[2];
  if (info) *info = 0;
  if (stv[0] & ST_TIMEOUT) return fail(HM_EDEVICE, "executor timed out waiting for a task");
  if (stv[0] & ST_BADOP) return fail(HM_EDEVICE, "internal: a task the executor does not run");
  if (stv[0] & ST_SINGULAR) {
    if (info) *info = stv[1];
    hm_lu_s* f = F.release();
    hm_lu_free(f);
    return fail(HM_ESINGULAR, "exact zero pivot in a diagonal leaf");
  }
  *out = F.release();
  // the columns beyond the fused panel are solved before a rank overflow is
  // reported, so that every column of B holds the solution either way
  if (fused && nrhs > nc) {
    hm_status st2 = h_solve(*out, nullptr, B + (int64_t)nc * ldb, ldb, nrhs - nc, 0.0, 0, stream, nullptr, nullptr);
    if (st2) return st2;
  }
  if (stv[2] > 0 && opts->max_rank == 0) return fail(HM_ERANK, "a truncation wanted more than 64 columns");
  return HM_OK;
}

hm_status h_lu(hm_matrix A, const hm_opts* opts, void* stream, hm_lu* out, int64_t* info) {
  return lu_impl(A, opts, stream, out, info, nullptr, 0, 0);
}

hm_status h_lu_solve(hm_matrix A, const hm_opts* opts, double* B, int64_t ldb, int64_t nrhs, void* stream, hm_lu* out,
                     int64_t* info) {
  if (!B && nrhs > 0) return fail(HM_EINVAL, "null pointer");
  if (nrhs < 0) return fail(HM_EINVAL, "nrhs < 0");
  return lu_impl(A, opts, stream, out, info, B, ldb, nrhs);
}

// ---------------------------------------------------------------------------
// h_lu_batched: the H-LUs of several matrices as one DAG on one launch
// ---------------------------------------------------------------------------
// The batch's factor storage: one arena per element type holding every
// instance's plan layout at its own base; released with the last handle.
struct BatchArena {
  DevBuf f64, f32, piv, ranks;
  ~BatchArena() {
    dev_free(f64);
    dev_free(f32);
    dev_free(piv);
    dev_free(ranks);
  }
};

// Span of the temporaries of one instance of a batch: the batch's total
// (HM_BATCH_TEMP_GB, default 16 GiB) shared in proportion to n, at least
// 64 MiB and at most the single-matrix span.
static int64_t batch_temp_budget(int64_t n, int64_t n_total) {
  double gb = 16.0;
  if (const char* e = getenv("HM_BATCH_TEMP_GB")) gb = std::max(1e-3, atof(e));
  const double total = gb * (double)(1ll << 30);
  int64_t b = (int64_t)(total * (double)n / (double)std::max<int64_t>(1, n_total));
  b = std::max<int64_t>(b, int64_t(64) << 20);
  return std::min<int64_t>(b, temp_budget()) >> 20 << 20;
}

static int64_t align64(int64_t x) { return (x + 63) / 64 * 64; }

// Shift a task record of instance-local storage to the batch arena.
static void relocate_task(Task& t, int64_t b64, int64_t b32, int64_t bpiv, int32_t brank, int32_t brow) {
  for (View* v : {&t.y, &t.a, &t.b, &t.x}) {
    if (v->type == VT_F64) v->off += b64;
    else if (v->type == VT_F32) v->off += b32;
    if (v->rank_id >= 0) v->rank_id += brank;
    if ((v->dyn & DYN_COLS2) && v->rank_id2 >= 0) v->rank_id2 += brank;
  }
  if ((t.op == OP_TRUNC || t.op == OP_TRUNC2) && t.lr >= 0) t.lr += brank;
  if ((t.op == OP_GETRF || t.op == OP_TRSM_L || t.op == OP_TRSM_UT || t.op == OP_TRSM_U) && t.piv >= 0)
    t.piv += bpiv;
  if (t.op == OP_GETRF) t.row0 += brow;
}

// Host side of a batch: every instance's traced plan and its bases in the
// batch arena and the combined DAG.
struct BatchLayout {
  std::vector<PlanEntry*> pes;
  std::vector<int64_t> b64, b32, bpiv, bt, be;
  std::vector<int32_t> brank, brow;
  int64_t n64 = 0, n32 = 0, npiv = 0, nrk = 0, ntask = 0, nedge = 0, nroot = 0, nrow = 0, nlev = 0;
  std::vector<int32_t> level_ptr;  // levels of the union (level l = every instance's level l)
};

// Trace every tree's plan (in parallel threads, host only) and lay the batch out.
static hm_status batch_layout(const std::vector<hm_tree>& trees, const hm_opts* opts, BatchLayout& L) {
  const int count = (int)trees.size();
  int64_t n_total = 0;
  for (hm_tree t : trees) n_total += t->t.n;
  L.pes.assign(count, nullptr);
  std::vector<hm_status> sts(count, HM_OK);
  std::vector<std::string> errs(count);
  {
    std::atomic<int> next{0};
    const int nth = std::max(1, std::min<int>(count, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int w = 0; w < nth; ++w)
      pool.emplace_back([&]() {
        for (int i = next++; i < count; i = next++) {
          sts[i] = get_plan(trees[i], opts->prec, opts->max_rank, opts->lazy, true, &L.pes[i],
                            batch_temp_budget(trees[i]->t.n, n_total), opts->coarsen);
          if (sts[i]) errs[i] = g_err;
        }
      });
    for (auto& th : pool) th.join();
  }
  for (int i = 0; i < count; ++i)
    if (sts[i]) return fail(sts[i], "instance " + std::to_string(i) + ": " + errs[i]);
  for (auto* v : {&L.b64, &L.b32, &L.bpiv, &L.bt, &L.be}) v->assign(count, 0);
  L.brank.assign(count, 0);
  L.brow.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    const Plan& p = L.pes[i]->plan;
    L.b64[i] = L.n64;
    L.b32[i] = L.n32;
    L.bpiv[i] = L.npiv;
    L.brank[i] = (int32_t)L.nrk;
    L.brow[i] = (int32_t)L.nrow;
    L.bt[i] = L.ntask;
    L.be[i] = L.nedge;
    L.n64 = align64(L.n64 + p.n_f64);
    L.n32 = align64(L.n32 + p.n_f32);
    L.npiv = align64(L.npiv + p.n_piv);
    L.nrk += p.nranks;
    L.nrow += trees[i]->t.n;
    L.ntask += (int64_t)p.lu.tasks.size();
    L.nedge += p.lu.nedges;
    L.nroot += (int64_t)p.lu.roots.size();
    L.nlev = std::max<int64_t>(L.nlev, (int64_t)p.lu.level_ptr.size() - 1);
  }
  if (L.ntask >= INT32_MAX || L.nedge >= INT32_MAX || L.nrk >= INT32_MAX || L.nrow >= INT32_MAX)
    return fail(HM_EINVAL, "batch too large for 32-bit task, edge or rank indices");
  L.level_ptr.assign((size_t)L.nlev + 1, 0);
  for (int i = 0; i < count; ++i) {
    const Dag& d = L.pes[i]->plan.lu;
    for (int64_t l = 0; l + 1 < (int64_t)d.level_ptr.size(); ++l)
      L.level_ptr[l + 1] += d.level_ptr[l + 1] - d.level_ptr[l];
  }
  for (int64_t l = 0; l < L.nlev; ++l) L.level_ptr[l + 1] += L.level_ptr[l];
  return HM_OK;
}

// Instance i's part of the combined DAG: relocated task records, successor
// pointers (without the final entry) and successor indices.
static void batch_instance(const BatchLayout& L, int i, std::vector<Task>& tk, std::vector<int32_t>& sp,
                           std::vector<int32_t>& si) {
  const Dag& d = L.pes[i]->plan.lu;
  tk = d.tasks;
  for (Task& t : tk) relocate_task(t, L.b64[i], L.b32[i], L.bpiv[i], L.brank[i], L.brow[i]);
  sp.assign(d.succ_ptr.begin(), d.succ_ptr.end() - 1);
  for (auto& x : sp) x += (int32_t)L.be[i];
  si = d.succ_idx;
  for (auto& x : si) x += (int32_t)L.bt[i];
}

// The low-rank descriptors of the batch, indexed like its rank slots (the
// slots of a solve's column count get an empty descriptor).
static std::vector<LrDesc> batch_lr(const BatchLayout& L) {
  std::vector<LrDesc> lr((size_t)L.nrk);
  std::memset(lr.data(), 0, lr.size() * sizeof(LrDesc));
  for (size_t i = 0; i < L.pes.size(); ++i) {
    const Plan& p = L.pes[i]->plan;
    for (size_t k = 0; k < p.lr.size(); ++k) {
      LrDesc d = p.lr[k];
      d.u_off += d.type == VT_F64 ? L.b64[i] : L.b32[i];
      d.v_off += d.type == VT_F64 ? L.b64[i] : L.b32[i];
      lr[(size_t)L.brank[i] + k] = d;
    }
  }
  return lr;
}

// Tasks of the union in level order (level l of every instance in turn).
static std::vector<int32_t> batch_order(const BatchLayout& L) {
  std::vector<int32_t> order((size_t)L.ntask);
  std::vector<int64_t> pos(L.level_ptr.begin(), L.level_ptr.end() - 1);
  for (size_t i = 0; i < L.pes.size(); ++i) {
    const Dag& d = L.pes[i]->plan.lu;
    for (int64_t l = 0; l + 1 < (int64_t)d.level_ptr.size(); ++l)
      for (int32_t k = d.level_ptr[l]; k < d.level_ptr[l + 1]; ++k)
        order[pos[l]++] = (int32_t)(d.level_order[k] + L.bt[i]);
  }
  return order;
}

// The device copy of the last batch's combined DAG, its low-rank descriptors
// and the copy descriptors of every instance's A, kept for the next call on
// the same plans (a batch refactored again skips the relocation and upload).
struct BatchCache {
  std::vector<PlanEntry*> key;
  int order_mode = 0;
  DevDag dd;
  DevBuf lr;
  std::vector<DevBuf> copies;
  ~BatchCache() {
    for (DevBuf* b : {&dd.tasks, &dd.indeg, &dd.succ_ptr, &dd.succ_idx, &dd.roots, &dd.order, &lr}) dev_free(*b);
    for (DevBuf& b : copies) dev_free(b);
  }
};
static std::mutex g_batch_mu;
static std::unique_ptr<BatchCache> g_batch;

static void batch_cache_drop(hm_tree t) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (!g_batch) return;
  for (auto& kv : t->plans)
    for (PlanEntry* pe : g_batch->key)
      if (pe == kv.second.get()) {
        g_batch.reset();
        return;
      }
}

// Relocate and upload the combined DAG of a batch.  order_mode 1 queues the
// roots of the instances with the most tasks first.
static hm_status batch_upload(const BatchLayout& L, const hm_matrix* As, int order_mode, hipStream_t s,
                              BatchCache& bc) {
  const int count = (int)L.pes.size();
  DevDag& dd = bc.dd;
  dd.ntasks = L.ntask;
  dd.nedges = L.nedge;
  dd.nlevels = L.nlev;
  dd.nroots = (int32_t)L.nroot;
  if (!dev_alloc(dd.tasks, (size_t)L.ntask * sizeof(Task), s) || !dev_alloc(dd.indeg, (size_t)L.ntask * 4, s) ||
      !dev_alloc(dd.succ_ptr, (size_t)(L.ntask + 1) * 4, s) ||
      !dev_alloc(dd.succ_idx, (size_t)std::max<int64_t>(1, L.nedge) * 4, s) ||
      !dev_alloc(dd.roots, (size_t)std::max<int64_t>(1, L.nroot) * 4, s) ||
      !dev_alloc(dd.order, (size_t)L.ntask * 4, s))
    return fail(HM_ENOMEM, "device allocation failed (batch DAG)");
  dd.level_ptr = L.level_ptr;
  std::vector<int> inst(count);
  for (int i = 0; i < count; ++i) inst[i] = i;
  if (order_mode == 1)
    std::stable_sort(inst.begin(), inst.end(), [&](int x, int y) {
      return L.pes[x]->plan.lu.tasks.size() > L.pes[y]->plan.lu.tasks.size();
    });
  std::vector<int32_t> roots_all;
  roots_all.reserve((size_t)L.nroot);
  for (int i : inst)
    for (int32_t r : L.pes[i]->plan.lu.roots) roots_all.push_back((int32_t)(r + L.bt[i]));
  // relocation on several host threads, uploads in instance order
  std::vector<std::vector<Task>> tk(count);
  std::vector<std::vector<int32_t>> sp(count), si(count);
  {
    std::atomic<int> next{0};
    const int nth = std::max(1, std::min<int>(count, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int w = 0; w < nth; ++w)
      pool.emplace_back([&]() {
        for (int i = next++; i < count; i = next++) batch_instance(L, i, tk[i], sp[i], si[i]);
      });
    for (auto& th : pool) th.join();
  }
  for (int i = 0; i < count; ++i) {
    const Dag& d = L.pes[i]->plan.lu;
    if (!tk[i].empty()) {
      HIPCHK(hipMemcpy((Task*)dd.tasks.p + L.bt[i], tk[i].data(), tk[i].size() * sizeof(Task),
                       hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy((int32_t*)dd.indeg.p + L.bt[i], d.indeg.data(), d.indeg.size() * 4, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy((int32_t*)dd.succ_ptr.p + L.bt[i], sp[i].data(), sp[i].size() * 4, hipMemcpyHostToDevice));
    }
    if (!si[i].empty())
      HIPCHK(hipMemcpy((int32_t*)dd.succ_idx.p + L.be[i], si[i].data(), si[i].size() * 4, hipMemcpyHostToDevice));
    std::vector<Task>().swap(tk[i]);
    std::vector<int32_t>().swap(sp[i]);
    std::vector<int32_t>().swap(si[i]);
  }
  const int32_t last = (int32_t)L.nedge;
  HIPCHK(hipMemcpy((int32_t*)dd.succ_ptr.p + L.ntask, &last, 4, hipMemcpyHostToDevice));
  if (!roots_all.empty())
    HIPCHK(hipMemcpy(dd.roots.p, roots_all.data(), roots_all.size() * 4, hipMemcpyHostToDevice));
  const std::vector<int32_t> order_all = batch_order(L);
  HIPCHK(hipMemcpy(dd.order.p, order_all.data(), order_all.size() * 4, hipMemcpyHostToDevice));
  hm_status st;
  if ((st = upload(bc.lr, batch_lr(L), s))) return st;
  // copy descriptors of every instance's A (assembly layout -> batch layout)
  bc.copies.resize(count);
  for (int i = 0; i < count; ++i) {
    hm_matrix A = As[i];
    const Plan& p = L.pes[i]->plan;
    const Plan& pa = A->pe->plan;
    const Tree& tr = A->tree->t;
    std::vector<CopyDesc> cd;
    for (size_t b = 0; b < tr.bl.size(); ++b) {
      const BlockNode& bn = tr.bl[b];
      if (bn.kind == BK_DENSE) {
        int64_t cnt = tr.cl[bn.tau].size() * tr.cl[bn.sigma].size();
        int64_t dst = p.data_off[b] + (p.data_type[b] == VT_F64 ? L.b64[i] : L.b32[i]);
        cd.push_back(CopyDesc{pa.data_off[b], dst, cnt, p.data_type[b], 0});
      } else if (bn.kind == BK_LOWRANK) {
        const LrDesc& da = pa.lr[pa.lr_index[b]];
        const LrDesc& dl = p.lr[p.lr_index[b]];
        const int64_t base = dl.type == VT_F64 ? L.b64[i] : L.b32[i];
        cd.push_back(CopyDesc{da.u_off, dl.u_off + base, (int64_t)da.m * da.cap, dl.type, 0});
        cd.push_back(CopyDesc{da.v_off, dl.v_off + base, (int64_t)da.n * da.cap, dl.type, 0});
      }
    }
    if ((st = upload(bc.copies[i], cd, s))) return st;
    HIPCHK(hipStreamSynchronize(s));
  }
  return HM_OK;
}

hm_status h_lu_batched(const hm_matrix* As, int count, const hm_opts* opts, void* stream, hm_lu* outs,
                       int64_t* infos) {
  if (!As || !outs || count < 1) return fail(HM_EINVAL, "null pointer or count < 1");
  if (!valid_opts(opts)) return fail(HM_EINVAL, "invalid options");
  for (int i = 0; i < count; ++i) {
    outs[i] = nullptr;
    if (infos) infos[i] = 0;
    if (!As[i]) return fail(HM_EINVAL, "null matrix in the batch");
    if (As[i]->max_rank != opts->max_rank) return fail(HM_EINVAL, "max_rank differs from an assembled matrix");
  }
  hm_status st = device_setup();
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<hm_tree> trees(count);
  for (int i = 0; i < count; ++i) trees[i] = As[i]->tree;
  BatchLayout L;
  if ((st = batch_layout(trees, opts, L))) return st;
  const std::vector<PlanEntry*>& pes = L.pes;
  const auto &b64 = L.b64, &b32 = L.b32, &bpiv = L.bpiv, &bt = L.bt, &be = L.be;
  const auto &brank = L.brank, &brow = L.brow;
  const int64_t n64 = L.n64, n32 = L.n32, npiv = L.npiv, nrk = L.nrk, ntask = L.ntask, nedge = L.nedge,
                nroot = L.nroot, nlev = L.nlev;
  for (int i = 0; i < count; ++i)
    if ((st = ensure_solve_uploaded(pes[i], s))) return st;
  auto arena = std::make_shared<BatchArena>();
  if (!dev_alloc(arena->f64, (size_t)std::max<int64_t>(1, n64) * 8, s) ||
      !dev_alloc(arena->f32, (size_t)std::max<int64_t>(1, n32) * 4, s) ||
      !dev_alloc(arena->piv, (size_t)std::max<int64_t>(1, npiv) * 4, s) ||
      !dev_alloc(arena->ranks, (size_t)std::max<int64_t>(1, nrk) * 4, s))
    return fail(HM_ENOMEM, "device allocation failed (batch factors)");
  std::lock_guard<std::mutex> cache_lock(g_batch_mu);
  const int order_mode = g_tuning.batch_order;
  if (!g_batch || g_batch->key != pes || g_batch->order_mode != order_mode) {
    g_batch.reset();
    auto bc = std::make_unique<BatchCache>();
    bc->key = pes;
    bc->order_mode = order_mode;
    if ((st = batch_upload(L, As, order_mode, s, *bc))) return st;
    g_batch = std::move(bc);
  }
  const DevDag& dd = g_batch->dd;
  // every instance's A into its part of the arena (FP64 copy, or FP32 conversion
  // of the off-diagonal blocks), ranks from the assembly
  hipLaunchKernelGGL(fill_i32_kernel, dim3(256), dim3(256), 0, s, (int32_t*)arena->ranks.p, 0, nrk);
  for (int i = 0; i < count; ++i) {
    HIPCHK(hipMemcpyAsync((int32_t*)arena->ranks.p + brank[i], As[i]->ranks.p, (size_t)pes[i]->plan.nlr_leaf * 4,
                          hipMemcpyDeviceToDevice, s));
    const DevBuf& cb = g_batch->copies[i];
    const int64_t ncd = (int64_t)(cb.bytes / sizeof(CopyDesc));
    if (ncd > 0)
      hipLaunchKernelGGL(convert_blocks_kernel, dim3((unsigned)ncd), dim3(256), 0, s, (const double*)As[i]->f64.p,
                         (double*)arena->f64.p, (float*)arena->f32.p, (const CopyDesc*)cb.p);
  }
  HIPCHK(hipGetLastError());
  ExecState es;
  if ((st = exec_state_alloc(es, ntask, s))) return st;
  DevBuf scratch;
  if (!dev_alloc(scratch, (size_t)g_nwg * kScratchPerWg * 8, s)) return fail(HM_ENOMEM, "device allocation failed");
  ExecArgs a = base_args((double*)arena->f64.p, (float*)arena->f32.p, (int32_t*)arena->piv.p,
                         (int32_t*)arena->ranks.p, (const LrDesc*)g_batch->lr.p, opts->eps, opts->max_rank);
  a.scratch = (double*)scratch.p;
  a.scratch_stride = kScratchPerWg;
  float ms = 0.f;
  st = run_dag(dd, a, es, opts->exec, s, &ms, DAG_LU);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(s));
  int32_t stv[4];
  unsigned long long ctr[kCtrSize];
  HIPCHK(hipMemcpy(stv, es.status.p, 16, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ctr, es.counters.p, sizeof(ctr), hipMemcpyDeviceToHost));
  dev_free(scratch);
  exec_state_free(es);
  if (stv[0] & ST_TIMEOUT) return fail(HM_EDEVICE, "executor timed out waiting for a task");
  if (stv[0] & ST_BADOP) return fail(HM_EDEVICE, "internal: a task the executor does not run");
  if (stv[0] & ST_SINGULAR) {
    // the first exact zero pivot (smallest batch row): report it at its instance
    int i = 0;
    while (i + 1 < count && brow[i + 1] <= stv[1]) ++i;
    if (infos)
      for (int k = 0; k < count; ++k) infos[k] = k == i ? stv[1] - brow[i] : -1;
    return fail(HM_ESINGULAR, "exact zero pivot in a diagonal leaf of instance " + std::to_string(i));
  }
  // one handle per instance over its slices of the arena
  hm_lu_stats bst;
  std::memset(&bst, 0, sizeof(bst));
  for (int k = 0; k < OP_COUNT; ++k) bst.op_busy_ms[k] = (double)ctr[kCtrBusy + k] / (double)g_clock_khz;
  for (int k = 0; k < 12; ++k) bst.trunc_phase_ms[k] = (double)ctr[kCtrPhase + k] / (double)g_clock_khz;
  double ntr = (double)std::max<unsigned long long>(1, ctr[kCtrCount + OP_TRUNC] + ctr[kCtrCount + OP_TRUNC2]);
  bst.trunc_mean_k = ctr[kCtrK] / ntr;
  bst.trunc_mean_mn = ctr[kCtrMN] / ntr;
  bst.ntasks = ntask;
  bst.nedges = nedge;
  bst.nlevels = nlev;
  bst.bytes_alg = (int64_t)ctr[0];
  bst.flops_alg = (int64_t)ctr[1];
  bst.exec_ms = ms;
  bst.rank_overflows = stv[2];
  for (int i = 0; i < count; ++i) {
    std::lock_guard<std::mutex> lk(As[i]->tree->mu);  // the counts are filled on first use
    const int64_t* c = lu_op_counts(pes[i]);
    for (int k = 0; k < OP_COUNT; ++k) bst.tasks_by_op[k] += c[k];
  }
  std::vector<std::unique_ptr<hm_lu_s>> made(count);
  for (int i = 0; i < count; ++i) {
    const Plan& p = pes[i]->plan;
    auto F = std::make_unique<hm_lu_s>();
    F->tree = As[i]->tree;
    F->pe = pes[i];
    F->prec = opts->prec;
    F->exec = opts->exec;
    F->eps = opts->eps;
    F->max_rank = opts->max_rank;
    F->dag_ntasks = 0;
    auto slice = [](DevBuf& dst, const DevBuf& src, int64_t off_bytes, int64_t bytes) {
      dst.p = (char*)src.p + off_bytes;
      dst.bytes = (size_t)bytes;
      dst.stream = src.stream;
      dst.owned = false;
    };
    slice(F->f64, arena->f64, b64[i] * 8, p.n_f64 * 8);
    slice(F->f32, arena->f32, b32[i] * 4, p.n_f32 * 4);
    slice(F->piv, arena->piv, bpiv[i] * 4, std::max<int64_t>(1, p.n_piv) * 4);
    slice(F->ranks, arena->ranks, (int64_t)brank[i] * 4, (int64_t)p.nranks * 4);
    F->arena = arena;
    if ((st = upload(F->perm, F->tree->t.perm, s))) return st;
    if ((st = exec_state_alloc(F->solve_st, pes[i]->solve.ntasks, s))) return st;
    F->stats = bst;
    made[i] = std::move(F);
  }
  HIPCHK(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) outs[i] = made[i].release();
  if (stv[2] > 0 && opts->max_rank == 0) return fail(HM_ERANK, "a truncation wanted more than 64 columns");
  return HM_OK;
}

hm_status hm_batch_dag_export(const hm_tree* trees, int count, const hm_opts* opts, int64_t* sizes, void* tasks,
                              int32_t* succ_ptr, int32_t* succ_idx, int32_t* order, int32_t* level_ptr, int64_t* lr,
                              int64_t* bases) {
  if (!trees || count < 1 || !opts || !sizes) return fail(HM_EINVAL, "bad argument");
  if (opts->max_rank < 0 || opts->max_rank > kMaxCap) return fail(HM_EINVAL, "max_rank must be in [0, 64]");
  std::vector<hm_tree> tv(trees, trees + count);
  for (hm_tree t : tv)
    if (!t) return fail(HM_EINVAL, "null tree in the batch");
  BatchLayout L;
  hm_status st = batch_layout(tv, opts, L);
  if (st) return st;
  sizes[0] = L.ntask;
  sizes[1] = L.nedge;
  sizes[2] = L.nlev;
  sizes[3] = L.n64;
  sizes[4] = L.n32;
  sizes[5] = L.npiv;
  sizes[6] = L.nrk;
  std::vector<Task> tk;
  std::vector<int32_t> sp, si;
  for (int i = 0; i < count; ++i) {
    if (!tasks && !succ_ptr && !succ_idx) break;
    batch_instance(L, i, tk, sp, si);
    if (tasks) std::memcpy((Task*)tasks + L.bt[i], tk.data(), tk.size() * sizeof(Task));
    if (succ_ptr) std::memcpy(succ_ptr + L.bt[i], sp.data(), sp.size() * 4);
    if (succ_idx) std::memcpy(succ_idx + L.be[i], si.data(), si.size() * 4);
  }
  if (succ_ptr) succ_ptr[L.ntask] = (int32_t)L.nedge;
  if (order) {
    const std::vector<int32_t> o = batch_order(L);
    std::memcpy(order, o.data(), o.size() * 4);
  }
  if (level_ptr) std::memcpy(level_ptr, L.level_ptr.data(), L.level_ptr.size() * 4);
  if (lr) {
    const std::vector<LrDesc> d = batch_lr(L);
    for (size_t k = 0; k < d.size(); ++k) {
      lr[6 * k] = d[k].u_off;
      lr[6 * k + 1] = d[k].v_off;
      lr[6 * k + 2] = d[k].m;
      lr[6 * k + 3] = d[k].n;
      lr[6 * k + 4] = d[k].cap;
      lr[6 * k + 5] = d[k].type;
    }
  }
  if (bases)
    for (int i = 0; i < count; ++i) {
      int64_t* b = bases + 8 * i;
      b[0] = L.b64[i];
      b[1] = L.b32[i];
      b[2] = L.bpiv[i];
      b[3] = L.brank[i];
      b[4] = L.brow[i];
      b[5] = L.bt[i];
      b[6] = L.be[i];
      b[7] = (int64_t)L.pes[i]->plan.lu.tasks.size();
    }
  return HM_OK;
}

void hm_lu_free(hm_lu F) {
  if (!F) return;
  for (DevBuf* b : {&F->f64, &F->f32, &F->piv, &F->ranks, &F->perm, &F->work}) dev_free(*b);
  exec_state_free(F->lu_st);
  exec_state_free(F->solve_st);
  delete F;
}

hm_status hm_lu_trace(hm_lu F, uint64_t* out, int64_t* ntasks, int64_t* clock_khz) {
  if (!F) return fail(HM_EINVAL, "null pointer");
  if (ntasks) *ntasks = F->dag_ntasks;
  if (clock_khz) *clock_khz = g_clock_khz;
  if (!out) return HM_OK;
  if (!F->lu_st.trace.p) return fail(HM_EINVAL, "no trace recorded (set HM_DEBUG_TRACE=1 before h_lu)");
  HIPCHK(hipMemcpy(out, F->lu_st.trace.p, (size_t)F->dag_ntasks * kTraceWords * 8, hipMemcpyDeviceToHost));
  return HM_OK;
}

hm_status hm_solve_trace(hm_lu F, uint64_t* out, int64_t* ntasks, int64_t* clock_khz) {
  if (!F) return fail(HM_EINVAL, "null pointer");
  const int64_t nt = F->pe->solve.ntasks;
  if (ntasks) *ntasks = nt;
  if (clock_khz) *clock_khz = g_clock_khz;
  if (!out) return HM_OK;
  if (!F->solve_st.trace.p) return fail(HM_EINVAL, "no trace recorded (set HM_DEBUG_TRACE=1 before h_lu)");
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(out, F->solve_st.trace.p, (size_t)nt * kTraceWords * 8, hipMemcpyDeviceToHost));
  return HM_OK;
}

hm_status hm_lu_stats_get(hm_lu F, hm_lu_stats* out) {
  if (!F || !out) return fail(HM_EINVAL, "null pointer");
  *out = F->stats;
  return HM_OK;
}

// Fixed device scratch of h_solve_noalloc (refinement vectors), so that the
// entry point allocates nothing.  Each device holds its own copy for the life
// of the process.  In host code `scratch` names a host-side stand-in, not a
// device address: kernels and copies take the address hipGetSymbolAddress
// returns for the current device.
constexpr int64_t kNoAllocScratchDoubles = int64_t(4) << 20;  // 32 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_ptr;  // device -> device address of `scratch`

static hm_status noalloc_scratch(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, (double*)ptr).first;
  }
  *out = it->second;
  return HM_OK;
}

// one pass of the traced forward/backward substitution on up to 64 columns in
// permuted order held in the factor's panel.  The executor status is not
// reset here: the caller clears it once per call, so that a failure of any
// pass survives until the call reads it.
static hm_status solve_pass(hm_lu F, int nc, hipStream_t s) {
  PlanEntry* pe = F->pe;
  hipLaunchKernelGGL(set_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)F->ranks.p + pe->plan.nrhs_slot, nc, 0, 0,
                     0, 1);
  ExecArgs a = base_args((double*)F->f64.p, (float*)F->f32.p, (int32_t*)F->piv.p, (int32_t*)F->ranks.p,
                         (const LrDesc*)pe->lr.p, F->eps, F->max_rank);
  // The substitution DAG runs on the persistent executor (a hand-off costs
  // less than a launch per level); HM_SOLVE_EXEC=level selects one launch
  // per level instead.
  int mode = HM_EXEC_DATAFLOW;
  if (const char* e = getenv("HM_SOLVE_EXEC")) mode = e[0] == 'l' ? HM_EXEC_LEVEL : HM_EXEC_DATAFLOW;
  return run_dag(pe->solve, a, F->solve_st, mode, s, nullptr, DAG_SOLVE, false);
}

static hm_status solve_status(hm_lu F) {
  int32_t stv[4];
  HIPCHK(hipMemcpy(stv, F->solve_st.status.p, 16, hipMemcpyDeviceToHost));
  if (stv[0] & ST_TIMEOUT) return fail(HM_EDEVICE, "executor timed out waiting for a task");
  if (stv[0] & ST_BADOP) return fail(HM_EDEVICE, "internal: a task the executor does not run");
  return HM_OK;
}

// Doubles of refinement work for a chunk of cw columns: a copy of b and the
// residual (n x cw each), norms (2 cw) and active flags (cw int32, rounded up).
static int64_t solve_work_doubles(int64_t n, int64_t cw) { return 2 * n * cw + 4 * cw; }

// The solve of h_solve, h_solve_async and h_solve_noalloc.  Columns go in
// chunks of cw <= 64 (each column's result does not depend on the chunk).
// work: solve_work_doubles(n, cw) doubles of device memory for refinement
// (unused without A).  With status_dev != NULL nothing synchronises and the
// executor status is written there stream-ordered instead of being returned.
static hm_status solve_impl(hm_lu F, hm_matrix A, double* B, int64_t ldb, int64_t nrhs, double rtol, int max_iter,
                            hipStream_t s, int* iters_host, double* relres_host, int64_t cw, double* work,
                            int32_t* status_dev, int* iters_max = nullptr) {
  const int64_t n = F->tree->t.n;
  const Plan& p = F->pe->plan;
  double* panel = (double*)F->f64.p + p.panel_off;
  hipLaunchKernelGGL(set_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)F->solve_st.status.p, 0, 0x7fffffff, 0, 0,
                     4);
  if (relres_host)
    for (int64_t c = 0; c < nrhs; ++c) relres_host[c] = std::nan("");
  double* bcopy = work;
  double* R = A ? bcopy + n * cw : nullptr;
  double* norms = A ? R + n * cw : nullptr;
  int32_t* active = A ? (int32_t*)(norms + 2 * cw) : nullptr;
  bool all_conv = true;
  hm_status st;
  for (int64_t c0 = 0; c0 < nrhs; c0 += cw) {
    const int nc = (int)std::min<int64_t>(cw, nrhs - c0);
    double* Bc = B + c0 * ldb;
    const int64_t tot = n * nc;
    const unsigned g = (unsigned)((tot + 255) / 256);
    if (A) HIPCHK(hipMemcpy2DAsync(bcopy, n * 8, Bc, ldb * 8, n * 8, nc, hipMemcpyDeviceToDevice, s));
    // x0 = U^{-1} L^{-1} P b
    hipLaunchKernelGGL(gather_rows_kernel, dim3(g), dim3(256), 0, s, (const double*)Bc, ldb,
                       (const int64_t*)F->perm.p, n, nc, panel, n);
    if ((st = solve_pass(F, nc, s))) return st;
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(g), dim3(256), 0, s, (const double*)panel, n,
                       (const int64_t*)F->perm.p, n, nc, Bc, ldb, 1.0, 0.0);
    HIPCHK(hipGetLastError());
    if (!A) continue;
    double bn[64], rn[64];
    int32_t act[64];
    hipLaunchKernelGGL(colnorm2_kernel, dim3(nc), dim3(kThreads), 0, s, (const double*)bcopy, n, n, norms);
    HIPCHK(hipMemcpyAsync(bn, norms, nc * 8, hipMemcpyDeviceToHost, s));
    int it = 0;
    for (;;) {
      // r = b - A x
      HIPCHK(hipMemcpyAsync(R, bcopy, n * nc * 8, hipMemcpyDeviceToDevice, s));
      if ((st = matvec_impl(A, -1.0, Bc, ldb, 1.0, R, n, nc, s))) return st;
      hipLaunchKernelGGL(colnorm2_kernel, dim3(nc), dim3(kThreads), 0, s, (const double*)R, n, n, norms);
      HIPCHK(hipMemcpyAsync(rn, norms, nc * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      // a failed substitution pass leaves x partly substituted: stop here
      if ((st = solve_status(F))) return st;
      bool done = true;
      for (int c = 0; c < nc; ++c) {
        double rel = bn[c] > 0 ? std::sqrt(rn[c] / bn[c]) : std::sqrt(rn[c]);
        if (relres_host) relres_host[c0 + c] = rel;
        act[c] = rel > rtol ? 1 : 0;
        if (act[c]) done = false;
      }
      if (done) break;
      if (it >= max_iter) {
        all_conv = false;
        break;
      }
      // x += solve(r) on the columns still above rtol
      HIPCHK(hipMemcpyAsync(active, act, nc * 4, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(gather_rows_kernel, dim3(g), dim3(256), 0, s, (const double*)R, n,
                         (const int64_t*)F->perm.p, n, nc, panel, n);
      if ((st = solve_pass(F, nc, s))) return st;
      hipLaunchKernelGGL(scatter_rows_kernel, dim3(g), dim3(256), 0, s, (const double*)panel, n,
                         (const int64_t*)F->perm.p, n, nc, R, n, 1.0, 0.0);
      hipLaunchKernelGGL(axpy_cols_kernel, dim3(g), dim3(256), 0, s, Bc, ldb, (const double*)R, n, n, nc,
                         (const int32_t*)active);
      HIPCHK(hipGetLastError());
      ++it;
    }
    if (iters_host) iters_host[c0 / cw] = it;
    if (iters_max) *iters_max = std::max(*iters_max, it);
  }
  if (status_dev) {
    hipLaunchKernelGGL(status_word_kernel, dim3(1), dim3(64), 0, s, (const int32_t*)F->solve_st.status.p,
                       status_dev);
    HIPCHK(hipGetLastError());
    return HM_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  if ((st = solve_status(F))) return st;
  if (!all_conv) return fail(HM_ENOCONV, "refinement did not reach rtol");
  return HM_OK;
}

static hm_status solve_args(hm_lu F, hm_matrix A, const double* B, int64_t ldb, int64_t nrhs, int max_iter) {
  if (!F || !B) return fail(HM_EINVAL, "null pointer");
  const int64_t n = F->tree->t.n;
  if (nrhs < 0 || ldb < n || max_iter < 0) return fail(HM_EINVAL, "bad nrhs, ldb or max_iter");
  if (A && A->tree != F->tree) return fail(HM_EINVAL, "matrix and factors are on different trees");
  return HM_OK;
}

hm_status h_solve(hm_lu F, hm_matrix A, double* B, int64_t ldb, int64_t nrhs, double rtol, int max_iter,
                  void* stream, int* iters_host, double* relres_host) {
  hm_status st = solve_args(F, A, B, ldb, nrhs, max_iter);
  if (st) return st;
  if (nrhs == 0) return HM_OK;
  if ((st = device_setup())) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = F->tree->t.n;
  const int64_t CW = F->pe->plan.nrhs_cap;
  if (A) {
    const size_t need = (size_t)solve_work_doubles(n, CW) * 8;
    if (F->work.bytes < need) {
      HIPCHK(hipStreamSynchronize(s));
      dev_free(F->work);
      if (!dev_alloc(F->work, need, s)) return fail(HM_ENOMEM, "device allocation failed (solve work)");
    }
  }
  return solve_impl(F, A, B, ldb, nrhs, rtol, max_iter, s, iters_host, relres_host, CW, (double*)F->work.p,
                    nullptr);
}

hm_status h_solve_noalloc(hm_lu F, hm_matrix A, double* B, int64_t ldb, int64_t nrhs, double rtol, int max_iter,
                          void* stream, int* iters_host, double* relres_host) {
  hm_status st = solve_args(F, A, B, ldb, nrhs, max_iter);
  if (st) return st;
  if (iters_host) *iters_host = 0;
  if (nrhs == 0) return HM_OK;
  if ((st = device_setup())) return st;
  double* work = nullptr;
  if ((st = noalloc_scratch(&work))) return st;
  const int64_t n = F->tree->t.n;
  int64_t cw = F->pe->plan.nrhs_cap;
  if (A) {
    while (cw > 0 && solve_work_doubles(n, cw) > kNoAllocScratchDoubles) --cw;
    if (cw < 1)
      return fail(HM_EINVAL, "n too large for the fixed scratch of h_solve_noalloc (refinement needs " +
                                 std::to_string(solve_work_doubles(n, 1) * 8) + " bytes, the scratch holds " +
                                 std::to_string(kNoAllocScratchDoubles * 8) + ")");
  }
  return solve_impl(F, A, B, ldb, nrhs, rtol, max_iter, (hipStream_t)stream, nullptr, relres_host, cw, work,
                    nullptr, iters_host);
}

hm_status h_solve_async(hm_lu F, double* B, int64_t ldb, int64_t nrhs, void* stream, int32_t* status_dev) {
  hm_status st = solve_args(F, nullptr, B, ldb, nrhs, 0);
  if (st) return st;
  if (!status_dev) return fail(HM_EINVAL, "null status word");
  if ((st = device_setup())) return st;
  hipStream_t s = (hipStream_t)stream;
  if (nrhs == 0) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, status_dev, 0, (int64_t)1);
    HIPCHK(hipGetLastError());
    return HM_OK;
  }
  return solve_impl(F, nullptr, B, ldb, nrhs, 0.0, 0, s, nullptr, nullptr, F->pe->plan.nrhs_cap, nullptr,
                    status_dev);
}

hm_status hm_footprint(const void* handle, int kind, size_t* bytes) {
  if (!handle || !bytes) return fail(HM_EINVAL, "null pointer");
  if (kind == 0) {
    *bytes = ((const hm_matrix_s*)handle)->bytes();
  } else if (kind == 1 || kind == 2) {
    const hm_lu_s* F = (const hm_lu_s*)handle;
    const Plan& p = F->pe->plan;
    size_t blocks = (size_t)p.blocks_f64 * 8 + (size_t)p.blocks_f32 * 4 + F->piv.bytes + F->ranks.bytes;
    size_t total = F->f64.bytes + F->f32.bytes + F->piv.bytes + F->ranks.bytes + F->perm.bytes + F->work.bytes +
                   F->lu_st.deps.bytes + F->lu_st.queue.bytes + F->solve_st.deps.bytes + F->solve_st.queue.bytes;
    *bytes = kind == 1 ? blocks : total - blocks;
  } else {
    return fail(HM_EINVAL, "kind must be 0, 1 or 2");
  }
  return HM_OK;
}

hm_status hm_export_leaf(const void* handle, int kind, int64_t block, double* data, int32_t* rank, int32_t* piv) {
  if (!handle || !rank) return fail(HM_EINVAL, "null pointer");
  hm_tree t;
  const Plan* p;
  const void* f64;
  const void* f32;
  const void* ranks;
  const void* pivs = nullptr;
  if (kind == 0) {
    const hm_matrix_s* A = (const hm_matrix_s*)handle;
    t = A->tree;
    p = &A->pe->plan;
    f64 = A->f64.p;
    f32 = nullptr;
    ranks = A->ranks.p;
  } else if (kind == 1) {
    const hm_lu_s* F = (const hm_lu_s*)handle;
    t = F->tree;
    p = &F->pe->plan;
    f64 = F->f64.p;
    f32 = F->f32.p;
    ranks = F->ranks.p;
    pivs = F->piv.p;
  } else {
    return fail(HM_EINVAL, "kind must be 0 or 1");
  }
  if (block < 0 || block >= (int64_t)t->t.bl.size()) return fail(HM_EINVAL, "block index out of range");
  const BlockNode& bn = t->t.bl[block];
  if (bn.kind == BK_STRUCT) return fail(HM_EINVAL, "not a leaf block");
  const int64_t m = t->t.cl[bn.tau].size(), n = t->t.cl[bn.sigma].size();
  auto fetch = [&](int64_t off, int type, int64_t count, double* dst) -> hm_status {
    if (type == VT_F64) {
      HIPCHK(hipMemcpy(dst, (const double*)f64 + off, count * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmp(count);
      HIPCHK(hipMemcpy(tmp.data(), (const float*)f32 + off, count * 4, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < count; ++i) dst[i] = tmp[i];
    }
    return HM_OK;
  };
  hm_status st;
  if (bn.kind == BK_DENSE) {
    *rank = -1;
    if (data && (st = fetch(p->data_off[block], p->data_type[block], m * n, data))) return st;
    if (piv && pivs && p->piv_off[block] >= 0)
      HIPCHK(hipMemcpy(piv, (const int32_t*)pivs + p->piv_off[block], m * 4, hipMemcpyDeviceToHost));
    return HM_OK;
  }
  const int li = p->lr_index[block];
  const LrDesc& d = p->lr[li];
  int32_t k = 0;
  HIPCHK(hipMemcpy(&k, (const int32_t*)ranks + li, 4, hipMemcpyDeviceToHost));
  *rank = k;
  if (data && k > 0) {
    if ((st = fetch(d.u_off, d.type, m * k, data))) return st;
    if ((st = fetch(d.v_off, d.type, n * k, data + m * k))) return st;
  }
  return HM_OK;
}

}  // extern "C"
