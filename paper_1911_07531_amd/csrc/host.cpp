// Host side of the H-LU library: trees (Def. 2.1, Def. 2.2), storage layout
// (Def. 2.3) and the symbolic trace of Algorithms 1-3 into a task DAG.
//
// The trace walks the recursion of hlu / htrsl / htrsu / hmul exactly as the
// sequential algorithm would run it and records, instead of arithmetic, one
// task per leaf-level block operation together with the storage it reads and
// writes (Def. 3.1).  Edges follow Def. 3.2 (an output intersecting a later
// input on the same storage) plus write-after-read and write-after-write
// ordering, so that every topological order of the DAG computes the
// sequential result.
#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <numeric>
#include <tuple>

namespace hm {

// ---------------------------------------------------------------------------
// Def. 2.1: cluster tree by geometric bisection of the longest axis
// ---------------------------------------------------------------------------
// Compiled with -ffp-contract=off: the bounding boxes, midpoints and the
// admissibility test must round exactly like a plain evaluation.
void build_cluster_tree(const double* pts, int64_t n, int dim, int leaf, Tree& t) {
  t.n = n;
  t.dim = dim;
  t.leaf = leaf;
  t.cl.clear();
  t.perm.clear();
  t.perm.reserve(n);
  std::vector<double> p3(3 * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d) p3[3 * i + d] = pts[i * dim + d];

  std::function<int(std::vector<int64_t>&, int)> rec = [&](std::vector<int64_t>& idx, int level) -> int {
    Cluster c;
    c.begin = (int64_t)t.perm.size();
    c.end = -1;
    c.son[0] = c.son[1] = -1;
    c.level = level;
    for (int d = 0; d < 3; ++d) {
      c.lo[d] = p3[3 * idx[0] + d];
      c.hi[d] = p3[3 * idx[0] + d];
    }
    for (int64_t i : idx)
      for (int d = 0; d < 3; ++d) {
        double v = p3[3 * i + d];
        if (v < c.lo[d]) c.lo[d] = v;
        if (v > c.hi[d]) c.hi[d] = v;
      }
    int me = (int)t.cl.size();
    t.cl.push_back(c);
    if ((int64_t)idx.size() > leaf) {
      int axis = 0;
      double best = c.hi[0] - c.lo[0];
      for (int d = 1; d < 3; ++d) {
        double e = c.hi[d] - c.lo[d];
        if (e > best) {
          best = e;
          axis = d;
        }
      }
      double mid = 0.5 * (c.lo[axis] + c.hi[axis]);
      std::vector<int64_t> left, right;
      left.reserve(idx.size());
      right.reserve(idx.size());
      for (int64_t i : idx) (p3[3 * i + axis] <= mid ? left : right).push_back(i);
      if (!left.empty() && !right.empty()) {
        std::vector<int64_t>().swap(idx);
        int s0 = rec(left, level + 1);
        int s1 = rec(right, level + 1);
        t.cl[me].son[0] = s0;
        t.cl[me].son[1] = s1;
      }
    }
    if (t.cl[me].son[0] < 0)
      for (int64_t i : idx) t.perm.push_back(i);
    t.cl[me].end = (int64_t)t.perm.size();
    return me;
  };
  std::vector<int64_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  rec(all, 0);
  t.pts_perm.assign(3 * n, 0.0);
  for (int64_t k = 0; k < n; ++k)
    for (int d = 0; d < 3; ++d) t.pts_perm[3 * k + d] = p3[3 * t.perm[k] + d];
}

static double diam(const Cluster& c) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    double e = c.hi[d] - c.lo[d];
    s = s + e * e;
  }
  return std::sqrt(s);
}

// Standard admissibility (Sec. 5.1) on bounding boxes; touching boxes are inadmissible.
static bool admissible(const Cluster& t, const Cluster& s, double eta) {
  double g2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    double g = std::max(0.0, std::max(s.lo[d] - t.hi[d], t.lo[d] - s.hi[d]));
    g2 = g2 + g * g;
  }
  double dist = std::sqrt(g2);
  if (dist <= 0.0) return false;
  return std::min(diam(t), diam(s)) <= eta * dist;
}

// Def. 2.2: sons(t, s) empty if admissible or a cluster is a leaf; pre-order numbering.
void build_block_tree(Tree& t, double eta) {
  t.eta = eta;
  t.bl.clear();
  std::function<int(int, int)> rec = [&](int tau, int sigma) -> int {
    BlockNode b;
    b.tau = tau;
    b.sigma = sigma;
    for (int k = 0; k < 4; ++k) b.son[k] = -1;
    int me = (int)t.bl.size();
    const Cluster& ct = t.cl[tau];
    const Cluster& cs = t.cl[sigma];
    if (admissible(ct, cs, eta))
      b.kind = BK_LOWRANK;
    else if (ct.leaf() || cs.leaf())
      b.kind = BK_DENSE;
    else
      b.kind = BK_STRUCT;
    t.bl.push_back(b);
    if (b.kind == BK_STRUCT) {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          int s = rec(ct.son[i], cs.son[j]);
          t.bl[me].son[2 * i + j] = s;
        }
    }
    return me;
  };
  rec(0, 0);
}

// ---------------------------------------------------------------------------
// Def. 2.3: storage of the leaves
// ---------------------------------------------------------------------------
static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

bool make_layout(const Tree& t, int prec, int max_rank, int nrhs_cap, Plan& p) {
  p.tree = &t;
  p.prec = prec;
  p.max_rank = max_rank;
  if (max_rank < 0 || max_rank > kMaxCap) {
    p.err = "max_rank must be in [0, 64]";
    return false;
  }
  p.cap = max_rank > 0 ? max_rank : kMaxCap;
  p.nrhs_cap = nrhs_cap;
  size_t nb = t.bl.size();
  p.data_off.assign(nb, -1);
  p.data_type.assign(nb, -1);
  p.lr_index.assign(nb, -1);
  p.piv_off.assign(nb, -1);
  p.inv_off.assign(nb, -1);
  p.lr.clear();
  p.lr_block.clear();
  p.diag_leaves.clear();
  int64_t f64 = 0, f32 = 0, piv = 0;
  const int64_t A = 32;
  for (size_t b = 0; b < nb; ++b) {
    const BlockNode& bn = t.bl[b];
    if (bn.kind == BK_STRUCT) continue;
    int64_t m = t.cl[bn.tau].size(), n = t.cl[bn.sigma].size();
    bool diag = bn.tau == bn.sigma;
    int type = (prec == 1 && !diag) ? VT_F32 : VT_F64;
    if (bn.kind == BK_DENSE) {
      if (diag && m > kMaxLeaf) {
        p.err = "diagonal leaf larger than 128 rows";
        return false;
      }
      int64_t& cur = type == VT_F64 ? f64 : f32;
      cur = align_up(cur, A);
      p.data_off[b] = cur;
      p.data_type[b] = type;
      cur += m * n;
      if (diag) {
        // LAPACK interchanges (m) followed by the resulting row permutation (m)
        p.piv_off[b] = piv;
        piv += 2 * m;
        p.diag_leaves.push_back((int)b);
      }
    } else {
      LrDesc d;
      d.m = (int32_t)m;
      d.n = (int32_t)n;
      d.cap = (int32_t)std::min<int64_t>(p.cap, std::min(m, n));
      d.type = type;
      int64_t& cur = type == VT_F64 ? f64 : f32;
      cur = align_up(cur, A);
      d.u_off = cur;
      cur += m * d.cap;
      cur = align_up(cur, A);
      d.v_off = cur;
      cur += n * d.cap;
      p.lr_index[b] = (int32_t)p.lr.size();
      p.lr.push_back(d);
      p.lr_block.push_back((int32_t)b);
    }
  }
  p.blocks_f64 = align_up(f64, A);
  p.blocks_f32 = align_up(f32, A);
  p.panel_off = p.blocks_f64;
  p.n_f64 = p.panel_off + t.n * (int64_t)nrhs_cap;
  // inverses of the factored diagonal leaves (for the substitution)
  for (int d : p.diag_leaves) {
    const int64_t m = t.cl[t.bl[d].tau].size();
    p.n_f64 = align_up(p.n_f64, A);
    p.inv_off[d] = p.n_f64;
    p.n_f64 += 2 * m * m;
  }
  p.n_f64 = align_up(p.n_f64, A);
  p.n_f32 = p.blocks_f32;
  p.n_piv = piv;
  p.nlr_leaf = (int)p.lr.size();
  p.nrhs_slot = (int)p.lr.size();
  p.nranks = p.nrhs_slot + 1;
  return true;
}

// ---------------------------------------------------------------------------
// Symbolic trace
// ---------------------------------------------------------------------------
namespace {

struct Rect {
  int32_t r0, r1, c0, c1;
};
static bool overlap(const Rect& a, const Rect& b) {
  return a.r0 < b.r1 && b.r0 < a.r1 && a.c0 < b.c1 && b.c0 < a.c1;
}
static bool covers(const Rect& a, const Rect& b) {
  return a.r0 <= b.r0 && a.r1 >= b.r1 && a.c0 <= b.c0 && a.c1 >= b.c1;
}

// A view plus the storage it touches: object id and the rectangle in the
// object's own (row, col) storage coordinates.
struct HView {
  View v;
  int obj;
  Rect rect;
  bool tr;
  int32_t pool_cls = -1, pool_slot = -1;  // temporaries: ring slot
};

struct Term {
  HView u, v;  // U (rows x k), V (cols x k)
  int32_t r0, c0;
  double alpha;
};

struct Rec {
  Rect r;
  int task;
};
struct ObjState {
  std::vector<Rec> writes, reads;
  // temporaries: accesses of the slot's earlier occupants (rectangles in
  // their own shapes, so they are kept whole: every access of this object
  // orders after them until a write covers the object's full extent)
  std::vector<Rec> inh_w, inh_r;
  Rect full{0, 0, 0, 0};
};

enum { ACC_R = 1, ACC_W = 2, ACC_RW = 3 };

class Tracer {
 public:
  Tracer(Plan& p, Dag& d, int64_t temp_budget_bytes) : p_(p), t_(*p.tree), d_(d) {
    tsize_ = p.prec == 1 ? 4 : 8;
    temp_type_ = p.prec == 1 ? VT_F32 : VT_F64;
    temp_budget_ = temp_budget_bytes / tsize_;
    size_t nb = t_.bl.size();
    obj_a_.assign(nb, -1);
    obj_b_.assign(nb, -1);
    inv_obj_.assign(nb, -1);
    for (int d : p.diag_leaves) inv_obj_[d] = new_obj();
    for (size_t b = 0; b < nb; ++b) {
      if (t_.bl[b].kind == BK_DENSE) obj_a_[b] = new_obj();
      if (t_.bl[b].kind == BK_LOWRANK) {
        obj_a_[b] = new_obj();
        obj_b_[b] = new_obj();
        owner_[obj_a_[b]] = (int)b;
        owner_[obj_b_[b]] = (int)b;
      }
    }
    lr_obj_.assign(p.lr.size(), {-1, -1});
    for (size_t i = 0; i < p.lr_block.size(); ++i)
      if (p.lr_block[i] >= 0) lr_obj_[i] = {obj_a_[p.lr_block[i]], obj_b_[p.lr_block[i]]};
    pending_.resize(nb);
    temp_base_ = p.prec == 1 ? p.blocks_f32 : p.n_f64;
    temp_top_ = temp_base_;
  }
  // Substitution DAGs: temporaries in FP64 after the factor's FP64 arena, and
  // low-rank products with a side of at least 2 * rows rows split into
  // partial products of about `rows` rows (0 = never split).
  void set_solve(int32_t split_rows, int32_t coarsen = 0) {
    tsize_ = 8;
    temp_type_ = VT_F64;
    temp_base_ = temp_top_ = p_.n_f64;
    split_ = split_rows;
    sub_ = true;
    solve_dag_ = true;
    coarsen_ = coarsen;
    if (coarsen_ > 0) {
      cb_of_row_.assign((size_t)t_.n, -1);
      coarse_blocks(0);
      cb_sweep_.assign(cb_begin_.size(), 0);
      deferred_.assign(cb_begin_.size(), {});
      def_lo_.assign(cb_begin_.size(), INT64_MAX);
      def_hi_.assign(cb_begin_.size(), -1);
      if (const char* e = getenv("HM_FOLD_REACH")) fold_reach_ = std::max(1, atoi(e));
    }
  }
  // +1 before the forward substitution, -1 before the backward one
  void set_sweep(int dir) { sweep_ = dir; }
  void set_temp_base(int64_t b) { temp_base_ = temp_top_ = b; }
  // tasks emitted from now on belong to a substitution (flag c1 = 1)
  void begin_substitution() { sub_ = true; }

  bool ok() const { return err_.empty(); }
  const std::string& err() const { return err_; }
  int64_t temp_end() const { return temp_top_; }

  // ---- views -------------------------------------------------------------
  HView dense(int b) {
    const BlockNode& bn = t_.bl[b];
    int32_t m = (int32_t)t_.cl[bn.tau].size(), n = (int32_t)t_.cl[bn.sigma].size();
    HView h;
    h.v = View{p_.data_off[b], m, n, 1, m, p_.data_type[b], 0, -1, 0};
    h.obj = obj_a_[b];
    h.rect = Rect{0, m, 0, n};
    h.tr = false;
    return h;
  }
  HView lr_u(int b) {
    const LrDesc& d = p_.lr[p_.lr_index[b]];
    HView h;
    h.v = View{d.u_off, d.m, d.cap, 1, d.m, d.type, DYN_COLS, p_.lr_index[b], 0};
    h.obj = obj_a_[b];
    h.rect = Rect{0, d.m, 0, d.cap};
    h.tr = false;
    return h;
  }
  HView lr_v(int b) {
    const LrDesc& d = p_.lr[p_.lr_index[b]];
    HView h;
    h.v = View{d.v_off, d.n, d.cap, 1, d.n, d.type, DYN_COLS, p_.lr_index[b], 0};
    h.obj = obj_b_[b];
    h.rect = Rect{0, d.n, 0, d.cap};
    h.tr = false;
    return h;
  }
  static HView ident(int32_t m) {
    HView h;
    h.v = View{0, m, m, 0, 0, VT_IDENT, 0, -1, 0};
    h.obj = -1;
    h.rect = Rect{0, 0, 0, 0};
    h.tr = false;
    return h;
  }
  static HView transpose(const HView& x) {
    HView h = x;
    std::swap(h.v.rows, h.v.cols);
    std::swap(h.v.rs, h.v.cs);
    int dyn = 0;
    if (x.v.dyn & DYN_ROWS) dyn |= DYN_COLS;
    if (x.v.dyn & DYN_COLS) dyn |= DYN_ROWS;
    h.v.dyn = dyn;
    h.tr = !x.tr;
    return h;
  }
  // Columns [a, b) of a view with a static column count.  A column slice of
  // an identity is materialised: an m x (b - a) temporary with ones at
  // (a + j, j).
  HView cols(const HView& x, int32_t a, int32_t b) {
    if (x.v.dyn & DYN_COLS) fail("column slice of a view with a run-time column count");
    if (x.v.type == VT_IDENT) {
      HView z = temp(x.v.rows, b - a, -1);
      zero(z);
      HView zr = rows(z, a, b);
      HView e = ident(b - a);
      Task t = blank(OP_COPY);
      t.y = zr.v;
      t.a = e.v;
      emit(t, {{&zr, ACC_W}});
      return z;
    }
    HView h = x;
    h.v.off = x.v.off + (int64_t)a * x.v.cs;
    h.v.cols = b - a;
    if (!x.tr) {
      h.rect.c0 = x.rect.c0 + a;
      h.rect.c1 = x.rect.c0 + b;
    } else {
      h.rect.r0 = x.rect.r0 + a;
      h.rect.r1 = x.rect.r0 + b;
    }
    return h;
  }
  HView rows(const HView& x, int32_t a, int32_t b) {
    if (x.v.dyn & DYN_ROWS) fail("row slice of a view with a run-time row count");
    HView h = x;
    if (x.v.type == VT_IDENT) {
      // a row slice of I is a shifted identity: only used through restriction,
      // which the trace expresses as a sub-view of a materialised factor
      fail("row slice of an identity view");
      return h;
    }
    h.v.off = x.v.off + (int64_t)a * x.v.rs;
    h.v.rows = b - a;
    if (!x.tr) {
      h.rect.r0 = x.rect.r0 + a;
      h.rect.r1 = x.rect.r0 + b;
    } else {
      h.rect.c0 = x.rect.c0 + a;
      h.rect.c1 = x.rect.c0 + b;
    }
    return h;
  }
  // Temporary panel rows x cols (cols may follow a rank slot), in the LU's
  // off-diagonal element type.  Temporaries live in rings per size class;
  // reusing a slot orders the new writer after every earlier access.
  HView temp(int32_t r, int32_t cols, int dyn_rank_id) {
    int64_t elems = (int64_t)r * cols;
    int cls = 0;
    int64_t sz = 1024;
    while (sz < elems) {
      sz <<= 1;
      ++cls;
    }
    if ((int)pools_.size() <= cls) pools_.resize(cls + 1);
    Pool& pool = pools_[cls];
    if (pool.limit == 0) pool.limit = std::max<int64_t>(64, std::min<int64_t>(1 << 16, temp_budget_ / 8 / sz));
    // next slot of the ring that no collected update still refers to
    int64_t slot = 0;
    for (int64_t tries = 0;; ++tries) {
      if (tries >= pool.limit) pool.limit *= 2;
      slot = pool.next % pool.limit;
      pool.next++;
      if (slot >= (int64_t)pool.off.size() || pool.pins[slot] == 0) break;
    }
    while (slot >= (int64_t)pool.off.size()) {
      temp_top_ = align_up(temp_top_, 32);
      pool.off.push_back(temp_top_);
      pool.obj.push_back(-1);
      pool.pins.push_back(0);
      temp_top_ += sz;
    }
    // a fresh object per occupant; the previous occupant (possibly of another
    // shape, so its rectangles do not compare with ours) hands over its
    // accesses, and any it had inherited itself
    const int ob = new_obj();
    const int prev = pool.obj[slot];
    if (prev >= 0) {
      ObjState& po = objs_[prev];
      ObjState& no = objs_[ob];
      no.inh_w = std::move(po.inh_w);
      no.inh_r = std::move(po.inh_r);
      no.inh_w.insert(no.inh_w.end(), po.writes.begin(), po.writes.end());
      no.inh_r.insert(no.inh_r.end(), po.reads.begin(), po.reads.end());
      std::vector<Rec>().swap(po.writes);
      std::vector<Rec>().swap(po.reads);
      std::vector<Rec>().swap(po.inh_w);
      std::vector<Rec>().swap(po.inh_r);
    }
    objs_[ob].full = Rect{0, r, 0, cols};
    pool.obj[slot] = ob;
    HView h;
    h.v = View{pool.off[slot], r, cols, 1, r, temp_type_, dyn_rank_id >= 0 ? DYN_COLS : 0, dyn_rank_id, 0};
    h.obj = ob;
    h.rect = Rect{0, r, 0, cols};
    h.tr = false;
    h.pool_cls = cls;
    h.pool_slot = (int32_t)slot;
    return h;
  }
  HView panel() {
    HView h;
    h.v = View{p_.panel_off, (int32_t)t_.n, p_.nrhs_cap, 1, (int32_t)t_.n, VT_F64, DYN_COLS, p_.nrhs_slot, 0};
    if (panel_obj_ < 0) panel_obj_ = new_obj();
    h.obj = panel_obj_;
    h.rect = Rect{0, (int32_t)t_.n, 0, p_.nrhs_cap};
    h.tr = false;
    return h;
  }

  // ---- task emission with dependency tracking (Def. 3.2 + WAR/WAW) -----------
  void emit(Task tk, std::initializer_list<std::pair<const HView*, int>> acc) {
    if (sub_) tk.c1 = 1;
    if (in_seq_) {
      seq_op(tk);
      return;
    }
    if (coarsen_ > 0 && sub_ && (tk.op == OP_GEMM || tk.op == OP_LRGEMM) && defer_neighbour(tk)) return;
    // a low-rank leaf with collected updates gets them applied before any
    // other task touches it
    for (auto& a : acc)
      if (a.first->obj >= 0) {
        int b = owner_[a.first->obj];
        if (b >= 0 && !pending_[b].empty()) flush(b);
      }
    int id = (int)d_.tasks.size();
    d_.tasks.push_back(tk);
    d_.task_call.push_back(call_);
    preds_.clear();
    // A view whose extent follows a rank must be ordered after the truncation
    // that set it: the task must also access that low-rank leaf's (or
    // accumulator's) U or V storage, which the truncation rewrites.
    for (auto& a : acc) {
      const View& v = a.first->v;
      if (!v.dyn || v.rank_id < 0 || v.rank_id >= (int)lr_obj_.size()) continue;
      auto ob = lr_obj_[v.rank_id];
      bool backed = false;
      for (auto& c : acc) backed |= c.first->obj == ob.first || c.first->obj == ob.second;
      if (!backed) fail("internal: a run-time extent follows a rank the task does not read");
    }
    for (auto& a : acc)
      if (a.first->obj >= 0 && (a.second & ACC_R)) access(id, a.first->obj, a.first->rect, false);
    for (auto& a : acc)
      if (a.first->obj >= 0 && (a.second & ACC_W)) access(id, a.first->obj, a.first->rect, true);
    std::sort(preds_.begin(), preds_.end());
    preds_.erase(std::unique(preds_.begin(), preds_.end()), preds_.end());
    int lvl = 0;
    for (int q : preds_) {
      edges_.push_back({q, id});
      lvl = std::max(lvl, d_.level[q] + 1);
    }
    d_.level.push_back(lvl);
    d_.indeg.push_back((int32_t)preds_.size());
  }

  // Static duration estimate of a task (microseconds; means measured per task
  // kind, truncations growing with the leaf's m + n), used only to flag the
  // tasks near the DAG's critical path.
  double cost_estimate(const Task& t) const {
    switch (t.op) {
      case OP_GETRF:
        return 75.0;
      case OP_TRSM_L:
      case OP_TRSM_UT:
      case OP_TRSM_U:
        return 25.0;
      case OP_GEMM:
        return 15.0;
      case OP_LRGEMM:
        return 40.0;
      case OP_TRUNC:
      case OP_TRUNC2:
        if (t.lr >= 0 && t.lr < (int)p_.lr.size()) return 100.0 + 0.1 * (p_.lr[t.lr].m + p_.lr[t.lr].n);
        return 150.0;
      case OP_TRTRI:
        return 30.0;
      default:
        return 10.0;
    }
  }
  // succ_crit: an edge's successor has slack (critical-path length minus the
  // longest path through it, both by the estimate) of at most 0.5 % of the
  // critical path; the executor runs such a successor on the workgroup that
  // releases it instead of queueing it behind the ready tasks off the path.
  void flag_critical() {
    const int nt = (int)d_.tasks.size();
    std::vector<float> cost(nt), bl(nt), tl(nt, 0.f);
    for (int i = 0; i < nt; ++i) cost[i] = (float)cost_estimate(d_.tasks[i]);
    for (int i = nt - 1; i >= 0; --i) {
      float m = 0.f;
      for (int32_t k = d_.succ_ptr[i]; k < d_.succ_ptr[i + 1]; ++k) m = std::max(m, bl[d_.succ_idx[k]]);
      bl[i] = cost[i] + m;
    }
    float cp = 0.f;
    for (int i = 0; i < nt; ++i) {
      cp = std::max(cp, tl[i] + bl[i]);
      for (int32_t k = d_.succ_ptr[i]; k < d_.succ_ptr[i + 1]; ++k) {
        const int s = d_.succ_idx[k];
        tl[s] = std::max(tl[s], tl[i] + cost[i]);
      }
    }
    // HM_CRIT_SLACK overrides the slack (a fraction of the critical path;
    // negative: no task flagged).  0.5 % measured best at n = 131072 (1.68 s
    // against 1.78 s unflagged; every task flagged: 1.72 s).
    const char* e = getenv("HM_CRIT_SLACK");
    const float thr = (float)(1.0 - (e ? atof(e) : 0.005)) * cp;
    d_.succ_crit.assign(d_.succ_idx.size(), 0);
    for (size_t k = 0; k < d_.succ_idx.size(); ++k) {
      const int s = d_.succ_idx[k];
      d_.succ_crit[k] = tl[s] + bl[s] >= thr ? 1 : 0;
    }

  }

  void finish() {
    int nt = (int)d_.tasks.size();
    d_.nedges = (int64_t)edges_.size();
    d_.succ_ptr.assign(nt + 1, 0);
    for (auto& e : edges_) d_.succ_ptr[e.first + 1]++;
    for (int i = 0; i < nt; ++i) d_.succ_ptr[i + 1] += d_.succ_ptr[i];
    d_.succ_idx.assign(edges_.size(), 0);
    std::vector<int32_t> fill(d_.succ_ptr.begin(), d_.succ_ptr.end() - 1);
    for (auto& e : edges_) d_.succ_idx[fill[e.first]++] = e.second;
    std::vector<std::pair<int, int>>().swap(edges_);
    if (!solve_dag_) flag_critical();
    int nl = 0;
    for (int l : d_.level) nl = std::max(nl, l + 1);
    d_.level_ptr.assign(nl + 1, 0);
    for (int l : d_.level) d_.level_ptr[l + 1]++;
    for (int i = 0; i < nl; ++i) d_.level_ptr[i + 1] += d_.level_ptr[i];
    d_.level_order.assign(nt, 0);
    std::vector<int32_t> pos(d_.level_ptr.begin(), d_.level_ptr.end() - 1);
    for (int i = 0; i < nt; ++i) d_.level_order[pos[d_.level[i]]++] = i;
    d_.roots.clear();
    for (int i = 0; i < nt; ++i)
      if (d_.indeg[i] == 0) d_.roots.push_back(i);
  }

  // ---- leaf operations ------------------------------------------------------
  static Task blank(int op) {
    Task t;
    std::memset(&t, 0, sizeof(t));
    t.op = op;
    t.lr = -1;
    t.piv = -1;
    View none{0, 0, 0, 0, 0, VT_NONE, 0, -1, 0};
    t.y = t.a = t.b = t.x = none;
    return t;
  }
  void gemm(const HView& y, double alpha, const HView& a, const HView& b, double beta) {
    Task t = blank(OP_GEMM);
    t.alpha = alpha;
    t.beta = beta;
    t.y = y.v;
    t.a = a.v;
    t.b = b.v;
    emit(t, {{&a, ACC_R}, {&b, ACC_R}, {&y, beta != 0.0 ? ACC_RW : ACC_W}});
  }
  void lrgemm(const HView& y, double alpha, const HView& a, const HView& b, const HView& x, double beta) {
    // a product whose target spans several coarse blocks and whose source
    // folds into the first of them (in sweep order): that block's rows as
    // their own product (folded into its task), the rest as a task
    if (const int32_t cut = fold_cut(y.v, x.v); cut > 0 && beta == 1.0 && !(a.v.dyn & DYN_ROWS)) {
      const int32_t m = y.v.rows;
      const int32_t f0 = sweep_ > 0 ? 0 : m - cut, f1 = sweep_ > 0 ? cut : m;
      const int32_t r0 = sweep_ > 0 ? cut : 0, r1 = sweep_ > 0 ? m : m - cut;
      lrgemm(rows(y, f0, f1), alpha, rows(a, f0, f1), b, x, beta);
      lrgemm(rows(y, r0, r1), alpha, rows(a, r0, r1), b, x, beta);
      return;
    }
    Task t = blank(OP_LRGEMM);
    t.alpha = alpha;
    t.beta = beta;
    t.y = y.v;
    t.a = a.v;
    t.b = b.v;
    t.x = x.v;
    emit(t, {{&a, ACC_R}, {&b, ACC_R}, {&x, ACC_R}, {&y, beta != 0.0 ? ACC_RW : ACC_W}});
  }
  // Clears the whole stored extent (capacity columns), so that it needs no
  // ordering against the rank that later accumulations follow.
  void zero(const HView& y) {
    Task t = blank(OP_ZERO);
    HView full = y;
    full.v.dyn = 0;
    full.v.rank_id = -1;
    t.y = full.v;
    emit(t, {{&full, ACC_W}});
  }
  // L^{-1} (inv = 0) or U^{-1} (inv = 1) of a factored diagonal leaf, or both
  // (inv = 2: the m x 2m region OP_TRTRI writes)
  HView inverse(int d, int inv) {
    const int32_t m = (int32_t)t_.cl[t_.bl[d].tau].size();
    HView h;
    const int64_t off = p_.inv_off[d] + (inv == 1 ? (int64_t)m * m : 0);
    const int32_t cols = inv == 2 ? 2 * m : m;
    h.v = View{off, m, cols, 1, m, VT_F64, 0, -1, 0};
    h.obj = inv_obj_[d];
    h.rect = Rect{0, m, inv == 1 ? m : 0, inv == 1 ? 2 * m : cols};
    h.tr = false;
    return h;
  }
  // In a substitution the leaf solves apply the inverses of the triangles
  // (computed once per factorization by OP_TRTRI): a product instead of a
  // chain of dependent steps.
  void trsm(int op, int d, const HView& x) {
    Task t = blank(op);
    HView a = dense(d);
    t.a = a.v;
    t.piv = p_.piv_off[d];
    t.x = x.v;
    if (sub_ && (op == OP_TRSM_L || op == OP_TRSM_U) && p_.inv_off[d] >= 0) {
      HView iv = inverse(d, op == OP_TRSM_L ? 0 : 1);
      t.b = iv.v;
      emit(t, {{&a, ACC_R}, {&iv, ACC_R}, {&x, ACC_RW}});
      return;
    }
    emit(t, {{&a, ACC_R}, {&x, ACC_RW}});
  }
  void trtri(int d) {
    Task t = blank(OP_TRTRI);
    HView a = dense(d);
    HView y = inverse(d, 2);
    t.a = a.v;
    t.y = y.v;
    t.piv = p_.piv_off[d];
    emit(t, {{&a, ACC_R}, {&y, ACC_W}});
  }
  void getrf(int d) {
    Task t = blank(OP_GETRF);
    HView a = dense(d);
    t.a = a.v;
    t.piv = p_.piv_off[d];
    t.row0 = (int32_t)t_.cl[t_.bl[d].tau].begin;
    emit(t, {{&a, ACC_RW}});
  }
  void trunc(int c, const Term& term) {
    HView cu = lr_u(c), cv = lr_v(c);
    trunc_lr(p_.lr_index[c], cu, cv, term);
  }
  // C <- T_eps(C + term) for the low-rank factors (cu, cv) of lr index li
  void trunc_lr(int li, const HView& cu, const HView& cv, const Term& term) {
    const LrDesc& d = p_.lr[li];
    int kb = term.u.v.cols;  // static bound of the term's rank
    if (d.cap + kb > kMaxK) fail("stacked rank above 128 in a truncated addition");
    Task t = blank(OP_TRUNC);
    t.lr = li;
    t.r0 = term.r0;
    t.c0 = term.c0;
    t.alpha = term.alpha;
    t.a = term.u.v;
    t.b = term.v.v;
    emit(t, {{&term.u, ACC_R}, {&term.v, ACC_R}, {&cu, ACC_RW}, {&cv, ACC_RW}});
  }

  // ---- exact products (no truncation) ---------------------------------------
  // y += alpha B x
  void hmat_mul_into(const HView& y, double alpha, int b, const HView& x) {
    const BlockNode& bn = t_.bl[b];
    if (bn.kind == BK_DENSE) {
      gemm(y, alpha, dense(b), x, 1.0);
    } else if (bn.kind == BK_LOWRANK) {
      lr_mul_into(y, alpha, lr_u(b), lr_v(b), x);
    } else {
      int64_t rb = t_.cl[bn.tau].begin, cb = t_.cl[bn.sigma].begin;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          int s = bn.son[2 * i + j];
          const Cluster& ct = t_.cl[t_.bl[s].tau];
          const Cluster& cs = t_.cl[t_.bl[s].sigma];
          hmat_mul_into(rows(y, (int32_t)(ct.begin - rb), (int32_t)(ct.end - rb)), alpha, s,
                        rows(x, (int32_t)(cs.begin - cb), (int32_t)(cs.end - cb)));
        }
    }
  }
  // y += alpha U (V^T x) for the factors U (m x k), V (n2 x k) of a low-rank
  // leaf.  Large ones become P partial products W_p = V_p^T x_p over row
  // chunks of x (one FP64 temporary, k x c each at a fixed stride) and Q
  // tasks y_q += alpha U_q (W_0 + ... + W_{P-1}) over row chunks of y, so
  // that one product runs on P + Q workgroups instead of one.
  void lr_mul_into(const HView& y, double alpha, const HView& U, const HView& V, const HView& x) {
    const int32_t m = y.v.rows, n2 = V.v.rows;
    if (split_ <= 0 || in_seq_ || folds_into_block(y.v, x.v) || std::max(m, n2) < 2 * split_) {
      lrgemm(y, alpha, U, transpose(V), x, 1.0);
      return;
    }
    const int32_t cap = U.v.cols, cw = x.v.cols;
    const int P = (n2 + split_ - 1) / split_, Q = (m + split_ - 1) / split_;
    HView W = temp(cap, cw * P, -1);
    const int64_t stride = (int64_t)cap * cw;
    auto part = [&](int p) {
      HView w = W;
      w.v.off = W.v.off + p * stride;
      w.v.cols = cw;
      w.v.dyn = DYN_ROWS | DYN_COLS2;
      w.v.rank_id = U.v.rank_id;
      w.v.rank_id2 = x.v.rank_id;
      w.rect = Rect{0, cap, p * cw, (p + 1) * cw};
      return w;
    };
    for (int p = 0; p < P; ++p) {
      const int32_t r0 = (int32_t)((int64_t)n2 * p / P), r1 = (int32_t)((int64_t)n2 * (p + 1) / P);
      gemm(part(p), 1.0, transpose(rows(V, r0, r1)), rows(x, r0, r1), 0.0);
    }
    HView w0 = part(0);
    w0.rect = W.rect;
    for (int q = 0; q < Q; ++q) {
      const int32_t r0 = (int32_t)((int64_t)m * q / Q), r1 = (int32_t)((int64_t)m * (q + 1) / Q);
      HView yq = rows(y, r0, r1), uq = rows(U, r0, r1);
      Task t = blank(OP_GEMMP);
      t.alpha = alpha;
      t.beta = 1.0;
      t.y = yq.v;
      t.a = uq.v;
      t.b = w0.v;
      t.r0 = P;
      t.piv = stride;
      emit(t, {{&uq, ACC_R}, {&w0, ACC_R}, {&yq, ACC_RW}});
    }
  }
  // y += alpha B^T x
  void hmat_tmul_into(const HView& y, double alpha, int b, const HView& x) {
    const BlockNode& bn = t_.bl[b];
    if (bn.kind == BK_DENSE) {
      gemm(y, alpha, transpose(dense(b)), x, 1.0);
    } else if (bn.kind == BK_LOWRANK) {
      lr_mul_into(y, alpha, lr_v(b), lr_u(b), x);
    } else {
      int64_t rb = t_.cl[bn.tau].begin, cb = t_.cl[bn.sigma].begin;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          int s = bn.son[2 * i + j];
          const Cluster& ct = t_.cl[t_.bl[s].tau];
          const Cluster& cs = t_.cl[t_.bl[s].sigma];
          hmat_tmul_into(rows(y, (int32_t)(cs.begin - cb), (int32_t)(cs.end - cb)), alpha, s,
                         rows(x, (int32_t)(ct.begin - rb), (int32_t)(ct.end - rb)));
        }
    }
  }

  // alpha A B as exact low-rank terms (the leaf-case products after Algorithm 1).
  void product_terms(double alpha, int a, int b, int32_t ro, int32_t co, std::vector<Term>& out) {
    const BlockNode& A = t_.bl[a];
    const BlockNode& B = t_.bl[b];
    int32_t ra = (int32_t)t_.cl[A.tau].size();
    int32_t cb_ = (int32_t)t_.cl[B.sigma].size();
    if (A.kind == BK_STRUCT && B.kind == BK_STRUCT) {
      int64_t rbase = t_.cl[A.tau].begin, cbase = t_.cl[B.sigma].begin;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int l = 0; l < 2; ++l) {
            int sa = A.son[2 * i + l], sb = B.son[2 * l + j];
            int32_t r = (int32_t)(t_.cl[t_.bl[sa].tau].begin - rbase);
            int32_t c = (int32_t)(t_.cl[t_.bl[sb].sigma].begin - cbase);
            product_terms(alpha, sa, sb, ro + r, co + c, out);
          }
      return;
    }
    Term tm;
    tm.r0 = ro;
    tm.c0 = co;
    tm.alpha = alpha;
    if (A.kind == BK_LOWRANK) {
      // U = U_A, V = B^T V_A
      int li = p_.lr_index[a];
      HView z = temp(cb_, p_.lr[li].cap, li);
      if (B.kind == BK_DENSE)
        gemm(z, 1.0, transpose(dense(b)), lr_v(a), 0.0);
      else if (B.kind == BK_LOWRANK)
        lrgemm(z, 1.0, lr_v(b), transpose(lr_u(b)), lr_v(a), 0.0);
      else {
        zero(z);
        hmat_tmul_into(z, 1.0, b, lr_v(a));
      }
      tm.u = lr_u(a);
      tm.v = z;
    } else if (B.kind == BK_LOWRANK) {
      // U = A U_B, V = V_B
      int li = p_.lr_index[b];
      HView y = temp(ra, p_.lr[li].cap, li);
      if (A.kind == BK_DENSE)
        gemm(y, 1.0, dense(a), lr_u(b), 0.0);
      else {
        zero(y);
        hmat_mul_into(y, 1.0, a, lr_u(b));
      }
      tm.u = y;
      tm.v = lr_v(b);
    } else if (A.kind == BK_DENSE && B.kind == BK_DENSE) {
      if (t_.cl[A.sigma].leaf()) {
        tm.u = dense(a);
        tm.v = transpose(dense(b));
      } else {
        HView y = temp(ra, cb_, -1);
        gemm(y, 1.0, dense(a), dense(b), 0.0);
        tm.u = y;
        tm.v = ident(cb_);
      }
    } else if (A.kind == BK_DENSE) {
      // B structured, row cluster of A is a leaf: U = I, V = B^T A^T
      HView z = temp(cb_, ra, -1);
      zero(z);
      hmat_tmul_into(z, 1.0, b, transpose(dense(a)));
      tm.u = ident(ra);
      tm.v = z;
    } else {
      // A structured, B dense, column cluster of B is a leaf: U = A B, V = I
      HView y = temp(ra, cb_, -1);
      zero(y);
      hmat_mul_into(y, 1.0, a, dense(b));
      tm.u = y;
      tm.v = ident(cb_);
    }
    out.push_back(tm);
  }

  // Restrict a term to rows [rl, rh) x cols [cl, ch) of its target (relative);
  // returns false if empty.  Identity factors are materialised when sliced.
  bool restrict_term(const Term& in, int32_t rl, int32_t rh, int32_t cl, int32_t ch, Term& out) {
    int32_t mu = in.u.v.rows, mv = in.v.v.rows;
    int32_t a0 = std::max(in.r0, rl), a1 = std::min(in.r0 + mu, rh);
    int32_t b0 = std::max(in.c0, cl), b1 = std::min(in.c0 + mv, ch);
    if (a0 >= a1 || b0 >= b1) return false;
    out = in;
    out.r0 = a0 - rl;
    out.c0 = b0 - cl;
    if (a0 != in.r0 || a1 != in.r0 + mu) out.u = slice_factor(in.u, a0 - in.r0, a1 - in.r0);
    if (b0 != in.c0 || b1 != in.c0 + mv) out.v = slice_factor(in.v, b0 - in.c0, b1 - in.c0);
    return true;
  }
  HView slice_factor(const HView& f, int32_t a, int32_t b) {
    if (f.v.type != VT_IDENT) return rows(f, a, b);
    // rows [a, b) of I_m: a (b-a) x m matrix with ones at (i, a+i)
    int32_t m = f.v.rows;
    HView z = temp(b - a, m, -1);
    zero(z);
    HView e = ident(b - a);
    // copy I_{b-a} into columns [a, b) of z
    HView zc = z;
    zc.v.off += (int64_t)a * z.v.cs;
    zc.v.cols = b - a;
    zc.rect.c0 = a;
    zc.rect.c1 = b;
    Task t = blank(OP_COPY);
    t.y = zc.v;
    t.a = e.v;
    emit(t, {{&zc, ACC_W}});
    return z;
  }

  void add_term_to_leaf(int c, const Term& tm) {
    const BlockNode& C = t_.bl[c];
    // A term wider than half the stacked-rank limit (a dense-dense product
    // over an inner leaf of more than 64 points, or an identity factor of
    // such a leaf) is added as column chunks of at most 64, so that a
    // truncation never stacks more than 128 columns.
    constexpr int32_t kChunk = kMaxK / 2;
    if (C.kind == BK_LOWRANK && tm.u.v.cols > kChunk) {
      const int32_t k = tm.u.v.cols;
      for (int32_t j0 = 0; j0 < k; j0 += kChunk) {
        const int32_t j1 = std::min(k, j0 + kChunk);
        Term part = tm;
        part.u = cols(tm.u, j0, j1);
        part.v = cols(tm.v, j0, j1);
        add_term_to_leaf(c, part);
      }
      return;
    }
    if (C.kind == BK_LOWRANK && lazy_ && scope_ > 0) {
      pin(tm.u, 1);
      pin(tm.v, 1);
      if (pending_[c].empty()) touched_.push_back(c);
      pending_[c].push_back(tm);
      return;
    }
    if (C.kind == BK_DENSE) {
      HView y = dense(c);
      HView ys = rows(y, tm.r0, tm.r0 + tm.u.v.rows);
      // column slice [c0, c0 + rows(V))
      ys.v.off += (int64_t)tm.c0 * ys.v.cs;
      ys.v.cols = tm.v.v.rows;
      ys.rect.c0 = tm.c0;
      ys.rect.c1 = tm.c0 + tm.v.v.rows;
      gemm(ys, tm.alpha, tm.u, transpose(tm.v), 1.0);
    } else {
      trunc(c, tm);
    }
  }

  void leaf_update(double alpha, int a, int b, int c) {
    std::vector<Term> terms;
    product_terms(alpha, a, b, 0, 0, terms);
    const BlockNode& C = t_.bl[c];
    if (C.kind != BK_STRUCT) {
      for (auto& tm : terms) add_term_to_leaf(c, tm);
      return;
    }
    if (terms.size() != 1) {
      fail("structured target with a multi-term product");
      return;
    }
    int64_t br = t_.cl[C.tau].begin, bc = t_.cl[C.sigma].begin;
    std::function<void(int)> visit = [&](int x) {
      const BlockNode& X = t_.bl[x];
      if (X.kind == BK_STRUCT) {
        for (int k = 0; k < 4; ++k) visit(X.son[k]);
        return;
      }
      const Cluster& ct = t_.cl[X.tau];
      const Cluster& cs = t_.cl[X.sigma];
      Term r;
      if (restrict_term(terms[0], (int32_t)(ct.begin - br), (int32_t)(ct.end - br), (int32_t)(cs.begin - bc),
                        (int32_t)(cs.end - bc), r))
        add_term_to_leaf(x, r);
    };
    visit(c);
  }

  // New accumulator: a low-rank buffer with the target's shape and capacity,
  // its own rank slot, storage from the temporaries.
  int new_accumulator(int c, HView& u, HView& v) {
    const LrDesc& dc = p_.lr[p_.lr_index[c]];
    int li = (int)p_.lr.size();
    u = temp(dc.m, dc.cap, -1);
    v = temp(dc.n, dc.cap, -1);
    LrDesc d;
    d.u_off = u.v.off;
    d.v_off = v.v.off;
    d.m = dc.m;
    d.n = dc.n;
    d.cap = dc.cap;
    d.type = temp_type_;
    p_.lr.push_back(d);
    p_.lr_block.push_back(-1);
    lr_obj_.push_back({u.obj, v.obj});
    u.v.dyn = v.v.dyn = DYN_COLS;
    u.v.rank_id = v.v.rank_id = li;
    return li;
  }
  // acc <- T(t1 + t2), returned as a term
  Term combine(int c, const Term& t1, const Term& t2) {
    HView u, v;
    int li = new_accumulator(c, u, v);
    int kb = t1.u.v.cols + t2.u.v.cols;
    if (kb > kMaxK) fail("stacked rank above 128 in a combined truncation");
    Task t = blank(OP_TRUNC2);
    t.lr = li;
    t.a = t1.u.v;
    t.b = t1.v.v;
    t.r0 = t1.r0;
    t.c0 = t1.c0;
    t.alpha = t1.alpha;
    t.x = t2.u.v;
    t.y = t2.v.v;
    t.row0 = t2.r0;
    t.c1 = t2.c0;
    t.beta = t2.alpha;
    emit(t, {{&t1.u, ACC_R}, {&t1.v, ACC_R}, {&t2.u, ACC_R}, {&t2.v, ACC_R}, {&u, ACC_W}, {&v, ACC_W}});
    Term r;
    r.u = u;
    r.v = v;
    r.r0 = r.c0 = 0;
    r.alpha = 1.0;
    pin(u, 1);
    pin(v, 1);
    return r;
  }
  // Apply the collected updates of low-rank leaf c: pairwise truncated
  // additions in a balanced tree, then one truncated addition into c.
  void flush(int c) {
    std::vector<Term> terms;
    terms.swap(pending_[c]);
    std::vector<Term> made;
    std::vector<Term> level = terms;
    while (level.size() > 1) {
      std::vector<Term> next;
      for (size_t i = 0; i + 1 < level.size(); i += 2) {
        next.push_back(combine(c, level[i], level[i + 1]));
        made.push_back(next.back());
      }
      if (level.size() % 2) next.push_back(level.back());
      level.swap(next);
    }
    if (!level.empty()) trunc(c, level[0]);
    for (auto& tm : terms) {
      pin(tm.u, -1);
      pin(tm.v, -1);
    }
    for (auto& tm : made) {
      pin(tm.u, -1);
      pin(tm.v, -1);
    }
  }
  void flush_all() {
    for (size_t b = 0; b < pending_.size(); ++b)
      if (!pending_[b].empty()) flush((int)b);
  }
  void set_lazy(bool v) { lazy_ = v; }

  // Algorithm 1.  With lazy updates a top-level call collects the updates it
  // makes to each low-rank leaf and applies them when it returns (hmul as
  // add_upd followed by apply_upd, Sec. 2.3).
  void hmul(double alpha, int a, int b, int c) {
    const bool top = scope_ == 0;
    ++scope_;
    const BlockNode& A = t_.bl[a];
    const BlockNode& B = t_.bl[b];
    const BlockNode& C = t_.bl[c];
    if (A.kind == BK_STRUCT && B.kind == BK_STRUCT && C.kind == BK_STRUCT) {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int l = 0; l < 2; ++l) hmul(alpha, A.son[2 * i + l], B.son[2 * l + j], C.son[2 * i + j]);
    } else {
      const int prev = begin_call(PT_HMUL, a, b, c);
      leaf_update(alpha, a, b, c);
      call_ = prev;
    }
    --scope_;
    if (top) {
      std::vector<int> leaves;
      leaves.swap(touched_);
      for (int x : leaves)
        if (!pending_[x].empty()) flush(x);
    }
  }

  // ---- accumulated updates (Sec. 2.3, Algorithms 4-8), lazy mode 2 --------
  // Every block that receives updates gets an accumulator: a dense m x n
  // temporary for a dense leaf, else low-rank factors (temporaries of the
  // block's shape and the plan's rank capacity, with their own rank slot)
  // truncated on every addition.  Products whose three blocks are structured
  // stay pending until shift_upd splits them one level.
  struct Acc {
    int li = -1;          // low-rank accumulator: its lr index, or -1
    HView u, v;           // its factors
    bool dense = false;   // dense accumulator of a dense leaf
    HView d;
    std::vector<std::tuple<double, int, int>> pend;  // pending (alpha, A, B)
  };
  Acc& acc(int c) {
    auto it = accs_.find(c);
    if (it == accs_.end()) it = accs_.emplace(c, Acc()).first;
    return it->second;
  }
  // U_C := U_C + term (one truncation, or a GEMM into a dense accumulator)
  void acc_add_term(int c, const Term& tm) {
    const BlockNode& C = t_.bl[c];
    const int32_t m = (int32_t)t_.cl[C.tau].size(), n = (int32_t)t_.cl[C.sigma].size();
    Acc& A = acc(c);
    if (C.kind == BK_DENSE) {
      if (!A.dense) {
        A.d = temp(m, n, -1);
        zero(A.d);
        pin(A.d, 1);
        A.dense = true;
      }
      HView ys = rows(A.d, tm.r0, tm.r0 + tm.u.v.rows);
      ys.v.off += (int64_t)tm.c0 * ys.v.cs;
      ys.v.cols = tm.v.v.rows;
      ys.rect.c0 = tm.c0;
      ys.rect.c1 = tm.c0 + tm.v.v.rows;
      gemm(ys, tm.alpha, tm.u, transpose(tm.v), 1.0);
      return;
    }
    if (A.li < 0) {
      LrDesc d;
      d.m = m;
      d.n = n;
      d.cap = (int32_t)std::min<int64_t>(p_.cap, std::min(m, n));
      A.u = temp(m, d.cap, -1);
      A.v = temp(n, d.cap, -1);
      d.u_off = A.u.v.off;
      d.v_off = A.v.v.off;
      d.type = temp_type_;
      A.li = (int)p_.lr.size();
      p_.lr.push_back(d);
      p_.lr_block.push_back(-1);
      lr_obj_.push_back({A.u.obj, A.v.obj});
      A.u.v.dyn = A.v.v.dyn = DYN_COLS;
      A.u.v.rank_id = A.v.v.rank_id = A.li;
      pin(A.u, 1);
      pin(A.v, 1);
    }
    // a term wider than half the stacked-rank limit goes in column chunks
    constexpr int32_t kChunk = kMaxK / 2;
    if (tm.u.v.cols > kChunk) {
      for (int32_t j0 = 0; j0 < tm.u.v.cols; j0 += kChunk) {
        const int32_t j1 = std::min(tm.u.v.cols, j0 + kChunk);
        Term part = tm;
        part.u = cols(tm.u, j0, j1);
        part.v = cols(tm.v, j0, j1);
        trunc_lr(A.li, A.u, A.v, part);
      }
      return;
    }
    trunc_lr(A.li, A.u, A.v, tm);
  }
  // Algorithm 4
  void add_upd(double alpha, int a, int b, int c) {
    const BlockNode& A = t_.bl[a];
    const BlockNode& B = t_.bl[b];
    const BlockNode& C = t_.bl[c];
    if (A.kind == BK_STRUCT && B.kind == BK_STRUCT && C.kind == BK_STRUCT) {
      acc(c).pend.emplace_back(alpha, a, b);
      return;
    }
    const int prev = begin_call(PT_HMUL, a, b, c);
    std::vector<Term> terms;
    product_terms(alpha, a, b, 0, 0, terms);
    for (const Term& tm : terms) acc_add_term(c, tm);
    call_ = prev;
  }
  // Algorithm 6 (C structured)
  void shift_upd(int c) {
    auto it = accs_.find(c);
    if (it == accs_.end()) return;
    Acc A = std::move(it->second);
    accs_.erase(it);
    const BlockNode& C = t_.bl[c];
    const int64_t rb = t_.cl[C.tau].begin, cb = t_.cl[C.sigma].begin;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        const int son = C.son[2 * i + j];
        const Cluster& ct = t_.cl[t_.bl[son].tau];
        const Cluster& cs = t_.cl[t_.bl[son].sigma];
        if (A.li >= 0) {
          Term r;
          r.u = rows(A.u, (int32_t)(ct.begin - rb), (int32_t)(ct.end - rb));
          r.v = rows(A.v, (int32_t)(cs.begin - cb), (int32_t)(cs.end - cb));
          r.r0 = r.c0 = 0;
          r.alpha = 1.0;
          acc_add_term(son, r);
        }
        for (auto& pd : A.pend) {
          const BlockNode& PA = t_.bl[std::get<1>(pd)];
          const BlockNode& PB = t_.bl[std::get<2>(pd)];
          for (int l = 0; l < 2; ++l) add_upd(std::get<0>(pd), PA.son[2 * i + l], PB.son[2 * l + j], son);
        }
      }
    if (A.li >= 0) {
      pin(A.u, -1);
      pin(A.v, -1);
    }
  }
  // Algorithm 5
  void apply_upd(int c) {
    const BlockNode& C = t_.bl[c];
    if (C.kind == BK_STRUCT) {
      shift_upd(c);
      for (int k = 0; k < 4; ++k) apply_upd(C.son[k]);
      return;
    }
    auto it = accs_.find(c);
    if (it == accs_.end()) return;
    Acc A = std::move(it->second);
    accs_.erase(it);
    if (A.dense) {
      const int32_t n = (int32_t)t_.cl[C.sigma].size();
      gemm(dense(c), 1.0, A.d, ident(n), 1.0);
      pin(A.d, -1);
    }
    if (A.li >= 0) {
      Term r;
      r.u = A.u;
      r.v = A.v;
      r.r0 = r.c0 = 0;
      r.alpha = 1.0;
      trunc(c, r);
      pin(A.u, -1);
      pin(A.v, -1);
    }
  }
  // Algorithm 8: L X = M (X overwrites M)
  void htrsl_acc(int ld, int m) {
    const BlockNode& M = t_.bl[m];
    const BlockNode& L = t_.bl[ld];
    if (M.kind == BK_STRUCT) {
      shift_upd(m);
      for (int j = 0; j < 2; ++j) htrsl_acc(L.son[0], M.son[j]);
      for (int j = 0; j < 2; ++j) add_upd(-1.0, L.son[2], M.son[j], M.son[2 + j]);
      for (int j = 0; j < 2; ++j) htrsl_acc(L.son[3], M.son[2 + j]);
    } else {
      apply_upd(m);
      const int prev = begin_call(PT_HTRSL, ld, m, m);
      solve_lower(ld, M.kind == BK_DENSE ? dense(m) : lr_u(m));
      call_ = prev;
    }
  }
  // the mirror of Algorithm 8: X U = M
  void htrsu_acc(int ud, int m) {
    const BlockNode& M = t_.bl[m];
    const BlockNode& U = t_.bl[ud];
    if (M.kind == BK_STRUCT) {
      shift_upd(m);
      for (int j = 0; j < 2; ++j) htrsu_acc(U.son[0], M.son[2 * j]);
      for (int j = 0; j < 2; ++j) add_upd(-1.0, M.son[2 * j], U.son[1], M.son[2 * j + 1]);
      for (int j = 0; j < 2; ++j) htrsu_acc(U.son[3], M.son[2 * j + 1]);
    } else {
      apply_upd(m);
      const int prev = begin_call(PT_HTRSU, ud, m, m);
      solve_upper_t(ud, M.kind == BK_DENSE ? transpose(dense(m)) : lr_v(m));
      call_ = prev;
    }
  }
  // Algorithm 7
  void hlu_acc(int a) {
    const BlockNode& A = t_.bl[a];
    if (A.kind == BK_STRUCT) {
      shift_upd(a);
      hlu_acc(A.son[0]);
      htrsu_acc(A.son[0], A.son[2]);
      htrsl_acc(A.son[0], A.son[1]);
      add_upd(-1.0, A.son[2], A.son[1], A.son[3]);
      hlu_acc(A.son[3]);
    } else {
      apply_upd(a);
      const int prev = begin_call(PT_HLU, a, a, a);
      getrf(a);
      trtri(a);
      call_ = prev;
    }
  }
  bool accs_empty() const { return accs_.empty(); }

  // Panel solves over a diagonal block (leaf or structured).
  void solve_lower(int d, const HView& x) {
    const BlockNode& D = t_.bl[d];
    if (coarsen_ > 0 && !in_seq_ && t_.cl[D.tau].size() <= coarsen_) {
      seq_block(d, x, false);
      return;
    }
    if (D.kind == BK_DENSE) {
      trsm(OP_TRSM_L, d, x);
      return;
    }
    int32_t n0 = (int32_t)t_.cl[t_.bl[D.son[0]].tau].size(), nn = (int32_t)t_.cl[D.tau].size();
    HView x0 = rows(x, 0, n0), x1 = rows(x, n0, nn);
    solve_lower(D.son[0], x0);
    hmat_mul_into(x1, -1.0, D.son[2], x0);
    solve_lower(D.son[3], x1);
  }
  void solve_upper_t(int d, const HView& x) {
    const BlockNode& D = t_.bl[d];
    if (D.kind == BK_DENSE) {
      trsm(OP_TRSM_UT, d, x);
      return;
    }
    int32_t n0 = (int32_t)t_.cl[t_.bl[D.son[0]].tau].size(), nn = (int32_t)t_.cl[D.tau].size();
    HView x0 = rows(x, 0, n0), x1 = rows(x, n0, nn);
    solve_upper_t(D.son[0], x0);
    hmat_tmul_into(x1, -1.0, D.son[1], x0);
    solve_upper_t(D.son[3], x1);
  }
  void solve_upper(int d, const HView& x) {
    const BlockNode& D = t_.bl[d];
    if (coarsen_ > 0 && !in_seq_ && t_.cl[D.tau].size() <= coarsen_) {
      seq_block(d, x, true);
      return;
    }
    if (D.kind == BK_DENSE) {
      trsm(OP_TRSM_U, d, x);
      return;
    }
    int32_t n0 = (int32_t)t_.cl[t_.bl[D.son[0]].tau].size(), nn = (int32_t)t_.cl[D.tau].size();
    HView x0 = rows(x, 0, n0), x1 = rows(x, n0, nn);
    solve_upper(D.son[3], x1);
    hmat_mul_into(x0, -1.0, D.son[1], x1);
    solve_upper(D.son[0], x0);
  }

  // ---- coarsened substitution (the remark after Algorithm 11) ---------------
  // Diagonal blocks of at most coarsen_ rows are the coarse blocks: the first
  // ones on each path from the root (a larger diagonal leaf is none).
  void coarse_blocks(int d) {
    const BlockNode& D = t_.bl[d];
    const Cluster& c = t_.cl[D.tau];
    if (c.size() <= coarsen_) {
      const int id = (int)cb_begin_.size();
      cb_begin_.push_back(c.begin);
      cb_end_.push_back(c.end);
      for (int64_t r = c.begin; r < c.end; ++r) cb_of_row_[(size_t)r] = id;
      return;
    }
    if (D.kind != BK_STRUCT) return;
    coarse_blocks(D.son[0]);
    coarse_blocks(D.son[3]);
  }
  bool is_panel(const View& v) const {
    return v.type == VT_F64 && (v.dyn & DYN_COLS) && v.rank_id == p_.nrhs_slot && v.off >= p_.panel_off &&
           v.off < p_.panel_off + t_.n;
  }
  // coarse block holding every row of a panel view, or -1
  int block_of(const View& v) const {
    const int64_t r = v.off - p_.panel_off;
    if (v.rows <= 0) return -1;
    const int b = cb_of_row_[(size_t)r];
    return b >= 0 && cb_of_row_[(size_t)(r + v.rows - 1)] == b ? b : -1;
  }
  // A product y += alpha A x (or alpha U (V^T x)) whose rows y lie in a coarse
  // block and whose source x is the whole neighbouring block just solved in
  // this sweep is folded into y's block task: it is the last update the block
  // waits for, and inside the task it needs no hand-off.
  // A product y += ... x with y inside coarse block by folds into by's task
  // when its source x lies in the coarse blocks among the fold_reach_
  // blocks before by in sweep order (with reach 1: the neighbour, the last
  // update by waits for; with more, products whose own task would finish
  // after the neighbour's block task).
  bool folds_into_block(const View& y, const View& x) const {
    if (coarsen_ <= 0 || !sub_ || !is_panel(y) || !is_panel(x) || x.rows <= 0) return false;
    const int by = block_of(y);
    if (by < 0 || cb_sweep_[by] == sweep_) return false;
    const int64_t r0 = x.off - p_.panel_off, r1 = r0 + x.rows;
    const int bf = cb_of_row_[(size_t)r0], bl = cb_of_row_[(size_t)(r1 - 1)];
    if (bf < 0 || bl < 0) return false;
    for (int k = bf; k < bl; ++k)
      if (cb_end_[k] != cb_begin_[k + 1]) return false;  // the blocks must tile x's rows
    if (sweep_ > 0) return bl < by && by - bf <= fold_reach_;
    return bf > by && bl - by <= fold_reach_;
  }
  // Rows of y's first coarse block (in sweep order) when y covers several
  // whole coarse blocks and x folds into that first block; else 0.
  int32_t fold_cut(const View& y, const View& x) const {
    if (coarsen_ <= 0 || !sub_ || in_seq_ || !is_panel(y) || y.rows <= 0) return 0;
    const int64_t r0 = y.off - p_.panel_off, r1 = r0 + y.rows;
    const int b0 = cb_of_row_[(size_t)r0], b1 = cb_of_row_[(size_t)(r1 - 1)];
    if (b0 < 0 || b1 < 0 || b0 == b1 || r0 != cb_begin_[b0] || r1 != cb_end_[b1]) return 0;
    for (int k = b0; k < b1; ++k)
      if (cb_end_[k] != cb_begin_[k + 1]) return 0;
    const int first = sweep_ > 0 ? b0 : b1;
    View yb = y;
    yb.off = p_.panel_off + cb_begin_[first];
    yb.rows = (int32_t)(cb_end_[first] - cb_begin_[first]);
    return folds_into_block(yb, x) ? yb.rows : 0;
  }
  bool defer_neighbour(const Task& tk) {
    const View& x = tk.op == OP_GEMM ? tk.b : tk.x;
    if (tk.beta != 1.0 || !folds_into_block(tk.y, x)) return false;
    const int by = block_of(tk.y);
    Task u = tk;
    u.y.off = tk.y.off - p_.panel_off - cb_begin_[by];
    u.y.dyn |= DYN_LOCAL;
    deferred_[by].push_back(u);
    const int64_t r0 = x.off - p_.panel_off;
    def_lo_[by] = std::min(def_lo_[by], r0);
    def_hi_[by] = std::max(def_hi_[by], r0 + x.rows);
    return true;
  }
  // micro-operation of the open block: panel views become block-local
  void seq_op(Task tk) {
    if (tk.op != OP_TRSM_L && tk.op != OP_TRSM_U && tk.op != OP_GEMM && tk.op != OP_LRGEMM)
      return fail("internal: task kind inside a coarsened block");
    if ((tk.op == OP_GEMM || tk.op == OP_LRGEMM) && tk.beta != 1.0)
      return fail("internal: overwriting product inside a coarsened block");
    for (View* v : {&tk.y, &tk.a, &tk.b, &tk.x}) {
      if (!is_panel(*v)) continue;
      const int64_t r = v->off - p_.panel_off - seq_w0_;
      if (r < 0 || r + v->rows > seq_W_ || v->rs != 1) return fail("internal: panel view outside its coarsened block");
      v->off = r;
      v->dyn |= DYN_LOCAL;
    }
    seq_cur_.push_back(tk);
  }
  // One task for the substitution of diagonal block d (rows x): its leaf
  // triangular solves and products in the order of the recursion, after the
  // product from the neighbouring block if that was folded in.
  void seq_block(int d, const HView& x, bool upper) {
    const int b = block_of(x.v);
    if (b < 0 || x.v.rows != cb_end_[b] - cb_begin_[b]) return fail("internal: coarsened block off its rows");
    in_seq_ = true;
    seq_w0_ = x.v.off - p_.panel_off;
    seq_W_ = x.v.rows;
    seq_cur_.assign(deferred_[b].begin(), deferred_[b].end());
    const bool folded = !deferred_[b].empty();
    const int64_t src_lo = def_lo_[b], src_hi = def_hi_[b];
    deferred_[b].clear();
    def_lo_[b] = INT64_MAX;
    def_hi_[b] = -1;
    if (upper)
      solve_upper(d, x);
    else
      solve_lower(d, x);
    in_seq_ = false;
    cb_sweep_[b] = sweep_;
    Task t = blank(OP_SEQ);
    t.y = x.v;
    t.piv = (int64_t)d_.seq.size();
    t.lr = (int32_t)seq_cur_.size();
    d_.seq.insert(d_.seq.end(), seq_cur_.begin(), seq_cur_.end());
    seq_cur_.clear();
    if (folded) {
      HView src = rows(panel(), (int32_t)src_lo, (int32_t)src_hi);
      emit(t, {{&src, ACC_R}, {&x, ACC_RW}});
    } else {
      emit(t, {{&x, ACC_RW}});
    }
  }

  // Algorithm 3: L X = M (X overwrites M)
  void htrsl(int ld, int m) {
    const BlockNode& M = t_.bl[m];
    const BlockNode& L = t_.bl[ld];
    if (M.kind == BK_STRUCT) {
      for (int j = 0; j < 2; ++j) htrsl(L.son[0], M.son[j]);
      for (int j = 0; j < 2; ++j) hmul(-1.0, L.son[2], M.son[j], M.son[2 + j]);
      for (int j = 0; j < 2; ++j) htrsl(L.son[3], M.son[2 + j]);
    } else {
      const int prev = begin_call(PT_HTRSL, ld, m, m);
      solve_lower(ld, M.kind == BK_DENSE ? dense(m) : lr_u(m));
      call_ = prev;
    }
  }
  // Mirror of Algorithm 3: X U = M (X overwrites M)
  void htrsu(int ud, int m) {
    const BlockNode& M = t_.bl[m];
    const BlockNode& U = t_.bl[ud];
    if (M.kind == BK_STRUCT) {
      for (int j = 0; j < 2; ++j) htrsu(U.son[0], M.son[2 * j]);
      for (int j = 0; j < 2; ++j) hmul(-1.0, M.son[2 * j], U.son[1], M.son[2 * j + 1]);
      for (int j = 0; j < 2; ++j) htrsu(U.son[3], M.son[2 * j + 1]);
    } else {
      const int prev = begin_call(PT_HTRSU, ud, m, m);
      solve_upper_t(ud, M.kind == BK_DENSE ? transpose(dense(m)) : lr_v(m));
      call_ = prev;
    }
  }
  // Algorithm 2
  void hlu(int a) {
    const BlockNode& A = t_.bl[a];
    if (A.kind == BK_STRUCT) {
      hlu(A.son[0]);
      htrsu(A.son[0], A.son[2]);
      htrsl(A.son[0], A.son[1]);
      hmul(-1.0, A.son[2], A.son[1], A.son[3]);
      hlu(A.son[3]);
    } else {
      const int prev = begin_call(PT_HLU, a, a, a);
      getrf(a);
      trtri(a);
      call_ = prev;
    }
  }

  void fail(const std::string& m) {
    if (err_.empty()) err_ = m;
  }
  // tasks emitted from now on belong to this paper-level leaf call; returns
  // the previous call
  int begin_call(int fn, int b0, int b1, int b2) {
    const int prev = call_;
    call_ = (int)(d_.calls.size() / 4);
    d_.calls.insert(d_.calls.end(), {fn, b0, b1, b2});
    return prev;
  }

 private:
  struct Pool {
    int64_t limit = 0;
    int64_t next = 0;
    std::vector<int64_t> off;
    std::vector<int> obj;
    std::vector<int> pins;  // collected updates still referring to the slot
  };
  void pin(const HView& h, int d) {
    if (h.pool_cls >= 0) pools_[h.pool_cls].pins[h.pool_slot] += d;
  }
  int new_obj() {
    objs_.emplace_back();
    owner_.push_back(-1);
    return (int)objs_.size() - 1;
  }
  void access(int task, int obj, const Rect& r, bool write) {
    ObjState& o = objs_[obj];
    if (!o.inh_w.empty() || !o.inh_r.empty()) {
      for (auto& w : o.inh_w)
        if (w.task != task) preds_.push_back(w.task);
      if (write) {
        for (auto& rd : o.inh_r)
          if (rd.task != task) preds_.push_back(rd.task);
        if (covers(r, o.full)) {
          std::vector<Rec>().swap(o.inh_w);
          std::vector<Rec>().swap(o.inh_r);
        }
      }
    }
    for (auto& w : o.writes)
      if (w.task != task && overlap(w.r, r)) preds_.push_back(w.task);
    if (write) {
      for (auto& rd : o.reads)
        if (rd.task != task && overlap(rd.r, r)) preds_.push_back(rd.task);
      o.writes.erase(std::remove_if(o.writes.begin(), o.writes.end(), [&](const Rec& x) { return covers(r, x.r); }),
                     o.writes.end());
      o.reads.erase(std::remove_if(o.reads.begin(), o.reads.end(), [&](const Rec& x) { return covers(r, x.r); }),
                    o.reads.end());
      o.writes.push_back({r, task});
    } else {
      o.reads.push_back({r, task});
    }
  }

  Plan& p_;
  const Tree& t_;
  Dag& d_;
  int tsize_;
  int temp_type_;
  int64_t temp_budget_;
  int64_t temp_base_, temp_top_;
  int panel_obj_ = -1;
  std::vector<int> obj_a_, obj_b_;
  std::vector<int> inv_obj_;                   // inverses of the diagonal leaves
  std::vector<ObjState> objs_;
  std::vector<int> owner_;                     // low-rank leaf owning an object, or -1
  std::vector<std::pair<int, int>> lr_obj_;    // U / V objects of every low-rank index
  std::vector<std::vector<Term>> pending_;     // collected updates per low-rank leaf
  std::vector<int> touched_;                   // leaves with collected updates in this call
  int scope_ = 0;                              // depth of nested hmul calls
  bool lazy_ = false;
  std::map<int, Acc> accs_;                    // accumulators of the accumulated H-LU (lazy mode 2)
  int32_t split_ = 0;                          // row chunk of split low-rank products (solve DAGs)
  // coarsened substitution (OP_SEQ): diagonal blocks of at most coarsen_ rows
  int32_t coarsen_ = 0;
  int sweep_ = 0;                              // +1 forward, -1 backward substitution
  std::vector<int32_t> cb_of_row_;             // coarse block of each panel row, -1 outside
  std::vector<int64_t> cb_begin_, cb_end_;     // panel rows of each coarse block
  std::vector<int> cb_sweep_;                  // the sweep whose block task was emitted
  std::vector<std::vector<Task>> deferred_;    // neighbour products folded into a block's task
  std::vector<int64_t> def_lo_, def_hi_;       // panel rows the folded products read
  int fold_reach_ = 1;                         // blocks back a folded product's source may reach
  bool in_seq_ = false;                        // collecting a block's micro-operations
  int64_t seq_w0_ = 0;
  int32_t seq_W_ = 0;
  std::vector<Task> seq_cur_;
  int32_t call_ = -1;                          // current paper-level leaf call (Dag::calls)
  bool sub_ = false;                           // emitting substitution tasks
  bool solve_dag_ = false;                     // a substitution DAG alone (every released task is kept)
  std::vector<Pool> pools_;
  std::vector<int> preds_;
  std::vector<std::pair<int, int>> edges_;
  std::string err_;
};

}  // namespace

bool trace_lu(Plan& p, int64_t temp_budget_bytes, int lazy) {
  p.lu = Dag();
  p.lr.resize(p.nlr_leaf);
  p.lr_block.resize(p.nlr_leaf);
  Tracer tr(p, p.lu, temp_budget_bytes);
  if (lazy == 2) {
    tr.hlu_acc(0);
    if (tr.ok() && !tr.accs_empty()) tr.fail("internal: accumulated updates never applied");
  } else {
    tr.set_lazy(lazy != 0);
    tr.hlu(0);
  }
  tr.flush_all();
  if (!tr.ok()) {
    p.err = tr.err();
    return false;
  }
  tr.finish();
  p.nrhs_slot = (int)p.lr.size();
  p.nranks = p.nrhs_slot + 1;
  int64_t end = tr.temp_end();
  p.lu_temp_base = p.prec == 1 ? p.blocks_f32 : p.n_f64;
  p.lu_temp_end = end;
  if (p.prec == 1) {
    p.temp_bytes = (end - p.blocks_f32) * 4;
    p.n_f32 = end;
  } else {
    p.temp_bytes = (end - p.n_f64) * 8;
    p.n_f64 = end;
  }
  return true;
}

bool trace_lu_solve(Plan& p, int64_t temp_budget_bytes, int lazy) {
  p.fused = Dag();
  // the H-LU part registers its accumulators again, in the same order
  const std::vector<LrDesc> lr_saved = p.lr;
  const std::vector<int32_t> blk_saved = p.lr_block;
  p.lr.resize(p.nlr_leaf);
  p.lr_block.resize(p.nlr_leaf);
  Tracer tr(p, p.fused, temp_budget_bytes);
  tr.set_temp_base(p.lu_temp_base);
  if (lazy == 2) {
    tr.hlu_acc(0);
  } else {
    tr.set_lazy(lazy != 0);
    tr.hlu(0);
  }
  tr.flush_all();
  tr.begin_substitution();
  HView x = tr.panel();
  tr.solve_lower(0, x);
  tr.solve_upper(0, x);
  bool same = p.lr.size() == lr_saved.size() && p.lr_block == blk_saved;
  for (size_t i = 0; same && i < p.lr.size(); ++i)
    same = p.lr[i].u_off == lr_saved[i].u_off && p.lr[i].v_off == lr_saved[i].v_off && p.lr[i].cap == lr_saved[i].cap;
  if (!tr.ok() || !same || tr.temp_end() != p.lu_temp_end) {
    p.lr = lr_saved;
    p.lr_block = blk_saved;
    p.fused = Dag();
    p.err = tr.ok() ? "internal: the fused trace differs from the H-LU trace" : tr.err();
    return false;
  }
  tr.finish();
  return true;
}

bool trace_solve(Plan& p, int32_t split_rows, int32_t coarsen) {
  p.solve = Dag();
  Tracer tr(p, p.solve, 0);
  tr.set_solve(split_rows, coarsen);
  HView x = tr.panel();
  tr.set_sweep(1);
  tr.solve_lower(0, x);
  tr.set_sweep(-1);
  tr.solve_upper(0, x);
  if (!tr.ok()) {
    p.err = tr.err();
    return false;
  }
  tr.finish();
  p.n_f64 = std::max(p.n_f64, tr.temp_end());
  return true;
}

}  // namespace hm
