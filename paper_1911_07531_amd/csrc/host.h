// Host-side structures: cluster tree, block tree, storage plan and task DAGs.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "hm_internal.h"

namespace hm {

enum BlockKind : int32_t { BK_STRUCT = 0, BK_DENSE = 1, BK_LOWRANK = 2 };

struct Cluster {
  int64_t begin, end;
  double lo[3], hi[3];
  int32_t son[2];
  int32_t level;
  int64_t size() const { return end - begin; }
  bool leaf() const { return son[0] < 0; }
};

struct BlockNode {
  int32_t tau, sigma;
  int32_t kind;
  int32_t son[4];  // (0,0),(0,1),(1,0),(1,1)
};

struct Tree {
  int64_t n = 0;
  int dim = 3;
  int leaf = 0;
  double eta = 0;
  std::vector<int64_t> perm;      // perm[k] = original index of permuted index k
  std::vector<double> pts_perm;   // n x 3 (z = 0 for dim 2), permuted order
  std::vector<Cluster> cl;        // depth-first pre-order
  std::vector<BlockNode> bl;      // depth-first pre-order
};

void build_cluster_tree(const double* pts, int64_t n, int dim, int leaf, Tree& t);
void build_block_tree(Tree& t, double eta);

// Storage of every leaf block inside the arenas, and the traced task DAGs.
// The paper's task kinds (Sec. 3): the leaf-level calls of Algorithms 1-3.
enum PaperFn { PT_HLU = 0, PT_HTRSL = 1, PT_HTRSU = 2, PT_HMUL = 3 };

struct Dag {
  std::vector<Task> tasks;
  // the paper-level leaf call (hlu, htrsl, htrsu, hmul on blocks) that each
  // task belongs to: task_call[i] indexes calls (4 ints: kind, three block
  // indices as in build_semiauto_dag), -1 outside any call
  std::vector<int32_t> task_call;
  std::vector<int32_t> calls;
  std::vector<int32_t> indeg;
  std::vector<int32_t> succ_ptr, succ_idx;
  std::vector<int32_t> level;       // longest-path level of each task
  std::vector<int32_t> level_order; // tasks sorted by level
  std::vector<int32_t> level_ptr;   // start of each level in level_order
  std::vector<int32_t> roots;
  int64_t nedges = 0;
  std::vector<Task> seq;            // micro-operations of the OP_SEQ tasks
  // per edge (aligned with succ_idx): the successor lies on or near the
  // critical path of a static duration estimate
  std::vector<uint8_t> succ_crit;
};

struct Plan {
  const Tree* tree = nullptr;
  int prec = 0;            // 0 = FP64, 1 = mixed (FP32 off-diagonal storage)
  int max_rank = 0;
  int cap = 0;             // stored rank capacity of low-rank leaves
  int nrhs_cap = 64;       // widest solve panel
  // per block (index = block id); -1 where not a leaf
  std::vector<int64_t> data_off;   // dense leaves
  std::vector<int32_t> data_type;
  std::vector<int32_t> lr_index;   // low-rank leaves
  std::vector<int64_t> piv_off;    // diagonal dense leaves
  std::vector<int64_t> inv_off;    // diagonal dense leaves: L^{-1} then U^{-1} (f64, m x m each)
  std::vector<LrDesc> lr;
  std::vector<int32_t> lr_block;
  std::vector<int32_t> diag_leaves;  // diagonal dense leaves in order
  int64_t n_f64 = 0, n_f32 = 0, n_piv = 0;
  int64_t blocks_f64 = 0, blocks_f32 = 0;  // arena prefix that holds block data
  int64_t panel_off = -1;  // solve panel (f64 arena), n x nrhs_cap
  int nranks = 0;          // rank slots (low-rank leaves, accumulators, nrhs slot)
  int nrhs_slot = 0;
  int nlr_leaf = 0;        // low-rank leaves (the first entries of lr); the rest are accumulators
  Dag lu, solve;
  Dag fused;               // H-LU followed by the substitution, one DAG (traced on demand)
  int64_t lu_temp_base = 0, lu_temp_end = 0;  // temporaries of the H-LU trace (its element type)
  int64_t temp_bytes = 0;
  std::string err;
};

// Storage layout for a tree.  prec = 0: every block FP64; prec = 1: diagonal
// leaves FP64, all other blocks FP32.
bool make_layout(const Tree& t, int prec, int max_rank, int nrhs_cap, Plan& p);
// Trace the H-LU (Algorithm 2) and the forward/backward solve into task DAGs.
// lazy: 0 truncate every update as produced (Algorithm 1's order); 1 collect
// the updates one top-level hmul call makes to each low-rank leaf and add them
// with a balanced tree of truncations when it returns; 2 the accumulated
// H-LU of Algorithms 4-8 (accumulators per block, shifted down level by level
// and added into a leaf right before it is factorized or solved).
bool trace_lu(Plan& p, int64_t temp_budget_bytes, int lazy);
// coarsen > 0: diagonal blocks of at most that many rows become one OP_SEQ
// task each (micro-operations in Dag::seq), with the product from the
// neighbouring block folded in.
bool trace_solve(Plan& p, int32_t split_rows, int32_t coarsen = 0);
// The H-LU and the forward/backward substitution traced as one DAG (the
// fusion of composed operations): a block row's substitution may start as
// soon as its factors are final.  The H-LU part is task for task the DAG of
// trace_lu (same temporaries, same accumulators); the substitution's tasks
// carry c1 = 1 and its low-rank products are not split.  Requires trace_lu.
bool trace_lu_solve(Plan& p, int64_t temp_budget_bytes, int lazy);
// The paper's semi-automatic construction of the H-LU task graph (Sec. 3,
// Algorithms 9-11; with sparsify, Algorithm 12 after every refinement step,
// paths of at most max_path edges, 0 = unbounded).  tasks: 4 ints per leaf
// task (kind, blocks: hlu (d, d, d), htrsl (L, M, M), htrsu (U, M, M), hmul
// (A, B, C)), in creation order; edges: pairs of task indices.
void build_semiauto_dag(const Tree& t, bool sparsify, int max_path, std::vector<int32_t>& tasks,
                        std::vector<int32_t>& edges);

}  // namespace hm
