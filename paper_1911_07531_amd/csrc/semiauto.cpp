// Semi-automatic task graph construction for the H-LU of Algorithm 2, at the
// granularity of the paper's tasks (hlu, htrsl, htrsu, hmul on blocks of the
// block tree): task refinement with inherited and refined dependencies
// (Sec. 3, Definition 3.2, Algorithms 9-11) and the removal of redundant edges
// (Sec. 4.1, Algorithm 12).  Host only.  The executed DAGs come from the
// leaf-level tracer (host.cpp); this construction is the paper's method, kept
// beside it so that the two can be compared task for task.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "host.h"

namespace hm {
namespace {

enum MatId { ID_A = 0, ID_L = 1, ID_U = 2 };

struct PTask {
  int fn;                 // PT_HLU, PT_HTRSL, PT_HTRSU, PT_HMUL
  int b[3];               // hlu (d, d, d); htrsl (L, M, M); htrsu (U, M, M); hmul (A, B, C)
  std::vector<int> sub;   // V_t, empty while the task is not refined
  std::vector<int> succ;  // S_t
};

struct Dep {
  int id, blk;
};

class Builder {
 public:
  explicit Builder(const Tree& t) : t_(t) {}

  // Algorithm 11, started from the task of the top-level call hlu(A, L, U)
  void compute(bool sparsify, int max_path) {
    tasks_.clear();
    final_.clear();
    std::vector<int> cur{add(PT_HLU, 0, 0, 0)};
    while (!cur.empty()) {
      for (int g : cur) refine(g);
      std::vector<int> next;
      for (int g : cur) {
        if (tasks_[g].sub.empty()) {
          std::vector<int> old = tasks_[g].succ;
          refine_loc_deps(g);
          if (tasks_[g].succ != old)
            next.push_back(g);
          else
            final_.push_back(g);
        } else {
          refine_sub_deps(g);
          next.insert(next.end(), tasks_[g].sub.begin(), tasks_[g].sub.end());
        }
      }
      if (sparsify)
        for (int g : cur) remove_redundant_around(g, max_path);
      cur.swap(next);
    }
  }

  void result(std::vector<int32_t>& tasks, std::vector<int32_t>& edges) const {
    std::vector<int> pos(tasks_.size(), -1);
    std::vector<int> order(final_);
    std::sort(order.begin(), order.end());
    for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int)i;
    tasks.clear();
    edges.clear();
    for (int g : order) {
      const PTask& x = tasks_[g];
      tasks.insert(tasks.end(), {x.fn, x.b[0], x.b[1], x.b[2]});
    }
    for (int g : order)
      for (int s : tasks_[g].succ) edges.insert(edges.end(), {pos[g], pos[s]});
  }

 private:
  int add(int fn, int b0, int b1, int b2) {
    tasks_.push_back(PTask{fn, {b0, b1, b2}, {}, {}});
    return (int)tasks_.size() - 1;
  }
  bool structured(int b) const { return t_.bl[b].kind == BK_STRUCT; }

  // input and output data of a task (the table of Sec. 3): the H-LU reads A
  // and writes L and U; the updates of A are hmul tasks that read L and U
  static void deps(const PTask& x, Dep* in, int& nin, Dep* out, int& nout) {
    switch (x.fn) {
      case PT_HLU:
        in[0] = {ID_A, x.b[0]};
        nin = 1;
        out[0] = {ID_L, x.b[0]};
        out[1] = {ID_U, x.b[0]};
        nout = 2;
        break;
      case PT_HTRSL:
        in[0] = {ID_L, x.b[0]};
        in[1] = {ID_A, x.b[1]};
        nin = 2;
        out[0] = {ID_U, x.b[1]};
        nout = 1;
        break;
      case PT_HTRSU:
        in[0] = {ID_U, x.b[0]};
        in[1] = {ID_A, x.b[1]};
        nin = 2;
        out[0] = {ID_L, x.b[1]};
        nout = 1;
        break;
      default:
        in[0] = {ID_L, x.b[0]};
        in[1] = {ID_U, x.b[1]};
        nin = 2;
        out[0] = {ID_A, x.b[2]};
        nout = 1;
    }
  }
  bool meet(int b1, int b2) const {
    const BlockNode &x = t_.bl[b1], &y = t_.bl[b2];
    const Cluster &xr = t_.cl[x.tau], &xc = t_.cl[x.sigma], &yr = t_.cl[y.tau], &yc = t_.cl[y.sigma];
    return xr.begin < yr.end && yr.begin < xr.end && xc.begin < yc.end && yc.begin < xc.end;
  }
  // Definition 3.2: an output of x meets an input of y in the same matrix
  bool precedes(int xi, int yi) const {
    Dep in_x[2], out_x[2], in_y[2], out_y[2];
    int a, b, c, d;
    deps(tasks_[xi], in_x, a, out_x, b);
    deps(tasks_[yi], in_y, c, out_y, d);
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < c; ++j)
        if (out_x[i].id == in_y[j].id && meet(out_x[i].blk, in_y[j].blk)) return true;
    return false;
  }

  // V_g and the local edges E_g: the sub-tasks of Algorithms 1-3 in their
  // sequential order, ordered among themselves by Definition 3.2
  void refine(int g) {
    const PTask x = tasks_[g];
    std::vector<int> v;
    if (x.fn == PT_HLU) {
      if (!structured(x.b[0])) return;
      const int* s = t_.bl[x.b[0]].son;
      v.push_back(add(PT_HLU, s[0], s[0], s[0]));
      v.push_back(add(PT_HTRSU, s[0], s[2], s[2]));
      v.push_back(add(PT_HTRSL, s[0], s[1], s[1]));
      v.push_back(add(PT_HMUL, s[2], s[1], s[3]));
      v.push_back(add(PT_HLU, s[3], s[3], s[3]));
    } else if (x.fn == PT_HTRSL) {
      if (!structured(x.b[0]) || !structured(x.b[1])) return;
      const int *l = t_.bl[x.b[0]].son, *m = t_.bl[x.b[1]].son;
      for (int j = 0; j < 2; ++j) v.push_back(add(PT_HTRSL, l[0], m[j], m[j]));
      for (int j = 0; j < 2; ++j) v.push_back(add(PT_HMUL, l[2], m[j], m[2 + j]));
      for (int j = 0; j < 2; ++j) v.push_back(add(PT_HTRSL, l[3], m[2 + j], m[2 + j]));
    } else if (x.fn == PT_HTRSU) {
      if (!structured(x.b[0]) || !structured(x.b[1])) return;
      const int *u = t_.bl[x.b[0]].son, *m = t_.bl[x.b[1]].son;
      for (int j = 0; j < 2; ++j) v.push_back(add(PT_HTRSU, u[0], m[2 * j], m[2 * j]));
      for (int j = 0; j < 2; ++j) v.push_back(add(PT_HMUL, m[2 * j], u[1], m[2 * j + 1]));
      for (int j = 0; j < 2; ++j) v.push_back(add(PT_HTRSU, u[3], m[2 * j + 1], m[2 * j + 1]));
    } else {
      if (!structured(x.b[0]) || !structured(x.b[1]) || !structured(x.b[2])) return;
      const int *a = t_.bl[x.b[0]].son, *b = t_.bl[x.b[1]].son, *c = t_.bl[x.b[2]].son;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int l = 0; l < 2; ++l) v.push_back(add(PT_HMUL, a[2 * i + l], b[2 * l + j], c[2 * i + j]));
    }
    for (size_t i = 0; i < v.size(); ++i)
      for (size_t j = i + 1; j < v.size(); ++j)
        if (precedes(v[i], v[j])) tasks_[v[i]].succ.push_back(v[j]);
    tasks_[g].sub = v;
  }

  // Algorithm 9: the dependencies of a refined task g pass to its sub-tasks,
  // towards the successors or their sub-tasks, where Definition 3.2 holds
  void refine_sub_deps(int g) {
    const std::vector<int> succ = tasks_[g].succ;
    const std::vector<int> sub = tasks_[g].sub;
    for (int s : succ) {
      std::vector<int> targets = tasks_[s].sub.empty() ? std::vector<int>{s} : tasks_[s].sub;
      for (int tp : sub)
        for (int x : targets)
          if (precedes(tp, x)) push_unique(tasks_[tp].succ, x);
    }
  }
  // Algorithm 10: an unrefined task keeps only the sub-tasks of a refined
  // successor that it precedes
  void refine_loc_deps(int g) {
    std::vector<int> out;
    for (int s : tasks_[g].succ) {
      if (tasks_[s].sub.empty()) {
        push_unique(out, s);
      } else {
        for (int x : tasks_[s].sub)
          if (precedes(g, x)) push_unique(out, x);
      }
    }
    tasks_[g].succ.swap(out);
  }
  static void push_unique(std::vector<int>& v, int x) {
    if (std::find(v.begin(), v.end(), x) == v.end()) v.push_back(x);
  }

  // Algorithm 12: within the neighbourhood of g (g or its sub-tasks, and its
  // successors or theirs), drop an edge (t', s) when s is also reached from
  // t' by a path of length >= 2 (at most max_path edges, 0 = unbounded)
  void remove_redundant_around(int g, int max_path) {
    std::vector<int> nb = tasks_[g].sub.empty() ? std::vector<int>{g} : tasks_[g].sub;
    for (int s : tasks_[g].succ) {
      if (tasks_[s].sub.empty())
        nb.push_back(s);
      else
        nb.insert(nb.end(), tasks_[s].sub.begin(), tasks_[s].sub.end());
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    auto inside = [&](int x) { return std::binary_search(nb.begin(), nb.end(), x); };
    const std::vector<int> starts = tasks_[g].sub.empty() ? std::vector<int>{g} : tasks_[g].sub;
    for (int tp : starts) {
      // nodes reached from a direct successor (paths of length >= 2 from tp)
      std::vector<int> seen, frontier;
      for (int u : tasks_[tp].succ)
        if (inside(u)) frontier.push_back(u);
      for (int depth = 2; !frontier.empty() && (max_path == 0 || depth <= max_path); ++depth) {
        std::vector<int> nxt;
        for (int u : frontier)
          for (int w : tasks_[u].succ)
            if (inside(w) && std::find(seen.begin(), seen.end(), w) == seen.end()) {
              seen.push_back(w);
              nxt.push_back(w);
            }
        frontier.swap(nxt);
      }
      std::vector<int>& st = tasks_[tp].succ;
      st.erase(std::remove_if(st.begin(), st.end(),
                              [&](int s) { return std::find(seen.begin(), seen.end(), s) != seen.end(); }),
               st.end());
    }
  }

  const Tree& t_;
  std::vector<PTask> tasks_;
  std::vector<int> final_;
};

}  // namespace

void build_semiauto_dag(const Tree& t, bool sparsify, int max_path, std::vector<int32_t>& tasks,
                        std::vector<int32_t>& edges) {
  Builder b(t);
  b.compute(sparsify, max_path);
  b.result(tasks, edges);
}

}  // namespace hm
