"""The paper's semi-automatic task graph construction (Sec. 3, Algorithms
9-11, with the edge sparsification of Sec. 4.1, Algorithm 12) against the
leaf-level tracer that produces the executed H-LU DAG (CPU only).

* both reach the same leaf tasks: every hlu / htrsl / htrsu / hmul call on
  blocks that the paper's refinement stops at is a call of the tracer, and
  no other;
* every dependency of the paper's graph (Definition 3.2), with or without
  sparsification, is enforced by the executed DAG (a path between the calls'
  tasks);
* sparsification removes only redundant edges: the transitive closure is
  unchanged;
* the executed DAG orders, beyond the paper's graph, only pairs of updates
  (hmul -> hmul) whose targets overlap: Definition 3.2 relates outputs to
  inputs only, and the paper serializes concurrent updates of one block at
  run time (Reading C-13).
"""
import collections

import numpy as np
import pytest

from paper_1911_07531_amd import hm, inputs


def _closure(nn, edges):
    succ = [[] for _ in range(nn)]
    indeg = np.zeros(nn, np.int64)
    for a, b in edges:
        succ[a].append(b)
        indeg[b] += 1
    order, q = [], collections.deque(np.nonzero(indeg == 0)[0].tolist())
    while q:
        x = q.popleft()
        order.append(x)
        for y in succ[x]:
            indeg[y] -= 1
            if indeg[y] == 0:
                q.append(y)
    assert len(order) == nn, "the graph has a cycle"
    reach = np.zeros((nn, (nn + 7) // 8), np.uint8)
    for x in reversed(order):
        for y in succ[x]:
            reach[x] |= reach[y]
            reach[x, y >> 3] |= np.uint8(1 << (y & 7))
    return reach


def _has(reach, a, b):
    return bool((reach[a, b >> 3] >> (b & 7)) & 1)


@pytest.mark.parametrize("geometry,n", [("sphere", 2048), ("line", 4096)])
def test_semiauto_dag_matches_traced_dag(geometry, n):
    pts = inputs.sphere_points(n, 0) if geometry == "sphere" else inputs.line_points(n)
    opts = hm.make_opts(leaf=32, eta=2.0, eps=1e-6, lazy=0)
    t = hm.Tree(pts, opts)
    tasks, edges = t.semiauto_dag(sparsify=False)
    stasks, sedges = t.semiauto_dag(sparsify=True)
    assert np.array_equal(tasks, stasks)
    assert 0 < len(sedges) < len(edges)
    calls, task_call = t.calls(opts, 0)
    assert (task_call >= 0).all()
    keys = {k: i for i, k in enumerate(map(tuple, calls.tolist()))}
    assert len(keys) == len(calls)
    assert set(keys) == set(map(tuple, tasks.tolist()))
    to_call = np.array([keys[k] for k in map(tuple, tasks.tolist())])
    # the executed DAG at the level of the calls
    d = t.dag(opts, 0)
    src = np.repeat(np.arange(len(task_call)), np.diff(d["succ_ptr"]))
    cu, cv = task_call[src], task_call[d["succ_idx"]]
    sel = cu != cv
    cedges = np.unique(np.stack([cu[sel], cv[sel]], 1), axis=0)
    reach_traced = _closure(len(calls), cedges.tolist())
    for e in (edges, sedges):
        mapped = np.stack([to_call[e[:, 0]], to_call[e[:, 1]]], 1)
        assert all(_has(reach_traced, a, b) for a, b in mapped)
    full = _closure(len(calls), np.stack([to_call[edges[:, 0]], to_call[edges[:, 1]]], 1).tolist())
    sparse = _closure(len(calls), np.stack([to_call[sedges[:, 0]], to_call[sedges[:, 1]]], 1).tolist())
    assert np.array_equal(full, sparse)
    # orderings of the executed DAG beyond the paper's graph: overlapping updates
    _, cl, _, bl = t.tables()

    def rect(b):
        r, c = cl[bl[b, 0]], cl[bl[b, 1]]
        return r[0], r[1], c[0], c[1]

    extra = [(a, b) for a, b in cedges if not _has(full, a, b)]
    for a, b in extra:
        assert calls[a][0] == 3 and calls[b][0] == 3, (calls[a], calls[b])
        ra, rb = rect(calls[a][3]), rect(calls[b][3])
        assert ra[0] < rb[1] and rb[0] < ra[1] and ra[2] < rb[3] and rb[2] < ra[3]
