"""The combined DAG of h_lu_batched on the CPU: every instance's traced H-LU
DAG relocated into one arena and one task list.

* every view, pivot offset, rank slot and low-rank index of the combined
  task list stays inside the batch arenas (the device runs these records);
* successor lists point inside each instance's own task range, so the union
  is the disjoint union of the instances' DAGs;
* replayed in NumPy in a random topological order of the union, every
  instance's factors are those of its own DAG replayed alone, bit for bit.
"""
import numpy as np

from oracle import hmatrix as H
from paper_1911_07531_amd import hm, inputs
from tests.dag_replay import Replay

VT_F64, VT_F32 = 0, 1
DYN_COLS2 = 4

CASES = [("sphere", 700, 32), ("cube", 600, 16), ("grid", 576, 64), ("sphere", 300, 128)]


def _instances(prec):
    out = []
    for geo, n, leaf in CASES:
        pts, diag = inputs.problem(geo, n, 3)
        kname = inputs.GEOMETRY_KERNEL[geo]
        opts = hm.make_opts(leaf=leaf, eta=2.0, eps=1e-4, max_rank=32, prec=prec)
        t = hm.Tree(pts, opts)
        perm, cl = H.build_cluster_tree(pts, leaf)
        root = H.build_block_tree(cl[0], 2.0)
        a = H.assemble(pts, perm, cl, root, diag, 1e-4, 32, kernel=kname)
        out.append((t, a))
    return out, hm.make_opts(leaf=32, eta=2.0, eps=1e-4, max_rank=32, prec=prec)


def _shifted(dag, base):
    """An instance's block table and low-rank table moved to its batch bases."""
    bo = dag["block_off"].copy()
    for r in bo:
        if r[0] >= 0:
            r[0] += base[0] if r[1] == VT_F64 else base[1]
        if r[2] >= 0:
            r[2] += base[3]
        if r[3] >= 0:
            r[3] += base[2]
    return bo


def test_batch_dag_bounds_and_disjoint_union():
    for prec in (hm.FP64, hm.MIXED):
        inst, opts = _instances(prec)
        bd = hm.batch_dag([t for t, _ in inst], opts)
        tasks, nt = bd["tasks"], len(bd["tasks"])
        size = {VT_F64: bd["n_f64"], VT_F32: bd["n_f32"]}
        for v in ("y", "a", "b", "x"):
            V = tasks[v]
            for typ in (VT_F64, VT_F32):
                sel = V["type"] == typ
                last = V["off"][sel] + (np.maximum(V["rows"][sel], 1) - 1) * V["rs"][sel] + \
                    (np.maximum(V["cols"][sel], 1) - 1) * V["cs"][sel]
                assert np.all(V["off"][sel] >= 0) and np.all(last < size[typ]), (v, typ)
            dyn = V["dyn"] != 0
            assert np.all(V["rank_id"][dyn] < bd["nranks"]) and np.all(V["rank_id"][dyn] >= 0)
            d2 = (V["dyn"] & DYN_COLS2) != 0
            assert np.all(V["rank_id2"][d2] < bd["nranks"])
        piv_ops = np.isin(tasks["op"], [1, 2, 3, 4])
        m = tasks["a"]["rows"][piv_ops]
        assert np.all(tasks["piv"][piv_ops] + 2 * m <= bd["n_piv"])
        tr = np.isin(tasks["op"], [7, 10])
        assert np.all((tasks["lr"][tr] >= 0) & (tasks["lr"][tr] < bd["nranks"]))
        # each instance's successors stay in its own task range
        for b in bd["bases"]:
            t0, cnt = int(b[5]), int(b[7])
            sp, si = bd["succ_ptr"], bd["succ_idx"]
            succ = si[sp[t0]:sp[t0 + cnt]]
            assert np.all((succ >= t0) & (succ < t0 + cnt))
        assert bd["succ_ptr"][-1] == bd["nedges"] and np.all(np.diff(bd["succ_ptr"]) >= 0)
        assert np.array_equal(np.sort(bd["order"]), np.arange(nt))


def test_batch_replay_equals_single_replays():
    inst, opts = _instances(hm.MIXED)
    trees = [t for t, _ in inst]
    bd = hm.batch_dag(trees, opts)
    rp = Replay(bd, 1e-4, 32)
    singles = []
    for (t, a), base in zip(inst, bd["bases"]):
        d = t.dag(opts, 0)
        blocks = {b.index: b for b in H.leaf_blocks(a.root)}
        rp.load_matrix(blocks, _shifted(d, base), bd["lr"])
        r1 = Replay(d, 1e-4, 32)
        r1.load_matrix(blocks, d["block_off"], d["lr"])
        r1.run(np.random.default_rng(5))
        singles.append((t, a, d, base, r1))
    rp.run(np.random.default_rng(6))
    for t, a, d, base, r1 in singles:
        sh = _shifted(d, base)
        for b in H.leaf_blocks(a.root):
            kind = 1 if b.kind == "D" else 2
            x = r1.leaf(b.index, kind, b.rows, b.cols, d["block_off"], d["lr"])
            y = rp.leaf(b.index, kind, b.rows, b.cols, sh, bd["lr"])
            assert x[0] == y[0]
            assert np.array_equal(x[1], y[1]), b.index
            if x[2] is not None:
                assert np.array_equal(x[2], y[2])
