"""C-ABI library on the CPU: exported symbols, exact tree parity with the
oracle (Def. 2.1, Def. 2.2), and invariants of the traced DAG (Def. 3.2:
every edge runs forward in the sequential order, so the graph is acyclic).
No compute call is made (no device here)."""
import ctypes
import subprocess

import numpy as np
import pytest

from oracle import hmatrix as H
from paper_1911_07531_amd import hm, inputs


@pytest.fixture(scope="module")
def L():
    return hm.lib()


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", hm.LIB_PATH], capture_output=True, text=True).stdout
    names = {line.split()[-1] for line in out.splitlines() if line.strip()}
    header = open(hm.os.path.join(hm._HERE, "..", "include", "hm.h")).read()
    for name in hm.exported_symbols():
        assert name in names, name
        assert name + "(" in header, name
        getattr(L, name)


@pytest.mark.parametrize("n,leaf,eta,seed", [(2048, 32, 2.0, 0), (3000, 64, 2.0, 1), (777, 20, 1.0, 2)])
def test_tree_parity_with_oracle(n, leaf, eta, seed):
    pts = inputs.sphere_points(n, seed)
    t = hm.Tree(pts, hm.make_opts(leaf=leaf, eta=eta))
    perm, cl, box, bl = t.tables()
    operm, ocl = H.build_cluster_tree(pts, leaf)
    oroot = H.build_block_tree(ocl[0], eta)
    assert np.array_equal(perm, operm)
    assert len(cl) == len(ocl)
    for i, c in enumerate(ocl):
        sons = [s.index for s in c.sons] if c.sons else [-1, -1]
        assert list(cl[i]) == [c.begin, c.end, sons[0], sons[1], c.level]
        assert np.array_equal(box[i, :3], c.lo) and np.array_equal(box[i, 3:], c.hi)
    oblocks = H.block_list(oroot)
    assert len(bl) == len(oblocks)
    kind = {"S": 0, "D": 1, "R": 2}
    for b in oblocks:
        row = bl[b.index]
        assert row[0] == b.tau.index and row[1] == b.sigma.index and row[2] == kind[b.kind]
        if b.kind == "S":
            assert list(row[3:]) == [b.sons[i][j].index for i in range(2) for j in range(2)]


def test_invalid_arguments_rejected(L):
    pts = np.zeros((4, 3))
    h = ctypes.c_void_p()
    bad = hm.make_opts(leaf=0)
    assert L.build_htree(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4, 3, ctypes.byref(bad),
                         ctypes.byref(h)) == hm.HM_EINVAL
    bad = hm.make_opts(eta=0.0)
    assert L.build_htree(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4, 3, ctypes.byref(bad),
                         ctypes.byref(h)) == hm.HM_EINVAL
    assert L.build_htree(None, 4, 3, ctypes.byref(hm.make_opts()), ctypes.byref(h)) == hm.HM_EINVAL
    assert b"n >= 1" in L.hm_last_error() or b"null" in L.hm_last_error()
    with pytest.raises(hm.HmError):
        hm.Tree(pts, hm.make_opts(leaf=-3))
    for dim in (0, 4):
        assert L.build_htree(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3, dim,
                             ctypes.byref(hm.make_opts()), ctypes.byref(h)) == hm.HM_EINVAL


@pytest.mark.parametrize("n,leaf", [(4096, 32), (3000, 64), (1, 8)])
def test_line_tree_parity_with_oracle(n, leaf):
    """Points on [0, 1] given with dim = 1: the host tree equals the oracle's,
    boxes padded with zero trailing coordinates."""
    pts = inputs.line_points(n)
    t = hm.Tree(pts, hm.make_opts(leaf=leaf, eta=2.0))
    perm, cl, box, bl = t.tables()
    operm, ocl = H.build_cluster_tree(pts, leaf)
    oroot = H.build_block_tree(ocl[0], 2.0)
    assert np.array_equal(perm, operm)
    assert len(cl) == len(ocl)
    for i, c in enumerate(ocl):
        assert box[i, 0] == c.lo[0] and box[i, 3] == c.hi[0]
        assert not box[i, [1, 2, 4, 5]].any()
        assert list(cl[i][:2]) == [c.begin, c.end]
    kind = {"S": 0, "D": 1, "R": 2}
    oblocks = H.block_list(oroot)
    assert len(bl) == len(oblocks)
    for b in oblocks:
        assert list(bl[b.index][:3]) == [b.tau.index, b.sigma.index, kind[b.kind]]


@pytest.mark.parametrize("prec", [hm.FP64, hm.MIXED])
def test_dag_is_forward_and_levels_consistent(prec):
    pts = inputs.sphere_points(2048, 0)
    opts = hm.make_opts(leaf=32, eta=2.0, eps=1e-6, max_rank=0, prec=prec)
    t = hm.Tree(pts, opts)
    for which in (0, 1, 2):
        d = t.dag(opts, which)
        sp, si, lv = d["succ_ptr"], d["succ_idx"], d["level"]
        n = len(d["tasks"])
        assert n > 0 and sp[-1] == len(si)
        src = np.repeat(np.arange(n), np.diff(sp))
        assert np.all(si > src)                 # edges run forward in trace order
        assert np.all(lv[si] >= lv[src] + 1)    # levels are a valid schedule
        assert lv.max() + 1 == d["nlevels"]
        ops = d["tasks"]["op"]
        # the substitution DAG alone holds sums of split partial products (11); the
        # factorization's DAGs invert the factored diagonal leaves (13) instead
        # coarsened diagonal blocks (12) with the default coarsening
        assert set(np.unique(ops)) <= (set(range(1, 13)) if which == 1 else set(range(1, 11)) | {13})
        if which != 1:
            assert (ops == 13).sum() == (ops == 1).sum()  # one inversion per factored leaf
    # every diagonal leaf is factored exactly once, in order along the diagonal
    d = t.dag(opts, 0)
    getrf = d["tasks"][d["tasks"]["op"] == 1]
    rows = getrf["row0"]
    assert np.all(np.diff(rows) > 0)
    _, cl, _, bl = t.tables()
    ndiag = sum(1 for b in bl if b[2] == 1 and b[0] == b[1])
    assert len(getrf) == ndiag


def test_fused_and_inspection_arguments_rejected(L):
    """h_lu_solve, hm_dag_calls and hm_semiauto_dag reject bad arguments
    before touching a device."""
    h = ctypes.c_void_p()
    info = ctypes.c_int64(0)
    opts = hm.make_opts()
    assert L.h_lu_solve(None, ctypes.byref(opts), None, 1, 1, None, ctypes.byref(h), ctypes.byref(info)) == hm.HM_EINVAL
    t = hm.Tree(inputs.sphere_points(256, 0), hm.make_opts(leaf=32))
    assert L.hm_semiauto_dag(t.h, 1, -1, None, None, None, None) == hm.HM_EINVAL
    assert L.hm_dag_calls(t.h, ctypes.byref(opts), 3, None, None, None) == hm.HM_EINVAL
    assert L.hm_dag_sizes(t.h, ctypes.byref(opts), 3, np.zeros(10, np.int64).ctypes.data) == hm.HM_EINVAL


def test_eps_below_the_truncation_route_rejected(L):
    """eps < 1e-8 (including the exact case eps = 0) is refused before any
    device work: the truncation's CholeskyQR resolves directions only down to
    about sqrt(u) of the largest."""
    t = hm.Tree(inputs.sphere_points(256, 0), hm.make_opts(leaf=32))
    h = ctypes.c_void_p()
    for eps in (0.0, 1e-10, 9.9e-9, -1.0):
        opts = hm.make_opts(leaf=32, eps=eps)
        assert L.h_assemble(t.h, hm.LAPLACE3D, 1.0, ctypes.byref(opts), None, ctypes.byref(h)) == hm.HM_EINVAL
        assert L.h_lu(None, ctypes.byref(opts), None, ctypes.byref(h), None) == hm.HM_EINVAL


def test_coarsening_range_and_seq_export(L):
    """hm_opts.coarsen outside [0, 1024] is refused; with coarsening the
    substitution DAG holds OP_SEQ tasks whose micro-operations (exported by
    hm_dag_seq_export) are leaf solves and products, every block-local panel
    view inside its block, and the task count falls."""
    t = hm.Tree(inputs.sphere_points(1024, 0), hm.make_opts(leaf=32))
    h = ctypes.c_void_p()
    for c in (-1, 1025):
        opts = hm.make_opts(leaf=32, coarsen=c)
        assert L.h_assemble(t.h, hm.LAPLACE3D, 1.0, ctypes.byref(opts), None, ctypes.byref(h)) == hm.HM_EINVAL
        n = ctypes.c_int64()
        assert L.hm_dag_seq_export(t.h, ctypes.byref(opts), 1, ctypes.byref(n), None) == hm.HM_EINVAL
    d0 = t.dag(hm.make_opts(leaf=32, coarsen=0), 1)
    d1 = t.dag(hm.make_opts(leaf=32, coarsen=128), 1)
    assert len(d0["seq"]) == 0 and not (d0["tasks"]["op"] == 12).any()
    seqt = d1["tasks"][d1["tasks"]["op"] == 12]
    assert len(seqt) > 0 and len(d1["tasks"]) < len(d0["tasks"])
    assert set(np.unique(d1["seq"]["op"])) <= {2, 4, 5, 6}
    assert int(seqt["lr"].sum()) == len(d1["seq"])  # every micro-operation belongs to one block
    for tk in seqt:
        W = int(tk["y"]["rows"])
        assert W <= 128
        for u in d1["seq"][int(tk["piv"]):int(tk["piv"]) + int(tk["lr"])]:
            for key in ("y", "a", "b", "x"):
                v = u[key]
                if int(v["dyn"]) & 8:  # block-local: rows inside the block
                    assert 0 <= int(v["off"]) and int(v["off"]) + int(v["rows"]) <= W


def test_solve_variants_reject_bad_arguments(L):
    """h_solve, h_solve_async and h_solve_noalloc check their arguments before
    touching a device."""
    st = ctypes.c_int32(0)
    assert L.h_solve(None, None, None, 1, 1, 1e-10, 5, None, None, None) == hm.HM_EINVAL
    assert L.h_solve_async(None, None, 1, 1, None, ctypes.byref(st)) == hm.HM_EINVAL
    assert L.h_solve_noalloc(None, None, None, 1, 1, 1e-10, 5, None, None, None) == hm.HM_EINVAL


def test_tuning_get_set_and_range(L):
    """hm_set_tuning keeps the launch choices the autotuner picks and refuses
    values outside their ranges (no device needed)."""
    old = hm.get_tuning()
    try:
        hm.set_tuning(exec_wg_per_cu=1, solve_wg=64, batch_order=1)
        assert hm.get_tuning() == {"exec_wg_per_cu": 1, "solve_wg": 64, "batch_order": 1}
        for bad in (dict(exec_wg_per_cu=3), dict(solve_wg=0), dict(batch_order=2)):
            with pytest.raises(hm.HmError) as ei:
                hm.set_tuning(**bad)
            assert ei.value.code == hm.HM_EINVAL
        assert hm.get_tuning()["exec_wg_per_cu"] == 1
    finally:
        hm.set_tuning(**old)


def test_batched_arguments_rejected(L):
    """h_lu_batched and hm_batch_dag_export reject bad arguments before any device work."""
    h = (ctypes.c_void_p * 2)()
    opts = hm.make_opts()
    assert L.h_lu_batched(None, 2, ctypes.byref(opts), None, h, None) == hm.HM_EINVAL
    assert L.h_lu_batched(h, 0, ctypes.byref(opts), None, h, None) == hm.HM_EINVAL
    mats = (ctypes.c_void_p * 2)(None, None)
    assert L.h_lu_batched(mats, 2, ctypes.byref(opts), None, h, None) == hm.HM_EINVAL
    sz = np.zeros(7, np.int64)
    assert L.hm_batch_dag_export(mats, 2, ctypes.byref(opts), sz.ctypes.data, None, None, None, None, None, None,
                                 None) == hm.HM_EINVAL


def test_import_arguments_rejected(L):
    """hm_import checks the leaf data against the block structure before any
    device work: a wrong value count is HM_EINVAL, a rank above the capacity
    HM_ERANK."""
    opts = hm.make_opts(leaf=32, eps=1e-6, max_rank=8)
    t = hm.Tree(inputs.sphere_points(512, 0), opts)
    _, cl, _, bl = t.tables()
    ranks = np.zeros(len(bl), np.int32)
    need = sum(int((cl[b[0], 1] - cl[b[0], 0]) * (cl[b[1], 1] - cl[b[1], 0])) for b in bl if b[2] == 1)
    data = np.zeros(need + 5)
    h = ctypes.c_void_p()
    assert L.hm_import(t.h, ctypes.byref(opts), ranks.ctypes.data, data.ctypes.data, need + 5, None,
                       ctypes.byref(h)) == hm.HM_EINVAL
    lr = int(np.nonzero(bl[:, 2] == 2)[0][0])
    ranks[lr] = 9
    assert L.hm_import(t.h, ctypes.byref(opts), ranks.ctypes.data, data.ctypes.data, need + 5, None,
                       ctypes.byref(h)) == hm.HM_ERANK
    assert L.hm_import(None, ctypes.byref(opts), ranks.ctypes.data, data.ctypes.data, 0, None,
                       ctypes.byref(h)) == hm.HM_EINVAL
