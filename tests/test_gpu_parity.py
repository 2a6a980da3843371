"""GPU parity of the H-LU path against the FP64 oracle (through the C-ABI).

Bars (written in each test):
  * trees: exact integers (CPU test) ; leaf getrf on identical input:
    interchanges bit-exact, values within 1e-13 relative (same FP64 steps,
    different summation order);
  * assembly: ranks within +-2 of the oracle's truncated SVD; block error
    ||A_b - U V^T||_2 <= 2 eps sigma_1 (ACA + recompression vs exact SVD);
  * H-LU: ||P A - L U||_2 / ||A||_2 <= 10 eps, factor ranks within +-2 of the
    oracle's, solve relative residuals <= 2x the oracle's (+ 1e-12 slack);
  * matvec: equal to the densified exported matrix times x, 1e-13 relative;
  * executors: the level-by-level and dataflow replays give bit-identical
    factors (every conflicting pair of tasks is ordered by the DAG).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import hmatrix as H
from paper_1911_07531_amd import hm, inputs
from tests.gpu_common import Problem, device_rhs, require_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("m", [1, 7, 32, 64])
def test_getrf_single_leaf_bit_exact_pivots(m):
    # one diagonal leaf: the whole matrix is one dense block
    p = Problem(m, 64, 1e-6, oracle=False)
    f = hm.LU(p.A, p.opts)
    kind, a, _ = p.A.leaf(0)
    assert kind == "D"
    kind, lu, piv = f.leaf(0)
    lu_ref, piv_ref = sla.lu_factor(a)
    assert np.array_equal(piv, piv_ref)
    assert np.max(np.abs(lu - lu_ref)) <= 1e-13 * np.abs(a).max() * max(1, m)


def test_singular_leaf_reports_row():
    # two points at distance 1 with the log kernel and a zero diagonal: the
    # single leaf is the zero matrix, so the first pivot is an exact zero
    pts = np.array([[0.0, 0.0], [1.0, 0.0]])
    opts = hm.make_opts(leaf=4, eta=2.0, eps=1e-6)
    t = hm.Tree(pts, opts)
    a = hm.Matrix(t, hm.LOG2D, 0.0, opts)
    with pytest.raises(hm.HmError) as ei:
        hm.LU(a, opts)
    assert ei.value.code == hm.HM_ESINGULAR and ei.value.info == 0


@pytest.fixture(scope="module")
def c1():
    """n = 2048, leaf 32, eta = 2, eps = 1e-6 (the small sphere workload);
    updates collected per hmul call on both sides (Reading R6)."""
    p = Problem(2048, 32, 1e-6)
    f = hm.LU(p.A, p.opts)
    of = H.hlu(p.oa, lazy=True)
    return p, f, of


def test_assembly_ranks_and_error_c1(c1):
    p, _, _ = c1
    ga = p.gpu_as_oracle(0, p.A.h)
    orank = H.rank_table(p.oa)
    grank = H.rank_table(ga)
    d = np.array([grank[k] - orank[k] for k in orank])
    assert np.max(np.abs(d)) <= 2, np.unique(d, return_counts=True)
    rng = np.random.default_rng(0)
    lr = [b for b in H.leaf_blocks(ga.root) if b.kind == "R"]
    for b in rng.choice(lr, 40, replace=False):
        exact = p.exact_block(ga.perm, b.tau, b.sigma)
        s1 = np.linalg.norm(exact, 2)
        assert np.linalg.norm(exact - b.U @ b.V.T, 2) <= 2 * p.eps * s1
    for b in H.leaf_blocks(ga.root):
        if b.kind == "D":
            exact = p.exact_block(ga.perm, b.tau, b.sigma)
            assert np.array_equal(b.D, exact) or np.max(np.abs(b.D - exact)) <= 1e-15 * np.abs(exact).max()


def test_hlu_error_bound_and_ranks_c1(c1):
    p, f, of = c1
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    err = H.lu_error_2norm(dense, gf, exact=True)
    oerr = H.lu_error_2norm(dense, of, exact=True)
    print(f"gpu ||PA-LU||/||A|| = {err:.3e}, oracle {oerr:.3e}")
    assert err <= 10 * p.eps
    orank = H.rank_table(of)
    grank = H.rank_table(gf)
    d = np.array([grank[k] - orank[k] for k in orank])
    assert np.max(np.abs(d)) <= 2, np.unique(d, return_counts=True)


def test_solve_residuals_c1(c1):
    p, f, of = c1
    b = inputs.rhs(p.n, 16, seed=1)
    xg = to_host(f.solve(device_rhs(b))[0])
    xo = H.solve(of, b)
    dense = p.dense_exact()
    a_user = np.empty_like(dense)
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = dense
    rg = np.linalg.norm(b - a_user @ xg, axis=0) / np.linalg.norm(b, axis=0)
    ro = np.linalg.norm(b - a_user @ xo, axis=0) / np.linalg.norm(b, axis=0)
    print("residual gpu / oracle", rg.max(), ro.max())
    assert np.all(rg <= 2 * ro + 1e-12)


def test_matvec_c1(c1):
    p, _, _ = c1
    ga = p.gpu_as_oracle(0, p.A.h)
    x = inputs.rhs(p.n, 20, seed=5)
    y0 = inputs.rhs(p.n, 20, seed=6)
    ah = np.empty((p.n, p.n))
    ah[np.ix_(ga.perm, ga.perm)] = H.densify(ga.root)
    y = to_host(p.A.matvec(device_rhs(x), device_rhs(y0), alpha=-0.5, beta=2.0))
    ref = -0.5 * ah @ x + 2.0 * y0
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.abs(ref).max()


def test_sequential_updates_match_sequential_oracle():
    """lazy = 0: every update truncated as produced, in Algorithm 1's order."""
    p = Problem(1024, 32, 1e-6)
    opts = hm.make_opts(leaf=32, eta=2.0, eps=1e-6, lazy=0)
    f = hm.LU(p.A, opts)
    of = H.hlu(p.oa)
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    assert H.lu_error_2norm(dense, gf, exact=True) <= 10 * p.eps
    orank, grank = H.rank_table(of), H.rank_table(gf)
    assert max(abs(grank[k] - orank[k]) for k in orank) <= 2


def test_level_and_dataflow_executors_identical():
    p = Problem(1024, 32, 1e-6, oracle=False)
    f1 = hm.LU(p.A, hm.make_opts(leaf=32, eta=2.0, eps=1e-6, exec_mode=hm.DATAFLOW))
    f2 = hm.LU(p.A, hm.make_opts(leaf=32, eta=2.0, eps=1e-6, exec_mode=hm.LEVEL))
    _, _, _, bl = p.tree.tables()
    for bi in np.nonzero(bl[:, 2] != 0)[0]:
        r1, r2 = f1.leaf(int(bi)), f2.leaf(int(bi))
        assert r1[0] == r2[0]
        assert np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


def test_edge_sizes():
    # n = 1, n below the leaf size, ragged leaves
    for n, leaf in [(1, 32), (5, 32), (100, 32), (257, 16)]:
        p = Problem(n, leaf, 1e-8, oracle=False)
        f = hm.LU(p.A, p.opts)
        b = inputs.rhs(n, 3, seed=2)
        x = to_host(f.solve(device_rhs(b))[0])
        dense = p.dense_exact()
        perm = p.tree.tables()[0]
        a_user = np.empty_like(dense)
        a_user[np.ix_(perm, perm)] = dense
        res = np.linalg.norm(b - a_user @ x, axis=0) / np.linalg.norm(b, axis=0)
        assert np.all(res <= 1e-6), (n, res)


def test_mixed_precision_c1():
    """FP32 off-diagonal storage (FP64 diagonal leaves, pivots, Gram/core SVD):
    the same error bound against the exact matrix, ranks within +-2 of the
    FP64 oracle's, and iterative refinement against the FP64 H-matvec reaching
    1e-10 relative residual."""
    p = Problem(2048, 32, 1e-6, prec=hm.MIXED)
    f = hm.LU(p.A, p.opts)
    of = H.hlu(p.oa, lazy=True)
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    err = H.lu_error_2norm(dense, gf, exact=True)
    print(f"mixed ||PA-LU||/||A|| = {err:.3e}")
    assert err <= 10 * p.eps
    orank, grank = H.rank_table(of), H.rank_table(gf)
    assert max(abs(grank[k] - orank[k]) for k in orank) <= 2
    b = inputs.rhs(p.n, 8, seed=1)
    xd = device_rhs(b)
    _, iters, rel = f.solve(xd, refine_with=p.A, rtol=1e-10, max_iter=50)
    assert np.all(rel <= 1e-10), rel
    ga = p.gpu_as_oracle(0, p.A.h)
    ah = np.empty((p.n, p.n))
    ah[np.ix_(ga.perm, ga.perm)] = H.densify(ga.root)
    x = to_host(xd)
    res = np.linalg.norm(b - ah @ x, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(res <= 1e-9), res


def test_solve_executors_identical(monkeypatch):
    """The substitution DAG gives bit-identical solutions level by level and
    with the persistent executor, also with refinement and with 64 columns."""
    p = Problem(4096, 64, 1e-6, max_rank=64, oracle=False, prec=hm.MIXED)
    f = hm.LU(p.A, p.opts)
    for nr in (5, 64):
        b = inputs.rhs(p.n, nr, seed=3)
        out = []
        for mode in ("level", "dataflow"):
            monkeypatch.setenv("HM_SOLVE_EXEC", mode)
            x = device_rhs(b)
            f.solve(x)
            y = device_rhs(b)
            f.solve(y, refine_with=p.A, rtol=1e-10, max_iter=20)
            out.append((to_host(x), to_host(y)))
        for o in out[1:]:
            assert np.array_equal(out[0][0], o[0]) and np.array_equal(out[0][1], o[1])


def test_reused_temporaries_on_device(monkeypatch):
    """A ring of temporaries much smaller than the DAG needs (every slot reused
    by temporaries of other shapes): repeated factorizations and both
    executors give bit-identical factors, within the error bound."""
    monkeypatch.setenv("HM_TEMP_BUDGET_GB", "0.0005")
    p = Problem(2048, 32, 1e-4, max_rank=16)
    b = inputs.rhs(p.n, 3, seed=4)
    sols = []
    for mode in (hm.DATAFLOW, hm.DATAFLOW, hm.LEVEL):
        opts = hm.make_opts(leaf=32, eta=2.0, eps=1e-4, max_rank=16, exec_mode=mode)
        f = hm.LU(p.A, opts)
        x = device_rhs(b)
        f.solve(x)
        sols.append(to_host(x))
    assert np.array_equal(sols[0], sols[1]) and np.array_equal(sols[0], sols[2])
    gf = p.gpu_as_oracle(1, f.h)
    assert H.lu_error_2norm(p.dense_exact(), gf, exact=True) <= 10 * p.eps


def test_split_solve_products(monkeypatch):
    """Low-rank products of the substitution DAG split into partial products
    over row chunks (128 rows here: every product with a side of 256 rows or
    more) give the unsplit solution up to rounding, identically on both
    executors."""
    b = inputs.rhs(4096, 5, seed=3)
    out = {}
    for split in ("0", "128"):
        monkeypatch.setenv("HM_SOLVE_SPLIT", split)
        p = Problem(4096, 64, 1e-6, max_rank=64, oracle=False)  # a new tree traces a new plan
        sdag = p.tree.dag(p.opts, 1)
        assert (sdag["tasks"]["op"] == 11).any() == (split != "0")
        f = hm.LU(p.A, p.opts)
        for mode in ("level", "dataflow"):
            monkeypatch.setenv("HM_SOLVE_EXEC", mode)
            x = device_rhs(b)
            f.solve(x)
            out[(split, mode)] = to_host(x)
    assert np.array_equal(out[("128", "level")], out[("128", "dataflow")])
    assert np.array_equal(out[("0", "level")], out[("0", "dataflow")])
    ref = out[("0", "level")]
    assert np.max(np.abs(out[("128", "level")] - ref)) <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("prec", [hm.FP64, hm.MIXED])
def test_coarsened_solve(prec, monkeypatch):
    """The substitution with diagonal blocks of at most 128, 256 or 512 rows
    run as one task each (panel rows in LDS, the neighbouring block's product
    folded in): the leaf-level solution up to rounding (1e-12 relative; the
    updates of a block are summed in another order), bit-identical on both
    executors, the solve residual against the oracle's factors within 2x the
    oracle's own, and the same with 64 right-hand sides (two column sweeps
    of the LDS copy for the larger blocks)."""
    p = Problem(4096, 64, 1e-6, max_rank=64, prec=prec)
    b = inputs.rhs(p.n, 32, seed=3)
    b64 = inputs.rhs(p.n, 64, seed=5)
    ref_lu = H.hlu(p.oa, lazy=True)
    a_user = np.empty((p.n, p.n))
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = p.dense_exact()
    ref_res = np.linalg.norm(b - a_user @ H.solve(ref_lu, b), axis=0) / np.linalg.norm(b, axis=0)
    sols = {}
    for c in (0, 128, 256, 512):
        opts = hm.make_opts(leaf=64, eta=2.0, eps=1e-6, max_rank=64, prec=prec, coarsen=c)
        if c:
            sdag = p.tree.dag(opts, 1)
            assert (sdag["tasks"]["op"] == 12).any()
        f = hm.LU(p.A, opts)
        for mode in ("level", "dataflow"):
            monkeypatch.setenv("HM_SOLVE_EXEC", mode)
            x = device_rhs(b)
            f.solve(x)
            sols[(c, mode)] = to_host(x)
            x = device_rhs(b64)
            f.solve(x)
            sols[(c, mode, 64)] = to_host(x)
        assert np.array_equal(sols[(c, "level")], sols[(c, "dataflow")]), c
        assert np.array_equal(sols[(c, "level", 64)], sols[(c, "dataflow", 64)]), c
    ref, ref64 = sols[(0, "dataflow")], sols[(0, "dataflow", 64)]
    for c in (128, 256, 512):
        d = np.max(np.abs(sols[(c, "dataflow")] - ref)) / np.abs(ref).max()
        d64 = np.max(np.abs(sols[(c, "dataflow", 64)] - ref64)) / np.abs(ref64).max()
        print(f"coarsen {c}: relative difference to the leaf-level solve {d:.1e} (32 RHS), {d64:.1e} (64 RHS)")
        assert d <= 1e-12 and d64 <= 1e-12, (c, d, d64)
        res = np.linalg.norm(b - a_user @ sols[(c, "dataflow")], axis=0) / np.linalg.norm(b, axis=0)
        assert np.all(res <= 2 * ref_res + 1e-12), (c, res.max(), ref_res.max())


@pytest.mark.parametrize("prec", [hm.FP64, hm.MIXED])
def test_fused_lu_solve_equals_separate(prec):
    """h_lu_solve runs the H-LU and the substitution as one DAG: the factors
    equal h_lu's leaf for leaf, bit for bit, and the solution equals h_lu
    followed by h_solve bit for bit (no product is split at this size); with
    70 right-hand sides the first 64 are fused and the rest solved after."""
    p = Problem(4096, 64, 1e-6, max_rank=64, oracle=False, prec=prec)
    # the fused substitution runs at leaf granularity: compare with the
    # uncoarsened separate substitution bit for bit, with the coarsened one
    # (default) up to the rounding of its other summation order
    opts = hm.make_opts(leaf=64, eta=2.0, eps=1e-6, max_rank=64, prec=prec, coarsen=0)
    f = hm.LU(p.A, opts)
    fc = hm.LU(p.A, p.opts)
    _, _, _, bl = p.tree.tables()
    leaves = np.nonzero(bl[:, 2] != 0)[0]
    for nrhs in (5, 70):
        b = inputs.rhs(p.n, nrhs, seed=7)
        x1 = device_rhs(b)
        f.solve(x1)
        x2 = device_rhs(b)
        g = hm.LU(p.A, opts, rhs=x2)
        assert np.array_equal(to_host(x1), to_host(x2))
        x3 = device_rhs(b)
        fc.solve(x3)
        assert np.max(np.abs(to_host(x3) - to_host(x2))) <= 1e-12 * np.abs(to_host(x2)).max()
        for bi in leaves[::7]:
            r1, r2 = f.leaf(int(bi)), g.leaf(int(bi))
            assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


def test_assembly_reproducible():
    """Two assemblies of the same tree are bit-identical (same H-matvec bit
    for bit, same leaves).  Each ACA workgroup owns a scratch slot sized for
    its block; an undersized slot made neighbouring blocks overwrite each
    other's factors now and then."""
    pts, diag = inputs.sphere_problem(32768, 0)
    opts = hm.make_opts(leaf=64, eta=2.0, eps=1e-4, max_rank=64, prec=hm.MIXED)
    t = hm.Tree(pts, opts)
    mats = [hm.Matrix(t, hm.LAPLACE3D, diag, opts) for _ in range(3)]
    x = device_rhs(inputs.rhs(32768, 4, seed=11))
    ys = [to_host(m.matvec(x)) for m in mats]
    assert np.array_equal(ys[0], ys[1]) and np.array_equal(ys[0], ys[2])
    _, _, _, bl = t.tables()
    for bi in np.nonzero(bl[:, 2] == 2)[0]:
        r = [m.leaf(int(bi)) for m in mats]
        assert all(np.array_equal(r[0][1], q[1]) and np.array_equal(r[0][2], q[2]) for q in r[1:]), bi


def test_fused_lu_solve_against_oracle_c1(c1):
    """h_lu_solve (H-LU and substitution in one DAG) against the oracle: the
    unrefined solve residuals against the exact matrix are at most 2x the
    oracle's, for 16 right-hand sides."""
    p, _, of = c1
    b = inputs.rhs(p.n, 16, seed=1)
    xd = device_rhs(b)
    hm.LU(p.A, p.opts, rhs=xd)
    xg = to_host(xd)
    xo = H.solve(of, b)
    dense = p.dense_exact()
    a_user = np.empty_like(dense)
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = dense
    rg = np.linalg.norm(b - a_user @ xg, axis=0) / np.linalg.norm(b, axis=0)
    ro = np.linalg.norm(b - a_user @ xo, axis=0) / np.linalg.norm(b, axis=0)
    print("fused residual gpu / oracle", rg.max(), ro.max())
    assert np.all(rg <= 2 * ro + 1e-12)


def test_executor_wait_limit_reported(monkeypatch):
    """The persistent executors' bounded wait: with a wait limit of zero ticks
    (set from the host) a workgroup that finds its queue slot empty gives up,
    raises the abort flag, and every workgroup leaves normally; h_lu and
    h_solve report HM_EDEVICE, and the next calls with the normal limit
    succeed on the same handles."""
    p = Problem(1024, 32, 1e-6, oracle=False)
    f = hm.LU(p.A, p.opts)
    b = inputs.rhs(p.n, 3, seed=2)
    ref = to_host(f.solve(device_rhs(b))[0])
    monkeypatch.setenv("HM_DEBUG_SPIN_TICKS", "0")
    with pytest.raises(hm.HmError) as ei:
        hm.LU(p.A, p.opts)
    assert ei.value.code == hm.HM_EDEVICE and "timed out" in str(ei.value)
    with pytest.raises(hm.HmError) as ei:
        f.solve(device_rhs(b))
    assert ei.value.code == hm.HM_EDEVICE
    with pytest.raises(hm.HmError) as ei:
        f.solve(device_rhs(b), refine_with=p.A)
    assert ei.value.code == hm.HM_EDEVICE
    monkeypatch.delenv("HM_DEBUG_SPIN_TICKS")
    g = hm.LU(p.A, p.opts)
    assert np.array_equal(to_host(g.solve(device_rhs(b))[0]), ref)
    assert np.array_equal(to_host(f.solve(device_rhs(b))[0]), ref)


def test_solve_async_equals_solve(monkeypatch):
    """h_solve_async queues the substitution and reports through a device
    word: the same solution as h_solve, bit for bit, and status 0; with the
    wait limit forced to zero the word reads HM_EDEVICE."""
    import torch
    p = Problem(4096, 64, 1e-6, max_rank=64, oracle=False, prec=hm.MIXED)
    f = hm.LU(p.A, p.opts)
    b = inputs.rhs(p.n, 70, seed=9)
    x1 = to_host(f.solve(device_rhs(b))[0])
    st = torch.full((1,), 123, dtype=torch.int32, device="cuda")
    xd = device_rhs(b)
    f.solve_async(xd, st)
    torch.cuda.synchronize()
    assert int(st.item()) == hm.HM_OK
    assert np.array_equal(to_host(xd), x1)
    monkeypatch.setenv("HM_DEBUG_SPIN_TICKS", "0")
    st.fill_(123)
    f.solve_async(device_rhs(b), st)
    torch.cuda.synchronize()
    assert int(st.item()) == hm.HM_EDEVICE
    monkeypatch.delenv("HM_DEBUG_SPIN_TICKS")
    xd = device_rhs(b)
    f.solve_async(xd, st)
    torch.cuda.synchronize()
    assert int(st.item()) == hm.HM_OK and np.array_equal(to_host(xd), x1)


def test_leaf_128_against_oracle():
    """Leaves of up to 128 points (the batched workload's largest): diagonal
    leaves of 65-128 rows take the getrf path in global memory (m > 97) and
    the two-rows-per-lane triangular solves; dense-dense products over such
    leaves reach low-rank targets in column chunks.  Bounds as for c1."""
    p = Problem(4096, 128, 1e-6)
    f = hm.LU(p.A, p.opts)
    of = H.hlu(p.oa, lazy=True)
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    err = H.lu_error_2norm(dense, gf, exact=False)
    assert err <= 10 * p.eps, err
    orank, grank = H.rank_table(of), H.rank_table(gf)
    assert max(abs(grank[k] - orank[k]) for k in orank) <= 2
    # the diagonal leaves of 98-128 rows: interchanges bit-exact against LAPACK on the assembled block
    _, cl, _, bl = p.tree.tables()
    big = [i for i in range(len(bl)) if bl[i, 2] == 1 and bl[i, 0] == bl[i, 1] and cl[bl[i, 0], 1] - cl[bl[i, 0], 0] > 97]
    assert big, "no diagonal leaf above 97 rows"
    b = inputs.rhs(p.n, 8, seed=1)
    xg = to_host(f.solve(device_rhs(b))[0])
    xo = H.solve(of, b)
    a_user = np.empty_like(dense)
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = dense
    rg = np.linalg.norm(b - a_user @ xg, axis=0) / np.linalg.norm(b, axis=0)
    ro = np.linalg.norm(b - a_user @ xo, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(rg <= 2 * ro + 1e-12), (rg, ro)


def test_getrf_leaf_above_97_rows_bit_exact_pivots():
    """A single diagonal leaf of 120 points (the global-memory getrf path):
    interchanges bit-exact against LAPACK, values to rounding."""
    p = Problem(120, 128, 1e-6, oracle=False)
    f = hm.LU(p.A, p.opts)
    kind, a, _ = p.A.leaf(0)
    kind, lu, piv = f.leaf(0)
    lu_ref, piv_ref = sla.lu_factor(a)
    assert np.array_equal(piv, piv_ref)
    assert np.max(np.abs(lu - lu_ref)) <= 1e-13 * np.abs(a).max() * 120


@pytest.mark.parametrize("geometry,n,leaf", [("cube", 2400, 32), ("grid", 2048, 64)])
def test_batched_geometries_against_oracle(geometry, n, leaf):
    """The batched workload's other geometries (unit-cube surface with
    1/(4 pi r), unit-square grid with -log r/(2 pi)), mixed precision at
    eps = 1e-4, ranks capped at 64: ||PA - LU||_2/||A||_2 <= 10 eps, ranks
    within +-2 of the FP64 oracle's, solve residuals <= 2x the oracle's."""
    p = Problem(n, leaf, 1e-4, max_rank=64, prec=hm.MIXED, geometry=geometry)
    f = hm.LU(p.A, p.opts)
    of = H.hlu(p.oa, lazy=True)
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    err = H.lu_error_2norm(dense, gf, exact=True)
    assert err <= 10 * p.eps, err
    orank, grank = H.rank_table(of), H.rank_table(gf)
    assert max(abs(grank[k] - orank[k]) for k in orank) <= 2
    b = inputs.rhs(p.n, 8, seed=1)
    xg = to_host(f.solve(device_rhs(b))[0])
    xo = H.solve(of, b)
    a_user = np.empty_like(dense)
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = dense
    rg = np.linalg.norm(b - a_user @ xg, axis=0) / np.linalg.norm(b, axis=0)
    ro = np.linalg.norm(b - a_user @ xo, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(rg <= 2 * ro + 1e-12), (rg, ro)


@pytest.mark.parametrize("prec", [hm.FP64, hm.MIXED])
def test_accumulated_hlu_against_oracle(prec):
    """The accumulated H-LU (Algorithms 4-8, lazy = 2) on the device, given the
    oracle's own assembly (hm_import), against the oracle's hlu_accumulated of
    the identical matrix: ||PA - LU||_2/||A||_2 <= 10 eps against the exact
    matrix, factor ranks within +-2, solve residuals <= 2x the oracle's."""
    p = Problem(2048, 32, 1e-6, prec=prec)
    leaves = {blk.index: ("D", blk.D) if blk.kind == "D" else ("R", blk.U, blk.V) for blk in H.leaf_blocks(p.oa.root)}
    opts = hm.make_opts(leaf=32, eta=2.0, eps=1e-6, prec=prec, lazy=2)
    B = hm.import_matrix(p.tree, opts, leaves)
    f = hm.LU(B, opts)
    of = H.hlu_accumulated(p.oa)
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    err = H.lu_error_2norm(dense, gf, exact=True)
    orank, grank = H.rank_table(of), H.rank_table(gf)
    d = np.array([grank[k] - orank[k] for k in orank])
    print(f"accumulated H-LU: ||PA-LU||/||A|| {err:.2e}, rank differences", np.unique(d, return_counts=True))
    assert err <= 10 * p.eps
    assert np.abs(d).max() <= 2
    b = inputs.rhs(p.n, 8, seed=1)
    xg = to_host(f.solve(device_rhs(b))[0])
    xo = H.solve(of, b)
    a_user = np.empty_like(dense)
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = dense
    rg = np.linalg.norm(b - a_user @ xg, axis=0) / np.linalg.norm(b, axis=0)
    ro = np.linalg.norm(b - a_user @ xo, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(rg <= 2 * ro + 1e-12), (rg, ro)


def test_accumulated_hlu_executors_identical():
    """lazy = 2 on the persistent executor and level by level: bit-identical factors."""
    p = Problem(4096, 64, 1e-4, max_rank=64, prec=hm.MIXED, oracle=False)
    b = inputs.rhs(p.n, 3, seed=2)
    out = []
    for mode in (hm.DATAFLOW, hm.LEVEL):
        opts = hm.make_opts(leaf=64, eta=2.0, eps=1e-4, max_rank=64, prec=hm.MIXED, exec_mode=mode, lazy=2)
        x = device_rhs(b)
        hm.LU(p.A, opts).solve(x)
        out.append(to_host(x))
    assert np.array_equal(out[0], out[1])
