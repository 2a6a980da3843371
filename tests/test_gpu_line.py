"""GPU parity on the one-dimensional model problem of Sec. 5.1: the log
kernel -log|x - y| / (2 pi) on n uniform cells of [0, 1], standard
admissibility with eta = 2 (a coarse block structure, three blocks per block
row on every level of a deep hierarchy).

Bars as for the sphere workload: assembly ranks within +-2 of the oracle's
truncated SVD and block errors <= 2 eps sigma_1; ||P A - L U||_2 / ||A||_2 <=
10 eps and factor ranks within +-2 of the oracle's; solve relative residuals
<= 2x the oracle's (+ 1e-12); mixed precision refined to 1e-10; the level and
dataflow executors bit-identical.  At n = 131072 (the benchmark's launch
configuration) properties that hold at any size: refinement to 1e-10 and a
componentwise residual of sampled exact-kernel rows within eps.
"""
import numpy as np
import pytest

from oracle import hmatrix as H
from paper_1911_07531_amd import hm, inputs
from tests.gpu_common import Problem, device_rhs, require_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def line():
    """n = 2048, leaf 32, eta = 2, eps = 1e-6 (updates collected per hmul call on both sides)."""
    p = Problem(2048, 32, 1e-6, geometry="line")
    f = hm.LU(p.A, p.opts)
    of = H.hlu(p.oa, lazy=True)
    return p, f, of


def _rank_diff(a, b):
    ra, rb = H.rank_table(a), H.rank_table(b)
    return np.array([ra[k] - rb[k] for k in rb])


def test_line_tree_shape(line):
    p, _, _ = line
    _, cl, _, bl = p.tree.tables()
    # 2048 / 32 = 64 leaves, 6 levels; dense leaves 3 * 64 - 2, low rank sum_{l=2}^{6} (3 * 2^l - 6)
    assert np.count_nonzero(bl[:, 2] == 1) == 3 * 64 - 2
    assert np.count_nonzero(bl[:, 2] == 2) == sum(3 * 2 ** l - 6 for l in range(2, 7))


def test_line_assembly(line):
    p, _, _ = line
    ga = p.gpu_as_oracle(0, p.A.h)
    d = _rank_diff(ga, p.oa)
    assert np.max(np.abs(d)) <= 2, np.unique(d, return_counts=True)
    for b in H.leaf_blocks(ga.root):
        exact = p.exact_block(ga.perm, b.tau, b.sigma)
        if b.kind == "R":
            assert np.linalg.norm(exact - b.U @ b.V.T, 2) <= 2 * p.eps * np.linalg.norm(exact, 2)
        else:
            assert np.max(np.abs(b.D - exact)) <= 1e-15 * np.abs(exact).max()


def test_line_hlu_error_and_ranks(line):
    p, f, of = line
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    err = H.lu_error_2norm(dense, gf, exact=True)
    oerr = H.lu_error_2norm(dense, of, exact=True)
    print(f"line: gpu ||PA-LU||/||A|| = {err:.3e}, oracle {oerr:.3e}")
    assert err <= 10 * p.eps
    d = _rank_diff(gf, of)
    assert np.max(np.abs(d)) <= 2, np.unique(d, return_counts=True)


def test_line_solve_residuals(line):
    p, f, of = line
    b = inputs.rhs(p.n, 16, seed=1)
    xg = to_host(f.solve(device_rhs(b))[0])
    xo = H.solve(of, b)
    dense = p.dense_exact()
    a_user = np.empty_like(dense)
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = dense
    rg = np.linalg.norm(b - a_user @ xg, axis=0) / np.linalg.norm(b, axis=0)
    ro = np.linalg.norm(b - a_user @ xo, axis=0) / np.linalg.norm(b, axis=0)
    print("line residual gpu / oracle", rg.max(), ro.max())
    assert np.all(rg <= 2 * ro + 1e-12)


def test_line_mixed_precision_refined():
    p = Problem(2048, 32, 1e-6, prec=hm.MIXED, geometry="line")
    f = hm.LU(p.A, p.opts)
    gf = p.gpu_as_oracle(1, f.h)
    err = H.lu_error_2norm(p.dense_exact(), gf, exact=True)
    print(f"line mixed ||PA-LU||/||A|| = {err:.3e}")
    assert err <= 10 * p.eps
    b = inputs.rhs(p.n, 4, seed=1)
    xd = device_rhs(b)
    _, iters, rel = f.solve(xd, refine_with=p.A, rtol=1e-10, max_iter=50)
    assert np.all(rel <= 1e-10), rel


def test_line_executors_identical():
    p = Problem(4096, 32, 1e-6, oracle=False, geometry="line")
    f1 = hm.LU(p.A, hm.make_opts(leaf=32, eta=2.0, eps=1e-6, exec_mode=hm.DATAFLOW))
    f2 = hm.LU(p.A, hm.make_opts(leaf=32, eta=2.0, eps=1e-6, exec_mode=hm.LEVEL))
    _, _, _, bl = p.tree.tables()
    for bi in np.nonzero(bl[:, 2] != 0)[0]:
        r1, r2 = f1.leaf(int(bi)), f2.leaf(int(bi))
        assert r1[0] == r2[0]
        assert np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


def test_line_full_size_refined_and_sampled_rows():
    n, eps = 131072, 1e-4
    pts, diag = inputs.line_problem(n)
    opts = hm.make_opts(leaf=64, eta=2.0, eps=eps, max_rank=64, prec=hm.MIXED)
    tree = hm.Tree(pts, opts)
    A = hm.Matrix(tree, hm.LOG2D, diag, opts)
    f = hm.LU(A, opts)
    b = inputs.rhs(n, 8, seed=1)
    xd = device_rhs(b)
    _, iters, rel = f.solve(xd, refine_with=A, rtol=1e-10, max_iter=50)
    print("line n=131072: IR iterations", iters.tolist(), "max relative residual", rel.max())
    assert np.all(rel <= 1e-10)
    x = to_host(xd)
    rows = np.random.default_rng(5).choice(n, 48, replace=False)
    # exact rows from the oracle's kernel: the sampled rows, then all columns
    perm = np.concatenate([rows, np.arange(n)])
    c = H.Cluster(0, 0, len(perm), np.zeros(1), np.zeros(1), 0)
    a = H.kernel_block(pts, perm, c, c, diag, r=(0, len(rows)), c=(len(rows), len(perm)), kernel="log2d")
    res = np.abs(b[rows] - a @ x)
    worst = (res / (np.abs(a) @ np.abs(x))).max()
    print("line n=131072: sampled componentwise residual against the exact kernel", worst)
    assert worst <= eps
