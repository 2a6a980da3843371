"""Pins for the oracle's arithmetic (CPU only).

* leaf getrf (Algorithm 2, leaf branch) against LAPACK's getrf via scipy on
  the same block: identical interchanges, equal values to rounding;
* compression and truncated addition (Sec. 2.3) against Eckart-Young on the
  dense SVD of the exact sum;
* every leaf-case product term (the special routines after Algorithm 1)
  against the dense product of the densified operands;
* whole H-LU at eps = 0 with full ranks against an independent dense
  right-looking block LU with leaf-local pivoting (Algorithm 2 in exact
  arithmetic), including the degenerate all-dense case (no admissible block)
  and the block-diagonal special case;
* the 10*eps bound of ||P A - L U||_2 / ||A||_2 at n = 2048 (exact 2-norm) and
  agreement of the power-iteration estimate with it;
* solve and matvec against dense products; iterative refinement;
* the log kernel of the one-dimensional model problem (Sec. 5.1): row sums
  of the matrix times h against the closed-form integral of the kernel over
  [0, 1] (midpoint rule, O(h) error), and the same eps = 0 and 10*eps pins
  on the line.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import hmatrix as H
from paper_1911_07531_amd import inputs


def _problem(n, leaf, eta, eps, max_rank=0, seed=0, geometry="sphere"):
    if geometry == "sphere":
        (pts, diag), kernel = inputs.sphere_problem(n, seed), "laplace3d"
    else:
        (pts, diag), kernel = inputs.line_problem(n), "log2d"
    perm, cl = H.build_cluster_tree(pts, leaf)
    root = H.build_block_tree(cl[0], eta)
    a = H.assemble(pts, perm, cl, root, diag, eps, max_rank, kernel=kernel)
    dense = H.kernel_block(pts, perm, cl[0], cl[0], diag, kernel=kernel)
    return a, dense


@pytest.mark.parametrize("m", [1, 2, 7, 32, 64])
def test_getrf_leaf_matches_lapack(m):
    rng = np.random.default_rng(m)
    a = rng.standard_normal((m, m))
    lu_ref, piv_ref = sla.lu_factor(a)
    b = a.copy()
    piv = H.getrf_leaf(b)
    assert np.array_equal(piv, piv_ref)
    assert np.allclose(b, lu_ref, rtol=0, atol=1e-13 * np.abs(a).max() * m)


def test_getrf_first_maximum_wins_ties():
    a = np.array([[1.0, 2.0, 0.0], [-1.0, 0.0, 1.0], [1.0, 1.0, 1.0]])
    piv = H.getrf_leaf(a.copy())
    assert piv[0] == 0  # |1| == |-1| == |1|: the first row is kept
    _, piv_ref = sla.lu_factor(np.array([[1.0, 2.0, 0.0], [-1.0, 0.0, 1.0], [1.0, 1.0, 1.0]]))
    assert np.array_equal(piv, piv_ref)


def test_getrf_zero_pivot_reports_row():
    a = np.zeros((4, 4))
    a[0, 0] = 1.0
    with pytest.raises(H.SingularError) as ei:
        H.getrf_leaf(a, row0=100)
    assert ei.value.row == 101


def test_apply_pivots_is_lapack_laswp():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((9, 9))
    lu, piv = sla.lu_factor(a)
    p, l, u = sla.lu(a)  # a = p l u
    x = rng.standard_normal((9, 4))
    y = x.copy()
    H.apply_pivots(piv, y)
    assert np.allclose(y, p.T @ x)


def test_compression_eckart_young():
    a, _ = _problem(2048, 32, 2.0, 1e-6)
    pts, diag = inputs.sphere_problem(2048, 0)
    lr = [b for b in H.leaf_blocks(a.root) if b.kind == "R"]
    rng = np.random.default_rng(0)
    for b in rng.choice(lr, 20, replace=False):
        exact = H.kernel_block(pts, a.perm, b.tau, b.sigma, diag)
        s = np.linalg.svd(exact, compute_uv=False)
        k = b.rank
        assert k == int(np.sum(s > 1e-6 * s[0]))
        err = np.linalg.norm(exact - b.U @ b.V.T, 2)
        tail = s[k] if k < len(s) else 0.0
        assert abs(err - tail) <= 1e-10 * s[0]
        assert err <= 1e-6 * s[0]
        # V has orthonormal columns, Sigma is carried by U
        assert np.allclose(b.V.T @ b.V, np.eye(k), atol=1e-12)


def test_randomized_compression_bound(monkeypatch):
    monkeypatch.setattr(H, "RANDOMIZED_MIN_SIDE", 100)
    pts, diag = inputs.sphere_problem(4096, 0)
    perm, cl = H.build_cluster_tree(pts, 64)
    root = H.build_block_tree(cl[0], 2.0)
    big = [b for b in H.block_list(root) if b.kind == "R" and min(b.rows, b.cols) > 100][:3]
    assert big
    for b in big:
        exact = H.kernel_block(pts, perm, b.tau, b.sigma, diag)
        s = np.linalg.svd(exact, compute_uv=False)
        sub = H.Block(0, b.tau, b.sigma, "R")
        leafs = H.HMatrix(sub, perm, cl, 4096, 1e-4, 0)
        del leafs
        H.assemble(pts, perm, cl, sub, diag, 1e-4, 0)
        err = np.linalg.norm(exact - sub.U @ sub.V.T, 2)
        assert err <= 1.5e-4 * s[0]
        assert abs(sub.rank - int(np.sum(s > 1e-4 * s[0]))) <= 2


@pytest.mark.parametrize("eps,max_rank", [(1e-6, 0), (1e-3, 0), (1e-8, 5), (0.0, 0)])
def test_truncated_add_eckart_young(eps, max_rank):
    rng = np.random.default_rng(7)
    m, n = 120, 90
    t = H.Cluster(0, 0, m, np.zeros(3), np.zeros(3), 0)
    s = H.Cluster(1, 0, n, np.zeros(3), np.zeros(3), 0)
    c = H.Block(0, t, s, "R")
    # a decaying low-rank C and a term on a sub-range
    c.U = rng.standard_normal((m, 12)) * np.logspace(0, -9, 12)
    c.V = np.linalg.qr(rng.standard_normal((n, 12)))[0]
    up = rng.standard_normal((40, 6)) * 1e-3
    vp = rng.standard_normal((30, 6))
    total = c.U @ c.V.T
    total[10:50, 20:50] += up @ vp.T
    H.truncated_add(c, 10, 20, up, vp, eps, max_rank)
    sv = np.linalg.svd(total, compute_uv=False)
    k = min(int(np.sum(sv > eps * sv[0])), 18)  # never above the stacked width
    if max_rank:
        k = min(k, max_rank)
    assert c.rank == k
    err = np.linalg.norm(total - c.U @ c.V.T, 2)
    tail = sv[k] if k < len(sv) else 0.0
    assert abs(err - tail) <= 1e-9 * sv[0]


def _rand_leaf(rng, kind, t, s, rank=5):
    b = H.Block(rng.integers(1 << 30), t, s, kind)
    if kind == "D":
        b.D = rng.standard_normal((t.size, s.size))
    else:
        b.U = rng.standard_normal((t.size, rank))
        b.V = rng.standard_normal((s.size, rank))
    return b


def test_product_terms_all_cases():
    rng = np.random.default_rng(11)
    pts = inputs.sphere_points(512, 4)
    perm, cl = H.build_cluster_tree(pts, 32)
    root = H.build_block_tree(cl[0], 2.0)
    a, _ = _problem(512, 32, 2.0, 1e-10)
    blocks = {b.index: b for b in H.block_list(a.root)}
    seen = set()
    # every (A, B) pair of blocks on a common inner cluster that hmul can meet
    for ab in blocks.values():
        for bb in blocks.values():
            if ab.sigma is not bb.tau:
                continue
            key = (ab.kind, bb.kind, ab.tau.is_leaf, ab.sigma.is_leaf, bb.sigma.is_leaf)
            if key in seen or (ab.kind == "S" and bb.kind == "S" and ab.rows > 128):
                continue
            seen.add(key)
            terms = H.product_terms(-0.5, ab, bb)
            dense = np.zeros((ab.rows, bb.cols))
            for (r, c, u, v) in terms:
                dense[r:r + u.shape[0], c:c + v.shape[0]] += u @ v.T
            ref = -0.5 * H.densify(ab) @ H.densify(bb)
            assert np.allclose(dense, ref, atol=1e-12 * max(1, np.abs(ref).max()))
    kinds = {(k[0], k[1]) for k in seen}
    assert {("R", "D"), ("D", "R"), ("D", "D"), ("S", "S"), ("R", "S"), ("S", "R")} <= kinds
    del rng, root


def _dense_block_lu(a, leaf_ranges):
    """Right-looking block LU with pivoting restricted to each diagonal leaf.

    Off-diagonal L blocks are left unpermuted (the swaps only touch the
    diagonal leaf and the columns to its right).  Written independently of the
    oracle's recursion; LAPACK's getrf factors each diagonal leaf.
    """
    a = a.copy()
    pivs = []
    for (r0, r1) in leaf_ranges:
        lu, piv = sla.lu_factor(a[r0:r1, r0:r1])
        a[r0:r1, r0:r1] = lu
        right = a[r0:r1, r1:]
        for j, p in enumerate(piv):
            right[[j, p]] = right[[p, j]]
        right[:] = sla.solve_triangular(lu, right, lower=True, unit_diagonal=True)
        below = sla.solve_triangular(lu, a[r1:, r0:r1].T, trans="T", lower=False).T
        a[r1:, r0:r1] = below
        a[r1:, r1:] -= below @ right
        pivs.append(piv)
    return a, pivs


@pytest.mark.parametrize("n,leaf,eta,geometry", [(512, 32, 2.0, "sphere"), (700, 24, 1.0, "sphere"),
                                                  (256, 32, 0.0, "sphere"), (512, 32, 2.0, "line"),
                                                  (600, 20, 2.0, "line")])
def test_hlu_eps0_equals_dense_block_lu(n, leaf, eta, geometry):
    a, dense = _problem(n, leaf, eta, 0.0, geometry=geometry)
    if eta == 0.0:
        assert all(b.kind != "R" for b in H.leaf_blocks(a.root))
    else:
        assert any(b.kind == "R" for b in H.leaf_blocks(a.root))
        # full rank: every admissible block kept at min(m, n) (numerically)
        assert np.allclose(H.densify(a.root), dense, atol=1e-12 * np.abs(dense).max())
    f = H.hlu(a)
    leaves = sorted({(c.begin, c.end) for c in a.clusters if c.is_leaf})
    ref, pivs = _dense_block_lu(dense, leaves)
    got = H.densify(f.root)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(dense).max() * 10
    diag = {b.tau.begin: b.piv for b in H.leaf_blocks(f.root) if b.tau is b.sigma}
    for (r0, _), piv in zip(leaves, pivs):
        assert np.array_equal(diag[r0], piv)


def test_hlu_block_diagonal_special_case():
    a, dense = _problem(512, 32, 2.0, 1e-8)
    for b in H.leaf_blocks(a.root):
        if b.tau is not b.sigma:
            if b.kind == "D":
                b.D[:] = 0.0
            else:
                b.U = np.zeros((b.rows, 0))
                b.V = np.zeros((b.cols, 0))
    f = H.hlu(a)
    for b in H.leaf_blocks(f.root):
        if b.tau is b.sigma:
            lu, piv = sla.lu_factor(H.densify(next(x for x in H.leaf_blocks(a.root) if x.index == b.index)))
            assert np.array_equal(b.piv, piv)
            assert np.allclose(b.D, lu, atol=1e-13 * np.abs(lu).max())
        elif b.kind == "R":
            assert b.rank == 0
        else:
            assert not b.D.any()


@pytest.fixture(scope="module")
def c1():
    """n = 2048, leaf 32, eta = 2, eps = 1e-6 (the small sphere workload)."""
    a, dense = _problem(2048, 32, 2.0, 1e-6)
    f = H.hlu(a)
    return a, dense, f


def test_hlu_error_bound_c1(c1):
    a, dense, f = c1
    err = H.lu_error_2norm(dense, f, exact=True)
    assert err <= 10 * 1e-6
    est = H.lu_error_2norm(dense, f, exact=False, iters=200)
    assert abs(est - err) <= 0.05 * err


def test_hlu_factor_identity_c1(c1):
    """P A_H = Lp U up to the truncation error (factors reproduce the H-matrix)."""
    a, dense, f = c1
    p, lp, u = H.lu_dense_factors(f)
    ah = H.densify(a.root)
    assert np.linalg.norm(ah[p] - lp @ u, 2) <= 10 * 1e-6 * np.linalg.norm(ah, 2)
    # L unit lower, U upper triangular
    assert np.allclose(np.diag(lp), 1.0)
    assert not np.triu(lp, 1).any()
    assert not np.tril(u, -1).any()


def test_solve_and_matvec_c1(c1):
    a, dense, f = c1
    b = inputs.rhs(2048, 16, seed=1)
    ah_user = np.empty_like(dense)
    ah_user[np.ix_(a.perm, a.perm)] = H.densify(a.root)
    y = H.matvec(a, b)
    assert np.allclose(y, ah_user @ b, atol=1e-13 * np.abs(ah_user @ b).max())
    y2 = H.matvec(a, b, alpha=2.0, beta=-1.0, y=y)
    assert np.allclose(y2, y, atol=1e-12 * np.abs(y).max())
    x = H.solve(f, b)
    p, lp, u = H.lu_dense_factors(f)
    # the solve inverts exactly the factors: Lp U x_perm = P b_perm
    xp = x[a.perm]
    bp = b[a.perm]
    assert np.allclose(lp @ (u @ xp), bp[p], atol=1e-10 * np.abs(bp).max())
    a_user = np.empty_like(dense)
    a_user[np.ix_(a.perm, a.perm)] = dense
    res = np.linalg.norm(b - a_user @ x, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(res <= 1e-4)


def test_refinement_converges_c1(c1):
    a, dense, f = c1
    b = inputs.rhs(2048, 4, seed=1)
    x, it, rel = H.refine(a, f, b, rtol=1e-10, max_iter=30)
    assert np.all(rel <= 1e-10)
    assert it <= 10


def test_hlu_lazy_eps0_equals_dense_block_lu():
    """Collected updates (Reading R6) change only the grouping of truncations:
    at eps = 0 the factors still equal the dense leaf-pivoted block LU."""
    a, dense = _problem(512, 32, 2.0, 0.0)
    f = H.hlu(a, lazy=True)
    leaves = sorted({(c.begin, c.end) for c in a.clusters if c.is_leaf})
    ref, pivs = _dense_block_lu(dense, leaves)
    assert np.max(np.abs(H.densify(f.root) - ref)) <= 1e-11 * np.abs(dense).max()
    assert all(not b.pending for b in H.leaf_blocks(f.root))


def test_hlu_lazy_error_bound_c1(c1):
    a, dense, _ = c1
    f = H.hlu(a, lazy=True)
    assert H.lu_error_2norm(dense, f, exact=True) <= 10 * 1e-6
    # one truncation per collected batch: the truncation of an exact sum is at
    # least as accurate as the sequential chain, so ranks are never much lower
    seq = H.rank_table(H.hlu(a))
    lz = H.rank_table(f)
    assert min(lz[i] - seq[i] for i in seq) >= -2


@pytest.mark.parametrize("geometry", ["sphere", "line"])
def test_hlu_accumulated_eps0_equals_dense_block_lu(geometry):
    """The accumulated H-LU (Algorithms 4-8) only regroups the updates: at
    eps = 0 (every accumulator and block kept at full rank) the factors equal
    the dense leaf-pivoted block LU, pivots included."""
    a, dense = _problem(512, 32, 2.0, 0.0, geometry=geometry)
    f = H.hlu_accumulated(a)
    leaves = sorted({(c.begin, c.end) for c in a.clusters if c.is_leaf})
    ref, pivs = _dense_block_lu(dense, leaves)
    assert np.max(np.abs(H.densify(f.root) - ref)) <= 1e-11 * np.abs(dense).max()
    diag = {b.tau.begin: b.piv for b in H.leaf_blocks(f.root) if b.tau is b.sigma}
    for (r0, _), piv in zip(leaves, pivs):
        assert np.array_equal(diag[r0], piv)


def test_hlu_accumulated_error_bound_and_fewer_truncations():
    """Accumulated updates meet the 10 eps bound against the exact matrix and
    need fewer truncated additions than the sequential H-LU of Algorithm 2
    (the saving the accumulators are for, Sec. 2.3)."""
    a, dense = _problem(1024, 32, 2.0, 1e-6)
    H.TRUNCATIONS[0] = 0
    fs = H.hlu(a)
    n_seq = H.TRUNCATIONS[0]
    H.TRUNCATIONS[0] = 0
    fa = H.hlu_accumulated(a)
    n_acc = H.TRUNCATIONS[0]
    assert H.lu_error_2norm(dense, fa, exact=True) <= 10 * 1e-6
    assert n_acc < n_seq, (n_acc, n_seq)
    # accumulators truncated against their own largest singular value keep a
    # little more than the sequential chain, never less
    rs, ra = H.rank_table(fs), H.rank_table(fa)
    assert min(ra[i] - rs[i] for i in rs) >= -2
    assert fs is not fa


def test_log_kernel_row_sums_are_the_integral():
    """h * sum_j a_ij approximates the integral of -log|x_i - y| / (2 pi) over
    [0, 1], which is (1 - x log x - (1 - x) log(1 - x)) / (2 pi): the own cell
    is exact (the diagonal is the cell mean) and the midpoint rule on the
    others errs by about h * zeta(2) / (12 * 2 pi) ~ 0.022 h.  A wrong sign,
    scale, logarithm base or self term misses this by more than 0.1 h."""
    import math
    for n in (256, 2048):
        pts, diag = inputs.line_problem(n)
        perm, cl = H.build_cluster_tree(pts, 32)
        a = H.kernel_block(pts, perm, cl[0], cl[0], diag, kernel="log2d")
        x = pts[perm, 0]
        exact = (1.0 - x * np.log(x) - (1.0 - x) * np.log1p(-x)) / (2.0 * math.pi)
        err = np.abs(a.sum(axis=1) / n - exact)
        assert err.max() <= 0.03 / n, err.max() * n
        assert err.max() >= 0.01 / n  # the midpoint rule's own error is visible


@pytest.mark.parametrize("lazy", [False, True])
def test_hlu_error_bound_line(lazy):
    a, dense = _problem(2048, 32, 2.0, 1e-6, geometry="line")
    f = H.hlu(a, lazy=lazy)
    err = H.lu_error_2norm(dense, f, exact=True)
    assert err <= 10 * 1e-6
    # the coarse 1D structure: ranks stay small (log-kernel blocks one cluster apart)
    ranks = [b.rank for b in H.leaf_blocks(f.root) if b.kind == "R"]
    assert 0 < max(ranks) <= 24
