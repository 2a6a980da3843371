"""The traced H-LU and solve DAGs, replayed in NumPy in random topological
orders, reproduce the oracle's sequential H-LU (Algorithm 2) and solve (CPU).

Same inputs on both sides (the oracle's assembled leaves are loaded into the
traced storage layout).  Truncation decisions follow the same order, so the
factors agree to rounding and the ranks agree exactly.
"""
import numpy as np
import pytest

from oracle import hmatrix as H
from paper_1911_07531_amd import hm, inputs
from tests.dag_replay import Replay


def _setup(n, leaf, eta, eps, max_rank, prec=hm.FP64, seed=0, lazy=0):
    pts, diag = inputs.sphere_problem(n, seed)
    opts = hm.make_opts(leaf=leaf, eta=eta, eps=eps, max_rank=max_rank, prec=prec, lazy=lazy)
    t = hm.Tree(pts, opts)
    perm, cl = H.build_cluster_tree(pts, leaf)
    root = H.build_block_tree(cl[0], eta)
    a = H.assemble(pts, perm, cl, root, diag, eps, max_rank)
    return t, opts, a


def _factors_from_replay(rp, t, a_template, dag):
    _, cl, _, bl = t.tables()
    f = H.hlu.__globals__["_copy_block"](a_template.root)
    for b in H.leaf_blocks(f):
        kind = "D" if b.kind == "D" else "R"
        m, n = b.rows, b.cols
        r = rp.leaf(b.index, 1 if kind == "D" else 2, m, n, dag["block_off"], dag["lr"])
        if kind == "D":
            b.D = r[1]
            if b.tau is b.sigma:
                b.piv = r[2]
        else:
            b.U, b.V = r[1], r[2]
    return H.HMatrix(f, a_template.perm, a_template.clusters, a_template.n, a_template.eps, a_template.max_rank)


@pytest.mark.parametrize("n,leaf,eps,max_rank,orders", [(512, 32, 1e-6, 0, 2), (1024, 24, 1e-4, 8, 1),
                                                        (600, 16, 1e-8, 0, 1)])
def test_replay_matches_oracle_hlu(n, leaf, eps, max_rank, orders):
    t, opts, a = _setup(n, leaf, 2.0, eps, max_rank)
    ref = H.hlu(a)
    dag = t.dag(opts, 0)
    blocks = {b.index: b for b in H.leaf_blocks(a.root)}
    ref_d = H.densify(ref.root)
    scale = np.abs(H.densify(a.root)).max()
    ref_ranks = H.rank_table(ref)
    for k in range(orders):
        rp = Replay(dag, eps, max_rank)
        rp.load_matrix(blocks, dag["block_off"], dag["lr"])
        rp.run(np.random.default_rng(k))
        f = _factors_from_replay(rp, t, a, dag)
        got = H.densify(f.root)
        assert np.max(np.abs(got - ref_d)) <= 1e-9 * scale
        ranks = H.rank_table(f)
        diff = [abs(ranks[i] - ref_ranks[i]) for i in ref_ranks]
        assert max(diff) <= 1 and sum(diff) <= max(2, len(diff) // 100)
        for b in H.leaf_blocks(f.root):
            if b.tau is b.sigma:
                ob = next(x for x in H.leaf_blocks(ref.root) if x.index == b.index)
                assert np.array_equal(b.piv, ob.piv)


@pytest.mark.parametrize("split,coarsen,reach", [(None, 0, 1), ("12", 0, 1), (None, 128, 1), ("12", 256, 1),
                                                (None, 40, 1), (None, 40, 3), ("12", 64, 4)])
def test_replay_solve_matches_oracle(split, coarsen, reach, monkeypatch):
    """The substitution DAG, with the large low-rank products split into
    partial products and their sums (split = 12 rows) or not, and with the
    diagonal blocks of at most `coarsen` rows run as one task each (the
    neighbouring block's product folded in) or not."""
    if split is not None:
        monkeypatch.setenv("HM_SOLVE_SPLIT", split)
    monkeypatch.setenv("HM_FOLD_REACH", str(reach))
    n, leaf, eps = 512, 32, 1e-6
    t, opts, a = _setup(n, leaf, 2.0, eps, 0)
    opts.coarsen = coarsen
    ref = H.hlu(a)
    dag = t.dag(opts, 0)
    sdag = t.dag(opts, 1)
    if coarsen == 0:
        assert (sdag["tasks"]["op"] == 11).any() == (split is not None)
    else:
        seq = sdag["seq"]
        assert (sdag["tasks"]["op"] == 12).any() and len(seq) > 0
        # some neighbour products were folded into the blocks' tasks (source rows outside the block)
        src_dyn = np.where(seq["op"] == 5, seq["b"]["dyn"], seq["x"]["dyn"])
        assert ((np.isin(seq["op"], (5, 6))) & ((src_dyn & 8) == 0)).any()
    blocks = {b.index: b for b in H.leaf_blocks(a.root)}
    rp = Replay(dag, eps, 0)
    rp.load_matrix(blocks, dag["block_off"], dag["lr"])
    rp.run(np.random.default_rng(3))
    # the solve DAG shares the storage layout; its panel sits in the f64 arena
    rs = Replay(sdag, eps, 0)
    rs.f64[:len(rp.f64)] = rp.f64[:len(rs.f64)] if len(rs.f64) <= len(rp.f64) else np.pad(rp.f64, (0, len(rs.f64) - len(rp.f64)))
    rs.piv[:] = rp.piv
    rs.ranks[:] = rp.ranks
    b = inputs.rhs(n, 5, seed=1)
    nrhs_slot = sdag["nranks"] - 1
    rs.ranks[nrhs_slot] = 5
    # the panel: the lowest offset a triangular solve or a coarsened block writes
    po = min([int(tk["x"]["off"]) for tk in sdag["tasks"] if tk["op"] in (2, 4)] +
             [int(tk["y"]["off"]) for tk in sdag["tasks"] if tk["op"] == 12])
    rs.f64[po:po + n * 5] = b[a.perm].flatten(order="F")
    rs.run(np.random.default_rng(4))
    x = np.empty((n, 5))
    x[a.perm] = rs.f64[po:po + n * 5].reshape(5, n).T
    ref_x = H.solve(ref, b)
    assert np.allclose(x, ref_x, rtol=0, atol=1e-9 * np.abs(ref_x).max())


@pytest.mark.parametrize("n,leaf,eps,max_rank", [(1024, 32, 1e-6, 0), (2048, 32, 1e-4, 16)])
def test_replay_lazy_updates_within_bounds(n, leaf, eps, max_rank):
    """Collected updates (balanced tree of truncations) stay within the parity
    bounds of the sequential H-LU: ||PA - LU||_2/||A||_2 <= 10 eps against the
    exact matrix, ranks within +-2 of the oracle's."""
    t, opts, a = _setup(n, leaf, 2.0, eps, max_rank, lazy=1)
    dag = t.dag(opts, 0)
    assert (dag["tasks"]["op"] == 10).any()
    blocks = {b.index: b for b in H.leaf_blocks(a.root)}
    rp = Replay(dag, eps, max_rank)
    rp.load_matrix(blocks, dag["block_off"], dag["lr"])
    rp.run(np.random.default_rng(7))
    f = _factors_from_replay(rp, t, a, dag)
    pts, diag = inputs.sphere_problem(n, 0)
    dense = H.kernel_block(pts, a.perm, a.clusters[0], a.clusters[0], diag)
    err = H.lu_error_2norm(dense, f, exact=True)
    assert err <= 10 * eps
    ref = H.hlu(a, lazy=True)
    rr, rg = H.rank_table(ref), H.rank_table(f)
    assert max(abs(rg[i] - rr[i]) for i in rr) <= 2
    assert H.lu_error_2norm(dense, ref, exact=True) <= 10 * eps


def test_replay_with_reused_temporaries(monkeypatch):
    """A ring of temporaries far smaller than the DAG needs: slots are reused by
    temporaries of other shapes, and every reuse must still be ordered after
    the slot's earlier accesses (random topological orders reproduce the
    collected-update H-LU within its bounds)."""
    n, leaf, eps, max_rank = 2048, 32, 1e-4, 16
    t_big, opts, a = _setup(n, leaf, 2.0, eps, max_rank, lazy=1)
    big = t_big.dag(opts, 0)
    monkeypatch.setenv("HM_TEMP_BUDGET_GB", "0.0005")
    t, _, _ = _setup(n, leaf, 2.0, eps, max_rank, lazy=1)
    dag = t.dag(opts, 0)
    assert dag["n_f32"] + dag["n_f64"] < big["n_f32"] + big["n_f64"]  # the small ring is reused
    blocks = {b.index: b for b in H.leaf_blocks(a.root)}
    pts, diag = inputs.sphere_problem(n, 0)
    dense = H.kernel_block(pts, a.perm, a.clusters[0], a.clusters[0], diag)
    ref = H.hlu(a, lazy=True)
    rr = H.rank_table(ref)
    for seed in (11, 12):
        rp = Replay(dag, eps, max_rank)
        rp.load_matrix(blocks, dag["block_off"], dag["lr"])
        rp.run(np.random.default_rng(seed))
        f = _factors_from_replay(rp, t, a, dag)
        assert H.lu_error_2norm(dense, f, exact=True) <= 10 * eps
        rg = H.rank_table(f)
        assert max(abs(rg[i] - rr[i]) for i in rr) <= 2


@pytest.mark.parametrize("lazy", [0, 1])
def test_fused_lu_solve_dag(lazy):
    """The H-LU and the substitution traced as one DAG (h_lu_solve): its first
    tasks are the H-LU DAG's tasks, record for record, with the same edges
    among them; replayed in random topological orders it gives the oracle's
    factors and solution."""
    n, leaf, eps = 512, 32, 1e-6
    t, opts, a = _setup(n, leaf, 2.0, eps, 0, lazy=lazy)
    dag = t.dag(opts, 0)
    fdag = t.dag(opts, 2)
    nl = len(dag["tasks"])
    assert len(fdag["tasks"]) > nl
    assert fdag["tasks"][:nl].tobytes() == dag["tasks"].tobytes()
    assert np.all(fdag["tasks"]["c1"][nl:] == 1)
    sp, si, fsp, fsi = dag["succ_ptr"], dag["succ_idx"], fdag["succ_ptr"], fdag["succ_idx"]
    for i in range(nl):
        own = fsi[fsp[i]:fsp[i + 1]]
        assert np.array_equal(np.sort(own[own < nl]), np.sort(si[sp[i]:sp[i + 1]]))
    assert np.all(fsi[fsp[nl]:] >= nl)  # no substitution task precedes an H-LU task
    ref = H.hlu(a, lazy=bool(lazy))
    b = inputs.rhs(n, 4, seed=2)
    ref_x = H.solve(ref, b)
    blocks = {bb.index: bb for bb in H.leaf_blocks(a.root)}
    for k in range(2):
        rp = Replay(fdag, eps, 0)
        rp.load_matrix(blocks, fdag["block_off"], fdag["lr"])
        rs = fdag["nranks"] - 1
        rp.ranks[rs] = 4
        po = min(int(tk["x"]["off"]) for tk in fdag["tasks"][nl:] if tk["op"] in (2, 4))
        rp.f64[po:po + n * 4] = b[a.perm].flatten(order="F")
        rp.run(np.random.default_rng(10 + k))
        x = np.empty((n, 4))
        x[a.perm] = rp.f64[po:po + n * 4].reshape(4, n).T
        if lazy:
            # collected updates: the device combines a batch by a tree of
            # truncations, the oracle in one; compare through the residual
            f = _factors_from_replay(rp, t, a, fdag)
            assert np.allclose(x, H.solve(f, b), rtol=0, atol=1e-9 * np.abs(x).max())
        else:
            assert np.allclose(x, ref_x, rtol=0, atol=1e-9 * np.abs(ref_x).max())


@pytest.mark.parametrize("lazy", [0, 1])
def test_replay_leaf_128_within_bounds(lazy):
    """Leaves of up to 128 points: dense-dense products over an inner leaf of
    more than 64 points (and identity factors of such leaves) reach a
    low-rank leaf as column chunks of at most 64, each truncated; the replay
    stays within the parity bounds of the oracle (10 eps, ranks +-2)."""
    n, leaf, eps = 1024, 128, 1e-6
    t, opts, a = _setup(n, leaf, 2.0, eps, 0, lazy=lazy)
    dag = t.dag(opts, 0)
    blocks = {b.index: b for b in H.leaf_blocks(a.root)}
    rp = Replay(dag, eps, 0)
    rp.load_matrix(blocks, dag["block_off"], dag["lr"])
    rp.run(np.random.default_rng(21))
    f = _factors_from_replay(rp, t, a, dag)
    pts, diag = inputs.sphere_problem(n, 0)
    dense = H.kernel_block(pts, a.perm, a.clusters[0], a.clusters[0], diag)
    assert H.lu_error_2norm(dense, f, exact=True) <= 10 * eps
    ref = H.hlu(a, lazy=bool(lazy))
    rr, rg = H.rank_table(ref), H.rank_table(f)
    assert max(abs(rg[i] - rr[i]) for i in rr) <= 2


def test_replay_accumulated_matches_oracle():
    """lazy mode 2 (the accumulated H-LU of Algorithms 4-8 on the device): the
    traced DAG replayed in a random topological order equals the oracle's
    hlu_accumulated to rounding, ranks exactly (accumulators, their shifts
    and the application before each leaf's factorization or solve)."""
    n, leaf, eps = 1024, 32, 1e-6
    t, opts, a = _setup(n, leaf, 2.0, eps, 0, lazy=2)
    dag = t.dag(opts, 0)
    blocks = {b.index: b for b in H.leaf_blocks(a.root)}
    rp = Replay(dag, eps, 0)
    rp.load_matrix(blocks, dag["block_off"], dag["lr"])
    rp.run(np.random.default_rng(13))
    f = _factors_from_replay(rp, t, a, dag)
    ref = H.hlu_accumulated(a)
    assert H.rank_table(f) == H.rank_table(ref)
    got, want = H.densify(f.root), H.densify(ref.root)
    assert np.max(np.abs(got - want)) <= 1e-9 * np.abs(want).max()
