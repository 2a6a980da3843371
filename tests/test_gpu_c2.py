"""The n = 32768 sphere workload in plain FP64 (leaf 64, eta = 2, eps = 1e-6,
ranks capped at 64) on the device, compared with the FP64 oracle's stored
results (tests/golden/c2_sphere.npz, written by tests/golden/make_golden.py
from the oracle alone):

  * every low-rank leaf's rank, of the assembled matrix and of the H-LU
    factors, within +-2 of the oracle's;
  * unrefined solve residuals against the exact kernel matrix, per right-hand
    side, at most 2x the oracle's;
  * ||P A - L U||_2 / ||A||_2 <= 10 eps with A the exact kernel matrix, by
    matrix-free power iteration (the factors applied from their exported
    leaves, A in row chunks);
  * the rank cap: how often it bound is reported (the oracle's ranks stay far
    below 64 here, so it must not bind).
"""
import os

import numpy as np
import pytest

from paper_1911_07531_amd import hm, inputs
from tests.exact_ops import Factors, exact_residuals, lu_error_estimate
from tests.gpu_common import device_rhs, require_gpu, to_host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_sphere.npz")


@pytest.fixture(scope="module")
def c2():
    require_gpu()
    g = np.load(GOLDEN)
    n, leaf, eps, cap = int(g["n"]), int(g["leaf"]), float(g["eps"]), int(g["max_rank"])
    pts, diag = inputs.sphere_problem(n, 0)
    opts = hm.make_opts(leaf=leaf, eta=float(g["eta"]), eps=eps, max_rank=cap, prec=hm.FP64, lazy=int(g["lazy"]))
    tree = hm.Tree(pts, opts)
    A = hm.Matrix(tree, hm.LAPLACE3D, diag, opts)
    f = hm.LU(A, opts)
    return g, pts, diag, tree, A, f


def _ranks(handle, kind, blocks):
    import ctypes
    r = ctypes.c_int32()
    out = np.empty(len(blocks), np.int32)
    for i, b in enumerate(blocks):
        hm._check(hm.lib().hm_export_leaf(handle, kind, int(b), None, ctypes.byref(r), None))
        out[i] = r.value
    return out


def test_ranks_within_two_of_oracle(c2):
    g, _, _, _, A, f = c2
    ga = _ranks(A.h, 0, g["blocks"])
    gf = _ranks(f.h, 1, g["blocks"])
    da = ga - g["assembly_rank"]
    df = gf - g["factor_rank"]
    print("assembly rank differences", np.unique(da, return_counts=True))
    print("factor rank differences", np.unique(df, return_counts=True))
    assert np.abs(da).max() <= 2
    assert np.abs(df).max() <= 2
    st = f.stats()
    print("truncations the cap or capacity bound:", st["rank_overflows"])
    assert st["rank_overflows"] == 0


def test_unrefined_residuals_within_twice_oracle(c2):
    g, pts, diag, _, _, f = c2
    b = inputs.rhs(len(pts), len(g["residual"]), seed=int(g["rhs_seed"]))
    x = to_host(f.solve(device_rhs(b))[0])
    r = exact_residuals(pts, diag, b, x)
    print("device residuals", r.min(), r.max(), "oracle", g["residual"].min(), g["residual"].max())
    assert np.all(r <= 2.0 * g["residual"])


def test_lu_error_bound_matrix_free(c2):
    g, pts, diag, tree, _, f = c2
    perm, _, _, _ = tree.tables()
    fac = Factors(f, tree)
    err = lu_error_estimate(pts[perm], diag, fac)
    print(f"||PA - LU||_2 / ||A||_2 ~ {err:.3e} (bound {10 * float(g['eps']):.1e})")
    assert err <= 10 * float(g["eps"])


def test_truncation_routes_exercised(c2, monkeypatch):
    """The comparisons above cover the device's truncation routes: the same
    factorization, repeated with the per-task timeline on (which does not
    change the arithmetic: the ranks must equal the untimed run's), records
    for every truncation its route and stacked width K.  Required: the
    small-rank route (K <= 32), the dense small-leaf route, and the Gram route
    both with K <= 64 (Gram matrices on the matrix cores) and with K > 64
    (tiled GEMM); the histogram is printed."""
    g, _, _, tree, A, f0 = c2
    opts = hm.make_opts(leaf=int(g["leaf"]), eta=float(g["eta"]), eps=float(g["eps"]), max_rank=int(g["max_rank"]),
                        prec=hm.FP64, lazy=int(g["lazy"]))
    monkeypatch.setenv("HM_DEBUG_TRACE", "1")
    f = hm.LU(A, opts)
    tl, _ = f.timeline()
    ops = tree.dag(opts, 0)["tasks"]["op"]
    tr = np.isin(ops, (hm.OP_NAMES.index("trunc"), hm.OP_NAMES.index("trunc2")))
    info, info2 = tl[tr, 2], tl[tr, 3]
    K = ((info >> 16) & 0xFFFF).astype(np.int64)
    route = (info2 & 0xFF).astype(np.int64)
    for r in np.unique(route):
        sel = route == r
        print(f"route {r}: {int(sel.sum())} truncations, K {int(K[sel].min())}..{int(K[sel].max())}")
    assert ((route == 1) & (K <= 32)).any()
    assert (route == 2).any()
    assert ((route == 3) & (K > 32) & (K <= 64)).any()
    assert ((route == 3) & (K > 64)).any()
    assert np.array_equal(_ranks(f.h, 1, g["blocks"]), _ranks(f0.h, 1, g["blocks"]))
