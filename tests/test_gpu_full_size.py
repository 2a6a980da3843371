"""The n = 131072 sphere workload (leaf 64, eps = 1e-4, ranks capped at 64,
FP32 off-diagonal storage) in the launch configuration the benchmark times:

  * against the FP64 oracle's stored results (tests/golden/c3_sphere.npz,
    written by tests/golden/make_golden.py from the oracle alone, about 2.5 h
    on a CPU): every low-rank leaf's rank, of the assembled matrix and of the
    H-LU factors, within +-2 of the oracle's, and the unrefined solve
    residuals against the exact kernel matrix at most 2x the oracle's;
  * properties that hold at any size: refinement converges to 1e-10 against
    the FP64 H-matvec; sampled rows of the exact kernel matrix give a
    componentwise residual within the truncation accuracy; the level and
    dataflow executors give bit-identical factors."""
import os

import numpy as np
import pytest

from paper_1911_07531_amd import hm, inputs
from tests.gpu_common import device_rhs, require_gpu, to_host

pytestmark = pytest.mark.gpu

N, LEAF, EPS, CAP = 131072, 64, 1e-4, 64


@pytest.fixture(scope="module")
def c3():
    require_gpu()
    pts, diag = inputs.sphere_problem(N, 0)
    opts = hm.make_opts(leaf=LEAF, eta=2.0, eps=EPS, max_rank=CAP, prec=hm.MIXED)
    tree = hm.Tree(pts, opts)
    A = hm.Matrix(tree, hm.LAPLACE3D, diag, opts)
    f = hm.LU(A, opts)
    return pts, diag, tree, A, f


def _exact_rows(pts, diag, rows):
    d = pts[rows][:, None, :] - pts[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    with np.errstate(divide="ignore"):
        a = 1.0 / (4.0 * np.pi * r)
    a[np.arange(len(rows)), rows] = diag
    return a


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3_sphere.npz")


def _ranks(handle, kind, blocks):
    import ctypes
    r = ctypes.c_int32()
    out = np.empty(len(blocks), np.int32)
    for i, b in enumerate(blocks):
        hm._check(hm.lib().hm_export_leaf(handle, kind, int(b), None, ctypes.byref(r), None))
        out[i] = r.value
    return out


def _exact_residuals_device(pts, diag, b, x, chunk=1024):
    """||b - A x||_2 / ||b||_2 per column with the exact kernel matrix A, its rows
    formed in chunks on the device with plain torch FP64 (test-side check)."""
    import torch
    P = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    X, B = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
    r2 = torch.zeros(B.shape[1], dtype=torch.float64, device="cuda")
    for r0 in range(0, len(pts), chunk):
        r1 = min(len(pts), r0 + chunk)
        d = P[r0:r1, None, :] - P[None, :, :]
        k = 1.0 / (4.0 * np.pi * torch.sqrt((d * d).sum(-1)))
        del d
        idx = torch.arange(r0, r1, device="cuda")
        k[idx - r0, idx] = diag
        res = B[r0:r1] - k @ X
        r2 += (res * res).sum(0)
    return (torch.sqrt(r2) / torch.linalg.norm(B, dim=0)).cpu().numpy()


def test_ranks_within_two_of_oracle_c3(c3):
    _, _, _, A, f = c3
    g = np.load(GOLDEN)
    assert int(g["n"]) == N and float(g["eps"]) == EPS and int(g["max_rank"]) == CAP
    da = _ranks(A.h, 0, g["blocks"]) - g["assembly_rank"]
    df = _ranks(f.h, 1, g["blocks"]) - g["factor_rank"]
    print("assembly rank differences", np.unique(da, return_counts=True))
    print("factor rank differences", np.unique(df, return_counts=True))
    assert np.abs(da).max() <= 2
    assert np.abs(df).max() <= 2
    assert f.stats()["rank_overflows"] == 0


def test_unrefined_residuals_within_twice_oracle_c3(c3):
    pts, diag, _, _, f = c3
    g = np.load(GOLDEN)
    b = inputs.rhs(N, len(g["residual"]), seed=int(g["rhs_seed"]))
    x = to_host(f.solve(device_rhs(b))[0])
    r = _exact_residuals_device(pts, diag, b, x)
    print("device residuals", r.min(), r.max(), "oracle", g["residual"].min(), g["residual"].max())
    assert np.all(r <= 2.0 * g["residual"])


def test_refined_solve_and_sampled_exact_rows(c3):
    pts, diag, _, A, f = c3
    b = inputs.rhs(N, 32, seed=1)
    xd = device_rhs(b)
    _, iters, rel = f.solve(xd, refine_with=A, rtol=1e-10, max_iter=50)
    print("IR iterations", iters.tolist(), "max relative residual", rel.max())
    assert np.all(rel <= 1e-10)
    x = to_host(xd)
    assert np.all(np.isfinite(x))
    rows = np.random.default_rng(5).choice(N, 48, replace=False)
    a = _exact_rows(pts, diag, rows)
    res = np.abs(b[rows] - a @ x)
    scale = np.abs(a) @ np.abs(x)
    worst = (res / scale).max()
    print("sampled componentwise residual against the exact kernel", worst)
    assert worst <= EPS


def test_level_and_dataflow_identical_full_size(c3):
    pts, diag, tree, A, f = c3
    opts = hm.make_opts(leaf=LEAF, eta=2.0, eps=EPS, max_rank=CAP, prec=hm.MIXED, exec_mode=hm.LEVEL)
    g = hm.LU(A, opts)
    b = inputs.rhs(N, 2, seed=2)
    x1, x2 = device_rhs(b), device_rhs(b)
    f.solve(x1)
    g.solve(x2)
    assert np.array_equal(to_host(x1), to_host(x2))


def test_fused_lu_solve_full_size(c3):
    """h_lu_solve at n = 131072: the same factors as h_lu (sampled leaves bit
    for bit) and the solution of h_lu + h_solve up to the rounding of the
    split products of the separate substitution."""
    pts, diag, tree, A, f = c3
    opts = hm.make_opts(leaf=LEAF, eta=2.0, eps=EPS, max_rank=CAP, prec=hm.MIXED)
    b = inputs.rhs(N, 4, seed=3)
    x1, x2 = device_rhs(b), device_rhs(b)
    f.solve(x1)
    g = hm.LU(A, opts, rhs=x2)
    x1, x2 = to_host(x1), to_host(x2)
    print("fused vs separate: max relative difference", np.abs(x1 - x2).max() / np.abs(x1).max())
    assert np.abs(x1 - x2).max() <= 1e-9 * np.abs(x1).max()
    _, _, _, bl = tree.tables()
    leaves = np.nonzero(bl[:, 2] != 0)[0]
    for bi in np.random.default_rng(1).choice(leaves, 200, replace=False):
        r1, r2 = f.leaf(int(bi)), g.leaf(int(bi))
        assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])
