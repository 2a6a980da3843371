"""hm_import (the parity hook that takes an H-matrix from host leaves) on the
device.

* export -> import round trip: the imported copy of an assembled matrix has
  the same H-matvec and factors to the same solutions, bit for bit;
* the oracle's own assembly (exact truncated SVDs of every admissible block)
  imported and factored on the device: the device H-LU and the oracle's H-LU
  of identical inputs agree within the parity bounds (factor ranks within +-2,
  ||PA - LU||_2/||A||_2 <= 10 eps against the exact matrix, solve residuals
  <= 2x the oracle's), so the comparison isolates the factorization from the
  assembly (ACA on the device, SVD in the oracle).
"""
import numpy as np
import pytest

from oracle import hmatrix as H
from paper_1911_07531_amd import hm, inputs
from tests.gpu_common import Problem, device_rhs, require_gpu, to_host

pytestmark = pytest.mark.gpu


def test_export_import_round_trip():
    require_gpu()
    p = Problem(4096, 64, 1e-6, max_rank=64, prec=hm.MIXED, oracle=False)
    _, _, _, bl = p.tree.tables()
    leaves = {b: p.A.leaf(b) for b in range(len(bl)) if bl[b, 2] != 0}
    B = hm.import_matrix(p.tree, p.opts, leaves)
    x = device_rhs(inputs.rhs(p.n, 5, seed=3))
    assert np.array_equal(to_host(p.A.matvec(x)), to_host(B.matvec(x)))
    b = inputs.rhs(p.n, 6, seed=4)
    x1, x2 = device_rhs(b), device_rhs(b)
    hm.LU(p.A, p.opts).solve(x1)
    hm.LU(B, p.opts).solve(x2)
    assert np.array_equal(to_host(x1), to_host(x2))


@pytest.mark.parametrize("geometry,n,leaf,eps", [("sphere", 2048, 32, 1e-6), ("cube", 2400, 32, 1e-4)])
def test_oracle_assembly_factored_on_device(geometry, n, leaf, eps):
    require_gpu()
    p = Problem(n, leaf, eps, geometry=geometry)
    leaves = {}
    for blk in H.leaf_blocks(p.oa.root):
        leaves[blk.index] = ("D", blk.D) if blk.kind == "D" else ("R", blk.U, blk.V)
    B = hm.import_matrix(p.tree, p.opts, leaves)
    f = hm.LU(B, p.opts)
    of = H.hlu(p.oa, lazy=True)
    gf = p.gpu_as_oracle(1, f.h)
    dense = p.dense_exact()
    err = H.lu_error_2norm(dense, gf, exact=True)
    oerr = H.lu_error_2norm(dense, of, exact=True)
    orank, grank = H.rank_table(of), H.rank_table(gf)
    d = np.array([grank[k] - orank[k] for k in orank])
    print(f"{geometry}: ||PA-LU||/||A|| device {err:.2e} oracle {oerr:.2e}; rank differences",
          np.unique(d, return_counts=True))
    assert err <= 10 * eps
    assert np.abs(d).max() <= 2
    b = inputs.rhs(p.n, 8, seed=1)
    xg = to_host(f.solve(device_rhs(b))[0])
    xo = H.solve(of, b)
    a_user = np.empty_like(dense)
    a_user[np.ix_(p.oa.perm, p.oa.perm)] = dense
    rg = np.linalg.norm(b - a_user @ xg, axis=0) / np.linalg.norm(b, axis=0)
    ro = np.linalg.norm(b - a_user @ xo, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(rg <= 2 * ro + 1e-12), (rg, ro)
