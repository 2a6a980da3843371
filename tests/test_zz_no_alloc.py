"""h_solve_noalloc (the solve for callers that cannot allocate) against
h_solve through the C-ABI: two calls in a row, the second on a smaller
problem with fewer right-hand sides, each bit-identical to h_solve (same
kernels, same 64-column chunks at these sizes), with and without refinement;
and a size where the fixed scratch holds fewer than 64 columns of refinement
vectors (n = 65536: chunks of 31 columns), which must still converge to the
same solution (each column's result does not depend on the other columns)."""
import numpy as np
import pytest

from paper_1911_07531_amd import hm, inputs
from tests.gpu_common import Problem, device_rhs, require_gpu, to_host

pytestmark = pytest.mark.gpu


def _both(f, A, b):
    xr = device_rhs(b)
    _, it_r, rel_r = f.solve(xr, refine_with=A, rtol=1e-10, max_iter=30)
    xn = device_rhs(b)
    _, it_n, rel_n = f.solve_noalloc(xn, refine_with=A, rtol=1e-10, max_iter=30)
    return to_host(xr), it_r, rel_r, to_host(xn), it_n, rel_n


def test_noalloc_solve_equals_solve_two_calls():
    require_gpu()
    for n, nrhs in ((4096, 70), (2048, 7)):
        print(f"h_solve_noalloc vs h_solve: n={n} nrhs={nrhs}", flush=True)
        p = Problem(n, 64, 1e-6, max_rank=64, prec=hm.MIXED, oracle=False)
        f = hm.LU(p.A, p.opts)
        b = inputs.rhs(p.n, nrhs, seed=13)
        xr, it_r, rel_r, xn, it_n, rel_n = _both(f, p.A, b)
        assert np.array_equal(xr, xn)
        assert np.array_equal(rel_r, rel_n) and np.all(rel_n <= 1e-10)
        assert it_n == int(it_r.max())
        # without refinement: the plain substitution
        x1, x2 = device_rhs(b), device_rhs(b)
        f.solve(x1)
        _, it0, rel0 = f.solve_noalloc(x2)
        assert np.array_equal(to_host(x1), to_host(x2)) and it0 == 0 and np.all(np.isnan(rel0))


def test_noalloc_solve_chunked_refinement():
    require_gpu()
    n, nrhs = 65536, 40
    print(f"h_solve_noalloc chunked refinement: n={n} nrhs={nrhs}", flush=True)
    p = Problem(n, 64, 1e-4, max_rank=64, prec=hm.MIXED, oracle=False)
    f = hm.LU(p.A, p.opts)
    b = inputs.rhs(p.n, nrhs, seed=17)
    xr, _, rel_r, xn, _, rel_n = _both(f, p.A, b)
    assert np.all(rel_r <= 1e-10) and np.all(rel_n <= 1e-10)
    assert np.abs(xr - xn).max() <= 1e-9 * np.abs(xr).max()
