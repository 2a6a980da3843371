"""Pins for the oracle's kernel entries (CPU only): each kernel matrix the
parity tests take as exact is checked against a closed-form integral of the
same kernel over the same surface, not against a second copy of its formula.

* sphere, a_ij = 1/(4 pi |x_i - x_j|), a_ii = 2/(4 pi h): the single layer
  potential of the unit sphere has (1/4pi) int_S |x - y|^{-1} dS(y) = 1 for
  every x on S, so (4 pi / n) sum_j a_ij = 1 - c h with c near 0.15;
* unit-cube surface, same kernel: h^2 sum_j a_ij against the exact integral
  of 1/(4 pi |x - y|) over the six faces (closed-form antiderivative of
  1/r over a rectangle), error c h with c near -0.14;
* unit-square grid, a_ij = -log|x_i - x_j| / (2 pi), a_ii = -log(h/2)/(2 pi):
  h^2 sum_j a_ij against the exact integral of -log r / (2 pi) over the
  square (closed-form antiderivative of log r^2), error c h^2 with c near
  -0.057 (the self term's defect against the cell mean dominates).

The closed forms themselves are checked against scipy's dblquad.  Every pin
also shows that a plausible mistake (a factor 2, a missing 4 pi or 2 pi, a
wrong power of r, a wrong sign or a wrong self term) falls outside its band.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import hmatrix as H
from paper_1911_07531_amd import inputs


def _matrix(pts, diag, kernel):
    perm, cl = H.build_cluster_tree(pts, 64)
    return H.kernel_block(pts, perm, cl[0], cl[0], diag, kernel=kernel), pts[perm]


def _log_rect_antideriv(x, y):
    """F with d^2 F / dx dy = log(x^2 + y^2): x y log(x^2+y^2) - 3 x y + x^2 atan(y/x) + y^2 atan(x/y)."""
    r2 = x * x + y * y
    t = np.where(r2 > 0, x * y * np.log(np.where(r2 > 0, r2, 1.0)), 0.0) - 3.0 * x * y
    t = t + np.where(x != 0, x * x * np.arctan(y / np.where(x != 0, x, 1.0)), 0.0)
    t = t + np.where(y != 0, y * y * np.arctan(x / np.where(y != 0, y, 1.0)), 0.0)
    return t


def _log_rect(px, py):
    """int_[0,1]^2 log((x - px)^2 + (y - py)^2) dx dy."""
    a0, a1, b0, b1 = -px, 1.0 - px, -py, 1.0 - py
    F = _log_rect_antideriv
    return F(a1, b1) - F(a0, b1) - F(a1, b0) + F(a0, b0)


def _inv_rect_antideriv(u, v, z):
    """G with d^2 G / du dv = 1/sqrt(u^2 + v^2 + z^2): u log(v + r) + v log(u + r) - z atan(u v / (z r))."""
    r = np.sqrt(u * u + v * v + z * z)
    t = u * np.log(np.where(v + r > 0, v + r, 1.0)) + v * np.log(np.where(u + r > 0, u + r, 1.0))
    zr = z * r
    return t - np.where(zr != 0, z * np.arctan(u * v / np.where(zr != 0, zr, 1.0)), 0.0)


def _inv_rect(pu, pv, pz):
    """int_[0,1]^2 1/sqrt((u - pu)^2 + (v - pv)^2 + pz^2) du dv."""
    a0, a1, b0, b1, z = -pu, 1.0 - pu, -pv, 1.0 - pv, np.abs(pz)
    G = _inv_rect_antideriv
    return G(a1, b1, z) - G(a0, b1, z) - G(a1, b0, z) + G(a0, b0, z)


def _cube_potential(p):
    """(1/4pi) int over the unit cube's surface of 1/|x - y| dS(y), for points p (m, 3)."""
    tot = np.zeros(len(p))
    for axis in range(3):
        free = [d for d in range(3) if d != axis]
        for val in (0.0, 1.0):
            tot += _inv_rect(p[:, free[0]], p[:, free[1]], p[:, axis] - val)
    return tot / (4.0 * math.pi)


def test_closed_forms_against_quadrature():
    for px, py in [(0.3, 0.7), (0.05, 0.5), (0.9, 0.1)]:
        num, _ = integrate.dblquad(lambda y, x: math.log((x - px) ** 2 + (y - py) ** 2), 0, 1, 0, 1, epsabs=1e-11)
        assert abs(float(_log_rect(np.array(px), np.array(py))) - num) <= 1e-8
    for pu, pv, pz in [(0.3, 0.7, 0.5), (0.5, 0.5, 1.0), (0.2, 0.9, 1e-4), (0.3, 0.6, 0.0)]:
        num, _ = integrate.dblquad(lambda v, u: 1.0 / math.sqrt((u - pu) ** 2 + (v - pv) ** 2 + pz ** 2),
                                   0, 1, 0, 1, epsabs=1e-10)
        assert abs(float(_inv_rect(np.array(pu), np.array(pv), np.array(pz))) - num) <= 1e-8


@pytest.mark.parametrize("n", [512, 2048, 8192])
def test_sphere_single_layer_row_sums(n):
    """(1 - (4 pi / n) sum_j a_ij) / h: mean in [0.14, 0.16], every row in [0.09, 0.20]."""
    pts, diag = inputs.sphere_problem(n, 0)
    h = inputs.sphere_spacing(n)
    perm, cl = H.build_cluster_tree(pts, 64)
    rs = np.zeros(n)
    for r0 in range(0, n, 1024):  # row chunks keep the distance array small
        r1 = min(n, r0 + 1024)
        rs[r0:r1] = H.kernel_block(pts, perm, cl[0], cl[0], diag, r=(r0, r1)).sum(axis=1)

    def c(rowsum):
        return (1.0 - 4.0 * math.pi / n * rowsum) / h

    def ok(rowsum):
        v = c(rowsum)
        return 0.14 <= v.mean() <= 0.16 and v.min() >= 0.09 and v.max() <= 0.20

    assert ok(rs), (c(rs).mean(), c(rs).min(), c(rs).max())
    # planted mistakes, computed from the same entries
    assert not ok(2.0 * rs)                         # kernel 1/(2 pi r)
    assert not ok(4.0 * math.pi * rs)               # kernel 1/r (4 pi dropped)
    assert not ok(rs - diag + diag / 2.0)           # self term 1/(4 pi h)
    assert not ok(rs - diag)                        # no self term
    if n <= 2048:                                   # kernel 1/(4 pi r^2)
        a = H.kernel_block(pts, perm, cl[0], cl[0], diag)
        off = a.copy()
        np.fill_diagonal(off, 0.0)
        d = np.where(off > 0, 1.0 / (4.0 * math.pi * np.where(off > 0, off, 1.0)), 0.0)
        sq = np.where(d > 0, 1.0 / (4.0 * math.pi * np.where(d > 0, d, 1.0) ** 2), 0.0).sum(axis=1) + diag
        assert not ok(sq)


@pytest.mark.parametrize("n", [600, 2400, 9600])
def test_cube_surface_row_sums(n):
    """(h^2 sum_j a_ij - exact surface integral) / h: mean in [-0.155, -0.13], rows in [-0.20, -0.08]."""
    pts, diag = inputs.cube_problem(n, 0)
    s = inputs.cube_side(n)
    h = 1.0 / s
    assert len(pts) == 6 * s * s
    a, p = _matrix(pts, diag, "laplace3d")
    ex = _cube_potential(p)
    rs = a.sum(axis=1)

    def ok(rowsum):
        v = (h * h * rowsum - ex) / h
        return -0.155 <= v.mean() <= -0.13 and v.min() >= -0.20 and v.max() <= -0.08

    assert ok(rs), ((h * h * rs - ex) / h).mean()
    assert not ok(2.0 * rs)
    assert not ok(4.0 * math.pi * rs)
    assert not ok(rs - diag / 2.0)
    assert not ok(rs - diag)


@pytest.mark.parametrize("n", [256, 1024, 4096])
def test_grid_log_kernel_row_sums(n):
    """(h^2 sum_j a_ij - exact integral) / h^2 in [-0.060, -0.054] for every row."""
    pts, diag = inputs.grid_problem(n)
    s = inputs.grid_side(n)
    h = 1.0 / s
    assert len(pts) == s * s
    a, p = _matrix(pts, diag, "log2d")
    ex = -_log_rect(p[:, 0], p[:, 1]) / (4.0 * math.pi)  # -log r / (2 pi) = -log(r^2) / (4 pi)
    rs = a.sum(axis=1)

    def ok(rowsum):
        v = (h * h * rowsum - ex) / (h * h)
        return v.min() >= -0.060 and v.max() <= -0.054

    assert ok(rs), ((h * h * rs - ex) / (h * h)).min()
    assert not ok(-rs)                                          # log r / (2 pi)
    assert not ok(2.0 * math.pi * rs)                           # 1/(2 pi) dropped
    assert not ok(rs - diag + (-math.log(h) / (2 * math.pi)))   # self term -log(h)/(2 pi)
    assert not ok(rs - diag)


def test_cube_and_grid_geometry():
    pts = inputs.cube_points(6 * 20 * 20, seed=3)
    on = (np.isclose(pts, 0.0) | np.isclose(pts, 1.0))
    assert np.all(on.sum(axis=1) == 1)            # every point on exactly one face
    face = np.argmax(on, axis=1) * 2 + np.isclose(pts[np.arange(len(pts)), np.argmax(on, axis=1)], 1.0)
    assert np.all(np.bincount(face, minlength=6) == 400)
    assert pts.min() >= 0.0 and pts.max() <= 1.0
    g = inputs.grid_points(1000)
    s = inputs.grid_side(1000)
    assert len(g) == s * s and np.allclose(np.sort(np.unique(g[:, 0])), (np.arange(s) + 0.5) / s)


def test_batched_instances_recipe():
    ins = inputs.batched_instances()
    assert len(ins) == 64
    ns = np.array([i["n"] for i in ins])
    assert ns.min() >= 4000 and ns.max() <= 66000
    assert {i["leaf"] for i in ins} == {32, 64, 128}
    assert [i["geometry"] for i in ins[:3]] == ["sphere", "cube", "grid"]
    assert ins == inputs.batched_instances()  # seeded
    # log-uniform sizes: the median of exp(U[ln a, ln b]) is sqrt(a b) = 16384
    assert 9000 <= np.median(ns) <= 30000
