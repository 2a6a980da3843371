"""Pins for the oracle's inputs, cluster tree and block tree (CPU only).

Cluster tree: Def. 2.1 (sons partition the parent); block tree: Def. 2.2
(leaves tile I x I exactly once; leaf kinds as in Def. 2.3); standard
admissibility (Sec. 5.1) checked by brute force on the bounding boxes.
"""
import math

import numpy as np
import pytest

from oracle import hmatrix as H
from paper_1911_07531_amd import inputs


def test_fibonacci_lattice_closed_form():
    n = 1000
    p = inputs.sphere_points(n, seed=0, jitter=0.0)
    i = np.arange(n)
    z = 1.0 - (2 * i + 1) / n
    phi = i * (math.pi * (3 - math.sqrt(5)))
    r = np.sqrt(1 - z * z)
    ref = np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)
    assert np.allclose(p, ref, atol=1e-15)


def test_jitter_stays_on_sphere_and_near_lattice():
    n = 2048
    h = inputs.sphere_spacing(n)
    p = inputs.sphere_points(n, seed=0)
    q = inputs.sphere_points(n, seed=0, jitter=0.0)
    assert np.allclose(np.linalg.norm(p, axis=1), 1.0, atol=1e-14)
    assert np.max(np.linalg.norm(p - q, axis=1)) <= 0.1 * h * math.sqrt(2) + 1e-12
    assert np.array_equal(p, inputs.sphere_points(n, seed=0))
    assert not np.array_equal(p, inputs.sphere_points(n, seed=3))
    # the self term quoted for n = 2048: h = 0.078332, a_ii = 2.0318
    assert abs(h - 0.078332) < 1e-6
    assert abs(inputs.sphere_self_term(n) - 2.0318) < 1e-4


@pytest.mark.parametrize("n,leaf", [(2048, 32), (1000, 17), (64, 64), (65, 64)])
def test_cluster_tree_partitions(n, leaf):
    pts = inputs.sphere_points(n, seed=2)
    perm, cl = H.build_cluster_tree(pts, leaf)
    assert np.array_equal(np.sort(perm), np.arange(n))
    root = cl[0]
    assert (root.begin, root.end) == (0, n)
    for c in cl:
        own = pts[perm[c.begin:c.end]]
        assert np.array_equal(own.min(0), c.lo) and np.array_equal(own.max(0), c.hi)
        if c.sons:
            s0, s1 = c.sons
            assert s0.begin == c.begin and s0.end == s1.begin and s1.end == c.end
            assert s0.size > 0 and s1.size > 0
            assert s0.index == c.index + 1
            ax = int(np.argmax(c.hi - c.lo))
            mid = 0.5 * (c.lo[ax] + c.hi[ax])
            assert np.all(pts[perm[s0.begin:s0.end], ax] <= mid)
            assert np.all(pts[perm[s1.begin:s1.end], ax] > mid)
            # input order is kept inside each son
            assert np.all(np.diff(perm[s0.begin:s0.end]) > 0) or s0.sons
        else:
            assert c.size <= leaf or np.all(own == own[0])


def test_block_tree_tiles_once_and_kinds():
    n, leaf, eta = 2048, 32, 2.0
    pts = inputs.sphere_points(n, seed=0)
    perm, cl = H.build_cluster_tree(pts, leaf)
    root = H.build_block_tree(cl[0], eta)
    cover = np.zeros((n // leaf + 1, n // leaf + 1))
    count = np.zeros((n, n), dtype=np.int32)
    blocks = H.block_list(root)
    assert [b.index for b in blocks] == list(range(len(blocks)))
    for b in blocks:
        t, s = b.tau, b.sigma
        gap = np.maximum(0, np.maximum(s.lo - t.hi, t.lo - s.hi))
        dist = math.sqrt(float(gap @ gap))
        adm = dist > 0 and min(t.diam(), s.diam()) <= eta * dist
        if b.kind == "R":
            assert adm
        elif b.kind == "D":
            assert not adm and (t.is_leaf or s.is_leaf)
        else:
            assert not adm and not t.is_leaf and not s.is_leaf
        if b.kind != "S":
            count[t.begin:t.end, s.begin:s.end] += 1
    del cover
    assert np.all(count == 1)
    # diagonal blocks are never admissible
    for b in blocks:
        if b.tau is b.sigma:
            assert b.kind in "SD"


def test_admissibility_brute_force_boxes():
    rng = np.random.default_rng(0)
    for _ in range(200):
        lo1 = rng.uniform(-1, 1, 3)
        hi1 = lo1 + rng.uniform(0, 0.5, 3)
        lo2 = rng.uniform(-1, 1, 3)
        hi2 = lo2 + rng.uniform(0, 0.5, 3)
        c1 = H.Cluster(0, 0, 1, lo1, hi1, 0)
        c2 = H.Cluster(1, 0, 1, lo2, hi2, 0)
        # brute-force box distance by dense sampling of the two boxes' corners/faces
        g = np.linspace(0, 1, 9)
        grid = np.stack(np.meshgrid(g, g, g), -1).reshape(-1, 3)
        a = lo1 + grid * (hi1 - lo1)
        b = lo2 + grid * (hi2 - lo2)
        dmin = np.min(np.linalg.norm(a[:, None] - b[None], axis=2))
        gap = np.maximum(0, np.maximum(lo2 - hi1, lo1 - hi2))
        d = math.sqrt(float(gap @ gap))
        assert d <= dmin + 1e-12
        assert dmin - d <= 0.5 * max(np.max(hi1 - lo1), np.max(hi2 - lo2)) / 8 * math.sqrt(3) + 1e-12
        eta = 2.0
        expect = d > 0 and min(np.linalg.norm(hi1 - lo1), np.linalg.norm(hi2 - lo2)) <= eta * d
        assert H.admissible(c1, c2, eta) == expect


def test_line_mesh_midpoints():
    x = inputs.line_points(8)[:, 0]
    assert x.shape == (8,)
    assert np.array_equal(x, np.array([1, 3, 5, 7, 9, 11, 13, 15]) / 16.0)
    # mean of -log|t| / (2 pi) over a cell of width h around its midpoint, by quadrature
    from scipy.integrate import quad
    for n in (1, 10, 1000):
        h = 1.0 / n
        v = 2 * quad(lambda t: -math.log(t), 0.0, 0.5 * h)[0] / h / (2 * math.pi)
        assert abs(inputs.line_self_term(n) - v) <= 1e-12 * abs(v)


@pytest.mark.parametrize("levels,leaf", [(3, 32), (5, 32), (6, 16), (4, 64)])
def test_line_block_tree_closed_form(levels, leaf):
    """Uniform points on [0, 1] with eta = 2 (Sec. 5.1, the 1D model problem):
    bisection halves every cluster, so level l holds 2^l clusters of equal
    width w_l.  Neighbours (gap h, diameter w_l - h > 2h once a cluster has
    more than 3 points) are inadmissible; clusters one cluster apart (gap
    w_l + h) are admissible.  Hence the inadmissible blocks of each level form
    the tridiagonal 3 * 2^l - 2, every adjacent pair of parents gives 3
    admissible son blocks on each side (3 * 2^l - 6 low-rank leaves on level
    l >= 1), and the leaves of level L = log2(n / leaf) are dense."""
    n = leaf << levels
    perm, cl = H.build_cluster_tree(inputs.line_points(n), leaf)
    assert np.array_equal(perm, np.arange(n))
    root = H.build_block_tree(cl[0], 2.0)
    by_level = {}
    for b in H.block_list(root):
        lt, ls = b.tau.level, b.sigma.level
        assert lt == ls
        w = b.tau.size
        i, j = b.tau.begin // w, b.sigma.begin // w
        assert b.sigma.size == w == n >> lt
        if abs(i - j) <= 1:
            assert b.kind == ("D" if lt == levels else "S")
        else:
            assert b.kind == "R" and abs(i // 2 - j // 2) == 1
        by_level.setdefault(lt, {"S": 0, "D": 0, "R": 0})[b.kind] += 1
    for l in range(levels + 1):
        c = by_level[l]
        assert c["S" if l < levels else "D"] == 3 * 2 ** l - 2
        assert c["R"] == max(0, 3 * 2 ** l - 6)
