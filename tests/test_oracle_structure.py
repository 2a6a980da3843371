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
