"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module produces *inputs only*: point clouds, the self-interaction value
placed on the diagonal, and right-hand sides.  It holds none of the H-matrix
arithmetic (no clustering, admissibility, kernel evaluation, compression or
factorisation), so both the CPU oracle and the device path may consume its
arrays without sharing any of the method's code.

The geometry stands in for the paper's model problem, the Laplace single layer
potential on the unit sphere (Sec. 5.1, "Model Problems"): a quasi-uniform
point set on the sphere replaces the piecewise-constant Galerkin mesh; the
paper notes that the entries do not matter for the block structure.

The second workload is the paper's one-dimensional model problem (Sec. 5.1,
the log-kernel integral equation on [0, 1]): n collocation points at the
midpoints of a uniform mesh of the unit interval.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))  # 2.39996...


def sphere_spacing(n: int) -> float:
    """Mean spacing h of n quasi-uniform points on the unit sphere: h = sqrt(4*pi/n)."""
    return math.sqrt(4.0 * math.pi / n)


def sphere_points(n: int, seed: int = 0, jitter: float = 0.1) -> np.ndarray:
    """n points on the unit sphere: Fibonacci lattice plus a seeded tangent jitter.

    z_i = 1 - (2i+1)/n, phi_i = i * golden angle; each point is moved by
    jitter*h*(u1 e1 + u2 e2) in its tangent plane (u ~ U[-1,1], PCG64(seed))
    and projected back onto the sphere.  Returns an (n, 3) float64 array in
    input order.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * GOLDEN_ANGLE
    p = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    h = sphere_spacing(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-1.0, 1.0, size=(n, 2))
    # tangent basis: e1 = normalize(axis x p) with axis = z unless p is near a pole
    axis = np.zeros_like(p)
    near_pole = np.abs(p[:, 2]) > 0.9
    axis[~near_pole, 2] = 1.0
    axis[near_pole, 0] = 1.0
    e1 = np.cross(axis, p)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(p, e1)
    q = p + jitter * h * (u[:, :1] * e1 + u[:, 1:] * e2)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return np.ascontiguousarray(q)


def sphere_self_term(n: int) -> float:
    """Diagonal value a_ii = 1/(4*pi*(h/2)) = 2/(4*pi*h): the kernel at half the mean spacing."""
    return 2.0 / (4.0 * math.pi * sphere_spacing(n))


def rhs(n: int, nrhs: int, seed: int = 1) -> np.ndarray:
    """N(0,1) right-hand sides, float64, column-major (n, nrhs) in the user's ordering."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.standard_normal((n, nrhs)))


def sphere_problem(n: int, seed: int = 0):
    """(points, diag) for the sphere single-layer workload of size n."""
    return sphere_points(n, seed), sphere_self_term(n)


def line_points(n: int) -> np.ndarray:
    """Midpoints x_i = (i + 1/2) / n of the n cells of a uniform mesh of [0, 1], as an (n, 1) array."""
    if n < 1:
        raise ValueError("n must be >= 1")
    return ((np.arange(n, dtype=np.float64) + 0.5) / n).reshape(n, 1)


def line_self_term(n: int) -> float:
    """Diagonal value for the kernel -log|x - y| / (2 pi) on the line: its mean over
    the cell [x_i - h/2, x_i + h/2] around the collocation point, h = 1/n,
    which is (1 - log(h/2)) / (2 pi)."""
    h = 1.0 / n
    return (1.0 - math.log(0.5 * h)) / (2.0 * math.pi)


def line_problem(n: int, seed: int = 0):
    """(points, diag) for the one-dimensional log-kernel workload of size n (no
    random draw: the mesh is uniform; ``seed`` is accepted for a common signature)."""
    return line_points(n), line_self_term(n)
