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


# ---------------------------------------------------------------------------
# Further geometries of the batched workload: the unit-cube surface with the
# 3D single layer kernel and a uniform grid on the unit square with the 2D
# logarithmic kernel.  The self term is the kernel at half the mean spacing,
# as for the sphere.
# ---------------------------------------------------------------------------
def cube_side(n: int) -> int:
    """Grid side s of the cube-surface point set nearest to n points: n is rounded to 6 s^2."""
    return max(1, int(round(math.sqrt(n / 6.0))))


def cube_points(n: int, seed: int = 0, jitter: float = 0.1) -> np.ndarray:
    """6 s^2 points on the surface of the unit cube [0, 1]^3, s = cube_side(n).

    Each face carries the s x s cell centres of a uniform grid (spacing
    h = 1/s), moved inside the face by jitter*h*(u1, u2), u ~ U[-1, 1]
    (PCG64(seed)).  Faces in the order x=0, x=1, y=0, y=1, z=0, z=1; inside a
    face row-major over its two free coordinates.  Returns (6 s^2, 3) float64.
    """
    s = cube_side(n)
    h = 1.0 / s
    g = (np.arange(s, dtype=np.float64) + 0.5) * h
    a, b = np.meshgrid(g, g, indexing="ij")
    a, b = a.ravel(), b.ravel()
    rng = np.random.Generator(np.random.PCG64(seed))
    faces = []
    for axis in range(3):
        free = [d for d in range(3) if d != axis]
        for val in (0.0, 1.0):
            u = rng.uniform(-1.0, 1.0, size=(s * s, 2))
            p = np.empty((s * s, 3))
            p[:, axis] = val
            p[:, free[0]] = a + jitter * h * u[:, 0]
            p[:, free[1]] = b + jitter * h * u[:, 1]
            faces.append(p)
    return np.ascontiguousarray(np.concatenate(faces))


def cube_self_term(n: int) -> float:
    """a_ii = 2 / (4 pi h) with h = 1/s = sqrt(6 / n_actual): the kernel 1/(4 pi r) at r = h/2."""
    return 2.0 / (4.0 * math.pi * (1.0 / cube_side(n)))


def grid_side(n: int) -> int:
    """Side s of the square grid nearest to n points: n is rounded to s^2."""
    return max(1, int(round(math.sqrt(n))))


def grid_points(n: int) -> np.ndarray:
    """The s x s cell centres ((i + 1/2)/s, (j + 1/2)/s) of the unit square, s = grid_side(n),
    row-major in i; returned as an (s^2, 2) float64 array (no random draw)."""
    s = grid_side(n)
    g = (np.arange(s, dtype=np.float64) + 0.5) / s
    a, b = np.meshgrid(g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([a.ravel(), b.ravel()], axis=1))


def grid_self_term(n: int) -> float:
    """a_ii = -log(h/2) / (2 pi) with h = 1/s: the kernel -log r / (2 pi) at r = h/2."""
    h = 1.0 / grid_side(n)
    return -math.log(0.5 * h) / (2.0 * math.pi)


def cube_problem(n: int, seed: int = 0):
    """(points, diag) for the cube-surface single-layer workload (about n points)."""
    return cube_points(n, seed), cube_self_term(n)


def grid_problem(n: int, seed: int = 0):
    """(points, diag) for the 2D logarithmic-kernel grid workload (about n points; no random draw)."""
    return grid_points(n), grid_self_term(n)


GEOMETRIES = ("sphere", "cube", "grid")
# the kernel each geometry is assembled with: "laplace3d" = 1/(4 pi r), "log2d" = -log(r)/(2 pi)
GEOMETRY_KERNEL = {"sphere": "laplace3d", "cube": "laplace3d", "grid": "log2d", "line": "log2d"}


def problem(geometry: str, n: int, seed: int = 0):
    """(points, diag) of a named geometry: sphere, cube, grid or line."""
    if geometry == "sphere":
        return sphere_problem(n, seed)
    if geometry == "cube":
        return cube_problem(n, seed)
    if geometry == "grid":
        return grid_problem(n, seed)
    if geometry == "line":
        return line_problem(n, seed)
    raise ValueError(f"unknown geometry {geometry!r}")


def batched_instances(count: int = 64, n_lo: int = 4096, n_hi: int = 65536, seed0: int = 100):
    """The batched workload: instance i draws, from PCG64(seed0 + i), its size
    n = round(exp(U[ln n_lo, ln n_hi])) and its leaf size from {32, 64, 128};
    its geometry is GEOMETRIES[i mod 3] (the cube and grid round n to their
    lattices).  Returns a list of dicts (geometry, kernel, n, leaf, seed)."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        leaf = int((32, 64, 128)[int(rng.integers(0, 3))])
        geo = GEOMETRIES[i % 3]
        if geo == "cube":
            n = 6 * cube_side(n) ** 2
        elif geo == "grid":
            n = grid_side(n) ** 2
        out.append(dict(geometry=geo, kernel=GEOMETRY_KERNEL[geo], n=n, leaf=leaf, seed=seed0 + i))
    return out
