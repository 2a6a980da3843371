"""Matrix-free checks against the exact kernel matrix for large n (test
infrastructure, GPU tests only).

The exact kernel matrix A (a_ij = k(|x_i - x_j|), a_ii = diag) is applied in
row chunks with plain torch FP64 operations on the device; the H-LU factors
are applied from their exported leaves with NumPy.  Neither side uses the
library's kernels or the oracle, so these give independent measurements of
||b - A x|| / ||b|| and of ||P A - L U||_2 / ||A||_2 (power iteration).
"""
from __future__ import annotations

import math

import numpy as np


def exact_apply(pts, diag, x, kernel="laplace3d", chunk=2048):
    """A x for the exact kernel matrix in the points' own ordering; x (n, k) float64 NumPy."""
    import torch
    dev = torch.device("cuda" if torch.cuda.is_available() else "cpu")
    P = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).to(dev)
    if P.shape[1] < 3:
        P = torch.nn.functional.pad(P, (0, 3 - P.shape[1]))
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)
    n = P.shape[0]
    out = torch.empty((n, X.shape[1]), dtype=torch.float64, device=dev)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        d = P[r0:r1, None, :] - P[None, :, :]
        r = torch.sqrt((d * d).sum(-1))
        del d
        if kernel == "laplace3d":
            k = 1.0 / (4.0 * math.pi * r)
        else:
            k = -torch.log(r) / (2.0 * math.pi)
        idx = torch.arange(r0, r1, device=dev)
        k[idx - r0, idx] = diag
        out[r0:r1] = k @ X
        del k, r
    return out.cpu().numpy()


def exact_residuals(pts, diag, b, x, kernel="laplace3d"):
    """||b - A x||_2 / ||b||_2 per column (user ordering)."""
    r = b - exact_apply(pts, diag, x, kernel)
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


class Factors:
    """The exported H-LU factors as operators in permuted ordering.

    P A = Lp U with the leaf-local pivots: diagonal leaves hold the packed
    LU (unit lower L, upper U) and their row permutation; off-diagonal lower
    blocks are stored unpermuted, so Lp = P_bd L_off + L_diag."""

    def __init__(self, lu, tree):
        from paper_1911_07531_amd import hm
        _, cl, _, bl = tree.tables()
        self.n = int(cl[0, 1] - cl[0, 0])
        self.lower, self.upper, self.diag = [], [], []
        self.p = np.arange(self.n)
        for b in range(len(bl)):
            tau, sigma, kind = bl[b, 0], bl[b, 1], bl[b, 2]
            if kind == 0:
                continue
            r0, r1, c0, c1 = int(cl[tau, 0]), int(cl[tau, 1]), int(cl[sigma, 0]), int(cl[sigma, 1])
            leaf = hm.export_leaf(lu.h, 1, b, tree)
            if tau == sigma:
                _, d, piv = leaf
                local = np.arange(r1 - r0)
                for i, pi in enumerate(piv):  # LAPACK interchanges, in order
                    local[i], local[pi] = local[pi], local[i]
                self.p[r0:r1] = r0 + local
                self.diag.append((r0, r1, np.tril(d, -1) + np.eye(r1 - r0), np.triu(d)))
            else:
                op = ("D", leaf[1]) if leaf[0] == "D" else ("R", leaf[1], leaf[2])
                (self.lower if r0 >= c1 else self.upper).append((r0, r1, c0, c1, op))

    @staticmethod
    def _mul(op, x, t=False):
        if op[0] == "D":
            return (op[1].T if t else op[1]) @ x
        u, v = op[1], op[2]
        return u @ (v.T @ x) if not t else v @ (u.T @ x)

    def lu_apply(self, x):
        """Lp U x (permuted ordering)."""
        y = np.zeros_like(x)
        for r0, r1, _, u in self.diag:
            y[r0:r1] += u @ x[r0:r1]
        for r0, r1, c0, c1, op in self.upper:
            y[r0:r1] += self._mul(op, x[c0:c1])
        z = np.zeros_like(x)
        for r0, r1, c0, c1, op in self.lower:
            z[r0:r1] += self._mul(op, y[c0:c1])
        out = z[self.p]  # P_bd L_off y
        for r0, r1, l, _ in self.diag:
            out[r0:r1] += l @ y[r0:r1]
        return out

    def lu_apply_t(self, w):
        """(Lp U)^T w = U^T (L_off^T P_bd^T w + L_diag^T w)."""
        pt = np.zeros_like(w)
        pt[self.p] = w  # P_bd^T w
        y = np.zeros_like(w)
        for r0, r1, c0, c1, op in self.lower:
            y[c0:c1] += self._mul(op, pt[r0:r1], t=True)
        for r0, r1, l, _ in self.diag:
            y[r0:r1] += l.T @ w[r0:r1]
        out = np.zeros_like(w)
        for r0, r1, _, u in self.diag:
            out[r0:r1] += u.T @ y[r0:r1]
        for r0, r1, c0, c1, op in self.upper:
            out[c0:c1] += self._mul(op, y[r0:r1], t=True)
        return out


def lu_error_estimate(pts_perm, diag, factors, kernel="laplace3d", iters=40, seed=5):
    """||P A - Lp U||_2 / ||A||_2 by power iteration on E^T E and on A^T A
    (A symmetric), A the exact kernel matrix in permuted ordering."""
    rng = np.random.default_rng(seed)
    n = factors.n

    def apply_e(v):
        av = exact_apply(pts_perm, diag, v, kernel)
        return av[factors.p] - factors.lu_apply(v)

    def apply_et(w):
        pt = np.zeros_like(w)
        pt[factors.p] = w
        return exact_apply(pts_perm, diag, pt, kernel) - factors.lu_apply_t(w)

    def power(f, ft):
        v = rng.standard_normal((n, 1))
        v /= np.linalg.norm(v)
        lam = 0.0
        for _ in range(iters):
            w = ft(f(v))
            new = float(np.linalg.norm(w))
            if new == 0.0:
                return 0.0
            v = w / new
            done = abs(new - lam) <= 1e-4 * new
            lam = new
            if done:
                break
        return math.sqrt(lam)

    ea = power(apply_e, apply_et)
    na = power(lambda v: exact_apply(pts_perm, diag, v, kernel), lambda v: exact_apply(pts_perm, diag, v, kernel))
    return ea / na
