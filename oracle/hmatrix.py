"""FP64 CPU oracle: cluster tree, block tree, compression and recursive H-LU.

TEST INFRASTRUCTURE ONLY.  Nothing in the device library imports, links or
calls this module; only tests/, the smoke check and the benchmark's CPU
baseline do.  It is deliberately plain: recursive Python over NumPy arrays,
float64 throughout, no blocking, fusion or reordering beyond what the
definitions and algorithms state.

Paper: Boerm, Christophersen, Kriemann, "Semi-Automatic Task Graph Construction
for H-Matrix Arithmetic" (arXiv 1911.07531).

  * cluster tree ........ Def. 2.1 (binary, Sec. 2.2); geometric bisection
  * block tree .......... Def. 2.2 with standard admissibility (Sec. 5.1)
  * H-matrix set ........ Def. 2.3 (dense leaves on leaf clusters, low rank
                          factors U V^T on admissible leaves)
  * hmul ................ Algorithm 1 (+ the leaf-case products below)
  * hlu ................. Algorithm 2
  * htrsl ............... Algorithm 3; htrsu is its mirror (Sec. 2.2)
  * truncation .......... Sec. 2.3: the rank of C + alpha A B is reduced to
                          precision eps after every update

Readings where the paper is silent (each one is listed in the design notes):
  R1  pivoting is leaf-local partial pivoting (LAPACK getrf convention, unit
      lower L, first maximum wins); off-diagonal L blocks are stored
      unpermuted, so P A = Lp U with Lp = P_bd L_off + L_diag.
  R2  truncation keeps sigma_i > eps * sigma_1 of the block (strict), then caps
      at max_rank (0 = no cap) and at min(m, n); Sigma is kept in U.
  R3  leaf-case products ("special routines" after Algorithm 1) are formed
      exactly as low-rank terms; a low-rank C whose A and B are both
      structured receives the terms of the recursive (i, j, l) expansion one
      by one, each with its own truncation; a structured C receives a
      low-rank product leaf by leaf (depth first), each leaf truncated.
  R4  htrsu recursion order mirrors Algorithm 3: both solves with U00, both
      updates with U01, both solves with U11.
  R5  adm(t, s) = dist(t, s) > 0 and min(diam t, diam s) <= eta * dist(t, s)
      with axis-aligned bounding boxes.
  R6  collected updates (hlu(..., lazy=True)): following the accumulator
      arithmetic of Sec. 2.3 (hmul as add_upd followed by apply_upd), each
      top-level hmul call collects the exact low-rank terms it produces for
      every low-rank leaf and applies them in one truncation,
      C <- T_eps(C + sum of terms), when it returns.
  R8  hlu_accumulated follows the accumulator H-LU of Algorithms 4-8: an
      accumulator per block, low-rank (truncated on every addition, same
      accuracy and cap as the blocks) or dense for dense leaves, pending
      structured products split one level at a time by shift_upd, and updates
      added into a leaf only right before it is factorized or solved.  A
      product that evaluates to several low-rank terms (the special routines
      after Algorithm 1) is added to the accumulator term by term.
  R7  the one-dimensional model problem of Sec. 5.1 uses the kernel
      -log|x - y| / (2 pi), a negative multiple of the printed log|x - y|
      (same block ranks, same pivot order in exact arithmetic, a positive
      definite operator on [0, 1]); the diagonal holds the kernel's mean over
      the collocation cell.

Parity is pinned in tests/test_oracle_*.py against: scipy's getrf on the same
leaf block, Eckart-Young for compression, brute-force tiling of the block
tree, the dense leaf-pivoted block LU at eps = 0, the 10*eps bound on tiny n,
and the dense product for matvec and solve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

__all__ = [
    "Cluster", "Block", "HMatrix", "SingularError",
    "build_cluster_tree", "build_block_tree", "admissible",
    "kernel_block", "assemble", "hlu", "solve", "matvec", "refine",
    "getrf_leaf", "apply_pivots", "truncated_add", "truncation_rank",
    "densify", "lu_dense_factors", "lu_error_2norm", "block_list",
    "leaf_blocks", "rank_table",
]

FOUR_PI = 4.0 * math.pi


class SingularError(ArithmeticError):
    """Exact zero pivot in a diagonal leaf; ``row`` is the permuted global row."""

    def __init__(self, row: int):
        super().__init__(f"zero pivot at row {row}")
        self.row = row


# ---------------------------------------------------------------------------
# Def. 2.1: cluster tree by geometric bisection
# ---------------------------------------------------------------------------
@dataclass
class Cluster:
    index: int
    begin: int
    end: int
    lo: np.ndarray
    hi: np.ndarray
    level: int
    sons: tuple = ()

    @property
    def size(self) -> int:
        return self.end - self.begin

    @property
    def is_leaf(self) -> bool:
        return not self.sons

    def diam(self) -> float:
        return math.sqrt(float(np.sum((self.hi - self.lo) ** 2)))


def build_cluster_tree(points: np.ndarray, leaf: int):
    """Binary cluster tree (Def. 2.1) by bisection of the longest bounding-box axis.

    Each cluster has the tight bounding box of its points; a cluster with more
    than ``leaf`` points is split at the midpoint of its longest axis (ties go
    to the lowest axis index); points with coordinate <= midpoint go to son 0,
    keeping input order in each son; the split is abandoned if a side would be
    empty.  Clusters are numbered in depth-first pre-order and the leaves in
    depth-first order define the permutation, so every cluster is a contiguous
    range [begin, end) of permuted indices.

    Returns (perm, clusters) with perm[k] = original index of permuted index k.
    """
    points = np.asarray(points, dtype=np.float64)
    perm: list = []
    clusters: list = []

    def rec(idx: np.ndarray, level: int) -> Cluster:
        pts = points[idx]
        c = Cluster(len(clusters), len(perm), -1, pts.min(axis=0), pts.max(axis=0), level)
        clusters.append(c)
        if len(idx) > leaf:
            ext = c.hi - c.lo
            axis = int(np.argmax(ext))
            mid = 0.5 * (c.lo[axis] + c.hi[axis])
            left = pts[:, axis] <= mid
            if left.any() and (~left).any():
                s0 = rec(idx[left], level + 1)
                s1 = rec(idx[~left], level + 1)
                c.sons = (s0, s1)
        if not c.sons:
            perm.extend(int(i) for i in idx)
        c.end = len(perm)
        return c

    rec(np.arange(len(points)), 0)
    return np.asarray(perm, dtype=np.int64), clusters


def admissible(t: Cluster, s: Cluster, eta: float) -> bool:
    """Standard admissibility (Sec. 5.1): min(diam t, diam s) <= eta * dist(t, s), dist > 0."""
    gap = np.maximum(0.0, np.maximum(s.lo - t.hi, t.lo - s.hi))
    dist = math.sqrt(float(np.sum(gap * gap)))
    if dist <= 0.0:
        return False
    return min(t.diam(), s.diam()) <= eta * dist


# ---------------------------------------------------------------------------
# Def. 2.2 / 2.3: block tree and H-matrix leaves
# ---------------------------------------------------------------------------
@dataclass
class Block:
    index: int
    tau: Cluster
    sigma: Cluster
    kind: str  # 'S' structured, 'D' dense leaf, 'R' low-rank leaf
    sons: list = field(default_factory=list)  # [[b00, b01], [b10, b11]]
    D: np.ndarray | None = None
    U: np.ndarray | None = None
    V: np.ndarray | None = None
    piv: np.ndarray | None = None  # diagonal dense leaves after hlu
    pending: list = field(default_factory=list)  # collected updates (Reading R6)

    @property
    def rows(self) -> int:
        return self.tau.size

    @property
    def cols(self) -> int:
        return self.sigma.size

    @property
    def rank(self) -> int:
        return 0 if self.U is None else self.U.shape[1]


def build_block_tree(root: Cluster, eta: float) -> Block:
    """Block tree (Def. 2.2): a block is a leaf if admissible or if a cluster is a leaf.

    Blocks are numbered in depth-first pre-order with sons (0,0),(0,1),(1,0),(1,1).
    """
    counter = [0]

    def rec(t: Cluster, s: Cluster) -> Block:
        b = Block(counter[0], t, s, "S")
        counter[0] += 1
        if admissible(t, s, eta):
            b.kind = "R"
        elif t.is_leaf or s.is_leaf:
            b.kind = "D"
        else:
            b.sons = [[None, None], [None, None]]
            for i in range(2):
                for j in range(2):
                    b.sons[i][j] = rec(t.sons[i], s.sons[j])
        return b

    return rec(root, root)


def block_list(b: Block) -> list:
    """All blocks in pre-order."""
    out = [b]
    if b.kind == "S":
        for i in range(2):
            for j in range(2):
                out.extend(block_list(b.sons[i][j]))
    return out


def leaf_blocks(b: Block) -> list:
    return [x for x in block_list(b) if x.kind != "S"]


@dataclass
class HMatrix:
    root: Block
    perm: np.ndarray
    clusters: list
    n: int
    eps: float
    max_rank: int


# ---------------------------------------------------------------------------
# Entries and compression (Sec. 2.1: admissible blocks approximable to eps)
# ---------------------------------------------------------------------------
KERNELS = ("laplace3d", "log2d")


def kernel_block(points, perm, rows: Cluster, cols: Cluster, diag: float, r=None, c=None,
                 kernel: str = "laplace3d") -> np.ndarray:
    """Entries a_ij = k(|x_i - x_j|), a_ii = diag, for permuted index ranges.

    kernel "laplace3d": k(d) = 1/(4 pi d), the single layer potential of the
    sphere problem (Sec. 5.1); "log2d": k(d) = -log(d)/(2 pi), the kernel of
    the one-dimensional model problem (Sec. 5.1) with the sign and scale of
    the 2D Laplace fundamental solution (Reading R7).
    """
    if kernel not in KERNELS:
        raise ValueError(f"unknown kernel {kernel!r}")
    ri = perm[rows.begin:rows.end] if r is None else perm[r[0]:r[1]]
    ci = perm[cols.begin:cols.end] if c is None else perm[c[0]:c[1]]
    x = points[ri]
    y = points[ci]
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(axis=2))
    same = ri[:, None] == ci[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        if kernel == "laplace3d":
            a = 1.0 / (FOUR_PI * d)
        else:
            a = -np.log(d) / (2.0 * math.pi)
    a[same] = diag
    return a


def _svd(a: np.ndarray, full_matrices: bool = True):
    """The SVD a = W diag(s) Z^T of a finite matrix.  LAPACK's divide-and-conquer
    driver (numpy's default) can report non-convergence on rare inputs; the
    decomposition is then taken from the QR-iteration driver, which computes
    the same factorization."""
    if not np.all(np.isfinite(a)):
        raise ValueError("non-finite entries in a matrix to be decomposed")
    try:
        return np.linalg.svd(a, full_matrices=full_matrices)
    except np.linalg.LinAlgError:
        return sla.svd(a, full_matrices=full_matrices, lapack_driver="gesvd")


def truncation_rank(s: np.ndarray, eps: float, max_rank: int, limit: int) -> int:
    """Reading R2: count sigma_i > eps*sigma_1, then cap by max_rank (0 = none) and limit."""
    if s.size == 0 or s[0] <= 0.0:
        return 0
    k = int(np.count_nonzero(s > eps * s[0]))
    if max_rank > 0:
        k = min(k, max_rank)
    return min(k, limit)


def _compress_dense(a: np.ndarray, eps: float, max_rank: int):
    w, s, zt = _svd(a, full_matrices=False)
    k = truncation_rank(s, eps, max_rank, min(a.shape))
    return w[:, :k] * s[:k], zt[:k].T.copy()


def _compress_randomized(apply, apply_t, m, n, eps, max_rank, seed):
    """Randomised truncated SVD (range finder with 2 power iterations, oversampling 10).

    apply(X) = A X, apply_t(Y) = A^T Y.  The sample width doubles until the
    smallest sampled singular value drops below eps*sigma_1/10.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ell = 32
    while True:
        ell = min(ell, min(m, n))
        y = apply(rng.standard_normal((n, ell)))
        q, _ = np.linalg.qr(y)
        for _ in range(2):
            z, _ = np.linalg.qr(apply_t(q))
            q, _ = np.linalg.qr(apply(z))
        bt = apply_t(q)  # n x ell = (Q^T A)^T
        zb, s, wt = _svd(bt, full_matrices=False)
        if ell >= min(m, n) or s[-1] <= eps * s[0] / 10.0:
            k = truncation_rank(s, eps, max_rank, min(m, n))
            u = q @ (wt.T[:, :k] * s[:k])
            v = zb[:, :k].copy()
            return u, v
        ell *= 2


RANDOMIZED_MIN_SIDE = 2048


def assemble(points, perm, clusters, root: Block, diag: float, eps: float, max_rank: int = 0,
             seed: int = 0, kernel: str = "laplace3d") -> HMatrix:
    """Fill the leaves of the block tree (Def. 2.3).

    Dense leaves hold the entries; admissible leaves hold the truncated SVD of
    the exact block (Reading R2), computed exactly when min(m, n) <= 2048 and
    by the randomised range finder above that.
    """
    points = np.asarray(points, dtype=np.float64)
    for b in leaf_blocks(root):
        if b.kind == "D":
            b.D = kernel_block(points, perm, b.tau, b.sigma, diag, kernel=kernel)
        else:
            m, n = b.rows, b.cols
            if min(m, n) <= RANDOMIZED_MIN_SIDE:
                b.U, b.V = _compress_dense(kernel_block(points, perm, b.tau, b.sigma, diag, kernel=kernel), eps,
                                           max_rank)
            else:
                chunk = 4096

                def apply(x, b=b):
                    out = np.zeros((b.rows, x.shape[1]))
                    for c0 in range(0, b.cols, chunk):
                        c1 = min(b.cols, c0 + chunk)
                        blk = kernel_block(points, perm, b.tau, b.sigma, diag,
                                           c=(b.sigma.begin + c0, b.sigma.begin + c1), kernel=kernel)
                        out += blk @ x[c0:c1]
                    return out

                def apply_t(y, b=b):
                    out = np.zeros((b.cols, y.shape[1]))
                    for c0 in range(0, b.cols, chunk):
                        c1 = min(b.cols, c0 + chunk)
                        blk = kernel_block(points, perm, b.tau, b.sigma, diag,
                                           c=(b.sigma.begin + c0, b.sigma.begin + c1), kernel=kernel)
                        out[c0:c1] = blk.T @ y
                    return out

                b.U, b.V = _compress_randomized(apply, apply_t, m, n, eps, max_rank, seed + b.index)
    return HMatrix(root, perm, clusters, len(perm), eps, max_rank)


# ---------------------------------------------------------------------------
# Exact block products (no truncation): B X and B^T X for any block kind
# ---------------------------------------------------------------------------
def hmat_mul(b: Block, x: np.ndarray) -> np.ndarray:
    """B x for a block of any kind; x has b.cols rows."""
    _use(b)
    if b.kind == "D":
        return b.D @ x
    if b.kind == "R":
        return b.U @ (b.V.T @ x)
    out = np.zeros((b.rows, x.shape[1]))
    for i in range(2):
        for j in range(2):
            s = b.sons[i][j]
            r0 = s.tau.begin - b.tau.begin
            c0 = s.sigma.begin - b.sigma.begin
            out[r0:r0 + s.rows] += hmat_mul(s, x[c0:c0 + s.cols])
    return out


def hmat_tmul(b: Block, x: np.ndarray) -> np.ndarray:
    """B^T x for a block of any kind; x has b.rows rows."""
    _use(b)
    if b.kind == "D":
        return b.D.T @ x
    if b.kind == "R":
        return b.V @ (b.U.T @ x)
    out = np.zeros((b.cols, x.shape[1]))
    for i in range(2):
        for j in range(2):
            s = b.sons[i][j]
            r0 = s.tau.begin - b.tau.begin
            c0 = s.sigma.begin - b.sigma.begin
            out[c0:c0 + s.cols] += hmat_tmul(s, x[r0:r0 + s.rows])
    return out


# ---------------------------------------------------------------------------
# Sec. 2.3: truncated low-rank addition
# ---------------------------------------------------------------------------
TRUNCATIONS = [0]  # truncated additions performed (for comparing update schemes)


def truncated_add_terms(c: Block, terms: list, eps: float, max_rank: int):
    """C <- T_eps(U_C V_C^T + sum of zero-padded terms (r0, c0, U_p, V_p)), one truncation."""
    TRUNCATIONS[0] += 1
    m, n = c.rows, c.cols
    kc = c.rank
    ks = [u.shape[1] for (_, _, u, _) in terms]
    k = kc + sum(ks)
    if k == 0:
        return
    us = np.zeros((m, k))
    vs = np.zeros((n, k))
    if kc:
        us[:, :kc] = c.U
        vs[:, :kc] = c.V
    col = kc
    for (r0, c0, up, vp) in terms:
        kp = up.shape[1]
        us[r0:r0 + up.shape[0], col:col + kp] = up
        vs[c0:c0 + vp.shape[0], col:col + kp] = vp
        col += kp
    qu, ru = np.linalg.qr(us)
    qv, rv = np.linalg.qr(vs)
    w, s, zt = _svd(ru @ rv.T)
    kk = truncation_rank(s, eps, max_rank, min(m, n))
    c.U = qu @ (w[:, :kk] * s[:kk])
    c.V = qv @ zt[:kk].T


class _Mode:
    """Whether updates of low-rank leaves are collected (Reading R6) during hlu."""
    lazy = False
    eps = 0.0
    max_rank = 0
    depth = 0          # nesting of hmul calls
    touched: list = []  # leaves with collected terms in the current top-level call


def _use(b: Block) -> None:
    """Apply the collected updates of a leaf before it is read (Reading R6)."""
    if b.kind == "R" and b.pending:
        terms, b.pending = b.pending, []
        truncated_add_terms(b, terms, _Mode.eps, _Mode.max_rank)


def truncated_add(c: Block, r0: int, c0: int, up: np.ndarray, vp: np.ndarray, eps: float, max_rank: int):
    """C <- T_eps(U_C V_C^T + pad(U_p) pad(V_p)^T).

    The term's factors are zero-padded: U_p occupies rows [r0, r0+len) of C,
    V_p columns [c0, c0+len).  Stack the factors, Householder-QR each side,
    SVD of the small core R_U R_V^T, keep the leading singular triplets
    (Reading R2) with Sigma folded into U.
    """
    TRUNCATIONS[0] += 1
    m, n = c.rows, c.cols
    kc = c.rank
    kp = up.shape[1]
    if kc + kp == 0:
        return
    us = np.zeros((m, kc + kp))
    vs = np.zeros((n, kc + kp))
    if kc:
        us[:, :kc] = c.U
        vs[:, :kc] = c.V
    us[r0:r0 + up.shape[0], kc:] = up
    vs[c0:c0 + vp.shape[0], kc:] = vp
    qu, ru = np.linalg.qr(us)
    qv, rv = np.linalg.qr(vs)
    w, s, zt = _svd(ru @ rv.T)
    k = truncation_rank(s, eps, max_rank, min(m, n))
    c.U = qu @ (w[:, :k] * s[:k])
    c.V = qv @ zt[:k].T


# ---------------------------------------------------------------------------
# Reading R3: products of leaves as exact low-rank terms
# ---------------------------------------------------------------------------
def product_terms(alpha: float, a: Block, b: Block) -> list:
    """alpha*A*B as a list of zero-padded terms (row offset, col offset, U, V).

    Relative to the row cluster of A and the column cluster of B.  Both
    operands structured: recurse over (i, j, l) in lexicographic order as in
    Algorithm 1.  Otherwise exactly one term:
      A low rank:  U = alpha U_A,        V = B^T V_A
      B low rank:  U = alpha A U_B,      V = V_B
      A, B dense, inner cluster a leaf:  U = alpha A, V = B^T
      A, B dense otherwise (outer leaves): U = alpha A B, V = I
      A dense, B structured (row leaf):  U = alpha I, V = B^T A^T
      A structured, B dense (col leaf):  U = alpha A B, V = I
    """
    _use(a)
    _use(b)
    if a.kind == "S" and b.kind == "S":
        out = []
        for i in range(2):
            for j in range(2):
                for l in range(2):
                    sa, sb = a.sons[i][l], b.sons[l][j]
                    ro = sa.tau.begin - a.tau.begin
                    co = sb.sigma.begin - b.sigma.begin
                    for (r, c, u, v) in product_terms(alpha, sa, sb):
                        out.append((ro + r, co + c, u, v))
        return out
    if a.kind == "R":
        return [(0, 0, alpha * a.U, hmat_tmul(b, a.V))]
    if b.kind == "R":
        return [(0, 0, alpha * hmat_mul(a, b.U), b.V)]
    if a.kind == "D" and b.kind == "D":
        if a.sigma.is_leaf:
            return [(0, 0, alpha * a.D, b.D.T.copy())]
        return [(0, 0, alpha * (a.D @ b.D), np.eye(b.cols))]
    if a.kind == "D":
        return [(0, 0, alpha * np.eye(a.rows), hmat_tmul(b, a.D.T))]
    return [(0, 0, alpha * hmat_mul(a, b.D), np.eye(b.cols))]


def _restrict(term, r_lo, r_hi, c_lo, c_hi):
    """Restrict a padded term to rows [r_lo, r_hi) x cols [c_lo, c_hi); None if empty."""
    r0, c0, u, v = term
    a0, a1 = max(r0, r_lo), min(r0 + u.shape[0], r_hi)
    b0, b1 = max(c0, c_lo), min(c0 + v.shape[0], c_hi)
    if a0 >= a1 or b0 >= b1:
        return None
    return a0 - r_lo, b0 - c_lo, u[a0 - r0:a1 - r0], v[b0 - c0:b1 - c0]


def _add_term_to_leaf(c: Block, term, eps, max_rank):
    r0, c0, u, v = term
    if c.kind == "R" and _Mode.lazy and _Mode.depth > 0:
        if not c.pending:
            _Mode.touched.append(c)
        c.pending.append(term)
        return
    if c.kind == "D":
        c.D[r0:r0 + u.shape[0], c0:c0 + v.shape[0]] += u @ v.T
    else:
        truncated_add(c, r0, c0, u, v, eps, max_rank)


def _leaf_update(alpha, a: Block, b: Block, c: Block, eps, max_rank):
    """Non-recursive branch of Algorithm 1 (the 'special routines', Reading R3)."""
    terms = product_terms(alpha, a, b)
    if c.kind != "S":
        for t in terms:
            _add_term_to_leaf(c, t, eps, max_rank)
        return
    assert len(terms) == 1
    base_r, base_c = c.tau.begin, c.sigma.begin
    for leaf in leaf_blocks(c):
        rt = _restrict(terms[0], leaf.tau.begin - base_r, leaf.tau.end - base_r,
                       leaf.sigma.begin - base_c, leaf.sigma.end - base_c)
        if rt is not None:
            _add_term_to_leaf(leaf, rt, eps, max_rank)


def hmul(alpha, a: Block, b: Block, c: Block, eps, max_rank):
    """Algorithm 1: C := C + alpha A B; recurse while none of the three blocks is a leaf.

    With collected updates (Reading R6) the outermost call applies the terms
    it collected for each low-rank leaf when it returns."""
    top = _Mode.depth == 0
    _Mode.depth += 1
    try:
        if a.kind == "S" and b.kind == "S" and c.kind == "S":
            for i in range(2):
                for j in range(2):
                    for l in range(2):
                        hmul(alpha, a.sons[i][l], b.sons[l][j], c.sons[i][j], eps, max_rank)
        else:
            _leaf_update(alpha, a, b, c, eps, max_rank)
    finally:
        _Mode.depth -= 1
    if top:
        leaves, _Mode.touched = _Mode.touched, []
        for x in leaves:
            _use(x)


# ---------------------------------------------------------------------------
# Leaf LU (Algorithm 2, non-recursive branch) and triangular panel solves
# ---------------------------------------------------------------------------
def getrf_leaf(a: np.ndarray, row0: int = 0) -> np.ndarray:
    """In-place LU with partial pivoting, LAPACK getrf convention (Reading R1).

    Column j: pivot = first row p >= j with maximal |a[p, j]|; swap full rows
    j and p; scale the column below the diagonal; rank-1 update.  Returns the
    0-based interchange vector ipiv.  Raises SingularError on an exact zero.
    """
    m = a.shape[0]
    ipiv = np.zeros(m, dtype=np.int64)
    for j in range(m):
        p = j + int(np.argmax(np.abs(a[j:, j])))
        ipiv[j] = p
        if a[p, j] == 0.0:
            raise SingularError(row0 + j)
        if p != j:
            a[[j, p], :] = a[[p, j], :]
        a[j + 1:, j] /= a[j, j]
        a[j + 1:, j + 1:] -= np.outer(a[j + 1:, j], a[j, j + 1:])
    return ipiv


def apply_pivots(ipiv: np.ndarray, x: np.ndarray) -> None:
    """x <- P x for the interchange sequence ipiv (in place, rows)."""
    for j, p in enumerate(ipiv):
        if p != j:
            x[[j, p]] = x[[p, j]]


def panel_solve_lower(d: Block, x: np.ndarray) -> None:
    """x <- Lp^{-1} P x over the diagonal block d (leaf or structured), in place.

    Diagonal leaf: apply the leaf interchanges then the unit-lower solve.
    Structured: solve with the first son, subtract L10 x0, solve with the second.
    """
    if d.kind == "D":
        apply_pivots(d.piv, x)
        x[:] = sla.solve_triangular(d.D, x, lower=True, unit_diagonal=True, check_finite=False)
        return
    n0 = d.sons[0][0].rows
    panel_solve_lower(d.sons[0][0], x[:n0])
    x[n0:] -= hmat_mul(d.sons[1][0], x[:n0])
    panel_solve_lower(d.sons[1][1], x[n0:])


def panel_solve_upper_t(d: Block, x: np.ndarray) -> None:
    """x <- U^{-T} x over the diagonal block d, in place (solve U^T y = x)."""
    if d.kind == "D":
        x[:] = sla.solve_triangular(d.D, x, trans="T", lower=False, check_finite=False)
        return
    n0 = d.sons[0][0].rows
    panel_solve_upper_t(d.sons[0][0], x[:n0])
    x[n0:] -= hmat_tmul(d.sons[0][1], x[:n0])
    panel_solve_upper_t(d.sons[1][1], x[n0:])


def panel_solve_upper(d: Block, x: np.ndarray) -> None:
    """x <- U^{-1} x over the diagonal block d, in place (backward substitution)."""
    if d.kind == "D":
        x[:] = sla.solve_triangular(d.D, x, lower=False, check_finite=False)
        return
    n0 = d.sons[0][0].rows
    panel_solve_upper(d.sons[1][1], x[n0:])
    x[:n0] -= hmat_mul(d.sons[0][1], x[n0:])
    panel_solve_upper(d.sons[0][0], x[:n0])


def htrsl(ld: Block, m: Block, eps, max_rank):
    """Algorithm 3: L X = M for M on rows of ld; X overwrites M."""
    _use(m)
    if m.kind == "S":
        for j in range(2):
            htrsl(ld.sons[0][0], m.sons[0][j], eps, max_rank)
        for j in range(2):
            hmul(-1.0, ld.sons[1][0], m.sons[0][j], m.sons[1][j], eps, max_rank)
        for j in range(2):
            htrsl(ld.sons[1][1], m.sons[1][j], eps, max_rank)
    elif m.kind == "D":
        panel_solve_lower(ld, m.D)
    else:
        panel_solve_lower(ld, m.U)


def htrsu(ud: Block, m: Block, eps, max_rank):
    """Mirror of Algorithm 3 (Reading R4): X U = M for M on columns of ud; X overwrites M."""
    _use(m)
    if m.kind == "S":
        for j in range(2):
            htrsu(ud.sons[0][0], m.sons[j][0], eps, max_rank)
        for j in range(2):
            hmul(-1.0, m.sons[j][0], ud.sons[0][1], m.sons[j][1], eps, max_rank)
        for j in range(2):
            htrsu(ud.sons[1][1], m.sons[j][1], eps, max_rank)
    elif m.kind == "D":
        xt = np.ascontiguousarray(m.D.T)
        panel_solve_upper_t(ud, xt)
        m.D = xt.T.copy()
    else:
        panel_solve_upper_t(ud, m.V)


def _hlu_rec(a: Block, eps, max_rank):
    """Algorithm 2 (recursive H-LU), in place."""
    if a.kind == "S":
        _hlu_rec(a.sons[0][0], eps, max_rank)
        htrsu(a.sons[0][0], a.sons[1][0], eps, max_rank)
        htrsl(a.sons[0][0], a.sons[0][1], eps, max_rank)
        hmul(-1.0, a.sons[1][0], a.sons[0][1], a.sons[1][1], eps, max_rank)
        _hlu_rec(a.sons[1][1], eps, max_rank)
    else:
        a.piv = getrf_leaf(a.D, a.tau.begin)


def _copy_block(b: Block) -> Block:
    c = Block(b.index, b.tau, b.sigma, b.kind)
    if b.kind == "S":
        c.sons = [[_copy_block(b.sons[i][j]) for j in range(2)] for i in range(2)]
    elif b.kind == "D":
        c.D = b.D.copy()
    else:
        c.U, c.V = b.U.copy(), b.V.copy()
    return c


def hlu(a: HMatrix, eps: float | None = None, max_rank: int | None = None, lazy: bool = False) -> HMatrix:
    """H-LU of a copy of ``a`` (Algorithm 2); the input is not modified.

    lazy=True collects the updates of low-rank leaves (Reading R6)."""
    eps = a.eps if eps is None else eps
    max_rank = a.max_rank if max_rank is None else max_rank
    f = HMatrix(_copy_block(a.root), a.perm, a.clusters, a.n, eps, max_rank)
    _Mode.lazy, _Mode.eps, _Mode.max_rank, _Mode.depth, _Mode.touched = lazy, eps, max_rank, 0, []
    try:
        _hlu_rec(f.root, eps, max_rank)
        for b in leaf_blocks(f.root):
            _use(b)
    finally:
        _Mode.lazy = False
    return f


# ---------------------------------------------------------------------------
# H-LU with accumulated updates (Sec. 2.3, Algorithms 4-8)
# ---------------------------------------------------------------------------
# Every block C_{t,s} owns an accumulator U_{t,s} (the sum of the updates whose
# product could be evaluated: a dense array for a dense leaf, else low-rank
# factors truncated on every addition) and a set P_{t,s} of pending products
# (alpha, A, B) whose three blocks are all structured.  add_upd (Alg. 4)
# collects, shift_upd (Alg. 6) moves U and P one level down, apply_upd (Alg. 5)
# reaches the leaves and adds U into them.  hlu (Alg. 7) and the triangular
# solves (Alg. 8 and its mirror) only collect updates and apply them when a
# leaf is factorized or solved.
class _Accumulators:
    def __init__(self, eps: float, max_rank: int):
        self.eps, self.max_rank = eps, max_rank
        self.u: dict = {}   # block index -> dense array, or (U, V)
        self.p: dict = {}   # block index -> list of (alpha, A, B)

    def add_terms(self, c: Block, terms) -> None:
        """U_{t,s} := U_{t,s} + sum of the terms (one truncated addition for low-rank form)."""
        if not terms:
            return
        if c.kind == "D":
            acc = self.u.get(c.index)
            if acc is None:
                acc = np.zeros((c.rows, c.cols))
            for (r0, c0, u, v) in terms:
                acc[r0:r0 + u.shape[0], c0:c0 + v.shape[0]] += u @ v.T
            self.u[c.index] = acc
            return
        holder = Block(-1, c.tau, c.sigma, "R")
        prev = self.u.get(c.index)
        holder.U, holder.V = prev if prev is not None else (np.zeros((c.rows, 0)), np.zeros((c.cols, 0)))
        truncated_add_terms(holder, list(terms), self.eps, self.max_rank)
        self.u[c.index] = (holder.U, holder.V)

    def add_upd(self, alpha: float, a: Block, b: Block, c: Block) -> None:
        """Algorithm 4.  A product that evaluates to several low-rank terms (both
        operands structured, target a leaf: the special routines after
        Algorithm 1) is added to the accumulator term by term (reading R8)."""
        if a.kind == "S" and b.kind == "S" and c.kind == "S":
            self.p.setdefault(c.index, []).append((alpha, a, b))
        else:
            for term in product_terms(alpha, a, b):
                self.add_terms(c, [term])

    def shift_upd(self, c: Block) -> None:
        """Algorithm 6 (C structured): U_{t',s'} += U_{t,s}|_{t',s'}; pending products split one level."""
        acc = self.u.pop(c.index, None)
        pend = self.p.pop(c.index, [])
        for i in range(2):
            for j in range(2):
                son = c.sons[i][j]
                r_lo, c_lo = son.tau.begin - c.tau.begin, son.sigma.begin - c.sigma.begin
                if acc is not None:
                    u, v = acc
                    rt = _restrict((0, 0, u, v), r_lo, r_lo + son.rows, c_lo, c_lo + son.cols)
                    if rt is not None and rt[2].shape[1] > 0:
                        self.add_terms(son, [rt])
                for (alpha, a, b) in pend:
                    for l in range(2):
                        self.add_upd(alpha, a.sons[i][l], b.sons[l][j], son)

    def apply_upd(self, c: Block) -> None:
        """Algorithm 5: reach the leaves and add the accumulated updates into them."""
        if c.kind == "S":
            self.shift_upd(c)
            for i in range(2):
                for j in range(2):
                    self.apply_upd(c.sons[i][j])
            return
        acc = self.u.pop(c.index, None)
        if acc is None:
            return
        if c.kind == "D":
            c.D += acc
        else:
            truncated_add(c, 0, 0, acc[0], acc[1], self.eps, self.max_rank)

    def htrsl(self, ld: Block, m: Block) -> None:
        """Algorithm 8: L X = M, X overwrites M (corrected indices, reading C-4)."""
        if m.kind == "S":
            self.shift_upd(m)
            for j in range(2):
                self.htrsl(ld.sons[0][0], m.sons[0][j])
            for j in range(2):
                self.add_upd(-1.0, ld.sons[1][0], m.sons[0][j], m.sons[1][j])
            for j in range(2):
                self.htrsl(ld.sons[1][1], m.sons[1][j])
            return
        self.apply_upd(m)
        panel_solve_lower(ld, m.D if m.kind == "D" else m.U)

    def htrsu(self, ud: Block, m: Block) -> None:
        """The mirror of Algorithm 8 for X U = M (reading R4)."""
        if m.kind == "S":
            self.shift_upd(m)
            for j in range(2):
                self.htrsu(ud.sons[0][0], m.sons[j][0])
            for j in range(2):
                self.add_upd(-1.0, m.sons[j][0], ud.sons[0][1], m.sons[j][1])
            for j in range(2):
                self.htrsu(ud.sons[1][1], m.sons[j][1])
            return
        self.apply_upd(m)
        if m.kind == "D":
            xt = np.ascontiguousarray(m.D.T)
            panel_solve_upper_t(ud, xt)
            m.D = xt.T.copy()
        else:
            panel_solve_upper_t(ud, m.V)

    def hlu(self, a: Block) -> None:
        """Algorithm 7 (update of A_{t1,t1} with L_{t1,t0} U_{t0,t1}, reading C-1)."""
        if a.kind == "S":
            self.shift_upd(a)
            self.hlu(a.sons[0][0])
            self.htrsu(a.sons[0][0], a.sons[1][0])
            self.htrsl(a.sons[0][0], a.sons[0][1])
            self.add_upd(-1.0, a.sons[1][0], a.sons[0][1], a.sons[1][1])
            self.hlu(a.sons[1][1])
            return
        self.apply_upd(a)
        a.piv = getrf_leaf(a.D, a.tau.begin)


def hlu_accumulated(a: HMatrix, eps: float | None = None, max_rank: int | None = None) -> HMatrix:
    """H-LU of a copy of ``a`` with accumulated updates (Algorithms 4-8); the input is not modified."""
    eps = a.eps if eps is None else eps
    max_rank = a.max_rank if max_rank is None else max_rank
    f = HMatrix(_copy_block(a.root), a.perm, a.clusters, a.n, eps, max_rank)
    acc = _Accumulators(eps, max_rank)
    acc.hlu(f.root)
    left = [k for k, v in acc.u.items() if v is not None] + [k for k, v in acc.p.items() if v]
    assert not left, f"accumulated updates never applied to blocks {left[:5]}"
    return f


# ---------------------------------------------------------------------------
# Solve, matvec, refinement (not in the paper: textbook block substitution)
# ---------------------------------------------------------------------------
def solve(f: HMatrix, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b through the H-LU factors; b and x in the user's ordering."""
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    b2 = b.reshape(b.shape[0], -1)
    y = b2[f.perm].copy()
    panel_solve_lower(f.root, y)
    panel_solve_upper(f.root, y)
    x = np.empty_like(y)
    x[f.perm] = y
    return x[:, 0] if vec else x


def matvec(a: HMatrix, x: np.ndarray, alpha: float = 1.0, beta: float = 0.0, y=None) -> np.ndarray:
    """y = alpha A_H x + beta y over all leaves; user ordering."""
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    x2 = x.reshape(x.shape[0], -1)
    t = hmat_mul(a.root, x2[a.perm])
    out = np.empty_like(t)
    out[a.perm] = t
    out *= alpha
    if y is not None and beta != 0.0:
        out += beta * np.asarray(y).reshape(out.shape)
    return out[:, 0] if vec else out


def refine(a: HMatrix, f: HMatrix, b: np.ndarray, rtol: float = 1e-10, max_iter: int = 50):
    """Iterative refinement: x += solve(b - A_H x) until ||r||/||b|| <= rtol (per column)."""
    b2 = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    x = solve(f, b2)
    bn = np.linalg.norm(b2, axis=0)
    it = 0
    while True:
        r = b2 - matvec(a, x)
        rel = np.linalg.norm(r, axis=0) / np.where(bn > 0, bn, 1.0)
        if np.all(rel <= rtol) or it >= max_iter:
            return x, it, rel
        x = x + solve(f, r)
        it += 1


# ---------------------------------------------------------------------------
# Dense views and error metrics
# ---------------------------------------------------------------------------
def densify(b: Block) -> np.ndarray:
    """Dense matrix of a block (the H-approximation), permuted ordering."""
    out = np.zeros((b.rows, b.cols))
    for leaf in leaf_blocks(b):
        r0 = leaf.tau.begin - b.tau.begin
        c0 = leaf.sigma.begin - b.sigma.begin
        out[r0:r0 + leaf.rows, c0:c0 + leaf.cols] = leaf.D if leaf.kind == "D" else leaf.U @ leaf.V.T
    return out


def lu_dense_factors(f: HMatrix):
    """(P, Lp, U) dense, permuted ordering, with P A_perm = Lp U (Reading R1).

    P is returned as a row-index vector: (P M) = M[p].
    """
    n = f.n
    lmat = np.zeros((n, n))
    umat = np.zeros((n, n))
    p = np.arange(n)
    for leaf in leaf_blocks(f.root):
        r0, r1, c0, c1 = leaf.tau.begin, leaf.tau.end, leaf.sigma.begin, leaf.sigma.end
        dense = leaf.D if leaf.kind == "D" else leaf.U @ leaf.V.T
        if leaf.tau is leaf.sigma:
            lmat[r0:r1, c0:c1] = np.tril(dense, -1) + np.eye(r1 - r0)
            umat[r0:r1, c0:c1] = np.triu(dense)
            local = np.arange(r1 - r0)
            apply_pivots(leaf.piv, local)
            p[r0:r1] = r0 + local
        elif r0 >= c1:
            lmat[r0:r1, c0:c1] = dense
        else:
            umat[r0:r1, c0:c1] = dense
    # off-diagonal L rows are stored unpermuted: Lp = P L_off + L_diag
    loff = lmat.copy()
    ldiag = np.zeros_like(lmat)
    for leaf in leaf_blocks(f.root):
        if leaf.tau is leaf.sigma:
            r0, r1 = leaf.tau.begin, leaf.tau.end
            ldiag[r0:r1, r0:r1] = lmat[r0:r1, r0:r1]
            loff[r0:r1, r0:r1] = 0.0
    lp = loff[p] + ldiag
    return p, lp, umat


def lu_error_2norm(a_dense_perm: np.ndarray, f: HMatrix, exact: bool | None = None, iters: int = 60,
                   seed: int = 5) -> float:
    """||P A - Lp U||_2 / ||A||_2 against a dense matrix in permuted ordering.

    Exact 2-norms for n <= 2048 (or exact=True), else power iteration on E^T E.
    """
    p, lp, umat = lu_dense_factors(f)
    e = a_dense_perm[p] - lp @ umat
    n = e.shape[0]
    if exact or (exact is None and n <= 2048):
        return float(np.linalg.norm(e, 2) / np.linalg.norm(a_dense_perm, 2))
    return _power_norm(e, iters, seed) / _power_norm(a_dense_perm, iters, seed)


def _power_norm(mat: np.ndarray, iters: int, seed: int) -> float:
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(mat.shape[1])
    v /= np.linalg.norm(v)
    prev = 0.0
    for _ in range(iters):
        w = mat.T @ (mat @ v)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            return 0.0
        v = w / lam
        if abs(lam - prev) <= 1e-4 * lam:
            prev = lam
            break
        prev = lam
    return math.sqrt(prev)


def rank_table(a: HMatrix) -> dict:
    """{block index: rank} for low-rank leaves."""
    return {b.index: b.rank for b in leaf_blocks(a.root) if b.kind == "R"}
