"""Write the oracle's reference values for the large sphere workloads.

Run from the repository root (CPU only, oracle and input generator only):

    python tests/golden/make_golden.py c2     # n = 32768,  leaf 64, eps 1e-6, ranks capped at 64
    python tests/golden/make_golden.py c3     # n = 131072, leaf 64, eps 1e-4, ranks capped at 64

Each writes tests/golden/<name>_sphere.npz with
  * the rank of every low-rank leaf of the assembled matrix and of the H-LU
    factors (block indices of the block tree, pre-order), computed by
    oracle.hmatrix with collected updates (Reading R6, the device default);
  * the relative residuals ||b - A x||_2 / ||b||_2 of the unrefined solve
    x = oracle.solve(F, b) for N(0, 1) right-hand sides (inputs.rhs, seed 1),
    with A the exact kernel matrix (not its H-approximation), evaluated in row
    chunks;
  * the oracle's H-LU wall time on this machine (context only).

The GPU tests compare the device's ranks (within +-2) and unrefined residuals
(at most 2x) with these values.  Nothing here touches the device library.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import hmatrix as H  # noqa: E402
from paper_1911_07531_amd import inputs  # noqa: E402

CONFIGS = {
    "c2": dict(n=32768, leaf=64, eta=2.0, eps=1e-6, max_rank=64, nrhs=16),
    "c3": dict(n=131072, leaf=64, eta=2.0, eps=1e-4, max_rank=64, nrhs=32),
}


def exact_residuals(pts, perm, root_cluster, diag, b, x, chunk=256):
    """||b - A x|| / ||b|| per column with the exact kernel matrix A, rows in chunks."""
    n = len(perm)
    bp, xp = b[perm], x[perm]
    r2 = np.zeros(b.shape[1])
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        a = H.kernel_block(pts, perm, root_cluster, root_cluster, diag, r=(r0, r1))
        r = bp[r0:r1] - a @ xp
        r2 += (r * r).sum(axis=0)
    return np.sqrt(r2) / np.linalg.norm(b, axis=0)


def save_assembly(path, a):
    """The oracle's assembled leaves in one flat array (no pickling)."""
    leaves = H.leaf_blocks(a.root)
    meta, chunks, off = [], [], 0
    for b in leaves:
        parts = [b.D] if b.kind == "D" else [b.U, b.V]
        k = -1 if b.kind == "D" else b.U.shape[1]
        meta.append((b.index, k, off))
        for x in parts:
            chunks.append(np.asarray(x, np.float64).ravel(order="F"))
            off += x.size
    np.savez(path, meta=np.array(meta, np.int64), data=np.concatenate(chunks))


def load_assembly(path, pts, perm, cl, root, c):
    z = np.load(path)
    meta, data = z["meta"], z["data"]
    blocks = {b.index: b for b in H.leaf_blocks(root)}
    for idx, k, off in meta:
        b = blocks[int(idx)]
        m, n = b.rows, b.cols
        if k < 0:
            b.D = data[off:off + m * n].reshape(n, m).T.copy()
        else:
            b.U = data[off:off + m * k].reshape(k, m).T.copy()
            b.V = data[off + m * k:off + (m + n) * k].reshape(k, n).T.copy()
    return H.HMatrix(root, perm, cl, len(perm), c["eps"], c["max_rank"])


def main(name: str):
    c = CONFIGS[name]
    t0 = time.time()
    pts, diag = inputs.sphere_problem(c["n"], 0)
    perm, cl = H.build_cluster_tree(pts, c["leaf"])
    root = H.build_block_tree(cl[0], c["eta"])
    print(f"[{name}] trees {time.time() - t0:.1f} s", flush=True)
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"hm_golden_{name}_assembly.npz")
    if os.path.exists(cache):  # the oracle's own assembly from an earlier run of this script
        a = load_assembly(cache, pts, perm, cl, root, c)
    else:
        a = H.assemble(pts, perm, cl, root, diag, c["eps"], c["max_rank"])
        save_assembly(cache, a)
    arank = H.rank_table(a)
    print(f"[{name}] assembled {time.time() - t0:.1f} s, {len(arank)} low-rank leaves", flush=True)
    t1 = time.time()
    f = H.hlu(a, lazy=True)
    t_lu = time.time() - t1
    frank = H.rank_table(f)
    print(f"[{name}] H-LU {t_lu:.1f} s", flush=True)
    b = inputs.rhs(c["n"], c["nrhs"], seed=1)
    x = H.solve(f, b)
    res = exact_residuals(pts, perm, cl[0], diag, b, x)
    print(f"[{name}] residuals {res.min():.3e} .. {res.max():.3e} ({time.time() - t0:.1f} s)", flush=True)
    keys = np.array(sorted(arank), dtype=np.int64)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_sphere.npz")
    np.savez_compressed(out, n=c["n"], leaf=c["leaf"], eta=c["eta"], eps=c["eps"], max_rank=c["max_rank"],
                        lazy=1, rhs_seed=1, blocks=keys,
                        assembly_rank=np.array([arank[k] for k in keys], dtype=np.int32),
                        factor_rank=np.array([frank[k] for k in keys], dtype=np.int32),
                        residual=res, oracle_lu_seconds=t_lu)
    print(f"[{name}] wrote {out}", flush=True)


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["c2"]:
        main(arg)
