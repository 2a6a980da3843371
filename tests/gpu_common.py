"""Shared fixtures for the GPU tests: device tensors, exported factors and
their comparison with the oracle (test infrastructure)."""
from __future__ import annotations

import numpy as np

from oracle import hmatrix as H
from paper_1911_07531_amd import hm, inputs


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test started without a visible HIP device")
    hm.lib()  # raises if libhm.so is missing


def device_rhs(b):
    import torch
    return torch.from_numpy(np.asfortranarray(b)).cuda().t().contiguous().t() if b.ndim == 2 else \
        torch.from_numpy(b).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


class Problem:
    """A workload on both sides: the oracle's tree/assembly and the GPU's.

    geometry "sphere": the single layer potential on the sphere; "line": the
    one-dimensional log-kernel model problem on [0, 1]; "cube": the single
    layer kernel on the unit cube's surface; "grid": the 2D logarithmic
    kernel on a uniform grid of the unit square (n rounded to the lattice)."""

    def __init__(self, n, leaf, eps, max_rank=0, eta=2.0, seed=0, prec=hm.FP64, exec_mode=hm.DATAFLOW,
                 oracle=True, geometry="sphere"):
        self.n, self.leaf, self.eps, self.max_rank = n, leaf, eps, max_rank
        self.pts, self.diag = inputs.problem(geometry, n, seed)
        self.kname = inputs.GEOMETRY_KERNEL[geometry]
        self.kernel = hm.LAPLACE3D if self.kname == "laplace3d" else hm.LOG2D
        n = self.n = len(self.pts)
        self.opts = hm.make_opts(leaf=leaf, eta=eta, eps=eps, max_rank=max_rank, prec=prec, exec_mode=exec_mode)
        self.tree = hm.Tree(self.pts, self.opts)
        self.A = hm.Matrix(self.tree, self.kernel, self.diag, self.opts)
        if oracle:
            perm, cl = H.build_cluster_tree(self.pts, leaf)
            root = H.build_block_tree(cl[0], eta)
            self.oa = H.assemble(self.pts, perm, cl, root, self.diag, eps, max_rank, kernel=self.kname)
        else:
            self.oa = None

    def gpu_as_oracle(self, handle_kind, handle):
        """Exported GPU leaves in the oracle's block structure (for densify etc.)."""
        perm, cl = H.build_cluster_tree(self.pts, self.leaf)
        root = H.build_block_tree(cl[0], self.opts.eta)
        for b in H.leaf_blocks(root):
            r = hm.export_leaf(handle, handle_kind, b.index, self.tree)
            if r[0] == "D":
                b.D = r[1]
                if b.tau is b.sigma and handle_kind == 1:
                    b.piv = r[2].astype(np.int64)
            else:
                b.U, b.V = r[1], r[2]
        return H.HMatrix(root, perm, cl, self.n, self.eps, self.max_rank)

    def dense_exact(self):
        """Exact kernel matrix in permuted order (small n only)."""
        perm, cl = H.build_cluster_tree(self.pts, self.leaf)
        return H.kernel_block(self.pts, perm, cl[0], cl[0], self.diag, kernel=self.kname)

    def exact_block(self, perm, tau, sigma):
        return H.kernel_block(self.pts, perm, tau, sigma, self.diag, kernel=self.kname)
