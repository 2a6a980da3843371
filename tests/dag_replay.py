"""Test-only replay of a traced task DAG in NumPy (no device).

Interprets the task records exported by the library (struct Task) on NumPy
arenas, in a random topological order of the DAG.  It checks on the CPU that
the trace of Algorithms 1-3 and its dependencies are right: the result must
match the oracle's sequential H-LU whatever order the DAG admits.  The task
semantics here are plain NumPy/SciPy; nothing of this is used by the library.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

VT_F64, VT_F32, VT_IDENT, VT_NONE = 0, 1, 2, 3
DYN_ROWS, DYN_COLS, DYN_COLS2, DYN_LOCAL = 1, 2, 4, 8


class Replay:
    def __init__(self, dag, eps, max_rank):
        self.d = dag
        # unwritten storage holds NaN, so a task that reads before its producer
        # (a missing edge) or past what was written shows up in the result
        self.f64 = np.full(max(1, dag["n_f64"]), np.nan)
        self.f32 = np.full(max(1, dag["n_f32"]), np.nan, np.float32)
        self.piv = np.zeros(max(1, dag["n_piv"]), np.int32)
        self.ranks = np.zeros(dag["nranks"], np.int32)
        self.eps = eps
        self.max_rank = max_rank
        self.inner = 0.1  # relative accuracy of inner (combining) truncations, in units of eps

    # -- views ---------------------------------------------------------------
    def dims(self, v):
        rows = self.ranks[v["rank_id"]] if v["dyn"] & DYN_ROWS else v["rows"]
        cols = self.ranks[v["rank_id"]] if v["dyn"] & DYN_COLS else v["cols"]
        if v["dyn"] & DYN_COLS2:
            cols = self.ranks[v["rank_id2"]]
        return int(rows), int(cols)

    def view(self, v):
        rows, cols = self.dims(v)
        t = int(v["type"])
        if t == VT_IDENT:
            return np.eye(rows, cols)
        arena = self.f64 if t == VT_F64 else self.f32
        off = int(v["off"])
        if rows == 0 or cols == 0:
            return np.zeros((rows, cols), arena.dtype)
        last = off + (rows - 1) * int(v["rs"]) + (cols - 1) * int(v["cs"])
        assert off >= 0 and last < arena.size, ("view out of its arena", off, rows, cols, v["rs"], v["cs"], arena.size)
        isz = arena.itemsize
        base = arena[off:]
        return np.lib.stride_tricks.as_strided(base, (rows, cols), (int(v["rs"]) * isz, int(v["cs"]) * isz))

    # -- storage ---------------------------------------------------------------
    def load_matrix(self, blocks_by_index, block_off, lr):
        """Fill the arenas from oracle leaves {block index: Block}."""
        for bi, b in blocks_by_index.items():
            off, typ, li, _ = block_off[bi]
            arena = self.f64 if typ == VT_F64 or li >= 0 and lr[li][5] == VT_F64 else self.f32
            if b.kind == "D":
                arena = self.f64 if typ == VT_F64 else self.f32
                arena[off:off + b.D.size] = b.D.flatten(order="F")
            elif b.kind == "R":
                u_off, v_off, m, n, cap, typ = lr[li]
                arena = self.f64 if typ == VT_F64 else self.f32
                k = b.rank
                assert k <= cap
                arena[u_off:u_off + m * k] = b.U.flatten(order="F")
                arena[v_off:v_off + n * k] = b.V.flatten(order="F")
                self.ranks[li] = k

    def leaf(self, bi, kind, m, n, block_off, lr):
        off, typ, li, poff = block_off[bi]
        if kind == 1:
            arena = self.f64 if typ == VT_F64 else self.f32
            d = np.asarray(arena[off:off + m * n], np.float64).reshape(n, m).T.copy()
            piv = self.piv[poff:poff + m].astype(np.int64) if poff >= 0 else None
            return "D", d, piv
        u_off, v_off, m_, n_, cap, typ = lr[li]
        arena = self.f64 if typ == VT_F64 else self.f32
        k = int(self.ranks[li])
        u = np.asarray(arena[u_off:u_off + m * k], np.float64).reshape(k, m).T.copy()
        v = np.asarray(arena[v_off:v_off + n * k], np.float64).reshape(k, n).T.copy()
        return "R", u, v

    # -- tasks -----------------------------------------------------------------
    def run_task(self, t):
        op = int(t["op"])
        if op == 1:  # getrf
            m = int(t["a"]["rows"])
            a = self.view(t["a"])
            lu, piv = sla.lu_factor(np.array(a, np.float64), check_finite=False)
            a[:] = lu
            self.piv[int(t["piv"]):int(t["piv"]) + m] = piv
            perm = np.arange(m)
            for j, q in enumerate(piv):  # (P x)[i] = x[perm[i]]
                perm[[j, q]] = perm[[q, j]]
            self.piv[int(t["piv"]) + m:int(t["piv"]) + 2 * m] = perm
        elif op in (2, 4) and int(t["b"]["type"]) == VT_F64:  # substitution with the leaf's inverse
            m = int(t["a"]["rows"])
            inv = np.array(self.view(t["b"]), np.float64)
            x = self.view(t["x"])
            xs = np.array(x, np.float64)
            if op == 2:
                xs = xs[self.piv[int(t["piv"]) + m:int(t["piv"]) + 2 * m]]
            x[:] = inv @ xs
        elif op == 13:  # inverses of the triangles of a factored diagonal leaf
            m = int(t["a"]["rows"])
            lu = np.array(self.view(t["a"]), np.float64)
            y = self.view(t["y"])
            eye = np.eye(m)
            y[:, :m] = sla.solve_triangular(lu, eye, lower=True, unit_diagonal=True, check_finite=False)
            y[:, m:] = sla.solve_triangular(lu, eye, lower=False, check_finite=False)
        elif op in (2, 3, 4):
            m = int(t["a"]["rows"])
            a = np.array(self.view(t["a"]), np.float64)
            x = self.view(t["x"])
            xs = np.array(x, np.float64)
            if op == 2:
                for j, p in enumerate(self.piv[int(t["piv"]):int(t["piv"]) + m]):
                    if p != j:
                        xs[[j, p]] = xs[[p, j]]
                xs = sla.solve_triangular(a, xs, lower=True, unit_diagonal=True, check_finite=False)
            elif op == 3:
                xs = sla.solve_triangular(a, xs, trans="T", lower=False, check_finite=False)
            else:
                xs = sla.solve_triangular(a, xs, lower=False, check_finite=False)
            x[:] = xs
        elif op == 5:
            y = self.view(t["y"])
            prod = np.asarray(self.view(t["a"]), np.float64) @ np.asarray(self.view(t["b"]), np.float64)
            out = t["alpha"] * prod
            if t["beta"] != 0.0:
                out = out + t["beta"] * np.asarray(y, np.float64)
            y[:] = out
        elif op == 6:
            y = self.view(t["y"])
            a = np.asarray(self.view(t["a"]), np.float64)
            b = np.asarray(self.view(t["b"]), np.float64)
            x = np.asarray(self.view(t["x"]), np.float64)
            out = t["alpha"] * (a @ (b @ x))
            if t["beta"] != 0.0:
                out = out + t["beta"] * np.asarray(y, np.float64)
            y[:] = out
        elif op == 7:
            self.trunc(t)
        elif op == 8:
            self.view(t["y"])[:] = 0.0
        elif op == 9:
            self.view(t["y"])[:] = self.view(t["a"])
        elif op == 10:
            self.trunc(t, two=True)
        elif op == 11:  # y += alpha a (b_0 + ... + b_{P-1}), b_p at offset b.off + p * piv
            y = self.view(t["y"])
            bsum = 0.0
            for p in range(int(t["r0"])):
                bv = t["b"].copy()
                bv["off"] = int(t["b"]["off"]) + p * int(t["piv"])
                bsum = bsum + np.asarray(self.view(bv), np.float64)
            y[:] = np.asarray(y, np.float64) + t["alpha"] * (np.asarray(self.view(t["a"]), np.float64) @ bsum)
        elif op == 12:  # coarsened substitution block: its micro-operations in order
            base = int(t["y"]["off"])
            first, count = int(t["piv"]), int(t["lr"])
            for k in range(first, first + count):
                u = self.d["seq"][k:k + 1].copy()
                for key in ("y", "a", "b", "x"):
                    if int(u[key]["dyn"][0]) & DYN_LOCAL:  # rows relative to the block
                        u[key]["off"][0] = base + int(u[key]["off"][0])
                        u[key]["dyn"][0] = int(u[key]["dyn"][0]) & ~DYN_LOCAL
                assert int(u["op"][0]) in (2, 4, 5, 6), int(u["op"][0])
                self.run_task(u[0])
        else:
            raise ValueError(op)

    def trunc(self, t, two=False):
        li = int(t["lr"])
        u_off, v_off, m, n, cap, typ = (int(x) for x in self.d["lr"][li])
        arena = self.f64 if typ == VT_F64 else self.f32
        kc = 0 if two else int(self.ranks[li])
        a = np.asarray(self.view(t["a"]), np.float64)
        b = np.asarray(self.view(t["b"]), np.float64)
        kp = a.shape[1]
        x = np.asarray(self.view(t["x"]), np.float64) if two else np.zeros((0, 0))
        y = np.asarray(self.view(t["y"]), np.float64) if two else np.zeros((0, 0))
        kp2 = x.shape[1] if two else 0
        K = kc + kp + kp2
        if K == 0:
            self.ranks[li] = 0
            return
        us = np.zeros((m, K))
        vs = np.zeros((n, K))
        us[:, :kc] = np.asarray(arena[u_off:u_off + m * kc], np.float64).reshape(kc, m).T
        vs[:, :kc] = np.asarray(arena[v_off:v_off + n * kc], np.float64).reshape(kc, n).T
        r0, c0 = int(t["r0"]), int(t["c0"])
        us[r0:r0 + a.shape[0], kc:kc + kp] = t["alpha"] * a
        vs[c0:c0 + b.shape[0], kc:kc + kp] = b
        if two:
            r1, c1 = int(t["row0"]), int(t["c1"])
            us[r1:r1 + x.shape[0], kc + kp:] = t["beta"] * x
            vs[c1:c1 + y.shape[0], kc + kp:] = y
        qu, ru = np.linalg.qr(us)
        qv, rv = np.linalg.qr(vs)
        w, s, zt = np.linalg.svd(ru @ rv.T)
        eps = self.eps * (self.inner if two else 1.0)
        k = 0 if s.size == 0 or s[0] <= 0 else int(np.count_nonzero(s > eps * s[0]))
        k = min(k, cap, m, n)
        unew = qu @ (w[:, :k] * s[:k])
        vnew = qv @ zt[:k].T
        arena[u_off:u_off + m * k] = unew.flatten(order="F")
        arena[v_off:v_off + n * k] = vnew.flatten(order="F")
        self.ranks[li] = k

    def run(self, rng=None):
        """Execute every task in a random topological order (Kahn with random picks)."""
        tasks = self.d["tasks"]
        n = len(tasks)
        sp, si = self.d["succ_ptr"], self.d["succ_idx"]
        indeg = np.zeros(n, np.int64)
        np.add.at(indeg, si, 1)
        ready = list(np.nonzero(indeg == 0)[0])
        done = 0
        while ready:
            k = rng.integers(len(ready)) if rng is not None else 0
            ready[k], ready[-1] = ready[-1], ready[k]
            i = ready.pop()
            self.run_task(tasks[i])
            done += 1
            for s in si[sp[i]:sp[i + 1]]:
                indeg[s] -= 1
                if indeg[s] == 0:
                    ready.append(s)
        assert done == n, "DAG has a cycle or unreachable tasks"
