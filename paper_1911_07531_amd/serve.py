"""A solve-serving loop over resident H-LU factors (continuous batching).

Factors stay on the device.  Requests arrive over time: a solve carries its
own right-hand sides (1-64 columns) for one factor; a refactorize request
replaces a factor by the H-LU of a new point set of the same size.  The loop

  * admits work by device footprint: a factor (matrix + factors + workspace,
    hm_footprint) or a request's right-hand-side buffer is admitted only
    while the bytes held stay within the budget; otherwise it waits;
  * batches continuously: whenever a factor's stream is idle, every solve
    request for that factor that has arrived (up to max_cols columns) is
    packed into one column-major buffer and substituted by one asynchronous
    h_solve_async on that factor's own stream, so requests for different
    factors overlap on the device and requests arriving meanwhile join the
    next batch;
  * refactorizes on a worker thread (tracing, assembly and h_lu on a stream
    of their own) and swaps the factor in when it is ready; solves queued for
    it meanwhile wait for the new factor;
  * reports, per request, the time from arrival to its result being ready on
    the device.

A column's solution does not depend on the other columns of its batch except
through rounding (the substitution's FP64 reductions are grouped by the
batch's column count), so a request's result is the same alone and in the
mix to about 1e-15 relative.  Every computation runs in the library's kernels; this
module only orders, packs and times the work.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import hm, inputs


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    factor: int             # index of the resident factor
    nrhs: int = 0           # solve: right-hand sides; 0 for a refactorize request
    seed: int = 0           # RHS seed (solve) or new point seed (refactorize)
    kind: str = "solve"
    t_done: float = float("nan")
    x: object = None        # device tensor (n, nrhs) with the solution
    batch: int = -1         # batch the request was served in
    status: int = 0


def rhs_device(n: int, nrhs: int, seed: int):
    """N(0, 1) right-hand sides of a request, drawn on the device from its own seed."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    return torch.randn((nrhs, n), generator=g, dtype=torch.float64, device="cuda").t()  # column-major (n, nrhs)


def poisson_stream(count: int, rate: float, factors: int, seed: int = 7, max_rhs: int = 64,
                   refactor_frac: float = 0.01):
    """Seeded request stream: exponential gaps at `rate` per second; each request picks
    a factor uniformly; a fraction refactorizes, the rest solve U{1..max_rhs} columns."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    f = rng.integers(0, factors, size=count)
    k = rng.integers(1, max_rhs + 1, size=count)
    refac = rng.random(count) < refactor_frac
    out = []
    for i in range(count):
        if refac[i]:
            out.append(Request(i, float(t[i]), int(f[i]), 0, 1000 + i, "refactor"))
        else:
            out.append(Request(i, float(t[i]), int(f[i]), int(k[i]), 10_000 + i))
    return out


class Resident:
    """One resident factorization: tree, assembled matrix, factors, its stream."""

    def __init__(self, geometry: str, n: int, seed: int, opts, kernel_name: str | None = None):
        import torch
        self.geometry, self.n, self.seed, self.opts = geometry, n, seed, opts
        pts, diag = inputs.problem(geometry, n, seed)
        kname = kernel_name or inputs.GEOMETRY_KERNEL[geometry]
        self.stream = torch.cuda.Stream()
        self.tree = hm.Tree(pts, opts)
        with torch.cuda.stream(self.stream):
            self.A = hm.Matrix(self.tree, hm.LAPLACE3D if kname == "laplace3d" else hm.LOG2D, diag, opts,
                               stream=self.stream)
            self.F = hm.LU(self.A, opts, stream=self.stream)
        self.n = self.tree.n
        self.status = torch.zeros(1, dtype=torch.int32, device="cuda")

    def footprint(self) -> int:
        return self.A.footprint() + self.F.footprint(1) + self.F.footprint(2)


class Server:
    def __init__(self, residents, budget_bytes: int, max_cols: int = 64):
        self.res = list(residents)
        self.budget = int(budget_bytes)
        self.max_cols = int(max_cols)
        self.held = sum(r.footprint() for r in self.res)
        if self.held > self.budget:
            raise ValueError(f"resident factors need {self.held} bytes, above the budget {self.budget}")
        self.lock = threading.Lock()
        self.batches = 0
        self.refactor_ms = []
        self.retries = 0
        # a refactorization holds a second factor plus its working set while it runs
        self.refactor_factor = 2.0

    # -- memory admission ----------------------------------------------------
    def _admit(self, nbytes: int) -> bool:
        with self.lock:
            if self.held + nbytes > self.budget:
                return False
            self.held += nbytes
            return True

    def _release(self, nbytes: int) -> None:
        with self.lock:
            self.held -= nbytes

    # -- the loop -----------------------------------------------------------
    def run(self, requests, poll_s: float = 20e-6):
        """Serve the requests (sorted by arrival) in real time; fills t_done / x / status."""
        import torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        nf = len(self.res)
        pending = [deque() for _ in range(nf)]
        inflight = [None] * nf          # (event, [(req, col0)], buffer, bytes, status copy)
        refactoring = [None] * nf       # worker thread and its result slot
        waiting_refac = deque()
        done = 0
        i = 0
        t0 = time.perf_counter()
        while done < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                r = reqs[i]
                i += 1
                if r.kind == "refactor":
                    waiting_refac.append(r)
                else:
                    pending[r.factor].append(r)
            progressed = False
            # completions
            for f in range(nf):
                fl = inflight[f]
                if fl is not None and fl[0].query():
                    ev, members, buf, nbytes, st_host = fl
                    st = int(st_host[0])
                    tdone = time.perf_counter() - t0
                    for r, c0 in members:
                        r.x = buf[:, c0:c0 + r.nrhs]
                        r.status = st
                        r.t_done = tdone
                        done += 1
                    self._release(nbytes)
                    inflight[f] = None
                    progressed = True
            # refactorizations: start when memory admits a second copy of the factor
            # plus its transient working set (traced DAG, executor state, scratch)
            while waiting_refac:
                r = waiting_refac[0]
                f = r.factor
                if refactoring[f] is not None or inflight[f] is not None:
                    break
                need = int(self.refactor_factor * self.res[f].footprint())
                if not self._admit(need):
                    break
                waiting_refac.popleft()
                slot = {}
                old = self.res[f]

                def work(old=old, r=r, slot=slot):
                    t1 = time.perf_counter()
                    try:
                        slot["res"] = Resident(old.geometry, old.n, r.seed, old.opts)  # h_lu synchronises its stream
                    except Exception as e:  # reported by the loop
                        slot["error"] = e
                    slot["ms"] = (time.perf_counter() - t1) * 1e3

                th = threading.Thread(target=work)
                th.start()
                refactoring[f] = (th, slot, r, need)
                progressed = True
            for f in range(nf):
                rf = refactoring[f]
                if rf is not None and not rf[0].is_alive():
                    th, slot, r, need = rf
                    th.join()
                    if "res" not in slot:
                        err = slot.get("error")
                        if isinstance(err, hm.HmError) and err.code == hm.HM_ENOMEM and self.retries < 100:
                            # the device could not hold it now: release, requeue, retry later
                            self._release(need)
                            refactoring[f] = None
                            waiting_refac.appendleft(r)
                            self.retries += 1
                            torch.cuda.empty_cache()
                            continue
                        raise RuntimeError(f"refactorization of factor {f} failed: {err}")
                    new = slot["res"]
                    old = self.res[f]
                    self.res[f] = new
                    self._release(old.footprint() + need - new.footprint())
                    self.refactor_ms.append(slot["ms"])
                    r.t_done = time.perf_counter() - t0
                    done += 1
                    refactoring[f] = None
                    del old
                    progressed = True
            # launches: one batch per idle factor
            for f in range(nf):
                if inflight[f] is not None or refactoring[f] is not None or not pending[f]:
                    continue
                res = self.res[f]
                members, cols = [], 0
                while pending[f] and (not members or cols + pending[f][0].nrhs <= self.max_cols):
                    r = pending[f].popleft()
                    members.append((r, cols))
                    cols += r.nrhs
                nbytes = res.n * cols * 8
                if not self._admit(nbytes):
                    for r, _ in reversed(members):
                        pending[f].appendleft(r)
                    continue
                with torch.cuda.stream(res.stream):
                    buf = torch.empty((cols, res.n), dtype=torch.float64, device="cuda").t()
                    for r, c0 in members:
                        buf[:, c0:c0 + r.nrhs] = rhs_device(res.n, r.nrhs, r.seed)
                    res.F.solve_async(buf, res.status, stream=res.stream)
                    st_host = torch.empty(1, dtype=torch.int32, pin_memory=True)
                    st_host.copy_(res.status, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(res.stream)
                for r, _ in members:
                    r.batch = self.batches
                self.batches += 1
                inflight[f] = (ev, members, buf, nbytes, st_host)
                progressed = True
            if not progressed:
                time.sleep(poll_s)
        return reqs

    def solve_alone(self, r: Request):
        """The same request served by itself (one h_solve_async of its columns only)."""
        import torch
        res = self.res[r.factor]
        with torch.cuda.stream(res.stream):
            buf = torch.empty((r.nrhs, res.n), dtype=torch.float64, device="cuda").t()
            buf[:, :] = rhs_device(res.n, r.nrhs, r.seed)
            res.F.solve_async(buf, res.status, stream=res.stream)
        res.stream.synchronize()
        return buf, int(res.status.item())


def latency_summary(reqs) -> dict:
    solves = [r for r in reqs if r.kind == "solve"]
    lat = np.array([(r.t_done - r.arrival) * 1e3 for r in solves])
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "solves": len(solves),
            "refactorizations": sum(1 for r in reqs if r.kind == "refactor"),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "solves_per_s": len(solves) / span, "rhs_per_s": sum(r.nrhs for r in solves) / span,
            "span_s": span, "failed": sum(1 for r in solves if r.status != 0)}
