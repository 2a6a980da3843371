"""Autotuner of the executors' launch choices, with a JSON cache.

The library exposes a few launch choices (hm_set_tuning): workgroups per
compute unit of the H-LU executors, workgroups of the persistent substitution
executor, and the queue order of a batch's instances.  Their best values
depend on the DAG's shape (a batch of many small matrices, one deep
factorization, a narrow substitution), so this module times each candidate on
the caller's own workload and keeps the fastest, keyed by the device and a
signature of the workload, in a JSON file (HM_TUNE_CACHE, default
~/.cache/hm_tuning.json).  Every timed call runs in the library's kernels;
this module only chooses among launch settings.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

from . import hm


def cache_path() -> str:
    return os.environ.get("HM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hm_tuning.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, rec: dict) -> None:
    data = _load()
    data[key] = rec
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _key(kind: str, sig) -> str:
    import torch
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    h = hashlib.sha1(json.dumps([kind, dev, sig], sort_keys=True).encode()).hexdigest()[:16]
    return f"{kind}:{h}"


def _time(fn, reps: int) -> float:
    import torch
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) * 1e3)
    return best


def tune_batched(mats, opts, reps: int = 1, use_cache: bool = True) -> dict:
    """Choose exec_wg_per_cu in {1, 2} and batch_order in {0, 1} for h_lu_batched
    of `mats`; applies the choice and returns {params, ms, cached}."""
    sig = sorted((int(m.tree.n), int(m.opts.leaf), int(m.opts.max_rank)) for m in mats) + \
        [int(opts.prec), float(opts.eps), int(opts.lazy), int(opts.exec)]
    key = _key("batched", sig)
    rec = _load().get(key) if use_cache else None
    if rec is None:
        hm.lu_batched(mats, opts)  # traces every plan once, outside the timing
        results = []
        for wg, order in itertools.product((1, 2), (0, 1)):
            hm.set_tuning(exec_wg_per_cu=wg, batch_order=order)
            ms = _time(lambda: hm.lu_batched(mats, opts), reps)
            results.append({"exec_wg_per_cu": wg, "batch_order": order, "ms": ms})
        best = min(results, key=lambda r: r["ms"])
        rec = {"params": {"exec_wg_per_cu": best["exec_wg_per_cu"], "batch_order": best["batch_order"]},
               "ms": best["ms"], "candidates": results}
        _store(key, rec)
        cached = False
    else:
        cached = True
    hm.set_tuning(**rec["params"])
    return dict(rec, cached=cached)


def tune_solve(f, nrhs: int, reps: int = 2, use_cache: bool = True) -> dict:
    """Choose the substitution executor's workgroups (solve_wg) for solves of
    nrhs columns on the factors f; applies it and returns {params, ms, cached}."""
    import numpy as np
    import torch
    from . import inputs
    sig = [int(f.tree.n), int(f.opts.leaf), int(f.opts.prec), int(nrhs)]
    key = _key("solve", sig)
    rec = _load().get(key) if use_cache else None
    if rec is None:
        b = torch.from_numpy(np.asfortranarray(inputs.rhs(f.tree.n, nrhs, seed=1))).cuda().t().contiguous().t()
        results = []
        for wg in (64, 128, 256):
            hm.set_tuning(solve_wg=wg)
            ms = _time(lambda: f.solve(b.clone().t().contiguous().t()), reps)
            results.append({"solve_wg": wg, "ms": ms})
        best = min(results, key=lambda r: r["ms"])
        rec = {"params": {"solve_wg": best["solve_wg"]}, "ms": best["ms"], "candidates": results}
        _store(key, rec)
        cached = False
    else:
        cached = True
    hm.set_tuning(**rec["params"])
    return dict(rec, cached=cached)
