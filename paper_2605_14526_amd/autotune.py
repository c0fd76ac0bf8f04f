"""Autotuner of a batch's launch shapes: the workgroup sizes of the local step
and of the K apply (tets per workgroup), the PD / adjoint iterations issued
between host checks, and graph replay.  Each candidate is timed on the
caller's own workload (a function that runs a few steps of the batch); the
winner is kept in a JSON cache keyed by the batch's shape."""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, Optional

BLOCKS = (64, 128, 256)
CHECKS = ((0, 0), (2, 0), (4, 0), (4, 1), (8, 1))


def batch_key(batch) -> str:
    sizes = sorted((int(sc.info()["n_tets"]), int(sc.info()["n_interface"])) for sc in batch.scenes)
    return f"n{len(sizes)}-tets{sum(a for a, _ in sizes)}-iface{sum(b for _, b in sizes)}"


def _time(run: Callable[[], None], torch, reps: int) -> float:
    run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def autotune(batch, run: Callable[[], None], torch, cache_path: Optional[str] = None, reps: int = 2,
             log: bool = False) -> Dict[str, int]:
    """Coordinate search (local-step workgroup, then K-apply workgroup, then
    host-check chunk and graph replay); applies and returns the best shape."""
    key = batch_key(batch)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            batch.config(**cache[key])
            return cache[key]
    else:
        cache = {}
    cfg = dict(block_local=256, block_applyK=256, iters_per_check=0, use_graph=0)
    timings = {}

    def trial(c):
        batch.config(**c)
        t = _time(run, torch, reps)
        timings[json.dumps(c, sort_keys=True)] = t
        if log:
            print(f"[autotune] {c}: {1e3 * t:.2f} ms", flush=True)
        return t

    for field, values in (("block_local", BLOCKS), ("block_applyK", BLOCKS)):
        best = None
        for v in values:
            c = dict(cfg, **{field: v})
            t = trial(c)
            if best is None or t < best[0]:
                best = (t, v)
        cfg[field] = best[1]
    best = None
    for chunk, graph in CHECKS:
        c = dict(cfg, iters_per_check=chunk, use_graph=graph)
        t = trial(c)
        if best is None or t < best[0]:
            best = (t, c)
    cfg = best[1]
    batch.config(**cfg)
    if cache_path:
        cache[key] = cfg
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return cfg
