"""Autotuner for the execution parameters of a plan.

Times forward + adjoint passes of a stack on the device for candidate
settings of the batch budget (``batch_mb``), the number of concurrent
streams (``streams``), the spreading tile shape
(``tile_w`` x ``tile_h``) and the spreading item size (``chunk``), one
parameter at a time (coordinate search from the defaults), and caches the
best setting per geometry and device in a JSON file.  Every candidate
computes the same operator; only the float32 summation order of the
spreading differs.
"""

from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Sequence

import numpy as np
import torch

from .radon import Plan, SliceGeometry

TILES = [(64, 32), (32, 32), (64, 64), (128, 32)]
CHUNKS = [256, 512, 1024]
BUDGETS_MB = [1, 160, 640, 1400, 2048]     # 1 MiB: every slice runs alone
STREAMS = [1, 2, 3, 6]
DEFAULTS = {"tile_w": 64, "tile_h": 32, "chunk": 1024, "batch_mb": 160, "streams": 2}


def default_cache_path() -> str:
    return os.path.join(os.path.expanduser("~"), ".cache", "nufftradon", "autotune.json")


def geometry_key(geoms: Sequence[SliceGeometry], width: int, device: torch.device) -> str:
    h = hashlib.sha1()
    h.update(torch.cuda.get_device_name(device).encode())
    h.update(str(width).encode())
    for g in geoms:
        h.update(np.array([g.n, g.n_det, len(g.angles)], dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(g.angles, dtype=np.float64).tobytes())
    return h.hexdigest()


def _time_pass(plan: Plan, x: torch.Tensor, s: torch.Tensor, g: torch.Tensor, reps: int) -> float:
    plan.fwd(x, s)
    plan.adj(s, g)
    torch.cuda.synchronize(plan.device)
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.fwd(x, s)
        plan.adj(s, g)
    torch.cuda.synchronize(plan.device)
    return (time.perf_counter() - t0) / reps


def autotune(geoms: Sequence[SliceGeometry], width: int = 7, device: torch.device | str | None = None,
             reps: int = 3, cache_path: str | None = None, use_cache: bool = True, verbose: bool = False) -> dict:
    """Best ``tuning`` dict for ``Plan(geoms, tuning=...)`` (measured, then cached)."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    cache_path = cache_path or default_cache_path()
    key = geometry_key(geoms, width, device)
    cache = {}
    if use_cache and os.path.exists(cache_path):
        try:
            with open(cache_path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key]["tuning"])

    plan = Plan(geoms, width=width, device=device, tuning=dict(DEFAULTS))
    gen = torch.Generator(device=device).manual_seed(0)
    x = torch.randn(plan.vol_numel, generator=gen, device=device, dtype=torch.float32)
    s = torch.empty(plan.sino_numel, device=device, dtype=torch.float32)
    g = torch.empty(plan.vol_numel, device=device, dtype=torch.float32)
    best = dict(DEFAULTS)
    best_t = _time_pass(plan, x, s, g, reps)
    trials = [("default", dict(best), best_t)]

    def consider(cand: dict):
        nonlocal best, best_t
        plan.retune(**cand)
        t = _time_pass(plan, x, s, g, reps)
        trials.append((str(cand), dict(cand), t))
        if verbose:
            print(f"[autotune] {cand}: {t * 1e3:.3f} ms")
        if t < best_t:
            best, best_t = dict(cand), t

    for mb in BUDGETS_MB:
        if mb != best["batch_mb"]:
            consider({**best, "batch_mb": mb})
    for ns in STREAMS:
        if ns != best["streams"]:
            consider({**best, "streams": ns})
    for tw, th in TILES:
        if (tw, th) != (best["tile_w"], best["tile_h"]):
            consider({**best, "tile_w": tw, "tile_h": th})
    for ch in CHUNKS:
        if ch != best["chunk"]:
            consider({**best, "chunk": ch})
    plan.retune(**best)

    cache[key] = {"tuning": best, "ms": best_t * 1e3,
                  "trials": [{"name": n, "ms": round(t * 1e3, 4)} for n, _, t in trials]}
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    except OSError:
        pass
    return dict(best)
