"""Autotuner for the brick decomposition and the LDS staging budget.

Each CV pass runs one workgroup per brick of cells and stages the brick's halo
in LDS.  Bigger bricks re-load fewer halo atoms and fill more lanes, but need
more LDS per workgroup (fewer workgroups per CU).  The tuner enumerates the
brick shapes whose expected halo fits a budget, times a few pipeline steps of
each on the real system, and keeps the fastest; results are cached by a key of
the CV kind, precision and atoms per cell.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import replace
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .binding import Params, Pipeline

SLOT_BYTES = {(0, False): 16, (0, True): 80, (1, False): 32, (1, True): 160}  # (precision, has rows)


def cells_per_axis(box: Sequence[float], r_list: float) -> Tuple[int, int, int]:
    return tuple(int(math.floor(b / r_list)) for b in box)


def candidates(n_atoms: int, box: Sequence[float], params: Params, lds_kb: Sequence[int] = (40, 48, 56, 64),
               limit: int = 10) -> List[Tuple[Tuple[int, int, int], int]]:
    """Feasible (brick, lds_kb) pairs, most owned atoms first."""
    nc = cells_per_axis(box, params.r_c + params.skin)
    rho = n_atoms / float(np.prod(nc))
    rec = SLOT_BYTES[(params.precision, params.cv_kind != 1)]
    out = []
    for kb in lds_kb:
        cap = (kb * 1024 - 2048) // rec
        for bx in range(1, min(4, nc[0]) + 1):
            for by in range(1, min(4, nc[1]) + 1):
                for bz in range(1, min(4, nc[2]) + 1):
                    halo = (bx + 2) * (by + 2) * (bz + 2) * rho
                    own = bx * by * bz * rho
                    # slots past the LDS capacity are read from global memory,
                    # so a halo somewhat above the capacity is still a candidate
                    if halo > 1.25 * cap or own > 1.2 * 256:
                        continue
                    out.append(((bx, by, bz), kb, own, halo / own))
    # prefer many owned atoms per workgroup up to one 256-thread pass, then low halo re-loads
    out.sort(key=lambda c: (-min(c[2], 240.0), c[3], c[1]))
    seen, picked = set(), []
    for b, kb, own, ratio in out:
        key = (tuple(sorted(b)), kb)
        if key in seen:
            continue
        seen.add(key)
        picked.append((b, kb))
        if len(picked) >= limit:
            break
    return picked


def _time_steps(pipe: Pipeline, pos4, force4, box, steps: int) -> float:
    import torch

    stream = pipe.stream
    pipe.build_neighbors_checked(pos4, box)
    with torch.cuda.stream(stream):
        pipe.step(pos4, force4)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            pipe.step(pos4, force4)
        e1.record(stream)
        e1.synchronize()
    pipe.check()
    return e0.elapsed_time(e1) / steps


def cache_key(n_atoms: int, box: Sequence[float], params: Params) -> str:
    nc = cells_per_axis(box, params.r_c + params.skin)
    rho = n_atoms / float(np.prod(nc))
    return f"kind{params.cv_kind}-p{params.precision}-rho{rho:.1f}-big{int(n_atoms >= 200000)}"


def autotune(pos4, box, params: Params, steps: int = 3, cache: Optional[str] = None,
             limit: int = 10) -> Tuple[Params, Dict[str, float]]:
    """Return params with the fastest (brick, lds_kb) and the timings (ms/step)."""
    n = pos4.shape[0]
    key = cache_key(n, box, params)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            known = json.load(f)
        if key in known:
            b, kb = known[key]["brick"], known[key]["lds_kb"]
            return replace(params, brick=tuple(b), lds_kb=kb), known[key]["timings"]
    import torch

    timings: Dict[str, float] = {}
    best = None
    force4 = torch.zeros((n, 4), dtype=torch.float64 if params.precision == 1 else torch.float32,
                         device=pos4.device)
    # the library's own choice (brick (0, 0, 0), default LDS budget) is always timed
    trials = [((0, 0, 0), 0)] + [c for c in candidates(n, box, params, limit=limit)
                                 if c != (tuple(params.brick), params.lds_kb)]
    for b, kb in trials:
        trial = replace(params, brick=b, lds_kb=kb)
        pipe = Pipeline(n, trial)
        pipe.hills_set(np.zeros((1, trial.dims)), np.zeros(1))
        try:
            ms = _time_steps(pipe, pos4, force4, box, steps)
        finally:
            pipe.close()
        timings["default" if kb == 0 else f"{b[0]}x{b[1]}x{b[2]}@{kb}KiB"] = ms
        if best is None or ms < best[0]:
            best = (ms, b, kb)
    if best is None:
        return params, timings
    tuned = replace(params, brick=best[1], lds_kb=best[2])
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
        known[key] = {"brick": list(best[1]), "lds_kb": best[2], "timings": timings}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(known, f, indent=1)
        os.replace(tmp, cache)
    return tuned, timings
