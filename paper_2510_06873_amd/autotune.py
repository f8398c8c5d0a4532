"""Autotuner for the brick decomposition, the LDS staging budget and the
lanes per atom.

Each CV pass runs one workgroup per brick of cells and stages the brick's halo
in LDS.  Bigger bricks re-load fewer halo atoms and fill more lanes, but need
more LDS per workgroup (fewer workgroups per CU); more lanes per atom split
each neighbour row over more lanes (more parallelism per brick, shorter rows
per lane, more combining of partial sums).  The tuner enumerates the brick
shapes whose expected halo fits a budget with the lane counts that fit a
workgroup, times a few pipeline steps of each on the real system, and keeps
the fastest; results are cached by a key of the CV kind, precision, atoms per
cell and size class (``size_class``), so that walkers of one class in a
serving loop share a tuning.
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


# lanes of one CV-pass workgroup (FP32, FP64)
BLOCK = {0: 512, 1: 256}


def candidates(n_atoms: int, box: Sequence[float], params: Params, lds_kb: Sequence[int] = (40, 48, 56, 64),
               limit: int = 10, tpas: Sequence[int] = (1, 2, 4)) -> List[Tuple[Tuple[int, int, int], int, int]]:
    """Feasible (brick, lds_kb, lanes per atom) triples, most busy lanes first."""
    nc = cells_per_axis(box, params.r_c + params.skin)
    rho = n_atoms / float(np.prod(nc))
    rec = SLOT_BYTES[(params.precision, params.cv_kind != 1)]
    blk = BLOCK[params.precision]
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
                    if halo > 1.25 * cap:
                        continue
                    for tpa in tpas:
                        # at most about one workgroup's worth of lanes
                        if own * tpa > 1.2 * blk:
                            continue
                        out.append(((bx, by, bz), kb, tpa, own * tpa, halo / own))
    # prefer many busy lanes per workgroup up to one pass over the workgroup,
    # then low halo re-loads, fewer lanes per atom, then the smaller budget
    out.sort(key=lambda c: (-min(c[3], 0.94 * blk), c[4], c[2], c[1]))
    seen, picked = set(), []
    for b, kb, tpa, lanes, ratio in out:
        key = (tuple(sorted(b)), kb, tpa)
        if key in seen:
            continue
        seen.add(key)
        picked.append((b, kb, tpa))
        if len(picked) >= limit:
            break
    return picked


def size_class(n_atoms: int) -> int:
    """Walker size class for tuning: 0 below 4,000 atoms, 1 below 32,000,
    2 below 200,000, 3 above."""
    return 0 if n_atoms < 4000 else (1 if n_atoms < 32000 else (2 if n_atoms < 200000 else 3))


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
    return f"kind{params.cv_kind}-p{params.precision}-rho{rho:.1f}-rc{params.r_c:g}-size{size_class(n_atoms)}"


def autotune(pos4, box, params: Params, steps: int = 3, cache: Optional[str] = None,
             limit: int = 10, lds_kb: Sequence[int] = (40, 48, 56, 64)) -> Tuple[Params, Dict[str, float]]:
    """Return params with the fastest (brick, lds_kb, tpa) and the timings
    (ms/step); lds_kb: the staging budgets (KiB) the candidates may use."""
    n = pos4.shape[0]
    key = cache_key(n, box, params)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            known = json.load(f)
        if key in known:
            e = known[key]
            return replace(params, brick=tuple(e["brick"]), lds_kb=e["lds_kb"], tpa=e.get("tpa", 0)), e["timings"]
    import torch

    timings: Dict[str, float] = {}
    best = None
    force4 = torch.zeros((n, 4), dtype=torch.float64 if params.precision == 1 else torch.float32,
                         device=pos4.device)
    # the library's own choice (brick (0, 0, 0), default LDS budget and lanes) is always timed
    trials = [((0, 0, 0), 0, 0)] + [c for c in candidates(n, box, params, lds_kb=lds_kb, limit=limit)
                                    if c != (tuple(params.brick), params.lds_kb, params.tpa)]
    for b, kb, tpa in trials:
        trial = replace(params, brick=b, lds_kb=kb, tpa=tpa)
        pipe = Pipeline(n, trial)
        pipe.hills_set(np.zeros((1, trial.dims)), np.zeros(1))
        try:
            ms = _time_steps(pipe, pos4, force4, box, steps)
        finally:
            pipe.close()
        timings["default" if kb == 0 else f"{b[0]}x{b[1]}x{b[2]}@{kb}KiB/tpa{tpa}"] = ms
        if best is None or ms < best[0]:
            best = (ms, b, kb, tpa)
    if best is None:
        return params, timings
    tuned = replace(params, brick=best[1], lds_kb=best[2], tpa=best[3])
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
        known[key] = {"brick": list(best[1]), "lds_kb": best[2], "tpa": best[3], "timings": timings}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(known, f, indent=1)
        os.replace(tmp, cache)
    return tuned, timings
