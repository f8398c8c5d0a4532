"""The autotuner on the GPU: it times the library's default and the feasible
brick/LDS candidates, caches its choice, and whatever geometry it picks gives
the oracle's CV and forces within the FP32 bars (the geometry changes only the
order of the sums)."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests.helpers import oracle_cvs, params_for, rel_force_err
from tests.test_gpu_parity import Q6CV, run_step

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_choice_cache_and_parity(orc, tmp_path):
    from paper_2510_06873_amd import Pipeline
    from paper_2510_06873_amd.autotune import autotune, candidates

    d = W.wurtzite_slab(nx=8, ny=4, nz=8, seed=5)
    pos, box, sp = d["pos"], d["box"], d["species"]
    n = len(pos)
    prm = params_for(Q6CV, max_neighbors=96)
    p4 = torch.from_numpy(W.as_float4(pos, sp)).to(torch.device("cuda", 0))
    cache = str(tmp_path / "tune.json")
    tuned, timings = autotune(p4, box, prm, steps=1, cache=cache, limit=3)
    assert "default" in timings and len(timings) >= 2 and all(t > 0 for t in timings.values())
    again, timings2 = autotune(p4, box, prm, steps=1, cache=cache, limit=3)
    assert (again.brick, again.lds_kb, again.tpa) == (tuned.brick, tuned.lds_kb, tuned.tpa) and timings2 == timings
    s_ref, g_ref, _ = oracle_cvs(orc, pos, box, Q6CV)
    F_in = W.external_forces(n, seed=9)
    geoms = [tuned] + [dataclasses.replace(prm, brick=b, lds_kb=kb, tpa=t)
                       for b, kb, t in candidates(n, box, prm, limit=3)]
    # every lane count, with the library's brick choice
    geoms += [dataclasses.replace(prm, tpa=t) for t in (1, 2, 4)]
    for trial in geoms:
        s, F = run_step(Pipeline(n, trial), pos, sp, box, F_in, [0.37])
        assert abs(s[0] - s_ref[0]) <= 1e-5 * abs(s_ref[0]), (trial.brick, trial.lds_kb, trial.tpa)
        assert rel_force_err(F[:, :3] - F_in[:, :3].astype(np.float64), -0.37 * g_ref[0]) <= 1e-4, trial.tpa
