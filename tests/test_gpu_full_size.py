"""Parity at the benchmark's full size: 1,024,000 atoms, 50,000 hills, the
launch configuration bench.py times (same parameters, brick choice, stream).

The oracle runs once over the whole system (tens of seconds); the cell list
is compared in full, neighbour rows on a seeded sample of atoms, the CV, the
bias at the GPU's s, and every atom's bias force (seeded with the GPU's dV/ds).
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import rel_force_err

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_wz1m_full_size_parity(orc):
    import bench

    S = bench.setup("wz1m")
    pipe, pos4, stream, n = S["pipe"], S["pos4"], S["stream"], S["n"]
    d = S["d"]
    pos, box = d["pos"], d["box"]
    F_in = S["F"].clone()
    with torch.cuda.stream(stream):
        bench.window(S)  # one full bench window: rebuild, 10 steps, deposit
        pipe.build_neighbors(pos4, box)
        F = F_in.clone()
        F0 = torch.zeros_like(F_in)
        s = pipe.cv_forward(pos4).clone()
        V, dV = pipe.bias_eval(s)
        pipe.cv_backward(pos4)
        pipe.apply_bias_forces(pos4, F, dV)
        pipe.apply_bias_forces(pos4, F0, dV)
        stream.synchronize()
    pipe.check()
    print(f"[full] N={n} s={s.item():.6f}", flush=True)

    # cell list: bit-exact in full
    nc, perm, start = pipe.cell_list()
    onc, _, operm, ostart = orc.cell_list(pos, box, 4.0)
    assert tuple(onc.tolist()) == nc
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(start.cpu().numpy(), ostart)

    # neighbour rows: bit-exact sets on a seeded sample of atoms
    off, nb = orc.neighbors(pos, box, 4.0)
    nbr, cnt = pipe.neighbor_lists()
    nbr, cnt, perm_h = nbr.cpu().numpy(), cnt.cpu().numpy(), perm.cpu().numpy()
    rank_of = np.empty(n, np.int64)
    rank_of[perm_h] = np.arange(n)
    for i in np.random.default_rng(0).choice(n, 4000, replace=False):
        t = rank_of[i]
        got = np.sort(perm_h[nbr[t, :cnt[t]]])
        assert np.array_equal(got, nb[off[i]:off[i + 1]]), i
    print("[full] neighbours ok", flush=True)

    # CV, bias and forces
    prm = orc.q6_params(3.6, 0.2, 0.7, 0.02, 5.5, 0.25)
    nl = (off, nb)
    s_ref = orc.q6_forward(pos, box, nl, prm)["s"]
    assert abs(s.item() - s_ref) <= 1e-5 * abs(s_ref)
    cen, hts = pipe.hills_get()
    Vr, dVr = orc.bias(cen, hts, S["wl"]["sigma"], [s.item()])
    assert abs(V.item() - Vr) <= 1e-12 * Vr
    assert abs(dV.item() - dVr[0]) <= 1e-12 * (abs(dVr[0]) + Vr / S["wl"]["sigma"][0])
    g_ref = orc.q6_gradient(pos, box, nl, prm)
    bias_ref = -dV.item() * g_ref
    # the bias force itself (into a zeroed array)
    err = rel_force_err(F0.cpu().numpy()[:, :3].astype(np.float64), bias_ref)
    print(f"[full] s rel err {abs(s.item() - s_ref) / s_ref:.2e}, dV/ds {dV.item():.3e}, "
          f"max |F_bias| {np.linalg.norm(bias_ref, axis=1).max():.3e}, force err {err:.2e}", flush=True)
    assert err <= 1e-4
    # added in place to N(0, 1) forces: exact up to the FP32 rounding of the stored sum
    Fo = F.cpu().numpy()[:, :3].astype(np.float64)
    Fi = F_in.cpu().numpy()[:, :3].astype(np.float64)
    bmax = np.linalg.norm(bias_ref, axis=1).max()
    assert np.max(np.abs(Fo - Fi - bias_ref)) <= 1e-4 * bmax + 2.0 ** -23 * np.max(np.abs(Fo))
