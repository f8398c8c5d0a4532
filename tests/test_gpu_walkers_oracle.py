"""Batched and served walkers against the FP64 oracle.

The batch and serving tests elsewhere show that a walker's results are bitwise
the same alone and in the mix; these tests anchor the mix itself to the
oracle, for each of the four walker kinds (fcc / wurtzite x coordination /
q6 count, FP32), including the FP32 coordination-only kernels.

Stage-wise parity (the oracle's bias and forces use the CV value the GPU
reported, as in the single-walker tests): the CV is checked against the
oracle's at 1e-5 relative, V and dV/ds against the oracle's hill sum at that
CV at 1e-12, and the bias force F_out - F_in against -sum_t dV_t ds/dx of the
oracle norm-wise at 1e-4.  External forces are zero here so that the FP32
force array holds the bias part alone (a unit-size external force would bury
a small bias force under its own rounding).
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import rel_force_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KINDS = (("fcc", "coord"), ("fcc", "q6"), ("wz", "coord"), ("wz", "q6"))


def walker_params(kind, cv, k_hills):
    from paper_2510_06873_amd import CV_COORD, CV_Q6COUNT, FP32, Params

    p = W.WALKER_CV[(kind, cv)]
    return Params(cv_kind=CV_COORD if cv == "coord" else CV_Q6COUNT, precision=FP32, r_c=p["r_c"], skin=p["skin"],
                  taper=p["taper"], cn_r0=p["cn_r0"], sigma=p["sigma"], w0=W.W0_EV, gamma=10.0, kBT=W.KBT_EV,
                  hill_capacity=k_hills + 16, max_neighbors=p["kmax"])


def walker_geometry(kind, n, seed):
    """fcc with 0.2 A jitter (about 2% of the atoms below the crystalline
    threshold; at the serving recipe's 0.1 A every c_i saturates and the q6
    force is near 1e-9) and wurtzite slabs with a random half, so that q6
    walkers have atoms off the saturated ends of the sigmoids."""
    if kind == "fcc":
        d = W.fcc_jittered(n=max(6, round((n / 4) ** (1 / 3))), jitter=0.2, seed=seed)
        return d["pos"], d["species"], d["box"]
    side = (n / 0.08745) ** (1 / 3)
    nx, ny, nz = max(4, round(side / 3.19)), max(3, round(side / (3.19 * np.sqrt(3)))), max(3, round(side / 5.19))
    d = W.wurtzite_slab(nx, ny, nz, seed=seed)
    return d["pos"], d["species"], d["box"]


def oracle_cv(orc, kind, cv, pos, box):
    """(s, ds/dx) of the oracle for a walker kind."""
    p = W.WALKER_CV[(kind, cv)]
    nl = orc.neighbors(pos, box, p["r_c"] + p["skin"])
    if cv == "coord":
        return orc.cn_forward(pos, box, nl, p["cn_r0"], p["r_c"]), orc.cn_gradient(pos, box, nl, p["cn_r0"], p["r_c"])
    prm = orc.q6_params(p["r_c"], p["taper"], 0.7, 0.02, 5.5, 0.25)
    return orc.q6_forward(pos, box, nl, prm)["s"], orc.q6_gradient(pos, box, nl, prm)


def replay(orc, s_gpu, centres, heights, sigma, steps, pace, grad):
    """The oracle's bias history of a walker stepped `steps` times at fixed
    positions with a well-tempered deposit after every `pace`-th step:
    (V and dV/ds of the last step, summed bias force, the hills)."""
    c = [list(x) for x in np.atleast_2d(centres)]
    h = list(heights)
    F = np.zeros_like(grad)
    for t in range(steps):
        V, dV = orc.bias(c, h, sigma, [s_gpu])
        F -= dV[0] * grad
        if (t + 1) % pace == 0:
            h.append(orc.wt_height(W.W0_EV, 10.0, W.KBT_EV, V))
            c.append([s_gpu])
    return V, dV[0], F, (np.array(c), np.array(h))


def check_walker(tag, s_gpu, s_ref, V_gpu, dV_gpu, V_ref, dV_ref, sigma, Fb_gpu, Fb_ref):
    assert abs(s_gpu - s_ref) <= 1e-5 * abs(s_ref), (tag, s_gpu, s_ref)
    assert abs(V_gpu - V_ref) <= 1e-12 * abs(V_ref), (tag, V_gpu, V_ref)
    # dV/ds against its natural scale V/sigma (it crosses zero between hills)
    assert abs(dV_gpu - dV_ref) <= 1e-12 * (abs(dV_ref) + abs(V_ref) / sigma), (tag, dV_gpu, dV_ref)
    assert np.linalg.norm(Fb_ref, axis=1).max() > 0, tag
    err = rel_force_err(Fb_gpu, Fb_ref)
    assert err <= 1e-4, (tag, err)
    return err


def test_batch_of_all_walker_kinds_matches_oracle(orc):
    """One Batch with the four walker kinds at uneven sizes: build, step,
    deposit, step; every walker's CV, V, dV/ds, bias force and hills against
    the oracle."""
    from paper_2510_06873_amd import Batch, Pipeline

    dev = torch.device("cuda", 0)
    sizes = {("fcc", "coord"): 2048, ("fcc", "q6"): 1400, ("wz", "coord"): 3000, ("wz", "q6"): 2600}
    pipes, pos, forces, ref = [], [], [], []
    for k, (kind, cv) in enumerate(KINDS):
        x, sp, box = walker_geometry(kind, sizes[(kind, cv)], seed=300 + k)
        s_ref, g_ref = oracle_cv(orc, kind, cv, x.astype(np.float64), box)
        sigma = W.WALKER_CV[(kind, cv)]["sigma"][0]
        rng = np.random.default_rng(400 + k)
        cen = s_ref + rng.uniform(-2 * sigma, 2 * sigma, (40, 1))
        hts = W.W0_EV * rng.uniform(0.2, 1.0, 40)
        pipe = Pipeline(len(x), walker_params(kind, cv, 40))
        pipe.hills_set(cen, hts)
        pipes.append(pipe)
        pos.append(torch.from_numpy(W.as_float4(x, sp)).to(dev))
        forces.append(torch.zeros((len(x), 4), dtype=torch.float32, device=dev))
        ref.append((x, box, s_ref, g_ref, cen, hts, sigma))
    batch = Batch(pipes, pos, forces)
    batch.build([r[1] for r in ref])
    batch.step()
    batch.deposit()
    batch.step()
    s, V = batch.values()
    dV = batch.gradients()
    torch.cuda.synchronize()
    for k, (kind, cv) in enumerate(KINDS):
        tag = f"{kind}/{cv}"
        assert pipes[k].status(True) == 0, tag
        x, box, s_ref, g_ref, cen, hts, sigma = ref[k]
        s_gpu = s[k, 0].item()
        V_ref, dV_ref, Fb_ref, (c_ref, h_ref) = replay(orc, s_gpu, cen, hts, [sigma], steps=2, pace=1, grad=g_ref)
        # the replay deposits after both steps; the batch deposited after the first only
        c_ref, h_ref = c_ref[:-1], h_ref[:-1]
        Fb = forces[k].cpu().numpy()[:, :3].astype(np.float64)
        check_walker(tag, s_gpu, s_ref, V[k].item(), dV[k, 0].item(), V_ref, dV_ref, sigma, Fb, Fb_ref)
        c_gpu, h_gpu = pipes[k].hills_get()
        assert np.array_equal(c_gpu, c_ref), tag  # the new hill sits at the GPU's CV value
        assert np.max(np.abs(h_gpu - h_ref) / h_ref) <= 1e-12, tag
    batch.close()
    for p in pipes:
        p.close()


def test_fp32_coordination_walker_matches_oracle(orc):
    """The FP32 coordination-only path on its own (the 864-atom fcc system of
    the FP64 coordination test, computed in FP32): CV at 1e-5 and the bias
    force at 1e-4 of the oracle's."""
    from paper_2510_06873_amd import Pipeline

    from tests.helpers import params_for

    dev = torch.device("cuda", 0)
    wl = dict(W.WORKLOADS["fcc864"], precision="fp32")
    d = W.structure(wl["structure"])
    x, box = d["pos"], d["box"]
    pos = x.astype(np.float64)
    nl = orc.neighbors(pos, box, wl["r_c"] + wl["skin"])
    s_ref = orc.cn_forward(pos, box, nl, wl["cn_r0"], wl["r_c"])
    g_ref = orc.cn_gradient(pos, box, nl, wl["cn_r0"], wl["r_c"])
    pipe = Pipeline(len(x), params_for(wl, max_neighbors=128))
    rng = np.random.default_rng(17)
    cen = s_ref + rng.uniform(-0.3, 0.3, (60, 1))
    hts = wl["w0"] * rng.uniform(0.2, 1.0, 60)
    pipe.hills_set(cen, hts)
    p4 = torch.from_numpy(W.as_float4(x)).to(dev)
    F = torch.zeros((len(x), 4), dtype=torch.float32, device=dev)
    pipe.build_neighbors_checked(p4, box)
    pipe.step(p4, F)
    torch.cuda.synchronize()
    assert pipe.status(True) == 0
    s_gpu = pipe.s.item()
    V_ref, dV_ref = orc.bias(cen, hts, wl["sigma"], [s_gpu])
    Fb = F.cpu().numpy()[:, :3].astype(np.float64)
    check_walker("fcc864/fp32", s_gpu, s_ref, pipe.V.item(), pipe.dVds.item(), V_ref, dV_ref[0], wl["sigma"][0], Fb,
                 -dV_ref[0] * g_ref)
    pipe.close()


def test_served_walkers_match_oracle(orc):
    """Continuous batching of requests of every walker kind (plus fillers, so
    that walkers join and leave the mix mid-run): each served walker's CV,
    bias and accumulated bias force over its steps, with its rebuilds and
    well-tempered deposits, against the oracle's replay of the same history."""
    from paper_2510_06873_amd.serving import Request, serve_batched

    sizes = {("fcc", "coord"): 1800, ("fcc", "q6"): 1200, ("wz", "coord"): 2500, ("wz", "q6"): 3200}
    reqs, ref = [], {}
    rid = 0
    for rep in range(2):
        for k, (kind, cv) in enumerate(KINDS):
            x, sp, box = walker_geometry(kind, sizes[(kind, cv)] // (rep + 1), seed=500 + 10 * rep + k)
            rng = np.random.default_rng(600 + rid)
            kh = int(rng.integers(20, 200))
            p = W.WALKER_CV[(kind, cv)]
            sigma = p["sigma"][0]
            if rep == 0:
                s_ref, g_ref = oracle_cv(orc, kind, cv, x.astype(np.float64), box)
                cen = s_ref + rng.uniform(-3 * sigma, 3 * sigma, (kh, 1))
                ref[rid] = (kind, cv, s_ref, g_ref, sigma)
            else:
                hi = (14.0 if kind == "fcc" else 8.0) if cv == "coord" else 1.05 * len(x)
                cen = rng.uniform(0.0, hi, (kh, 1))
            hts = W.W0_EV * rng.uniform(0.2, 1.0, kh)
            zero = np.zeros((len(x), 4), np.float32)
            r = Request(rid, 0.002 * rid, W.as_float4(x, sp), box, walker_params(kind, cv, kh + 8), cen, hts, zero,
                        steps=23 + 3 * k, pace=10)
            reqs.append((r, cen, hts))
            rid += 1
    results, stats = serve_batched([r for r, _, _ in reqs], hbm_budget=64 << 30, max_slots=3, keep_forces=True)
    assert len(results) == len(reqs)
    by_id = {r.rid: r for r in results}
    for r, cen, hts in reqs:
        if r.rid not in ref:
            continue
        kind, cv, s_ref, g_ref, sigma = ref[r.rid]
        res = by_id[r.rid]
        s_gpu = float(res.s[0])
        V_ref, dV_ref, Fb_ref, _ = replay(orc, s_gpu, cen, hts, [sigma], steps=r.steps, pace=r.pace, grad=g_ref)
        # the served result carries V of the last step; dV/ds is checked through the force sum
        assert abs(res.V - V_ref) <= 1e-12 * abs(V_ref), (kind, cv, res.V, V_ref)
        assert abs(s_gpu - s_ref) <= 1e-5 * abs(s_ref), (kind, cv, s_gpu, s_ref)
        err = rel_force_err(res.forces[:, :3], Fb_ref)
        assert err <= 1e-4, (kind, cv, err)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
