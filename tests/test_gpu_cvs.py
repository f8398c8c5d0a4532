"""HIP path of the small CVs and the free-energy estimators against the FP64
oracle on the same seeded inputs.

Bars: CV values 1e-12 (FP64 on both sides from the same FP32 coordinates,
libm vs device transcendental functions); bias forces added to FP32 force
arrays within FP32 rounding of the stored sums (1e-6 relative, norm-wise), to
FP64 arrays 1e-12; periodic hill heights and V 1e-12 relative; free energies
within 1e-10 kBT where finite, +inf in the same bins.
"""
import math

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * math.pi


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    return t.to(device=dev(), dtype=dtype or t.dtype).contiguous()


def test_torsions_and_forces(orc):
    import paper_2510_06873_amd as P

    d = W.peptide_in_solvent()
    pos, box, quads = d["pos"], d["box"], d["quads"]
    n, m = len(pos), len(quads)
    p4 = to_dev(W.as_float4(pos))
    q = to_dev(quads, torch.int32)
    phi = P.torsions(p4, q, box)
    torch.cuda.synchronize()
    phi_ref, g_ref = orc.torsions(pos, box, quads)
    assert np.max(np.abs(phi.cpu().numpy() - phi_ref)) < 1e-12
    dV = np.random.default_rng(1).normal(0.0, 2.0, m)
    ref = np.zeros((n, 3))
    for t in range(m):
        for k in range(4):
            ref[quads[t, k]] -= dV[t] * g_ref[t, k]
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 1e-6)):
        F = torch.zeros((n, 4), dtype=dtype, device=dev())
        P.torsion_forces(p4, q, box, to_dev(dV), F)
        torch.cuda.synchronize()
        got = F.cpu().numpy()[:, :3].astype(np.float64)
        err = np.linalg.norm(got - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max()
        assert err <= tol, (dtype, err)
        assert np.all(F.cpu().numpy()[:, 3] == 0)


def test_torsion_bad_index_gives_nan_and_no_force():
    import paper_2510_06873_amd as P

    d = W.peptide_in_solvent()
    pos, box, quads = d["pos"], d["box"], d["quads"][:3].copy()
    quads[1, 2] = len(pos) + 5  # out of range: never dereferenced
    p4 = to_dev(W.as_float4(pos))
    q = to_dev(quads, torch.int32)
    phi = P.torsions(p4, q, box).cpu().numpy()
    assert np.isfinite(phi[0]) and np.isnan(phi[1]) and np.isfinite(phi[2])
    F = torch.zeros((len(pos), 4), dtype=torch.float64, device=dev())
    P.torsion_forces(p4, q, box, to_dev(np.array([0.0, 1.0, 0.0])), F)
    torch.cuda.synchronize()
    assert float(F.abs().sum()) == 0.0  # torsion 1 skipped, the others have dV = 0


def test_nearest_distance_and_forces(orc):
    import paper_2510_06873_amd as P

    d = W.surface_water()
    pos, box, c, h = d["pos"], d["box"], d["centre"], d["hydrogens"]
    n = len(pos)
    p4 = to_dev(W.as_float4(pos))
    mem = to_dev(h, torch.int32)
    arg = torch.zeros(1, dtype=torch.int32, device=dev())
    s = P.nearest_distance(p4, c, mem, box, nearest=arg)
    torch.cuda.synchronize()
    s_ref, a_ref, u = orc.nearest_distance(pos, box, c, h)
    assert abs(s.item() - s_ref) < 1e-12 and arg.item() == a_ref
    dV = torch.tensor([0.75], dtype=torch.float64, device=dev())
    F = torch.zeros((n, 4), dtype=torch.float64, device=dev())
    P.nearest_distance_forces(p4, c, mem, box, dV, F)
    torch.cuda.synchronize()
    ref = np.zeros((n, 3))
    ref[c] += 0.75 * u
    ref[a_ref] -= 0.75 * u
    assert np.max(np.abs(F.cpu().numpy()[:, :3] - ref)) < 1e-12
    # the centre inside the member set is skipped; a bad member gives NaN
    h2 = np.concatenate([[c], h])
    s2 = P.nearest_distance(p4, c, to_dev(h2, torch.int32), box)
    assert abs(s2.item() - s_ref) < 1e-12
    h3 = h.copy()
    h3[7] = -4
    assert math.isnan(P.nearest_distance(p4, c, to_dev(h3, torch.int32), box).item())


def test_external_context_periodic_hills(orc):
    from paper_2510_06873_amd import CV_EXTERNAL, Params, Pipeline

    kBT = W.KBT_KJMOL
    prm = Params(cv_kind=CV_EXTERNAL, external_dims=2, sigma=[0.35, 0.35], period=[TWO_PI, TWO_PI], w0=1.2,
                 gamma=10.0, kBT=kBT, hill_capacity=512)
    pipe = Pipeline(0, prm)
    cen = W.hill_centres(300, [-math.pi, -math.pi], [math.pi, math.pi], seed=44)
    s = torch.empty(2, dtype=torch.float64, device=dev())
    for k in range(cen.shape[0]):
        s.copy_(torch.as_tensor(cen[k]))
        pipe.deposit_hill(s)
    pipe.check()
    c_gpu, h_gpu = pipe.hills_get()
    h_ref = orc.deposit_sequence(cen, [0.35, 0.35], 1.2, 10.0, kBT, period=[TWO_PI, TWO_PI])
    assert np.array_equal(c_gpu, cen)
    assert np.max(np.abs(h_gpu - h_ref) / h_ref) < 1e-12
    pts = np.array([[math.pi - 0.01, -math.pi + 0.02], [-3.0, 3.1], [0.3, -0.7], [math.pi, math.pi]])
    for x in pts:
        V, dV = pipe.bias_eval(to_dev(x))
        Vr, dVr = orc.bias(cen, h_ref, [0.35, 0.35], x, period=[TWO_PI, TWO_PI])
        assert abs(V.item() - Vr) <= 1e-12 * Vr
        assert np.max(np.abs(dV.cpu().numpy() - dVr)) <= 1e-12 * (np.abs(dVr).max() + Vr / 0.35)
    # the atom calls are not for this kind of context
    from paper_2510_06873_amd import GmError
    with pytest.raises(GmError):
        pipe.deposit_hill()  # no forward pass to take s from
    # free energy from the hills on a 64 x 48 grid
    lo, hi, nb = [-math.pi, -math.pi], [math.pi, math.pi], [64, 48]
    F = pipe.fes_hills(lo, hi, nb).cpu().numpy()
    Fr = orc.fes_hills(cen, h_ref, [0.35, 0.35], lo, hi, nb, gamma=10.0, period=[TWO_PI, TWO_PI])
    assert np.max(np.abs(F - Fr)) <= 1e-12 * np.abs(Fr).max()


@pytest.mark.parametrize("dims,nb", [(2, [72, 60]), (1, [20000])])
def test_fes_reweight(orc, dims, nb):
    import paper_2510_06873_amd as P

    s, V = W.biased_trace(T=200000, dims=dims, seed=45 + dims)
    kBT = W.KBT_KJMOL
    lo = [-math.pi] * dims
    hi = [math.pi] * dims
    F = P.fes_reweight(to_dev(s), to_dev(V), lo, hi, nb, kBT).cpu().numpy()
    Fr = orc.fes_reweight(s, V, lo, hi, nb, kBT)
    fin = np.isfinite(Fr)
    assert np.array_equal(np.isfinite(F), fin)
    assert fin.sum() > 0.5 * fin.size
    assert np.max(np.abs(F[fin] - Fr[fin])) <= 1e-10 * kBT
