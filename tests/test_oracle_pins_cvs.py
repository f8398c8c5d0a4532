"""Pins of the oracle's other CVs and free-energy estimators against facts
other than their own formulas: constructed torsions of known angle, finite
differences, invariances, a k-d tree, closed forms for periodic hills and for
reweighted histograms."""
import math

import numpy as np
import pytest

TWO_PI = 2.0 * math.pi


def _wrap(a):
    return (a + math.pi) % TWO_PI - math.pi


# ---------------------------------------------------------------------------
# Torsion angles (alanine dipeptide Phi/Psi)
# ---------------------------------------------------------------------------
def _quad_at(theta, origin=(0.0, 0.0, 0.0)):
    """Four atoms with torsion theta by construction: x2 at the origin, x3 on
    +z, x1's projection on +x, x4's projection at angle theta counterclockwise
    about +z (the bond x2->x3).  Components along the axis do not change the
    angle."""
    o = np.asarray(origin, np.float64)
    x1 = o + [1.2, 0.0, -0.4]
    x2 = o + [0.0, 0.0, 0.0]
    x3 = o + [0.0, 0.0, 1.5]
    x4 = o + [1.3 * math.cos(theta), 1.3 * math.sin(theta), 1.9]
    return np.stack([x1, x2, x3, x4])


@pytest.mark.parametrize("deg", [-179.0, -120.0, -60.0, -1e-3, 0.0, 1e-3, 45.0, 90.0, 150.0, 180.0])
def test_torsion_constructed_angles(orc, deg):
    # IUPAC: looking along x2 -> x3, x1 turned clockwise by phi eclipses x4
    theta = math.radians(deg)
    box = np.array([30.0, 30.0, 30.0])
    pos = _quad_at(theta, origin=(5.0, 6.0, 7.0))
    phi, _ = orc.torsions(pos, box, [[0, 1, 2, 3]])
    assert abs(_wrap(phi[0] - theta)) < 1e-12
    # the same molecule wrapped across the faces of the box (minimum images)
    phi2, _ = orc.torsions((pos - [5.0, 6.0, 7.4]) % box, box, [[0, 1, 2, 3]])
    assert abs(_wrap(phi2[0] - theta)) < 1e-12


def _random_quads(rng, n_atoms, m):
    return np.stack([rng.choice(n_atoms, 4, replace=False) for _ in range(m)]).astype(np.int32)


def test_torsion_gradient_finite_differences(orc):
    rng = np.random.default_rng(1)
    box = np.array([12.0, 13.0, 14.0])
    pos = rng.random((30, 3)) * box
    quads = _random_quads(rng, 30, 12)
    phi, g = orc.torsions(pos, box, quads)
    h = 1e-5
    for t in range(quads.shape[0]):
        for k in range(4):
            for a in range(3):
                def f(dx):
                    p = pos.copy()
                    p[quads[t, k], a] += dx
                    return orc.torsions(p, box, quads[t:t + 1])[0][0]
                d1 = _wrap(f(h) - f(-h)) / (2 * h)
                d2 = _wrap(f(h / 2) - f(-h / 2)) / h
                fd = (4 * d2 - d1) / 3  # Richardson
                assert abs(fd - g[t, k, a]) <= 1e-7 * max(1.0, abs(g[t, k, a])), (t, k, a)


def test_torsion_invariances(orc):
    rng = np.random.default_rng(2)
    box = np.array([40.0, 40.0, 40.0])
    pos = 15.0 + rng.random((20, 3)) * 8.0
    quads = _random_quads(rng, 20, 10)
    phi, g = orc.torsions(pos, box, quads)
    # rigid rotation about the centre: same angles
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    c = pos.mean(0)
    phi_r, _ = orc.torsions((pos - c) @ q.T + c, box, quads)
    assert np.max(np.abs(_wrap(phi_r - phi))) < 1e-12
    # a mirror image flips every sign
    phi_m, _ = orc.torsions(pos * [-1.0, 1.0, 1.0] + [40.0, 0.0, 0.0], box, quads)
    assert np.max(np.abs(_wrap(phi_m + phi))) < 1e-12
    # no net force and no net torque from a torsion
    x = pos[quads]  # (m, 4, 3)
    assert np.max(np.abs(g.sum(1))) < 1e-12
    assert np.max(np.abs(np.cross(x, g).sum(1))) < 1e-10


# ---------------------------------------------------------------------------
# Distance to the nearest atom of a set (rutile surface O - nearest H)
# ---------------------------------------------------------------------------
def test_nearest_distance_against_kdtree(orc):
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(3)
    box = np.array([20.0, 18.0, 25.0])
    pos = rng.random((600, 3)) * box
    members = np.sort(rng.choice(600, 150, replace=False)).astype(np.int32)
    tree = cKDTree(pos[members], boxsize=box)
    for centre in rng.choice(600, 40, replace=False):
        s, arg, u = orc.nearest_distance(pos, box, centre, members)
        dd, ii = tree.query(pos[centre], k=2)
        k = 1 if members[ii[0]] == centre else 0
        assert abs(s - dd[k]) < 1e-12
        assert arg == members[ii[k]]
        assert abs(np.linalg.norm(u) - 1.0) < 1e-12


def test_nearest_distance_hand_case(orc):
    box = np.array([10.0, 10.0, 10.0])
    pos = np.array([[0.5, 5.0, 5.0],   # centre
                    [9.7, 5.0, 5.0],   # 0.8 across the x face
                    [0.5, 6.0, 5.0],   # 1.0
                    [3.0, 5.0, 5.0]])  # 2.5
    s, arg, u = orc.nearest_distance(pos, box, 0, [0, 3, 2, 1])  # the centre itself is skipped
    assert abs(s - 0.8) < 1e-12 and arg == 1
    assert np.allclose(u, [-1.0, 0.0, 0.0], atol=1e-12)


# ---------------------------------------------------------------------------
# Periodic hills
# ---------------------------------------------------------------------------
def test_periodic_hill_across_the_boundary(orc):
    h, sigma = 1.7, 0.35
    c = np.array([math.pi - 0.05])
    s = -math.pi + 0.05  # 0.1 ahead of the centre through the boundary
    V, dV = orc.bias(c, [h], [sigma], [s], period=[TWO_PI])
    e = h * math.exp(-0.1 ** 2 / (2 * sigma ** 2))
    assert abs(V - e) < 1e-14
    assert abs(dV[0] - (-e * 0.1 / sigma ** 2)) < 1e-13
    # without the period the hill is a whole turn away
    V0, _ = orc.bias(c, [h], [sigma], [s])
    assert V0 < 1e-30


def test_periodic_bias_is_periodic_and_matches_images(orc):
    rng = np.random.default_rng(4)
    sigma = [0.35, 0.35]
    cen = rng.uniform(-math.pi, math.pi, (300, 2))
    hts = rng.uniform(0.5, 1.5, 300)
    for s in rng.uniform(-math.pi, math.pi, (20, 2)):
        V, dV = orc.bias(cen, hts, sigma, s, period=[TWO_PI, TWO_PI])
        V2, dV2 = orc.bias(cen, hts, sigma, s + [TWO_PI, -TWO_PI], period=[TWO_PI, TWO_PI])
        assert abs(V - V2) <= 1e-12 * V and np.max(np.abs(dV - dV2)) <= 1e-11 * (1 + np.abs(dV).max())
        # brute force over the 9 nearest images of every hill (sigma << 2 pi)
        Vb = 0.0
        for kx in (-1, 0, 1):
            for ky in (-1, 0, 1):
                x = s - (cen + [kx * TWO_PI, ky * TWO_PI])
                Vb += np.sum(hts * np.exp(-np.sum(x * x, 1) / (2 * 0.35 ** 2)))
        assert abs(V - Vb) <= 1e-10 * Vb


def test_periodic_deposit_sequence(orc):
    rng = np.random.default_rng(5)
    cen = rng.uniform(-math.pi, math.pi, (50, 2))
    h = orc.deposit_sequence(cen, [0.35, 0.35], 1.2, 10.0, 2.494, period=[TWO_PI, TWO_PI])
    for k in range(50):
        V, _ = orc.bias(cen[:k], h[:k], [0.35, 0.35], cen[k], period=[TWO_PI, TWO_PI])
        assert abs(h[k] - 1.2 * math.exp(-V / (2.494 * 9.0))) <= 1e-14


# ---------------------------------------------------------------------------
# Free energy by reweighting and from the hills
# ---------------------------------------------------------------------------
def _bins(s, lo, hi, nb):
    w = (hi - lo) / nb
    return np.floor((s - lo) / w)


def test_fes_reweight_unbiased_is_the_histogram(orc):
    rng = np.random.default_rng(6)
    s = rng.normal(0.0, 1.0, 20000)
    kBT = 2.5
    F = orc.fes_reweight(s, np.zeros_like(s), -3.0, 3.0, 30, kBT)
    b = _bins(s, -3.0, 3.0, 30)
    counts = np.array([np.sum(b == i) for i in range(30)])
    ref = np.where(counts > 0, -kBT * np.log(np.maximum(counts, 1) / len(s)), np.inf)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(F), fin)
    assert np.max(np.abs(F[fin] - ref[fin])) < 1e-12


def test_fes_reweight_two_states_closed_form(orc):
    kBT = 2.494
    nA, nB, VA, VB = 300, 700, 4.0, 1.0
    s = np.concatenate([np.full(nA, 0.25), np.full(nB, 0.75), np.full(50, 3.0)])  # 50 outside the grid
    V = np.concatenate([np.full(nA, VA), np.full(nB, VB), np.full(50, 2.0)])
    F = orc.fes_reweight(s, V, 0.0, 1.0, 2, kBT)
    wA, wB, wO = nA * math.exp(VA / kBT), nB * math.exp(VB / kBT), 50 * math.exp(2.0 / kBT)
    assert abs(F[0] + kBT * math.log(wA / (wA + wB + wO))) < 1e-12
    assert abs(F[1] + kBT * math.log(wB / (wA + wB + wO))) < 1e-12
    # a constant added to the bias cancels
    F2 = orc.fes_reweight(s, V + 123.0, 0.0, 1.0, 2, kBT)
    assert np.max(np.abs(F2 - F)) < 1e-12


def test_fes_reweight_2d_bin_layout(orc):
    # one sample per chosen bin: bin id i0 + nb0 i1
    s = np.array([[0.05, 0.05], [0.95, 0.05], [0.05, 0.95], [0.55, 0.45]])
    F = orc.fes_reweight(s, np.zeros(4), [0.0, 0.0], [1.0, 1.0], [10, 5], 1.0)
    hit = np.flatnonzero(np.isfinite(F))
    assert list(hit) == sorted([0, 9, 40, 5 + 10 * 2])
    assert np.allclose(F[hit], -math.log(0.25), atol=1e-15)


def test_fes_hills_closed_form(orc):
    h, sigma, c = 1.3, 0.2, 0.4
    lo, hi, nb = 0.0, 1.0, 10
    g = lo + (np.arange(nb) + 0.5) * ((hi - lo) / nb)
    ref = -h * np.exp(-(g - c) ** 2 / (2 * sigma ** 2))
    assert np.max(np.abs(orc.fes_hills([c], [h], [sigma], lo, hi, nb) - ref)) < 1e-15
    assert np.max(np.abs(orc.fes_hills([c], [h], [sigma], lo, hi, nb, gamma=10.0) - ref * 10.0 / 9.0)) < 1e-14
