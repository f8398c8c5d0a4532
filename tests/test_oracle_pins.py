"""Pins of the FP64 oracle against what the mathematics and the literature fix.

None of these re-types an oracle formula: each compares the oracle with an
independent route (a library routine, a published table, a closed-form lattice
sum, an identity such as the Legendre addition theorem, finite differences,
symmetry, or a high-precision replay).
"""
import json
import os

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
Q6CV = dict(r_c=3.6, taper=0.2, bond_d0=0.7, bond_w=0.02, count_n0=5.5, count_w=0.25)


def rand_units(n, seed):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# Spherical harmonics: the library routine (scipy) is the reference.
# --------------------------------------------------------------------------
def test_ylm6_matches_scipy(orc):
    for u in rand_units(200, 1):
        theta = np.arccos(np.clip(u[2], -1, 1))
        phi = np.arctan2(u[1], u[0])
        ref = np.array([sph_harm_y(6, m, theta, phi) for m in range(7)])
        got = orc.ylm6_complex(u)
        assert np.max(np.abs(got - ref)) < 1e-13


def test_ylm6_real_vector_dot_is_complex_sum(orc):
    """v(u).v(w) = sum_{m=-6..6} Y_6m(u) conj(Y_6m(w)) = 13/(4 pi) P_6(u.w)."""
    us, ws = rand_units(100, 2), rand_units(100, 3)
    for u, w in zip(us, ws):
        lhs = orc.ylm6_real(u) @ orc.ylm6_real(w)
        rhs = 13.0 / (4 * np.pi) * eval_legendre(6, u @ w)
        assert abs(lhs - rhs) < 1e-13


# --------------------------------------------------------------------------
# Steinhardt q6 of ideal clusters: published values.
# --------------------------------------------------------------------------
def _lattice(kind):
    if kind == "fcc":
        pos, box = W.fcc_ideal(4, 3.615)
        return pos, box, 3.2
    if kind == "sc":
        a, n = 2.5, 5
        g = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3) * a
        return g.astype(float), np.array([n * a] * 3), 3.0
    if kind == "bcc":
        a, n = 3.0, 5
        g = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3) * a
        return np.concatenate([g, g + a / 2]).astype(float), np.array([n * a] * 3), 3.6
    if kind == "hcp":
        a = 2.5
        c = a * np.sqrt(8.0 / 3.0)
        cell, sp, L = W.wurtzite_ortho_cell(a, c, 0.0)
        cell = cell[sp == 0]  # the cation sublattice of wurtzite is hcp
        nx, ny, nz = 6, 4, 4
        g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
        pos = (g[:, None, :] * L + cell[None]).reshape(-1, 3)
        return pos, L * np.array([nx, ny, nz]), 3.0
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["fcc", "hcp", "bcc", "sc"])
def test_steinhardt_lattices(orc, kind):
    gold = json.load(open(os.path.join(HERE, "golden", "steinhardt_q6.json")))
    pos, box, rc = _lattice(kind)
    nl = orc.neighbors(pos, box, rc + 0.4)
    out = orc.q6_forward(pos, box, nl, orc.q6_params(rc, 0.2, 0.7, 0.02, 5.5, 0.25))
    want = gold["Q6"][kind]
    assert np.all(np.abs(out["q6"] - want) < 0.6 * 10.0 ** -gold["printed_decimals"])


def test_steinhardt_icosahedron(orc):
    gold = json.load(open(os.path.join(HERE, "golden", "steinhardt_q6.json")))
    phi = (1 + 5 ** 0.5) / 2
    v = []
    for s1 in (-1, 1):
        for s2 in (-1, 1):
            v += [(0, s1, s2 * phi), (s1, s2 * phi, 0), (s2 * phi, 0, s1)]
    v = np.array(v, float)
    v = 2.5 * v / np.linalg.norm(v, axis=1, keepdims=True)
    box = np.array([40.0, 40.0, 40.0])
    pos = np.concatenate([[[20.0, 20.0, 20.0]], 20.0 + v])
    nl = orc.neighbors(pos, box, 3.0)
    out = orc.q6_forward(pos, box, nl, orc.q6_params(2.6, 0.05, 0.7, 0.02, 5.5, 0.25))
    assert abs(out["q6"][0] - gold["Q6"]["icosahedron"]) < 0.6e-5


def test_sc_q6_closed_form(orc):
    """Six axis neighbours: Q6^2 = (1/36)(12 P6(1) + 24 P6(0)) = 1/8 exactly."""
    pos, box, rc = _lattice("sc")
    nl = orc.neighbors(pos, box, rc + 0.4)
    out = orc.q6_forward(pos, box, nl, orc.q6_params(rc, 0.2, 0.7, 0.02, 5.5, 0.25))
    assert np.max(np.abs(out["q6"] - np.sqrt(1 / 8))) < 1e-13


# --------------------------------------------------------------------------
# Addition theorem: |Q_i|^2 and the bond dots from Legendre polynomials only.
# --------------------------------------------------------------------------
def _taper(r, rc, D):
    return np.where(r <= rc - D, 1.0, np.where(r < rc, 0.5 * (1 + np.cos(np.pi * (r - rc + D) / D)), 0.0))


def _shell(pos, box, i, rc):
    d = pos - pos[i]
    d -= box * np.rint(d / box)
    r = np.linalg.norm(d, axis=1)
    m = (r < rc) & (np.arange(len(pos)) != i)
    return d[m] / r[m, None], r[m]


def test_qnorm_and_dots_by_addition_theorem(orc):
    d = W.small_wurtzite_slab()
    pos, box = d["pos"].astype(np.float64), d["box"]
    nl = orc.neighbors(pos, box, 4.0)
    out = orc.q6_forward(pos, box, nl, orc.q6_params(**Q6CV))
    rng = np.random.default_rng(5)
    for i in rng.choice(len(pos), 40, replace=False):
        ui, ri = _shell(pos, box, i, 3.6)
        fi = _taper(ri, 3.6, 0.2)
        q2 = 13 / (4 * np.pi) * fi @ eval_legendre(6, ui @ ui.T) @ fi
        assert abs(out["qnorm"][i] ** 2 - q2) < 1e-12 * max(1.0, q2)
        off, nbr = nl
        for j in nbr[off[i]:off[i + 1]][:6]:
            uj, rj = _shell(pos, box, j, 3.6)
            fj = _taper(rj, 3.6, 0.2)
            cross = 13 / (4 * np.pi) * fi @ eval_legendre(6, ui @ uj.T) @ fj
            dot = cross / (out["qnorm"][i] * out["qnorm"][j])
            assert abs(out["qhat"][i] @ out["qhat"][j] - dot) < 1e-12


def test_wurtzite_bond_dot_spectrum(orc):
    """Perfect wurtzite (a=3.19, c=5.19, u=0.377): 17 neighbours inside 3.6 A,
    only m in {0, +-3, +-6} survive, and the bond dots take two values, the
    second given by the addition theorem on the two shells."""
    pos, sp, box = W.wurtzite_ideal(6, 3, 4)
    nl = orc.neighbors(pos, box, 4.0)
    out = orc.q6_forward(pos, box, nl, orc.q6_params(**Q6CV))
    off, nbr = nl
    i = 0
    ui, ri = _shell(pos, box, i, 3.6)
    assert len(ri) == 17
    Q = out["Q"][i]
    # components 1,2 (m=1), 3,4 (m=2), 7,8 (m=4), 9,10 (m=5) vanish by the 3-fold axis
    assert np.max(np.abs(Q[[1, 2, 3, 4, 7, 8, 9, 10]])) < 1e-12
    dots = sorted(out["qhat"][i] @ out["qhat"][j] for j in nbr[off[i]:off[i + 1]] if np.linalg.norm(
        (pos[j] - pos[i]) - box * np.rint((pos[j] - pos[i]) / box)) < 3.6)
    vals = np.unique(np.round(dots, 9))
    assert len(vals) == 2 and abs(vals[1] - 1.0) < 1e-9
    # the second value is the cross term between the two site types
    j_other = [j for j in nbr[off[i]:off[i + 1]] if abs(out["qhat"][i] @ out["qhat"][j] - 1) > 1e-6][0]
    uj, rj = _shell(pos, box, j_other, 3.6)
    cross = (13 / (4 * np.pi)) * np.ones(17) @ eval_legendre(6, ui @ uj.T) @ np.ones(17)
    assert abs(vals[0] - cross / (out["qnorm"][i] * out["qnorm"][j_other])) < 1e-9


# --------------------------------------------------------------------------
# Coordination number: closed-form lattice sum over fcc shells.
# --------------------------------------------------------------------------
def test_fcc_coordination_shell_sum(orc):
    a, r0, rc = 3.615, 3.0, 6.0
    pos, box = W.fcc_ideal(6, a)
    nl = orc.neighbors(pos, box, 6.5)
    s = orc.cn_forward(pos, box, nl, r0, rc)
    # fcc shells: n = 12, 6, 24, 12, 24, 8 at a*sqrt(k/2), k = 1..6
    shells = [(12, 1), (6, 2), (24, 3), (12, 4), (24, 5), (8, 6)]
    ref = 0.0
    for cnt, k in shells:
        r = a * np.sqrt(k / 2)
        if r < rc:
            x = r / r0
            ref += cnt * (1 - x ** 6) / (1 - x ** 12)  # the switch as the workload states it
    assert abs(s - ref) < 1e-12 * ref
    assert abs(s - 13.2361817553) < 1e-9


def test_cn_switch_at_r0_is_half(orc):
    box = np.array([30.0, 30.0, 30.0])
    pos = np.array([[10.0, 10.0, 10.0], [13.0, 10.0, 10.0]])
    nl = orc.neighbors(pos, box, 6.5)
    assert abs(orc.cn_forward(pos, box, nl, 3.0, 6.0) - 0.5) < 1e-15


# --------------------------------------------------------------------------
# Neighbour sets: brute force against cell binning; cell-list properties.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,n,L,rl", [(1, 500, (12.0, 13.5, 14.2), 4.0), (2, 2000, (20.0, 21.0, 19.5), 4.0),
                                         (3, 300, (12.0, 12.0, 12.0), 3.999999), (4, 64, (9.0, 9.3, 9.1), 3.0),
                                         (5, 4096, (30.1, 25.7, 28.3), 6.5)])
def test_neighbors_brute_equals_cells(orc, seed, n, L, rl):
    rng = np.random.default_rng(seed)
    box = np.array(L)
    pos = (rng.random((n, 3)) * box).astype(np.float32)
    a = orc.neighbors(pos, box, rl, method="brute")
    b = orc.neighbors(pos, box, rl, method="cells")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # symmetric relation
    off, nbr = a
    rows = np.repeat(np.arange(n), np.diff(off))
    fwd = set(zip(rows.tolist(), nbr.tolist()))
    assert all((j, i) in fwd for i, j in fwd)


def test_neighbors_tiny_hand_case(orc):
    box = np.array([10.0, 10.0, 10.0])
    pos = np.array([[0.5, 5, 5], [9.6, 5, 5], [3.0, 5, 5], [0.5, 5, 8.4]], np.float32)
    off, nbr = orc.neighbors(pos, box, 3.0, method="brute")
    # 0-1 through the x face (0.9), 0-2 (2.5), 0-3 (3.4: out), 1-2 (3.4: out)
    assert off.tolist() == [0, 2, 3, 4, 4]
    assert nbr.tolist() == [1, 2, 0, 0]


def test_box_too_small(orc):
    with pytest.raises(ValueError):
        orc.cell_grid(np.array([11.9, 20.0, 20.0]), 4.0)
    assert orc.cell_grid(np.array([12.0, 20.0, 20.0]), 4.0).tolist() == [3, 5, 5]


def test_cell_list_properties(orc):
    d = W.small_wurtzite_slab()
    pos, box = d["pos"], d["box"]
    nc, cell, perm, start = orc.cell_list(pos, box, 4.0)
    n = len(pos)
    assert sorted(perm.tolist()) == list(range(n))
    key = cell[perm].astype(np.int64) * n + perm
    assert np.all(np.diff(key) > 0)
    assert np.array_equal(np.diff(start), np.bincount(cell, minlength=int(np.prod(nc))))
    # each atom lies in its cell's slab on every axis (to rounding)
    cx = np.stack([cell % nc[0], (cell // nc[0]) % nc[1], cell // (nc[0] * nc[1])], 1)
    w = box / nc
    x = pos.astype(np.float64)
    assert np.all(x >= cx * w - 1e-9) and np.all(x < (cx + 1) * w + 1e-9)


# --------------------------------------------------------------------------
# Gradients: central differences, zero net force, invariances.
# --------------------------------------------------------------------------
def _fd(fun, x, idx, h=1e-4):
    """Central differences at h and h/2, Richardson-extrapolated (error O(h^4));
    the sharp bond and count sigmoids make plain O(h^2) differences at h = 1e-4
    too coarse for a 1e-6 comparison."""
    def central(i, a, step):
        xp = x.copy()
        xp[i, a] += step
        xm = x.copy()
        xm[i, a] -= step
        return (fun(xp) - fun(xm)) / (2 * step)

    return np.array([(4 * central(i, a, h / 2) - central(i, a, h)) / 3 for (i, a) in idx])


def _slab():
    d = W.wurtzite_slab(4, 3, 4, seed=31)
    return d["pos"].astype(np.float64), d["box"]


def test_q6_gradient_finite_differences(orc):
    pos, box = _slab()
    nl = orc.neighbors(pos, box, 4.0)
    prm = orc.q6_params(**Q6CV)
    g = orc.q6_gradient(pos, box, nl, prm)
    rng = np.random.default_rng(7)
    # coordinates of the atoms with the largest gradients, plus random ones
    big = np.argsort(-np.linalg.norm(g, axis=1))[:20]
    idx = [(i, a) for i in big for a in range(3)] + [(int(i), int(a)) for i, a in
                                                      zip(rng.integers(0, len(pos), 60), rng.integers(0, 3, 60))]
    fd = _fd(lambda x: orc.q6_forward(x, box, nl, prm)["s"], pos, idx)
    an = np.array([g[i, a] for i, a in idx])
    assert np.max(np.abs(fd - an)) <= 1e-6 * np.max(np.abs(g)) + 1e-9
    assert np.max(np.abs(g)) > 1e-2  # the slab's interface makes the test non-vacuous


def test_cn_gradient_finite_differences(orc):
    pos, box = _slab()
    nl = orc.neighbors(pos, box, 4.0)
    g = orc.cn_gradient(pos, box, nl, 2.5, 3.6)
    # skip coordinates of atoms with a pair within 10 h of the hard cutoff
    off, nbr = nl
    idx = []
    rng = np.random.default_rng(8)
    for i in rng.choice(len(pos), 60, replace=False):
        d = pos[nbr[off[i]:off[i + 1]]] - pos[i]
        d -= box * np.rint(d / box)
        if np.all(np.abs(np.linalg.norm(d, axis=1) - 3.6) > 1e-3):
            idx += [(int(i), a) for a in range(3)]
    assert len(idx) > 60
    fd = _fd(lambda x: orc.cn_forward(x, box, nl, 2.5, 3.6), pos, idx)
    an = np.array([g[i, a] for i, a in idx])
    assert np.max(np.abs(fd - an)) <= 1e-8 * np.max(np.abs(g))


def test_bias_force_finite_differences(orc):
    """F_fd = -[V(s(x+h)) - V(s(x-h))]/2h against the chain-rule force, 2-D CV."""
    pos, box = _slab()
    nl = orc.neighbors(pos, box, 4.0)
    prm = orc.q6_params(**Q6CV)
    s0 = np.array([orc.cn_forward(pos, box, nl, 2.5, 3.6), orc.q6_forward(pos, box, nl, prm)["s"]])
    sigma = np.array([0.05, 20.0])
    cen = W.hill_centres(300, s0 - 3 * sigma, s0 + 3 * sigma, seed=9)
    hts = orc.deposit_sequence(cen, sigma, W.W0_EV, 10.0, W.KBT_EV)

    def V(x):
        s = [orc.cn_forward(x, box, nl, 2.5, 3.6), orc.q6_forward(x, box, nl, prm)["s"]]
        return orc.bias(cen, hts, sigma, np.array(s))[0]

    _, dV = orc.bias(cen, hts, sigma, s0)
    grads = [orc.cn_gradient(pos, box, nl, 2.5, 3.6), orc.q6_gradient(pos, box, nl, prm)]
    F = orc.bias_forces(np.zeros((len(pos), 3)), grads, dV)
    big = np.argsort(-np.linalg.norm(F, axis=1))[:15]
    idx = [(int(i), a) for i in big for a in range(3)]
    fd = -_fd(V, pos, idx)
    an = np.array([F[i, a] for i, a in idx])
    assert np.max(np.abs(fd - an)) <= 1e-6 * np.max(np.linalg.norm(F, axis=1))


def test_zero_net_force_and_translation(orc):
    pos, box = _slab()
    nl = orc.neighbors(pos, box, 4.0)
    prm = orc.q6_params(**Q6CV)
    for g in (orc.q6_gradient(pos, box, nl, prm), orc.cn_gradient(pos, box, nl, 2.5, 3.6)):
        gmax = np.max(np.linalg.norm(g, axis=1))
        assert np.linalg.norm(g.sum(0)) <= 1e-12 * np.sqrt(len(pos)) * gmax
    s = orc.q6_forward(pos, box, nl, prm)["s"]
    shifted = np.mod(pos + np.array([1.37, -2.11, 4.05]), box)
    nl2 = orc.neighbors(shifted, box, 4.0)
    assert abs(orc.q6_forward(shifted, box, nl2, prm)["s"] - s) < 1e-10 * s


def test_rotation_and_permutation_invariance(orc):
    """A non-periodic cluster in a large box: s is invariant under rotation and
    relabelling; the gradient rotates and permutes with the atoms."""
    rng = np.random.default_rng(12)
    ideal, sp, _ = W.wurtzite_ideal(3, 2, 2)
    cl = ideal - ideal.mean(0) + rng.normal(0, 0.08, ideal.shape)
    box = np.array([60.0, 60.0, 60.0])
    prm = orc.q6_params(**Q6CV)

    def run(x):
        xb = x + 30.0
        nl = orc.neighbors(xb, box, 4.0)
        return orc.q6_forward(xb, box, nl, prm)["s"], orc.q6_gradient(xb, box, nl, prm)

    s0, g0 = run(cl)
    A = rng.normal(size=(3, 3))
    R, _ = np.linalg.qr(A)
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    s1, g1 = run(cl @ R.T)
    assert abs(s1 - s0) < 1e-11 * max(1.0, abs(s0))
    assert np.max(np.abs(g1 - g0 @ R.T)) < 1e-10 * np.max(np.abs(g0))
    p = rng.permutation(len(cl))
    s2, g2 = run(cl[p])
    assert abs(s2 - s0) < 1e-11 * max(1.0, abs(s0))
    assert np.max(np.abs(g2 - g0[p])) < 1e-12 * np.max(np.abs(g0))


def test_perfect_fcc_cn_forces_vanish(orc):
    pos, box = W.fcc_ideal(6, 3.615)
    nl = orc.neighbors(pos, box, 6.5)
    g = orc.cn_gradient(pos, box, nl, 3.0, 6.0)
    assert np.max(np.abs(g)) < 1e-12


# --------------------------------------------------------------------------
# Hills and well-tempered heights.
# --------------------------------------------------------------------------
def test_single_hill(orc):
    V, g = orc.bias([[1.5]], [0.7], [0.2], [1.5])
    assert V == 0.7 and g[0] == 0.0
    V, g = orc.bias([[1.5, -2.0]], [0.7], [0.2, 3.0], [1.7, 1.0])
    assert abs(V - 0.7 * np.exp(-0.5) * np.exp(-0.5)) < 1e-16


def test_hill_integral_closed_form(orc):
    """int V ds = sqrt(2 pi) sigma sum_k h_k (1-D), by trapezoidal quadrature."""
    cen = W.hill_centres(50, [0.0], [3.0], seed=3)
    h = np.random.default_rng(4).random(50) + 0.5
    s = np.linspace(-3.0, 6.0, 20001)
    V = np.array([orc.bias(cen, h, [0.2], [x])[0] for x in s])
    integral = np.sum((V[1:] + V[:-1]) * 0.5 * np.diff(s))
    assert abs(integral - np.sqrt(2 * np.pi) * 0.2 * h.sum()) < 1e-10 * integral


def test_bias_derivative_fd(orc):
    cen = W.hill_centres(40, [0.0, -1.0], [2.0, 1.0], seed=5)
    h = np.linspace(0.1, 1.0, 40)
    sig = [0.3, 0.25]
    s = np.array([0.9, 0.1])
    _, g = orc.bias(cen, h, sig, s)
    for d in range(2):
        e = np.zeros(2)
        e[d] = 1e-5
        fd = (orc.bias(cen, h, sig, s + e)[0] - orc.bias(cen, h, sig, s - e)[0]) / 2e-5
        assert abs(fd - g[d]) < 1e-8


def test_wt_first_height_and_plain_metad(orc):
    cen = W.hill_centres(20, [0.0], [1.0], seed=6)
    h = orc.deposit_sequence(cen, [0.1], 1.2, 10.0, W.KBT_KJMOL)
    assert h[0] == 1.2 and np.all(h[1:] < 1.2) and np.all(h > 0)
    assert np.all(orc.deposit_sequence(cen, [0.1], 1.2, 0.0, W.KBT_KJMOL) == 1.2)


def test_wt_colocated_recursion_high_precision(orc):
    """Hills at one point: V_{n+1} = V_n + w0 exp(-V_n / (kT (gamma-1))).
    Replayed with 40-digit arithmetic; 50,000 deposits stay within 1e-12."""
    import mpmath

    K = 50000
    w0, gamma, kT = 1.2, 10.0, W.KBT_KJMOL
    cen = np.zeros((K, 1))
    # the co-located recursion only needs V at the shared point, so deposit in
    # blocks through the oracle's own height rule and bias sum
    h = np.empty(K)
    V = 0.0
    chunk = 2000
    for k0 in range(0, K, chunk):
        hh = []
        for k in range(k0, min(K, k0 + chunk)):
            hk = orc.wt_height(w0, gamma, kT, V)
            hh.append(hk)
            V += hk
        h[k0:k0 + len(hh)] = hh
        V = orc.bias(cen[:k0 + len(hh)], h[:k0 + len(hh)], [0.1], [0.0])[0]
    mpmath.mp.dps = 40
    Vm = mpmath.mpf(0)
    a = mpmath.mpf(kT) * (mpmath.mpf(gamma) - 1)
    for k in range(K):
        Vm += mpmath.mpf(w0) * mpmath.exp(-Vm / a)
    assert abs(V - float(Vm)) < 1e-12 * float(Vm)
    # continuous-limit bound: V_n lies near a ln(1 + n w0 / a)
    cont = float(a * mpmath.log(1 + K * w0 / a))
    assert abs(V - cont) / cont < 0.01


def test_deposit_sequence_matches_stepwise(orc):
    cen = W.hill_centres(200, [0.0, 0.0], [1.0, 2.0], seed=8)
    sig = [0.1, 0.3]
    h = orc.deposit_sequence(cen, sig, 1.2, 10.0, W.KBT_KJMOL)
    for k in (0, 1, 57, 199):
        V = orc.bias(cen[:k], h[:k], sig, cen[k])[0]
        assert h[k] == orc.wt_height(1.2, 10.0, W.KBT_KJMOL, V)


# --------------------------------------------------------------------------
# The crystalline-count stage (bond dots -> b_ij -> n_i -> c_i -> s), pinned
# by geometry: the bond dots come from the Legendre addition theorem over the
# two atoms' shells (never from the oracle's harmonics), the taper weights from
# the pair distances, and the logistics are the workload's definition.
# --------------------------------------------------------------------------
def _logistic(x, centre, width):
    return 1.0 / (1.0 + np.exp(-(x - centre) / width))


def _shell_dots(pos, box, rc, D, pairs):
    """d_ij = Q_i.Q_j / (|Q_i||Q_j|) by the addition theorem, for each (i, j)."""
    cache = {}

    def shell(i):
        if i not in cache:
            u, r = _shell(pos, box, i, rc)
            cache[i] = (u, _taper(r, rc, D))
        return cache[i]

    out = []
    for i, j in pairs:
        ui, fi = shell(i)
        uj, fj = shell(j)
        qii = fi @ eval_legendre(6, ui @ ui.T) @ fi
        qjj = fj @ eval_legendre(6, uj @ uj.T) @ fj
        qij = fi @ eval_legendre(6, ui @ uj.T) @ fj
        out.append(qij / np.sqrt(qii * qjj))
    return np.array(out)


def test_count_stage_perfect_wurtzite_closed_form(orc):
    """Perfect wurtzite: every atom has 9 bond dots of exactly 1 (its own site
    type) and 8 of one value d2 (the other type, from the addition theorem),
    all weights 1, so n_i = 9 b(1) + 8 b(d2) and s = N c(n) for every atom."""
    pos, sp, box = W.wurtzite_ideal(6, 3, 4)
    nl = orc.neighbors(pos, box, 4.0)
    out = orc.q6_forward(pos, box, nl, orc.q6_params(**Q6CV))
    n = len(pos)
    # an atom of the other site type among atom 0's neighbours (dot != 1)
    u0, r0 = _shell(pos, box, 0, 3.6)
    assert len(r0) == 17 and np.all(r0 < 3.6 - 0.2)  # all weights are 1
    d = pos - pos[0]
    d -= box * np.rint(d / box)
    cand = [j for j in range(1, n) if np.linalg.norm(d[j]) < 3.6]
    dots = _shell_dots(pos, box, 3.6, 0.2, [(0, j) for j in cand])
    same = np.abs(dots - 1.0) < 1e-9
    assert same.sum() == 9 and (~same).sum() == 8
    d2 = dots[~same]
    assert np.ptp(d2) < 1e-12 and abs(d2[0] - 0.6610857) < 1e-7
    n_ref = 9 * _logistic(1.0, 0.7, 0.02) + 8 * _logistic(d2[0], 0.7, 0.02)
    c_ref = _logistic(n_ref, 5.5, 0.25)
    assert abs(n_ref - 10.0001686) < 1e-7
    assert np.max(np.abs(out["nb"] - n_ref)) < 1e-12
    assert np.max(np.abs(out["c"] - c_ref)) < 1e-15
    assert abs(out["s"] - n * c_ref) < 1e-12 * n
    assert abs(out["s"] / n - (1 - 1.5e-8)) < 1e-9


def test_count_stage_taper_and_slopes(orc):
    """A jittered fcc cluster whose first shell straddles the taper (r_c 2.8,
    taper 0.4), with bond and count widths chosen so that the dots and counts
    lie on the logistics' slopes: n_i = sum_j f(r_ij) b(d_ij) per atom, c_i =
    c(n_i), c'_i = c(1 - c)/w_c and s = sum_i c_i against the weights and
    dots computed from the geometry.  A dropped weight, swapped widths or a
    flipped sign each fail it."""
    rng = np.random.default_rng(17)
    ideal, _ = W.fcc_ideal(3, 3.615)
    ideal = ideal[np.linalg.norm(ideal - ideal.mean(0), axis=1) < 5.5]
    pos = ideal - ideal.mean(0) + 20.0 + rng.normal(0.0, 0.18, ideal.shape)
    box = np.array([40.0, 40.0, 40.0])
    rc, D, d0, wb, n0, wc = 2.8, 0.4, 0.6, 0.08, 4.0, 1.5
    prm = orc.q6_params(rc, D, d0, wb, n0, wc)
    nl = orc.neighbors(pos, box, rc + 0.4)
    out = orc.q6_forward(pos, box, nl, prm)
    n = len(pos)
    nb_ref = np.zeros(n)
    pairs, w = [], []
    for i in range(n):
        u, r = _shell(pos, box, i, rc)
        d = pos - pos[i]
        d -= box * np.rint(d / box)
        js = [j for j in range(n) if j != i and np.linalg.norm(d[j]) < rc]
        pairs += [(i, j) for j in js]
        w += list(_taper(np.linalg.norm(d[js], axis=1), rc, D))
    dots = _shell_dots(pos, box, rc, D, pairs)
    w = np.array(w)
    np.add.at(nb_ref, [i for i, _ in pairs], w * _logistic(dots, d0, wb))
    c_ref = _logistic(nb_ref, n0, wc)
    # the case exercises every term: weights inside the taper, dots and counts on the slopes
    assert np.sum((w > 0.05) & (w < 0.95)) > 20
    assert np.sum(np.abs(dots - d0) < 2 * wb) > 20
    assert np.sum(np.abs(nb_ref - n0) < wc) > 5
    assert np.max(np.abs(out["nb"] - nb_ref)) < 1e-12 * max(1.0, nb_ref.max())
    assert np.max(np.abs(out["c"] - c_ref)) < 1e-12
    assert np.max(np.abs(out["dc"] - c_ref * (1 - c_ref) / wc)) < 1e-12
    assert abs(out["s"] - c_ref.sum()) < 1e-12 * n
