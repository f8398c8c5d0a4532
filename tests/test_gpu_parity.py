"""HIP path against the FP64 oracle, stage by stage, on the same seeded inputs.

Bars (written here, derived in the design notes):
  * cell permutation, cell starts and neighbour sets: bit-exact;
  * CV: |s_gpu - s_ref| <= 1e-5 |s_ref| in FP32 (1e-10 in FP64);
  * bias forces (F_out - F_in), seeded with the same dV/ds on both sides:
    max_i |dF_i| / max_i |F_ref_i| <= 1e-4 in FP32 (1e-10 in FP64);
  * V, dV/ds and hill heights at the same s: 1e-12 relative (FP64 both sides).
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import oracle_cvs, params_for, rel_force_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q6CV = dict(cv="q6", precision="fp32", r_c=3.6, skin=0.4, taper=0.2, cn_r0=2.5, bond_d0=0.7, bond_w=0.02,
            count_n0=5.5, count_w=0.25, sigma=[20.0], w0=W.W0_EV, gamma=10.0, kBT=W.KBT_EV,
            hills=dict(k=64))


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype).contiguous()


def make_pipe(wl, n, **kw):
    from paper_2510_06873_amd import Pipeline

    return Pipeline(n, params_for(wl, **kw))


def gpu_neighbor_sets(pipe):
    """Rows of the GPU neighbour lists mapped back to atom ids, as sorted arrays."""
    _, perm, _ = pipe.cell_list()
    nbr, cnt = pipe.neighbor_lists()
    perm = perm.cpu().numpy()
    nbr = nbr.cpu().numpy()
    cnt = cnt.cpu().numpy()
    rows = {}
    for t in range(len(perm)):
        rows[int(perm[t])] = np.sort(perm[nbr[t, :cnt[t]]])
    return rows


# ---------------------------------------------------------------------------
# Cell list and neighbour sets: bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("spec", [dict(nx=4, ny=3, nz=6, seed=21), dict(nx=7, ny=5, nz=5, seed=22),
                                  dict(nx=40, ny=20, nz=15, seed=2)])
def test_cell_list_and_neighbors_bit_exact(orc, spec):
    d = W.wurtzite_slab(**spec)
    pos, box = d["pos"], d["box"]
    n = len(pos)
    pipe = make_pipe(Q6CV, n)
    p4 = to_dev(W.as_float4(pos, d["species"]))
    pipe.build_neighbors(p4, box)
    assert pipe.status(True) == 0
    nc, perm, start = pipe.cell_list()
    onc, ocell, operm, ostart = orc.cell_list(pos, box, 4.0)
    assert tuple(onc.tolist()) == nc
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(start.cpu().numpy(), ostart)
    off, nb = orc.neighbors(pos, box, 4.0)
    rows = gpu_neighbor_sets(pipe)
    for i in range(n):
        assert np.array_equal(rows[i], nb[off[i]:off[i + 1]]), i
    mx, tot = pipe.neighbor_stats()
    assert tot == len(nb) and mx == int(np.diff(off).max())


def test_neighbors_random_boxes_edge(orc):
    """Uniform random atoms in boxes just above 3 cells per axis, skin 0."""
    from paper_2510_06873_amd import Params, Pipeline

    rng = np.random.default_rng(3)
    for L in ((12.0, 12.3, 12.9), (12.0000001, 13.7, 16.2)):
        box = np.array(L)
        pos = (rng.random((700, 3)) * box).astype(np.float32)
        pipe = Pipeline(700, Params(cv_kind=2, r_c=4.0, skin=0.0, sigma=[1.0], hill_capacity=4, max_neighbors=200))
        pipe.build_neighbors(to_dev(W.as_float4(pos)), box)
        assert pipe.status(True) == 0
        off, nb = orc.neighbors(pos, box, 4.0, method="brute")
        rows = gpu_neighbor_sets(pipe)
        for i in range(700):
            assert np.array_equal(rows[i], nb[off[i]:off[i + 1]])


def test_neighbors_pairs_at_the_cutoff(orc):
    """Simple-cubic lattice with spacing r_list (4 A), jittered by about one
    FP32 ulp: every nearest pair lies within a few ulps of r_list, where the
    build's FP32 test defers to the FP64 one; pairs across the faces included."""
    from paper_2510_06873_amd import Params, Pipeline

    rng = np.random.default_rng(11)
    m = 7
    box = np.full(3, 4.0 * m)
    idx = np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = (idx * 4.0 + rng.normal(0.0, 2e-6, idx.shape)) % box
    pos = pos.astype(np.float32)
    n = len(pos)
    pipe = Pipeline(n, Params(cv_kind=2, r_c=4.0, skin=0.0, sigma=[1.0], hill_capacity=4, max_neighbors=64))
    pipe.build_neighbors(to_dev(W.as_float4(pos)), box)
    assert pipe.status(True) == 0
    off, nb = orc.neighbors(pos, box, 4.0, method="brute")
    counts = np.diff(off)
    assert 0 < counts.sum() < 6 * n  # some of the nearest pairs fall inside, some outside
    rows = gpu_neighbor_sets(pipe)
    for i in range(n):
        assert np.array_equal(rows[i], nb[off[i]:off[i + 1]]), i


# ---------------------------------------------------------------------------
# q6 count: CV, per-atom values, gradient and forces
# ---------------------------------------------------------------------------
def run_step(pipe, pos, species, box, F_in, seed_dv):
    p4 = to_dev(W.as_float4(pos, species))
    pipe.build_neighbors_checked(p4, box)
    s = pipe.cv_forward(p4).clone()
    pipe.cv_backward(p4)
    F = to_dev(F_in, pipe.fdtype)
    dv = torch.tensor(seed_dv, dtype=torch.float64, device=dev())
    pipe.apply_bias_forces(p4, F, dv)
    torch.cuda.synchronize()
    assert pipe.status(True) == 0
    return s.cpu().numpy(), F.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("precision,tol_s,tol_f", [("fp32", 1e-5, 1e-4), ("fp64", 1e-10, 1e-10)])
@pytest.mark.parametrize("spec", [dict(nx=4, ny=3, nz=6, seed=21), dict(nx=8, ny=4, nz=8, seed=5)])
def test_q6_cv_and_forces(orc, spec, precision, tol_s, tol_f):
    d = W.wurtzite_slab(**spec)
    pos, box, sp = d["pos"], d["box"], d["species"]
    n = len(pos)
    wl = dict(Q6CV, precision=precision)
    pipe = make_pipe(wl, n)
    F_in = W.external_forces(n, seed=9)
    dv = [0.37]
    s, F = run_step(pipe, pos, sp, box, F_in, dv)
    s_ref, g_ref, nl = oracle_cvs(orc, pos, box, wl)
    assert abs(s[0] - s_ref[0]) <= tol_s * abs(s_ref[0])
    F_ref_bias = -dv[0] * g_ref[0]
    assert rel_force_err(F[:, :3] - F_in[:, :3].astype(np.float64), F_ref_bias) <= tol_f
    assert np.array_equal(F[:, 3], F_in[:, 3])
    # per-atom Steinhardt q6 and bond counts
    prm = orc.q6_params(3.6, 0.2, 0.7, 0.02, 5.5, 0.25)
    o = orc.q6_forward(pos, box, nl, prm)
    from paper_2510_06873_amd import ATOM_C, ATOM_NB, ATOM_Q6

    tol_a = 1e-4 if precision == "fp32" else 1e-10
    assert np.max(np.abs(pipe.atom_values(ATOM_Q6).cpu().numpy() - o["q6"])) <= tol_a
    assert np.max(np.abs(pipe.atom_values(ATOM_NB).cpu().numpy() - o["nb"])) <= 50 * tol_a
    assert np.max(np.abs(pipe.atom_values(ATOM_C).cpu().numpy() - o["c"])) <= 50 * tol_a


@pytest.mark.parametrize("precision,tol_s,tol_f", [("fp32", 1e-5, 1e-4), ("fp64", 1e-10, 1e-10)])
def test_dense_cluster_in_gas(orc, precision, tol_s, tol_f):
    """Bricks sized for the mean density (3.9 atoms per cell): next to the
    cluster (about 33 atoms per cell) a brick's halo holds some 1,300 slots,
    more than the neighbour build and the CV passes stage in LDS (998), so
    both read the rest from global memory, and such a brick owns more atoms
    than its workgroup has threads.  The rows start 96 wide and overflow
    (131 neighbours in the cluster), so the checked build grows them.  Bond
    and count thresholds are lowered (0.4 and 2 bonds, width 0.5) so that the
    disordered atoms sit on the slopes of both logistics (s ~ 1,700 of 3,900)."""
    d = W.cluster_in_gas()
    pos, box = d["pos"], d["box"]
    n = len(pos)
    wl = dict(Q6CV, precision=precision, bond_d0=0.4, count_n0=2.0, count_w=0.5)
    pipe = make_pipe(wl, n, max_neighbors=96)
    p4 = to_dev(W.as_float4(pos))
    pipe.build_neighbors_checked(p4, box)
    off, nb = orc.neighbors(pos, box, 4.0)
    assert np.diff(off).max() > 96
    rows = gpu_neighbor_sets(pipe)
    for i in range(n):
        assert np.array_equal(rows[i], nb[off[i]:off[i + 1]]), i
    F_in = W.external_forces(n, seed=12)
    dv = [0.53]
    s, F = run_step(pipe, pos, None, box, F_in, dv)
    s_ref, g_ref, _ = oracle_cvs(orc, pos, box, wl, nl=(off, nb))
    assert abs(s[0] - s_ref[0]) <= tol_s * abs(s_ref[0])
    assert rel_force_err(F[:, :3] - F_in[:, :3].astype(np.float64), -dv[0] * g_ref[0]) <= tol_f


@pytest.mark.parametrize("precision,brick,tol_s,tol_f", [("fp32", (1, 1, 1), 1e-5, 1e-4), ("fp32", (2, 2, 2), 1e-5, 1e-4),
                                                          ("fp32", (3, 3, 3), 1e-5, 1e-4),
                                                          ("fp64", (1, 1, 1), 1e-10, 1e-10)])
def test_rows_ending_on_16_byte_boundaries(orc, precision, brick, tol_s, tol_f):
    """A simple cubic lattice (a = 1.6 A, 14^3 atoms, 0.02 A jitter) with r_c
    3.45 and skin 0.3: every atom has exactly 32 neighbours inside r_c (shells
    1.6, 2.26, 2.77 and 3.2 A) and 56 in its list (plus 3.58 A), so with 4, 2
    or 1 threads per atom (bricks of 1, 8 and 27 cells) every in-cutoff
    sub-row holds 8, 16 or 32 slots: each row walk ends exactly on a 16-byte
    chunk, and every row write ends with a full chunk and no partial tail.
    The 3x3x3 bricks stage less than their halo (the whole system), so their
    walks also take the path that reads records from global memory.  Bond and
    count thresholds (0.96 / 0.02 and 27 / 0.5) put the atoms on the slopes
    of both logistics (s ~ 1,360 of 2,744)."""
    a, L = 1.6, 14
    g = np.arange(L) * a
    box = np.full(3, L * a)
    rng = np.random.default_rng(7)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = np.mod(pos + rng.uniform(-0.02, 0.02, pos.shape), box).astype(np.float32)
    pos[pos >= box.astype(np.float32)] = 0.0  # the oracle sees the FP32 coordinates the GPU gets
    pos = pos.astype(np.float64)
    n = len(pos)
    wl = dict(Q6CV, precision=precision, r_c=3.45, skin=0.3, bond_d0=0.96, bond_w=0.02, count_n0=27.0,
              count_w=0.5)
    prm = params_for(wl)
    prm.brick = brick
    from paper_2510_06873_amd import Pipeline

    pipe = Pipeline(n, prm)
    off, nb = orc.neighbors(pos, box, 3.75)
    assert np.diff(off).min() == np.diff(off).max() == 56
    F_in = W.external_forces(n, seed=13)
    dv = [0.41]
    s, F = run_step(pipe, pos, None, box, F_in, dv)
    rows = gpu_neighbor_sets(pipe)
    for i in range(n):
        assert np.array_equal(rows[i], nb[off[i]:off[i + 1]]), i
    _, _, cut = pipe.neighbor_stats(cutoff_pairs=True)
    assert cut == 32 * n
    s_ref, g_ref, _ = oracle_cvs(orc, pos, box, wl, nl=(off, nb))
    assert 0.3 * n < s_ref[0] < 0.7 * n
    assert abs(s[0] - s_ref[0]) <= tol_s * abs(s_ref[0])
    assert rel_force_err(F[:, :3] - F_in[:, :3].astype(np.float64), -dv[0] * g_ref[0]) <= tol_f


def test_q6_forces_wrapped_pairs_long_box(orc):
    """Pairs across the periodic faces of a 204 A box: the minimum-image
    difference must not round at the magnitude of the box length (FP32 ulp at
    200 A is 1.5e-5 A).  Forming x_j - x_i before removing the image shift put
    a 4e-4 relative force error on the atoms at the faces; with the shift taken
    from the coordinate near the far face their error stays at the FP32 level
    of the interior (~1e-5), so the bar for the face atoms is tighter than the
    general one."""
    d = W.wurtzite_slab(64, 3, 4, seed=31)
    pos, box, sp = d["pos"], d["box"], d["species"]
    n = len(pos)
    assert box[0] > 200.0
    pipe = make_pipe(Q6CV, n)
    F_in = np.zeros((n, 4), np.float32)
    dv = [1.0]
    s, F = run_step(pipe, pos, sp, box, F_in, dv)
    s_ref, g_ref, _ = oracle_cvs(orc, pos, box, Q6CV)
    assert abs(s[0] - s_ref[0]) <= 1e-6 * abs(s_ref[0])
    err = rel_force_err(F[:, :3], -g_ref[0])
    # atoms within 2 A of an x face against the rest
    face = np.minimum(pos[:, 0], box[0] - pos[:, 0]) < 2.0
    gmax = np.linalg.norm(g_ref[0], axis=1).max()
    err_face = np.linalg.norm(F[face, :3] + g_ref[0][face], axis=1).max() / gmax
    print(f"[wrap] N={n} force err {err:.2e}, at the x faces {err_face:.2e}")
    assert err <= 1e-4
    assert err_face <= 2e-5


def test_q6_coordinates_outside_the_box(orc):
    """Coordinates given in other periodic images (shifted by whole box
    lengths, as an MD code that never wraps would pass them).  The box has
    11 cells per axis, so most bricks keep off the faces and take plain pair
    differences while every coordinate is inside the box; a step with shifted
    coordinates must switch every brick to the minimum image (the gather
    flags them), with or without a rebuild in between."""
    d = W.wurtzite_slab(14, 8, 9, seed=33)
    pos, box, sp = d["pos"], d["box"], d["species"]
    n = len(pos)
    assert min(np.floor(box / 4.0)) >= 11
    k = np.random.default_rng(4).integers(-1, 2, size=(n, 3))
    k[np.random.default_rng(5).random(n) < 0.7] = 0  # most atoms stay in the box
    pos_u = (pos.astype(np.float64) + k * box).astype(np.float32)
    pipe = make_pipe(Q6CV, n)

    def step(p):
        p4 = to_dev(W.as_float4(p, sp))
        s = pipe.cv_forward(p4).clone()
        pipe.cv_backward(p4)
        F = torch.zeros((n, 4), dtype=torch.float32, device=dev())
        pipe.apply_bias_forces(p4, F, torch.ones(1, dtype=torch.float64, device=dev()))
        torch.cuda.synchronize()
        assert pipe.status(True) == 0
        return s.item(), F.cpu().numpy()[:, :3].astype(np.float64)

    refs = {}
    for tag, p in (("in", pos), ("out", pos_u)):
        s_ref, g_ref, _ = oracle_cvs(orc, p, box, Q6CV)
        refs[tag] = (s_ref[0], -g_ref[0])
    pipe.build_neighbors_checked(to_dev(W.as_float4(pos, sp)), box)
    for tag, p in (("in", pos), ("out", pos_u), ("out", pos_u)):  # lists from the wrapped coordinates
        s, F = step(p)
        assert abs(s - refs[tag][0]) <= 1e-5 * abs(refs[tag][0]), tag
        assert rel_force_err(F, refs[tag][1]) <= 1e-4, tag
    pipe.build_neighbors_checked(to_dev(W.as_float4(pos_u, sp)), box)  # lists from the shifted ones
    off_u, nb_u = orc.neighbors(pos_u, box, 4.0)
    rows = gpu_neighbor_sets(pipe)
    for i in np.random.default_rng(6).choice(n, 500, replace=False):
        assert np.array_equal(rows[i], nb_u[off_u[i]:off_u[i + 1]]), i
    for tag, p in (("out", pos_u), ("in", pos)):
        s, F = step(p)
        assert abs(s - refs[tag][0]) <= 1e-5 * abs(refs[tag][0]), tag
        assert rel_force_err(F, refs[tag][1]) <= 1e-4, tag


def test_q6_backward_gradient_output(orc):
    d = W.wurtzite_slab(5, 3, 5, seed=23)
    pos, box = d["pos"], d["box"]
    n = len(pos)
    pipe = make_pipe(Q6CV, n)
    p4 = to_dev(W.as_float4(pos))
    pipe.build_neighbors(p4, box)
    pipe.cv_forward(p4)
    g = torch.full((n, 4), 7.0, dtype=torch.float32, device=dev())
    pipe.cv_backward(p4, None, g)
    torch.cuda.synchronize()
    _, g_ref, _ = oracle_cvs(orc, pos, box, Q6CV)
    g = g.cpu().numpy().astype(np.float64)
    assert rel_force_err(g[:, :3], g_ref[0]) <= 1e-4
    assert np.all(g[:, 3] == 7.0)
    # zero net gradient (translation invariance), FP32 bound
    gmax = np.linalg.norm(g[:, :3], axis=1).max()
    assert np.linalg.norm(g[:, :3].sum(0)) <= 1e-5 * np.sqrt(n) * gmax


# ---------------------------------------------------------------------------
# 2-D CV (coordination + q6 count) and coordination alone (FP64)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,tol_s,tol_f", [("fp32", 1e-5, 1e-4), ("fp64", 1e-10, 1e-10)])
def test_coord_q6_2d(orc, precision, tol_s, tol_f):
    wl = dict(W.WORKLOADS["wz2048"], precision=precision)
    d = W.structure(wl["structure"])
    pos, box = d["pos"], d["box"]
    n = len(pos)
    pipe = make_pipe(wl, n)
    F_in = W.external_forces(n, seed=10)
    dv = [0.11, -0.023]
    s, F = run_step(pipe, pos, d["species"], box, F_in, dv)
    s_ref, g_ref, _ = oracle_cvs(orc, pos, box, wl)
    assert np.all(np.abs(s - s_ref) <= tol_s * np.abs(s_ref))
    F_ref_bias = -(dv[0] * g_ref[0] + dv[1] * g_ref[1])
    assert rel_force_err(F[:, :3] - F_in[:, :3].astype(np.float64), F_ref_bias) <= tol_f


def test_fcc864_coordination_fp64(orc):
    wl = W.WORKLOADS["fcc864"]
    d = W.structure(wl["structure"])
    pos, box = d["pos"], d["box"]
    n = len(pos)
    pipe = make_pipe(wl, n)
    F_in = np.zeros((n, 4))
    F_in[:, :3] = W.external_forces(n, seed=11)[:, :3]
    dv = [-3.3]
    s, F = run_step(pipe, pos, None, box, F_in, dv)
    s_ref, g_ref, _ = oracle_cvs(orc, pos, box, wl)
    assert abs(s[0] - s_ref[0]) <= 1e-10 * abs(s_ref[0])
    assert rel_force_err(F[:, :3] - F_in[:, :3], -dv[0] * g_ref[0]) <= 1e-10


# ---------------------------------------------------------------------------
# Hills: deposition replay, bias evaluation, checkpoint
# ---------------------------------------------------------------------------
def test_deposit_replay_and_bias_fcc864(orc):
    wl = W.WORKLOADS["fcc864"]
    hp = wl["hills"]
    cen = W.hill_centres(hp["k"], hp["lo"], hp["hi"], hp["seed"])
    pipe = make_pipe(wl, 864)
    cdev = to_dev(cen, torch.float64)
    for k in range(len(cen)):
        pipe.deposit_hill(cdev[k])
    gc, gh = pipe.hills_get()
    h_ref = orc.deposit_sequence(cen, wl["sigma"], wl["w0"], wl["gamma"], wl["kBT"])
    assert np.array_equal(gc, cen)
    assert np.max(np.abs(gh - h_ref) / h_ref) <= 1e-12
    for sval in (13.2, 0.0, 7.77, 20.0):
        s = torch.tensor([sval], dtype=torch.float64, device=dev())
        V, dV = pipe.bias_eval(s)
        Vr, dVr = orc.bias(cen, h_ref, wl["sigma"], [sval])
        assert abs(V.item() - Vr) <= 1e-12 * max(Vr, 1e-300)
        assert abs(dV.item() - dVr[0]) <= 1e-12 * (abs(dVr[0]) + Vr / wl["sigma"][0])


def test_bias_2d_and_checkpoint_roundtrip(orc):
    wl = W.WORKLOADS["wz2048"]
    pipe = make_pipe(wl, 100)
    cen = W.hill_centres(3000, [5.0, 900.0], [6.0, 1100.0], seed=3)
    hts = np.random.default_rng(1).random(3000) * 0.01
    pipe.hills_set(cen, hts)
    s = torch.tensor([5.5, 1000.0], dtype=torch.float64, device=dev())
    V, dV = pipe.bias_eval(s)
    V1, dV1 = V.item(), dV.cpu().numpy().copy()
    Vr, dVr = orc.bias(cen, hts, wl["sigma"], [5.5, 1000.0])
    assert abs(V1 - Vr) <= 1e-12 * Vr
    assert np.all(np.abs(dV1 - dVr) <= 1e-12 * (np.abs(dVr) + Vr / np.array(wl["sigma"])))
    c2, h2 = pipe.hills_get()
    pipe2 = make_pipe(wl, 100)
    pipe2.hills_set(c2, h2)
    V2, dV2 = pipe2.bias_eval(s)
    assert V2.item() == V1 and np.array_equal(dV2.cpu().numpy(), dV1)


def test_deposit_sampled_heights_wz1m_hills(orc):
    """50,000 deposits (the 1.02M-atom workload's history); every 997th height
    is recomputed by the oracle from the GPU's own earlier hills."""
    wl = W.WORKLOADS["wz1m"]
    hp = wl["hills"]
    cen = W.hill_centres(hp["k"], hp["lo"], hp["hi"], hp["seed"])
    pipe = make_pipe(wl, 1000)
    cdev = to_dev(cen, torch.float64)
    for k in range(len(cen)):
        pipe.deposit_hill(cdev[k])
    gc, gh = pipe.hills_get()
    assert len(gh) == hp["k"] and gh[0] == wl["w0"]
    for k in range(1, hp["k"], 997):
        V, _ = orc.bias(gc[:k], gh[:k], wl["sigma"], gc[k])
        assert abs(gh[k] - orc.wt_height(wl["w0"], wl["gamma"], wl["kBT"], V)) <= 1e-12 * gh[k]


# ---------------------------------------------------------------------------
# Determinism, call order and the sticky errors
# ---------------------------------------------------------------------------
def test_bitwise_determinism():
    d = W.wurtzite_slab(8, 4, 8, seed=5)
    n = len(d["pos"])
    p4 = to_dev(W.as_float4(d["pos"]))
    outs = []
    for _ in range(2):
        pipe = make_pipe(Q6CV, n)
        pipe.hills_set([[float(n) * 0.4]], [0.01])
        pipe.build_neighbors(p4, d["box"])
        F = torch.zeros((n, 4), dtype=torch.float32, device=dev())
        pipe.step(p4, F)
        torch.cuda.synchronize()
        outs.append((pipe.s.cpu().numpy().copy(), F.cpu().numpy().copy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_errors_and_call_order():
    from paper_2510_06873_amd import GmError

    d = W.wurtzite_slab(4, 3, 6, seed=21)
    n = len(d["pos"])
    p4 = to_dev(W.as_float4(d["pos"]))
    pipe = make_pipe(Q6CV, n, max_neighbors=8)
    with pytest.raises(GmError, match="STATE"):
        pipe.cv_forward(p4)
    with pytest.raises(GmError, match="BOX_TOO_SMALL"):
        pipe.build_neighbors(p4, [11.9, 30.0, 30.0])
    pipe.build_neighbors(p4, d["box"])
    assert pipe.status(True) == -5  # rows of ~26 > 8
    assert pipe.status(True) == 0   # cleared
    pipe.build_neighbors_checked(p4, d["box"])
    pipe.cv_forward(p4)
    F = torch.zeros((n, 4), dtype=torch.float32, device=dev())
    with pytest.raises(GmError, match="STATE"):
        pipe.apply_bias_forces(p4, F)
    # backward and the force pass need the positions of the last forward
    other = p4.clone()
    with pytest.raises(GmError, match="STATE"):
        pipe.cv_backward(other)
    pipe.cv_backward(p4)
    with pytest.raises(GmError, match="STATE"):
        pipe.apply_bias_forces(other, F)
    pipe.apply_bias_forces(p4, F)
    bad = p4.clone()
    bad[3, 1] = float("nan")
    pipe.cv_forward(bad)
    assert pipe.status(True) == -7
    small = make_pipe(dict(Q6CV, hills=dict(k=0)), n, hill_capacity=2)
    s = torch.tensor([1.0], dtype=torch.float64, device=dev())
    for _ in range(3):
        small.deposit_hill(s)
    assert small.status(True) == -6
    assert len(small.hills_get()[1]) == 2


# ---------------------------------------------------------------------------
# torch.autograd: V(s(x)).backward() through the hand-written adjoint
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["stored", "recompute", "interleaved"])
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("fp64", 1e-6)])
def test_autograd_2d_bias_gradient(orc, mode, precision, tol):
    from paper_2510_06873_amd.autograd import GaussianBias, cv

    wl = dict(W.WORKLOADS["wz2048"], precision=precision)
    d = W.structure(wl["structure"])
    pos, box = d["pos"], d["box"]
    n = len(pos)
    s_ref, g_ref, _ = oracle_cvs(orc, pos, box, wl)
    sig = np.array(wl["sigma"])
    cen = W.hill_centres(200, s_ref - 3 * sig, s_ref + 3 * sig, seed=15)
    hts = orc.deposit_sequence(cen, sig, wl["w0"], wl["gamma"], wl["kBT"])
    pipe = make_pipe(wl, n)
    pipe.hills_set(cen, hts)
    p4 = to_dev(W.as_float4(pos)).requires_grad_(True)
    pipe.build_neighbors_checked(p4.detach(), box)
    s = cv(p4, pipe, "recompute" if mode == "recompute" else "stored")
    V = GaussianBias.apply(s, pipe)
    if mode == "interleaved":
        pipe.cv_forward(p4.detach())  # a second forward in between: backward must recompute
    V.backward()
    torch.cuda.synchronize()
    s_gpu = s.detach().cpu().numpy()
    assert np.all(np.abs(s_gpu - s_ref) <= (1e-5 if precision == "fp32" else 1e-10) * np.abs(s_ref))
    Vr, dVr = orc.bias(cen, hts, sig, s_gpu)
    assert abs(V.item() - Vr) <= 1e-12 * Vr
    grad_ref = dVr[0] * g_ref[0] + dVr[1] * g_ref[1]
    g = p4.grad.cpu().numpy().astype(np.float64)
    assert rel_force_err(g[:, :3], grad_ref) <= tol
    assert np.all(g[:, 3] == 0)


def test_recompute_mode_holds_no_rows_between_calls():
    """The "recompute" autograd mode gives the per-atom q6 rows back after the
    forward and after the backward, so the context holds 2 x 16 floats per
    atom less between calls, and its gradient equals the stored mode's bit
    for bit (the same kernels on the same state)."""
    from paper_2510_06873_amd.autograd import bias_energy

    wl = dict(W.WORKLOADS["wz2048"], precision="fp32")
    d = W.structure(wl["structure"])
    pos, box = d["pos"], d["box"]
    n = len(pos)
    grads, held = {}, {}
    for mode in ("stored", "recompute"):
        pipe = make_pipe(wl, n)
        p4 = to_dev(W.as_float4(pos))
        pipe.build_neighbors_checked(p4, box)
        s0 = pipe.cv_forward(p4).cpu().numpy().copy()
        sig = np.array(wl["sigma"])
        pipe.hills_set(W.hill_centres(100, s0 - 2 * sig, s0 + 2 * sig, seed=19), np.full(100, wl["w0"]))
        x = p4.clone().requires_grad_(True)
        before = pipe.device_bytes()
        V = bias_energy(x, pipe, mode)
        between = pipe.device_bytes()
        V.backward()
        torch.cuda.synchronize()
        held[mode] = (before, between, pipe.device_bytes())
        grads[mode] = x.grad.cpu().numpy().copy()
        assert pipe.status(True) == 0
        # a forward after the release allocates the rows again
        pipe.step(p4, torch.zeros((n, 4), dtype=torch.float32, device=dev()))
        torch.cuda.synchronize()
        assert pipe.status(True) == 0
        pipe.close()
    rows = 2 * 16 * 4 * n
    b, m, a = held["stored"]
    assert b == m == a
    b_r, m_r, a_r = held["recompute"]
    assert b_r == b and m_r == b - rows and a_r == b - rows
    assert np.array_equal(grads["stored"], grads["recompute"])


def test_autograd_against_finite_differences_of_the_gpu_path():
    """d V(s(x)) / dx from the autograd wrappers against central differences
    of the GPU path itself (FP64 context, 2-D CV, 2,048 atoms): coordinates
    moved by 2^-13 A (exact in FP32 at these magnitudes), Richardson
    extrapolation over h and h/2, lists kept from the unperturbed build."""
    from paper_2510_06873_amd.autograd import bias_energy

    wl = dict(W.WORKLOADS["wz2048"], precision="fp64")
    d = W.structure(wl["structure"])
    pos, box = d["pos"], d["box"]
    n = len(pos)
    pipe = make_pipe(wl, n)
    p4 = to_dev(W.as_float4(pos))
    pipe.build_neighbors_checked(p4, box)
    s0 = pipe.cv_forward(p4).cpu().numpy().copy()
    sig = np.array(wl["sigma"])
    cen = W.hill_centres(300, s0 - 2 * sig, s0 + 2 * sig, seed=17)
    pipe.hills_set(cen, np.full(len(cen), wl["w0"]))
    x = p4.clone().requires_grad_(True)
    bias_energy(x, pipe, "recompute").backward()
    grad = x.grad.cpu().numpy().astype(np.float64)

    def V_at(delta, i, a):
        q = pos.copy()
        q[i, a] = np.float32(np.float64(q[i, a]) + delta)
        assert np.float64(q[i, a]) - np.float64(pos[i, a]) == delta  # the move is exact
        pipe.cv_forward(to_dev(W.as_float4(q)))
        V, _ = pipe.bias_eval()
        return V.item()

    h = 2.0 ** -13
    rng = np.random.default_rng(8)
    big = np.argsort(-np.linalg.norm(grad[:, :3], axis=1))[:6]
    for i in list(big) + list(rng.choice(n, 6, replace=False)):
        for a in range(3):
            d1 = (V_at(h, i, a) - V_at(-h, i, a)) / (2 * h)
            d2 = (V_at(h / 2, i, a) - V_at(-h / 2, i, a)) / h
            fd = (4 * d2 - d1) / 3
            assert abs(fd - grad[i, a]) <= 1e-6 * np.abs(grad[:, :3]).max(), (i, a, fd, grad[i, a])
