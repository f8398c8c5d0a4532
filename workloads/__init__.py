"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle's.

This module holds no arithmetic of the method (no CV, bias or force); it only
builds atom positions, external forces and hill centres from seeds, plus the
parameter sets of the standard workloads.  Both sides read the same FP32
positions; the oracle promotes them to FP64.

Workloads (the GaN-like and Cu-like systems stand in for the paper's GaN NEP
runs and benchmarks, whose datasets and trained potentials are not available):

* ``fcc864``   fcc 6x6x6 cells, a = 3.615 A, jitter N(0, 0.1 A); coordination CV,
               FP64; 1-D well-tempered bias from 1,000 hills.
* ``wz96k``    wurtzite 40x40x15 hexagonal cells as a 40x20x15 orthohexagonal
               grid (8 atoms each); lower z half crystal (jitter 0.05 A), upper
               half random sequential addition at the same density with a
               1.6 A minimum distance; q6 crystalline count, 10,000 hills.
* ``wz1m``     the same recipe at 80x40x40 orthohexagonal cells, 1,024,000 atoms,
               50,000 hills, external forces N(0, 1 eV/A).
* ``wz2048``   8x4x8 slab, 2-D CV (coordination + q6 count), 5,000 hills.
* ``wz262k``   64x32x16 orthohexagonal crystal slab, 2-D CV, timing size.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

# 1.2 kJ/mol expressed in eV, and k_B T at 300 K in kJ/mol and in eV.
KJMOL_PER_EV = 96.48533212
KB_EV = 8.617333262e-5
KB_KJMOL = 0.0083144626


def _cache_dir():
    d = os.environ.get("GPUMETAD_CACHE", "/tmp/gpumetad_inputs")
    os.makedirs(d, exist_ok=True)
    return d


def _cached(tag: str, spec: dict, fn):
    key = hashlib.sha1(json.dumps(spec, sort_keys=True).encode()).hexdigest()[:16]
    path = os.path.join(_cache_dir(), f"{tag}_{key}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return {k: z[k] for k in z.files}
    out = fn()
    tmp = path + ".tmp%d.npz" % os.getpid()
    np.savez(tmp, **out)
    os.replace(tmp, path)
    return out


def _wrap_f32(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Wrap into [0, L), round to FP32; a value that rounds up to L becomes 0."""
    w = np.mod(x, box)
    f = w.astype(np.float32)
    for a in range(3):
        col = f[:, a]
        col[col.astype(np.float64) >= box[a]] = np.float32(0.0)
        col[col < 0] = np.float32(0.0)
    return f


# --------------------------------------------------------------------------
# Lattices
# --------------------------------------------------------------------------
def fcc_ideal(n: int, a: float):
    """Ideal fcc positions (4 n^3 atoms) and the cubic box."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    pos = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return pos, np.array([n * a] * 3, dtype=np.float64)


def wurtzite_ortho_cell(a: float, c: float, u: float):
    """8-atom orthohexagonal wurtzite cell (a, a*sqrt3, c); species 0 (Ga), 1 (N)."""
    s3 = np.sqrt(3.0)
    ga = np.array([[0.0, a * s3 / 3.0, 0.0],
                   [a / 2.0, a * s3 / 6.0, c / 2.0],
                   [a / 2.0, 5.0 * a * s3 / 6.0, 0.0],
                   [0.0, 2.0 * a * s3 / 3.0, c / 2.0]])
    n = ga + np.array([0.0, 0.0, u * c])
    pos = np.concatenate([ga, n])
    species = np.array([0] * 4 + [1] * 4, dtype=np.int32)
    return pos, species, np.array([a, a * s3, c])


def wurtzite_ideal(nx: int, ny: int, nz: int, a=3.19, c=5.19, u=0.377):
    """Ideal wurtzite on an nx x ny x nz grid of orthohexagonal cells."""
    cell, sp, L = wurtzite_ortho_cell(a, c, u)
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    pos = (g[:, None, :] * L[None, None, :] + cell[None, :, :]).reshape(-1, 3)
    species = np.tile(sp, g.shape[0])
    return pos, species, L * np.array([nx, ny, nz], dtype=np.float64)


# --------------------------------------------------------------------------
# Random sequential addition
# --------------------------------------------------------------------------
def rsa_fill(fixed: np.ndarray, n_new: int, box: np.ndarray, zlo: float, zhi: float,
             dmin: float, rng: np.random.Generator, batch: int = 60000) -> np.ndarray:
    """Place n_new points uniformly in z in [zlo, zhi), one after another, each
    accepted only if it is at least dmin (periodic) from every point already
    placed, fixed points included.  Candidates are drawn in batches; inside a
    batch they are accepted greedily in draw order, which is the sequential rule."""
    from scipy.spatial import cKDTree

    if n_new == 0:
        return np.zeros((0, 3))
    span = np.array([box[0], box[1], zhi - zlo])
    lo = np.array([0.0, 0.0, zlo])
    # Only fixed points within dmin of the slab (through periodic z) can interfere.
    zf = np.mod(fixed[:, 2], box[2])
    inside = (zf >= zlo) & (zf < zhi)
    below = np.mod(zlo - zf, box[2]) < dmin
    above = np.mod(zf - zhi, box[2]) < dmin
    constraint = np.mod(fixed[inside | below | above], box)
    placed = []
    n_acc = 0
    while n_acc < n_new:
        pts = np.concatenate([constraint] + placed) if placed else constraint
        tree = cKDTree(np.mod(pts, box), boxsize=box)
        nb = int(min(batch, max(256, 2 * (n_new - n_acc))))
        cand = lo + rng.random((nb, 3)) * span
        cand[:, 2] = np.minimum(cand[:, 2], np.nextafter(zhi, zlo))
        d, _ = tree.query(cand, k=1, distance_upper_bound=dmin)
        surv = cand[~(d < dmin)]
        if surv.shape[0] == 0:
            continue
        pairs = cKDTree(surv, boxsize=box).query_pairs(dmin, output_type="ndarray")
        ok = np.ones(surv.shape[0], dtype=bool)
        if pairs.size:
            pairs = pairs[np.argsort(pairs[:, 1], kind="stable")]
            for i, j in pairs:
                if ok[i]:
                    ok[j] = False
        acc = surv[ok][: n_new - n_acc]
        placed.append(acc)
        n_acc += acc.shape[0]
    return np.concatenate(placed)


def wurtzite_slab(nx, ny, nz, a=3.19, c=5.19, u=0.377, jitter=0.05, dmin=1.6, seed=0,
                  random_half=True):
    """Wurtzite slab: atoms whose ideal z < Lz/2 keep the crystal sites plus
    N(0, jitter) noise; the rest are replaced by random sequential addition in
    [Lz/2, Lz) at the same count (so N and the density are unchanged)."""
    spec = dict(kind="wz_slab", nx=nx, ny=ny, nz=nz, a=a, c=c, u=u, jitter=jitter, dmin=dmin,
                seed=seed, random_half=random_half, v=3)

    def make():
        rng = np.random.default_rng(seed)
        ideal, species, box = wurtzite_ideal(nx, ny, nz, a, c, u)
        pos = ideal + rng.normal(0.0, jitter, ideal.shape)
        if random_half:
            crystal = ideal[:, 2] < box[2] / 2.0
            n_rand = int((~crystal).sum())
            keep = np.mod(pos[crystal], box)
            rnd = rsa_fill(keep, n_rand, box, box[2] / 2.0, box[2], dmin, rng)
            pos = np.concatenate([pos[crystal], rnd])
            species = np.concatenate([species[crystal], species[~crystal]])
            n_crystal = int(crystal.sum())
        else:
            n_crystal = pos.shape[0]
        return dict(pos=_wrap_f32(pos, box), species=species.astype(np.int32), box=box,
                    n_crystal=np.array(n_crystal))

    return _cached("wz", spec, make)


def fcc_jittered(n=6, a=3.615, jitter=0.1, seed=1):
    spec = dict(kind="fcc", n=n, a=a, jitter=jitter, seed=seed, v=1)

    def make():
        rng = np.random.default_rng(seed)
        ideal, box = fcc_ideal(n, a)
        pos = ideal + rng.normal(0.0, jitter, ideal.shape)
        return dict(pos=_wrap_f32(pos, box), species=np.zeros(pos.shape[0], np.int32), box=box,
                    n_crystal=np.array(pos.shape[0]))

    return _cached("fcc", spec, make)


def as_float4(pos: np.ndarray, species: np.ndarray | None = None) -> np.ndarray:
    """(N, 4) float32: x, y, z and the species id in the fourth lane."""
    out = np.zeros((pos.shape[0], 4), np.float32)
    out[:, :3] = pos[:, :3]
    if species is not None:
        out[:, 3] = species.astype(np.float32)
    return out


def external_forces(n: int, sigma: float = 1.0, seed: int = 4) -> np.ndarray:
    """(N, 4) float32 forces from the interatomic potential stand-in: N(0, sigma)."""
    rng = np.random.default_rng(seed)
    f = np.zeros((n, 4), np.float32)
    f[:, :3] = rng.normal(0.0, sigma, (n, 3)).astype(np.float32)
    return f


def hill_centres(k: int, lo, hi, seed: int) -> np.ndarray:
    """(K, dims) float64 centres drawn uniformly in [lo, hi) per dimension, in
    deposition order."""
    lo = np.atleast_1d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(hi, dtype=np.float64))
    rng = np.random.default_rng(seed)
    return lo + rng.random((k, lo.shape[0])) * (hi - lo)


# --------------------------------------------------------------------------
# Standard workloads: geometry recipe + CV / bias parameters
# --------------------------------------------------------------------------
W0_EV = 1.2 / KJMOL_PER_EV
KBT_EV = KB_EV * 300.0
KBT_KJMOL = KB_KJMOL * 300.0

Q6_CV = dict(r_c=3.6, skin=0.4, taper=0.2, bond_d0=0.7, bond_w=0.02, count_n0=5.5, count_w=0.25)

WORKLOADS = {
    "fcc864": dict(structure=dict(kind="fcc", n=6, a=3.615, jitter=0.1, seed=1),
                   cv="coord", precision="fp64", r_c=6.0, skin=0.5, cn_r0=3.0, taper=0.0,
                   hills=dict(k=1000, lo=[0.0], hi=[14.0], seed=11), sigma=[0.1],
                   w0=1.2, gamma=10.0, kBT=KBT_KJMOL),
    "wz96k": dict(structure=dict(kind="wz", nx=40, ny=20, nz=15, seed=2),
                  cv="q6", precision="fp32", **Q6_CV, cn_r0=2.5,
                  hills=dict(k=10000, lo=[0.0], hi=[96000.0], seed=12), sigma=[20.0],
                  w0=W0_EV, gamma=10.0, kBT=KBT_EV),
    "wz1m": dict(structure=dict(kind="wz", nx=80, ny=40, nz=40, seed=3),
                 cv="q6", precision="fp32", **Q6_CV, cn_r0=2.5,
                 hills=dict(k=50000, lo=[0.0], hi=[1.02e6], seed=13), sigma=[200.0],
                 w0=W0_EV, gamma=10.0, kBT=KBT_EV, force_seed=4),
    "wz2048": dict(structure=dict(kind="wz", nx=8, ny=4, nz=8, seed=5),
                   cv="coord_q6", precision="fp32", **Q6_CV, cn_r0=2.5,
                   hills=dict(k=5000, centre_rel=10.0, seed=15), sigma=[0.05, 20.0],
                   w0=W0_EV, gamma=10.0, kBT=KBT_EV),
    "wz262k": dict(structure=dict(kind="wz", nx=64, ny=32, nz=16, seed=6),
                   cv="coord_q6", precision="fp32", **Q6_CV, cn_r0=2.5,
                   hills=dict(k=5000, centre_rel=10.0, seed=16), sigma=[0.05, 20.0],
                   w0=W0_EV, gamma=10.0, kBT=KBT_EV),
}


def structure(spec: dict):
    """Positions (N,3) float32, species, box, n_crystal for a structure spec."""
    s = dict(spec)
    kind = s.pop("kind")
    if kind == "fcc":
        return fcc_jittered(**s)
    if kind == "wz":
        return wurtzite_slab(**s)
    raise ValueError(kind)


def small_wurtzite_slab(nx=4, ny=3, nz=6, seed=21, jitter=0.05):
    """A small slab (a few hundred atoms) with crystal and random halves."""
    return wurtzite_slab(nx, ny, nz, jitter=jitter, seed=seed)


# --------------------------------------------------------------------------
# Serving: many uneven walkers with Poisson arrivals
# --------------------------------------------------------------------------
WALKER_CV = {
    # (structure, cv): CV parameters
    ("fcc", "coord"): dict(cv="coord", r_c=6.0, skin=0.5, cn_r0=3.0, taper=0.2, sigma=[0.1], kmax=128),
    ("fcc", "q6"): dict(cv="q6", r_c=3.2, skin=0.4, cn_r0=2.5, taper=0.2, sigma=[20.0], kmax=48),
    ("wz", "coord"): dict(cv="coord", r_c=3.6, skin=0.4, cn_r0=2.5, taper=0.2, sigma=[0.1], kmax=48),
    ("wz", "q6"): dict(cv="q6", r_c=3.6, skin=0.4, cn_r0=2.5, taper=0.2, sigma=[20.0], kmax=48),
}


def walker_structure(kind: str, n_target: int, seed: int):
    """Near-cubic crystal of about n_target atoms with N(0, jitter) noise
    (fcc a = 3.615, jitter 0.1; wurtzite jitter 0.05), large enough for 3 cells
    of the walker's neighbour cutoff on every axis."""
    rng = np.random.default_rng(seed)
    if kind == "fcc":
        n = max(6, int(round((n_target / 4) ** (1 / 3))))
        ideal, box = fcc_ideal(n, 3.615)
        jit = 0.1
        species = np.zeros(ideal.shape[0], np.int32)
    else:
        side = (n_target / 0.08745) ** (1 / 3)
        nx = max(4, int(round(side / 3.19)))
        ny = max(3, int(round(side / (3.19 * np.sqrt(3)))))
        nz = max(3, int(round(side / 5.19)))
        ideal, species, box = wurtzite_ideal(nx, ny, nz)
        jit = 0.05
    pos = ideal + rng.normal(0.0, jit, ideal.shape)
    return _wrap_f32(pos, box), species, box


def serving_requests(count=256, n_lo=1000, n_hi=200000, rate=2000.0, k_lo=100, k_hi=20000, seed=7):
    """Walker requests: atom counts log-uniform in [n_lo, n_hi], fcc or wurtzite
    and coordination or q6 count with equal odds, hill histories log-uniform in
    [k_lo, k_hi] (centres around the range the CV can take, heights in
    [0.2, 1] w0), Poisson arrival times at `rate` per second.  Plain arrays and
    parameter dicts; the caller turns them into library objects."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for i in range(count):
        n_t = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        kind = "fcc" if rng.random() < 0.5 else "wz"
        cv = "coord" if rng.random() < 0.5 else "q6"
        pos, species, box = walker_structure(kind, n_t, seed=1000 + i)
        n = pos.shape[0]
        prm = dict(WALKER_CV[(kind, cv)])
        k = int(np.exp(rng.uniform(np.log(k_lo), np.log(k_hi))))
        hi = (14.0 if kind == "fcc" else 8.0) if cv == "coord" else 1.05 * n
        centres = rng.uniform(0.0, hi, (k, 1))
        w0 = W0_EV
        heights = w0 * rng.uniform(0.2, 1.0, k)
        forces = external_forces(n, seed=5000 + i)
        out.append(dict(rid=i, arrival=float(t[i]), pos=as_float4(pos, species), box=box, kind=kind, params=prm,
                        centres=centres, heights=heights, forces=forces, w0=w0, kBT=KBT_EV))
    return out


# --------------------------------------------------------------------------
# Stand-ins for the paper's small-CV studies (their molecules, NEP models and
# trajectories are not available): geometry and random numbers only.
# --------------------------------------------------------------------------
def peptide_in_solvent(n_solvent=3000, box=(32.0, 32.0, 32.0), seed=41):
    """An alanine-dipeptide-sized chain (22 atoms: a random backbone walk of
    1.5 A bonds at ~111 degree angles, side atoms hung off it) in a box of
    random solvent sites.  Returns positions (float32, wrapped), the box, the
    22 chain atom ids and two backbone quadruples standing for Phi(C-N-CA-C)
    and Psi(N-CA-C-N), plus 30 further random quadruples of chain atoms."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, np.float64)
    chain = np.zeros((22, 3))
    chain[0] = box / 2
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    turn = np.radians(180.0 - 111.0)  # direction change for a 111 degree bond angle
    for i in range(1, 10):  # backbone
        nd = rng.normal(size=3)
        nd -= nd.dot(d) * d
        nd /= np.linalg.norm(nd)
        d = np.cos(turn) * d + np.sin(turn) * nd
        chain[i] = chain[i - 1] + 1.5 * d
    for i in range(10, 22):  # side atoms, 1.1 A off a backbone atom
        v = rng.normal(size=3)
        chain[i] = chain[rng.integers(0, 10)] + 1.1 * v / np.linalg.norm(v)
    solvent = rng.random((n_solvent, 3)) * box
    pos = np.concatenate([chain, solvent])
    order = rng.permutation(len(pos))  # the chain scattered through the atom order
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    pos = pos[order]
    ids = inv[:22]
    quads = [[ids[2], ids[3], ids[4], ids[5]], [ids[3], ids[4], ids[5], ids[6]]]
    for _ in range(30):
        quads.append(list(rng.choice(ids, 4, replace=False)))
    return dict(pos=_wrap_f32(pos, box), box=box, chain=ids.astype(np.int32), quads=np.asarray(quads, np.int32))


def surface_water(n_atoms=4000, n_h=800, box=(26.0, 26.0, 40.0), seed=43):
    """A rutile-surface-with-water stand-in: random sites in the box, a chosen
    centre (the surface oxygen) and a set of hydrogen sites.  Returns
    positions (float32), box, centre id and the hydrogen ids."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, np.float64)
    pos = rng.random((n_atoms, 3)) * box
    h = np.sort(rng.choice(n_atoms, n_h, replace=False)).astype(np.int32)
    others = np.setdiff1d(np.arange(n_atoms), h)
    return dict(pos=_wrap_f32(pos, box), box=box, centre=int(rng.choice(others)), hydrogens=h)


def biased_trace(T=200000, dims=2, seed=45, periodic=True):
    """Samples (s_t, V_t) of a biased run stand-in: s from a mixture of
    Gaussians (wrapped to [-pi, pi) when periodic), V from a sum of 64 random
    Gaussian hills at those points (float64)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-2.5, 2.5, (4, dims))
    comp = rng.integers(0, 4, T)
    s = mu[comp] + rng.normal(0.0, 0.6, (T, dims))
    if periodic:
        s = (s + np.pi) % (2 * np.pi) - np.pi
    c = rng.uniform(-np.pi, np.pi, (64, dims))
    h = rng.uniform(0.5, 2.0, 64)
    V = np.zeros(T)
    for k in range(64):
        V += h[k] * np.exp(-np.sum((s - c[k]) ** 2, axis=1) / (2 * 0.5 ** 2))
    return s.reshape(T, dims) if dims > 1 else s[:, 0], V


def cluster_in_gas(n_cluster=900, n_gas=3000, box=(40.0, 40.0, 40.0), edge=12.0, corner=(13.3, 9.7, 21.1),
                   dmin=1.1, seed=47):
    """A dense cluster in a gas: n_cluster atoms in a cube of the given edge
    (about 0.5 atoms/A^3) and n_gas atoms over the whole box, no two closer
    than dmin through the periodic faces (random sequential addition).  Bricks
    sized for the mean density then see halos far larger than expected near
    the cluster.  Returns positions (float32) and the box."""
    spec = dict(n_cluster=n_cluster, n_gas=n_gas, box=list(box), edge=edge, corner=list(corner), dmin=dmin,
                seed=seed)

    def make():
        rng = np.random.default_rng(seed)
        L = np.asarray(box, np.float64)
        placed = np.zeros((n_cluster + n_gas, 3))
        count = 0
        for n, lo, span in ((n_cluster, np.asarray(corner, np.float64), np.full(3, edge)),
                            (n_gas, np.zeros(3), L)):
            got = 0
            while got < n:
                x = lo + rng.random(3) * span
                d = placed[:count] - x
                d -= L * np.rint(d / L)
                if count == 0 or np.min(np.einsum("ij,ij->i", d, d)) >= dmin * dmin:
                    placed[count] = x
                    count += 1
                    got += 1
        return dict(pos=_wrap_f32(placed, L), box=L)

    return _cached("cluster_in_gas", spec, make)
