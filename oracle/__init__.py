"""Plain FP64 CPU oracle for the metadynamics bias pipeline (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports, links or calls anything here, and this package
imports nothing from the product.

The arithmetic lives in ``oracle.c`` (double precision, single threaded, no FMA
contraction); this module only compiles it with gcc and marshals numpy arrays.
Each function names the passage of the method it follows; the C source carries
the formulas.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class Q6Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("r_c", "taper", "bond_d0", "bond_w", "count_n0", "count_w")]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = C.CDLL(build())
    dp, ip32, ip64 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    lib.gmo_cell_grid.argtypes = [dp, C.c_double, ip32]
    lib.gmo_cell_grid.restype = C.c_int
    lib.gmo_cell_ids.argtypes = [dp, C.c_int64, dp, ip32, ip32]
    lib.gmo_cell_sort.argtypes = [ip32, C.c_int64, C.c_int64, ip32, ip32]
    for f in (lib.gmo_neighbors_brute, lib.gmo_neighbors_cells):
        f.argtypes = [dp, C.c_int64, dp, C.c_double, ip64, ip32, C.c_int64]
        f.restype = C.c_int64
    lib.gmo_cn_forward.argtypes = [dp, C.c_int64, dp, ip64, ip32, C.c_double, C.c_double, dp]
    lib.gmo_cn_forward.restype = C.c_double
    lib.gmo_cn_gradient.argtypes = [dp, C.c_int64, dp, ip64, ip32, C.c_double, C.c_double, dp]
    lib.gmo_ylm6_complex.argtypes = [dp, dp, dp]
    lib.gmo_ylm6_real.argtypes = [dp, dp]
    lib.gmo_q6_forward.argtypes = [dp, C.c_int64, dp, ip64, ip32, C.POINTER(Q6Params)] + [dp] * 7
    lib.gmo_q6_forward.restype = C.c_double
    lib.gmo_q6_gradient.argtypes = [dp, C.c_int64, dp, ip64, ip32, C.POINTER(Q6Params), dp]
    lib.gmo_bias.argtypes = [dp, dp, C.c_int64, C.c_int, dp, dp, dp, dp, dp]
    lib.gmo_wt_height.argtypes = [C.c_double] * 4
    lib.gmo_wt_height.restype = C.c_double
    lib.gmo_deposit_sequence.argtypes = [dp, C.c_int64, C.c_int, dp, dp, C.c_double, C.c_double, C.c_double, dp]
    lib.gmo_torsions.argtypes = [dp, dp, ip32, C.c_int64, dp, dp]
    lib.gmo_nearest_distance.argtypes = [dp, dp, C.c_int32, ip32, C.c_int64, ip32, dp]
    lib.gmo_nearest_distance.restype = C.c_double
    lib.gmo_fes_reweight.argtypes = [dp, dp, C.c_int64, C.c_int, dp, dp, ip32, C.c_double, dp]
    lib.gmo_fes_hills.argtypes = [dp, dp, C.c_int64, C.c_int, dp, dp, C.c_double, dp, dp, ip32, dp]
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def _positions(pos):
    """Oracle positions: the FP32 input values promoted to FP64, shape (N, 3)."""
    pos = np.asarray(pos)
    return _d(pos[:, :3].astype(np.float64))


# --------------------------------------------------------------------------
# Cell list and neighbour sets
# --------------------------------------------------------------------------
def cell_grid(box, r_list):
    """Cells per axis, n_a = floor(L_a / r_list) (>= 3), or raises ValueError."""
    lib = _load()
    nc = np.zeros(3, np.int32)
    rc = lib.gmo_cell_grid(_p(_d(box)), float(r_list), _p(nc, C.c_int32))
    if rc != 0:
        raise ValueError("box too small for r_list" if rc == -4 else "invalid r_list")
    return nc


def cell_list(pos, box, r_list):
    """(ncell[3], cell[N], perm[N], cell_start[ncells+1]) of the counting sort."""
    lib = _load()
    x = _positions(pos)
    n = x.shape[0]
    nc = cell_grid(box, r_list)
    ncells = int(nc[0]) * int(nc[1]) * int(nc[2])
    cell = np.zeros(n, np.int32)
    perm = np.zeros(n, np.int32)
    start = np.zeros(ncells + 1, np.int32)
    lib.gmo_cell_ids(_p(x), n, _p(_d(box)), _p(nc, C.c_int32), _p(cell, C.c_int32))
    lib.gmo_cell_sort(_p(cell, C.c_int32), n, ncells, _p(perm, C.c_int32), _p(start, C.c_int32))
    return nc, cell, perm, start


def neighbors(pos, box, r_list, method="cells"):
    """Full neighbour lists as CSR (offsets[N+1] int64, nbr int32), rows ascending."""
    lib = _load()
    x = _positions(pos)
    n = x.shape[0]
    fn = lib.gmo_neighbors_cells if method == "cells" else lib.gmo_neighbors_brute
    off = np.zeros(n + 1, np.int64)
    cap = max(64 * n, 1)
    nbr = np.zeros(cap, np.int32)
    tot = fn(_p(x), n, _p(_d(box)), float(r_list), _p(off, C.c_int64), _p(nbr, C.c_int32), cap)
    if tot < 0:
        raise ValueError("box too small for r_list")
    if tot > cap:
        nbr = np.zeros(tot, np.int32)
        tot = fn(_p(x), n, _p(_d(box)), float(r_list), _p(off, C.c_int64), _p(nbr, C.c_int32), tot)
    return off, nbr[:tot].copy()


# --------------------------------------------------------------------------
# Collective variables
# --------------------------------------------------------------------------
def cn_forward(pos, box, nl, r0, r_c, per_atom=False):
    """Mean coordination number s_CN and optionally per-atom sums."""
    lib = _load()
    x = _positions(pos)
    off, nbr = nl
    out = np.zeros(x.shape[0]) if per_atom else None
    s = lib.gmo_cn_forward(_p(x), x.shape[0], _p(_d(box)), _p(off, C.c_int64), _p(nbr, C.c_int32),
                           float(r0), float(r_c), _p(out))
    return (s, out) if per_atom else s


def cn_gradient(pos, box, nl, r0, r_c):
    """ds_CN/dx, shape (N, 3)."""
    lib = _load()
    x = _positions(pos)
    off, nbr = nl
    g = np.zeros_like(x)
    lib.gmo_cn_gradient(_p(x), x.shape[0], _p(_d(box)), _p(off, C.c_int64), _p(nbr, C.c_int32),
                        float(r0), float(r_c), _p(g))
    return g


def ylm6_complex(u):
    """Complex Y_6m(u) for m = 0..6 (orthonormal, Condon-Shortley phase)."""
    lib = _load()
    re = np.zeros(7)
    im = np.zeros(7)
    lib.gmo_ylm6_complex(_p(_d(u)), _p(re), _p(im))
    return re + 1j * im


def ylm6_real(u):
    """Real 13-vector (Y_60, sqrt2 Re/Im Y_6m for m = 1..6)."""
    lib = _load()
    v = np.zeros(13)
    lib.gmo_ylm6_real(_p(_d(u)), _p(v))
    return v


def q6_params(r_c, taper, bond_d0, bond_w, count_n0, count_w):
    return Q6Params(r_c, taper, bond_d0, bond_w, count_n0, count_w)


def q6_forward(pos, box, nl, prm: Q6Params):
    """q6 crystalline count and its intermediates, as a dict of numpy arrays."""
    lib = _load()
    x = _positions(pos)
    n = x.shape[0]
    off, nbr = nl
    out = {k: np.zeros((n, 13)) for k in ("Q", "qhat")}
    out.update({k: np.zeros(n) for k in ("qnorm", "nb", "c", "dc", "fsum")})
    s = lib.gmo_q6_forward(_p(x), n, _p(_d(box)), _p(off, C.c_int64), _p(nbr, C.c_int32), C.byref(prm),
                           _p(out["Q"]), _p(out["qhat"]), _p(out["qnorm"]), _p(out["nb"]), _p(out["c"]),
                           _p(out["dc"]), _p(out["fsum"]))
    out["s"] = s
    fs = np.where(out["fsum"] > 0, out["fsum"], 1.0)
    # Steinhardt q6_i = sqrt(4 pi / 13 sum_m |Q_im / sum_j f_ij|^2)
    out["q6"] = np.sqrt(4 * np.pi / 13.0) * out["qnorm"] / fs
    return out


def q6_gradient(pos, box, nl, prm: Q6Params):
    """ds_Q6/dx, shape (N, 3)."""
    lib = _load()
    x = _positions(pos)
    off, nbr = nl
    g = np.zeros_like(x)
    lib.gmo_q6_gradient(_p(x), x.shape[0], _p(_d(box)), _p(off, C.c_int64), _p(nbr, C.c_int32),
                        C.byref(prm), _p(g))
    return g


# --------------------------------------------------------------------------
# Bias and hills
# --------------------------------------------------------------------------
def _period(period, dims):
    return None if period is None else _d(np.broadcast_to(np.asarray(period, np.float64), (dims,)))


def bias(centres, heights, sigma, s, period=None):
    """(V, dV/ds) of the Gaussian-hill sum at CV value s; period[d] > 0 makes
    dimension d periodic (nearest image of s - c)."""
    lib = _load()
    s = _d(np.atleast_1d(s))
    dims = s.shape[0]
    c = _d(np.asarray(centres).reshape(-1, dims))
    h = _d(heights)
    V = np.zeros(1)
    g = np.zeros(dims)
    per = _period(period, dims)
    lib.gmo_bias(_p(c), _p(h), h.shape[0], dims, _p(_d(np.atleast_1d(sigma))), _p(per) if per is not None else None,
                 _p(s), _p(V), _p(g))
    return float(V[0]), g


def wt_height(w0, gamma, kBT, V):
    return _load().gmo_wt_height(float(w0), float(gamma), float(kBT), float(V))


def deposit_sequence(centres, sigma, w0, gamma, kBT, period=None):
    """Heights of hills deposited in index order at the given centres."""
    lib = _load()
    sigma = _d(np.atleast_1d(sigma))
    dims = sigma.shape[0]
    c = _d(np.asarray(centres).reshape(-1, dims))
    h = np.zeros(c.shape[0])
    per = _period(period, dims)
    lib.gmo_deposit_sequence(_p(c), c.shape[0], dims, _p(sigma), _p(per) if per is not None else None,
                             float(w0), float(gamma), float(kBT), _p(h))
    return h


def torsions(pos, box, quads):
    """(phi[m], grad[m][4][3]) of the torsion angles of the atom quadruples
    (IUPAC sign, minimum images)."""
    lib = _load()
    x = _d(np.asarray(pos)[:, :3])
    q = np.ascontiguousarray(np.asarray(quads, np.int32).reshape(-1, 4))
    phi = np.zeros(q.shape[0])
    g = np.zeros((q.shape[0], 4, 3))
    lib.gmo_torsions(_p(x), _p(_d(box)), q.ctypes.data_as(C.POINTER(C.c_int32)), q.shape[0], _p(phi), _p(g))
    return phi, g


def nearest_distance(pos, box, centre, members):
    """(s, nearest atom, unit vector centre -> nearest) over the member set."""
    lib = _load()
    x = _d(np.asarray(pos)[:, :3])
    m = np.ascontiguousarray(np.asarray(members, np.int32))
    arg = np.zeros(1, np.int32)
    u = np.zeros(3)
    s = lib.gmo_nearest_distance(_p(x), _p(_d(box)), int(centre), m.ctypes.data_as(C.POINTER(C.c_int32)),
                                 m.shape[0], arg.ctypes.data_as(C.POINTER(C.c_int32)), _p(u))
    return float(s), int(arg[0]), u


def fes_reweight(s, V, lo, hi, nbins, kBT):
    """F per bin (bin id i0 + nb0 i1) from samples (s_t, V_t) of a biased run."""
    lib = _load()
    s = np.asarray(s, np.float64)
    dims = 1 if s.ndim == 1 else s.shape[1]
    s = _d(s.reshape(-1, dims))
    V = _d(V)
    nb = np.ascontiguousarray(np.atleast_1d(nbins).astype(np.int32))
    F = np.zeros(int(np.prod(nb)))
    lib.gmo_fes_reweight(_p(s), _p(V), s.shape[0], dims, _p(_d(np.atleast_1d(lo))), _p(_d(np.atleast_1d(hi))),
                         nb.ctypes.data_as(C.POINTER(C.c_int32)), float(kBT), _p(F))
    return F


def fes_hills(centres, heights, sigma, lo, hi, nbins, gamma=0.0, period=None):
    """F = -V (or -gamma/(gamma-1) V, well-tempered) on the grid of bin centres."""
    lib = _load()
    sigma = _d(np.atleast_1d(sigma))
    dims = sigma.shape[0]
    c = _d(np.asarray(centres).reshape(-1, dims))
    h = _d(heights)
    nb = np.ascontiguousarray(np.atleast_1d(nbins).astype(np.int32))
    F = np.zeros(int(np.prod(nb)))
    per = _period(period, dims)
    lib.gmo_fes_hills(_p(c), _p(h), h.shape[0], dims, _p(sigma), _p(per) if per is not None else None,
                      float(gamma), _p(_d(np.atleast_1d(lo))), _p(_d(np.atleast_1d(hi))),
                      nb.ctypes.data_as(C.POINTER(C.c_int32)), _p(F))
    return F


# --------------------------------------------------------------------------
# Whole pipeline step
# --------------------------------------------------------------------------
def bias_forces(F_in, grads, dVds):
    """F_out = F_in - sum_d dV/ds_d * ds_d/dx  (biased potential U_b = U_0 + V_b)."""
    F = np.asarray(F_in, dtype=np.float64)[:, :3].copy()
    for g, dv in zip(grads, np.atleast_1d(dVds)):
        F -= dv * g
    return F
