"""ctypes binding of libgpumetad (the C-ABI in include/gpumetad.h).

Argument marshalling only: every step of the pipeline runs in the HIP library.
Tensors are torch CUDA tensors (device memory and streams); their data
pointers go straight to the C calls.  There is no CPU fallback: if the library
is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpumetad.so")

GM_OK = 0
ERRORS = {
    -1: "GM_ERR_INVALID_ARG", -2: "GM_ERR_OOM", -3: "GM_ERR_HIP", -4: "GM_ERR_BOX_TOO_SMALL",
    -5: "GM_ERR_NEIGHBOR_OVERFLOW", -6: "GM_ERR_HILL_CAPACITY", -7: "GM_ERR_NONFINITE", -8: "GM_ERR_STATE",
    -9: "GM_ERR_TOO_LARGE",
}
CV_COORD, CV_Q6COUNT, CV_COORD_Q6, CV_EXTERNAL = 1, 2, 3, 4
FP32, FP64 = 0, 1
ATOM_Q6, ATOM_NB, ATOM_C, ATOM_CN = 1, 2, 3, 4

# Every symbol include/gpumetad.h declares.
EXPORTS = (
    "gm_create", "gm_destroy", "gm_set_stream", "gm_build_neighbors", "gm_cv_forward", "gm_bias_eval",
    "gm_cv_backward", "gm_apply_bias_forces", "gm_deposit_hill", "gm_hills_get", "gm_hills_set", "gm_status",
    "gm_strerror", "gm_neighbor_stats", "gm_release_rows", "gm_device_bytes", "gm_hills_set_device",
    "gm_status_copy", "gm_status_decode", "gm_reserve_neighbors",
    "gm_copy_cell_list", "gm_copy_neighbors", "gm_atom_values", "gm_version",
    "gm_batch_create", "gm_batch_destroy", "gm_batch_update", "gm_batch_build", "gm_batch_build_some",
    "gm_batch_step", "gm_batch_deposit", "gm_batch_deposit_some", "gm_batch_values",
    "gm_torsions", "gm_torsion_forces", "gm_nearest_distance", "gm_nearest_distance_forces",
    "gm_lattice_virial", "gm_fes_reweight", "gm_fes_reweight_noalloc", "gm_fes_hills",
)


class GmError(RuntimeError):
    def __init__(self, code: int, call: str):
        self.code = code
        msg = _lib.gm_strerror(code).decode() if _lib is not None else ""
        super().__init__(f"{call}: {ERRORS.get(code, code)} ({msg})")


class GmParams(C.Structure):
    _fields_ = [
        ("cv_kind", C.c_int32), ("precision", C.c_int32),
        ("r_c", C.c_double), ("skin", C.c_double), ("taper", C.c_double), ("cn_r0", C.c_double),
        ("bond_d0", C.c_double), ("bond_w", C.c_double), ("count_n0", C.c_double), ("count_w", C.c_double),
        ("sigma", C.c_double * 2), ("w0", C.c_double), ("gamma", C.c_double), ("kBT", C.c_double),
        ("hill_capacity", C.c_int64), ("max_neighbors", C.c_int32), ("brick", C.c_int32 * 3), ("lds_kb", C.c_int32),
        ("period", C.c_double * 2), ("dims", C.c_int32), ("tpa", C.c_int32),
    ]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_06873_amd.build` "
                          "(hipcc, gfx950); there is no CPU fallback")
    # torch ships its own HIP runtime; load it first so that the library binds
    # to the same one (two runtimes in one process do not share device memory
    # or streams, and the library's allocations then fail)
    import torch  # noqa: F401

    lib = C.CDLL(LIB_PATH)
    vp, dp, ip32, ip64 = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sig = {
        "gm_create": ([C.POINTER(C.c_void_p), C.POINTER(GmParams), C.c_int64, vp], C.c_int),
        "gm_destroy": ([vp], C.c_int),
        "gm_set_stream": ([vp, vp], C.c_int),
        "gm_build_neighbors": ([vp, vp, dp], C.c_int),
        "gm_cv_forward": ([vp, vp, vp], C.c_int),
        "gm_bias_eval": ([vp, vp, vp, vp], C.c_int),
        "gm_cv_backward": ([vp, vp, vp, vp], C.c_int),
        "gm_apply_bias_forces": ([vp, vp, vp, vp], C.c_int),
        "gm_deposit_hill": ([vp, vp], C.c_int),
        "gm_hills_get": ([vp, dp, dp, C.c_int64, ip64], C.c_int),
        "gm_hills_set": ([vp, dp, dp, C.c_int64], C.c_int),
        "gm_status": ([vp, C.c_int], C.c_int),
        "gm_strerror": ([C.c_int], C.c_char_p),
        "gm_neighbor_stats": ([vp, ip32, ip64, ip64], C.c_int),
        "gm_reserve_neighbors": ([vp, C.c_int32], C.c_int),
        "gm_release_rows": ([vp], C.c_int),
        "gm_hills_set_device": ([vp, vp, vp, C.c_int64], C.c_int),
        "gm_status_copy": ([vp, vp], C.c_int),
        "gm_status_decode": ([C.c_int32], C.c_int),
        "gm_device_bytes": ([vp, vp], C.c_int),
        "gm_copy_cell_list": ([vp, vp, vp, ip32], C.c_int),
        "gm_copy_neighbors": ([vp, vp, vp, ip32], C.c_int),
        "gm_atom_values": ([vp, C.c_int, vp], C.c_int),
        "gm_version": ([], C.c_char_p),
        "gm_batch_create": ([C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p),
                             C.POINTER(C.c_void_p), vp], C.c_int),
        "gm_batch_destroy": ([vp], C.c_int),
        "gm_batch_update": ([vp, C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)],
                            C.c_int),
        "gm_batch_build": ([vp, dp], C.c_int),
        "gm_batch_build_some": ([vp, C.POINTER(C.c_int32), C.c_int32, dp, vp], C.c_int),
        "gm_batch_step": ([vp], C.c_int),
        "gm_batch_deposit": ([vp], C.c_int),
        "gm_batch_deposit_some": ([vp, C.POINTER(C.c_int32), C.c_int32], C.c_int),
        "gm_batch_values": ([vp, vp, vp, vp], C.c_int),
        "gm_torsions": ([vp, C.c_int64, vp, C.c_int32, dp, vp, vp], C.c_int),
        "gm_torsion_forces": ([vp, C.c_int64, vp, C.c_int32, dp, vp, vp, C.c_int32, vp], C.c_int),
        "gm_nearest_distance": ([vp, C.c_int64, C.c_int32, vp, C.c_int32, dp, vp, vp, vp], C.c_int),
        "gm_nearest_distance_forces": ([vp, C.c_int64, C.c_int32, vp, C.c_int32, dp, vp, vp, C.c_int32, vp],
                                       C.c_int),
        "gm_lattice_virial": ([dp, dp, C.c_int32, dp], C.c_int),
        "gm_fes_reweight": ([vp, vp, C.c_int64, C.c_int32, dp, dp, ip32, C.c_double, vp, vp], C.c_int),
        "gm_fes_reweight_noalloc": ([vp, vp, C.c_int64, C.c_int32, dp, dp, ip32, C.c_double, vp, vp], C.c_int),
        "gm_fes_hills": ([vp, dp, dp, ip32, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib: Optional[C.CDLL] = _load()


def lib() -> C.CDLL:
    return _lib


def _check(rc: int, call: str):
    if rc != GM_OK:
        raise GmError(rc, call)


def _ptr(t, numel: Optional[int] = None, dtype=None, name: str = "tensor") -> Optional[int]:
    """Device pointer of a contiguous tensor, after checking its size and type."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device (CUDA/HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: expected at least {numel} elements, got {t.numel()}")
    return t.data_ptr()


@dataclass
class Params:
    """Mirror of gm_params (see include/gpumetad.h)."""
    cv_kind: int = CV_Q6COUNT
    precision: int = FP32
    r_c: float = 3.6
    skin: float = 0.4
    taper: float = 0.2
    cn_r0: float = 2.5
    bond_d0: float = 0.7
    bond_w: float = 0.02
    count_n0: float = 5.5
    count_w: float = 0.25
    sigma: Sequence[float] = field(default_factory=lambda: [20.0])
    w0: float = 1.2
    gamma: float = 10.0
    kBT: float = 2.494
    hill_capacity: int = 100000
    max_neighbors: int = 64
    brick: Sequence[int] = (0, 0, 0)  # cells per brick and axis; 0 = chosen per build
    lds_kb: int = 0                   # LDS staging budget per workgroup; 0 = auto
    period: Sequence[float] = (0.0, 0.0)  # per CV dimension; 0 = not periodic (2 pi for an angle)
    external_dims: int = 1            # CV dimensions of a CV_EXTERNAL context
    tpa: int = 0                      # lanes per atom in the CV passes (1, 2, 4); 0 = chosen per build

    @property
    def dims(self) -> int:
        if self.cv_kind == CV_EXTERNAL:
            return int(self.external_dims)
        return 2 if self.cv_kind == CV_COORD_Q6 else 1

    def to_c(self) -> GmParams:
        sig = list(self.sigma) + [0.0] * (2 - len(self.sigma))
        per = list(self.period) + [0.0] * (2 - len(self.period))
        return GmParams(self.cv_kind, self.precision, self.r_c, self.skin, self.taper, self.cn_r0,
                        self.bond_d0, self.bond_w, self.count_n0, self.count_w, (C.c_double * 2)(*sig[:2]),
                        self.w0, self.gamma, self.kBT, self.hill_capacity, self.max_neighbors,
                        (C.c_int32 * 3)(*[int(b) for b in self.brick]), int(self.lds_kb),
                        (C.c_double * 2)(*[float(x) for x in per[:2]]), int(self.external_dims), int(self.tpa))


class Pipeline:
    """One gm_ctx: a system of n atoms, its lists, CV state and hill history."""

    def __init__(self, n_atoms: int, params: Params, stream=None):
        import torch

        self.torch = torch
        self.params = params
        self.n = int(n_atoms)
        self.dims = params.dims
        self.fdtype = torch.float64 if params.precision == FP64 else torch.float32
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._cp = params.to_c()
        h = C.c_void_p()
        _check(_lib.gm_create(C.byref(h), C.byref(self._cp), self.n, C.c_void_p(self.stream.cuda_stream)),
               "gm_create")
        self.h = h
        dev = torch.device("cuda", torch.cuda.current_device())
        self.s = torch.zeros(self.dims, dtype=torch.float64, device=dev)
        self.V = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dVds = torch.zeros(self.dims, dtype=torch.float64, device=dev)
        self.generation = 0  # number of cv_forward calls (autograd checks it)
        self._begin()  # the context stream must see the zero-filled buffers

    def close(self):
        if getattr(self, "h", None):
            _lib.gm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        _check(_lib.gm_set_stream(self.h, C.c_void_p(stream.cuda_stream)), "gm_set_stream")

    # ---- the six pipeline calls --------------------------------------------
    def _pos(self, pos4):
        return _ptr(pos4, 4 * self.n, self.torch.float32, "pos4")

    def _vec(self, t, name):
        return _ptr(t, self.dims, self.torch.float64, name)

    def _arr4(self, t, name):
        return _ptr(t, 4 * self.n, self.fdtype, name)

    def build_neighbors(self, pos4, box):
        box_c = (C.c_double * 3)(*[float(b) for b in box])
        _check(_lib.gm_build_neighbors(self.h, self._pos(pos4), box_c), "gm_build_neighbors")

    def cv_forward(self, pos4, s=None):
        s = self.s if s is None else s
        _check(_lib.gm_cv_forward(self.h, self._pos(pos4), self._vec(s, "s")), "gm_cv_forward")
        self.generation += 1
        return s

    def bias_eval(self, s=None, V=None, dVds=None):
        s = self.s if s is None else s
        V = self.V if V is None else V
        dVds = self.dVds if dVds is None else dVds
        _check(_lib.gm_bias_eval(self.h, self._vec(s, "s"), _ptr(V, 1, self.torch.float64, "V"),
                                 self._vec(dVds, "dVds")), "gm_bias_eval")
        return V, dVds

    def cv_backward(self, pos4, seed=None, grad4=None):
        _check(_lib.gm_cv_backward(self.h, self._pos(pos4), self._vec(seed, "seed"), self._arr4(grad4, "grad4")),
               "gm_cv_backward")
        return grad4

    def apply_bias_forces(self, pos4, force4, dVds=None):
        dVds = self.dVds if dVds is None else dVds
        _check(_lib.gm_apply_bias_forces(self.h, self._pos(pos4), self._vec(dVds, "dVds"),
                                         self._arr4(force4, "force4")), "gm_apply_bias_forces")
        return force4

    def deposit_hill(self, s=None):
        """Deposit at s (device double[dims]); None = at the last forward's CV."""
        _check(_lib.gm_deposit_hill(self.h, self._vec(s, "s") if s is not None else None), "gm_deposit_hill")

    # ---- one MD step's bias pipeline ---------------------------------------
    def step(self, pos4, force4):
        self.cv_forward(pos4)
        self.bias_eval()
        self.cv_backward(pos4)
        self.apply_bias_forces(pos4, force4)

    # ---- state, checkpoint, inspection -------------------------------------
    def status(self, sync: bool = True) -> int:
        return _lib.gm_status(self.h, 1 if sync else 0)

    def check(self):
        _check(self.status(True), "gm_status")

    def hills_get(self):
        import numpy as np

        k = C.c_int64()
        _check(_lib.gm_hills_get(self.h, None, None, 0, C.byref(k)), "gm_hills_get")
        K = k.value
        cen = np.zeros((max(K, 1), self.dims))
        hts = np.zeros(max(K, 1))
        _check(_lib.gm_hills_get(self.h, cen.ctypes.data_as(C.POINTER(C.c_double)),
                                 hts.ctypes.data_as(C.POINTER(C.c_double)), max(K, 1), C.byref(k)), "gm_hills_get")
        return cen[:K], hts[:K]

    def fes_hills(self, lo, hi, nbins, F=None):
        """F = -V (or -gamma/(gamma-1) V) on the grid of bin centres, bin id i0 + nb0 i1."""
        lo, hi, nb = _grid(lo, hi, nbins, self.dims)
        total = 1
        for x in nb:
            total *= x
        F = self.torch.empty(total, dtype=self.torch.float64, device=self.s.device) if F is None else F
        _check(_lib.gm_fes_hills(self.h, lo, hi, nb, _ptr(F, total, self.torch.float64, "F")), "gm_fes_hills")
        return F

    def hills_set(self, centres, heights):
        import numpy as np

        cen = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, self.dims)
        hts = np.ascontiguousarray(heights, dtype=np.float64)
        _check(_lib.gm_hills_set(self.h, cen.ctypes.data_as(C.POINTER(C.c_double)),
                                 hts.ctypes.data_as(C.POINTER(C.c_double)), hts.shape[0]), "gm_hills_set")

    def neighbor_stats(self, cutoff_pairs: bool = False):
        """(max row length, total list entries[, ordered pairs inside r_c])."""
        m = C.c_int32()
        t = C.c_int64()
        cp = C.c_int64()
        _check(_lib.gm_neighbor_stats(self.h, C.byref(m), C.byref(t), C.byref(cp) if cutoff_pairs else None),
               "gm_neighbor_stats")
        return (m.value, t.value, cp.value) if cutoff_pairs else (m.value, t.value)

    def hills_set_device(self, centres, heights):
        """Hill history from device tensors (double [k, dims] and [k]), enqueued
        without waiting; the tensors must stay alive until the stream has run it."""
        k = int(heights.shape[0])
        _check(_lib.gm_hills_set_device(self.h, _ptr(centres, k * self.dims, self.torch.float64, "centres"),
                                        _ptr(heights, k, self.torch.float64, "heights"), k), "gm_hills_set_device")

    def status_copy(self, dst):
        """Enqueue a copy of the sticky error word into dst (int32 tensor of one
        element, device or pinned host); decode it with status_decode once the
        stream has passed this point."""
        if dst.dtype != self.torch.int32 or dst.numel() < 1:
            raise ValueError("dst must hold one int32")
        _check(_lib.gm_status_copy(self.h, C.c_void_p(dst.data_ptr())), "gm_status_copy")

    @staticmethod
    def status_decode(word: int) -> int:
        return _lib.gm_status_decode(int(word))

    def release_rows(self):
        """Give the per-atom q6 rows back to the pool until the next forward."""
        _check(_lib.gm_release_rows(self.h), "gm_release_rows")

    def device_bytes(self) -> int:
        """Bytes of device memory the context holds now."""
        b = C.c_int64()
        _check(_lib.gm_device_bytes(self.h, C.byref(b)), "gm_device_bytes")
        return int(b.value)

    def reserve_neighbors(self, kmax: int):
        _check(_lib.gm_reserve_neighbors(self.h, int(kmax)), "gm_reserve_neighbors")

    def build_neighbors_checked(self, pos4, box):
        """Build; on a neighbour-list overflow grow the rows and rebuild (synchronises)."""
        self.build_neighbors(pos4, box)
        rc = self.status(True)
        if rc == -5:
            m, _ = self.neighbor_stats()
            self.reserve_neighbors(m + 8)
            self.build_neighbors(pos4, box)
            rc = self.status(True)
        _check(rc, "gm_build_neighbors")

    def _begin(self):
        """Order the context stream after the caller's stream (for tensors the
        binding allocates on the caller's stream and the library writes)."""
        cur = self.torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _end(self, *tensors):
        """Make the caller's stream wait for the library's writes."""
        cur = self.torch.cuda.current_stream()
        if cur != self.stream:
            cur.wait_stream(self.stream)
            for t in tensors:
                t.record_stream(self.stream)

    def cell_list(self):
        torch = self.torch
        perm = torch.empty(self.n, dtype=torch.int32, device=self.s.device)
        nc = (C.c_int32 * 3)()
        _check(_lib.gm_copy_cell_list(self.h, _ptr(perm), None, nc), "gm_copy_cell_list")
        ncells = nc[0] * nc[1] * nc[2]
        start = torch.empty(ncells + 1, dtype=torch.int32, device=self.s.device)
        self._begin()
        _check(_lib.gm_copy_cell_list(self.h, _ptr(perm), _ptr(start), nc), "gm_copy_cell_list")
        self._end(perm, start)
        return (nc[0], nc[1], nc[2]), perm, start

    def neighbor_lists(self):
        torch = self.torch
        w = C.c_int32()
        _check(_lib.gm_copy_neighbors(self.h, None, None, C.byref(w)), "gm_copy_neighbors")
        nbr = torch.empty((self.n, w.value), dtype=torch.int32, device=self.s.device)
        cnt = torch.empty(self.n, dtype=torch.int32, device=self.s.device)
        self._begin()
        _check(_lib.gm_copy_neighbors(self.h, _ptr(nbr), _ptr(cnt), C.byref(w)), "gm_copy_neighbors")
        self._end(nbr, cnt)
        return nbr, cnt

    def atom_values(self, what: int):
        out = self.torch.empty(self.n, dtype=self.torch.float64, device=self.s.device)
        self._begin()
        _check(_lib.gm_atom_values(self.h, int(what), _ptr(out, self.n, self.torch.float64, "out")),
               "gm_atom_values")
        self._end(out)
        return out


class Batch:
    """Many walkers (Pipelines) stepped together: one launch per pass for all
    walkers of a CV kind (gm_batch_*).  pos4[w] / force4[w] are the walkers'
    resident device arrays; they must outlive the batch."""

    def __init__(self, pipes, pos4, force4, stream=None):
        import torch

        self.torch = torch
        pipes, pos4, force4 = self._members(pipes, pos4, force4)
        if not pipes:
            raise ValueError("a batch starts with at least one walker")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        w, hs, xs, fs = self._tables(pipes, pos4, force4)
        h = C.c_void_p()
        _check(_lib.gm_batch_create(C.byref(h), hs, w, xs, fs, C.c_void_p(self.stream.cuda_stream)), "gm_batch_create")
        self.h = h
        self._adopt(pipes, pos4, force4)
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)

    @staticmethod
    def _members(pipes, pos4, force4):
        pipes, pos4, force4 = list(pipes), list(pos4), list(force4)
        if not (len(pos4) == len(force4) == len(pipes)):
            raise ValueError("one position and one force array per walker")
        for p, x, f in zip(pipes, pos4, force4):
            p._pos(x)
            p._arr4(f, "force4")
        return pipes, pos4, force4

    @staticmethod
    def _tables(pipes, pos4, force4):
        w = len(pipes)
        hs = (C.c_void_p * max(w, 1))(*[p.h.value for p in pipes])
        xs = (C.c_void_p * max(w, 1))(*[x.data_ptr() for x in pos4])
        fs = (C.c_void_p * max(w, 1))(*[f.data_ptr() for f in force4])
        return w, hs, xs, fs

    def _adopt(self, pipes, pos4, force4):
        torch = self.torch
        self.pipes, self.pos4, self.force4 = pipes, pos4, force4
        for p in pipes:
            p.stream = self.stream
        w = len(pipes)
        if getattr(self, "s", None) is None or self.s.shape[0] != w:
            dev = pos4[0].device if pos4 else self.s.device
            self.s = torch.zeros((w, 2), dtype=torch.float64, device=dev)
            self.V = torch.zeros(w, dtype=torch.float64, device=dev)
            self.dVds = torch.zeros((w, 2), dtype=torch.float64, device=dev)

    def update(self, pipes, pos4, force4):
        """Replace the members (gm_batch_update): the device tables and the
        entries of walkers that stay are kept.  Remove a walker this way
        before closing its Pipeline."""
        pipes, pos4, force4 = self._members(pipes, pos4, force4)
        w, hs, xs, fs = self._tables(pipes, pos4, force4)
        _check(_lib.gm_batch_update(self.h, hs, w, xs, fs), "gm_batch_update")
        self._adopt(pipes, pos4, force4)

    def close(self):
        if getattr(self, "h", None):
            _lib.gm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, boxes):
        import numpy as np

        b = np.ascontiguousarray(boxes, dtype=np.float64).reshape(len(self.pipes), 3)
        _check(_lib.gm_batch_build(self.h, b.ctypes.data_as(C.POINTER(C.c_double))), "gm_batch_build")

    def build_some(self, which, boxes, stream=None):
        """Rebuild the lists of the member indices in `which` (boxes: one row
        per listed walker), batched where the walkers allow; on `stream`
        (default: the batch stream), ordered by the caller."""
        import numpy as np

        if not len(which):
            return
        b = np.ascontiguousarray(boxes, dtype=np.float64).reshape(len(which), 3)
        idx = (C.c_int32 * len(which))(*[int(i) for i in which])
        st = C.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(_lib.gm_batch_build_some(self.h, idx, len(which), b.ctypes.data_as(C.POINTER(C.c_double)), st),
               "gm_batch_build_some")

    def step(self):
        _check(_lib.gm_batch_step(self.h), "gm_batch_step")
        for p in self.pipes:
            p.generation += 1

    def deposit(self, which=None):
        """One hill per walker, or only for the member indices in `which`."""
        if which is None:
            _check(_lib.gm_batch_deposit(self.h), "gm_batch_deposit")
            return
        idx = (C.c_int32 * max(len(which), 1))(*[int(i) for i in which])
        _check(_lib.gm_batch_deposit_some(self.h, idx, len(which)), "gm_batch_deposit_some")

    def values(self):
        """(s[W, 2], V[W]) device tensors, enqueued on the batch stream."""
        _check(_lib.gm_batch_values(self.h, self.s.data_ptr(), self.V.data_ptr(), None), "gm_batch_values")
        return self.s, self.V

    def gradients(self):
        """dV/ds[W, 2] of every walker's last step (device tensor, enqueued on the batch stream)."""
        _check(_lib.gm_batch_values(self.h, None, None, self.dVds.data_ptr()), "gm_batch_values")
        return self.dVds


def version() -> str:
    return _lib.gm_version().decode()


# ---- CVs of a few atoms, lattice parameters, free energy ---------------------
def _grid(lo, hi, nbins, dims):
    lo = [float(x) for x in (lo if hasattr(lo, "__len__") else [lo])]
    hi = [float(x) for x in (hi if hasattr(hi, "__len__") else [hi])]
    nb = [int(x) for x in (nbins if hasattr(nbins, "__len__") else [nbins])]
    if not (len(lo) == len(hi) == len(nb) == dims):
        raise ValueError(f"expected {dims} grid dimensions")
    return (C.c_double * dims)(*lo), (C.c_double * dims)(*hi), (C.c_int32 * dims)(*nb)


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _box(box):
    return (C.c_double * 3)(*[float(b) for b in box])


def _force(force4, n):
    import torch

    if force4.dtype not in (torch.float32, torch.float64):
        raise ValueError("force4: expected float32 or float64")
    return _ptr(force4, 4 * n, None, "force4"), (FP64 if force4.dtype == torch.float64 else FP32)


def torsions(pos4, quads, box, phi=None, stream=None):
    """Torsion angles (IUPAC sign) of the atom quadruples quads (dev int32 [m][4])."""
    import torch

    n, m = pos4.shape[0], quads.shape[0]
    phi = torch.empty(m, dtype=torch.float64, device=pos4.device) if phi is None else phi
    _check(_lib.gm_torsions(_ptr(pos4, 4 * n, torch.float32, "pos4"), n, _ptr(quads, 4 * m, torch.int32, "quads"),
                            m, _box(box), _ptr(phi, m, torch.float64, "phi"), _stream(stream)), "gm_torsions")
    return phi


def torsion_forces(pos4, quads, box, dVdphi, force4, stream=None):
    """force4 -= sum_t dV/dphi_t dphi_t/dx (in place)."""
    import torch

    n, m = pos4.shape[0], quads.shape[0]
    fp, prec = _force(force4, n)
    _check(_lib.gm_torsion_forces(_ptr(pos4, 4 * n, torch.float32, "pos4"), n,
                                  _ptr(quads, 4 * m, torch.int32, "quads"), m, _box(box),
                                  _ptr(dVdphi, m, torch.float64, "dVdphi"), fp, prec, _stream(stream)),
           "gm_torsion_forces")
    return force4


def nearest_distance(pos4, centre, members, box, s=None, nearest=None, stream=None):
    """Distance from atom centre to the nearest atom of members (dev int32 [k])."""
    import torch

    n, k = pos4.shape[0], members.shape[0]
    s = torch.empty(1, dtype=torch.float64, device=pos4.device) if s is None else s
    _check(_lib.gm_nearest_distance(_ptr(pos4, 4 * n, torch.float32, "pos4"), n, int(centre),
                                    _ptr(members, k, torch.int32, "members"), k, _box(box),
                                    _ptr(s, 1, torch.float64, "s"), _ptr(nearest, 1, torch.int32, "nearest"),
                                    _stream(stream)), "gm_nearest_distance")
    return s


def nearest_distance_forces(pos4, centre, members, box, dVds, force4, stream=None):
    import torch

    n, k = pos4.shape[0], members.shape[0]
    fp, prec = _force(force4, n)
    _check(_lib.gm_nearest_distance_forces(_ptr(pos4, 4 * n, torch.float32, "pos4"), n, int(centre),
                                           _ptr(members, k, torch.int32, "members"), k, _box(box),
                                           _ptr(dVds, 1, torch.float64, "dVds"), fp, prec, _stream(stream)),
           "gm_nearest_distance_forces")
    return force4


def lattice_virial(box, dVdL):
    """W_aa = -L_a dV/dL_a for lattice-parameter CVs (host values)."""
    d = len(dVdL)
    out = (C.c_double * d)()
    _check(_lib.gm_lattice_virial((C.c_double * 3)(*[float(b) for b in box]),
                                  (C.c_double * d)(*[float(x) for x in dVdL]), d, out), "gm_lattice_virial")
    return list(out)


def fes_reweight(s, V, lo, hi, nbins, kBT, F=None, stream=None):
    """F per bin from samples s (dev double [T] or [T][dims]) and their bias V (dev double [T])."""
    import torch

    T = V.shape[0]
    dims = 1 if s.dim() == 1 else s.shape[1]
    lo_c, hi_c, nb_c = _grid(lo, hi, nbins, dims)
    total = 1
    for i in range(dims):
        total *= nb_c[i]
    F = torch.empty(total, dtype=torch.float64, device=V.device) if F is None else F
    _check(_lib.gm_fes_reweight(_ptr(s, T * dims, torch.float64, "s"), _ptr(V, T, torch.float64, "V"), T, dims,
                                lo_c, hi_c, nb_c, float(kBT), _ptr(F, total, torch.float64, "F"), _stream(stream)),
           "gm_fes_reweight")
    return F


def fes_reweight_noalloc(s, V, lo, hi, nbins, kBT, F, stream=None):
    """fes_reweight into the caller's F (dev double [prod nbins]) with no device
    allocation (the library's fixed scratch; at most 65536 bins)."""
    import torch

    T = V.shape[0]
    dims = 1 if s.dim() == 1 else s.shape[1]
    lo_c, hi_c, nb_c = _grid(lo, hi, nbins, dims)
    total = 1
    for i in range(dims):
        total *= nb_c[i]
    _check(_lib.gm_fes_reweight_noalloc(_ptr(s, T * dims, torch.float64, "s"), _ptr(V, T, torch.float64, "V"), T,
                                        dims, lo_c, hi_c, nb_c, float(kBT), _ptr(F, total, torch.float64, "F"),
                                        _stream(stream)),
           "gm_fes_reweight_noalloc")
    return F
