"""Continuous batching of bias-force requests from many independent walkers.

A request is one walker (its own atoms, box, CV kind and resident hill
history) that needs ``steps`` MD steps of the bias pipeline, with a neighbour
rebuild and a hill deposit every ``pace`` steps of its own.  The server keeps
each admitted walker's lists and hills on the device, admits new requests at
tick boundaries while a slot and HBM budget are free, and advances every
active walker by one step per tick with one launch per pass for all of them
(one ``Batch`` for the whole run, whose members change in place); the walkers
due for a neighbour rebuild or a hill deposit at a tick get them in one
launch per stage as well.  Finished walkers free their slot and memory for
the queue.

Nothing in the loop waits for the device while walkers run.  A request's
arrays are page-locked before the run (the server receives them into pinned
host buffers), so an admission is a chain of enqueued work on an admission
stream: context creation, the position, force and hill uploads and the first
neighbour build, closed by an event.  The walker joins the batch at once; the
batch stream waits for that event only (not for later admissions), so no
host thread waits for the admission either.  A finished walker's CV, bias,
forces and (sticky) error word are copied to pinned memory behind an event
that the loop polls, and its buffers go back to the library's stream-ordered
pool in stream order.  The error word is checked only then: a walker whose
neighbour rows overflowed (the row width carries a margin, so this is rare)
has its result discarded and its request queued again with rows twice as
wide.

Walkers are prepared ahead: while a tick's step runs on the device, the loop
admits queued requests (within the HBM budget, which counts them) into a
staging list, so that when a group of walkers finishes together the next ones
join at once instead of being created one by one while the device idles.

``serve_sequential`` runs the same requests one after another with the
per-walker calls, the baseline the batched loop is measured against.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .binding import Batch, Params, Pipeline


@dataclass
class Request:
    rid: int
    arrival: float              # seconds after the start of the run
    pos: np.ndarray             # (N, 4) float32 positions
    box: np.ndarray             # (3,) float64
    params: Params
    centres: np.ndarray         # (K, dims) hill centres
    heights: np.ndarray         # (K,) hill heights
    forces: np.ndarray          # (N, 4) external forces (float32)
    steps: int = 100
    pace: int = 10
    pinned: Optional[dict] = None  # page-locked copies of the arrays (pin())

    @property
    def n(self) -> int:
        return self.pos.shape[0]

    def pin(self, torch):
        """Page-locked host copies of the request's arrays, so that its
        uploads are enqueued without a host wait."""
        if self.pinned is None:
            dims = self.params.dims
            self.pinned = {
                "pos": torch.from_numpy(np.ascontiguousarray(self.pos, np.float32)).pin_memory(),
                "forces": torch.from_numpy(np.ascontiguousarray(self.forces, np.float32)).pin_memory(),
                "centres": torch.from_numpy(np.ascontiguousarray(np.reshape(self.centres, (-1, dims)),
                                                                 np.float64)).pin_memory(),
                "heights": torch.from_numpy(np.ascontiguousarray(self.heights, np.float64)).pin_memory(),
            }
        return self.pinned


@dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    finished: float
    s: np.ndarray
    V: float
    forces: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def device_bytes(req: Request) -> int:
    """Device memory a walker holds while admitted (library buffers plus its
    resident positions and forces), from the sizes the library allocates."""
    p = req.params
    n = req.n
    t = 8 if p.precision == 1 else 4
    kmax = (max(p.max_neighbors, 4) + 3) // 4 * 4
    per_atom = 16 + 16 * t                      # caller positions + forces
    per_atom += 4 * 7 + 2 * 2 * kmax            # cell, perm, owned tables, counts, neighbour + cutoff rows
    per_atom += 4 * t + 2 * t                   # sorted positions, bond count, coordination
    if p.cv_kind != 1:
        per_atom += 16 * t * 2                  # q-hat and adjoint rows
    per_atom += 4 * 8                           # halo slot table (bounded by 8 halo copies per atom)
    hills = p.hill_capacity * (p.dims + 1) * 8
    return int(n * per_atom + hills + (1 << 20))


class _Walker:
    """An admitted request: its context, resident arrays and hill history,
    all enqueued on `stream` (the current stream while this runs), ending
    with the first neighbour build, a copy of the error word and `ready`."""

    def __init__(self, req: Request, dev, torch, stream):
        self.req = req
        h = req.pin(torch)
        self.pipe = Pipeline(req.n, req.params, stream=stream)
        self.pos = h["pos"].to(dev, non_blocking=True)
        self.F = h["forces"].to(device=dev, non_blocking=True)
        if self.pipe.fdtype != torch.float32:
            self.F = self.F.to(self.pipe.fdtype)
        self.cen = h["centres"].to(dev, non_blocking=True)
        self.hts = h["heights"].to(dev, non_blocking=True)
        self.pipe.hills_set_device(self.cen, self.hts)
        self.pipe.build_neighbors(self.pos, req.box)
        self.ready = torch.cuda.Event()
        self.ready.record(stream)
        self.err = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self.done = 0
        self.bytes = device_bytes(req)

    def close(self):
        self.pipe.close()


def _finish(w: _Walker, t: float, admitted: float, keep_forces: bool) -> Result:
    s = w.pipe.s.cpu().numpy().copy() if w.pipe.s is not None else None
    return Result(w.req.rid, w.req.n, w.req.arrival, admitted, t, s, float(w.pipe.V.item()),
                  w.F.cpu().numpy().copy() if keep_forces else None)


@dataclass
class _Retiring:
    """Walkers that finished at one tick: host copies of their results and
    error words land behind ``event`` on the batch stream."""
    event: object
    walkers: list
    s: object                   # pinned (W, 2) CVs of the whole batch at that tick
    V: object                   # pinned (W,) biases
    rows: list                  # row of each walker in s / V
    forces: list                # pinned force copies (keep_forces) or None


def tune_requests(requests: List[Request], cache: Optional[str] = None, steps: int = 5, limit: int = 6,
                  device=None) -> Tuple[List[Request], dict]:
    """The autotuner's brick shape and lanes per atom, chosen once per tuning
    class (CV kind, precision, cutoff, walker size class and atoms per cell
    rounded to an integer) on the largest request of the class and given to
    every request of the class.  The LDS budget stays the library's: a batched
    pass runs every walker of a CV kind with the largest staging any of them
    asks for, so a smaller budget for one walker would not take effect.
    Returns the tuned requests and the choice per class."""
    from dataclasses import replace

    import torch

    from .autotune import autotune, cells_per_axis, size_class

    def key_of(r):
        p = r.params
        rho = r.n / float(np.prod(cells_per_axis(r.box, p.r_c + p.skin)))
        return f"kind{p.cv_kind}-p{p.precision}-rc{p.r_c:g}-size{size_class(r.n)}-rho{round(rho)}"

    dev = device or torch.device("cuda", 0)
    largest = {}
    for r in requests:
        k = key_of(r)
        if k not in largest or r.n > largest[k].n:
            largest[k] = r
    chosen = {}
    for k, r in largest.items():
        pos4 = torch.from_numpy(np.ascontiguousarray(r.pos, np.float32)).to(dev)
        tuned, _ = autotune(pos4, r.box, r.params, steps=steps, cache=cache, limit=limit, lds_kb=(80,))
        chosen[k] = (tuple(tuned.brick), tuned.tpa)
    out = []
    for r in requests:
        b, tpa = chosen[key_of(r)]
        out.append(replace(r, params=replace(r.params, brick=b, tpa=tpa), pinned=None))
    return out, chosen


def _wider(req: Request) -> Request:
    """The same request with neighbour rows twice as wide."""
    from dataclasses import replace

    return replace(req, params=replace(req.params, max_neighbors=2 * max(int(req.params.max_neighbors), 4)))


def serve_batched(requests: List[Request], hbm_budget: int, max_slots: int = 64, keep_forces: bool = False,
                  device=None, stage_ahead: Optional[int] = None):
    """Run the requests with continuous batching; returns (results, stats).

    stage_ahead: most walkers prepared ahead of a free slot (default max_slots;
    0 admits only into free slots).  A request that would not fit the budget
    even alone is rejected before anything runs (it could never be admitted)."""
    for r in requests:
        if device_bytes(r) > hbm_budget:
            raise ValueError(f"request {r.rid} needs {device_bytes(r)} bytes of device memory, "
                             f"more than the whole budget of {hbm_budget}")
    import torch

    from .binding import GmError

    dev = device or torch.device("cuda", 0)
    for r in requests:
        r.pin(torch)
    stream = torch.cuda.Stream(device=dev)
    adm = torch.cuda.Stream(device=dev)
    pending = sorted(requests, key=lambda r: r.arrival)
    active: List[_Walker] = []
    staged: List[_Walker] = []
    stage_cap = max(max_slots if stage_ahead is None else int(stage_ahead), 1)
    retiring: List[_Retiring] = []
    admitted_at = {}
    results: List[Result] = []
    used = 0
    peak_used = 0
    ticks = 0
    batch = None
    members = None
    t0 = time.perf_counter()

    def retire(entry: _Retiring):
        nonlocal used
        entry.event.synchronize()  # completed already unless the loop is idle
        t = time.perf_counter() - t0
        for w, k, F in zip(entry.walkers, entry.rows, entry.forces):
            code = Pipeline.status_decode(int(w.err[0]))
            used -= w.bytes
            if code == -5:  # rows overflowed: run the request again with wider rows
                w.close()
                pending.insert(0, _wider(w.req))
                continue
            if code != 0:
                raise GmError(code, f"walker {w.req.rid}")
            results.append(Result(w.req.rid, w.req.n, w.req.arrival, admitted_at[w.req.rid], t,
                                  entry.s[k, :w.pipe.dims].numpy().copy(), float(entry.V[k]),
                                  F.numpy().copy() if F is not None else None))
            w.close()  # buffers back to the pool in order on the batch stream

    def can_prepare():
        return (pending and pending[0].arrival <= time.perf_counter() - t0
                and used + device_bytes(pending[0]) <= hbm_budget)

    def prepare():
        nonlocal used, peak_used
        req = pending.pop(0)
        with torch.cuda.stream(adm):
            w = _Walker(req, dev, torch, adm)
        w.pos.record_stream(stream)
        w.F.record_stream(stream)
        used += w.bytes
        peak_used = max(peak_used, used)
        return w

    with torch.cuda.stream(stream):
        while pending or active or retiring or staged:
            while retiring and retiring[0].event.query():
                retire(retiring.pop(0))
            # free slots take the staged walkers first, then fresh admissions;
            # the batch stream waits for each one's admission work
            while len(active) < max_slots and (staged or can_prepare()):
                w = staged.pop(0) if staged else prepare()
                stream.wait_event(w.ready)
                active.append(w)
                admitted_at[w.req.rid] = time.perf_counter() - t0
            if not active:
                if retiring:
                    retire(retiring.pop(0))
                elif pending:
                    time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            ids = tuple(w.req.rid for w in active)
            if ids != members:
                # one batch for the whole run: a change of members keeps its
                # device tables (no allocation or free per change)
                pipes, xs, fs = [w.pipe for w in active], [w.pos for w in active], [w.F for w in active]
                if batch is None:
                    batch = Batch(pipes, xs, fs, stream=stream)
                else:
                    batch.update(pipes, xs, fs)
                members = ids
            # rebuilds due at each walker's own step count, one launch per
            # stage of the rebuild for all of them
            due = [k for k, w in enumerate(active) if w.done > 0 and w.done % w.req.pace == 0]
            if due:
                batch.build_some(due, [active[k].req.box for k in due])
            batch.step()
            ticks += 1
            due = []
            for k, w in enumerate(active):
                w.done += 1
                if w.done % w.req.pace == 0:
                    due.append(k)
            if due:
                batch.deposit(due)  # one launch pair for the walkers due
            # prepare walkers for the next free slots while the step runs
            step_done = torch.cuda.Event()
            step_done.record(stream)
            made = 0
            while len(staged) < stage_cap and can_prepare() and (made == 0 or not step_done.query()):
                staged.append(prepare())
                made += 1
            finished = [w for w in active if w.done >= w.req.steps]
            if finished:
                s, V = batch.values()
                # pinned buffers of one size for every retirement, so that the
                # host allocator serves them from its cache
                s_h = torch.empty((max_slots, 2), dtype=s.dtype, pin_memory=True)
                V_h = torch.empty((max_slots,), dtype=V.dtype, pin_memory=True)
                s_h[:s.shape[0]].copy_(s, non_blocking=True)
                V_h[:V.shape[0]].copy_(V, non_blocking=True)
                forces = []
                for w in finished:
                    w.pipe.status_copy(w.err)
                    if keep_forces:
                        F_h = torch.empty(w.F.shape, dtype=w.F.dtype, pin_memory=True)
                        F_h.copy_(w.F, non_blocking=True)
                        forces.append(F_h)
                    else:
                        forces.append(None)
                ev = torch.cuda.Event()
                ev.record(stream)
                retiring.append(_Retiring(ev, finished, s_h, V_h, [members.index(w.req.rid) for w in finished],
                                          forces))
                active = [w for w in active if w.done < w.req.steps]
                # the finished walkers leave the batch before their contexts close
                batch.update([w.pipe for w in active], [w.pos for w in active], [w.F for w in active])
                members = tuple(w.req.rid for w in active)
        stream.synchronize()
        if batch is not None:
            batch.close()
    wall = time.perf_counter() - t0
    return results, _stats(results, wall, ticks=ticks, peak_bytes=peak_used)


def serve_sequential(requests: List[Request], keep_forces: bool = False, device=None):
    """Baseline: one walker at a time, per-walker launches, arrival order."""
    import torch

    dev = device or torch.device("cuda", 0)
    for r in requests:
        r.pin(torch)
    stream = torch.cuda.Stream(device=dev)
    results = []
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for req in sorted(requests, key=lambda r: r.arrival):
            now = time.perf_counter() - t0
            if req.arrival > now:
                time.sleep(req.arrival - now)
            admitted = time.perf_counter() - t0
            w = _Walker(req, dev, torch, stream)
            while w.pipe.status(True) == -5:  # the first build overflowed its rows
                w.close()
                w = _Walker(_wider(w.req), dev, torch, stream)
            w.pipe.check()
            for step in range(req.steps):
                if step > 0 and step % req.pace == 0:
                    w.pipe.build_neighbors(w.pos, req.box)
                w.pipe.step(w.pos, w.F)
                if (step + 1) % req.pace == 0:
                    w.pipe.deposit_hill()
            stream.synchronize()
            w.pipe.check()
            results.append(_finish(w, time.perf_counter() - t0, admitted, keep_forces))
            w.close()
    wall = time.perf_counter() - t0
    return results, _stats(results, wall)


def _stats(results: List[Result], wall: float, **extra) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    out = {
        "requests": len(results),
        "wall_s": wall,
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_ms": float(lat.mean()) if len(lat) else None,
        "atoms": int(sum(r.n for r in results)),
    }
    out.update(extra)
    return out


def summarize(results: List[Result], stats: dict, steps: int) -> dict:
    """Aggregate atom-steps/s over the makespan plus the latency percentiles."""
    total = sum(r.n for r in results) * steps
    d = dict(stats)
    d["atom_steps_per_s"] = total / stats["wall_s"] if stats["wall_s"] > 0 else None
    return d
