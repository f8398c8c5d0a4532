"""Throughput of the per-step metadynamics bias pipeline on one MI355X.

A bench step is one window of the hot path at 1,024,000 atoms (wurtzite
GaN-like slab, q6 crystalline-count CV, 50,000 deposited hills, external
forces N(0, 1 eV/A)):
    1 x build_neighbors
    10 x (cv_forward, bias_eval, cv_backward, apply_bias_forces)
    1 x deposit_hill
i.e. 10 MD steps = 10 N atom-steps.  Inputs are resident in HBM before the
timed region.  Inside it, HIP events bracket only the force calls (their
kernel is the roofline's); the time of every call comes from a few more
windows timed call by call afterwards.  Prints one JSON line.

The line also carries the walker-serving workload (256 requests of 1k-200k
atoms, continuous batching against sequential launches: p50/p99 latency and
aggregate atom-steps/s) and the oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--graph] [--no-cpu] [--no-serving]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

MD_STEPS_PER_WINDOW = 10
HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (packed FP32: two lanes' FMAs per
# instruction), and the ceiling without packed FP32, which this library's
# kernels are built without: 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 157.3
ALU_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# Algorithmic flops of k_pass4 per ordered pair inside r_c (FMA = 2): pair
# vector and r^2 8, 1/r and unit vector 5, g_i + g_j 13, E_m(z) 22, S and its
# gradient by the complex recurrence 144, tangential projection and
# accumulation 18.  The minimum image (bookkeeping, not arithmetic of the
# method) and the taper terms of the pairs in the last 0.2 A are not counted.
FLOPS_PER_PAIR_P4 = 210
# k_pass4's HBM traffic as measured by the FETCH_SIZE / WRITE_SIZE counters
# (scaled by a plain copy kernel of known size), with a digest of the kernel
# sources it was taken on: reported only while those sources are unchanged.
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "k_pass4_wz1m_hbm_traffic.txt")
KERNEL_SOURCES = ("gm_cv.hip", "gm_device.h", "gm_internal.h")
# k_pass4 per owned atom: slot/rank tables 8, cutoff count 4, position 16, adjoint
# row 64 (its last three lanes hold the taper term), permutation 4, force read +
# write 32
P4_BYTES_PER_ATOM = 128
# one MD step per atom: gather (perm 4, positions 16 read + 16 write), pass 1
# (positions 16, q-hat row write 64), pass 2 (q-hat row 64, c' 4, count 4),
# pass 3 (q-hat row 64, adjoint row write 64), pass 4 (as above), plus the
# per-step cutoff rows (2 B per pair, written once and read three times,
# counted as 8 B per pair) and the rebuild / 10
STEP_BYTES_PER_ATOM = 36 + 80 + 72 + 128 + 128


def model_bytes_per_atom_step(k_mean):
    """The algorithmic HBM bytes of one q6 atom-step in the layout-independent
    model: positions 16, force in + out 32, the neighbour list read once
    4 (K + 1), the 13-float q-hat and adjoint rows written and read
    (2 x 52 each), c' written and read (2 x 4), and the rebuild (positions 16,
    cell id and permutation 12, list write 4 (K + 1)) over 10 steps; K is the
    mean list length.  About 380 B at K = 24.5."""
    nl = 4.0 * (k_mean + 1.0)
    return 16 + 32 + nl + 2 * 52 + 2 * 4 + 2 * 52 + (16 + 12 + nl) / MD_STEPS_PER_WINDOW


def kernel_digest():
    import hashlib

    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2510_06873_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(root, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """Bytes per k_pass4 launch from the committed counter summary, or None if
    it is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if line.startswith(("sources_digest:", "bytes_per_launch:")))
    except OSError:
        return None
    if kv.get("sources_digest", "").strip() != kernel_digest():
        return None
    return int(kv["bytes_per_launch"].strip())


def copy_probe(mib):
    """A plain device copy of known size (the calibration run for the HBM
    byte counters): 5 launches of dst.copy_(src) over `mib` MiB."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="wz1m")
    ap.add_argument("--graph", action="store_true", help="replay each window as a captured HIP graph")
    ap.add_argument("--no-graph-too", dest="graph_too", action="store_false",
                    help="skip the graph-replayed windows timed after the eager ones")
    ap.add_argument("--call-windows", type=int, default=5,
                    help="windows after the timed region with an event pair around every call (per_call_us)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving workload")
    ap.add_argument("--autograd", action="store_true",
                    help="only time the autograd wrappers (stored vs recompute) on the 262,144-atom 2-D CV")
    ap.add_argument("--fes", action="store_true", help="only time the free energy from hills on a grid")
    ap.add_argument("--autotune", action="store_true",
                    help="time candidate brick shapes / LDS budgets on this system first and use the fastest")
    ap.add_argument("--brick", default=None, help="force the brick shape, e.g. 3x3x4")
    ap.add_argument("--lds-kb", type=int, default=0, help="LDS staging budget per workgroup (KiB)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--no-serving", action="store_true", help="skip the walker-serving block of the default line")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help=argparse.SUPPRESS)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup(wl_name, args=None):
    import torch

    import workloads as W
    from paper_2510_06873_amd import FP32, FP64, Params, Pipeline

    wl = W.WORKLOADS[wl_name]
    d = W.structure(wl["structure"])
    n = d["pos"].shape[0]
    kind = {"coord": 1, "q6": 2, "coord_q6": 3}[wl["cv"]]
    prm = Params(cv_kind=kind, precision=FP64 if wl["precision"] == "fp64" else FP32, r_c=wl["r_c"],
                 skin=wl["skin"], taper=wl.get("taper") or 0.2, cn_r0=wl["cn_r0"], bond_d0=wl.get("bond_d0", 0.7),
                 bond_w=wl.get("bond_w", 0.02), count_n0=wl.get("count_n0", 5.5), count_w=wl.get("count_w", 0.25),
                 sigma=wl["sigma"], w0=wl["w0"], gamma=wl["gamma"], kBT=wl["kBT"],
                 hill_capacity=wl["hills"]["k"] + 1024, max_neighbors=48)
    if args is not None and args.brick:
        prm.brick = tuple(int(x) for x in args.brick.split("x"))
    if args is not None and args.lds_kb:
        prm.lds_kb = args.lds_kb
    tuned = None
    if args is not None and args.autotune:
        from paper_2510_06873_amd.autotune import autotune

        p4 = torch.from_numpy(W.as_float4(d["pos"], d["species"])).to(torch.device("cuda", 0))
        prm, timings = autotune(p4, d["box"], prm, steps=3, limit=16)
        tuned = {"brick": list(prm.brick), "lds_kb": prm.lds_kb, "tpa": prm.tpa, "ms_per_md_step": timings}
        log(f"[bench] autotune: {tuned}")
    stream = torch.cuda.Stream()
    dev = torch.device("cuda", 0)
    with torch.cuda.stream(stream):
        pipe = Pipeline(n, prm, stream=stream)
        pos4 = torch.from_numpy(W.as_float4(d["pos"], d["species"])).to(dev)
        F_in = torch.from_numpy(W.external_forces(n, seed=wl.get("force_seed", 4))).to(dev)
        if prm.precision == FP64:
            F_in = F_in.double()
        F = F_in.clone()
        pipe.build_neighbors_checked(pos4, d["box"])
        hp = wl["hills"]
        if "lo" in hp:
            cen = W.hill_centres(hp["k"], hp["lo"], hp["hi"], hp["seed"])
        else:
            s0 = pipe.cv_forward(pos4).cpu().numpy()
            sig = np.array(wl["sigma"])
            cen = W.hill_centres(hp["k"], s0 - hp["centre_rel"] * sig, s0 + hp["centre_rel"] * sig, hp["seed"])
        cdev = torch.from_numpy(cen).to(dev)
        t = time.time()
        for k in range(cen.shape[0]):
            pipe.deposit_hill(cdev[k])
        stream.synchronize()
        log(f"[bench] {wl_name}: N={n}, hills deposited: {cen.shape[0]} in {time.time() - t:.1f}s")
        pipe.check()
    return dict(wl=wl, d=d, n=n, pipe=pipe, pos4=pos4, F=F, stream=stream, cen=cen, box=d["box"], tuned=tuned)


CALLS_PER_WINDOW = 2 + 4 * MD_STEPS_PER_WINDOW


def event_pool(count):
    """Timing events created ahead of the timed region (creating an event
    costs host time that would otherwise sit between the launches)."""
    import torch

    return [torch.cuda.Event(enable_timing=True) for _ in range(count)]


def window(S, ev=None, pool=None, only=None):
    """One window; ev collects (name, start, end) event pairs around the calls
    (only those named in `only`, when given), taken from pool (a list,
    consumed from the end) when given."""
    import torch

    pipe, pos4, F, box = S["pipe"], S["pos4"], S["F"], S["box"]

    def timed(name, fn, *a):
        if ev is None or (only is not None and name not in only):
            fn(*a)
            return
        if pool:
            e0, e1 = pool.pop(), pool.pop()
        else:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
        e0.record(S["stream"])
        fn(*a)
        e1.record(S["stream"])
        ev.append((name, e0, e1))

    timed("build_neighbors", pipe.build_neighbors, pos4, box)
    for _ in range(MD_STEPS_PER_WINDOW):
        timed("cv_forward", pipe.cv_forward, pos4)
        timed("bias_eval", pipe.bias_eval)
        timed("cv_backward", pipe.cv_backward, pos4)
        timed("apply_bias_forces", pipe.apply_bias_forces, pos4, F)
    timed("deposit_hill", pipe.deposit_hill)


def cpu_leg(wl_name, seconds):
    """One process of the CPU baseline: the oracle as it stands (plain C,
    single threaded, FP64) on a workload's full input (all its hills):
    repeated MD steps of the bias pipeline (a neighbour build amortised over
    10 steps, q6 forward, bias, q6 gradient and forces) for about `seconds`,
    at least one.  Runs in a child process of its own, with no GPU."""
    import oracle as orc
    import workloads as W

    wl = W.WORKLOADS[wl_name]
    d = W.structure(wl["structure"])
    pos, box = d["pos"], d["box"]
    n = pos.shape[0]
    prm = orc.q6_params(wl["r_c"], wl["taper"], wl["bond_d0"], wl["bond_w"], wl["count_n0"], wl["count_w"])
    hp = wl["hills"]
    cen = W.hill_centres(hp["k"], hp["lo"], hp["hi"], hp["seed"])
    hts = np.full(cen.shape[0], wl["w0"])
    F_in = W.external_forces(n, seed=wl.get("force_seed", 4))
    t_nl = t_step = 0.0
    reps = 0
    t_all = time.time()
    while reps < 1 or time.time() - t_all < seconds:
        t0 = time.time()
        nl = orc.neighbors(pos, box, wl["r_c"] + wl["skin"])
        t1 = time.time()
        s = orc.q6_forward(pos, box, nl, prm)["s"]
        _, dv = orc.bias(cen, hts, wl["sigma"], [s])
        g = orc.q6_gradient(pos, box, nl, prm)
        orc.bias_forces(F_in, [g], dv)
        t2 = time.time()
        t_nl += t1 - t0
        t_step += t2 - t1
        reps += 1
    per_step = (t_nl / MD_STEPS_PER_WINDOW + t_step) / reps
    return {"workload": wl_name, "atoms": n, "hills": int(cen.shape[0]), "reps": reps,
            "s_per_md_step": per_step, "atom_steps_per_s": n / per_step, "wall_s": time.time() - t_all}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def _run_legs(specs):
    """Run `bench.py --cpu-leg` children concurrently; their JSON results."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-leg", wl, "--cpu-seconds",
                               str(sec)], stdout=subprocess.PIPE, env=env) for wl, sec in specs]
    out = []
    for p in procs:
        stdout, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"CPU baseline leg exited with {p.returncode}")
        out.append(json.loads(stdout.decode().strip().splitlines()[-1]))
    return out


def cpu_baseline():
    """The oracle timed on the host cores, in child processes (no GPU): one
    thread on the 96,000-atom slab; one such process per core of this
    process's CPU share (at most 16), concurrently (the oracle is single
    threaded; independent processes on the same sample make the all-core
    figure); and one MD step at the full 1,024,000 atoms.  `value` is the
    all-core aggregate."""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    procs = max(1, min(16, cores))
    t = time.time()
    one = _run_legs([("wz96k", 8.0)])[0]
    many = _run_legs([("wz96k", 8.0)] * procs)
    full = _run_legs([("wz1m", 0.0)])[0]
    agg = sum(r["atom_steps_per_s"] for r in many)
    return {"value": agg, "unit": "atom-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"wz96k: 96000 atoms (the slab recipe of the 1,024,000-atom workload, all 10,000 hills): "
                      f"{procs} concurrent single-threaded processes x >= 8 s of MD steps (neighbour build / 10 + "
                      f"q6 forward + bias + q6 gradient + forces), FP64; total {time.time() - t:.1f} s with the legs "
                      f"below",
            "cpu_model": cpu_model(), "cpu_share": cores,
            "legs": {"one_thread_96k": round(one["atom_steps_per_s"], 1),
                     "all_cores_96k": round(agg, 1), "all_cores_processes": procs,
                     "one_thread_1m": round(full["atom_steps_per_s"], 1),
                     "one_thread_1m_s_per_md_step": round(full["s_per_md_step"], 2),
                     "one_thread_1m_hills": full["hills"]}}


def autograd_bench(steps=20, warmup=3):
    """The differentiation workload: 262,144 atoms, 2-D CV (coordination + q6
    count) on a 2-D Gaussian bias of 5,000 hills placed around the CV value.
    Times V(s(x)).backward() through the torch.autograd wrappers with the
    per-atom state stored by the forward or recomputed in the backward, next
    to the explicit calls (forward, bias, backward with the gradient out)."""
    import torch

    import workloads as W
    from paper_2510_06873_amd import CV_COORD_Q6, FP32, Params, Pipeline
    from paper_2510_06873_amd.autograd import bias_energy

    wl = W.WORKLOADS["wz262k"]
    d = W.structure(wl["structure"])
    n = d["pos"].shape[0]
    prm = Params(cv_kind=CV_COORD_Q6, precision=FP32, r_c=wl["r_c"], skin=wl["skin"], taper=wl["taper"],
                 cn_r0=wl["cn_r0"], bond_d0=wl["bond_d0"], bond_w=wl["bond_w"], count_n0=wl["count_n0"],
                 count_w=wl["count_w"], sigma=wl["sigma"], w0=wl["w0"], gamma=wl["gamma"], kBT=wl["kBT"],
                 hill_capacity=wl["hills"]["k"] + 16, max_neighbors=64)
    pipe = Pipeline(n, prm)
    dev = torch.device("cuda", 0)
    pos4 = torch.from_numpy(W.as_float4(d["pos"], d["species"])).to(dev)
    pipe.build_neighbors_checked(pos4, d["box"])
    s0 = pipe.cv_forward(pos4).cpu().numpy().copy()
    sig = np.array(wl["sigma"])
    cen = W.hill_centres(wl["hills"]["k"], s0 - 3 * sig, s0 + 3 * sig, seed=wl["hills"]["seed"])
    st = torch.empty(2, dtype=torch.float64, device=dev)
    for c in cen:
        st.copy_(torch.as_tensor(c))
        pipe.deposit_hill(st)
    pipe.check()
    x = pos4.clone().requires_grad_(True)
    grad4 = torch.zeros((n, 4), dtype=torch.float32, device=dev)

    def explicit():
        pipe.cv_forward(pos4)
        pipe.bias_eval()
        pipe.cv_backward(pos4, pipe.dVds, grad4)

    def through_autograd(mode):
        x.grad = None
        bias_energy(x, pipe, mode).backward()

    out = {"workload": f"wz262k: {n} atoms, 2-D CV (coordination, q6 count), {len(cen)} hills, FP32",
           "unit": "ms per forward + backward"}
    for name, fn in (("explicit", explicit), ("stored", lambda: through_autograd("stored")),
                     ("recompute", lambda: through_autograd("recompute"))):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        e1.synchronize()
        out[name + "_ms"] = round(e0.elapsed_time(e1) / steps, 4)
        # device memory the context holds between two calls
        out[name + "_context_bytes"] = pipe.device_bytes()
        log(f"[bench] autograd {name}: {out[name + '_ms']} ms, context holds {out[name + '_context_bytes']} B")
    pipe.check()
    return out


def fes_bench(steps=5, warmup=1):
    """The free energy from deposited hills on a grid (gm_fes_hills): 20,000
    hills of a 2-D periodic CV (torsion-like, sigma 0.35 rad) on a 256 x 256
    grid of bin centres."""
    import math

    import torch

    import workloads as W
    from paper_2510_06873_amd import CV_EXTERNAL, Params, Pipeline

    prm = Params(cv_kind=CV_EXTERNAL, external_dims=2, sigma=[0.35, 0.35], w0=1.2, gamma=10.0, kBT=W.KBT_KJMOL,
                 hill_capacity=20000, period=[2 * math.pi, 2 * math.pi])
    pipe = Pipeline(0, prm)
    cen = W.hill_centres(20000, [-math.pi, -math.pi], [math.pi, math.pi], seed=21)
    pipe.hills_set(cen, np.full(len(cen), 1.2))
    lo, hi, nb = [-math.pi, -math.pi], [math.pi, math.pi], [256, 256]
    F = torch.empty(nb[0] * nb[1], dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        pipe.fes_hills(lo, hi, nb, F)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pipe.fes_hills(lo, hi, nb, F)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"workload": "2-D periodic CV, 20000 hills, 256 x 256 grid", "ms_per_grid": round(ms, 3),
            "hill_evaluations_per_s": 20000 * nb[0] * nb[1] / (ms * 1e-3)}


def serving_requests(count=256, seed=7, n_hi=200000):
    """The serving workload as library requests."""
    import workloads as W
    from paper_2510_06873_amd import FP32, Params
    from paper_2510_06873_amd.serving import Request

    out = []
    for r in W.serving_requests(count=count, seed=seed, n_hi=n_hi):
        p = r["params"]
        kind = {"coord": 1, "q6": 2}[p["cv"]]
        prm = Params(cv_kind=kind, precision=FP32, r_c=p["r_c"], skin=p["skin"], taper=p["taper"], cn_r0=p["cn_r0"],
                     sigma=p["sigma"], w0=r["w0"], gamma=10.0, kBT=r["kBT"],
                     hill_capacity=r["centres"].shape[0] + 64, max_neighbors=p["kmax"])
        out.append(Request(r["rid"], r["arrival"], r["pos"], r["box"], prm, r["centres"], r["heights"], r["forces"]))
    return out


def serving(args):
    """p50/p99 request latency and aggregate atom-steps/s, batched vs sequential.

    The server first tunes brick shape and lanes per atom once per walker
    class (``tune_requests``, a start-up cost reported as ``tuning_s``); the
    batched and sequential runs use the tuned requests, and the batched run
    with the library's own choice is reported beside them."""
    from paper_2510_06873_amd.serving import serve_batched, serve_sequential, summarize, tune_requests

    reqs = serving_requests(count=args.serving_requests)
    warm = serving_requests(count=4, seed=99, n_hi=5000)
    serve_batched(warm, hbm_budget=64 << 30)
    serve_sequential(warm)
    t0 = time.perf_counter()
    tuned, chosen = tune_requests(reqs)
    tune_s = time.perf_counter() - t0
    log(f"[bench] serving: {len(reqs)} requests, {sum(r.n for r in reqs)} atoms, "
        f"{len(chosen)} tuning classes in {tune_s:.1f} s")
    # one untimed pass of the same requests: the measured runs see a warm
    # memory pool and warm clocks, as a long-running server would
    serve_batched(tuned, hbm_budget=64 << 30, max_slots=64)
    rb, sb = serve_batched(tuned, hbm_budget=64 << 30, max_slots=64)
    log(f"[bench] batched: {sb['wall_s']:.2f} s")
    rs, ss = serve_sequential(tuned)
    log(f"[bench] sequential: {ss['wall_s']:.2f} s")
    serve_batched(reqs, hbm_budget=64 << 30, max_slots=64)
    rd, sd = serve_batched(reqs, hbm_budget=64 << 30, max_slots=64)
    log(f"[bench] batched with the library's default geometry: {sd['wall_s']:.2f} s")
    steps = reqs[0].steps
    b = summarize(rb, sb, steps)
    q = summarize(rs, ss, steps)
    return {"requests": len(reqs), "steps_per_request": steps, "arrival_rate_per_s": 2000.0,
            "hbm_budget_gib": 64, "slots": 64, "tuning_classes": len(chosen), "tuning_s": round(tune_s, 2),
            "batched": b, "sequential": q, "batched_library_default": summarize(rd, sd, steps),
            "speedup_atom_steps": b["atom_steps_per_s"] / q["atom_steps_per_s"]}


def main():
    args = parse()
    if args.cpu_leg:
        print(json.dumps(cpu_leg(args.cpu_leg, args.cpu_seconds)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving(args)}), flush=True)
        return
    if args.autograd:
        print(json.dumps({"autograd": autograd_bench()}), flush=True)
        return
    if args.fes:
        print(json.dumps({"fes_hills": fes_bench()}), flush=True)
        return
    S = setup(args.workload, args)
    n = S["n"]
    stream = S["stream"]
    graph = None
    if args.graph:
        # capture one window; the hill count lives on the device, so replays keep depositing
        with torch.cuda.stream(stream):
            window(S)
            stream.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                window(S)
        log("[bench] captured one window as a HIP graph")
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            graph.replay() if graph is not None else window(S)
        stream.synchronize()
        S["pipe"].check()
        log(f"[bench] warmup done ({args.warmup} windows)")
        # Inside the timed region only the force calls are bracketed by events
        # (the roofline's k_pass4 launches): an event pair around every call
        # adds about 0.3 ms to a 5 ms window.  The other calls are timed in
        # instrumented windows after it.
        ev = [] if graph is None else None
        pool = event_pool(2 * MD_STEPS_PER_WINDOW * args.steps) if graph is None else None
        e_win = event_pool(args.steps)  # an event at every window boundary (per-window spread)
        e_start = torch.cuda.Event(enable_timing=True)
        e_stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e_start.record(stream)
        for i in range(args.steps):
            if graph is not None:
                graph.replay()
            else:
                window(S, ev, pool, only=("apply_bias_forces",))
            e_win[i].record(stream)
        e_stop.record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    S["pipe"].check()
    gpu_ms = e_start.elapsed_time(e_stop)
    win_ms = [e_start.elapsed_time(e_win[0])] + [a.elapsed_time(b) for a, b in zip(e_win, e_win[1:])]
    spread = {"median": round(float(np.median(win_ms)), 4), "p10": round(float(np.percentile(win_ms, 10)), 4),
              "p90": round(float(np.percentile(win_ms, 90)), 4)}
    graph_line = None
    if graph is None and args.graph_too:
        # the same window captured once as a HIP graph and replayed (no
        # per-call events can be recorded inside a graph on this runtime)
        with torch.cuda.stream(stream):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                window(S)
            for _ in range(2):
                g.replay()
            stream.synchronize()
            ge = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
            ge[0].record(stream)
            for i in range(args.steps):
                g.replay()
                ge[i + 1].record(stream)
            stream.synchronize()
        S["pipe"].check()
        gw = [a.elapsed_time(b) for a, b in zip(ge, ge[1:])]
        gmean = ge[0].elapsed_time(ge[-1]) / args.steps
        graph_line = {"ms_per_step": round(gmean, 4), "value": n * MD_STEPS_PER_WINDOW / (gmean * 1e-3),
                      "window_ms": {"median": round(float(np.median(gw)), 4),
                                    "p10": round(float(np.percentile(gw, 10)), 4),
                                    "p90": round(float(np.percentile(gw, 90)), 4)}}
        log(f"[bench] graph-replayed windows: {gmean:.3f} ms each")
    ms_per_window = gpu_ms / args.steps
    atom_steps = n * MD_STEPS_PER_WINDOW * args.steps
    value = atom_steps / (gpu_ms / 1e3)
    log(f"[bench] {args.steps} windows: {gpu_ms:.2f} ms GPU, {wall * 1e3:.2f} ms wall")

    per_call = {}
    if ev:
        for name, e0, e1 in ev:
            per_call.setdefault(name, []).append(e0.elapsed_time(e1))
    timed_us = {k: 1e3 * float(np.mean(v)) for k, v in per_call.items()}
    # every call of a few more windows, each bracketed by events (not part of
    # the throughput figure)
    per_call_us = {}
    if graph is None and args.call_windows > 0:
        ev2, pool2 = [], event_pool(2 * CALLS_PER_WINDOW * args.call_windows)
        with torch.cuda.stream(stream):
            for _ in range(args.call_windows):
                window(S, ev2, pool2)
            stream.synchronize()
        S["pipe"].check()
        calls = {}
        for name, e0, e1 in ev2:
            calls.setdefault(name, []).append(e0.elapsed_time(e1))
        per_call_us = {k: round(1e3 * float(np.mean(v)), 2) for k, v in calls.items()}

    mx, total_entries, cut_pairs = S["pipe"].neighbor_stats(cutoff_pairs=True)
    roofline = None
    if "apply_bias_forces" in timed_us:
        # Dominant launch: k_pass4 (apply_bias_forces, one launch per call), bound
        # by FP32 VALU work: the fraction of the published FP32 peak, and of the
        # ceiling without packed FP32 (which these kernels do not use).  Its
        # average over every launch of the timed region.
        t_us = timed_us["apply_bias_forces"]
        flops = FLOPS_PER_PAIR_P4 * cut_pairs
        achieved = flops / (t_us * 1e-6) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                    "peak_nonpacked": round(ALU_NONPACKED_TFLOPS, 1),
                    "frac_nonpacked": round(achieved / ALU_NONPACKED_TFLOPS, 4),
                    "traffic": measured_traffic() if args.workload == "wz1m" else None,
                    "kernel": "k_pass4 (apply_bias_forces)", "avg_launch_us": round(t_us, 2),
                    "flops_per_launch": int(flops), "pairs_in_cutoff": int(cut_pairs),
                    "hbm_bytes_per_launch": int(n * P4_BYTES_PER_ATOM + 2 * cut_pairs)}
    # Whole step against HBM: the layout-independent model's algorithmic bytes
    # per atom-step, and beside it this layout's own (its 16-wide rows, cutoff
    # rows and tables, each counted once per write and once per read).
    step_s = ms_per_window / MD_STEPS_PER_WINDOW * 1e-3
    bpas = model_bytes_per_atom_step(total_entries / n)
    step_hbm = n * bpas / step_s / 1e9
    layout_bytes = n * STEP_BYTES_PER_ATOM + 2 * 4 * cut_pairs + n * (4 * (total_entries / n) + 40) / MD_STEPS_PER_WINDOW
    out = {
        "metric": "atom-steps/s for q6-CV+bias+force at 1.02M atoms (%HBM roofline); p50/p99 req latency",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_window,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 CV sum and hill sums)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: wurtzite GaN-like slab, {n} atoms (half crystal, half RSA), "
                               f"q6 crystalline-count CV, r_c 3.6 + skin 0.4, {S['cen'].shape[0]} hills, "
                               f"window = 1 rebuild + 10 x (cv_forward, bias_eval, cv_backward, "
                               f"apply_bias_forces) + 1 deposit",
                   "atoms": n, "md_steps_per_step": MD_STEPS_PER_WINDOW, "graph": bool(args.graph),
                   "neighbor_entries": int(total_entries), "autotuned": S["tuned"]},
        "window_ms": spread,
        "graph_replay": graph_line,
        "per_call_us": per_call_us,
        "per_call_from": (f"{args.call_windows} windows after the timed region, an event pair around every call "
                          f"(inside the timed region only apply_bias_forces is bracketed)"),
        "roofline": roofline,
        "step_hbm": {"achieved_gbs": round(step_hbm, 1), "peak_gbs": HBM_PEAK_GBS,
                     "frac": round(step_hbm / HBM_PEAK_GBS, 4), "bytes_per_atom_step": round(bpas, 1),
                     "bytes_per_step": int(n * bpas), "layout_bytes_per_step": int(layout_bytes),
                     "layout_frac": round(layout_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4)},
    }
    if not args.no_serving and args.workload == "wz1m":
        log("[bench] serving workload ...")
        out["serving"] = serving(args)
    if not args.no_cpu:
        log("[bench] timing the oracle on the host cores ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
