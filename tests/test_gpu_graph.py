"""A window of the pipeline (rebuild, three MD steps, one deposit) captured as
a HIP graph and replayed several times, with eager work and synchronisations
between the replays, against the same windows run eagerly: CV, bias, forces
and the hill history after every replay are bitwise those of the eager run
(the window's kernels take every scalar from device memory and clear their
counters with kernels, so a replay repeats the eager launches exactly)."""
import numpy as np
import pytest

import workloads as W
from tests.helpers import params_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q6_2D = dict(cv="coord_q6", precision="fp32", r_c=3.6, skin=0.4, taper=0.2, cn_r0=2.5, bond_d0=0.7, bond_w=0.02,
             count_n0=5.5, count_w=0.25, sigma=[0.2, 20.0], w0=W.W0_EV, gamma=10.0, kBT=W.KBT_EV,
             hills=dict(k=64))


def window(pipe, p4, F, box):
    pipe.build_neighbors(p4, box)
    for _ in range(3):
        pipe.cv_forward(p4)
        pipe.bias_eval()
        pipe.cv_backward(p4)
        pipe.apply_bias_forces(p4, F)
    pipe.deposit_hill()


def snapshot(pipe, F):
    pipe.stream.synchronize()
    c, h = pipe.hills_get()
    return pipe.s.cpu().numpy().copy(), pipe.V.cpu().numpy().copy(), F.cpu().numpy().copy(), c, h


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_window_graph_replays_match_eager(precision):
    from paper_2510_06873_amd import Pipeline

    dev = torch.device("cuda", 0)
    d = W.wurtzite_slab(nx=8, ny=4, nz=8, seed=5)
    pos, box, sp = d["pos"], d["box"], d["species"]
    n = len(pos)
    wl = dict(Q6_2D, precision=precision)
    p4 = torch.from_numpy(W.as_float4(pos, sp)).to(dev)
    probe = Pipeline(n, params_for(wl, max_neighbors=96))
    probe.build_neighbors_checked(p4, box)
    s0 = probe.cv_forward(p4).cpu().numpy()
    probe.close()
    sig = np.array(wl["sigma"])
    cen = W.hill_centres(40, s0 - 2 * sig, s0 + 2 * sig, seed=8)

    def make(stream):
        with torch.cuda.stream(stream):
            pipe = Pipeline(n, params_for(wl, max_neighbors=96), stream=stream)
            pipe.hills_set(cen, np.full(40, wl["w0"]))
            F = torch.from_numpy(W.external_forces(n, seed=3)).to(device=dev, dtype=pipe.fdtype)
            pipe.build_neighbors_checked(p4, box)
        return pipe, F

    replays = 4
    se = torch.cuda.Stream(device=dev)
    pe, Fe = make(se)
    eager = []
    with torch.cuda.stream(se):
        for _ in range(replays + 1):
            window(pe, p4, Fe, box)
            eager.append(snapshot(pe, Fe))
    assert pe.status(True) == 0

    sg = torch.cuda.Stream(device=dev)
    pg, Fg = make(sg)
    with torch.cuda.stream(sg):
        window(pg, p4, Fg, box)  # the first window eagerly (sizes every buffer), as the eager run
        got = [snapshot(pg, Fg)]
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=sg):
            window(pg, p4, Fg, box)
        for _ in range(replays):
            graph.replay()
            got.append(snapshot(pg, Fg))
            Fg.add_(0.0)  # eager work on the same stream between replays
    assert pg.status(True) == 0
    for k, (a, b) in enumerate(zip(eager, got)):
        for name, x, y in zip(("s", "V", "F", "centres", "heights"), a, b):
            assert np.array_equal(x, y), (k, name)
    assert len(got[-1][4]) == 40 + replays + 1


def test_batch_graph_replays_match_eager():
    """A batch of uneven walkers (all three CV kinds): one step for all of them
    and a deposit, captured once and replayed; every walker's CV, bias,
    forces and hills after each replay equal the eager batch's bitwise."""
    from paper_2510_06873_amd import Batch, Pipeline

    dev = torch.device("cuda", 0)
    kinds = [dict(Q6_2D, cv="q6", sigma=[20.0]), dict(Q6_2D, cv="coord", sigma=[0.2]), dict(Q6_2D)]
    structs = [W.wurtzite_slab(nx=4, ny=3, nz=6, seed=21), W.wurtzite_slab(nx=8, ny=4, nz=8, seed=5),
               W.wurtzite_slab(nx=6, ny=4, nz=4, seed=9)]

    def make(stream):
        pipes, pos, forces, boxes = [], [], [], []
        with torch.cuda.stream(stream):
            for k, (wl, d) in enumerate(zip(kinds, structs)):
                n = len(d["pos"])
                pipe = Pipeline(n, params_for(wl, max_neighbors=96), stream=stream)
                p4 = torch.from_numpy(W.as_float4(d["pos"], d["species"])).to(dev)
                pipe.build_neighbors_checked(p4, d["box"])
                s0 = pipe.cv_forward(p4).cpu().numpy()
                sig = np.array(wl["sigma"])
                pipe.hills_set(W.hill_centres(20, s0 - 2 * sig, s0 + 2 * sig, seed=30 + k), np.full(20, wl["w0"]))
                pipes.append(pipe)
                pos.append(p4)
                forces.append(torch.from_numpy(W.external_forces(n, seed=40 + k)).to(dev))
                boxes.append(d["box"])
            batch = Batch(pipes, pos, forces, stream=stream)
            batch.build(boxes)
        return batch, pipes, forces

    def iteration(batch):
        batch.step()
        batch.deposit()

    def snapshot(batch, pipes, forces):
        s, V = batch.values()
        batch.stream.synchronize()
        return [(s[k].cpu().numpy().copy(), V[k].item(), forces[k].cpu().numpy().copy(), *p.hills_get())
                for k, p in enumerate(pipes)]

    replays = 3
    se = torch.cuda.Stream(device=dev)
    be, pe, fe = make(se)
    eager = []
    with torch.cuda.stream(se):
        for _ in range(replays + 1):
            iteration(be)
            eager.append(snapshot(be, pe, fe))
    sg = torch.cuda.Stream(device=dev)
    bg, pg, fg = make(sg)
    with torch.cuda.stream(sg):
        iteration(bg)
        got = [snapshot(bg, pg, fg)]
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=sg):
            iteration(bg)
        for _ in range(replays):
            graph.replay()
            got.append(snapshot(bg, pg, fg))
    for p in pe + pg:
        assert p.status(True) == 0
    for r, (a, b) in enumerate(zip(eager, got)):
        for k in range(len(kinds)):
            for name, x, y in zip(("s", "V", "F", "centres", "heights"), a[k], b[k]):
                assert np.array_equal(x, y), (r, k, name)


def test_per_call_graphs_match_eager():
    """Each call of a window captured as its own graph (as the benchmark
    replays them, with events between the replays) and replayed in the
    window's order for several windows: CV, bias, forces and hills equal
    those of the same windows run eagerly, bit for bit."""
    from paper_2510_06873_amd import Pipeline

    dev = torch.device("cuda", 0)
    d = W.wurtzite_slab(nx=8, ny=4, nz=8, seed=5)
    pos, box, sp = d["pos"], d["box"], d["species"]
    n = len(pos)
    wl = dict(Q6_2D, cv="q6", sigma=[20.0])
    p4 = torch.from_numpy(W.as_float4(pos, sp)).to(dev)

    def make(stream):
        with torch.cuda.stream(stream):
            pipe = Pipeline(n, params_for(wl, max_neighbors=96), stream=stream)
            pipe.build_neighbors_checked(p4, box)
            s0 = pipe.cv_forward(p4).cpu().numpy()
            pipe.hills_set(W.hill_centres(30, s0 - 40.0, s0 + 40.0, seed=12), np.full(30, wl["w0"]))
            F = torch.from_numpy(W.external_forces(n, seed=6)).to(dev)
        return pipe, F

    windows = 3
    se = torch.cuda.Stream(device=dev)
    pe, Fe = make(se)
    eager = []
    with torch.cuda.stream(se):
        for _ in range(windows + 1):
            window(pe, p4, Fe, box)
            eager.append(snapshot(pe, Fe))
    sg = torch.cuda.Stream(device=dev)
    pg, Fg = make(sg)
    with torch.cuda.stream(sg):
        window(pg, p4, Fg, box)
        got = [snapshot(pg, Fg)]
        calls = (("build", pg.build_neighbors, (p4, box)), ("fwd", pg.cv_forward, (p4,)), ("bias", pg.bias_eval, ()),
                 ("bwd", pg.cv_backward, (p4,)), ("force", pg.apply_bias_forces, (p4, Fg)),
                 ("dep", pg.deposit_hill, ()))
        graphs = {}
        for name, fn, a in calls:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=sg):
                fn(*a)
            graphs[name] = g
        for _ in range(windows):
            e = torch.cuda.Event(enable_timing=True)
            graphs["build"].replay()
            for _ in range(3):
                for name in ("fwd", "bias", "bwd", "force"):
                    graphs[name].replay()
                    e.record(sg)
            graphs["dep"].replay()
            got.append(snapshot(pg, Fg))
    assert pe.status(True) == 0 and pg.status(True) == 0
    for k, (a, b) in enumerate(zip(eager, got)):
        for name, x, y in zip(("s", "V", "F", "centres", "heights"), a, b):
            assert np.array_equal(x, y), (k, name)
