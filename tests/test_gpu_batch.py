"""Batched walkers: one launch per pass for many uneven systems gives, per
walker, bitwise the same CV, bias, forces and hills as stepping it alone."""
import numpy as np
import pytest

import workloads as W
from tests.helpers import params_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q6 = dict(cv="q6", precision="fp32", r_c=3.6, skin=0.4, taper=0.2, cn_r0=2.5, bond_d0=0.7, bond_w=0.02,
          count_n0=5.5, count_w=0.25, sigma=[20.0], w0=W.W0_EV, gamma=10.0, kBT=W.KBT_EV, hills=dict(k=64))


def walkers():
    """(workload params, structure) of uneven walkers with all three CV kinds."""
    out = []
    for spec in (dict(nx=4, ny=3, nz=6, seed=21), dict(nx=8, ny=4, nz=8, seed=5), dict(nx=12, ny=6, nz=6, seed=7)):
        out.append((Q6, W.wurtzite_slab(**spec)))
    out.append((dict(W.WORKLOADS["wz2048"], precision="fp32"), W.structure(W.WORKLOADS["wz2048"]["structure"])))
    out.append((dict(W.WORKLOADS["fcc864"], precision="fp32"), W.structure(W.WORKLOADS["fcc864"]["structure"])))
    return out


def setup(wl, d, dev, k):
    from paper_2510_06873_amd import Pipeline

    n = len(d["pos"])
    pipe = Pipeline(n, params_for(wl, max_neighbors=96))
    p4 = torch.from_numpy(W.as_float4(d["pos"], d["species"])).to(dev)
    F = torch.from_numpy(W.external_forces(n, seed=100 + k)).to(dev)
    pipe.build_neighbors_checked(p4, d["box"])
    s0 = pipe.cv_forward(p4).cpu().numpy()
    sig = np.array(wl["sigma"])
    cen = W.hill_centres(50, s0 - 2 * sig, s0 + 2 * sig, seed=200 + k)
    pipe.hills_set(cen, np.full(50, wl["w0"]))
    return pipe, p4, F


def test_batch_bitwise_equals_solo():
    from paper_2510_06873_amd import Batch

    dev = torch.device("cuda", 0)
    ws = walkers()
    solo = []
    for k, (wl, d) in enumerate(ws):
        pipe, p4, F = setup(wl, d, dev, k)
        for step in range(3):
            if step == 1:
                pipe.deposit_hill()
            pipe.step(p4, F)
        torch.cuda.synchronize()
        assert pipe.status(True) == 0
        solo.append((pipe.s.cpu().numpy().copy(), pipe.V.cpu().numpy().copy(), F.cpu().numpy().copy(),
                     pipe.hills_get()))
    pipes, pos, forces = [], [], []
    for k, (wl, d) in enumerate(ws):
        pipe, p4, F = setup(wl, d, dev, k)
        pipes.append(pipe)
        pos.append(p4)
        forces.append(F)
    batch = Batch(pipes, pos, forces)
    batch.build([d["box"] for _, d in ws])
    for step in range(3):
        if step == 1:
            batch.deposit()
        batch.step()
    s, V = batch.values()
    torch.cuda.synchronize()
    for k, p in enumerate(pipes):
        assert p.status(True) == 0
        s_solo, V_solo, F_solo, (c_solo, h_solo) = solo[k]
        dims = p.dims
        assert np.array_equal(s[k, :dims].cpu().numpy(), s_solo[:dims]), k
        assert V[k].item() == V_solo[0], k
        assert np.array_equal(forces[k].cpu().numpy(), F_solo), k
        c, h = p.hills_get()
        assert np.array_equal(c, c_solo) and np.array_equal(h, h_solo), k


def _run_solo(wl, d, dev, k, steps):
    pipe, p4, F = setup(wl, d, dev, k)
    for step in range(steps):
        if step == 1:
            pipe.deposit_hill()
        pipe.step(p4, F)
    return pipe, F


def test_context_churn_on_another_stream():
    """Contexts created, stepped and destroyed on one stream while another
    context steps on a second stream: every result is bitwise that of a quiet
    run on the default stream (buffers are allocated, zero-filled and released
    in stream order, with no device-wide wait to keep them apart)."""
    dev = torch.device("cuda", 0)
    ws = walkers()
    long_k, long_steps = 3, 12
    ref = {}
    for k, (wl, d) in enumerate(ws):
        pipe, F = _run_solo(wl, d, dev, k, long_steps if k == long_k else 3)
        torch.cuda.synchronize()
        ref[k] = (pipe.s.cpu().numpy().copy(), pipe.V.item(), F.cpu().numpy().copy(), pipe.hills_get())
        pipe.close()
    sA, sB = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    with torch.cuda.stream(sA):
        wl, d = ws[long_k]
        pA, FA = _run_solo(wl, d, dev, long_k, long_steps)  # enqueued on sA, not waited for
    for rnd in range(2):
        for k in (0, 1, 2, 4):
            with torch.cuda.stream(sB):
                pipe, F = _run_solo(ws[k][0], ws[k][1], dev, k, 3)
                got = (pipe.s.cpu().numpy().copy(), pipe.V.item(), F.cpu().numpy().copy(), pipe.hills_get())
                assert pipe.status(True) == 0
                pipe.close()
            s, V, Fr, (c, h) = ref[k]
            assert np.array_equal(got[0], s) and got[1] == V, (rnd, k)
            assert np.array_equal(got[2], Fr), (rnd, k)
            assert np.array_equal(got[3][0], c) and np.array_equal(got[3][1], h), (rnd, k)
    sA.synchronize()
    with torch.cuda.stream(sA):
        assert pA.status(True) == 0
        s, V, Fr, (c, h) = ref[long_k]
        assert np.array_equal(pA.s.cpu().numpy(), s) and pA.V.item() == V
        assert np.array_equal(FA.cpu().numpy(), Fr)
        cA, hA = pA.hills_get()
        assert np.array_equal(cA, c) and np.array_equal(hA, h)
        pA.close()


def test_context_with_a_smaller_lds_budget_created_later():
    """The kernels' LDS limit is shared by all contexts: a context created
    later with a smaller staging budget (as the autotuner makes) must leave an
    earlier context's launches working and its results unchanged."""
    from paper_2510_06873_amd import Pipeline

    dev = torch.device("cuda", 0)
    wl, d = walkers()[3]
    ref, F_ref = _run_solo(wl, d, dev, 3, 2)
    torch.cuda.synchronize()
    s_ref, F_ref = ref.s.cpu().numpy().copy(), F_ref.cpu().numpy().copy()
    ref.close()
    pipe, p4, F = setup(wl, d, dev, 3)  # default budget (78 KiB)
    prm = params_for(wl, max_neighbors=96)
    prm.lds_kb = 40
    later = Pipeline(len(d["pos"]), prm)
    for step in range(2):
        if step == 1:
            pipe.deposit_hill()
        pipe.step(p4, F)
    torch.cuda.synchronize()
    assert pipe.status(True) == 0
    assert np.array_equal(pipe.s.cpu().numpy(), s_ref)
    assert np.array_equal(F.cpu().numpy(), F_ref)
    later.close()


def test_batch_update_members_bitwise_equals_solo():
    """One batch whose members change between steps (walkers join, finish and
    leave, the member list ends empty): every walker's CV, bias, forces and
    hills are bitwise those of stepping it alone, and contexts closed after
    leaving the batch do not disturb the ones that stay."""
    from paper_2510_06873_amd import Batch

    dev = torch.device("cuda", 0)
    ws = walkers()
    solo = {}
    for k, (wl, d) in enumerate(ws):
        pipe, F = _run_solo(wl, d, dev, k, 3)
        torch.cuda.synchronize()
        solo[k] = (pipe.s.cpu().numpy().copy(), pipe.V.item(), F.cpu().numpy().copy(), pipe.hills_get())
        pipe.close()
    made = {k: setup(wl, d, dev, k) for k, (wl, d) in enumerate(ws)}
    joins = {0: [0, 1, 2], 1: [3], 2: [4]}
    active, done, batch = [], {}, None
    for tick in range(8):
        active += joins.get(tick, [])
        if not active:
            break
        args = ([made[k][0] for k in active], [made[k][1] for k in active], [made[k][2] for k in active])
        if batch is None:
            batch = Batch(*args)
        else:
            batch.update(*args)
        for k in active:
            if done.get(k, 0) == 1:
                made[k][0].deposit_hill()
        batch.step()
        s, V = batch.values()
        s, V = s.cpu().numpy(), V.cpu().numpy()
        for row, k in enumerate(active):
            done[k] = done.get(k, 0) + 1
        finished = [k for k in active if done[k] == 3]
        for k in finished:
            row = active.index(k)
            pipe, p4, F = made[k]
            assert pipe.status(True) == 0, k
            s_solo, V_solo, F_solo, (c_solo, h_solo) = solo[k]
            assert np.array_equal(s[row, :pipe.dims], s_solo[:pipe.dims]), (tick, k)
            assert V[row] == V_solo, (tick, k)
            assert np.array_equal(F.cpu().numpy(), F_solo), (tick, k)
            c, h = pipe.hills_get()
            assert np.array_equal(c, c_solo) and np.array_equal(h, h_solo), (tick, k)
        active = [k for k in active if k not in finished]
        batch.update([made[k][0] for k in active], [made[k][1] for k in active], [made[k][2] for k in active])
        for k in finished:
            made[k][0].close()
    assert sorted(done) == list(range(len(ws))) and all(v == 3 for v in done.values())
    batch.close()


def test_batch_deposit_some_bitwise_equals_solo():
    """Deposits for some members only (one launch pair): the depositing
    walkers' hills are bitwise those of gm_deposit_hill on each alone, the
    others get none; repeated or out-of-range indices are refused."""
    from paper_2510_06873_amd import Batch
    from paper_2510_06873_amd.binding import GmError

    dev = torch.device("cuda", 0)
    ws = walkers()
    solo = {}
    for k, (wl, d) in enumerate(ws):
        pipe, p4, F = setup(wl, d, dev, k)
        pipe.step(p4, F)
        if k in (1, 3):
            pipe.deposit_hill()
        pipe.step(p4, F)
        torch.cuda.synchronize()
        solo[k] = (pipe.hills_get(), F.cpu().numpy().copy())
        pipe.close()
    made = [setup(wl, d, dev, k) for k, (wl, d) in enumerate(ws)]
    batch = Batch([m[0] for m in made], [m[1] for m in made], [m[2] for m in made])
    batch.step()
    for bad in ([1, 1], [len(ws)], [-1]):
        with pytest.raises(GmError):
            batch.deposit(bad)
    batch.deposit([3, 1])
    batch.step()
    torch.cuda.synchronize()
    for k, (pipe, p4, F) in enumerate(made):
        assert pipe.status(True) == 0
        (c_solo, h_solo), F_solo = solo[k]
        c, h = pipe.hills_get()
        assert np.array_equal(c, c_solo) and np.array_equal(h, h_solo), k
        assert np.array_equal(F.cpu().numpy(), F_solo), k
    batch.close()


def test_batch_build_some_bitwise_equals_solo():
    """Rebuilds of some members in one launch per stage (and a system too
    large for the one-workgroup scans, rebuilt alone in the same call, on a
    second stream): cell lists, neighbour rows and the step that follows are
    bitwise those of gm_build_neighbors; bad indices are refused."""
    from paper_2510_06873_amd import Batch, Pipeline
    from paper_2510_06873_amd.binding import GmError

    dev = torch.device("cuda", 0)
    ws = walkers()
    big = W.walker_structure("wz", 120000, seed=77)
    big_wl = dict(Q6, cv="q6")
    ws.append((big_wl, dict(pos=big[0], species=big[1], box=big[2])))
    solo = []
    for k, (wl, d) in enumerate(ws):
        pipe, p4, F = setup(wl, d, dev, k)
        pipe.step(p4, F)
        torch.cuda.synchronize()
        _, perm, start = pipe.cell_list()
        nbr, cnt = pipe.neighbor_lists()
        solo.append((perm.cpu().numpy(), start.cpu().numpy(), nbr.cpu().numpy(), cnt.cpu().numpy(),
                     pipe.s.cpu().numpy().copy(), F.cpu().numpy().copy()))
        pipe.close()
    made = [setup(wl, d, dev, k) for k, (wl, d) in enumerate(ws)]
    # lists built from shifted positions first, so that the batched rebuild
    # has to replace every table
    for k, (pipe, p4, F) in enumerate(made):
        box = torch.tensor(np.asarray(ws[k][1]["box"], np.float64), device=dev)
        shifted = p4.clone()
        shifted[:, :3] = torch.remainder(p4[:, :3].double() + 1.37, box).float()
        pipe.build_neighbors_checked(shifted, ws[k][1]["box"])
        torch.cuda.synchronize()
    batch = Batch([m[0] for m in made], [m[1] for m in made], [m[2] for m in made])
    for bad in ([0, 0], [len(ws)]):
        with pytest.raises(GmError):
            batch.build_some(bad, [ws[0][1]["box"]] * len(bad))
    side = torch.cuda.Stream(device=dev)
    order = [5, 0, 3, 1, 4, 2]
    side.wait_stream(batch.stream)
    batch.build_some(order, [ws[k][1]["box"] for k in order], stream=side)
    batch.stream.wait_stream(side)
    batch.step()
    s_b = batch.values()[0].cpu().numpy()
    torch.cuda.synchronize()
    for k, (pipe, p4, F) in enumerate(made):
        assert pipe.status(True) == 0, k
        perm0, start0, nbr0, cnt0, s0, F0 = solo[k]
        _, perm, start = pipe.cell_list()
        nbr, cnt = pipe.neighbor_lists()
        assert np.array_equal(perm.cpu().numpy(), perm0) and np.array_equal(start.cpu().numpy(), start0), k
        cnt, nbr = cnt.cpu().numpy(), nbr.cpu().numpy()
        assert np.array_equal(cnt, cnt0), k
        # entries past a row's count are not written by the copy
        used = np.arange(nbr.shape[1])[None, :] < np.minimum(cnt, nbr.shape[1])[:, None]
        assert np.array_equal(nbr[used], nbr0[used]), k
        assert np.array_equal(s_b[k, :pipe.dims], s0[:pipe.dims]), k
        assert np.array_equal(F.cpu().numpy(), F0), k
    batch.close()


def test_batch_build_some_fp64_and_changed_box():
    """The batched rebuild in FP64 (its gather and neighbour rows in double),
    and a walker rebuilt with a different box (new cell geometry: its device
    argument block is rewritten), both bitwise equal to gm_build_neighbors."""
    from paper_2510_06873_amd import Batch

    dev = torch.device("cuda", 0)
    wl = W.WORKLOADS["fcc864"]
    ds = [W.fcc_jittered(n=6, a=3.615, jitter=0.1, seed=s) for s in (1, 2, 3)]
    # the same atoms in a box 6% larger on x: other cells, same pairs
    big = dict(ds[2])
    big["box"] = np.asarray(big["box"], np.float64) * np.array([1.06, 1.0, 1.0])

    def lists(pipe):
        _, perm, start = pipe.cell_list()
        nbr, cnt = pipe.neighbor_lists()
        cnt, nbr = cnt.cpu().numpy(), nbr.cpu().numpy()
        used = np.arange(nbr.shape[1])[None, :] < np.minimum(cnt, nbr.shape[1])[:, None]
        return perm.cpu().numpy(), start.cpu().numpy(), cnt, nbr[used]

    def setup64(d, k):
        pipe, p4, F = setup(wl, d, dev, k)
        return pipe, p4, F.to(pipe.fdtype)

    solo, hills = [], []
    for k, d in enumerate(ds[:2] + [big]):
        pipe, p4, F = setup64(d, k)
        hills.append(pipe.hills_get())
        pipe.step(p4, F)
        torch.cuda.synchronize()
        solo.append((lists(pipe), pipe.s.cpu().numpy().copy(), F.cpu().numpy().copy()))
        pipe.close()
    made = [setup64(d, k) for k, d in enumerate(ds)]
    for (pipe, _, _), (cen, hts) in zip(made, hills):
        pipe.hills_set(cen, hts)  # walker 2's hills were placed around its CV in the larger box
    assert all(m[0].fdtype == torch.float64 for m in made)
    batch = Batch([m[0] for m in made], [m[1] for m in made], [m[2] for m in made])
    batch.build_some([0, 1, 2], [ds[0]["box"], ds[1]["box"], ds[2]["box"]])  # argument blocks uploaded
    batch.build_some([2, 0, 1], [big["box"], ds[0]["box"], ds[1]["box"]])  # walker 2: new grid
    batch.step()
    s_b = batch.values()[0].cpu().numpy()
    torch.cuda.synchronize()
    for k, (pipe, p4, F) in enumerate(made):
        assert pipe.status(True) == 0, k
        (perm0, start0, cnt0, nbr0), s0, F0 = solo[k]
        perm, start, cnt, nbr = lists(pipe)
        assert np.array_equal(perm, perm0) and np.array_equal(start, start0), k
        assert np.array_equal(cnt, cnt0) and np.array_equal(nbr, nbr0), k
        assert np.array_equal(s_b[k, :1], s0), k
        assert np.array_equal(F.cpu().numpy(), F0), k
    batch.close()
