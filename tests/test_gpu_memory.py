"""Device memory handed out again: contexts destroyed and created in turn on two
streams (each new context may receive blocks that a destroyed one left, with
their old contents) give bitwise the results of the first context, and the
first context's results match the oracle (CV at 1e-5 relative, bias force
norm-wise at 1e-4; external forces zero, as in the walker tests).  Also: the
coordination CV alone, which keeps no in-cutoff rows, still reports their
total length."""
import numpy as np
import pytest

from tests.helpers import rel_force_err
from tests.test_gpu_walkers_oracle import oracle_cv, walker_geometry, walker_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run_once(prm, pos, species, box, stream):
    import workloads as W
    from paper_2510_06873_amd import Pipeline

    n = len(pos)
    dev = torch.device("cuda", 0)
    with torch.cuda.stream(stream):
        pipe = Pipeline(n, prm, stream=stream)
        p4 = torch.from_numpy(W.as_float4(pos, species)).to(dev)
        F = torch.zeros((n, 4), dtype=torch.float32, device=dev)
        pipe.build_neighbors_checked(p4, box)
        s0 = pipe.cv_forward(p4).cpu().numpy()
        sig = np.array(prm.sigma[:1])
        pipe.hills_set(W.hill_centres(20, s0 - sig, s0 + sig, seed=3), np.full(20, W.W0_EV))
        pipe.step(p4, F)
        stream.synchronize()
        assert pipe.status(True) == 0
        out = (pipe.s.cpu().numpy().copy(), pipe.dVds.cpu().numpy().copy(), F.cpu().numpy().copy())
    pipe.close()
    return out


@pytest.mark.parametrize("kind,cv", [("fcc", "coord"), ("wz", "q6")])
def test_contexts_on_reused_memory_match_the_first(kind, cv):
    import oracle as orc

    pos, species, box = walker_geometry(kind, 3000, seed=5)
    prm = walker_params(kind, cv, 20)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    first = run_once(prm, pos, species, box, streams[0])
    for k in range(1, 7):
        again = run_once(prm, pos, species, box, streams[k % 2])
        for a, b in zip(first, again):
            assert np.array_equal(a, b), (kind, cv, k)
    s_ref, g_ref = oracle_cv(orc, kind, cv, pos, box)
    s, dV, F = first
    assert abs(s[0] - s_ref) <= 1e-5 * abs(s_ref), (s[0], s_ref)
    assert rel_force_err(F[:, :3], -dV[0] * g_ref) <= 1e-4


@pytest.mark.parametrize("kind", ["fcc", "wz"])
def test_coordination_cutoff_pair_count(kind):
    """The coordination CV alone keeps only the lengths of its in-cutoff rows:
    their sum (gm_neighbor_stats) is the number of ordered pairs inside r_c
    (pairs within 1e-5 A of r_c may fall either way: FP32 on the device, FP64
    here)."""
    import oracle as orc
    import workloads as W
    from paper_2510_06873_amd import Pipeline

    pos, species, box = walker_geometry(kind, 3000, seed=9)
    prm = walker_params(kind, "coord", 4)
    p = W.WALKER_CV[(kind, "coord")]
    n = len(pos)
    dev = torch.device("cuda", 0)
    pipe = Pipeline(n, prm)
    p4 = torch.from_numpy(W.as_float4(pos, species)).to(dev)
    pipe.build_neighbors_checked(p4, box)
    pipe.cv_forward(p4)
    torch.cuda.synchronize()
    _, _, cut = pipe.neighbor_stats(cutoff_pairs=True)
    off, nb = orc.neighbors(pos, box, p["r_c"] + p["skin"])
    i = np.repeat(np.arange(n), np.diff(off))
    d = pos[nb] - pos[i]
    L = np.asarray(box, dtype=np.float64)
    d -= L * np.rint(d / L)
    r = np.linalg.norm(d, axis=1)
    lo, hi = int((r < p["r_c"] - 1e-5).sum()), int((r < p["r_c"] + 1e-5).sum())
    assert lo <= cut <= hi, (cut, lo, hi)
    pipe.close()
