"""The allocation-free reweighting (gm_fes_reweight_noalloc) against the
allocating call it mirrors (gm_fes_reweight), through the C-ABI: the same
free energies on two calls in a row, the second with fewer samples and a
smaller grid (so the fixed scratch still holds the first call's values
beyond what the second one uses), on the LDS-histogram and the global-sum
paths, and the grid limit rejected before any device work."""
import math

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def _same(F_new, F_ref, kBT):
    """Same empty bins; finite values equal up to the order of the FP64
    atomic adds of the per-bin sums (1e-12 kBT)."""
    fin = np.isfinite(F_ref)
    assert np.array_equal(np.isfinite(F_new), fin)
    assert fin.sum() > 0
    assert np.max(np.abs(F_new[fin] - F_ref[fin])) <= 1e-12 * kBT


@pytest.mark.parametrize("dims,grids", [
    (2, ([200, 180], [40, 30])),       # 36,000 bins (global sums) then 1,200 (LDS histograms)
    (1, ([65536], [5000])),            # the largest grid the scratch holds, then a smaller one
])
def test_noalloc_equals_allocating_call_twice(dims, grids):
    import paper_2510_06873_amd as P

    kBT = W.KBT_KJMOL
    lo, hi = [-math.pi] * dims, [math.pi] * dims
    for k, (T, nb) in enumerate(zip((200000, 30000), grids)):
        s, V = W.biased_trace(T=T, dims=dims, seed=60 + 7 * k + dims)
        sd, Vd = _dev(s), _dev(V)
        total = int(np.prod(nb))
        F_ref = P.fes_reweight(sd, Vd, lo, hi, nb, kBT)
        F_new = torch.full((total,), float("nan"), dtype=torch.float64, device=sd.device)
        out = P.fes_reweight_noalloc(sd, Vd, lo, hi, nb, kBT, F_new)
        torch.cuda.synchronize()
        assert out is F_new
        _same(F_new.cpu().numpy(), F_ref.cpu().numpy(), kBT)


def test_noalloc_rejects_grids_beyond_its_scratch():
    import paper_2510_06873_amd as P

    s, V = W.biased_trace(T=1000, dims=1, seed=3)
    sd, Vd = _dev(s), _dev(V)
    F = torch.zeros(65537, dtype=torch.float64, device=sd.device)
    with pytest.raises(P.GmError, match="TOO_LARGE"):
        P.fes_reweight_noalloc(sd, Vd, [-math.pi], [math.pi], [65537], W.KBT_KJMOL, F)
