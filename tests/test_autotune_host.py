"""Host logic of the brick autotuner (no GPU needed): cell counts, the
feasible candidates and their order, the cache key."""
import math

import numpy as np
import pytest

import workloads as W


def _params(**kw):
    from paper_2510_06873_amd import Params

    return Params(**kw)


@pytest.fixture(scope="module")
def at():
    try:
        from paper_2510_06873_amd import autotune
    except ImportError:
        pytest.skip("library not built")
    return autotune


def test_cells_per_axis(at):
    assert at.cells_per_axis([12.0, 12.3, 16.2], 4.0) == (3, 3, 4)
    assert at.cells_per_axis([255.2, 221.0, 207.6], 4.0) == (63, 55, 51)


def test_candidates_are_feasible_ordered_and_unique(at):
    d = W.wurtzite_slab(nx=16, ny=8, nz=12, seed=3)
    n, box = len(d["pos"]), d["box"]
    prm = _params(cv_kind=2, r_c=3.6, skin=0.4, sigma=[20.0], hill_capacity=8)
    nc = at.cells_per_axis(box, 4.0)
    rho = n / float(np.prod(nc))
    cands = at.candidates(n, box, prm, limit=8)
    assert 0 < len(cands) <= 8
    keys = set()
    owns = []
    for (bx, by, bz), kb, tpa in cands:
        assert kb in (40, 48, 56, 64) and tpa in (1, 2, 4)
        assert 1 <= bx <= min(4, nc[0]) and 1 <= by <= min(4, nc[1]) and 1 <= bz <= min(4, nc[2])
        cap = (kb * 1024 - 2048) // 80  # q6 slots: position and a 16-float row
        assert (bx + 2) * (by + 2) * (bz + 2) * rho <= 1.25 * cap
        own = bx * by * bz * rho
        assert own * tpa <= 1.2 * 512  # lanes of one FP32 workgroup
        owns.append(min(own * tpa, 0.94 * 512))
        key = (tuple(sorted((bx, by, bz))), kb, tpa)
        assert key not in keys  # one brick shape per permutation, budget and lane count
        keys.add(key)
    assert owns == sorted(owns, reverse=True)  # most busy lanes first
    assert len({c[2] for c in at.candidates(n, box, prm, limit=40)}) > 1  # lane counts are searched


def test_cache_key_separates_kind_precision_and_density(at):
    box = [40.0, 40.0, 40.0]
    a = _params(cv_kind=2, r_c=3.6, skin=0.4, sigma=[20.0], hill_capacity=8)
    b = _params(cv_kind=1, r_c=3.6, skin=0.4, sigma=[20.0], hill_capacity=8)
    c = _params(cv_kind=2, precision=1, r_c=3.6, skin=0.4, sigma=[20.0], hill_capacity=8)
    k = at.cache_key(5000, box, a)
    assert k == at.cache_key(5000, box, a)
    assert len({k, at.cache_key(5000, box, b), at.cache_key(5000, box, c), at.cache_key(9000, box, a)}) == 4
    # walkers of one size class share a key; the classes differ
    assert at.cache_key(5000, box, a) == at.cache_key(5010, box, a)
    assert [at.size_class(n) for n in (1000, 5000, 50000, 500000)] == [0, 1, 2, 3]
