"""Continuous batching: every walker's CV, bias and forces are bitwise the
same whether it is served in the mix or alone; admission honours the budget."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def requests(count=10):
    import bench

    return bench.serving_requests(count=count, seed=3, n_hi=6000)


def test_serving_results_same_alone_and_in_mix():
    from paper_2510_06873_amd.serving import serve_batched, serve_sequential

    reqs = requests()
    for r in reqs:
        r.steps = 25
    rb, sb = serve_batched(reqs, hbm_budget=64 << 30, max_slots=4, keep_forces=True)
    rs, ss = serve_sequential(reqs, keep_forces=True)
    assert len(rb) == len(rs) == len(reqs)
    alone = {r.rid: r for r in rs}
    for r in rb:
        a = alone[r.rid]
        assert np.array_equal(r.s, a.s), r.rid
        assert r.V == a.V, r.rid
        assert np.array_equal(r.forces, a.forces), r.rid
        assert r.latency > 0
    assert sb["p99_ms"] >= sb["p50_ms"] > 0


def test_admission_respects_budget():
    from paper_2510_06873_amd.serving import device_bytes, serve_batched

    reqs = requests(6)
    for r in reqs:
        r.steps = 10
    budget = max(device_bytes(r) for r in reqs) + 1
    rb, sb = serve_batched(reqs, hbm_budget=budget, max_slots=8)
    assert len(rb) == len(reqs)
    assert sb["peak_bytes"] <= budget


def test_overflowing_walker_is_run_again_with_wider_rows():
    """A request whose neighbour rows are far too narrow (8 entries for some
    17-30 neighbours): the batched loop finds the overflow in the error word
    at retirement, discards that result and runs the request again with rows
    twice as wide until it fits; the results equal the sequential run's."""
    from dataclasses import replace

    from paper_2510_06873_amd.serving import serve_batched, serve_sequential

    reqs = requests(5)
    for r in reqs:
        r.steps = 12
    narrow = [i for i, r in enumerate(reqs) if r.params.cv_kind == 2][:1] or [0]
    for i in narrow:
        reqs[i].params = replace(reqs[i].params, max_neighbors=8)
    rb, _ = serve_batched(reqs, hbm_budget=64 << 30, max_slots=3, keep_forces=True)
    rs, _ = serve_sequential(reqs, keep_forces=True)
    assert sorted(r.rid for r in rb) == sorted(r.rid for r in reqs)
    alone = {r.rid: r for r in rs}
    for r in rb:
        a = alone[r.rid]
        assert np.array_equal(r.s, a.s) and r.V == a.V, r.rid
        assert np.array_equal(r.forces, a.forces), r.rid


def test_tuned_requests_match_untuned_and_serve_bitwise_alone():
    """Requests tuned per class (brick shape and lanes per atom): served in
    the mix they equal their own sequential run bitwise, and they agree with
    the library's default geometry within the FP32 bars (the geometry only
    reorders the sums)."""
    from paper_2510_06873_amd.serving import serve_batched, serve_sequential, tune_requests

    reqs = requests(8)
    for r in reqs:
        r.steps = 12
    tuned, chosen = tune_requests(reqs, steps=2, limit=3)
    assert len(tuned) == len(reqs) and chosen
    for r, t in zip(reqs, tuned):
        assert t.rid == r.rid and t.params.cv_kind == r.params.cv_kind and t.params.lds_kb == r.params.lds_kb
    rt, _ = serve_batched(tuned, hbm_budget=64 << 30, max_slots=4, keep_forces=True)
    ra, _ = serve_sequential(tuned, keep_forces=True)
    rd, _ = serve_batched(reqs, hbm_budget=64 << 30, max_slots=4, keep_forces=True)
    alone = {r.rid: r for r in ra}
    default = {r.rid: r for r in rd}
    for r in rt:
        a, d = alone[r.rid], default[r.rid]
        assert np.array_equal(r.s, a.s) and r.V == a.V and np.array_equal(r.forces, a.forces), r.rid
        assert np.allclose(r.s, d.s, rtol=1e-5, atol=1e-6), r.rid
        f, fd = r.forces[:, :3].astype(np.float64), d.forces[:, :3].astype(np.float64)
        assert np.max(np.abs(f - fd)) <= 1e-4 * max(np.max(np.abs(fd)), 1.0), r.rid
