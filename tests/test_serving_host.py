"""Host-side logic of the serving loop (no GPU needed)."""
import numpy as np
import pytest


def test_serving_rejects_a_request_larger_than_the_budget():
    """A walker that alone exceeds the HBM budget could never be admitted: the
    server refuses the request set up front instead of waiting for it."""
    try:
        from paper_2510_06873_amd import Params
        from paper_2510_06873_amd.serving import Request, device_bytes, serve_batched
    except ImportError:
        pytest.skip("library not built")
    pos = np.zeros((1000, 4), np.float32)
    req = Request(0, 0.0, pos, np.full(3, 20.0), Params(cv_kind=2, sigma=[1.0], hill_capacity=8),
                  np.zeros((0, 1)), np.zeros(0), pos.copy())
    with pytest.raises(ValueError, match="budget"):
        serve_batched([req], hbm_budget=device_bytes(req) - 1)
