"""torch.autograd wrappers around the CV and bias calls.

The paper obtains bias forces from PyTorch's automatic differentiation
(Results, "Frameworks of GPU-MetaD").  Here the derivative is the library's
hand-written adjoint: `CollectiveVariable.backward` calls `gm_cv_backward`
with the incoming gradient as the seed and gets `sum_d seed_d ds_d/dx` in one
pass, so `V(s(x)).backward()` runs the same kernels as `gm_apply_bias_forces`.

Two ways to hold the per-atom forward state (q-hat rows, bond counts):

* ``"stored"``    backward uses the state the forward left in the context;
                  if another forward ran on the same context in between, it is
                  recomputed (the context holds one state at a time).
* ``"recompute"`` backward always reruns the forward passes first and gives
                  the per-atom rows back to the library's pool when it is
                  done (``gm_release_rows``), so the context holds no
                  per-atom CV state between calls (128 B per atom in FP32).
"""
from __future__ import annotations

import torch

from .binding import Pipeline


class CollectiveVariable(torch.autograd.Function):
    """s = CV(pos4); d(loss)/d(pos4) = sum_d d(loss)/ds_d * ds_d/dx."""

    @staticmethod
    def forward(ctx, pos4: torch.Tensor, pipe: Pipeline, mode: str = "stored"):
        if mode not in ("stored", "recompute"):
            raise ValueError("mode must be 'stored' or 'recompute'")
        s = torch.empty(pipe.dims, dtype=torch.float64, device=pos4.device)
        pipe.cv_forward(pos4.detach(), s)
        if mode == "recompute":
            pipe.release_rows()  # the backward computes them again
        ctx.pipe = pipe
        ctx.mode = mode
        ctx.generation = pipe.generation
        ctx.save_for_backward(pos4)
        return s

    @staticmethod
    def backward(ctx, grad_s: torch.Tensor):
        (pos4,) = ctx.saved_tensors
        pipe: Pipeline = ctx.pipe
        p = pos4.detach()
        if ctx.mode == "recompute" or pipe.generation != ctx.generation:
            pipe.cv_forward(p, torch.empty(pipe.dims, dtype=torch.float64, device=p.device))
        seed = grad_s.detach().to(torch.float64).contiguous()
        grad4 = torch.zeros((pipe.n, 4), dtype=pipe.fdtype, device=p.device)
        pipe.cv_backward(p, seed, grad4)
        if ctx.mode == "recompute":
            pipe.release_rows()
        return grad4.to(pos4.dtype), None, None


class GaussianBias(torch.autograd.Function):
    """V = sum_k h_k exp(-sum_d (s_d - c_kd)^2 / 2 sigma_d^2) over the context's
    hills (paper, Methods: the equation for V_b); dV/ds from the same kernel."""

    @staticmethod
    def forward(ctx, s: torch.Tensor, pipe: Pipeline):
        V = torch.empty(1, dtype=torch.float64, device=s.device)
        dV = torch.empty(pipe.dims, dtype=torch.float64, device=s.device)
        pipe.bias_eval(s.detach().contiguous(), V, dV)
        ctx.save_for_backward(dV)
        return V[0]

    @staticmethod
    def backward(ctx, grad_V: torch.Tensor):
        (dV,) = ctx.saved_tensors
        return grad_V * dV, None


def cv(pos4: torch.Tensor, pipe: Pipeline, mode: str = "stored") -> torch.Tensor:
    return CollectiveVariable.apply(pos4, pipe, mode)


def bias_energy(pos4: torch.Tensor, pipe: Pipeline, mode: str = "stored") -> torch.Tensor:
    """V(s(pos4)) as a differentiable scalar: -grad is the bias force."""
    return GaussianBias.apply(CollectiveVariable.apply(pos4, pipe, mode), pipe)
