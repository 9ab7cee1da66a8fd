"""torch.autograd wrappers around the C ABI (forward step and its hand-written adjoint).

`sdc_step(x, sdc, dt, M, K)` returns the state after one dSDC step; its backward calls
sdc_step_adjoint, which recomputes the node stages of that step from the saved input.  A loop of
steps therefore keeps one checkpoint per step (the step's input state) and recomputes each step's
stages during the backward pass.  With taped=True the forward keeps the step's stage grid fields
in a device tape (sdc_tape_size bytes per step) and the backward reads them instead of
recomputing (same gradient, bitwise).  `sht_inverse(spec, sdc)` is the scalar synthesis with its
transpose as backward.  Gradients follow the real inner product over (Re, Im) of every stored
coefficient; the imaginary parts of m = 0 entries of state gradients are zero.
"""
from __future__ import annotations

import torch


class _SDCStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, sdc, dt, M, K, taped):
        y = x.detach().clone().contiguous()
        if taped:
            tape = sdc.new_tape(M, K)
            sdc.step_taped(y, dt, tape, M, K)
            ctx.save_for_backward(tape)
        else:
            sdc.step(y, dt, M, K)
            ctx.save_for_backward(x.detach())
        ctx.sdc, ctx.dt, ctx.M, ctx.K, ctx.taped = sdc, dt, M, K, taped
        return y

    @staticmethod
    def backward(ctx, gy):
        (saved,) = ctx.saved_tensors
        lam = gy.detach().contiguous().clone()
        out = torch.empty_like(lam)
        if ctx.taped:
            ctx.sdc.step_adjoint_taped(saved, lam, out, ctx.dt, ctx.M, ctx.K)
        else:
            ctx.sdc.step_adjoint(saved.contiguous(), lam, out, ctx.dt, ctx.M, ctx.K)
        return out, None, None, None, None, None


class _SHTInverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, spec, sdc):
        grid = torch.empty(sdc.grid_shape, dtype=torch.float64, device=spec.device)
        sdc.sht_inverse(spec.detach().contiguous(), grid)
        ctx.sdc = sdc
        return grid

    @staticmethod
    def backward(ctx, gg):
        spec = torch.empty(ctx.sdc.spec_shape, dtype=torch.float64, device=gg.device)
        ctx.sdc.sht_inverse_adjoint(gg.detach().contiguous(), spec)
        return spec, None


def sdc_step(x, sdc, dt: float, M: int = None, K: int = None, taped: bool = False):
    return _SDCStep.apply(x, sdc, float(dt), M or sdc.M, K or sdc.K, bool(taped))


def sht_inverse(spec, sdc):
    return _SHTInverse.apply(spec, sdc)


def height_loss(x, phi_target, sdc, gravity: float):
    """0.5 * sum over grid points of (h - h_target)^2 with h = (Phi_bar + Phi')/g and
    h_target = H + Phi'_target/g (the mean depth cancels): Phi' is field 0 of the state."""
    diff = sht_inverse((x[:, 0] - phi_target).contiguous(), sdc) / gravity
    return 0.5 * torch.sum(diff * diff)
