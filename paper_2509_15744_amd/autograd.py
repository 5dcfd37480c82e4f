"""The misfit as a differentiable function of the material.

``FdMisfit.apply(c, problem, k)`` returns J(c) (Eq. cost1) and records the forward
sweep of Alg. 1 (``fd_sens_forward``: propagation, cost, adjoint force and K(u,u)
accumulation).  Its backward is the superposed backward sweep
(``fd_sens_backward``): dJ/dc from (K(v,v) - K(u,u)) / (2k) (Eq. superposedkernel),
scaled by the incoming gradient.  The state carried between the two is four
device arrays of the grid size plus the residual rows: no forward history.

The backward consumes that state, so a graph built by one ``apply`` can be
differentiated once (``retain_graph`` is not supported).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import fdwave


@dataclass
class SensProblem:
    """Everything except the speed field that fixes J: grid spacing and order,
    acquisition (host cell indices, device wavelet [nt, nsrc]), observed data
    (device [nt, nrec]), time axis, and kernel options."""
    dx: float
    order: int
    src: np.ndarray
    rec: np.ndarray
    wavelet: torch.Tensor
    observed: torch.Tensor
    dt: float
    nt: int
    acc_dtype: str | None = None
    variant: int = 0
    chunk: int = 0
    shots: tuple | None = None      # (src_shot, rec_shot, nshot) for a batch of shots


class FdMisfit(torch.autograd.Function):
    """J(c) with the memory-efficient adjoint as its backward."""

    @staticmethod
    def forward(ctx, c: torch.Tensor, prob: SensProblem, k: float):
        c = c.contiguous()
        nshot = prob.shots[2] if prob.shots is not None else 1
        state = fdwave.SweepState(c, prob.nt, len(prob.rec), acc_dtype=prob.acc_dtype, nshot=nshot)
        J = fdwave.fd_sens_forward(c, prob.dx, prob.order, prob.src, prob.wavelet, prob.rec,
                                   prob.dt, prob.nt, prob.observed, state, shots=prob.shots,
                                   acc_dtype=prob.acc_dtype, variant=prob.variant,
                                   chunk=prob.chunk)
        ctx.save_for_backward(c)
        ctx.state = state
        ctx.prob = prob
        ctx.k = float(k)
        return torch.tensor(J, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        (c,) = ctx.saved_tensors
        if ctx.state is None:
            raise RuntimeError("FdMisfit: the backward sweep consumes the forward state; "
                               "differentiate each apply() once")
        prob = ctx.prob
        grad = fdwave.fd_sens_backward(c, prob.dx, prob.order, prob.src, prob.wavelet, prob.rec,
                                       prob.dt, prob.nt, ctx.k, ctx.state,
                                       grad_scale=float(gJ.item()), shots=prob.shots,
                                       acc_dtype=prob.acc_dtype, variant=prob.variant,
                                       chunk=prob.chunk)
        ctx.state = None
        return grad, None, None


def misfit(c: torch.Tensor, prob: SensProblem, k: float) -> torch.Tensor:
    """J(c) as a differentiable scalar (float64 tensor on c's device)."""
    return FdMisfit.apply(c, prob, k)


class FdVdMisfit(torch.autograd.Function):
    """J(m, b) of the variable-material second-order scheme (the paper's Sec. 3.1
    flux form, mass m and stiffness b) with Alg. 1 as its backward: the forward records
    the forward sweep (``fd_vd_sens_forward``), the backward runs the superposed sweep
    (``fd_vd_sens_backward``) and returns (dJ/dm, dJ/db) scaled by the incoming
    gradient.  ``prob.order`` is ignored (the scheme is second order)."""

    @staticmethod
    def forward(ctx, m: torch.Tensor, b: torch.Tensor, prob: SensProblem, k: float):
        m, b = m.contiguous(), b.contiguous()
        nshot = prob.shots[2] if prob.shots is not None else 1
        state = fdwave.VdSweepState(m, prob.nt, len(prob.rec), acc_dtype=prob.acc_dtype, nshot=nshot)
        J = fdwave.fd_vd_sens_forward(m, b, prob.dx, prob.src, prob.wavelet, prob.rec, prob.dt, prob.nt,
                                      prob.observed, state, shots=prob.shots, acc_dtype=prob.acc_dtype,
                                      variant=prob.variant, chunk=prob.chunk)
        ctx.save_for_backward(m, b)
        ctx.state = state
        ctx.prob = prob
        ctx.k = float(k)
        return torch.tensor(J, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        m, b = ctx.saved_tensors
        if ctx.state is None:
            raise RuntimeError("FdVdMisfit: the backward sweep consumes the forward state; "
                               "differentiate each apply() once")
        prob = ctx.prob
        gm, gb = fdwave.fd_vd_sens_backward(m, b, prob.dx, prob.src, prob.wavelet, prob.rec, prob.dt, prob.nt,
                                            ctx.k, ctx.state, grad_scale=float(gJ.item()), shots=prob.shots,
                                            acc_dtype=prob.acc_dtype, variant=prob.variant, chunk=prob.chunk)
        ctx.state = None
        return gm, gb, None, None


def vd_misfit(m: torch.Tensor, b: torch.Tensor, prob: SensProblem, k: float) -> torch.Tensor:
    """J(m, b) as a differentiable scalar (float64 tensor on m's device)."""
    return FdVdMisfit.apply(m, b, prob, k)
