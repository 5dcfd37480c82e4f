"""Gradient-based design with the memory-efficient sensitivities (Sec. 2.3 and the
update of Eq. gradientdescent, with Adam as the optimiser).

One design iteration is five calls into the library, all on the device:

1. ``fd_design_map``: design field gamma on a box of cells -> density filter ->
   projection -> clip -> material (m, b) of the variable-material scheme;
2. ``fd_vd_sens_forward``: forward sweep, J, adjoint force, forward kernel sums;
3. ``fd_vd_sens_backward``: the superposed backward sweep (Alg. 1), dC/dm and dC/db
   with C = scale * J applied as the gradient scale;
4. ``fd_design_adjoint``: dC/dgamma by the chain rule of step 1;
5. ``fd_adam_step``: the Adam update of gamma and its clip to the admissible interval.

Objectives: the data misfit of Eq. cost1 (full waveform inversion: observed traces,
scale 1) and the region objective of Eq. cost2 for topology optimisation,
C = (1/A) int_T int_{Omega_s} u^2, which is the misfit with a receiver on every cell of
Omega_s, zero observed data and scale 2 / (number of cells): with
J = dt/2 sum_n sum_r u_r^2 and A = cells * dx^d the two agree, and the adjoint force
-scale * u / dt is the paper's -2u/A in the scheme's units (Eq. adjointSource2).
A negative scale maximises C (the amplifying design of the paper's example).

``AdamDesign`` also runs the beta-continuation of the projection (beta grows by a
factor every few iterations).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import calibrate, fdwave


@dataclass
class DesignProblem:
    """Everything but the design field: the box and its chain (``fdwave.make_design``),
    the material outside the box (device fields of the grid shape; box cells are
    overwritten by each map), acquisition, objective and time axis."""
    design: fdwave.fd_design
    m: torch.Tensor
    b: torch.Tensor
    dx: float
    src: np.ndarray
    wavelet: torch.Tensor
    rec: np.ndarray
    observed: torch.Tensor
    dt: float
    nt: int
    scale: float = 1.0
    acc_dtype: str | None = None
    variant: int = 0
    chunk: int = 0


def region_receivers(shape, origin, extent) -> np.ndarray:
    """Flat C-order cell indices of every cell of a box (the receivers of the region
    objective)."""
    idx = np.indices(tuple(int(e) for e in extent)).reshape(len(shape), -1)
    idx = idx + np.asarray(origin, dtype=np.int64).reshape(-1, 1)
    return np.ravel_multi_index(tuple(idx), tuple(shape)).astype(np.int64)


def region_scale(ncells: int, maximize: bool = False) -> float:
    """C / J of the region objective: 2 / cells (negated to maximise)."""
    return (-2.0 if maximize else 2.0) / ncells


def stable_dt(material, lo: float, hi: float, dx: float, ndim: int, frac: float = 0.95,
              samples: int = 2001) -> float:
    """A time step that passes the library's stability check for EVERY design: the
    largest Gershgorin row sum 2d max_{g_i, g_j} h(b_i, b_j)(1/m_i + 1/sqrt(m_i m_j))
    over material values g in [lo, hi] (sampled), times frac of its limit."""
    m0, dm, b0, db = material
    g = np.linspace(lo, hi, samples)
    m = m0 + g * dm
    b = b0 + g * db
    if (m <= 0).any() or (b <= 0).any():
        raise ValueError("the material map gives a non-positive coefficient on [lo, hi]")
    bi, bj = b[:, None], b[None, :]
    mi, mj = m[:, None], m[None, :]
    face = 2 * bi * bj / (bi + bj) * (1 / mi + 1 / np.sqrt(mi * mj))
    row = 2 * ndim * face.max()
    return frac * 2.0 * dx / math.sqrt(row)


class AdamDesign:
    """Adam on the design field with the memory-efficient gradient.  ``k`` is the
    superposition factor (None: ``calibrate.auto_k`` from the first forward sweep);
    [lo, hi] the admissible interval of gamma; the projection's beta is multiplied by
    ``beta_growth`` every ``beta_every`` iterations (continuation)."""

    def __init__(self, prob: DesignProblem, gamma0: torch.Tensor, lr: float, k: float | None = None,
                 betas=(0.9, 0.999), eps: float = 1e-8, lo: float = 0.0, hi: float = 1.0,
                 beta_growth: float = 1.1, beta_every: int = 5):
        self.prob = prob
        self.gamma = gamma0.detach().clone().contiguous()
        self.m1 = torch.zeros_like(self.gamma)
        self.m2 = torch.zeros_like(self.gamma)
        self.grad = torch.empty_like(self.gamma)
        self.lr, self.betas, self.eps, self.lo, self.hi = lr, betas, eps, lo, hi
        self.beta_growth, self.beta_every = beta_growth, beta_every
        self.k = k
        self.it = 0
        self.state = fdwave.VdSweepState(prob.m, prob.nt, len(prob.rec), acc_dtype=prob.acc_dtype)
        self.grad_m = torch.empty_like(prob.m)
        self.grad_b = torch.empty_like(prob.m)
        self.history: list[float] = []
        self.sweep_opts: dict = {}   # extra fd_opts fields for the two sweeps (e.g. timing)

    def _opts(self):
        p = self.prob
        return dict(acc_dtype=p.acc_dtype, variant=p.variant, chunk=p.chunk, **self.sweep_opts)

    def evaluate(self) -> float:
        """C at the current gamma and dC/dgamma into ``self.grad`` (no update)."""
        p = self.prob
        fdwave.fd_design_map(p.design, self.gamma, p.m, p.b)
        J = fdwave.fd_vd_sens_forward(p.m, p.b, p.dx, p.src, p.wavelet, p.rec, p.dt, p.nt, p.observed,
                                      self.state, **self._opts())
        if self.k is None:
            wn = float(torch.linalg.vector_norm(p.wavelet.double()))
            self.k = calibrate.auto_k(J, p.dt, wn, p.dx, p.design.ndim)
        fdwave.fd_vd_sens_backward(p.m, p.b, p.dx, p.src, p.wavelet, p.rec, p.dt, p.nt, self.k, self.state,
                                   grad_scale=p.scale, grad_m=self.grad_m, grad_b=self.grad_b, **self._opts())
        fdwave.fd_design_adjoint(p.design, self.gamma, self.grad_m, self.grad_b, self.grad)
        return p.scale * J

    def step(self) -> float:
        """One iteration: evaluate, Adam update with clip, beta continuation.  Returns C
        before the update."""
        C = self.evaluate()
        self.it += 1
        fdwave.fd_adam_step(self.gamma, self.grad, self.m1, self.m2, self.it, self.lr, self.betas[0],
                            self.betas[1], self.eps, self.lo, self.hi)
        d = self.prob.design
        if d.beta > 0 and self.beta_every > 0 and self.it % self.beta_every == 0:
            d.beta *= self.beta_growth
        self.history.append(C)
        return C
