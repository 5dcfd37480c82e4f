"""Choice of the superposition factor k (Sec. 4.1).

The approximation error of Alg. 1 grows linearly in k (the k^2 K(u_dagger, u_dagger)
term of the superposed kernel), while a small k makes K(v,v) - K(u,u) a difference of
nearly equal sums, so the gradient of a low-precision run drifts away from the
high-precision one.  The paper's rule takes the smallest k at which single and double
precision still agree.  Two helpers:

* ``auto_k``: a scale-free k from quantities known between the two sweeps, the norm
  of the source term and of the adjoint force (||f_dagger|| follows from J).
* ``sweep_k``: the paper's rule as a decade sweep on the device: for each k the f32 and
  f64 gradients of Alg. 1 and the f64 exact gradient (re-simulation), reporting the
  gap to the exact gradient and the f32-vs-f64 disagreement, and the smallest k whose
  disagreement is within a tolerance.

Everything runs through the C-ABI (``fdwave``); this module only loops and compares.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import torch

from . import fdwave as fdw


def adjoint_force_norm(J: float, dt: float) -> float:
    """||f_dagger|| over all receivers and steps: f_dagger^n = -residual^n / dt and
    J = dt/2 sum residual^2, so ||f_dagger|| = sqrt(2 J / dt) / dt."""
    return math.sqrt(2.0 * J / dt) / dt


def auto_k(J: float, dt: float, wavelet_norm: float, dx: float, ndim: int, beta: float = 0.005) -> float:
    """k = beta ||f|| / ||f_dagger|| with ||f|| = ||wavelet|| / dx^ndim: the superposed
    force f + k f_dagger then carries a fixed share beta of adjoint force, whatever the
    units of the data.  Returns 1.0 when there is no adjoint force (J = 0)."""
    fd = adjoint_force_norm(J, dt)
    if not (fd > 0.0) or not math.isfinite(fd):
        return 1.0
    return beta * (wavelet_norm / dx ** ndim) / fd


@dataclass
class KPoint:
    k: float
    gap: float        # ||g64(k) - g_exact|| / ||g_exact||
    fp32_err: float   # ||g32(k) - g64(k)|| / ||g64(k)||
    g64: Optional[torch.Tensor] = None   # with keep=True: the two device gradients at k
    g32: Optional[torch.Tensor] = None


def _rel(a: torch.Tensor, b: torch.Tensor) -> float:
    a64, b64 = a.double(), b.double()
    nb = float(torch.linalg.vector_norm(b64))
    return float(torch.linalg.vector_norm(a64 - b64)) / (nb if nb > 0 else 1.0)


def sweep_k(c: torch.Tensor, dx: float, order: int, src, wavelet: torch.Tensor, rec, dt: float, nt: int,
            observed: torch.Tensor, ks, tol: float = 1e-4, shots=None, keep: bool = False, **opts):
    """Decade sweep of k (the paper's calibration rule).  c, wavelet and observed are
    device tensors (any float dtype; they are run in both f32 and f64).  Returns
    (points, k_best): one KPoint per k in ascending order, and the smallest k whose
    fp32_err <= tol (None if none qualifies).  With keep the points also hold the f64
    and f32 gradients, and the exact gradient is returned third."""
    c64, w64, o64 = c.double(), wavelet.double(), observed.double()
    c32, w32, o32 = c.float(), wavelet.float(), observed.float()
    g_ex, _ = fdw.fd_adjoint_exact(c64, dx, order, src, w64, rec, dt, nt, o64, shots=shots, **opts)
    points = []
    for k in sorted(float(x) for x in ks):
        g64, _ = fdw.fd_adjoint_sensitivity(c64, dx, order, src, w64, rec, dt, nt, o64, k, shots=shots, **opts)
        g32, _ = fdw.fd_adjoint_sensitivity(c32, dx, order, src, w32, rec, dt, nt, o32, k, shots=shots, **opts)
        points.append(KPoint(k, _rel(g64, g_ex), _rel(g32, g64), g64 if keep else None, g32 if keep else None))
    best = next((p.k for p in points if p.fp32_err <= tol), None)
    return (points, best, g_ex) if keep else (points, best)
