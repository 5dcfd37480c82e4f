"""FP64 oracle of the design chain around the sweeps (arXiv:2509.15744, Sec. 2.3,
"Constraints", and the update of Eq. gradientdescent with Adam).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the product path never
imports it, and it shares no code with the GPU library.

Plain numpy, written from the definitions:

* density filter with linear decay: gt_i = sum_k w(x_i - x_k) gamma_k / sum_k w(x_i - x_k),
  w(x) = r_f - |x| for |x| < r_f (cells), k over the design cells;
* smoothed Heaviside projection
  H(gt) = (tanh(beta eta) + tanh(beta (gt - eta))) / (tanh(beta eta) + tanh(beta (1 - eta)))
  and its slope beta / ((tanh(beta eta) + tanh(beta (1 - eta))) cosh^2(beta (gt - eta)));
* clip of the projected field to [lo, hi] (the paper clips it to [0, 1]);
* the material maps, both affine in the clipped field: rho-scaling
  (Eq. scalarwaveequation: m = g rho0, b = g rho0 c0^2) and the two-material map of
  Eq. wavetopopt (m = 1/kappa1 + g (1/kappa2 - 1/kappa1), b = 1/rho1 + g (1/rho2 - 1/rho1));
* the chain rule dC/dgamma = dC/dg * dg/dgt * dgt/dgamma with the filter's Jacobian
  d gt_i / d gamma_k = w_ik / sum_k w_ik (the paper's expression; applied as the
  transposed product, which is what the chain rule asks for);
* Adam (Kingma and Ba, 2015, Algorithm 1: bias-corrected moments, epsilon added to the
  square root of the corrected second moment), followed by the clip of the design
  field.

Readings: "no filter" is r_f <= 1 (the neighbourhood is the cell itself), "no
projection" is beta <= 0; the derivative of the clip is 1 on the closed interval and
0 outside.
"""
from __future__ import annotations

import itertools

import numpy as np


def filter_offsets(rf: float, ndim: int):
    """[(offset, weight)] with |offset| < rf (offsets in cells), weight rf - |offset|."""
    rf = max(float(rf), 1.0)
    R = int(np.ceil(rf)) - 1
    out = []
    for off in itertools.product(range(-R, R + 1), repeat=ndim):
        dist = np.sqrt(float(sum(o * o for o in off)))
        if dist < rf:
            out.append((off, rf - dist))
    return out


def _shifted(x: np.ndarray, off):
    """y[i] = x[i + off] where i + off lies in the array, and a validity mask."""
    y = np.zeros_like(x)
    mask = np.zeros(x.shape, dtype=bool)
    dst, src = [], []
    for o, n in zip(off, x.shape):
        dst.append(slice(max(0, -o), min(n, n - o)))
        src.append(slice(max(0, o), min(n, n + o)))
    y[tuple(dst)] = x[tuple(src)]
    mask[tuple(dst)] = True
    return y, mask


def filter_weight_sums(shape, rf: float) -> np.ndarray:
    """W_i = sum over the design cells k in the neighbourhood of i of w_ik."""
    W = np.zeros(shape)
    for off, w in filter_offsets(rf, len(shape)):
        _, mask = _shifted(np.zeros(shape), off)
        W += w * mask
    return W


def density_filter(gamma: np.ndarray, rf: float) -> np.ndarray:
    """gt_i = sum_k w_ik gamma_k / W_i over the design cells."""
    gamma = np.asarray(gamma, dtype=np.float64)
    num = np.zeros(gamma.shape)
    for off, w in filter_offsets(rf, gamma.ndim):
        y, _ = _shifted(gamma, off)
        num += w * y
    return num / filter_weight_sums(gamma.shape, rf)


def density_filter_transpose(y: np.ndarray, rf: float) -> np.ndarray:
    """z_k = sum_i (d gt_i / d gamma_k) y_i = sum_i w_ik y_i / W_i."""
    y = np.asarray(y, dtype=np.float64)
    t = y / filter_weight_sums(y.shape, rf)
    out = np.zeros(y.shape)
    for off, w in filter_offsets(rf, y.ndim):
        s, _ = _shifted(t, off)
        out += w * s
    return out


def projection(gt, beta: float, eta: float):
    if beta <= 0:
        return np.asarray(gt, dtype=np.float64).copy()
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (np.tanh(beta * eta) + np.tanh(beta * (np.asarray(gt) - eta))) / den


def projection_slope(gt, beta: float, eta: float):
    if beta <= 0:
        return np.ones(np.shape(gt))
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return beta / (den * np.cosh(beta * (np.asarray(gt) - eta)) ** 2)


def rho_scaling(rho0: float, c0: float):
    """(m0, dm, b0, db) of Eq. scalarwaveequation."""
    return 0.0, rho0, 0.0, rho0 * c0 * c0


def two_material(rho1: float, rho2: float, kappa1: float, kappa2: float):
    """(m0, dm, b0, db) of Eq. wavetopopt with the linear maps of kappa^-1 and rho^-1."""
    return 1.0 / kappa1, 1.0 / kappa2 - 1.0 / kappa1, 1.0 / rho1, 1.0 / rho2 - 1.0 / rho1


def design_map(gamma, rf, beta, eta, lo, hi, material):
    """(g, m_box, b_box): clipped projected filtered field and the material on the box."""
    gt = density_filter(gamma, rf)
    g = np.clip(projection(gt, beta, eta), lo, hi)
    m0, dm, b0, db = material
    return g, m0 + g * dm, b0 + g * db


def design_adjoint(gamma, rf, beta, eta, lo, hi, material, grad_m_box, grad_b_box):
    """dC/dgamma from dC/dm and dC/db on the box."""
    gt = density_filter(gamma, rf)
    h = projection(gt, beta, eta)
    _, dm, _, db = material
    dC_dg = np.asarray(grad_m_box) * dm + np.asarray(grad_b_box) * db
    dC_dgt = dC_dg * ((h >= lo) & (h <= hi)) * projection_slope(gt, beta, eta)
    return density_filter_transpose(dC_dgt, rf)


def box_slices(origin, extent):
    return tuple(slice(o, o + e) for o, e in zip(origin, extent))


def adam(x, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, lo=-np.inf, hi=np.inf):
    """One step of Adam on copies; returns (x, m1, m2)."""
    g = np.asarray(grad, dtype=np.float64)
    m1 = beta1 * np.asarray(m1) + (1.0 - beta1) * g
    m2 = beta2 * np.asarray(m2) + (1.0 - beta2) * g * g
    mhat = m1 / (1.0 - beta1 ** step)
    vhat = m2 / (1.0 - beta2 ** step)
    x = np.asarray(x, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return np.clip(x, lo, hi), m1, m2
