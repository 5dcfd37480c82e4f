"""k calibration helpers: host arithmetic of auto_k (CPU) and the decade sweep of the
paper's rule on the device (the gap is linear in k, the f32-vs-f64 disagreement
falls as k grows, the chosen k is the smallest within the tolerance)."""
import math

import numpy as np
import pytest
import torch

from paper_2509_15744_amd import workloads as wl
from helpers import say, to_dev


def test_auto_k_closed_form():
    from paper_2509_15744_amd import calibrate
    # J = dt/2 sum r^2 with residual r: ||fdag|| = ||r|| / dt
    r = np.array([0.3, -0.4, 1.2])
    dt = 0.25
    J = 0.5 * dt * float((r ** 2).sum())
    assert math.isclose(calibrate.adjoint_force_norm(J, dt), np.linalg.norm(r) / dt, rel_tol=1e-14)
    wnorm, dx = 2.0, 0.5
    k = calibrate.auto_k(J, dt, wnorm, dx, 2, beta=0.01)
    assert math.isclose(k, 0.01 * (wnorm / dx ** 2) / (np.linalg.norm(r) / dt), rel_tol=1e-14)
    assert calibrate.auto_k(0.0, dt, wnorm, dx, 2) == 1.0


@pytest.mark.gpu
def test_sweep_k_follows_the_paper_rule():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import calibrate, fdwave as fdw
    p = wl.inclusion_2d(nt=400)
    f64 = torch.float64
    obs = fdw.fd_forward(to_dev(p.c_ref, f64), p.dx, p.order, p.src, to_dev(p.wavelet, f64), p.rec, p.dt, p.nt)
    ks = [1e-3, 1e-2, 1e-1, 1.0, 10.0]
    say("k sweep on the inclusion workload")
    pts, best = calibrate.sweep_k(to_dev(p.c, f64), p.dx, p.order, p.src, to_dev(p.wavelet, f64), p.rec,
                                  p.dt, p.nt, obs, ks, tol=1e-4)
    for q in pts:
        say(f"  k {q.k:.0e}: gap {q.gap:.3e}, f32 vs f64 {q.fp32_err:.3e}")
    gaps = np.array([q.gap for q in pts])
    # linear in k (the k^2 term of the superposed kernel over k)
    assert np.allclose(gaps[1:] / gaps[:-1], 10.0, rtol=0.02)
    errs = np.array([q.fp32_err for q in pts])
    assert errs[0] > errs[-1]
    assert best is not None
    i = [q.k for q in pts].index(best)
    assert pts[i].fp32_err <= 1e-4 and all(q.fp32_err > 1e-4 for q in pts[:i])


@pytest.mark.gpu
def test_sweep_k_against_the_oracle():
    """The decade sweep on the device against the FP64 oracle on the same inputs (the
    inclusion workload, observed data from the oracle's forward solve): the device
    exact gradient equals the oracle's stored-history adjoint, each f64 gradient the
    oracle's Alg. 1 at that k (1e-9), the device gap(k) the oracle's gap(k), which is
    k times the closed-form gap per unit k (sum of squared adjoint increments over c^3),
    and the paper's rule (smallest k whose f32 gradient is within the tolerance of the
    double-precision one) picks the same k with the oracle's gradients as the reference."""
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    import oracle
    from paper_2509_15744_amd import calibrate
    from helpers import rel
    p = wl.inclusion_2d(nt=400)
    obs, _, _ = oracle.forward(p.c_ref, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec)
    g_ex_o, _, s2, _ = oracle.exact_gradient(p.c, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec, obs)
    gap1 = np.linalg.norm(s2 / p.c ** 3) / np.linalg.norm(g_ex_o)
    f64 = torch.float64
    ks = [1e-3, 1e-2, 1e-1, 1.0, 10.0]
    tol = 1e-4
    say("k sweep against the oracle")
    pts, best, g_ex = calibrate.sweep_k(to_dev(p.c, f64), p.dx, p.order, p.src, to_dev(p.wavelet, f64), p.rec,
                                        p.dt, p.nt, to_dev(obs, f64), ks, tol=tol, keep=True)
    assert rel(g_ex.cpu().numpy(), g_ex_o) < 1e-9
    errs_o = []
    for q in pts:
        g_ap_o, _, _ = oracle.superposition_gradient(p.c, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec,
                                                     obs, q.k)
        gap_o = rel(g_ap_o, g_ex_o)
        g64 = q.g64.cpu().numpy()
        g32 = q.g32.cpu().numpy()
        errs_o.append(rel(g32, g_ap_o))
        say(f"  k {q.k:.0e}: gap {q.gap:.4e} (oracle {gap_o:.4e}, k gap1 {q.k * gap1:.4e}), "
            f"f32 {q.fp32_err:.3e} (vs oracle {errs_o[-1]:.3e})")
        assert rel(g64, g_ap_o) < 1e-9
        assert abs(gap_o - q.k * gap1) <= 1e-9 * q.k * gap1
        assert abs(q.gap - gap_o) <= 1e-7 * gap_o
        assert abs(q.fp32_err - errs_o[-1]) <= 1e-3 * errs_o[-1] + 1e-12
    best_o = next((q.k for q, e in zip(pts, errs_o) if e <= tol), None)
    assert best is not None and best == best_o
