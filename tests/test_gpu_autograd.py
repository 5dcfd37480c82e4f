"""FdMisfit (torch.autograd.Function whose backward is the superposed sweep) against
the oracle, central finite differences and the exact stored-history adjoint.

The 256^3 case (smooth speed in [1, 3], order 8, nt = 2000) compares against
``tests/golden/smooth3d_256_nt2000.npz``, written by
``tests/golden/make_smooth3d_256.py`` with the oracle only (checkpointed exact
adjoint and Alg. 1 at the same k, sampled on every 8th cell per axis).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2509_15744_amd import workloads as wl
from helpers import OracleCase, rel, say, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "smooth3d_256_nt2000.npz")


@pytest.fixture(scope="module")
def ag():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import autograd, fdwave
    return autograd, fdwave


def _prob(ag, p, obs, dtype):
    autograd, fdwave = ag
    return autograd.SensProblem(dx=p.dx, order=p.order, src=p.src, rec=p.rec,
                                wavelet=to_dev(p.wavelet, dtype), observed=to_dev(obs, dtype),
                                dt=p.dt, nt=p.nt)


def test_autograd_equals_oracle_and_scales(ag):
    """f64: J and c.grad equal the oracle's Alg. 1 at the same k to rounding; an outer
    factor on the loss scales the gradient (the backward's grad_scale)."""
    autograd, fdwave = ag
    p = wl.small_random((17, 12, 40), order=8, nt=45, dtype="f64", seed=31)
    case = OracleCase(p, k=0.03)
    say("autograd small f64")
    c = to_dev(p.c, torch.float64).requires_grad_(True)
    prob = _prob(ag, p, case.obs, torch.float64)
    J = autograd.misfit(c, prob, case.k)
    assert abs(J.item() - case.J) < 1e-12 * case.J
    (3.0 * J).backward()
    assert rel(c.grad.cpu().numpy(), 3.0 * case.g_approx) < 1e-9
    # the +k / -k average is the exact discrete adjoint gradient
    c2 = to_dev(p.c, torch.float64).requires_grad_(True)
    autograd.misfit(c2, prob, -case.k).backward()
    avg = 0.5 * (c.grad.cpu().numpy() / 3.0 + c2.grad.cpu().numpy())
    assert rel(avg, case.g_exact) < 1e-9


def test_backward_twice_is_refused(ag):
    autograd, fdwave = ag
    p = wl.small_random((10, 10, 16), order=4, nt=10, dtype="f32", seed=2)
    c = to_dev(p.c, torch.float32).requires_grad_(True)
    obs = np.zeros((p.nt, len(p.rec)))
    J = autograd.misfit(c, _prob(ag, p, obs, torch.float32), 0.1)
    J.backward(retain_graph=True)
    with pytest.raises(RuntimeError):
        J.backward()


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle reference not generated")
def test_autograd_256_cubed(ag):
    """256^3, f32, order 8, nt = 2000: c.grad vs the oracle's Alg. 1 (same k) within
    1e-4; the gap to the exact adjoint reported and matched; the +/-k average vs the
    exact adjoint; central FD (f64, eps = 1e-6) on 64 cells vs the exact adjoint."""
    autograd, fdwave = ag
    ref = np.load(GOLDEN)
    k = float(ref["k"])
    s = (slice(None, None, int(ref["stride"])),) * 3
    p = wl.smooth_3d(n=256, nt=2000)
    say("autograd 256^3 f32, k", k)
    prob = _prob(ag, p, p.observed, torch.float32)
    c = to_dev(p.c, torch.float32).requires_grad_(True)
    J = autograd.misfit(c, prob, k)
    J.backward()
    g = c.grad[s].double().cpu().numpy()
    e_par = rel(g, ref["approx_sample"])
    gap_gpu = rel(g, ref["exact_sample"])
    gap_ref = rel(ref["approx_sample"], ref["exact_sample"])
    say(f"  J {J.item():.9e} (oracle {float(ref['J']):.9e}); parity {e_par:.3e}; "
        f"gap {gap_gpu:.4e} (oracle {gap_ref:.4e}, full field "
        f"{float(ref['gap_norm']) / float(ref['exact_norm']):.4e})")
    assert abs(J.item() - float(ref["J"])) < 1e-4 * float(ref["J"])
    assert e_par < 1e-4
    assert abs(gap_gpu - gap_ref) < 1e-4 + 1e-3 * gap_ref

    cm = to_dev(p.c, torch.float32).requires_grad_(True)
    autograd.misfit(cm, prob, -k).backward()
    g_avg = 0.5 * (c.grad + cm.grad)[s].double().cpu().numpy()
    e_avg = rel(g_avg, ref["exact_sample"])
    say(f"  +/-k average vs exact adjoint {e_avg:.3e}")
    assert e_avg < 1e-3

    # central finite differences of the f64 discrete J at 64 cells of the sample where
    # |g_exact| >= 1e-3 max |g_exact|
    ex = ref["exact_sample"]
    cand = np.argwhere(np.abs(ex) >= 1e-3 * np.abs(ex).max())
    rng = np.random.default_rng(64)
    pick = cand[rng.choice(len(cand), size=min(64, len(cand)), replace=False)]
    stride = int(ref["stride"])
    c64 = to_dev(p.c, torch.float64)
    w64 = to_dev(p.wavelet, torch.float64)
    o64 = to_dev(p.observed, torch.float64)
    eps = 1e-6
    fd, exv, gv = [], [], []
    for cell in pick:
        idx = tuple(int(v) * stride for v in cell)
        jj = []
        for sgn in (1.0, -1.0):
            cp = c64.clone()
            cp[idx] += sgn * eps
            tr = fdwave.fd_forward(cp, p.dx, p.order, p.src, w64, p.rec, p.dt, p.nt)
            jj.append(fdwave.fd_misfit(tr, o64, p.dt))
        fd.append((jj[0] - jj[1]) / (2 * eps))
        exv.append(ex[tuple(cell)])
        gv.append(g_avg[tuple(cell)])
    fd, exv, gv = np.array(fd), np.array(exv), np.array(gv)
    r_fd = np.abs(fd - exv) / np.abs(exv)
    r_gpu = np.abs(gv - fd) / np.abs(fd)
    say(f"  FD vs exact adjoint: median {np.median(r_fd):.2e} max {r_fd.max():.2e}; "
        f"GPU +/-k vs FD: median {np.median(r_gpu):.2e} max {r_gpu.max():.2e}")
    assert np.median(r_fd) < 1e-5 and r_fd.max() < 1e-3
    assert np.median(r_gpu) < 1e-3
