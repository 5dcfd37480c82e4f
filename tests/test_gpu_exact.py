"""Exact discrete gradient by re-simulation (fd_adjoint_exact): u stepped back from its
end levels together with the adjoint field, cross kernel accumulated in the same fused
launch.  Checked element by element against the oracle's stored-history exact adjoint,
against the +/-k average of the superposition on the device (the gap is odd in k), the
per-cell sign of the gap, and at 256^3 against the oracle's checkpointed reference.

Tolerances: f64 1e-9 relative L2 (the re-simulated u carries the rounding of the
backward recursion, ~1e-13 here); f32 1e-4 relative L2.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2509_15744_amd import workloads as wl
from helpers import rel, say, shot_problem, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "smooth3d_256_nt2000.npz")


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def _oracle_exact(p):
    obs, _, _ = oracle.forward(p.c_ref, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec)
    g, J, s2, tr = oracle.exact_gradient(p.c, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec, obs)
    return obs, g, J, s2, tr


def _run_exact(fdw, p, obs, dtype, **opts):
    c, w, o = to_dev(p.c, dtype), to_dev(p.wavelet, dtype), to_dev(obs, dtype)
    tr = torch.empty((p.nt, len(p.rec)), dtype=dtype, device="cuda")
    g, J = fdw.fd_adjoint_exact(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, o, traces=tr, **opts)
    torch.cuda.synchronize()
    return g.double().cpu().numpy(), J, tr.double().cpu().numpy()


@pytest.mark.parametrize("shape,order,nt,seed", [
    ((50, 70), 8, 90, 1),          # 2D, ragged tail along the contiguous axis
    ((37, 130), 4, 70, 2),         # 2D, several tiles plus a tail
    ((14, 11, 70), 8, 40, 3),      # 3D, ragged in both in-plane axes
    ((20, 18, 130), 2, 50, 4),
])
def test_exact_matches_oracle_f64(fdw, shape, order, nt, seed):
    p = wl.small_random(shape, order=order, nt=nt, dtype="f64", seed=seed, nrec=9)
    obs, g_o, J_o, _, tr_o = _oracle_exact(p)
    for variant in [v for v in fdw.variants_for(shape) if v <= 2]:
        say("exact f64", shape, order, nt, "variant", variant)
        g, J, tr = _run_exact(fdw, p, obs, torch.float64, variant=variant)
        assert rel(tr, tr_o) < 1e-12
        assert abs(J - J_o) <= 1e-12 * J_o
        assert rel(g, g_o) < 1e-9, rel(g, g_o)


@pytest.mark.parametrize("acc", ["f64", "f32"])
def test_exact_f32(fdw, acc):
    """f32 fields, either accumulator (the cross kernel has no cancellation, so an f32
    accumulator keeps the bound)."""
    p = wl.small_random((21, 16, 64), order=8, nt=200, dtype="f32", seed=7, nrec=12)
    obs, g_o, J_o, _, _ = _oracle_exact(p)
    say("exact f32, acc", acc)
    g, J, _ = _run_exact(fdw, p, obs, torch.float32, acc_dtype=acc)
    assert abs(J - J_o) < 1e-4 * J_o
    assert rel(g, g_o) < 1e-4, rel(g, g_o)


@pytest.mark.parametrize("shape,nshot,order", [((14, 11, 70), 3, 8), ((40, 66), 5, 4)])
def test_exact_shots(fdw, shape, nshot, order):
    """f64 shot batch: the sum of the per-shot exact gradients of the oracle."""
    P = shot_problem(shape, nshot, order, 31, "f64", seed=11 + nshot)
    g_o = np.zeros(shape)
    J_o = 0.0
    for s in range(nshot):
        si = np.where(P["src_shot"] == s)[0]
        ri = np.where(P["rec_shot"] == s)[0]
        gs, Js, _, _ = oracle.exact_gradient(P["c"], 1.0, order, P["dt"], P["nt"], P["src"][si],
                                             P["wavelet"][:, si], P["rec"][ri], P["obs"][:, ri])
        g_o += gs
        J_o += Js
    f64 = torch.float64
    say("exact shots", shape, nshot, order)
    g, J = fdw.fd_adjoint_exact(to_dev(P["c"], f64), 1.0, order, P["src"], to_dev(P["wavelet"], f64),
                                P["rec"], P["dt"], P["nt"], to_dev(P["obs"], f64),
                                shots=(P["src_shot"], P["rec_shot"], nshot))
    assert abs(J - J_o) <= 1e-12 * J_o
    assert rel(g.cpu().numpy(), g_o) < 1e-9


def test_exact_is_the_pm_k_average_and_below_the_approximation(fdw):
    """f64: [approx(+k) + approx(-k)] / 2 on the device equals the re-simulated exact
    gradient, and approx(+k) - exact = (k / c^3) sum (mu^{n+1} - mu^n)^2 >= 0 per cell
    (the oracle's adjoint field gives the right-hand side)."""
    p = wl.small_random((26, 19, 70), order=8, nt=80, dtype="f64", seed=21, nrec=10)
    obs, g_o, _, s2, _ = _oracle_exact(p)
    f64 = torch.float64
    c, w, o = to_dev(p.c, f64), to_dev(p.wavelet, f64), to_dev(obs, f64)
    say("exact vs +/-k average")
    g_ex, _ = fdw.fd_adjoint_exact(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, o)
    k = 0.02
    g_p, _ = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, o, k)
    g_m, _ = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, o, -k)
    g_ex, g_p, g_m = (t.cpu().numpy() for t in (g_ex, g_p, g_m))
    assert rel(0.5 * (g_p + g_m), g_ex) < 1e-9
    gap = g_p - g_ex
    want = k * s2 / p.c ** 3
    assert rel(gap, want) < 1e-6
    assert gap.min() >= -1e-9 * np.abs(g_ex).max()


def test_exact_edge_cases(fdw):
    """One step (only the terminal interval), no receivers (zero gradient and J), a
    variant that cannot carry two fields (rejected), k-free signature."""
    p = wl.small_random((12, 10, 64), order=8, nt=1, dtype="f64", seed=5)
    obs, g_o, J_o, _, _ = _oracle_exact(p)
    say("exact nt=1")
    g, J, _ = _run_exact(fdw, p, obs, torch.float64)
    assert abs(J - J_o) <= 1e-12 * max(J_o, 1e-300)
    assert rel(g, g_o) < 1e-12

    p0 = wl.small_random((12, 10, 64), order=8, nt=20, dtype="f64", seed=6, nrec=0)
    f64 = torch.float64
    say("exact no receivers")
    g0, J0 = fdw.fd_adjoint_exact(to_dev(p0.c, f64), 1.0, 8, p0.src, to_dev(p0.wavelet, f64),
                                  p0.rec, p0.dt, p0.nt, torch.zeros((20, 0), dtype=f64, device="cuda"))
    assert J0 == 0.0 and float(g0.abs().max()) == 0.0

    p3 = wl.small_random((12, 10, 64), order=8, nt=5, dtype="f32", seed=8)
    one_field = [v for v in range(1, fdw.lib().fd_variant_count(3) + 1)
                 if fdw.fd_variant_info(3, v)["max_fields"] < 2]
    assert one_field
    with pytest.raises(fdw.FdError) as e:
        _run_exact(fdw, p3, np.zeros((5, len(p3.rec))), torch.float32, variant=one_field[0])
    assert e.value.code == fdw.FD_E_ARG


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle reference not generated")
def test_exact_256_cubed(fdw):
    """256^3, f32, order 8, nt = 2000: the re-simulated exact gradient against the
    oracle's checkpointed exact adjoint on the sampled cells."""
    ref = np.load(GOLDEN)
    s = (slice(None, None, int(ref["stride"])),) * 3
    p = wl.smooth_3d(n=256, nt=2000)
    f32 = torch.float32
    say("exact 256^3 f32")
    g, J = fdw.fd_adjoint_exact(to_dev(p.c, f32), p.dx, p.order, p.src, to_dev(p.wavelet, f32), p.rec,
                                p.dt, p.nt, to_dev(p.observed, f32))
    e = rel(g[s].double().cpu().numpy(), ref["exact_sample"])
    say(f"  J {J:.9e} (oracle {float(ref['J']):.9e}); exact vs oracle exact {e:.3e}")
    assert abs(J - float(ref["J"])) < 1e-4 * float(ref["J"])
    assert e < 1e-4
