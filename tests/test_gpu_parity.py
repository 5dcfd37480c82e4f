"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, element by element
on seeded inputs that span several tiles with ragged tails, plus edge cases, closed
forms and error paths on the device.

Tolerances: f64 grids agree with the oracle to rounding (traces 1e-12, gradients
1e-9 relative L2, the gradient carrying the K(u,u) - K(v,v) cancellation); f32 grids
must agree within 1e-4 relative L2 on traces and on the sensitivity field at the same
k (the acceptance bound for runs of up to 4000 steps).
"""
import ctypes
import functools
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2509_15744_amd import workloads as wl
from helpers import OracleCase, rel, say, to_dev, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def run_sens(fdw, p, case, variant=0, acc_dtype=None, k=None):
    dt_ = torch_dtype(p.dtype)
    c = to_dev(p.c, dt_)
    w = to_dev(p.wavelet, dt_)
    obs = to_dev(case.obs, dt_)
    traces = torch.empty((p.nt, len(p.rec)), dtype=dt_, device="cuda")
    grad, J = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs,
                                         case.k if k is None else k, traces=traces,
                                         acc_dtype=acc_dtype, variant=variant)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), J, traces.cpu().numpy()


@functools.lru_cache(maxsize=None)
def inclusion_case():
    return OracleCase(wl.inclusion_2d(), gap=0.01)


def _layered_ragged():
    p = wl.layered_2d(n=300, nt=1500, seed=12, rec_every=3)
    # make the second axis ragged for every tile width: 300 x 270
    c = p.c[:, :270].copy()
    c_ref = p.c_ref[:, :270].copy()
    shape = c.shape
    rec = wl.flat(shape, [[0, 3 * q + 1] for q in range(90)])
    src = wl.flat(shape, [[0, 135]])
    return wl.Problem("layered2d-ragged", shape, 8, "f32", 1.0, p.dt, p.nt, c, c_ref, src, rec,
                      p.wavelet, meta=p.meta)


@functools.lru_cache(maxsize=None)
def layered_ragged_case():
    return OracleCase(_layered_ragged(), gap=0.02)


def _smooth3d_ragged():
    shape = (45, 38, 70)
    pn = wl.smooth_noise(shape, 6.0, 21)
    c = 1.0 + (pn - pn.min()) * (2.0 / (pn.max() - pn.min()))
    c_ref = np.full(shape, 2.0)
    rec = wl.flat(shape, [[0, a, b] for a in range(2, 38, 6) for b in range(1, 70, 5)])
    src = wl.flat(shape, [[0, 19, 35]])
    dt = 0.4 / 3.0
    return wl.Problem("smooth3d-ragged", shape, 8, "f32", 1.0, dt, 300, c, c_ref, src, rec,
                      wl.ricker(300, dt, 0.05).reshape(300, 1))


@functools.lru_cache(maxsize=None)
def smooth3d_case():
    return OracleCase(_smooth3d_ragged(), gap=0.02)


# ---------------------------------------------------------------------------
# parity on the workloads
# ---------------------------------------------------------------------------

def test_inclusion_fp64_parity(fdw):
    """128 x 128, f64, order 4, nt = 600, inclusion medium: traces, J and the
    sensitivity at the same k agree with the oracle to rounding; the gap to the
    exact stored-history adjoint is the closed-form k/c^3 sum (dmu)^2 (1%)."""
    case = inclusion_case()
    p = case.p
    say("inclusion fp64", p.shape, p.nt, "k", case.k)
    for variant in fdw.variants_for(p.shape):
        grad, J, traces = run_sens(fdw, p, case, variant=variant)
        assert rel(traces, case.traces) < 1e-12
        assert abs(J - case.J) < 1e-12 * case.J
        assert rel(grad, case.g_approx) < 1e-9
        gap = rel(grad, case.g_exact)
        assert abs(gap - 0.01) < 1e-6, gap


def test_layered2d_fp32_parity(fdw):
    """300 x 270 layered medium (ragged for every tile width), f32, order 8,
    nt = 1500, 90 receivers on the top row: traces and the sensitivity within 1e-4."""
    case = layered_ragged_case()
    p = case.p
    say("layered2d fp32", p.shape, p.nt, "k", case.k)
    grad, J, traces = run_sens(fdw, p, case)
    e_tr, e_g = rel(traces, case.traces), rel(grad, case.g_approx)
    say("  traces", e_tr, "grad", e_g, "J", J, case.J)
    assert e_tr < 1e-4
    assert abs(J - case.J) < 1e-4 * case.J
    assert e_g < 1e-4


def test_smooth3d_fp32_parity(fdw):
    """45 x 38 x 70 smooth medium (ragged on all axes), f32, order 8, nt = 300,
    a 6 x 14 receiver grid on the top face: traces and the sensitivity within 1e-4,
    for every 3D tile variant."""
    case = smooth3d_case()
    p = case.p
    for variant in fdw.variants_for(p.shape):
        say("smooth3d fp32 variant", variant, p.shape, p.nt)
        grad, J, traces = run_sens(fdw, p, case, variant=variant)
        e_tr, e_g = rel(traces, case.traces), rel(grad, case.g_approx)
        say("  traces", e_tr, "grad", e_g)
        assert e_tr < 1e-4
        assert e_g < 1e-4


@pytest.mark.parametrize("shape,order,nt,seed", [
    ((9, 11), 2, 37, 1),
    ((4, 4), 8, 25, 2),            # minimal extents: n = r
    ((5, 130), 4, 1, 3),           # a single step
    ((70, 66), 8, 2, 4),           # two steps
    ((6, 5, 4), 8, 30, 5),         # minimal 3D
    ((17, 9, 131), 4, 23, 6),
    ((33, 20, 65), 2, 19, 7),
    ((8, 71, 9), 8, 15, 8),
    ((12, 9, 132), 8, 21, 9),      # multiple of 4, ragged for 128- and 256-wide tiles
    ((20, 17, 68), 4, 17, 10),
    ((30, 260), 8, 25, 11),
    ((7, 6, 8), 8, 9, 12),         # narrower than every vector tile
])
def test_edge_cases_fp64(fdw, shape, order, nt, seed):
    """Random media, duplicate receivers, a receiver on a source cell, cells anywhere
    (walls and corners included), very short runs: f64 parity to rounding."""
    p = wl.small_random(shape, order=order, nt=nt, dtype="f64", seed=seed, nsrc=3, nrec=9)
    case = OracleCase(p, k=0.05)
    say("edge", shape, order, nt)
    for variant in fdw.variants_for(shape):
        grad, J, traces = run_sens(fdw, p, case, variant=variant)
        assert rel(traces, case.traces) < 1e-12
        assert abs(J - case.J) <= 1e-12 * max(case.J, 1e-300)
        assert rel(grad, case.g_approx) < 1e-9


def test_cells_on_every_wall_and_corner(fdw):
    """Sources and receivers on all eight corners and the centres of all six faces."""
    shape = (13, 10, 67)
    corners = [[a, b, c] for a in (0, 12) for b in (0, 9) for c in (0, 66)]
    faces = [[0, 5, 33], [12, 5, 33], [6, 0, 33], [6, 9, 33], [6, 5, 0], [6, 5, 66]]
    rng = np.random.default_rng(3)
    c = 1.0 + rng.random(shape)
    nt = 40
    dt = 0.4 * oracle.cfl_limit(3, 8) / c.max()
    p = wl.Problem("walls", shape, 8, "f64", 1.0, dt, nt, c, np.full(shape, 1.5),
                   wl.flat(shape, corners), wl.flat(shape, corners + faces),
                   rng.standard_normal((nt, 8)))
    case = OracleCase(p, k=0.1)
    say("walls and corners")
    grad, J, traces = run_sens(fdw, p, case)
    assert rel(traces, case.traces) < 1e-12
    assert rel(grad, case.g_approx) < 1e-9


@pytest.mark.parametrize("copies", [1, 3])
def test_dense_receiver_planes(fdw, copies):
    """Every cell of the first row is a receiver, `copies` times over, and several
    sources share it: with 3 copies a block's plane holds more events than the kernel
    stages in LDS (128), which takes the global-memory path; both paths match the
    oracle to rounding in every 2D variant."""
    shape = (26, 300)
    rng = np.random.default_rng(40 + copies)
    c = 1.0 + rng.random(shape)
    nt = 24
    dt = 0.4 * oracle.cfl_limit(2, 4) / c.max()
    row = [[0, j] for j in range(shape[1])]
    rec = wl.flat(shape, row * copies)
    src = wl.flat(shape, [[0, 7], [0, 7], [0, 150], [3, 299]])
    p = wl.Problem("dense", shape, 4, "f64", 1.0, dt, nt, c, np.full(shape, 1.5), src, rec,
                   rng.standard_normal((nt, len(src))))
    case = OracleCase(p, k=0.05)
    for variant in fdw.variants_for(shape):
        say("dense receiver plane, copies", copies, "variant", variant)
        grad, J, traces = run_sens(fdw, p, case, variant=variant)
        assert rel(traces, case.traces) < 1e-12
        assert abs(J - case.J) <= 1e-12 * case.J
        assert rel(grad, case.g_approx) < 1e-9


def test_variants_are_bitwise_identical(fdw):
    """The per-cell arithmetic does not depend on the tile shape."""
    p = wl.small_random((19, 23, 132), order=8, nt=20, dtype="f32", seed=9)
    case = OracleCase(p, k=0.05, exact=False)
    assert len(fdw.variants_for(p.shape)) == fdw.fd_variant_count(3)
    ref = None
    for variant in fdw.variants_for(p.shape):
        say("bitwise variant", variant)
        out = run_sens(fdw, p, case, variant=variant)
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[2], ref[2])
            assert out[1] == ref[1]


def test_second_launch_shape_is_bitwise_identical(fdw):
    """Launches that touch no accumulator may run another tile shape (variant_plain,
    chunk_plain): the per-cell arithmetic is the same, so the gradient, J and traces are
    bitwise those of a single launch shape."""
    p = wl.small_random((33, 20, 128), order=8, nt=30, dtype="f32", seed=17)
    case = OracleCase(p, k=0.05, exact=False)
    say("second launch shape")
    g1, J1, t1 = run_sens(fdw, p, case, variant=2)
    for vp, cp in ((7, 0), (3, 8), (6, 16), (1, 33)):
        dt_ = torch_dtype(p.dtype)
        tr = torch.empty((p.nt, len(p.rec)), dtype=dt_, device="cuda")
        g2, J2 = fdw.fd_adjoint_sensitivity(to_dev(p.c, dt_), p.dx, p.order, p.src, to_dev(p.wavelet, dt_), p.rec,
                                            p.dt, p.nt, to_dev(case.obs, dt_), case.k, traces=tr, variant=2,
                                            variant_plain=vp, chunk_plain=cp)
        assert J2 == J1 and np.array_equal(g2.cpu().numpy(), g1) and np.array_equal(tr.cpu().numpy(), t1)


def test_variant_needing_wider_rows_is_rejected(fdw):
    p = wl.small_random((10, 10, 70), order=4, nt=5, dtype="f32", seed=1)
    bad = [v for v in range(1, fdw.fd_variant_count(3) + 1)
           if 70 % fdw.fd_variant_info(3, v)["cells_per_lane"]]
    assert bad
    c, w = to_dev(p.c, torch.float32), to_dev(p.wavelet, torch.float32)
    with pytest.raises(fdw.FdError) as e:
        fdw.fd_forward(c, 1.0, 4, p.src, w, p.rec, p.dt, 5, variant=bad[0])
    assert e.value.code == fdw.FD_E_ARG and "multiple of" in str(e.value)


def test_chunking_is_bitwise_identical(fdw):
    """The axis-0 chunk length (planes per block) changes only the decomposition."""
    p = wl.small_random((37, 20, 70), order=8, nt=12, dtype="f32", seed=10)
    case = OracleCase(p, k=0.05, exact=False)
    dt_ = torch.float32
    c, w, obs = to_dev(p.c, dt_), to_dev(p.wavelet, dt_), to_dev(case.obs, dt_)
    ref = None
    for chunk in (0, 1, 5, 16, 37, 1000):
        say("chunk", chunk)
        st = fdw.SweepState(c, p.nt, len(p.rec))
        J = fdw.fd_sens_forward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, st,
                                chunk=chunk)
        g = fdw.fd_sens_backward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, case.k, st,
                                 chunk=chunk)
        out = (J, g.cpu().numpy())
        if ref is None:
            ref = out
            assert rel(out[1], case.g_approx) < 1e-4
        else:
            assert out[0] == ref[0] and np.array_equal(out[1], ref[1])


def test_timing_record(fdw):
    p = wl.small_random((16, 16, 64), order=8, nt=9, dtype="f32", seed=12)
    dt_ = torch.float32
    c, w = to_dev(p.c, dt_), to_dev(p.wavelet, dt_)
    obs = torch.zeros((p.nt, len(p.rec)), dtype=dt_, device="cuda")
    tf, tb = fdw.fd_timing(), fdw.fd_timing()
    st = fdw.SweepState(c, p.nt, len(p.rec))
    fdw.fd_sens_forward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, st, timing=tf)
    fdw.fd_sens_backward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, 0.1, st, timing=tb)
    assert tf.fwd_launches == 9 and tb.bwd_launches == 8
    assert tf.fwd_ms > 0 and tb.bwd_ms > 0


def test_runs_are_deterministic(fdw):
    p = _layered_ragged()
    dt_ = torch.float32
    c, w = to_dev(p.c, dt_), to_dev(p.wavelet, dt_)
    obs = torch.zeros((p.nt, len(p.rec)), dtype=dt_, device="cuda")
    say("determinism")
    g1, J1 = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, 0.01)
    g1 = g1.clone()
    g2, J2 = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, 0.01)
    assert J1 == J2
    assert torch.equal(g1, g2)


def test_split_sweeps_equal_fused_call(fdw):
    """fd_sens_forward + fd_sens_backward (the autograd pair) equals
    fd_adjoint_sensitivity bitwise, and grad_scale scales the result."""
    p = wl.small_random((40, 75), order=8, nt=50, dtype="f32", seed=11)
    case = OracleCase(p, k=0.05, exact=False)
    dt_ = torch.float32
    c, w, obs = to_dev(p.c, dt_), to_dev(p.wavelet, dt_), to_dev(case.obs, dt_)
    say("split sweeps")
    g_fused, J_fused = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt,
                                                  obs, case.k)
    st = fdw.SweepState(c, p.nt, len(p.rec))
    J = fdw.fd_sens_forward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, st)
    g = fdw.fd_sens_backward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, case.k, st, grad_scale=1.0)
    assert J == J_fused
    assert torch.equal(g, g_fused)
    st2 = fdw.SweepState(c, p.nt, len(p.rec))
    fdw.fd_sens_forward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, st2)
    g3 = fdw.fd_sens_backward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, case.k, st2, grad_scale=-2.5)
    assert torch.allclose(g3, -2.5 * g_fused, rtol=1e-6, atol=0)


def test_forward_and_misfit(fdw):
    """fd_forward traces and fd_misfit (J and residual) against the oracle."""
    p = wl.small_random((31, 5, 77), order=4, nt=60, dtype="f64", seed=13)
    traces_o, _, _ = oracle.forward(p.c, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec)
    obs = np.random.default_rng(1).standard_normal(traces_o.shape) * 1e-3
    J_o, res_o = oracle.misfit(traces_o, obs, p.dt)
    say("forward + misfit")
    dt_ = torch.float64
    tr = fdw.fd_forward(to_dev(p.c, dt_), p.dx, p.order, p.src, to_dev(p.wavelet, dt_), p.rec, p.dt, p.nt)
    res = torch.empty_like(tr)
    J = fdw.fd_misfit(tr, to_dev(obs, dt_), p.dt, residual=res)
    assert rel(tr.cpu().numpy(), traces_o) < 1e-12
    assert abs(J - J_o) < 1e-11 * J_o
    assert rel(res.cpu().numpy(), res_o) < 1e-11


def test_misfit_fp32_and_empty(fdw):
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal((333, 17)), rng.standard_normal((333, 17))
    J_o, _ = oracle.misfit(a.astype(np.float32), b.astype(np.float32), 0.3)
    J = fdw.fd_misfit(to_dev(a, torch.float32), to_dev(b, torch.float32), 0.3)
    assert abs(J - J_o) < 1e-6 * J_o         # differences rounded to f32, sums in f64
    z = torch.zeros((5, 0), dtype=torch.float32, device="cuda")
    assert fdw.fd_misfit(z, z, 0.3) == 0.0


# ---------------------------------------------------------------------------
# closed forms on the device
# ---------------------------------------------------------------------------

def _mode(shape, modes):
    v = np.ones(shape)
    for ax, (n, m) in enumerate(zip(shape, modes)):
        s = [1] * len(shape)
        s[ax] = n
        v = v * np.cos(math.pi * m / n * (np.arange(n) + 0.5)).reshape(s)
    return v


_A = {2: [1.0], 4: [4 / 3, -1 / 12], 8: [8 / 5, -1 / 5, 8 / 315, -1 / 560]}


def _lam(order, theta):
    a = _A[order]
    return 2.0 * sum(aj * (math.cos((j + 1) * theta) - 1.0) for j, aj in enumerate(a))


@pytest.mark.parametrize("shape,order,modes,dtype", [
    ((96, 70), 8, (5, 3), "f64"),
    ((30, 21, 67), 4, (2, 3, 5), "f64"),
    ((40, 33, 130), 8, (1, 4, 7), "f64"),
    ((256, 200), 8, (9, 4), "f32"),
    ((64, 48, 80), 8, (3, 2, 5), "f32"),
])
def test_standing_wave_on_device(fdw, shape, order, modes, dtype):
    """fd_propagate on the exact standing wave: u^n = cos(n phi) v."""
    dx, c0 = 1.0, 1.1
    dt = 0.45 * oracle.cfl_limit(len(shape), order) / c0
    v = _mode(shape, modes)
    lam = sum(_lam(order, math.pi * m / n) for n, m in zip(shape, modes))
    cphi = 1.0 + 0.5 * dt * dt * c0 * c0 * lam
    phi = math.acos(cphi)
    dt_ = torch_dtype(dtype)
    coef = torch.full(shape, dt * dt * c0 * c0, dtype=dt_, device="cuda")
    up, uc = to_dev(cphi * v, dt_), to_dev(v, dt_)
    nsteps = 301
    say("standing wave", shape, order, dtype)
    fdw.fd_propagate(coef, up, uc, nsteps, dx, order)
    tol = 1e-11 if dtype == "f64" else 1e-4
    assert rel(uc.cpu().numpy(), math.cos(nsteps * phi) * v) < tol
    assert rel(up.cpu().numpy(), math.cos((nsteps - 1) * phi) * v) < tol


# ---------------------------------------------------------------------------
# error paths on the device
# ---------------------------------------------------------------------------

def test_cfl_violation_is_rejected(fdw):
    p = wl.small_random((20, 20), order=8, nt=10, dtype="f32", seed=1)
    c = to_dev(p.c, torch.float32)
    w = to_dev(p.wavelet, torch.float32)
    dt_bad = 0.6 / float(p.c.max())          # Courant 0.6 > 0.5546
    with pytest.raises(fdw.FdError) as e:
        fdw.fd_forward(c, 1.0, 8, p.src, w, p.rec, dt_bad, 10)
    assert e.value.code == fdw.FD_E_CFL


def test_bad_speed_is_rejected(fdw):
    p = wl.small_random((20, 20), order=4, nt=10, dtype="f32", seed=1)
    w = to_dev(p.wavelet, torch.float32)
    for bad in (-1.0, 0.0, float("nan"), float("inf")):
        c = p.c.copy()
        c[3, 4] = bad
        with pytest.raises(fdw.FdError) as e:
            fdw.fd_forward(to_dev(c, torch.float32), 1.0, 4, p.src, w, p.rec, p.dt, 10)
        assert e.value.code == fdw.FD_E_NONFINITE


def test_host_and_undersized_buffers_are_rejected(fdw):
    p = wl.small_random((20, 20), order=4, nt=10, dtype="f32", seed=1)
    c = to_dev(p.c, torch.float32)
    w = to_dev(p.wavelet, torch.float32)
    g = fdw.make_grid(p.shape, 1.0, 4, fdw.FD_F32)
    acq = fdw.Acquisition(p.src, w, p.rec)
    host = np.zeros(400, dtype=np.float32)
    tr = torch.empty((10, len(p.rec)), dtype=torch.float32, device="cuda")
    rc = fdw.lib().fd_forward(ctypes.byref(g), ctypes.c_void_p(host.ctypes.data), ctypes.byref(acq.c),
                              p.dt, 10, ctypes.c_void_p(tr.data_ptr()), None, None)
    assert rc == fdw.FD_E_ARG and "not a device allocation" in fdw.lib().fd_last_error().decode()
    small = torch.empty(100, dtype=torch.float32, device="cuda")
    big_grid = fdw.make_grid((20000, 20000), 1.0, 4, fdw.FD_F32)
    rc = fdw.lib().fd_forward(ctypes.byref(big_grid), ctypes.c_void_p(small.data_ptr()),
                              ctypes.byref(fdw.fd_acq()), p.dt, 10, None, None, None)
    assert rc == fdw.FD_E_ARG and "smaller than required" in fdw.lib().fd_last_error().decode()
