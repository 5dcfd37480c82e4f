"""Parity at the full benchmark sizes, in the launch configuration the benchmark uses
(library-chosen shape, variant 0): 1024^3 layered (order 8, f32, 16384 receivers) and
2048^2 layered (order 8, f32, 512 receivers).

The oracle cannot run these grids for thousands of steps, so:

* a few steps (nt = 4) of the full sensitivity are compared on sampled cells: the
  oracle runs on a window around the samples that keeps the true walls and reaches
  farther than the domain of dependence (2 r nt cells: nt forward and nt - 1 backward
  steps), so the window's cut edges cannot reach the samples;
* the wavefield is exactly zero beyond r nt cells of the source, so far receivers
  record exact zeros and contribute exactly (dt/2) obs^2 to J;
* the exact standing wave holds at full size over hundreds of steps.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2509_15744_amd import workloads as wl
from helpers import rel, say, to_dev

pytestmark = pytest.mark.gpu
NT = 4


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def _window_check(fdw, p, c_dev, centre, half, k):
    """Full-size run of nt = NT steps vs the oracle on the window around ``centre``."""
    shape = p.shape
    nd = len(shape)
    rng = np.random.default_rng(7)
    obs = 1e-3 * rng.standard_normal((NT, len(p.rec)))
    w = p.wavelet[:NT]
    f32 = torch.float32
    tr = torch.empty((NT, len(p.rec)), dtype=f32, device="cuda")
    g, J = fdw.fd_adjoint_sensitivity(c_dev, p.dx, p.order, p.src, to_dev(w, f32), p.rec, p.dt, NT,
                                      to_dev(obs, f32), k, traces=tr)
    torch.cuda.synchronize()
    r = p.order // 2
    reach = 2 * r * NT
    lo = [max(0, centre[a] - half) for a in range(nd)]
    hi = [min(shape[a], centre[a] + half + 1) for a in range(nd)]
    win = tuple(slice(lo[a], hi[a]) for a in range(nd))
    cw = c_dev[win].double().cpu().numpy()
    wshape = cw.shape

    def inside(cells):
        co = np.array(np.unravel_index(cells, shape)).T
        m = np.all([(co[:, a] >= lo[a]) & (co[:, a] < hi[a]) for a in range(nd)], axis=0)
        return m, co - np.array(lo)

    ms, cs = inside(p.src)
    mr, cr = inside(p.rec)
    g_o, J_o, tr_o = oracle.superposition_gradient(
        cw, p.dx, p.order, p.dt, NT, wl.flat(wshape, cs[ms]), w[:, ms], wl.flat(wshape, cr[mr]),
        obs[:, mr], k)
    # cells whose domain of dependence stays inside the window
    core = []
    for a in range(nd):
        a0 = lo[a] if lo[a] == 0 else lo[a] + reach
        a1 = hi[a] if hi[a] == shape[a] else hi[a] - reach
        core.append(slice(a0 - lo[a], a1 - lo[a]))
    core = tuple(core)
    g_gpu = g[win].double().cpu().numpy()
    e_g = rel(g_gpu[core], g_o[core])
    # receivers in the core: traces
    rec_core = mr & np.all([(np.array(np.unravel_index(p.rec, shape)).T[:, a] >= lo[a] + core[a].start)
                            & (np.array(np.unravel_index(p.rec, shape)).T[:, a] < lo[a] + core[a].stop)
                            for a in range(nd)], axis=0)
    idx_in_win = np.cumsum(mr) - 1
    tr_gpu = tr.double().cpu().numpy()
    e_tr = rel(tr_gpu[:, rec_core], tr_o[:, idx_in_win[rec_core]])
    # far receivers: exact zeros
    sx = np.array(np.unravel_index(p.src, shape)).T
    rx = np.array(np.unravel_index(p.rec, shape)).T
    dist = np.min(np.abs(rx[:, None, :] - sx[None, :, :]).max(axis=2), axis=1)
    far = dist > r * NT
    J_far = 0.5 * p.dt * float(np.sum(obs[:, far] ** 2))
    J_near = 0.5 * p.dt * float(np.sum((tr_o[:, idx_in_win[~far]] - obs[:, ~far]) ** 2))
    say(f"  window {wshape}: grad core {e_g:.2e} ({int(np.prod([s.stop - s.start for s in core]))} cells), "
        f"traces {e_tr:.2e} ({int(rec_core.sum())} receivers), far receivers {int(far.sum())}")
    assert np.all(~far <= mr), "every receiver near the source must lie in the window"
    assert e_g < 1e-4 and e_tr < 1e-4
    assert np.all(tr_gpu[:, far] == 0.0)
    assert abs(J - (J_far + J_near)) < 1e-5 * J
    return g


def test_fullsize_3d_sampled_parity(fdw):
    p = wl.layered_3d(n=1024, nt=NT, device="cuda")
    c = p.c.float().contiguous()
    say("1024^3 layered, nt", NT)
    g = _window_check(fdw, p, c, (0, 512, 512), 64, k=0.5)
    # far from every source and receiver the gradient is exactly zero
    assert torch.count_nonzero(g[600:]).item() == 0


def test_fullsize_2d_sampled_parity(fdw):
    p = wl.layered_2d(n=2048, nt=NT)
    c = torch.as_tensor(p.c, dtype=torch.float32, device="cuda")
    say("2048^2 layered, nt", NT)
    _window_check(fdw, p, c, (0, 1024), 96, k=0.5)


@pytest.mark.parametrize("shape,modes,nsteps", [((1024, 1024, 1024), (3, 5, 2), 150),
                                                ((2048, 2048), (7, 4), 400)])
def test_fullsize_standing_wave(fdw, shape, modes, nsteps):
    """Exact standing wave at full size, through fd_propagate in the library's launch shape."""
    c0, order = 1.5, 8
    dt = 0.45 * oracle.cfl_limit(len(shape), order) / c0
    a = [8 / 5, -1 / 5, 8 / 315, -1 / 560]
    lam = sum(2.0 * sum(aj * (math.cos((j + 1) * math.pi * m / n) - 1.0) for j, aj in enumerate(a))
              for n, m in zip(shape, modes))
    cphi = 1.0 + 0.5 * dt * dt * c0 * c0 * lam
    phi = math.acos(cphi)
    f32 = torch.float32
    v = torch.ones(shape, dtype=f32, device="cuda")
    for ax, (n, m) in enumerate(zip(shape, modes)):
        s = [1] * len(shape)
        s[ax] = n
        v = v * torch.cos(math.pi * m / n * (torch.arange(n, device="cuda", dtype=torch.float64) + 0.5)).float().view(s)
    coef = torch.full(shape, dt * dt * c0 * c0, dtype=f32, device="cuda")
    up, uc = (cphi * v).contiguous(), v.clone()
    say("standing wave", shape, nsteps)
    fdw.fd_propagate(coef, up, uc, nsteps, 1.0, order)
    torch.cuda.synchronize()
    want = math.cos(nsteps * phi)
    err = float(torch.linalg.vector_norm((uc - want * v).double()) / torch.linalg.vector_norm(v.double()))
    say(f"  rel error {err:.2e}")
    assert err < 1e-4
