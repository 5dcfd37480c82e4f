"""Parity at the full benchmark sizes, in the launch configuration the benchmark uses
(library-chosen shape): 1024^3 layered (order 8, f32, 16384 receivers), 2048^2
layered (order 8, f32, 512 receivers) and the 1024^3 layered material of the
variable-material scheme (order 2, f32, 16384 receivers, both sensitivities).

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


def _window_check(shape, src, rec, wavelet, dt, r, centre, half, run_gpu, run_oracle):
    """Full-size run of nt = NT steps (``run_gpu(w, obs)`` -> (gradient fields, J, traces),
    device tensors) vs the oracle on the window around ``centre`` (``run_oracle(win,
    src_w, w_w, rec_w, obs_w)`` -> (gradient fields, J, traces) on the window)."""
    nd = len(shape)
    rng = np.random.default_rng(7)
    obs = 1e-3 * rng.standard_normal((NT, len(rec)))
    w = wavelet[:NT]
    grads, J, tr = run_gpu(w, obs)
    torch.cuda.synchronize()
    reach = 2 * r * NT
    lo = [max(0, centre[a] - half) for a in range(nd)]
    hi = [min(shape[a], centre[a] + half + 1) for a in range(nd)]
    win = tuple(slice(lo[a], hi[a]) for a in range(nd))
    wshape = tuple(hi[a] - lo[a] for a in range(nd))

    def inside(cells):
        co = np.array(np.unravel_index(cells, shape)).T
        m = np.all([(co[:, a] >= lo[a]) & (co[:, a] < hi[a]) for a in range(nd)], axis=0)
        return m, co - np.array(lo)

    ms, cs = inside(src)
    mr, cr = inside(rec)
    grads_o, J_o, tr_o = run_oracle(win, wl.flat(wshape, cs[ms]), w[:, ms], wl.flat(wshape, cr[mr]),
                                    obs[:, mr])
    # cells whose domain of dependence stays inside the window
    core = []
    for a in range(nd):
        a0 = lo[a] if lo[a] == 0 else lo[a] + reach
        a1 = hi[a] if hi[a] == shape[a] else hi[a] - reach
        core.append(slice(a0 - lo[a], a1 - lo[a]))
    core = tuple(core)
    errs = [rel(g[win].double().cpu().numpy()[core], go[core]) for g, go in zip(grads, grads_o)]
    # receivers in the core: traces
    rx = np.array(np.unravel_index(rec, shape)).T
    rec_core = mr & np.all([(rx[:, a] >= lo[a] + core[a].start) & (rx[:, a] < lo[a] + core[a].stop)
                            for a in range(nd)], axis=0)
    idx_in_win = np.cumsum(mr) - 1
    tr_gpu = tr.double().cpu().numpy()
    e_tr = rel(tr_gpu[:, rec_core], tr_o[:, idx_in_win[rec_core]])
    # far receivers: exact zeros
    sx = np.array(np.unravel_index(src, shape)).T
    dist = np.min(np.abs(rx[:, None, :] - sx[None, :, :]).max(axis=2), axis=1)
    far = dist > r * NT
    J_far = 0.5 * dt * float(np.sum(obs[:, far] ** 2))
    J_near = 0.5 * dt * float(np.sum((tr_o[:, idx_in_win[~far]] - obs[:, ~far]) ** 2))
    say(f"  window {wshape}: gradient core {', '.join(f'{e:.2e}' for e in errs)} "
        f"({int(np.prod([s.stop - s.start for s in core]))} cells), traces {e_tr:.2e} "
        f"({int(rec_core.sum())} receivers), far receivers {int(far.sum())}")
    assert np.all(~far <= mr), "every receiver near the source must lie in the window"
    assert max(errs) < 1e-4 and e_tr < 1e-4
    assert np.all(tr_gpu[:, far] == 0.0)
    assert abs(J - (J_far + J_near)) < 1e-5 * J
    return grads


def _constant_density(fdw, p, c_dev, centre, half, k):
    f32 = torch.float32

    def run_gpu(w, obs):
        tr = torch.empty((NT, len(p.rec)), dtype=f32, device="cuda")
        g, J = fdw.fd_adjoint_sensitivity(c_dev, p.dx, p.order, p.src, to_dev(w, f32), p.rec, p.dt, NT,
                                          to_dev(obs, f32), k, traces=tr)
        return (g,), J, tr

    def run_oracle(win, src_w, w_w, rec_w, obs_w):
        cw = c_dev[win].double().cpu().numpy()
        g, J, tr = oracle.superposition_gradient(cw, p.dx, p.order, p.dt, NT, src_w, w_w, rec_w, obs_w, k)
        return (g,), J, tr

    return _window_check(p.shape, p.src, p.rec, p.wavelet, p.dt, p.order // 2, centre, half,
                         run_gpu, run_oracle)[0]


def test_fullsize_3d_sampled_parity(fdw):
    p = wl.layered_3d(n=1024, nt=NT, device="cuda")
    c = p.c.float().contiguous()
    say("1024^3 layered, nt", NT)
    g = _constant_density(fdw, p, c, (0, 512, 512), 64, k=0.5)
    # far from every source and receiver the gradient is exactly zero
    assert torch.count_nonzero(g[600:]).item() == 0


def test_fullsize_2d_sampled_parity(fdw):
    p = wl.layered_2d(n=2048, nt=NT)
    c = torch.as_tensor(p.c, dtype=torch.float32, device="cuda")
    say("2048^2 layered, nt", NT)
    _constant_density(fdw, p, c, (0, 1024), 96, k=0.5)


def test_fullsize_vd_sampled_parity(fdw):
    """The variable-material second-order scheme on the 1024^3 layered material of the
    vd3d benchmark (f32, the library's launch shape): both sensitivities and the traces
    on the window core against the oracle's vdoracle.c."""
    q = wl.layered_material_3d(n=1024, nt=NT, device="cuda")
    del q["m_ref"], q["b_ref"]
    f32 = torch.float32
    k = 0.5

    def run_gpu(w, obs):
        tr = torch.empty((NT, len(q["rec"])), dtype=f32, device="cuda")
        gm, gb, J = fdw.fd_vd_adjoint_sensitivity(q["m"], q["b"], q["dx"], q["src"], to_dev(w, f32), q["rec"],
                                                  q["dt"], NT, to_dev(obs, f32), k, traces=tr)
        return (gm, gb), J, tr

    def run_oracle(win, src_w, w_w, rec_w, obs_w):
        mw = q["m"][win].double().cpu().numpy()
        bw = q["b"][win].double().cpu().numpy()
        gm, gb, J, tr = oracle.vd_superposition_gradient(mw, bw, q["dx"], q["dt"], NT, src_w, w_w, rec_w,
                                                         obs_w, k)
        return (gm, gb), J, tr

    say("1024^3 variable material, nt", NT)
    gm, gb = _window_check(q["shape"], q["src"], q["rec"], q["wavelet"], q["dt"], 1, (0, 512, 512), 48,
                           run_gpu, run_oracle)
    assert torch.count_nonzero(gm[200:]).item() == 0 and torch.count_nonzero(gb[200:]).item() == 0


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
