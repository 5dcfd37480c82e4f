"""Gradient-based design on the device (fd_design_map, fd_design_adjoint, fd_adam_step
and the loop in paper_2509_15744_amd/design.py) against the oracle's design chain
(oracle/design.py) and its variable-material Alg. 1 (oracle/vdoracle.c).

Tolerances: map and chain rule f64 1e-13 relative L2 (f32 2e-6); Adam f64 1e-14
absolute (f32 1e-6); design loops (f64) 1e-9 on the design field after each
iteration and 1e-12 on the objective.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import design as od
from helpers import rel, say, to_dev

pytestmark = pytest.mark.gpu

TATO = (1.204, 2643.0, 1.419e5, 6.87e8)   # rho1, rho2, kappa1, kappa2 (air, solid)


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def _box(origin, extent):
    return tuple(slice(o, o + e) for o, e in zip(origin, extent))


CASES = [
    # shape, origin, extent, rf, beta, eta, lo, hi, material
    ((37, 130), (5, 17), (23, 70), 1.5, 2.0, 0.5, 0.0, 1.0, "two"),
    ((29, 40), (0, 0), (29, 40), 3.2, 8.0, 0.4, 0.1, 0.9, "rho"),        # box = grid, clipping
    ((14, 11, 70), (2, 3, 5), (9, 6, 41), 2.2, 1.0, 0.5, 0.0, 1.0, "two"),
    ((20, 33), (4, 1), (7, 31), 0.0, 0.0, 0.5, 1e-5, 1.0, "rho"),        # FWI form: no filter, no projection
    ((6, 5, 9), (1, 0, 2), (5, 5, 1), 1.5, 3.0, 0.5, 0.0, 1.0, "two"),   # one-cell-thin box
    ((40, 50), (3, 4), (30, 40), 12.0, 2.0, 0.5, 0.0, 1.0, "two"),       # the appendix's radius 12
]


def _material(name, fdw=None):
    mod = fdw if fdw is not None else od
    return mod.two_material(*TATO) if name == "two" else mod.rho_scaling(2700.0, 6000.0)


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_design_map_and_adjoint_match_oracle(fdw, case, dtype):
    shape, origin, extent, rf, beta, eta, lo, hi, mat = CASES[case]
    rng = np.random.default_rng(10 + case)
    gamma = -0.2 + 1.4 * rng.random(extent)
    material = _material(mat)
    box = _box(origin, extent)
    g_o, m_o, b_o = od.design_map(gamma, rf, beta, eta, lo, hi, material)
    gm = rng.standard_normal(shape) / abs(material[1])
    gb = rng.standard_normal(shape) / abs(material[3])
    grad_o = od.design_adjoint(gamma, rf, beta, eta, lo, hi, material, gm[box], gb[box])

    code = fdw.FD_F64 if dtype == torch.float64 else fdw.FD_F32
    d = fdw.make_design(shape, origin, extent, code, fdw.two_material(*TATO) if mat == "two"
                        else fdw.rho_scaling(2700.0, 6000.0), rf, beta, eta, lo, hi)
    m0 = rng.random(shape)
    m = to_dev(m0, dtype)
    b = to_dev(m0 + 1.0, dtype)
    gd = to_dev(gamma, dtype)
    gbar = torch.empty_like(gd)
    say("design map", case, dtype)
    fdw.fd_design_map(d, gd, m, b, gbar)
    grad = fdw.fd_design_adjoint(d, gd, to_dev(gm, dtype), to_dev(gb, dtype))
    torch.cuda.synchronize()
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    mh, bh = m.double().cpu().numpy(), b.double().cpu().numpy()
    assert rel(gbar.double().cpu().numpy(), g_o) < tol
    assert rel(mh[box], m_o) < tol and rel(bh[box], b_o) < tol
    outside = np.ones(shape, dtype=bool)
    outside[box] = False
    m_in = torch.as_tensor(m0, dtype=dtype).double().numpy()
    b_in = torch.as_tensor(m0 + 1.0, dtype=dtype).double().numpy()
    assert np.array_equal(mh[outside], m_in[outside]) and np.array_equal(bh[outside], b_in[outside])
    assert rel(grad.double().cpu().numpy(), grad_o) < (1e-12 if dtype == torch.float64 else 2e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_adam_matches_oracle(fdw, dtype):
    rng = np.random.default_rng(20)
    n = 3000
    x = rng.random(n)
    xs, m1, m2 = x.copy(), np.zeros(n), np.zeros(n)
    xd = to_dev(x, dtype)
    m1d, m2d = torch.zeros_like(xd), torch.zeros_like(xd)
    say("adam", dtype)
    for t in range(1, 6):
        g = rng.standard_normal(n) * 10.0 ** rng.uniform(-10, 2, n)
        xs, m1, m2 = od.adam(xs, g, m1, m2, t, lr=0.05, beta1=0.9, beta2=0.99, eps=1e-8, lo=0.0, hi=1.0)
        fdw.fd_adam_step(xd, to_dev(g, dtype), m1d, m2d, t, 0.05, 0.9, 0.99, 1e-8, 0.0, 1.0)
    out = xd.double().cpu().numpy()
    assert np.abs(out - xs).max() < (1e-14 if dtype == torch.float64 else 1e-6)
    assert out.min() >= 0.0 and out.max() <= 1.0 and (out == 0.0).any()


def _sine_burst(nt, dt, freq, cycles, amp):
    t = np.arange(nt) * dt
    w = 2 * np.pi * freq
    s = amp * np.sin(w * t) * np.sin(w * t / (2 * cycles)) ** 2
    s[t > 2 * np.pi * cycles / w] = 0.0
    return s.reshape(nt, 1)


def _tato(fdw):
    """A small acoustic-black-hole set-up (Eq. wavetopopt materials, 20 cells per
    wavelength in air at 5 kHz as in the paper's example): air background, a design
    box between the source and the region whose time-integrated u^2 is the objective."""
    from paper_2509_15744_amd import design as dz
    shape, dx = (48, 96), 1.0 / 300.0
    origin, extent = (8, 30), (32, 24)
    r_origin, r_extent = (18, 75), (12, 10)
    mat = od.two_material(*TATO)
    dmat = fdw.two_material(*TATO)
    dt = dz.stable_dt(dmat, 0.0, 1.0, dx, 2)
    nt = 300
    src = np.array([24 * shape[1] + 10], dtype=np.int64)
    w = _sine_burst(nt, dt, 5000.0, 2, 100.0)
    rec = dz.region_receivers(shape, r_origin, r_extent)
    return dict(shape=shape, dx=dx, origin=origin, extent=extent, mat=mat, dmat=dmat, dt=dt, nt=nt, src=src, w=w,
                rec=rec, scale=dz.region_scale(len(rec)), oscale=2.0 / (r_extent[0] * r_extent[1]), rf=1.5,
                beta=1.0, eta=0.5, lo=0.0, hi=1.0, obs=None, background=(1 / TATO[2], 1 / TATO[0]))


def _fwi(fdw):
    """A small full-waveform-inversion set-up (rho-scaling, Eq. scalarwaveequation;
    gamma in [1e-5, 1] on the whole grid, no filter or projection): observed traces of
    a medium with a void, the design starting from the homogeneous medium."""
    from paper_2509_15744_amd import design as dz
    shape, dx = (40, 64), 8e-5
    mat = od.rho_scaling(2700.0, 6000.0)
    dmat = fdw.rho_scaling(2700.0, 6000.0)
    dt = dz.stable_dt(dmat, 1e-5, 1.0, dx, 2)
    nt = 260
    src = np.array([0 * shape[1] + 32], dtype=np.int64)
    w = _sine_burst(nt, dt, 6000.0 / (25 * dx), 2, 1e12)
    rec = np.concatenate([np.arange(0, shape[1], 4), (shape[0] - 1) * shape[1] + np.arange(0, shape[1], 4)])
    true = np.ones(shape)
    true[15:24, 24:36] = 1e-5
    tr, _, _ = oracle.vd_forward(true * 2700.0, true * 2700.0 * 6000.0 ** 2, dx, dt, nt, src, w, rec)
    return dict(shape=shape, dx=dx, origin=(0, 0), extent=shape, mat=mat, dmat=dmat, dt=dt, nt=nt, src=src, w=w,
                rec=rec, scale=1.0, oscale=1.0, rf=0.0, beta=0.0, eta=0.5, lo=1e-5, hi=1.0, obs=tr,
                background=(0.0, 0.0))


def _fwi3d(fdw):
    """The 3D FWI form on a small grid: rho-scaling on the whole grid, a void ball in the
    true medium, receivers on the top and bottom faces."""
    from paper_2509_15744_amd import design as dz
    shape, dx = (16, 14, 20), 1e-4
    mat = od.rho_scaling(2700.0, 6000.0)
    dmat = fdw.rho_scaling(2700.0, 6000.0)
    dt = dz.stable_dt(dmat, 1e-5, 1.0, dx, 3)
    nt = 120
    src = np.array([7 * shape[2] + 10], dtype=np.int64)
    w = _sine_burst(nt, dt, 6000.0 / (12 * dx), 2, 1e12)
    face = [(a * shape[1] + i) * shape[2] + j for a in (0, shape[0] - 1)
            for i in range(0, shape[1], 2) for j in range(0, shape[2], 2)]
    rec = np.array(face, dtype=np.int64)
    x, y, z = np.indices(shape)
    true = np.ones(shape)
    true[(x - 9) ** 2 + (y - 6) ** 2 + (z - 9) ** 2 <= 9] = 1e-5
    tr, _, _ = oracle.vd_forward(true * 2700.0, true * 2700.0 * 6000.0 ** 2, dx, dt, nt, src, w, rec)
    return dict(shape=shape, dx=dx, origin=(0, 0, 0), extent=shape, mat=mat, dmat=dmat, dt=dt, nt=nt, src=src,
                w=w, rec=rec, scale=1.0, oscale=1.0, rf=0.0, beta=0.0, eta=0.5, lo=1e-5, hi=1.0, obs=tr,
                background=(0.0, 0.0))


def _oracle_loop(p, gamma0, k, iters, lr):
    shape, box = p["shape"], _box(p["origin"], p["extent"])
    obs = p["obs"] if p["obs"] is not None else np.zeros((p["nt"], len(p["rec"])))
    gamma = gamma0.copy()
    m1, m2 = np.zeros_like(gamma), np.zeros_like(gamma)
    out = []
    for t in range(1, iters + 1):
        _, mb, bb = od.design_map(gamma, p["rf"], p["beta"], p["eta"], p["lo"], p["hi"], p["mat"])
        m = np.full(shape, p["background"][0])
        b = np.full(shape, p["background"][1])
        m[box], b[box] = mb, bb
        gm, gb, J, _ = oracle.vd_superposition_gradient(m, b, p["dx"], p["dt"], p["nt"], p["src"], p["w"],
                                                        p["rec"], obs, k)
        grad = od.design_adjoint(gamma, p["rf"], p["beta"], p["eta"], p["lo"], p["hi"], p["mat"],
                                 p["oscale"] * gm[box], p["oscale"] * gb[box])
        gamma, m1, m2 = od.adam(gamma, grad, m1, m2, t, lr=lr, lo=p["lo"], hi=p["hi"])
        out.append((p["oscale"] * J, gamma.copy()))
    return out


@pytest.mark.parametrize("setup", ["tato", "fwi", "fwi3d"])
def test_design_loop_matches_oracle_loop(fdw, setup):
    """Three Adam iterations of the device loop equal the same loop built from the
    oracle's pieces at the same k (f64): objective and design field after each."""
    from paper_2509_15744_amd import design as dz
    p = {"tato": _tato, "fwi": _fwi, "fwi3d": _fwi3d}[setup](fdw)
    rng = np.random.default_rng(30)
    gamma0 = (0.5 + 0.1 * rng.standard_normal(p["extent"])).clip(0, 1) if setup == "tato" else np.ones(p["extent"])
    f64 = torch.float64
    m = torch.full(p["shape"], p["background"][0], dtype=f64, device="cuda")
    b = torch.full(p["shape"], p["background"][1], dtype=f64, device="cuda")
    obs = p["obs"] if p["obs"] is not None else np.zeros((p["nt"], len(p["rec"])))
    d = fdw.make_design(p["shape"], p["origin"], p["extent"], fdw.FD_F64, p["dmat"], p["rf"], p["beta"],
                        p["eta"], p["lo"], p["hi"])
    prob = dz.DesignProblem(design=d, m=m, b=b, dx=p["dx"], src=p["src"], wavelet=to_dev(p["w"], f64),
                            rec=p["rec"], observed=to_dev(obs, f64), dt=p["dt"], nt=p["nt"], scale=p["scale"])
    lr = 0.05 if setup == "tato" else 0.02
    loop = dz.AdamDesign(prob, to_dev(gamma0, f64), lr=lr, lo=p["lo"], hi=p["hi"])
    say("design loop", setup)
    got = [(loop.step(), loop.gamma.cpu().numpy().copy()) for _ in range(3)]
    ref = _oracle_loop(p, gamma0, loop.k, 3, lr)
    for (C, g), (Co, go) in zip(got, ref):
        assert abs(C - Co) <= 1e-12 * abs(Co)
        assert rel(g, go) < 1e-9
    assert np.abs(got[-1][1] - gamma0).max() > 0.01     # the design moved


def test_design_loop_reduces_region_energy(fdw):
    """Suppression (the paper's first design goal): six iterations from a grey design
    lower the region objective; beta-continuation raised beta after five."""
    from paper_2509_15744_amd import design as dz
    p = _tato(fdw)
    f64 = torch.float64
    m = torch.full(p["shape"], p["background"][0], dtype=f64, device="cuda")
    b = torch.full(p["shape"], p["background"][1], dtype=f64, device="cuda")
    d = fdw.make_design(p["shape"], p["origin"], p["extent"], fdw.FD_F64, p["dmat"], p["rf"], p["beta"],
                        p["eta"], p["lo"], p["hi"])
    prob = dz.DesignProblem(design=d, m=m, b=b, dx=p["dx"], src=p["src"], wavelet=to_dev(p["w"], f64),
                            rec=p["rec"], observed=torch.zeros((p["nt"], len(p["rec"])), dtype=f64, device="cuda"),
                            dt=p["dt"], nt=p["nt"], scale=p["scale"])
    loop = dz.AdamDesign(prob, torch.full(p["extent"], 0.5, dtype=f64, device="cuda"), lr=0.1)
    say("design loop descent")
    hist = [loop.step() for _ in range(6)]
    assert hist[-1] < hist[0], hist
    assert math.isclose(d.beta, 1.1)
    g = loop.gamma.cpu().numpy()
    assert g.min() >= 0.0 and g.max() <= 1.0


def test_design_error_paths(fdw):
    f64 = torch.float64
    m = torch.ones((10, 12), dtype=f64, device="cuda")
    gam = torch.ones((4, 4), dtype=f64, device="cuda")
    bad = [
        fdw.make_design((10, 12), (8, 0), (4, 4), fdw.FD_F64, (0, 1, 0, 1)),               # box outside
        fdw.make_design((10, 12), (0, 0), (4, 4), fdw.FD_F64, (0, 1, 0, 1), 40.0),         # radius
        fdw.make_design((10, 12), (0, 0), (4, 4), fdw.FD_F64, (0, 1, 0, 1), 1.5, 2.0, 1.5),  # eta
        fdw.make_design((10, 12), (0, 0), (4, 4), fdw.FD_F64, (0, 1, 0, 1), lo=1.0, hi=0.0),
        fdw.make_design((10, 12), (0, 0), (4, 4), fdw.FD_F64, (0, float("nan"), 0, 1)),
    ]
    for d in bad:
        with pytest.raises(fdw.FdError) as e:
            fdw.fd_design_map(d, gam, m, m.clone())
        assert e.value.code == fdw.FD_E_ARG
    small = torch.ones((3, 4), dtype=f64, device="cuda")
    ok = fdw.make_design((10, 12), (0, 0), (4, 4), fdw.FD_F64, (0, 1, 0, 1))
    with pytest.raises(ValueError):                 # gamma smaller than the box
        fdw.fd_design_map(ok, small, m, m.clone())
    x = torch.zeros(8, dtype=f64, device="cuda")
    for kw in (dict(step=0), dict(beta1=1.0), dict(eps=-1.0)):
        args = dict(step=1, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8)
        args.update(kw)
        with pytest.raises(fdw.FdError):
            fdw.fd_adam_step(x, x, x.clone(), x.clone(), args["step"], args["lr"], args["beta1"], args["beta2"],
                             args["eps"])


def test_design_loop_amplifies_with_negative_scale(fdw):
    """The amplifying design (the paper's second example, signs of Eqs. cost2 and
    adjointSource2 inverted): a negative scale makes the loop raise the region energy."""
    from paper_2509_15744_amd import design as dz
    p = _tato(fdw)
    f64 = torch.float64
    m = torch.full(p["shape"], p["background"][0], dtype=f64, device="cuda")
    b = torch.full(p["shape"], p["background"][1], dtype=f64, device="cuda")
    d = fdw.make_design(p["shape"], p["origin"], p["extent"], fdw.FD_F64, p["dmat"], p["rf"], p["beta"],
                        p["eta"], p["lo"], p["hi"])
    prob = dz.DesignProblem(design=d, m=m, b=b, dx=p["dx"], src=p["src"], wavelet=to_dev(p["w"], f64),
                            rec=p["rec"], observed=torch.zeros((p["nt"], len(p["rec"])), dtype=f64, device="cuda"),
                            dt=p["dt"], nt=p["nt"], scale=dz.region_scale(len(p["rec"]), maximize=True))
    loop = dz.AdamDesign(prob, torch.full(p["extent"], 0.5, dtype=f64, device="cuda"), lr=0.1)
    say("design loop ascent")
    hist = [loop.step() for _ in range(5)]
    assert all(h < 0 for h in hist)
    assert hist[-1] < hist[0], hist        # -C decreases: the region energy grows
