"""Pins of the FP64 oracle to facts fixed outside it: textbook stencil weights,
exact discrete solutions, closed-form Green's functions, conservation laws,
operator symmetry, adjoint identities and brute-force finite differences.

Each test names the passage of the paper it pins and the mistake it would
catch.  None of them needs a GPU.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2509_15744_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _textbook_weights():
    out = {}
    with open(os.path.join(GOLDEN, "central_weights.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out[int(parts[0])] = [Fraction(p) for p in parts[1:]]
    return out


# ---------------------------------------------------------------------------
# stencil weights (paper Sec. 3.1, extended to order 2r)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("order", [2, 4, 8])
def test_weights_match_textbook_table(order):
    """Fornberg's recursion reproduces the published table exactly."""
    assert oracle.central_weights(order) == _textbook_weights()[order]


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12])
def test_weights_match_closed_form(order):
    """a_j = 2 (-1)^(j+1) (r!)^2 / (j^2 (r-j)! (r+j)!), a_0 = -2 sum a_j."""
    r = order // 2
    a = oracle.central_weights(order)
    for j in range(1, r + 1):
        cf = Fraction(2 * (-1) ** (j + 1) * math.factorial(r) ** 2,
                      j * j * math.factorial(r - j) * math.factorial(r + j))
        assert a[j] == cf
    assert a[0] == -2 * sum(a[1:])


def _half_sample_mode(shape, modes):
    v = np.ones(shape)
    for ax, (n, m) in enumerate(zip(shape, modes)):
        th = math.pi * m / n
        s = [1] * len(shape)
        s[ax] = n
        v = v * np.cos(th * (np.arange(n) + 0.5)).reshape(s)
    return v


def _symbol(order, theta):
    a = [float(x) for x in _textbook_weights()[order]]
    return a[0] + 2.0 * sum(a[j] * math.cos(j * theta) for j in range(1, len(a)))


@pytest.mark.parametrize("order", [2, 4, 8])
def test_stencil_accuracy_order(order):
    """The Rayleigh quotient of L on the wall-compatible cosine mode of wavenumber
    theta approaches -theta^2 with error ~ theta^(order+2): catches a wrong weight
    that keeps symmetry but loses accuracy."""
    n = 256
    errs, ths = [], []
    for m in (8, 16, 32):
        v = _half_sample_mode((n,), (m,))
        lv = oracle.laplacian(v, 1.0, order)
        lam = float(v @ lv / (v @ v))
        th = math.pi * m / n
        errs.append(abs(lam + th * th))
        ths.append(th)
    slopes = np.diff(np.log(errs)) / np.diff(np.log(ths))
    assert np.all(np.abs(slopes - (order + 2)) < 0.15), slopes


@pytest.mark.parametrize("shape,order,modes,dx", [
    ((64,), 2, (5,), 1.0),
    ((48, 40), 8, (7, 3), 0.5),
    ((20, 18, 16), 4, (2, 5, 3), 2.5),
    ((16, 12, 10), 8, (1, 0, 4), 1.0),
])
def test_standing_wave_is_exact(shape, order, modes, dx):
    """Homogeneous medium, initial levels cos(phi) v and v with v the half-sample
    cosine mode: the scheme gives u^n = cos(n phi) v exactly, 2 cos(phi) = 2 +
    dt^2 c^2 lambda.  Pins the weights, the mirror walls (a whole-sample mirror
    breaks the eigenvector), the leapfrog form and coef = dt^2 c^2."""
    c0 = 1.3
    dt = 0.45 * oracle.cfl_limit(len(shape), order) * dx / c0
    v = _half_sample_mode(shape, modes)
    lam = sum(_symbol(order, math.pi * m / n) for n, m in zip(shape, modes)) / dx ** 2
    cphi = 1.0 + 0.5 * dt * dt * c0 * c0 * lam
    phi = math.acos(cphi)
    coef = np.full(shape, dt * dt * c0 * c0)
    nsteps = 400
    up, uc = oracle.propagate(coef, cphi * v, v, nsteps, dx, order)
    assert np.abs(uc - math.cos(nsteps * phi) * v).max() < 1e-11
    assert np.abs(up - math.cos((nsteps - 1) * phi) * v).max() < 1e-11


def test_dalembert_courant_one():
    """1D, order 2, Courant number 1: the leapfrog reproduces d'Alembert's solution
    exactly, u^n_i = (G_{i-n} + G_{i+n}) / 2 with G the even extension of the
    initial pulse about the wall faces (paper Eq. BC)."""
    n = 120
    i = np.arange(n)
    g = np.exp(-0.5 * ((i - 30.0) / 4.0) ** 2) + 0.5 * np.exp(-0.5 * ((i - 90.0) / 3.0) ** 2)

    def G(x):
        x = np.mod(x, 2 * n)
        return g[np.where(x < n, x, 2 * n - 1 - x)]

    coef = np.ones(n)                       # c dt / dx = 1
    u_m1 = 0.5 * (G(i - 1) + G(i + 1))      # level -1 equals level 1: zero velocity
    steps = 700                             # several wall reflections
    up, uc = oracle.propagate(coef, u_m1, g, steps, 1.0, 2)
    exact = 0.5 * (G(i - steps) + G(i + steps))
    assert np.abs(uc - exact).max() < 1e-12


@pytest.mark.parametrize("shape,order", [((13,), 2), ((9, 11), 4), ((7, 6, 9), 8), ((8, 8), 8)])
def test_laplacian_is_symmetric(shape, order):
    """<L x, y> = <x, L y>: the mirror walls make L self-adjoint in the plain
    inner product, which the superposition method requires (paper Sec. 4)."""
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(shape), rng.standard_normal(shape)
    lx, ly = oracle.laplacian(x, 0.7, order), oracle.laplacian(y, 0.7, order)
    a, b = float(np.sum(lx * y)), float(np.sum(x * ly))
    assert abs(a - b) <= 1e-13 * max(abs(a), 1.0)
    assert abs(float(lx.sum())) < 1e-11 * np.abs(lx).sum()   # constants are in the kernel


def test_energy_is_conserved_source_free():
    """E^{n+1/2} = sum m (u^{n+1}-u^n)^2 / (2 dt^2) - (u^{n+1})^T L u^n / 2 is
    constant without sources in a heterogeneous medium (m = 1/c^2)."""
    rng = np.random.default_rng(2)
    shape, order, dx = (24, 20), 8, 1.0
    c = 1.0 + rng.random(shape)
    dt = 0.4 * dx / c.max()
    coef = dt * dt * c * c
    m = 1.0 / (c * c)
    u0 = wl.smooth_noise(shape, 2.0, 3)
    um = u0 * 0.99
    energies = []
    for _ in range(30):
        up, uc = oracle.propagate(coef, um, u0, 10, dx, order)
        e = np.sum(m * (uc - up) ** 2) / (2 * dt * dt) - 0.5 * np.sum(uc * oracle.laplacian(up, dx, order))
        energies.append(e)
        um, u0 = up, uc
    energies = np.array(energies)
    assert energies.min() > 0
    assert np.abs(energies - energies[0]).max() < 1e-12 * energies[0]


def test_energy_balance_with_source():
    """With a point force: E^{n+1/2} - E^{n-1/2} = (f^n)^T (u^{n+1} - u^{n-1}) / 2,
    f^n = wavelet[n] / dx^d at the source (paper Eq. source1).  Pins the source
    scaling coef * f against the operator."""
    shape, order, dx = (20, 22), 4, 0.8
    rng = np.random.default_rng(5)
    c = 1.0 + 0.5 * rng.random(shape)
    dt = 0.45 * dx / c.max()
    nt = 80
    src = wl.flat(shape, [[7, 9]])
    w = wl.ricker(nt, dt, 0.1).reshape(nt, 1)
    _, hist, _ = oracle.forward(c, dx, order, dt, nt, src, w, wl.flat(shape, [[0, 0]]), history=True)
    m = 1.0 / (c * c)

    def energy(n):   # E^{n+1/2}
        return (np.sum(m * (hist[n + 1] - hist[n]) ** 2) / (2 * dt * dt)
                - 0.5 * np.sum(hist[n + 1] * oracle.laplacian(hist[n], dx, order)))

    e_scale = max(abs(energy(n)) for n in range(nt))
    for n in range(1, nt):
        lhs = energy(n) - energy(n - 1)
        f = w[n, 0] / dx ** 2
        rhs = 0.5 * f * (hist[n + 1].flat[src[0]] - hist[n - 1].flat[src[0]])
        assert abs(lhs - rhs) < 1e-12 * e_scale


@pytest.mark.parametrize("shape,order", [((40,), 2), ((15, 17), 4), ((8, 9, 10), 8)])
def test_dot_product_forward_adjoint(shape, order):
    """<F w, d> = <w, F^T d> for the linear map wavelet -> traces, with F^T the
    backward sweep of the same operator (paper Sec. 2.2, self-adjoint problem):
    mismatch <= 1e-12."""
    rng = np.random.default_rng(7)
    c = 1.0 + rng.random(shape)
    nt = 70
    dt = 0.4 * oracle.cfl_limit(len(shape), order) / c.max()
    n = int(np.prod(shape))
    src = rng.choice(n, 3, replace=False)
    rec = rng.choice(n, 4, replace=False)
    w = rng.standard_normal((nt, 3))
    d = rng.standard_normal((nt, 4))
    traces, _, _ = oracle.forward(c, 1.0, order, dt, nt, src, w, rec)
    _, mu_src = oracle.adjoint(c, 1.0, order, dt, nt, rec, d / dt ** 2, src=src)
    lhs = float(np.sum(traces * d))
    rhs = float(np.sum(w * mu_src)) * dt * dt
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_reciprocity_heterogeneous():
    """Trace at r from a force at s equals the trace at s from the same force at r
    (symmetric mass and stiffness), heterogeneous medium."""
    shape, order = (30, 26), 8
    rng = np.random.default_rng(9)
    c = 1.0 + rng.random(shape)
    nt = 150
    dt = 0.45 * oracle.cfl_limit(2, order) / c.max()
    a, b = wl.flat(shape, [[3, 4]]), wl.flat(shape, [[25, 19]])
    w = wl.ricker(nt, dt, 0.08).reshape(nt, 1)
    tab, _, _ = oracle.forward(c, 1.0, order, dt, nt, a, w, b)
    tba, _, _ = oracle.forward(c, 1.0, order, dt, nt, b, w, a)
    assert np.abs(tab - tba).max() < 1e-13 * np.abs(tab).max()


# ---------------------------------------------------------------------------
# homogeneous-medium Green's functions (continuous limit of the scheme)
# ---------------------------------------------------------------------------

def _images(pos, shape, reach):
    """Mirror images of a point in the box with walls at the half-cell faces."""
    per_axis = []
    for p, n in zip(pos, shape):
        lst = []
        mmax = int(reach // (2 * n)) + 2
        for m in range(-mmax, mmax + 1):
            lst.append(p + 2 * n * m)
            lst.append(-1 - p + 2 * n * m)
        per_axis.append(lst)
    return per_axis


def _green_3d_trace(shape, s, r, c, t, wavelet_fn):
    out = np.zeros_like(t)
    reach = c * t.max() + 1
    ims = _images(s, shape, reach)
    for x in ims[0]:
        for y in ims[1]:
            for z in ims[2]:
                R = math.sqrt((x - r[0]) ** 2 + (y - r[1]) ** 2 + (z - r[2]) ** 2)
                if R <= reach:
                    out += wavelet_fn(t - R / c) / (4 * math.pi * R)
    return out


def _green_2d_trace(shape, s, r, c, t, wavelet_fn):
    """u = (1/2pi) int_0^{acosh(ct/R)} s(t - (R/c) cosh eta) d eta per image."""
    out = np.zeros_like(t)
    reach = c * t.max() + 1
    ims = _images(s, shape, reach)
    eta_q = np.linspace(0.0, 1.0, 4001)
    for x in ims[0]:
        for y in ims[1]:
            R = math.sqrt((x - r[0]) ** 2 + (y - r[1]) ** 2)
            for q, tq in enumerate(t):
                if c * tq <= R:
                    continue
                top = math.acosh(c * tq / R)
                eta = eta_q * top
                vals = wavelet_fn(tq - (R / c) * np.cosh(eta))
                out[q] += np.trapezoid(vals, eta) / (2 * math.pi)
    return out


def _ricker_fn(f, t0):
    def fn(t):
        a = (math.pi * f * (t - t0)) ** 2
        return (1 - 2 * a) * np.exp(-a)
    return fn


@pytest.mark.parametrize("ndim", [2, 3])
def test_homogeneous_green_function(ndim):
    """Homogeneous c: receiver traces converge to the closed-form Green's function
    of (1/c^2) u_tt - Delta u = s(t) delta(x) (3D: s(t - R/c) / (4 pi R); 2D: the
    c / (2 pi sqrt(c^2 t^2 - R^2)) convolution), summed over wall images.  Pins
    the point-source scaling 1/dx^d and the time origin; the error shrinks as
    the wavelength is resolved by more cells."""
    c0, order = 1.0, 8
    errs = []
    for cells_per_wl in (10, 20):
        f = c0 / cells_per_wl
        t0 = 1.5 / f
        n = 40 if ndim == 3 else 96
        shape = (n,) * ndim
        s = (n // 2,) * ndim
        r = (n // 2, n // 2 + 9) + ((n // 2,) if ndim == 3 else ())
        if ndim == 2:
            r = (n // 2 + 7, n // 2 + 9)
        dt = 0.3 / c0
        tmax = 2 * t0 + 40
        nt = int(tmax / dt)
        w = wl.ricker(nt, dt, f, t0).reshape(nt, 1)
        c = np.full(shape, c0)
        tr, _, _ = oracle.forward(c, 1.0, order, dt, nt, wl.flat(shape, [s]), w, wl.flat(shape, [r]))
        t = np.arange(1, nt + 1) * dt
        green = (_green_3d_trace if ndim == 3 else _green_2d_trace)(shape, s, r, c0, t, _ricker_fn(f, t0))
        errs.append(np.linalg.norm(tr[:, 0] - green) / np.linalg.norm(green))
    assert errs[1] < 0.02, errs
    assert errs[1] < 0.5 * errs[0], errs


# ---------------------------------------------------------------------------
# gradients (paper Sec. 2.2 sensitivity analysis, Sec. 4 superposition)
# ---------------------------------------------------------------------------

def _tiny(shape, order, seed, nt=40):
    rng = np.random.default_rng(seed)
    c = 1.0 + 0.5 * rng.random(shape)
    dt = 0.45 * oracle.cfl_limit(len(shape), order) / c.max()
    n = int(np.prod(shape))
    src = rng.choice(n, 2, replace=False)
    rec = rng.choice(n, 3, replace=False)
    w = rng.standard_normal((nt, 2))
    obs = 0.05 * rng.standard_normal((nt, 3))
    return c, dt, nt, src, w, rec, obs


@pytest.mark.parametrize("shape,order", [((12,), 2), ((9, 11), 4), ((5, 6, 7), 8)])
def test_exact_gradient_matches_brute_force_fd(shape, order):
    """Stored-history adjoint gradient dJ/dc equals central finite differences of
    the discrete J at every cell (eps = 1e-6): pins the dt factor of J, the
    adjoint force -residual/dt, the kernel's time differences and -2/c^3."""
    c, dt, nt, src, w, rec, obs = _tiny(shape, order, 11)
    g, J, _, _ = oracle.exact_gradient(c, 1.0, order, dt, nt, src, w, rec, obs)
    fd = oracle.fd_gradient(c, 1.0, order, dt, nt, src, w, rec, obs, np.arange(c.size))
    assert np.abs(fd - g.ravel()).max() < 1e-7 * np.abs(g).max()


@pytest.mark.parametrize("seg", [1, 7, 40, 1000])
def test_checkpointed_adjoint_equals_stored_history(seg):
    """Uniform checkpointing recomputes the same levels: identical gradient, J, traces
    and sum (dmu)^2 as the stored-history adjoint, for any segment length."""
    c, dt, nt, src, w, rec, obs = _tiny((7, 6, 9), 8, 19, nt=40)
    g, J, s2, tr = oracle.exact_gradient(c, 1.0, 8, dt, nt, src, w, rec, obs)
    gc, Jc, s2c, trc = oracle.exact_gradient_ckpt(c, 1.0, 8, dt, nt, src, w, rec, obs, seg=seg)
    assert np.array_equal(tr, trc) and J == Jc
    assert np.abs(gc - g).max() <= 1e-12 * np.abs(g).max()
    assert np.abs(s2c - s2).max() <= 1e-12 * np.abs(s2).max()


@pytest.mark.parametrize("shape,order", [((9, 11), 4), ((5, 6, 7), 8)])
def test_superposition_gap_closed_form(shape, order):
    """K(u+k mu, u+k mu) - K(u,u) = 2k K(u,mu) + k^2 K(mu,mu) (paper Eq.
    superposedkernel1), so approx - exact = (k / c^3) sum_n (mu^{n+1} - mu^n)^2
    cell by cell, and the +k / -k average is exact."""
    c, dt, nt, src, w, rec, obs = _tiny(shape, order, 13)
    g, J, s2, tr = oracle.exact_gradient(c, 1.0, order, dt, nt, src, w, rec, obs)
    scale = np.abs(g).max()
    for k in (1e-1, 1e-3):
        ga, Ja, tra = oracle.superposition_gradient(c, 1.0, order, dt, nt, src, w, rec, obs, k)
        assert np.abs(ga - g - k / c ** 3 * s2).max() < 1e-9 * scale
        assert abs(Ja - J) < 1e-13 * J
        assert np.array_equal(tra, tr)
        gm, _, _ = oracle.superposition_gradient(c, 1.0, order, dt, nt, src, w, rec, obs, -k)
        assert np.abs(0.5 * (ga + gm) - g).max() < 1e-9 * scale


def test_superposition_without_adjoint_force_is_zero():
    """Observed data equal to the simulated traces: no adjoint force, v = u level by
    level, and the kernel difference vanishes to rounding (the forward and backward
    interval sets coincide)."""
    shape, order = (14, 12), 8
    c, dt, nt, src, w, rec, _ = _tiny(shape, order, 17, nt=60)
    tr, _, _ = oracle.forward(c, 1.0, order, dt, nt, src, w, rec)
    ga, J, _ = oracle.superposition_gradient(c, 1.0, order, dt, nt, src, w, rec, tr, 1e-2)
    assert J == 0.0
    u_scale = np.abs(tr).max() ** 2 / 1e-2
    assert np.abs(ga).max() < 1e-9 * u_scale


def test_cfl_limits_match_symbol():
    """The stability limit 2 / sqrt(d max|symbol|) equals the tabulated values."""
    want = {(2, 2): 0.7071, (2, 4): 0.6124, (2, 8): 0.5546,
            (3, 2): 0.5774, (3, 4): 0.5000, (3, 8): 0.4529}
    for (d, p), v in want.items():
        assert abs(oracle.cfl_limit(d, p) - v) < 1e-4
