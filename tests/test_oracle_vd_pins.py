"""Pins of the oracle's variable-material scheme (the paper's second-order flux form,
Sec. 3.1, Eqs. FDstencil1/FDstencil2 as m u_tt - div(b grad u) = f with
harmonic-mean faces) against facts fixed independently of its code:

* with b = 1 it is the constant-density order-2 scheme of the other oracle;
* the exact steady solution of (b u')' = 0 in a two-material bar (piecewise
  linear, slopes in the ratio of the materials) is annihilated at every interior
  cell: the series-conductance face value is the harmonic mean, an arithmetic mean
  fails this;
* L_b is symmetric, negative semi-definite and annihilates constants;
* the discrete energy is conserved without forces;
* the forward map and the backward sweep are transposes (dot-product test);
* the exact gradient equals brute-force central differences of J in m and in b at
  every cell of tiny grids;
* Alg. 1 differs from the exact gradient by the closed forms -(k/2) sum (dmu)^2
  (mass) and (dt^2/dx^2)(k/2) sum_faces dh/db (dmu)^2 (stiffness); the +/-k average
  is exact;
* the per-cell stability bound (Gershgorin row sums of M^-1/2 K M^-1/2) covers the
  largest eigenvalue of M^-1 K from a dense eigen-solve, reaches the closed-form
  Neumann eigenvalue's bound in a homogeneous medium, and leapfrog runs are bounded
  just below 2/sqrt(lambda_max) and blow up just above it.
"""
import numpy as np
import pytest

import oracle
from helpers import gershgorin_rows


def _medium(shape, seed):
    rng = np.random.default_rng(seed)
    m = 0.5 + rng.random(shape)
    b = 0.5 + rng.random(shape)
    dt = 0.4 / np.sqrt(len(shape) * b.max() / m.min())
    return rng, m, b, dt


@pytest.mark.parametrize("shape", [(40,), (21, 17), (9, 8, 11)])
def test_constant_stiffness_is_the_order2_scheme(shape):
    """b = 1, m = 1/c^2: traces equal the constant-density order-2 oracle and
    dJ/dc = -(2/c^3) dJ/dm."""
    rng = np.random.default_rng(3)
    c = 1.0 + rng.random(shape)
    n = int(np.prod(shape))
    nt = 40
    dt = 0.4 * oracle.cfl_limit(len(shape), 2) / c.max()
    src, rec = rng.choice(n, 2, replace=False), rng.choice(n, 5, replace=False)
    w = rng.standard_normal((nt, 2))
    obs = 0.1 * rng.standard_normal((nt, 5))
    tr_v, _, _ = oracle.vd_forward(1.0 / c ** 2, np.ones(shape), 1.0, dt, nt, src, w, rec)
    tr_c, _, _ = oracle.forward(c, 1.0, 2, dt, nt, src, w, rec)
    assert np.abs(tr_v - tr_c).max() <= 1e-12 * np.abs(tr_c).max()
    gm, gb, J, _, _, _ = oracle.vd_exact_gradient(1.0 / c ** 2, np.ones(shape), 1.0, dt, nt, src, w,
                                                  rec, obs)
    gc, Jc, _, _ = oracle.exact_gradient(c, 1.0, 2, dt, nt, src, w, rec, obs)
    assert abs(J - Jc) <= 1e-12 * Jc
    assert np.abs(-2.0 / c ** 3 * gm - gc).max() <= 1e-9 * np.abs(gc).max()


@pytest.mark.parametrize("dx", [1.0, 0.25])
def test_two_material_bar_steady_state(dx):
    """(b u')' = 0 with b = b1 left of a face and b2 right of it: u is linear on each
    side with u'_2 / u'_1 = b1 / b2 and continuous at the face.  Sampled at the cell
    centres, L_b u = 0 at every interior cell (only the wall cells, where the mirror
    imposes zero flux, differ).  The arithmetic face mean does not annihilate it."""
    n, cut = 30, 13                     # face between cells cut-1 and cut
    b1, b2 = 0.7, 3.1
    b = np.where(np.arange(n) < cut, b1, b2).astype(float)
    xf = cut * dx                       # face position (cells centred at (i + 1/2) dx)
    x = (np.arange(n) + 0.5) * dx
    s1 = 1.0
    s2 = s1 * b1 / b2
    u = np.where(x < xf, s1 * (x - xf), s2 * (x - xf)) + 2.0
    lu = oracle.vd_operator(b, u, dx)
    interior = lu[1:-1]
    assert np.abs(interior).max() <= 1e-12 * np.abs(u).max() / dx ** 2
    # with the arithmetic mean the interface cells would see a net flux
    am = 0.5 * (b1 + b2)
    flux_left = am * (u[cut] - u[cut - 1]) / dx ** 2
    flux_in = b1 * (u[cut - 1] - u[cut - 2]) / dx ** 2
    assert abs(flux_left - flux_in) > 1e-3 * abs(flux_in)


@pytest.mark.parametrize("shape", [(25,), (11, 9), (6, 7, 5)])
def test_operator_symmetric_negative_and_annihilates_constants(shape):
    rng = np.random.default_rng(5)
    b = 0.3 + rng.random(shape)
    x, y = rng.standard_normal(shape), rng.standard_normal(shape)
    lx, ly = oracle.vd_operator(b, x, 0.7), oracle.vd_operator(b, y, 0.7)
    assert abs(np.sum(lx * y) - np.sum(x * ly)) <= 1e-13 * np.abs(lx).sum() * np.abs(y).max()
    assert np.sum(x * lx) < 0.0
    assert np.abs(oracle.vd_operator(b, np.full(shape, 3.7), 0.7)).max() == 0.0


def test_energy_is_conserved_source_free():
    """E^{n+1/2} = 1/2 (u^{n+1}-u^n)^T M (u^{n+1}-u^n) / dt^2 - 1/2 (u^{n+1})^T L_b u^n is
    constant once the source has stopped (heterogeneous m and b)."""
    shape = (24, 19)
    rng, m, b, dt = _medium(shape, 11)
    nt = 160
    src = np.array([5 * 19 + 7])
    w = np.zeros((nt, 1))
    w[:20, 0] = rng.standard_normal(20)
    _, hist, _ = oracle.vd_forward(m, b, 1.0, dt, nt, src, w, np.array([0]), history=True)
    E = []
    for n in range(25, nt):
        du = hist[n + 1] - hist[n]
        E.append(0.5 * np.sum(m * du * du) / dt ** 2
                 - 0.5 * np.sum(hist[n + 1] * oracle.vd_operator(b, hist[n], 1.0)))
    E = np.array(E)
    assert np.abs(E - E[0]).max() <= 1e-12 * abs(E[0])


@pytest.mark.parametrize("shape", [(19, 15), (7, 6, 9)])
def test_dot_product_forward_adjoint(shape):
    """<F w, d> = <w, F^T d> for wavelet -> traces, F^T the backward sweep with the
    force d / dt^2 (the same operator): mismatch <= 1e-12."""
    rng, m, b, dt = _medium(shape, 7)
    nt = 60
    n = int(np.prod(shape))
    src, rec = rng.choice(n, 3, replace=False), rng.choice(n, 4, replace=False)
    w, d = rng.standard_normal((nt, 3)), rng.standard_normal((nt, 4))
    traces, _, _ = oracle.vd_forward(m, b, 1.0, dt, nt, src, w, rec)
    hist = oracle.vd_adjoint(m, b, 1.0, dt, nt, rec, d / dt ** 2)
    mu_src = hist[:nt].reshape(nt, -1)[:, src]
    lhs = float(np.sum(traces * d))
    rhs = float(np.sum(w * mu_src)) * dt * dt
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("shape", [(13,), (8, 7), (5, 4, 6)])
def test_exact_gradient_matches_brute_force_fd(shape):
    """dJ/dm and dJ/db of the exact discrete adjoint vs central differences of J
    (eps = 1e-6) at every cell: max error <= 1e-6 of the largest entry."""
    rng, m, b, dt = _medium(shape, 13)
    nt = 30
    n = int(np.prod(shape))
    src, rec = rng.choice(n, 2, replace=False), rng.choice(n, 3, replace=False)
    w = rng.standard_normal((nt, 2))
    obs = 0.1 * rng.standard_normal((nt, 3))
    gm, gb, _, _, _, _ = oracle.vd_exact_gradient(m, b, 1.0, dt, nt, src, w, rec, obs)
    cells = np.arange(n)
    fm = oracle.vd_fd_gradient(m, b, "m", 1.0, dt, nt, src, w, rec, obs, cells)
    fb = oracle.vd_fd_gradient(m, b, "b", 1.0, dt, nt, src, w, rec, obs, cells)
    assert np.abs(fm - gm.reshape(-1)).max() <= 1e-6 * np.abs(gm).max()
    assert np.abs(fb - gb.reshape(-1)).max() <= 1e-6 * np.abs(gb).max()


@pytest.mark.parametrize("shape,dx", [((17, 13), 1.0), ((6, 5, 8), 0.5)])
def test_superposition_gap_closed_form(shape, dx):
    """Alg. 1 minus the exact gradient: -(k/2) s2_m for m and (dt^2/dx^2)(k/2) s2_b for b,
    to rounding; the +/-k average is the exact gradient."""
    rng, m, b, dt = _medium(shape, 17)
    dt *= dx
    nt = 45
    n = int(np.prod(shape))
    src, rec = rng.choice(n, 2, replace=False), rng.choice(n, 5, replace=False)
    w = rng.standard_normal((nt, 2))
    obs = 0.1 * rng.standard_normal((nt, 5))
    gm, gb, J, s2m, s2b, tr = oracle.vd_exact_gradient(m, b, dx, dt, nt, src, w, rec, obs)
    k = 0.02
    am, ab, Ja, tra = oracle.vd_superposition_gradient(m, b, dx, dt, nt, src, w, rec, obs, k)
    bm, bb, _, _ = oracle.vd_superposition_gradient(m, b, dx, dt, nt, src, w, rec, obs, -k)
    assert J == Ja and np.array_equal(tr, tra)
    assert np.abs((am - gm) + 0.5 * k * s2m).max() <= 1e-10 * np.abs(gm).max()
    assert np.abs((ab - gb) - 0.5 * k * dt ** 2 / dx ** 2 * s2b).max() <= 1e-10 * np.abs(gb).max()
    assert np.abs(0.5 * (am + bm) - gm).max() <= 1e-10 * np.abs(gm).max()
    assert np.abs(0.5 * (ab + bb) - gb).max() <= 1e-10 * np.abs(gb).max()


def _stiffness_matrix(b, dx):
    """K = -L_b as a dense matrix, column by column from the oracle's operator."""
    n = b.size
    K = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        K[:, j] = -oracle.vd_operator(b, e.reshape(b.shape), dx).reshape(-1)
    return K


def test_stability_bound_homogeneous_closed_form():
    """Homogeneous medium: lambda_max(M^-1 K) is the cell-centred Neumann eigenvalue
    (b/m)(4/dx^2) sum_ax sin^2(pi (n_ax - 1) / (2 n_ax)), below the row-sum bound
    4 d b / (m dx^2), which the interior rows reach."""
    import scipy.linalg
    shape, dx, mv, bv = (7, 5), 0.5, 1.7, 2.3
    K = _stiffness_matrix(np.full(shape, bv), dx)
    lam = scipy.linalg.eigh(K, np.eye(K.shape[0]) * mv, eigvals_only=True)
    want = bv / mv * 4 / dx ** 2 * sum(np.sin(np.pi * (n - 1) / (2 * n)) ** 2 for n in shape)
    assert abs(lam.max() - want) < 1e-12 * want
    s = gershgorin_rows(np.full(shape, mv), np.full(shape, bv))
    assert abs(s.max() / dx ** 2 - 4 * len(shape) * bv / mv / dx ** 2) < 1e-12 * s.max()


@pytest.mark.parametrize("shape,seed", [((6, 5), 1), ((4, 3, 5), 2)])
def test_stability_bound_covers_lambda_max(shape, seed):
    """Air/solid-like mixtures (Eq. wavetopopt materials scaled to unit order): the
    per-cell bound is at least lambda_max, and well below the global
    4 d max b / (min m dx^2), which pairs one material's stiffness with the other's mass."""
    import scipy.linalg
    rng = np.random.default_rng(seed)
    solid = rng.random(shape) < 0.5
    m = np.where(solid, 1.46e-9, 7.05e-6) * 1e6
    b = np.where(solid, 3.78e-4, 0.83)
    dx = 1.0
    K = _stiffness_matrix(b, dx)
    lam = scipy.linalg.eigh(K, np.diag(m.reshape(-1)), eigvals_only=True).max()
    s = gershgorin_rows(m, b).max() / dx ** 2
    assert lam <= s * (1 + 1e-12)
    assert s < 0.05 * 4 * len(shape) * b.max() / m.min() / dx ** 2


def test_leapfrog_limit_is_lambda_max():
    """Oracle runs driven by a +/- impulse pair (no net force, so the Neumann zero mode
    stays at rest) stay bounded at dt = 0.999 * 2/sqrt(lambda_max) and grow without
    bound at 1.02 times it: the limit the bound guards is the right one."""
    import scipy.linalg
    rng = np.random.default_rng(4)
    shape = (6, 7)
    m = 0.5 + rng.random(shape)
    b = 0.5 + rng.random(shape)
    K = _stiffness_matrix(b, 1.0)
    lam = scipy.linalg.eigh(K, np.diag(m.reshape(-1)), eigvals_only=True).max()
    nt = 3000
    w = np.zeros((nt, 2))
    w[0] = (1.0, -1.0)
    src = np.array([9, 30], dtype=np.int64)
    rec = np.arange(m.size, dtype=np.int64)
    tr, _, _ = oracle.vd_forward(m, b, 1.0, 0.999 * 2 / np.sqrt(lam), nt, src, w, rec)
    assert np.abs(tr[nt // 2:]).max() < 2.0 * np.abs(tr[:nt // 2]).max()
    with np.errstate(all="ignore"):
        tr, _, _ = oracle.vd_forward(m, b, 1.0, 1.02 * 2 / np.sqrt(lam), nt, src, w, rec)
        grown = np.abs(tr[nt // 2:]).max() / np.abs(tr[:nt // 2]).max()
    assert not np.isfinite(tr).all() or grown > 1e6
