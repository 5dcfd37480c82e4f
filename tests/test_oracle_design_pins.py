"""Pins of the oracle's design chain (``oracle/design.py``: density filter, projection,
clip, material maps, their chain rule and Adam) against facts fixed outside its code:

* the filter's values for a unit impulse at r_f = 1.5 (the paper's radius) in 2D and
  3D, worked out by hand from w = r_f - |x|; a brute-force double loop over all cell
  pairs on tiny grids; constants are kept everywhere and linear fields at cells whose
  neighbourhood lies inside the box; the transpose passes the dot-product test;
* the projection maps 0 to 0, 1 to 1 and eta to tanh(beta eta) / normaliser, tends
  to the identity as beta -> 0, and its slope equals central differences;
* the whole chain's gradient equals central differences of a linear functional of
  (m, b) at every design cell of tiny boxes, with clipping active;
* Adam's first step is lr g / (|g| + eps) per coordinate (m_hat = g, v_hat = g^2),
  and twenty steps agree with torch.optim.Adam, an independent implementation of the
  same published algorithm; the clip holds.
"""
import numpy as np
import pytest

from oracle import design as od


def test_filter_impulse_2d_closed_form():
    """Weights 1.5 (centre), 0.5 (4 edge neighbours), 1.5 - sqrt 2 (4 diagonal ones):
    an impulse spreads as w / W with W = 9.5 - 4 sqrt 2 at interior cells."""
    g = np.zeros((9, 9))
    g[4, 4] = 1.0
    gt = od.density_filter(g, 1.5)
    W = 9.5 - 4 * np.sqrt(2)
    assert abs(gt[4, 4] - 1.5 / W) < 1e-15
    for q in [(3, 4), (5, 4), (4, 3), (4, 5)]:
        assert abs(gt[q] - 0.5 / W) < 1e-15
    for q in [(3, 3), (3, 5), (5, 3), (5, 5)]:
        assert abs(gt[q] - (1.5 - np.sqrt(2)) / W) < 1e-15
    assert np.count_nonzero(gt) == 9


def test_filter_impulse_3d_closed_form():
    """19 taps in 3D at r_f = 1.5 (|x|^2 in {0, 1, 2}): W = 22.5 - 12 sqrt 2."""
    g = np.zeros((5, 5, 5))
    g[2, 2, 2] = 1.0
    gt = od.density_filter(g, 1.5)
    W = 22.5 - 12 * np.sqrt(2)
    assert abs(gt[2, 2, 2] - 1.5 / W) < 1e-15
    assert abs(gt[2, 2, 3] - 0.5 / W) < 1e-15
    assert abs(gt[2, 3, 3] - (1.5 - np.sqrt(2)) / W) < 1e-15
    assert gt[3, 3, 3] == 0.0
    assert np.count_nonzero(gt) == 19


@pytest.mark.parametrize("shape,rf", [((4, 5), 2.3), ((3, 3, 4), 1.5), ((6, 3), 1.0), ((5, 4), 3.7)])
def test_filter_brute_force(shape, rf):
    rng = np.random.default_rng(1)
    g = rng.random(shape)
    cells = list(np.ndindex(*shape))
    want = np.zeros(shape)
    for i in cells:
        num = den = 0.0
        for k in cells:
            dist = np.sqrt(sum((a - b) ** 2 for a, b in zip(i, k)))
            if dist < max(rf, 1.0):
                w = max(rf, 1.0) - dist
                num += w * g[k]
                den += w
        want[i] = num / den
    assert np.abs(od.density_filter(g, rf) - want).max() < 1e-14


@pytest.mark.parametrize("rf", [1.5, 2.5, 4.2])
def test_filter_keeps_constants_and_interior_linear_fields(rf):
    shape = (14, 17)
    assert np.abs(od.density_filter(np.full(shape, 0.37), rf) - 0.37).max() < 1e-15
    i, j = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    lin = 0.3 + 0.02 * i - 0.05 * j
    R = int(np.ceil(rf)) - 1
    inner = (slice(R, shape[0] - R), slice(R, shape[1] - R))
    assert np.abs(od.density_filter(lin, rf)[inner] - lin[inner]).max() < 1e-14
    # at the edge the truncated neighbourhood is one-sided: the value moves inward
    assert abs(od.density_filter(lin, rf)[0, 8] - lin[0, 8]) > 1e-3


@pytest.mark.parametrize("shape,rf", [((7, 9), 1.5), ((4, 5, 6), 2.2)])
def test_filter_transpose_dot_product(shape, rf):
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(shape), rng.standard_normal(shape)
    a = np.sum(od.density_filter(x, rf) * y)
    b = np.sum(x * od.density_filter_transpose(y, rf))
    assert abs(a - b) < 1e-13 * np.abs(x).sum()


@pytest.mark.parametrize("beta,eta", [(1.0, 0.5), (8.0, 0.5), (3.0, 0.3), (20.0, 0.7)])
def test_projection_fixed_points_and_slope(beta, eta):
    den = np.tanh(beta * eta) + np.tanh(beta * (1 - eta))
    assert abs(od.projection(0.0, beta, eta)) < 1e-15
    assert abs(od.projection(1.0, beta, eta) - 1.0) < 1e-15
    assert abs(od.projection(eta, beta, eta) - np.tanh(beta * eta) / den) < 1e-15
    x = np.linspace(-0.2, 1.2, 29)
    h = 1e-6
    fd = (od.projection(x + h, beta, eta) - od.projection(x - h, beta, eta)) / (2 * h)
    assert np.abs(od.projection_slope(x, beta, eta) - fd).max() < 1e-6 * max(1.0, beta)


def test_projection_small_beta_is_identity():
    x = np.linspace(0, 1, 11)
    assert np.abs(od.projection(x, 1e-5, 0.5) - x).max() < 1e-9
    assert np.array_equal(od.projection(x, 0.0, 0.5), x)


MATERIALS = [od.rho_scaling(2700.0, 6000.0), od.two_material(1.204, 2643.0, 1.419e5, 6.87e8)]


@pytest.mark.parametrize("shape,rf,beta,eta,lo,hi,mat,spread", [
    ((5, 6), 1.5, 4.0, 0.5, 0.0, 1.0, 0, 1.0),
    ((4, 3, 5), 2.2, 2.0, 0.4, 0.25, 0.75, 1, 3.0),    # clipping active on both sides
    ((6, 4), 1.0, 0.0, 0.5, 1e-5, 1.0, 0, 1.0),        # no filter, no projection (FWI form)
])
def test_chain_rule_matches_central_differences(shape, rf, beta, eta, lo, hi, mat, spread):
    """L(gamma) = sum (a m + c b): its gradient from design_adjoint equals central
    differences at every design cell (cells whose projected value sits within the step
    of a clip bound are skipped, the map has a kink there)."""
    rng = np.random.default_rng(3)
    gamma = 0.5 + spread * (rng.random(shape) - 0.5)
    material = MATERIALS[mat]
    scale = np.array([1.0 / abs(material[1]), 1.0 / abs(material[3])])
    a = rng.standard_normal(shape) * scale[0]
    c = rng.standard_normal(shape) * scale[1]

    def L(gm):
        _, m, b = od.design_map(gm, rf, beta, eta, lo, hi, material)
        return np.sum(a * m + c * b)

    grad = od.design_adjoint(gamma, rf, beta, eta, lo, hi, material, a, c)
    h = 1e-6
    gt = od.density_filter(gamma, rf)
    proj = od.projection(gt, beta, eta)
    near = (np.abs(proj - lo) < 1e-4) | (np.abs(proj - hi) < 1e-4)
    R = int(np.ceil(max(rf, 1.0))) - 1
    checked = 0
    for i in np.ndindex(*shape):
        lo_i = tuple(max(0, q - R) for q in i)
        hi_i = tuple(q + R + 1 for q in i)
        if near[tuple(slice(l, u) for l, u in zip(lo_i, hi_i))].any():
            continue
        e = np.zeros(shape)
        e[i] = h
        fd = (L(gamma + e) - L(gamma - e)) / (2 * h)
        assert abs(fd - grad[i]) < 1e-6 * (abs(fd) + 1e-3), (i, fd, grad[i])
        checked += 1
    assert checked >= 0.3 * gamma.size
    if spread > 1:
        g, _, _ = od.design_map(gamma, rf, beta, eta, lo, hi, material)
        assert (g == lo).any() and (g == hi).any()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    x0, g = rng.random(50), rng.standard_normal(50)
    x1, _, _ = od.adam(x0, g, np.zeros(50), np.zeros(50), 1, lr=0.1, eps=1e-8)
    assert np.abs(x1 - (x0 - 0.1 * g / (np.abs(g) + 1e-8))).max() < 1e-15


def test_adam_matches_torch_and_clips():
    import torch
    rng = np.random.default_rng(5)
    x0 = rng.random(40)
    grads = rng.standard_normal((20, 40))
    p = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.8, 0.95), eps=1e-6)
    x, m1, m2 = x0.copy(), np.zeros(40), np.zeros(40)
    for t, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g)
        opt.step()
        x, m1, m2 = od.adam(x, g, m1, m2, t, lr=0.01, beta1=0.8, beta2=0.95, eps=1e-6)
    assert np.abs(x - p.detach().numpy()).max() < 1e-14
    xc, _, _ = od.adam(x0, np.full(40, -1.0), np.zeros(40), np.zeros(40), 1, lr=0.5, lo=0.0, hi=1.0)
    assert xc.max() == 1.0 and xc.min() >= 0.0 and (xc == 1.0).sum() == (x0 >= 0.5).sum()
