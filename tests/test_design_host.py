"""Host-side pieces of the design loop (no GPU): stable_dt keeps every design under the
per-cell stability bound that the variable-material calls check, for both of the
paper's material maps; the region receivers and the objective scale."""
import numpy as np
import pytest

from helpers import gershgorin_rows


@pytest.fixture(scope="module")
def dz():
    from paper_2509_15744_amd import design
    return design


def _maps():
    from paper_2509_15744_amd import fdwave
    return [(fdwave.rho_scaling(2700.0, 6000.0), 1e-5, 1.0, 1e-4),
            (fdwave.two_material(1.204, 2643.0, 1.419e5, 6.87e8), 0.0, 1.0, 1.0 / 300.0)]


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("ndim", [2, 3])
def test_stable_dt_covers_every_design(dz, which, ndim):
    """Random designs, lo/hi checkerboards and fields whose neighbour ratio sits at the
    worst value of the face term all satisfy dt^2 max_i s_i <= 4 dx^2 at stable_dt."""
    material, lo, hi, dx = _maps()[which]
    m0, dm, b0, db = material
    dt = dz.stable_dt(material, lo, hi, dx, ndim)
    rng = np.random.default_rng(3 + which + 10 * ndim)
    shape = (9, 10) if ndim == 2 else (6, 7, 8)
    fields = [lo + (hi - lo) * rng.random(shape) for _ in range(20)]
    idx = np.indices(shape).sum(axis=0)
    fields.append(np.where(idx % 2 == 0, lo, hi))
    for g2 in np.linspace(lo, hi, 9):                # a cell of one value among others
        f = np.full(shape, hi)
        f[idx % 2 == 0] = g2
        fields.append(f)
        fields.append(np.where(idx % 2 == 0, lo + 0.17 * (hi - lo), g2))
    worst = 0.0
    for g in fields:
        m, b = m0 + g * dm, b0 + g * db
        worst = max(worst, dt * dt * gershgorin_rows(m, b).max() / (4 * dx * dx))
    assert worst <= 0.95 ** 2 * (1 + 1e-9)


def test_region_receivers_and_scale(dz):
    rec = dz.region_receivers((5, 7), (1, 2), (2, 3))
    assert rec.tolist() == [9, 10, 11, 16, 17, 18]
    rec3 = dz.region_receivers((4, 5, 6), (1, 0, 2), (1, 2, 2))
    assert rec3.tolist() == [32, 33, 38, 39]
    assert dz.region_scale(8) == 0.25 and dz.region_scale(8, maximize=True) == -0.25
