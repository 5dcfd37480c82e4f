"""Seeded synthetic inputs for the acoustic sensitivity workloads.

This module only generates inputs (wave-speed fields, source wavelets,
source and receiver cells, time step); it holds none of the method's
arithmetic and is the one piece shared by the GPU path and the oracle.
Every generator is deterministic in its seed.

The paper's own inputs (a CT-scanned specimen and acquisition files
published separately) are not available; these recipes stand in for them
with the same structure: smooth heterogeneous media, a point source near the
top face and a line or plane of receivers.

Conventions: grids are C-order with axis 0 the depth (slowest) axis and the
last axis contiguous; cells are addressed by flat C-order indices (int64);
the wavelet is ``[nt, nsrc]`` with row n at t = n dt; dx = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One sensitivity problem: model, acquisition and time axis."""
    name: str
    shape: tuple
    order: int
    dtype: str                 # "f32" or "f64": arithmetic type of the GPU fields
    dx: float
    dt: float
    nt: int
    c: object                  # numpy array (or torch tensor for device-generated grids)
    c_ref: object              # model whose traces serve as the observed data
    src: np.ndarray            # int64 [nsrc] flat cells
    rec: np.ndarray            # int64 [nrec] flat cells
    wavelet: np.ndarray        # float64 [nt, nsrc]
    meta: dict = field(default_factory=dict)
    observed: np.ndarray | None = None   # [nt, nrec] data given directly (c_ref is then None)

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def ncell(self):
        return int(np.prod(self.shape))


def ricker(nt: int, dt: float, f_peak: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet w(t) = (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0,
    sampled at t = n dt, n = 0..nt-1; t0 defaults to 1.5 / f_peak."""
    if t0 is None:
        t0 = 1.5 / f_peak
    t = np.arange(nt, dtype=np.float64) * dt
    a = (math.pi * f_peak * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def flat(shape, coords) -> np.ndarray:
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, len(shape))
    return np.ravel_multi_index(tuple(coords.T), tuple(shape)).astype(np.int64)


def time_step(c_max: float, dx: float, courant: float) -> float:
    """dt from the Courant number c_max dt / dx."""
    return courant * dx / c_max


# ---------------------------------------------------------------------------
# media
# ---------------------------------------------------------------------------

def smooth_noise(shape, sigma: float, seed: int) -> np.ndarray:
    """White Gaussian noise, Gaussian-smoothed (reflecting edges), scaled to max |P| = 1."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    p = gaussian_filter(rng.standard_normal(shape), sigma=sigma, mode="reflect")
    return p / np.abs(p).max()


def layered_speed(shape, n_layers: int, c_lo: float, c_hi: float, seed: int) -> np.ndarray:
    """Piecewise-constant speed along axis 0: interfaces at sorted uniform depths,
    layer speeds uniform in [c_lo, c_hi]."""
    rng = np.random.default_rng(seed)
    n0 = shape[0]
    cuts = np.sort(rng.uniform(0.0, n0, size=n_layers - 1))
    speeds = rng.uniform(c_lo, c_hi, size=n_layers)
    depth = np.arange(n0) + 0.5
    layer = np.searchsorted(cuts, depth)
    prof = speeds[layer]
    return np.broadcast_to(prof.reshape((n0,) + (1,) * (len(shape) - 1)), shape).copy()


def layered_perturbed(shape, seed: int, n_layers=8, c_lo=1.5, c_hi=4.5, sigma=8.0, amp=0.05):
    """Layered medium times (1 + amp P) with P smoothed noise; returns (c, c_layers)."""
    base = layered_speed(shape, n_layers, c_lo, c_hi, seed)
    pert = smooth_noise(shape, sigma, seed + 1)
    return base * (1.0 + amp * pert), base


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def inclusion_2d(n: int = 128, nt: int = 600, order: int = 4, dtype: str = "f64",
                 radius: float = 16.0, c_in: float = 1.2, courant: float = 0.5,
                 nrec: int = 32) -> Problem:
    """Homogeneous c = 1 with a circular inclusion of speed ``c_in``; Ricker source
    at the top centre (20 cells per wavelength at c = 1), receivers on the bottom row;
    observed data come from the inclusion-free medium."""
    shape = (n, n)
    i, j = np.meshgrid(np.arange(n) + 0.0, np.arange(n) + 0.0, indexing="ij")
    ctr = (n - 1) / 2.0
    c = np.where((i - ctr) ** 2 + (j - ctr) ** 2 <= radius ** 2, c_in, 1.0)
    c_ref = np.ones(shape)
    dt = time_step(c.max(), 1.0, courant)
    f_peak = 1.0 / 20.0
    step = max(1, n // nrec)
    rec = flat(shape, [[n - 1, step * q + step // 2] for q in range(nrec)])
    src = flat(shape, [[0, n // 2]])
    return Problem("inclusion2d", shape, order, dtype, 1.0, dt, nt, c, c_ref, src, rec,
                   ricker(nt, dt, f_peak).reshape(nt, 1),
                   meta={"courant": courant, "f_peak": f_peak})


def layered_2d(n: int = 2048, nt: int = 4000, order: int = 8, dtype: str = "f32",
               seed: int = 2, courant: float = 0.5, rec_every: int = 4,
               src_cols=None) -> Problem:
    """Eight random layers (c in [1.5, 4.5]) times a 5% smoothed (sigma = 8) perturbation;
    Ricker source(s) on the top row at 20 cells per wavelength of the slowest speed;
    receivers on the top row every ``rec_every`` cells; observed data from the
    unperturbed layers."""
    shape = (n, n)
    c, c_ref = layered_perturbed(shape, seed)
    dt = time_step(c.max(), 1.0, courant)
    f_peak = c.min() / 20.0
    if src_cols is None:
        src_cols = [n // 2]
    src = flat(shape, [[0, s] for s in src_cols])
    rec = flat(shape, [[0, rec_every * q + rec_every // 2] for q in range(n // rec_every)])
    w = ricker(nt, dt, f_peak)
    wavelet = np.repeat(w.reshape(nt, 1), len(src), axis=1)
    return Problem("layered2d", shape, order, dtype, 1.0, dt, nt, c, c_ref, src, rec, wavelet,
                   meta={"courant": courant, "f_peak": f_peak, "seed": seed})


def ricker_fn(f_peak: float, t0: float | None = None):
    """The Ricker wavelet as a function of continuous time."""
    if t0 is None:
        t0 = 1.5 / f_peak

    def fn(t):
        a = (math.pi * f_peak * (np.asarray(t) - t0)) ** 2
        return (1.0 - 2.0 * a) * np.exp(-a)
    return fn


def green3d_traces(shape, src_pos, rec_pos, c0, dt, nt, wavelet_fn, dx=1.0):
    """Closed-form data of a homogeneous 3D box of speed c0 with reflecting walls at the
    half-cell faces: sum over wall images of s(t - R/c0) / (4 pi R) for
    (1/c0^2) u_tt - Lap u = s(t) delta, sampled at t = n dt, n = 1..nt.
    Positions are cell indices (cell centres); returns [nt, nrec]."""
    t = np.arange(1, nt + 1) * dt
    reach = c0 * t[-1] / dx + 1.0
    per_axis = []
    for p, n in zip(src_pos, shape):
        m = int(reach // (2 * n)) + 2
        per_axis.append(np.array([p + 2 * n * k for k in range(-m, m + 1)]
                                 + [-1 - p + 2 * n * k for k in range(-m, m + 1)], dtype=np.float64))
    ix, iy, iz = np.meshgrid(*per_axis, indexing="ij")
    imgs = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    rec_pos = np.asarray(rec_pos, dtype=np.float64)
    out = np.zeros((nt, len(rec_pos)))
    for q, r in enumerate(rec_pos):
        R = np.sqrt(((imgs - r) ** 2).sum(axis=1)) * dx
        R = R[R <= reach * dx]
        tau = t[:, None] - R[None, :] / c0
        out[:, q] = (wavelet_fn(tau) / (4.0 * math.pi * R[None, :])).sum(axis=1)
    return out


def smooth_3d(n: int = 256, nt: int = 2000, order: int = 8, dtype: str = "f32", seed: int = 4,
              sigma: float = 6.0, courant: float = 0.4, rec_every: int = 8,
              observed: str = "green") -> Problem:
    """Smooth random speed in [1, 3] (white noise, Gaussian sigma, affine map); Ricker
    source at the centre of the top face (f = 1/20); receiver grid on the face
    x0 = 0 every ``rec_every`` cells.  Observed data: the closed-form traces of the
    homogeneous c = 2 box (``observed="green"``, no solve needed) or the traces of a
    c = 2 solve (``observed="solve"``, c_ref set)."""
    shape = (n, n, n)
    p = smooth_noise(shape, sigma, seed)
    c = 1.0 + (p - p.min()) * (2.0 / (p.max() - p.min()))
    dt = time_step(3.0, 1.0, courant)
    f_peak = 1.0 / 20.0
    src_pos = [0, n // 2, n // 2]
    src = flat(shape, [src_pos])
    h = rec_every // 2
    rec_pos = [[0, rec_every * a + h, rec_every * b + h]
               for a in range(n // rec_every) for b in range(n // rec_every)]
    rec = flat(shape, rec_pos)
    obs, c_ref = None, None
    if observed == "green":
        obs = green3d_traces(shape, src_pos, rec_pos, 2.0, dt, nt, ricker_fn(f_peak))
    else:
        c_ref = np.full(shape, 2.0)
    return Problem("smooth3d", shape, order, dtype, 1.0, dt, nt, c, c_ref, src, rec,
                   ricker(nt, dt, f_peak).reshape(nt, 1),
                   meta={"courant": courant, "f_peak": f_peak, "seed": seed}, observed=obs)


def layered_3d(n: int = 1024, nt: int = 3000, order: int = 8, dtype: str = "f32", seed: int = 5,
               courant: float = 0.4, rec_every: int = 8, shots=None, device=None) -> Problem:
    """3D version of the layered recipe (layers along axis 0, 5% smoothed perturbation,
    sigma = 8); source(s) on the top face; receiver plane on x0 = 0 every ``rec_every``
    cells.  With ``device`` (a torch device) the field is generated there, which keeps
    billion-cell grids off the host; c and c_ref are then torch tensors."""
    shape = (n, n, n)
    if device is None:
        c, c_ref = layered_perturbed(shape, seed)
        c_min, c_max = float(c.min()), float(c.max())
    else:
        c, c_ref = _layered_perturbed_torch(shape, seed, device)
        c_min, c_max = float(c.min()), float(c.max())
    dt = time_step(c_max, 1.0, courant)
    f_peak = c_min / 20.0
    if shots is None:
        shots = [(n // 2, n // 2)]
    src = flat(shape, [[0, a, b] for (a, b) in shots])
    h = rec_every // 2
    rec = flat(shape, [[0, rec_every * a + h, rec_every * b + h]
                       for a in range(n // rec_every) for b in range(n // rec_every)])
    w = ricker(nt, dt, f_peak)
    wavelet = np.repeat(w.reshape(nt, 1), len(src), axis=1)
    return Problem("layered3d", shape, order, dtype, 1.0, dt, nt, c, c_ref, src, rec, wavelet,
                   meta={"courant": courant, "f_peak": f_peak, "seed": seed})


def layered_material_3d(n: int = 1024, nt: int = 3000, seed: int = 5, rec_every: int = 8,
                        bound_frac: float = 0.9, device=None) -> dict:
    """Variable-material twin of ``layered_3d`` for the second-order flux-form scheme
    m u_tt - div(b grad u) = f: mass m = 1/c^2 of the perturbed layered medium,
    stiffness b = a second layered profile (8 layers, values in [0.5, 1.5]) times the
    same 5% smoothed perturbation (b / b_layers = c / c_layers); the reference medium of
    the observed data is m_ref = 1/c_ref^2, b_ref = 1.  dt is ``bound_frac`` of the
    stability bound dt sqrt(3 max b / min m) <= dx (dx = 1).  Source at the top-face
    centre, receiver plane on x0 = 0 every ``rec_every`` cells, Ricker at 20 cells per
    wavelength of the slowest speed sqrt(min b / max m).  With ``device`` the fields are
    generated there (torch tensors, float32)."""
    import torch
    shape = (n, n, n)
    c, c_ref = _layered_perturbed_torch(shape, seed, device)
    prof = layered_speed((n, 1), 8, 0.5, 1.5, seed + 7)[:, 0]
    b_lay = torch.as_tensor(prof, device=device, dtype=torch.float32).view(n, 1, 1)
    m = (1.0 / (c * c)).contiguous()
    b = (b_lay * (c / c_ref)).contiguous()
    m_ref = (1.0 / (c_ref * c_ref)).contiguous()
    b_ref = torch.ones_like(m_ref)
    bmax = max(float(b.max()), 1.0)
    mmin = min(float(m.min()), float(m_ref.min()))
    dt = bound_frac / math.sqrt(3.0 * bmax / mmin)
    slow = math.sqrt(min(float(b.min()), 1.0) / max(float(m.max()), float(m_ref.max())))
    src = flat(shape, [[0, n // 2, n // 2]])
    h = rec_every // 2
    rec = flat(shape, [[0, rec_every * a + h, rec_every * q + h]
                       for a in range(n // rec_every) for q in range(n // rec_every)])
    wavelet = ricker(nt, dt, slow / 20.0).reshape(nt, 1)
    return dict(shape=shape, dx=1.0, dt=dt, nt=nt, m=m, b=b, m_ref=m_ref, b_ref=b_ref, src=src,
                rec=rec, wavelet=wavelet)


def _layered_perturbed_torch(shape, seed, device, n_layers=8, c_lo=1.5, c_hi=4.5,
                             sigma=8.0, amp=0.05):
    """Device-side twin of ``layered_perturbed`` for grids too large for host smoothing:
    same recipe, torch's generator instead of numpy's (float32 result)."""
    import torch
    base_prof = layered_speed((shape[0], 1), n_layers, c_lo, c_hi, seed)[:, 0]
    g = torch.Generator(device=device)
    g.manual_seed(seed + 1)
    p = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    rad = int(math.ceil(4 * sigma))
    x = torch.arange(-rad, rad + 1, device=device, dtype=torch.float32)
    ker = torch.exp(-0.5 * (x / sigma) ** 2)
    ker = ker / ker.sum()
    for ax in range(len(shape)):
        p = _smooth_axis(p, ker, rad, ax)
    p = p / p.abs().max()
    base = torch.as_tensor(base_prof, device=device, dtype=torch.float32)
    base = base.view((shape[0],) + (1,) * (len(shape) - 1)).expand(shape)
    c = base * (1.0 + amp * p)
    return c.contiguous(), base.contiguous()


def _smooth_axis(p, ker, rad, ax):
    """1D convolution of ``p`` along ``ax`` with reflecting edges (numpy's and
    scipy's "reflect": the edge sample repeats), as a sum of shifted slices."""
    import torch
    n = p.shape[ax]
    idx = torch.arange(-rad, n + rad, device=p.device)
    idx = torch.where(idx < 0, -1 - idx, idx)
    idx = torch.where(idx >= n, 2 * n - 1 - idx, idx)
    padded = torch.index_select(p, ax, idx)
    out = torch.zeros_like(p)
    for j in range(2 * rad + 1):
        out.add_(padded.narrow(ax, j, n), alpha=float(ker[j]))
    return out


def small_random(shape, order: int = 8, nt: int = 60, dtype: str = "f32", seed: int = 0,
                 nsrc: int = 2, nrec: int = 7, courant: float = 0.4) -> Problem:
    """Tiny heterogeneous problem with random cells for sources and receivers
    (duplicates and wall cells included on purpose), for parity edge cases."""
    rng = np.random.default_rng(seed)
    c = 1.0 + rng.random(shape)
    c_ref = np.full(shape, 1.5)
    dt = time_step(c.max(), 1.0, courant)
    n = int(np.prod(shape))
    src = rng.integers(0, n, size=nsrc).astype(np.int64)
    rec = rng.integers(0, n, size=nrec).astype(np.int64)
    if nrec >= 2:
        rec[-1] = rec[0]                       # a duplicate receiver
    if nsrc >= 1 and nrec >= 3:
        rec[1] = src[0]                        # a receiver on a source cell
    wavelet = rng.standard_normal((nt, nsrc))
    return Problem("random", tuple(shape), order, dtype, 1.0, dt, nt, c, c_ref, src, rec,
                   wavelet, meta={"courant": courant, "seed": seed})


def sine_burst(nt: int, dt: float, freq: float, cycles: int, amp: float) -> np.ndarray:
    """The sine burst of Eq. source2: amp sin(w t) sin^2(w t / (2 cycles)) for
    0 <= t <= 2 pi cycles / w, zero after; w = 2 pi freq, t = n dt.  [nt]."""
    t = np.arange(nt) * dt
    w = 2.0 * np.pi * freq
    s = amp * np.sin(w * t) * np.sin(w * t / (2 * cycles)) ** 2
    s[t > 2.0 * np.pi * cycles / w] = 0.0
    return s


# Air and the solid of the topology-optimisation example (Sec. 2.3): densities and
# bulk moduli (the solid's modulus as reduced in the paper for larger time steps).
TATO_MATERIALS = dict(rho1=1.204, rho2=2643.0, kappa1=1.419e5, kappa2=6.87e8)


def tato_2d(n0: int = 2703, n1: int = 5403, nt: int = 17184, dx: float = 1.0 / 300.0,
            dt: float = 4.58e-6) -> dict:
    """The two-dimensional acoustic black-hole problem at the paper's size (Tab.
    problemsetupTopOpt: 18 m x 9 m, 5403 x 2703 grid points, N = 17184 steps,
    dt ~ 4.58e-6 s, 5 kHz two-cycle sine burst of amplitude 1e2 s^-2).  The paper gives
    the layout only as a figure; here: axis 1 (contiguous) is the 18 m side, the
    source sits at mid-depth 3 m from the left wall, the design box covers 6..12 m by
    1.5..7.5 m, and the objective region is a 0.5 m x 0.5 m box centred 14.75 m from the
    left wall at mid-depth.  Returns host data: shape, dx, dt, nt, src, wavelet [nt, 1],
    design box (origin, extent), region box (origin, extent), materials."""
    shape = (n0, n1)
    cells = lambda metres: int(round(metres / dx))   # noqa: E731
    src = flat(shape, [[n0 // 2, cells(3.0)]])
    origin = (cells(1.5), cells(6.0))
    extent = (min(cells(6.0), n0 - origin[0]), min(cells(6.0), n1 - origin[1]))
    r_ext = (cells(0.5), cells(0.5))
    r_org = (n0 // 2 - r_ext[0] // 2, cells(14.75) - r_ext[1] // 2)
    wavelet = sine_burst(nt, dt, 5000.0, 2, 1e2).reshape(nt, 1)
    return dict(shape=shape, dx=dx, dt=dt, nt=nt, src=src, wavelet=wavelet, design_origin=origin,
                design_extent=extent, region_origin=r_org, region_extent=r_ext, materials=dict(TATO_MATERIALS))


def fwi_3d(n0: int = 976, n1: int = 503, n2: int = 503, nt: int = 7200, dt: float = 9e-9, seed: int = 11,
           n_voids: int = 24, rec_every: int = 8, dx: float = 0.05 / 503, device=None) -> dict:
    """A stand-in for the paper's three-dimensional FWI specimen at its size (Tab.
    problemsetupFWI: 0.05 m x 0.05 m x 0.0973 m, 503 x 503 x 976 grid points, N = 7200,
    dt = 9e-9 s, 2 MHz two-cycle sine burst of 1e12, rho-scaling with rho0 = 2700,
    c0 = 6000).  The CT scan is not available: the true indicator is a solid cylinder
    along axis 0 (radius 0.45 of the side, gamma = 1, void gamma = 1e-5 outside) holding
    ``n_voids`` seeded spherical voids (radius 6..20 cells, less on small grids) and the paper's added
    16 x 16 x 16 cubical void at the centre; the starting design is the cylinder without
    voids.  Source at the centre of the top face (x0 = 0), receivers on the top and
    bottom faces every ``rec_every`` cells; cells of the paper's size (0.05 m / 503)
    whatever the extents.  gamma fields are float32 on ``device``."""
    import torch
    shape = (n0, n1, n2)
    rng = np.random.default_rng(seed)
    y = torch.arange(n1, device=device, dtype=torch.float32).view(1, n1, 1) - (n1 - 1) / 2
    z = torch.arange(n2, device=device, dtype=torch.float32).view(1, 1, n2) - (n2 - 1) / 2
    inside = (y * y + z * z) <= (0.45 * n1) ** 2
    eps = 1e-5
    start = torch.where(inside, 1.0, eps).expand(shape).contiguous()
    true = start.clone()
    x = torch.arange(n0, device=device, dtype=torch.float32).view(n0, 1, 1)
    r_hi = min(20.0, 0.15 * n1)
    for _ in range(n_voids):
        r = float(rng.uniform(min(6.0, r_hi / 2), r_hi))
        cx = float(rng.uniform(r, n0 - r))
        ang, rad = rng.uniform(0, 2 * np.pi), rng.uniform(0, 0.45 * n1 - r)
        cy, cz = rad * np.cos(ang), rad * np.sin(ang)
        ball = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r
        true = torch.where(ball, eps, true)
    c0, c1, c2 = n0 // 2, n1 // 2, n2 // 2
    true[c0 - 8:c0 + 8, c1 - 8:c1 + 8, c2 - 8:c2 + 8] = eps
    src = flat(shape, [[0, c1, c2]])
    h = rec_every // 2
    face = [[a, rec_every * i + h, rec_every * j + h] for a in (0, n0 - 1)
            for i in range(n1 // rec_every) for j in range(n2 // rec_every)]
    rec = flat(shape, face)
    wavelet = sine_burst(nt, dt, 2e6, 2, 1e12).reshape(nt, 1)
    return dict(shape=shape, dx=dx, dt=dt, nt=nt, src=src, rec=rec, wavelet=wavelet, gamma_true=true.contiguous(),
                gamma_start=start, rho0=2700.0, c0=6000.0, eps=eps)
