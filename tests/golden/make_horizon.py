"""Write the long-horizon FP64 references of the layered workloads:

* ``layered2d_2048_nt4000.npz``: 2048^2, order 8, nt = 4000, c_max dt/dx = 0.5, eight
  random layers times a 5% smoothed perturbation, one Ricker source at the top centre,
  512 receivers on the top row (every 4th cell);
* ``layered3d_256_nt3000.npz``: the same recipe in 3D at 256^3, order 8, nt = 3000,
  c_max dt/dx = 0.4, source at the top-face centre, a receiver plane on x0 = 0 every
  16 cells (256 receivers).

Calls only ``oracle`` and the input generators.  The oracle is fed exactly what an f32
device run is fed: speeds, wavelet and observed data rounded to float32 first.  The
observed data are the oracle's traces in the unperturbed layers, rounded to float32
and stored whole (they are an input of the gradient).  Stored besides (float64):

* ``k``: factor of the superposition, k = 0.005 ||f|| / ||fdag|| with
  ||f|| = ||wavelet|| / dx^d and ||fdag|| = sqrt(2 J / dt) / dt;
* ``J``: the misfit of the FP64 forward solve in the perturbed medium;
* ``traces_sample``: its traces at every ``rec_stride``-th receiver, all nt levels;
* ``exact_sample``, ``approx_sample``: dJ/dc of the exact discrete adjoint (uniform
  checkpoints) and of the superposition at ``k`` on every ``stride``-th cell per axis;
* ``exact_norm``, ``approx_norm``, ``gap_norm``: full-field L2 norms of the exact
  gradient, the approximation and their difference.

Run from the repository root: ``python tests/golden/make_horizon.py [2d|3d]`` (on 8
cores about 12 minutes for 2d and 45 minutes for 3d; the 3d case takes ~25 GB of host
memory).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_15744_amd import workloads as wl  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
BETA = 0.005

CASES = {
    "2d": dict(out="layered2d_2048_nt4000.npz", make=lambda: wl.layered_2d(n=2048, nt=4000),
               stride=8, rec_stride=8, seg=64),
    "3d": dict(out="layered3d_256_nt3000.npz",
               make=lambda: wl.layered_3d(n=256, nt=3000, rec_every=16),
               stride=8, rec_stride=4, seg=55),
}


def r32(x):
    """The value an f32 device array holds, back in float64."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def run(name):
    case = CASES[name]
    t0 = time.time()
    p = case["make"]()
    c, c_ref, w = r32(p.c), r32(p.c_ref), r32(p.wavelet)
    nd = len(p.shape)
    print(f"[{name}] inputs {time.time() - t0:.1f}s, grid {p.shape}, nt {p.nt}, "
          f"{len(p.rec)} receivers, threads {oracle.num_threads()}", flush=True)
    obs_full, _, _ = oracle.forward(c_ref, p.dx, p.order, p.dt, p.nt, p.src, w, p.rec)
    obs32 = obs_full.astype(np.float32)
    obs = obs32.astype(np.float64)
    print(f"[{name}] observed {time.time() - t0:.1f}s", flush=True)
    g_ex, J, _, traces = oracle.exact_gradient_ckpt(c, p.dx, p.order, p.dt, p.nt, p.src, w,
                                                    p.rec, obs, seg=case["seg"])
    print(f"[{name}] exact {time.time() - t0:.1f}s J={J:.9e}", flush=True)
    f_norm = float(np.linalg.norm(w)) / p.dx ** nd
    k = BETA * f_norm / (np.sqrt(2.0 * J / p.dt) / p.dt)
    g_ap, J_ap, _ = oracle.superposition_gradient(c, p.dx, p.order, p.dt, p.nt, p.src, w, p.rec,
                                                  obs, k)
    print(f"[{name}] approx {time.time() - t0:.1f}s k={k:.6e}", flush=True)
    s = (slice(None, None, case["stride"]),) * nd
    rs = case["rec_stride"]
    out = os.path.join(HERE, case["out"])
    np.savez_compressed(
        out, k=np.float64(k), J=np.float64(J), J_approx=np.float64(J_ap),
        stride=np.int64(case["stride"]), rec_stride=np.int64(rs), observed=obs32,
        traces_sample=traces[:, ::rs].copy(),
        exact_sample=g_ex[s].copy(), approx_sample=g_ap[s].copy(),
        exact_norm=np.float64(np.linalg.norm(g_ex)), approx_norm=np.float64(np.linalg.norm(g_ap)),
        gap_norm=np.float64(np.linalg.norm(g_ap - g_ex)))
    print(f"[{name}] wrote {out} ({os.path.getsize(out) / 1e6:.1f} MB); "
          f"gap {np.linalg.norm(g_ap - g_ex) / np.linalg.norm(g_ex):.4e}", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["2d", "3d"]):
        run(name)
