"""FP32 parity at the full time horizon of the layered workloads, against FP64 oracle
references written by tests/golden/make_horizon.py (oracle only):

* 2048^2, order 8, nt = 4000, 512 receivers on the top row;
* 256^3, order 8, nt = 3000, the 3D layered recipe, a receiver plane every 16 cells.

The device runs in f32 with the f64 accumulator, in the launch shape the autotuner
picks for the grid (as the bench does), on exactly the inputs the oracle saw (speeds,
wavelet and observed data rounded to float32).  Bound: relative L2 <= 1e-4 on the
traces, the superposition gradient at the oracle's k and the exact (re-simulated)
gradient; J to 1e-5; the gap between them matches the oracle's.  These are the
long-horizon cases where f32 phase drift and the cancellation of K(v,v) - K(u,u)
would show (Sec. 4.1)."""
import os

import numpy as np
import pytest
import torch

from paper_2509_15744_amd import workloads as wl
from helpers import rel, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CASES = {
    "layered2d_2048_nt4000": lambda: wl.layered_2d(n=2048, nt=4000),
    "layered3d_256_nt3000": lambda: wl.layered_3d(n=256, nt=3000, rec_every=16),
}


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp32_full_horizon(fdw, name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not written yet (tests/golden/make_horizon.py)")
    ref = np.load(path)
    p = CASES[name]()
    f32 = torch.float32
    c = torch.as_tensor(np.asarray(p.c, dtype=np.float32)).cuda()
    w = torch.as_tensor(np.asarray(p.wavelet, dtype=np.float32)).cuda()
    obs = torch.as_tensor(ref["observed"]).cuda()
    assert obs.dtype == f32 and obs.shape == (p.nt, len(p.rec))
    k = float(ref["k"])
    best, _ = fdw.fd_autotune(p.shape, p.dx, p.order, f32, nshot=1, steps=4)
    shape = {key: best[key] for key in ("variant", "chunk", "max_group", "variant_plain", "chunk_plain")}
    say("horizon", name, "k", k, "launch shape", shape)
    tr = torch.empty((p.nt, len(p.rec)), dtype=f32, device="cuda")
    g, J = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, k, traces=tr, **shape)
    say("horizon exact", name)
    g_ex, J_ex = fdw.fd_adjoint_exact(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs)
    torch.cuda.synchronize()
    st = int(ref["stride"])
    rs = int(ref["rec_stride"])
    s = (slice(None, None, st),) * len(p.shape)
    ap = g[s].double().cpu().numpy()
    ex = g_ex[s].double().cpu().numpy()
    e_tr = rel(tr[:, ::rs].double().cpu().numpy(), ref["traces_sample"])
    e_ap = rel(ap, ref["approx_sample"])
    e_ex = rel(ex, ref["exact_sample"])
    e_J = abs(J - float(ref["J"])) / float(ref["J"])
    gap_dev = rel(ap, ex)
    gap_or = rel(ref["approx_sample"], ref["exact_sample"])
    say(f"  traces {e_tr:.3e}  grad {e_ap:.3e}  exact {e_ex:.3e}  J {e_J:.3e}  "
        f"gap {gap_dev:.5f} (oracle {gap_or:.5f}, full field {float(ref['gap_norm'] / ref['exact_norm']):.5f})")
    assert e_tr <= 1e-4
    assert e_ap <= 1e-4
    assert e_ex <= 1e-4
    assert e_J <= 1e-5 and abs(J_ex - J) <= 1e-5 * J
    assert abs(gap_dev - gap_or) <= 2e-4
