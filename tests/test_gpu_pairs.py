"""Two time steps per launch (fd_opts.pairs): the constant-density 3D sweeps of one shot
advance levels n+1 and n+2 in one launch, recomputing level n+1 on a ring of width r
around each tile.  The results equal those of one step per launch bit for bit (the
same arithmetic in the same order, the ring cells past a wall standing for the mirrored
cells), and the oracle's Alg. 1 to rounding: ragged extents (padded rows, partial tiles,
extents down to twice the stencil radius), sources and receivers on walls, edges and
corners, odd and even nt, orders 2, 4 and 8, f64 and f32 (f32 partial sums), the fused
call and the two halves."""
import numpy as np
import pytest
import torch

import oracle
from paper_2509_15744_amd import workloads as wl
from helpers import rel, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def _walls(shape, rng, n):
    """Cells on faces, edges and corners of the grid."""
    cells = []
    for _ in range(n):
        c = [int(rng.integers(0, s)) for s in shape]
        for ax in rng.choice(3, size=int(rng.integers(1, 4)), replace=False):
            c[ax] = 0 if rng.random() < 0.5 else shape[ax] - 1
        cells.append(c)
    return wl.flat(shape, cells)


CASES = [
    # shape, order, nt, dtype
    ((24, 20, 70), 8, 31, "f64"),
    ((24, 20, 70), 8, 30, "f32"),
    ((17, 9, 130), 4, 25, "f64"),
    ((8, 8, 8), 8, 12, "f64"),       # every extent = 2r: the ring reaches past both walls
    ((40, 16, 64), 2, 41, "f32"),
    ((70, 13, 66), 8, 2, "f64"),
    ((70, 13, 66), 8, 3, "f32"),
]


@pytest.mark.parametrize("shape,order,nt,dtype", CASES)
def test_pairs_equal_one_step_and_oracle(fdw, shape, order, nt, dtype):
    rng = np.random.default_rng(sum(shape) + order + nt)
    q = wl.small_random(shape, order=order, nt=nt, dtype=dtype, seed=int(rng.integers(1 << 30)), nsrc=3, nrec=9)
    src = np.concatenate([q.src, _walls(shape, rng, 3)])
    rec = np.concatenate([q.rec, _walls(shape, rng, 9)])
    wav = np.concatenate([q.wavelet, rng.standard_normal((nt, 3))], axis=1)
    obs, _, _ = oracle.forward(q.c_ref, q.dx, order, q.dt, nt, src, wav, rec)
    # f32 loses digits in the differences of the superposed field as k shrinks; the
    # larger f32 k keeps its rounding below the 1e-4 bound on the shortest runs
    k = 0.05 if dtype == "f64" else 0.4
    g_o, J_o, tr_o = oracle.superposition_gradient(q.c, q.dx, order, q.dt, nt, src, wav, rec, obs, k)
    t = torch.float64 if dtype == "f64" else torch.float32
    c, w, o = to_dev(q.c, t), to_dev(wav, t), to_dev(obs, t)
    tr1 = torch.empty((nt, len(rec)), dtype=t, device="cuda")
    tr2 = torch.empty_like(tr1)
    say("pairs", shape, order, nt, dtype)
    g1, J1 = fdw.fd_adjoint_sensitivity(c, q.dx, order, src, w, rec, q.dt, nt, o, k, traces=tr1, pairs=-1)
    tm = fdw.fd_timing()
    g2, J2 = fdw.fd_adjoint_sensitivity(c, q.dx, order, src, w, rec, q.dt, nt, o, k, traces=tr2, pairs=1, timing=tm)
    torch.cuda.synchronize()
    assert tm.fwd_pair_launches == nt // 2 and tm.bwd_pair_launches == (nt - 1) // 2
    assert torch.equal(tr1, tr2), float((tr1 - tr2).abs().max())
    assert J1 == J2
    assert torch.equal(g1, g2), float((g1 - g2).abs().max())
    tol = 1e-9 if dtype == "f64" else 1e-4
    assert rel(tr2.cpu().numpy(), tr_o) < (1e-12 if dtype == "f64" else 1e-5)
    assert rel(g2.cpu().numpy(), g_o) < tol
    assert abs(J2 - J_o) < tol * J_o


@pytest.mark.parametrize("nt", [20, 21])
def test_pairs_split_halves(fdw, nt):
    """The two halves with caller-owned state and two steps per launch equal the fused
    call (the forward half leaves u^{nt-1}, u^nt where the backward half expects them,
    whatever the parity of the number of two-step launches)."""
    shape = (30, 12, 100)
    q = wl.small_random(shape, order=8, nt=nt, dtype="f32", seed=nt)
    obs, _, _ = oracle.forward(q.c_ref, q.dx, 8, q.dt, nt, q.src, q.wavelet, q.rec)
    f32 = torch.float32
    c, w, o = to_dev(q.c, f32), to_dev(q.wavelet, f32), to_dev(obs, f32)
    say("pairs halves", nt)
    g, J = fdw.fd_adjoint_sensitivity(c, q.dx, 8, q.src, w, q.rec, q.dt, nt, o, 0.05, pairs=1)
    st = fdw.SweepState(c, nt, len(q.rec))
    J2 = fdw.fd_sens_forward(c, q.dx, 8, q.src, w, q.rec, q.dt, nt, o, st, pairs=1)
    st1 = fdw.SweepState(c, nt, len(q.rec))
    fdw.fd_sens_forward(c, q.dx, 8, q.src, w, q.rec, q.dt, nt, o, st1, pairs=-1)
    torch.cuda.synchronize()
    # the forward half's end levels, accumulator and residuals equal the one-step half's
    for name in ("u_a", "u_b", "acc", "residual"):
        assert torch.equal(getattr(st, name), getattr(st1, name)), name
    g2 = fdw.fd_sens_backward(c, q.dx, 8, q.src, w, q.rec, q.dt, nt, 0.05, st, pairs=1)
    torch.cuda.synchronize()
    assert J2 == J and torch.equal(g2, g)
