"""fd_workspace_bytes bounds what one fd_adjoint_sensitivity call takes from the
stream-ordered pool: the default pool's high-water mark of used memory (reset before
the call, HIP's hipMemPoolAttrUsedMemHigh) minus what was in use before is at most the
bound, and close to it (the state arrays dominate)."""
import ctypes

import numpy as np
import pytest
import torch

from helpers import say, shot_problem, to_dev

pytestmark = pytest.mark.gpu

USED_CURRENT, USED_HIGH = 0x7, 0x8   # hipMemPoolAttrUsedMemCurrent, hipMemPoolAttrUsedMemHigh


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def _pool():
    hip = ctypes.CDLL("libamdhip64.so")
    pool = ctypes.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(ctypes.byref(pool), torch.cuda.current_device()) == 0
    return hip, pool


def _attr(hip, pool, which):
    v = ctypes.c_uint64()
    assert hip.hipMemPoolGetAttribute(pool, which, ctypes.byref(v)) == 0
    return v.value


@pytest.mark.parametrize("shape,nshot,order", [((24, 20, 70), 3, 8), ((130, 96), 1, 4)])
def test_workspace_bound_covers_the_pool_peak(fdw, shape, nshot, order):
    P = shot_problem(shape, nshot, order, 40, "f32", seed=7)
    hip, pool = _pool()
    torch.cuda.synchronize()
    before = _attr(hip, pool, USED_CURRENT)
    zero = ctypes.c_uint64(0)
    assert hip.hipMemPoolSetAttribute(pool, USED_HIGH, ctypes.byref(zero)) == 0
    say("workspace", shape, nshot, order)
    f32 = torch.float32
    shots = (P["src_shot"], P["rec_shot"], nshot) if nshot > 1 else None
    fdw.fd_adjoint_sensitivity(to_dev(P["c"], f32), 1.0, order, P["src"], to_dev(P["wavelet"], f32), P["rec"],
                               P["dt"], P["nt"], to_dev(P["obs"], f32), 0.05, shots=shots)
    torch.cuda.synchronize()
    used = _attr(hip, pool, USED_HIGH) - before
    bound = fdw.fd_workspace_bytes(shape, order, fdw.FD_F32, P["nt"], nsrc=len(P["src"]), nrec=len(P["rec"]),
                                   nshots=nshot)
    # wavefields, f64 accumulator, f32 partial sums of the kernel terms, residual rows
    state = 2 * nshot * int(np.prod(shape)) * 4 + int(np.prod(shape)) * 12 + P["nt"] * len(P["rec"]) * 4
    assert state <= used <= bound, (state, used, bound)
