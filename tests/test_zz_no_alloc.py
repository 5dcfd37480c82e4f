"""fd_adjoint_sensitivity_noalloc: the gradient with every scratch array in the
library's fixed per-device array.  Two calls in a row (the second on a smaller
problem) equal fd_adjoint_sensitivity on the same inputs and the oracle, take nothing
from the stream-ordered pool, and a problem beyond the array is refused with an
error that names both sizes."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2509_15744_amd import workloads as wl
from helpers import rel, say, to_dev

pytestmark = pytest.mark.gpu

USED_CURRENT, USED_HIGH = 0x7, 0x8   # hipMemPoolAttrUsedMemCurrent, hipMemPoolAttrUsedMemHigh


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def _pool_peak_reset():
    hip = ctypes.CDLL("libamdhip64.so")
    pool = ctypes.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(ctypes.byref(pool), torch.cuda.current_device()) == 0
    v = ctypes.c_uint64()
    assert hip.hipMemPoolGetAttribute(pool, USED_CURRENT, ctypes.byref(v)) == 0
    zero = ctypes.c_uint64(0)
    assert hip.hipMemPoolSetAttribute(pool, USED_HIGH, ctypes.byref(zero)) == 0

    def grown():
        h = ctypes.c_uint64()
        assert hip.hipMemPoolGetAttribute(pool, USED_HIGH, ctypes.byref(h)) == 0
        return max(0, h.value - v.value)
    return grown


def _case(fdw, q, dtype, k):
    obs, _, _ = oracle.forward(q.c_ref, q.dx, q.order, q.dt, q.nt, q.src, q.wavelet, q.rec)
    g_o, J_o, tr_o = oracle.superposition_gradient(q.c, q.dx, q.order, q.dt, q.nt, q.src, q.wavelet, q.rec,
                                                   obs, k)
    c, w, o = to_dev(q.c, dtype), to_dev(q.wavelet, dtype), to_dev(obs, dtype)
    return c, w, o, g_o, J_o, tr_o


def test_noalloc_matches_the_allocating_call(fdw):
    cases = [  # the second problem is smaller than the first
        (wl.small_random((30, 22, 70), order=8, nt=40, dtype="f32", seed=3), torch.float32, 1e-4),
        (wl.small_random((40, 66), order=4, nt=50, dtype="f64", seed=4), torch.float64, 1e-9),
    ]
    k = 0.05
    for q, dtype, tol in cases:
        c, w, o, g_o, J_o, tr_o = _case(fdw, q, dtype, k)
        grad = torch.empty_like(c)
        tr = torch.empty((q.nt, len(q.rec)), dtype=dtype, device="cuda")
        g_ref, J_ref = fdw.fd_adjoint_sensitivity(c, q.dx, q.order, q.src, w, q.rec, q.dt, q.nt, o, k)
        torch.cuda.synchronize()
        grown = _pool_peak_reset()
        say("noalloc", q.shape, dtype)
        g, J = fdw.fd_adjoint_sensitivity_noalloc(c, q.dx, q.order, q.src, w, q.rec, q.dt, q.nt, o, k,
                                                  grad=grad, traces=tr)
        torch.cuda.synchronize()
        assert grown() == 0
        # the same launches as the allocating call: the same result
        assert torch.equal(g, g_ref) and J == J_ref
        assert rel(g.cpu().numpy(), g_o) < tol
        assert rel(tr.cpu().numpy(), tr_o) < tol
        assert abs(J - J_o) < tol * J_o


def test_noalloc_refuses_problems_beyond_the_array(fdw):
    q = wl.small_random((256, 128, 256), order=8, nt=4, dtype="f32", seed=5)
    f32 = torch.float32
    c, w = to_dev(q.c, f32), to_dev(q.wavelet, f32)
    o = torch.zeros((q.nt, len(q.rec)), dtype=f32, device="cuda")
    with pytest.raises(fdw.FdError) as e:
        fdw.fd_adjoint_sensitivity_noalloc(c, q.dx, q.order, q.src, w, q.rec, q.dt, q.nt, o, 0.05)
    assert e.value.code == fdw.FD_E_ARG and "FD_NOALLOC_BYTES" in str(e.value)
    # the array is intact: a small call still matches after the refusal
    q = wl.small_random((20, 90), order=8, nt=30, dtype="f64", seed=6)
    c, w, o, g_o, J_o, _ = _case(fdw, q, torch.float64, 0.05)
    g, J = fdw.fd_adjoint_sensitivity_noalloc(c, q.dx, q.order, q.src, w, q.rec, q.dt, q.nt, o, 0.05)
    assert rel(g.cpu().numpy(), g_o) < 1e-9
