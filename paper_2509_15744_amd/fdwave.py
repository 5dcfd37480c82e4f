"""ctypes binding of ``libfdwave.so`` (declared in ``include/fdwave.h``).

Argument marshalling only: torch tensors become device pointers, index arrays
become host int64 arrays, and every call runs on torch's current HIP stream.
All arithmetic happens in the library's HIP kernels.  Importing this module
raises if the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdwave.so")

FD_OK, FD_E_ARG, FD_E_CFL, FD_E_NOMEM, FD_E_DEVICE, FD_E_NONFINITE = 0, 1, 2, 3, 4, 5
FD_F32, FD_F64 = 0, 1
_CODES = {1: "FD_E_ARG", 2: "FD_E_CFL", 3: "FD_E_NOMEM", 4: "FD_E_DEVICE", 5: "FD_E_NONFINITE"}


class FdError(RuntimeError):
    """A non-zero return code of the library, with its fd_last_error() text."""

    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class fd_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int64 * 3), ("dx", ctypes.c_double),
                ("order", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class fd_acq(ctypes.Structure):
    _fields_ = [("nsrc", ctypes.c_int32), ("src_cell", ctypes.POINTER(ctypes.c_int64)),
                ("wavelet", ctypes.c_void_p), ("nrec", ctypes.c_int32),
                ("rec_cell", ctypes.POINTER(ctypes.c_int64))]


class fd_timing(ctypes.Structure):
    _fields_ = [("fwd_ms", ctypes.c_double), ("fwd_launches", ctypes.c_int32),
                ("bwd_ms", ctypes.c_double), ("bwd_launches", ctypes.c_int32)]


class fd_opts(ctypes.Structure):
    _fields_ = [("acc_dtype", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("timing", ctypes.POINTER(fd_timing)), ("chunk", ctypes.c_int32)]


class fd_state(ctypes.Structure):
    _fields_ = [("u_a", ctypes.c_void_p), ("u_b", ctypes.c_void_p), ("acc", ctypes.c_void_p),
                ("residual", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2509_15744_amd.build` (no fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    G, A, O, S = (ctypes.POINTER(fd_grid), ctypes.POINTER(fd_acq), ctypes.POINTER(fd_opts),
                  ctypes.POINTER(fd_state))
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "fd_last_error": ([], ctypes.c_char_p),
        "fd_cfl_limit": ([I, I], D),
        "fd_variant_count": ([I], I),
        "fd_forward": ([G, P, A, D, I, P, O, P], ctypes.c_int),
        "fd_misfit": ([I, I, I, D, P, P, P, DP, P], ctypes.c_int),
        "fd_adjoint_sensitivity": ([G, P, A, D, I, P, D, P, DP, P, O, P], ctypes.c_int),
        "fd_sens_forward": ([G, P, A, D, I, P, S, P, DP, O, P], ctypes.c_int),
        "fd_sens_backward": ([G, P, A, D, I, D, S, D, P, O, P], ctypes.c_int),
        "fd_propagate": ([G, P, P, P, I, O, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _raise(rc):
    if rc != FD_OK:
        raise FdError(rc, _lib.fd_last_error().decode())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return FD_F32
    if t.dtype == torch.float64:
        return FD_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, what):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_grid(shape, dx, order, dtype_code) -> fd_grid:
    g = fd_grid()
    g.ndim = len(shape)
    for i, s in enumerate(shape):
        g.shape[i] = int(s)
    g.dx = float(dx)
    g.order = int(order)
    g.dtype = int(dtype_code)
    return g


class Acquisition:
    """Host cell arrays + device wavelet, kept alive for the duration of calls."""

    def __init__(self, src_cells, wavelet: torch.Tensor, rec_cells):
        self.src = np.ascontiguousarray(np.asarray(src_cells, dtype=np.int64).reshape(-1))
        self.rec = np.ascontiguousarray(np.asarray(rec_cells, dtype=np.int64).reshape(-1))
        self.wavelet = wavelet
        a = fd_acq()
        a.nsrc = len(self.src)
        a.src_cell = self.src.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        a.wavelet = _dev(wavelet, "wavelet") if len(self.src) else None
        a.nrec = len(self.rec)
        a.rec_cell = self.rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        self.c = a


def make_opts(acc_dtype=None, variant=0, timing: "fd_timing | None" = None, chunk=0) -> fd_opts:
    o = fd_opts()
    o.chunk = int(chunk)
    if timing is not None:
        o.timing = ctypes.pointer(timing)
    if acc_dtype is None or acc_dtype in ("f64", torch.float64, FD_F64):
        o.acc_dtype = FD_F64
    elif acc_dtype in ("f32", torch.float32, FD_F32):
        o.acc_dtype = FD_F32
    else:
        raise ValueError(f"acc_dtype {acc_dtype!r}")
    o.variant = int(variant)
    return o


def fd_cfl_limit(ndim: int, order: int) -> float:
    return float(_lib.fd_cfl_limit(ndim, order))


def fd_variant_count(ndim: int) -> int:
    return int(_lib.fd_variant_count(ndim))


def fd_forward(c, dx, order, src, wavelet, rec, dt, nt, traces=None, acc_dtype=None, variant=0,
               timing=None, chunk=0):
    """Receiver traces [nt, nrec] of the forward solve."""
    acq = Acquisition(src, wavelet, rec)
    if traces is None:
        traces = torch.empty((nt, len(acq.rec)), dtype=c.dtype, device=c.device)
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(acc_dtype, variant, timing, chunk)
    _raise(_lib.fd_forward(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt),
                           _dev(traces, "traces"), ctypes.byref(o), _stream()))
    return traces


def fd_misfit(traces, observed, dt, residual=None) -> float:
    """J = dt/2 sum (traces - observed)^2; fills ``residual`` when given."""
    nt, nrec = traces.shape
    J = ctypes.c_double()
    _raise(_lib.fd_misfit(int(nt), int(nrec), _dtype_code(traces), float(dt),
                          _dev(traces, "traces"), _dev(observed, "observed"),
                          _dev(residual, "residual"), ctypes.byref(J), _stream()))
    return J.value


def fd_adjoint_sensitivity(c, dx, order, src, wavelet, rec, dt, nt, observed, k, grad=None,
                           traces=None, acc_dtype=None, variant=0, timing=None, chunk=0):
    """(grad_c, J) of the memory-efficient method at factor ``k``."""
    acq = Acquisition(src, wavelet, rec)
    if grad is None:
        grad = torch.empty_like(c)
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(acc_dtype, variant, timing, chunk)
    J = ctypes.c_double()
    _raise(_lib.fd_adjoint_sensitivity(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt),
                                       int(nt), _dev(observed, "observed"), float(k),
                                       _dev(grad, "grad"), ctypes.byref(J), _dev(traces, "traces"),
                                       ctypes.byref(o), _stream()))
    return grad, J.value


class SweepState:
    """Caller-owned device state between fd_sens_forward and fd_sens_backward."""

    def __init__(self, c: torch.Tensor, nt: int, nrec: int, acc_dtype=None):
        acc_t = torch.float32 if (make_opts(acc_dtype).acc_dtype == FD_F32
                                  and c.dtype == torch.float32) else torch.float64
        self.u_a = torch.empty_like(c)
        self.u_b = torch.empty_like(c)
        self.acc = torch.empty(c.shape, dtype=acc_t, device=c.device)
        self.residual = torch.empty((nt, nrec), dtype=c.dtype, device=c.device)

    def c_struct(self) -> fd_state:
        s = fd_state()
        s.u_a = self.u_a.data_ptr()
        s.u_b = self.u_b.data_ptr()
        s.acc = self.acc.data_ptr()
        s.residual = self.residual.data_ptr()
        return s


def fd_sens_forward(c, dx, order, src, wavelet, rec, dt, nt, observed, state: SweepState,
                    traces=None, acc_dtype=None, variant=0, timing=None, chunk=0) -> float:
    acq = Acquisition(src, wavelet, rec)
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(acc_dtype, variant, timing, chunk)
    st = state.c_struct()
    J = ctypes.c_double()
    _raise(_lib.fd_sens_forward(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt),
                                _dev(observed, "observed"), ctypes.byref(st), _dev(traces, "traces"),
                                ctypes.byref(J), ctypes.byref(o), _stream()))
    return J.value


def fd_sens_backward(c, dx, order, src, wavelet, rec, dt, nt, k, state: SweepState, grad_scale=1.0,
                     grad=None, acc_dtype=None, variant=0, timing=None, chunk=0):
    acq = Acquisition(src, wavelet, rec)
    if grad is None:
        grad = torch.empty_like(c)
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(acc_dtype, variant, timing, chunk)
    st = state.c_struct()
    _raise(_lib.fd_sens_backward(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt),
                                 float(k), ctypes.byref(st), float(grad_scale), _dev(grad, "grad"),
                                 ctypes.byref(o), _stream()))
    return grad


def fd_propagate(coef, u_prev, u_cur, nsteps, dx, order, variant=0, chunk=0):
    """In place: (u_prev, u_cur) advance by ``nsteps`` source-free steps."""
    g = make_grid(coef.shape, dx, order, _dtype_code(coef))
    o = make_opts(None, variant, None, chunk)
    _raise(_lib.fd_propagate(ctypes.byref(g), _dev(coef, "coef"), _dev(u_prev, "u_prev"),
                             _dev(u_cur, "u_cur"), int(nsteps), ctypes.byref(o), _stream()))
    return u_prev, u_cur
