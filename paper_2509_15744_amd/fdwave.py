"""ctypes binding of ``libfdwave.so`` (declared in ``include/fdwave.h``).

Argument marshalling only: torch tensors become device pointers, index arrays
become host int64 arrays, and every call runs on torch's current HIP stream.
All arithmetic happens in the library's HIP kernels.  Importing this module
raises if the library has not been built; there is no fallback path.

Keyword options accepted by the solver calls (``**opts``): ``acc_dtype`` ("f64",
default, or "f32"), ``variant`` (tile variant, 0 = library choice), ``chunk``
(planes per block, 0 = library choice), ``max_group`` (shots per launch, 0/1/2/4),
``graph`` (batched calls: capture each sweep in a hipGraph), ``timing`` (an
``fd_timing`` record to fill).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdwave.so")

FD_OK, FD_E_ARG, FD_E_CFL, FD_E_NOMEM, FD_E_DEVICE, FD_E_NONFINITE = 0, 1, 2, 3, 4, 5
FD_F32, FD_F64 = 0, 1
FD_NOALLOC_BYTES = 64 << 20   # the fixed scratch array of the no-allocation entry point
_CODES = {1: "FD_E_ARG", 2: "FD_E_CFL", 3: "FD_E_NOMEM", 4: "FD_E_DEVICE", 5: "FD_E_NONFINITE"}


class FdError(RuntimeError):
    """A non-zero return code of the library, with its fd_last_error() text."""

    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)


class fd_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int64 * 3), ("dx", ctypes.c_double),
                ("order", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class fd_acq(ctypes.Structure):
    _fields_ = [("nsrc", ctypes.c_int32), ("src_cell", _I64P), ("wavelet", ctypes.c_void_p),
                ("nrec", ctypes.c_int32), ("rec_cell", _I64P), ("nshot", ctypes.c_int32),
                ("src_shot", _I32P), ("rec_shot", _I32P)]


class fd_timing(ctypes.Structure):
    _fields_ = [("fwd_ms", ctypes.c_double), ("fwd_launches", ctypes.c_int32),
                ("bwd_ms", ctypes.c_double), ("bwd_launches", ctypes.c_int32),
                ("fwd_pair_launches", ctypes.c_int32), ("bwd_pair_launches", ctypes.c_int32),
                ("persistent_blocks", ctypes.c_int32)]


class fd_opts(ctypes.Structure):
    _fields_ = [("acc_dtype", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("timing", ctypes.POINTER(fd_timing)), ("chunk", ctypes.c_int32),
                ("max_group", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("barrier_timeout_us", ctypes.c_int32),
                ("variant_plain", ctypes.c_int32), ("chunk_plain", ctypes.c_int32),
                ("no_partials", ctypes.c_int32), ("pairs", ctypes.c_int32)]


class fd_state(ctypes.Structure):
    _fields_ = [("u_a", ctypes.c_void_p), ("u_b", ctypes.c_void_p), ("acc", ctypes.c_void_p),
                ("residual", ctypes.c_void_p)]


class fd_problem(ctypes.Structure):
    _fields_ = [("grid", fd_grid), ("c", ctypes.c_void_p), ("acq", fd_acq), ("dt", ctypes.c_double),
                ("nt", ctypes.c_int32), ("observed", ctypes.c_void_p), ("k", ctypes.c_double),
                ("grad_c", ctypes.c_void_p), ("traces", ctypes.c_void_p)]


class fd_design(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int64 * 3), ("origin", ctypes.c_int64 * 3),
                ("extent", ctypes.c_int64 * 3), ("dtype", ctypes.c_int32), ("filter_radius", ctypes.c_double),
                ("beta", ctypes.c_double), ("eta", ctypes.c_double), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("m0", ctypes.c_double), ("dm", ctypes.c_double),
                ("b0", ctypes.c_double), ("db", ctypes.c_double)]


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
        "fd_workspace_bytes": ([G, A, I, I], ctypes.c_size_t),
        "fd_variant_count": ([I], I),
        "fd_variant_info": ([I, I, _I32P, _I32P, _I32P, _I32P, _I32P], ctypes.c_int),
        "fd_forward": ([G, P, A, D, I, P, O, P], ctypes.c_int),
        "fd_misfit": ([I, I, I, D, P, P, P, DP, P], ctypes.c_int),
        "fd_adjoint_sensitivity": ([G, P, A, D, I, P, D, P, DP, P, O, P], ctypes.c_int),
        "fd_adjoint_sensitivity_noalloc": ([G, P, A, D, I, P, D, P, DP, P, O, P], ctypes.c_int),
        "fd_adjoint_exact": ([G, P, A, D, I, P, P, DP, P, O, P], ctypes.c_int),
        "fd_vd_forward": ([G, P, P, A, D, I, P, O, P], ctypes.c_int),
        "fd_vd_adjoint_sensitivity": ([G, P, P, A, D, I, P, D, P, P, DP, P, O, P], ctypes.c_int),
        "fd_vd_sens_forward": ([G, P, P, A, D, I, P, S, P, P, DP, O, P], ctypes.c_int),
        "fd_vd_sens_backward": ([G, P, P, A, D, I, D, S, P, D, P, P, O, P], ctypes.c_int),
        "fd_sens_forward": ([G, P, A, D, I, P, S, P, DP, O, P], ctypes.c_int),
        "fd_sens_backward": ([G, P, A, D, I, D, S, D, P, O, P], ctypes.c_int),
        "fd_adjoint_sensitivity_batched": ([ctypes.POINTER(fd_problem), I, DP, O, P], ctypes.c_int),
        "fd_batch_plan_create": ([ctypes.POINTER(fd_problem), I, O, P, ctypes.POINTER(P)], ctypes.c_int),
        "fd_batch_run": ([P, P, P], ctypes.c_int),
        "fd_batch_timing": ([P, ctypes.POINTER(fd_timing)], ctypes.c_int),
        "fd_batch_plan_destroy": ([P, P], ctypes.c_int),
        "fd_propagate": ([G, P, P, P, I, O, P], ctypes.c_int),
        "fd_autotune": ([G, I, O, I, O, DP, P], ctypes.c_int),
        "fd_design_map": ([ctypes.POINTER(fd_design), P, P, P, P, P], ctypes.c_int),
        "fd_design_adjoint": ([ctypes.POINTER(fd_design), P, P, P, P, P], ctypes.c_int),
        "fd_adam_step": ([ctypes.c_int64, I, P, P, P, P, I, D, D, D, D, D, D, P], ctypes.c_int),
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


def _fits(t, n, like, what):
    """The library reads or writes n values of the field dtype through t's pointer:
    t (when given) must hold at least n values of like's dtype.  The library's own
    range check sees whole allocator blocks, so undersized tensors are caught here."""
    if t is None:
        return
    if t.dtype != like.dtype:
        raise TypeError(f"{what} is {t.dtype}, the field is {like.dtype}")
    if t.numel() < n:
        raise ValueError(f"{what} has {t.numel()} values, {n} are needed")


def _check_io(field, nt, acq, wavelet=None, observed=None, traces=None, extra_fields=()):
    """Sizes of the arrays a sweep touches: wavelet [nt][nsrc], observed and traces
    [nt][nrec], other grid fields [ncell]."""
    n = field.numel()
    nt = int(nt)
    _fits(wavelet if wavelet is not None else acq.wavelet, nt * acq.c.nsrc, field, "wavelet")
    _fits(observed, nt * acq.c.nrec, field, "observed")
    _fits(traces, nt * acq.c.nrec, field, "traces")
    for what, t in extra_fields:
        _fits(t, n, field, what)


def _check_state(field, nt, acq, state, nshot=1):
    n = field.numel()
    ns = max(int(nshot), 1)
    for what, t, need in (("state.u_a", state.u_a, ns * n), ("state.u_b", state.u_b, ns * n),
                          ("state.residual", state.residual, int(nt) * acq.c.nrec)):
        _fits(t, need, field, what)
    for what in ("acc", "acc_b"):
        t = getattr(state, what, None)
        if t is not None and t.numel() < n:
            raise ValueError(f"state.{what} has {t.numel()} values, {n} are needed")


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
    """Host cell (and shot) arrays + device wavelet, kept alive for the calls."""

    def __init__(self, src_cells, wavelet: torch.Tensor, rec_cells, src_shot=None, rec_shot=None,
                 nshot=0):
        self.src = np.ascontiguousarray(np.asarray(src_cells, dtype=np.int64).reshape(-1))
        self.rec = np.ascontiguousarray(np.asarray(rec_cells, dtype=np.int64).reshape(-1))
        self.wavelet = wavelet
        self.nshot = int(nshot)
        a = fd_acq()
        a.nsrc = len(self.src)
        a.src_cell = self.src.ctypes.data_as(_I64P)
        a.wavelet = _dev(wavelet, "wavelet") if len(self.src) else None
        a.nrec = len(self.rec)
        a.rec_cell = self.rec.ctypes.data_as(_I64P)
        a.nshot = self.nshot
        if self.nshot > 1:
            self.src_shot = np.ascontiguousarray(np.asarray(src_shot, dtype=np.int32).reshape(-1))
            self.rec_shot = np.ascontiguousarray(np.asarray(rec_shot, dtype=np.int32).reshape(-1))
            if len(self.src_shot) != len(self.src) or len(self.rec_shot) != len(self.rec):
                raise ValueError("one shot tag per source and per receiver")
            a.src_shot = self.src_shot.ctypes.data_as(_I32P)
            a.rec_shot = self.rec_shot.ctypes.data_as(_I32P)
        self.c = a

    @property
    def shots(self):
        return max(self.nshot, 1)


def make_opts(acc_dtype=None, variant=0, timing=None, chunk=0, max_group=0, graph=False,
              persistent=False, barrier_timeout_us=0, variant_plain=0, chunk_plain=0,
              no_partials=False, pairs=0) -> fd_opts:
    o = fd_opts()
    o.no_partials = int(bool(no_partials))
    o.pairs = int(pairs)
    o.variant_plain = int(variant_plain)
    o.chunk_plain = int(chunk_plain)
    o.persistent = int(bool(persistent))
    o.barrier_timeout_us = int(barrier_timeout_us)
    if acc_dtype is None or acc_dtype in ("f64", torch.float64, FD_F64):
        o.acc_dtype = FD_F64
    elif acc_dtype in ("f32", torch.float32, FD_F32):
        o.acc_dtype = FD_F32
    else:
        raise ValueError(f"acc_dtype {acc_dtype!r}")
    o.variant = int(variant)
    if timing is not None:
        o.timing = ctypes.pointer(timing)
    o.chunk = int(chunk)
    o.max_group = int(max_group)
    o.graph = int(bool(graph))
    return o


def fd_cfl_limit(ndim: int, order: int) -> float:
    return float(_lib.fd_cfl_limit(ndim, order))


def fd_variant_count(ndim: int) -> int:
    return int(_lib.fd_variant_count(ndim))


def fd_variant_info(ndim: int, variant: int) -> dict:
    """Tile shape of a kernel variant: tile_z, tile_y, threads, cells_per_lane, max_fields."""
    out = [ctypes.c_int32() for _ in range(5)]
    _raise(_lib.fd_variant_info(int(ndim), int(variant), *[ctypes.byref(o) for o in out]))
    return dict(zip(("tile_z", "tile_y", "threads", "cells_per_lane", "max_fields"),
                    (o.value for o in out)))


def variants_for(shape) -> list:
    """Kernel variants that can run on a grid of this shape."""
    nd = len(shape)
    return [v for v in range(1, fd_variant_count(nd) + 1)
            if shape[-1] % fd_variant_info(nd, v)["cells_per_lane"] == 0]


def _acq(src, wavelet, rec, shots):
    if isinstance(src, Acquisition):
        return src
    src_shot, rec_shot, nshot = shots if shots is not None else (None, None, 0)
    return Acquisition(src, wavelet, rec, src_shot, rec_shot, nshot)


def fd_forward(c, dx, order, src, wavelet, rec, dt, nt, traces=None, shots=None, **opts):
    """Receiver traces [nt, nrec] of the forward solve.  ``shots`` = (src_shot, rec_shot,
    nshot) tags a batch of shots."""
    acq = _acq(src, wavelet, rec, shots)
    if traces is None:
        traces = torch.empty((nt, len(acq.rec)), dtype=c.dtype, device=c.device)
    _check_io(c, nt, acq, traces=traces)
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(**opts)
    _raise(_lib.fd_forward(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt),
                           _dev(traces, "traces"), ctypes.byref(o), _stream()))
    return traces


def fd_misfit(traces, observed, dt, residual=None) -> float:
    """J = dt/2 sum (traces - observed)^2; fills ``residual`` when given."""
    nt, nrec = traces.shape
    _fits(observed, traces.numel(), traces, "observed")
    _fits(residual, traces.numel(), traces, "residual")
    J = ctypes.c_double()
    _raise(_lib.fd_misfit(int(nt), int(nrec), _dtype_code(traces), float(dt),
                          _dev(traces, "traces"), _dev(observed, "observed"),
                          _dev(residual, "residual"), ctypes.byref(J), _stream()))
    return J.value


def _sensitivity(fn, c, dx, order, src, wavelet, rec, dt, nt, observed, k, grad, traces, shots, opts):
    acq = _acq(src, wavelet, rec, shots)
    if grad is None:
        grad = torch.empty_like(c)
    _check_io(c, nt, acq, observed=observed, traces=traces, extra_fields=[("grad", grad)])
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(**opts)
    J = ctypes.c_double()
    _raise(fn(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt), _dev(observed, "observed"),
              float(k), _dev(grad, "grad"), ctypes.byref(J), _dev(traces, "traces"), ctypes.byref(o), _stream()))
    return grad, J.value


def fd_adjoint_sensitivity(c, dx, order, src, wavelet, rec, dt, nt, observed, k, grad=None,
                           traces=None, shots=None, **opts):
    """(grad_c, J) of the memory-efficient method at factor ``k``."""
    return _sensitivity(_lib.fd_adjoint_sensitivity, c, dx, order, src, wavelet, rec, dt, nt, observed, k,
                        grad, traces, shots, opts)


def fd_adjoint_sensitivity_noalloc(c, dx, order, src, wavelet, rec, dt, nt, observed, k, grad=None,
                                   traces=None, shots=None, **opts):
    """``fd_adjoint_sensitivity`` with the library's scratch in its fixed per-device
    array (no device allocation inside the call; pass ``grad`` to allocate nothing at
    all).  Problems beyond ``FD_NOALLOC_BYTES`` of scratch raise FD_E_ARG."""
    return _sensitivity(_lib.fd_adjoint_sensitivity_noalloc, c, dx, order, src, wavelet, rec, dt, nt, observed,
                        k, grad, traces, shots, opts)


def fd_adjoint_exact(c, dx, order, src, wavelet, rec, dt, nt, observed, grad=None, traces=None,
                     shots=None, **opts):
    """(grad_c, J) of the exact discrete adjoint by re-simulation (no factor k)."""
    acq = _acq(src, wavelet, rec, shots)
    if grad is None:
        grad = torch.empty_like(c)
    _check_io(c, nt, acq, observed=observed, traces=traces, extra_fields=[("grad", grad)])
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(**opts)
    J = ctypes.c_double()
    _raise(_lib.fd_adjoint_exact(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt),
                                 _dev(observed, "observed"), _dev(grad, "grad"), ctypes.byref(J),
                                 _dev(traces, "traces"), ctypes.byref(o), _stream()))
    return grad, J.value


def fd_vd_forward(m, b, dx, src, wavelet, rec, dt, nt, traces=None, shots=None, **opts):
    """Traces [nt][nrec] of the variable-material second-order scheme (mass m, stiffness b)."""
    acq = _acq(src, wavelet, rec, shots)
    if traces is None:
        traces = torch.empty((int(nt), acq.c.nrec), dtype=m.dtype, device=m.device)
    _check_io(m, nt, acq, traces=traces, extra_fields=[("b", b)])
    g = make_grid(m.shape, dx, 2, _dtype_code(m))
    o = make_opts(**opts)
    _raise(_lib.fd_vd_forward(ctypes.byref(g), _dev(m, "m"), _dev(b, "b"), ctypes.byref(acq.c), float(dt),
                              int(nt), _dev(traces, "traces"), ctypes.byref(o), _stream()))
    return traces


def fd_vd_adjoint_sensitivity(m, b, dx, src, wavelet, rec, dt, nt, observed, k, grad_m=None, grad_b=None,
                              traces=None, shots=None, **opts):
    """(grad_m, grad_b, J) of Alg. 1 for the variable-material second-order scheme."""
    acq = _acq(src, wavelet, rec, shots)
    grad_m = torch.empty_like(m) if grad_m is None else grad_m
    grad_b = torch.empty_like(m) if grad_b is None else grad_b
    _check_io(m, nt, acq, observed=observed, traces=traces,
              extra_fields=[("b", b), ("grad_m", grad_m), ("grad_b", grad_b)])
    g = make_grid(m.shape, dx, 2, _dtype_code(m))
    o = make_opts(**opts)
    J = ctypes.c_double()
    _raise(_lib.fd_vd_adjoint_sensitivity(ctypes.byref(g), _dev(m, "m"), _dev(b, "b"), ctypes.byref(acq.c),
                                          float(dt), int(nt), _dev(observed, "observed"), float(k),
                                          _dev(grad_m, "grad_m"), _dev(grad_b, "grad_b"), ctypes.byref(J),
                                          _dev(traces, "traces"), ctypes.byref(o), _stream()))
    return grad_m, grad_b, J.value


class SweepState:
    """Caller-owned device state between fd_sens_forward and fd_sens_backward."""

    def __init__(self, c: torch.Tensor, nt: int, nrec: int, acc_dtype=None, nshot: int = 1):
        acc_t = torch.float32 if (make_opts(acc_dtype).acc_dtype == FD_F32
                                  and c.dtype == torch.float32) else torch.float64
        ns = max(int(nshot), 1)
        self.u_a = torch.empty((ns,) + tuple(c.shape), dtype=c.dtype, device=c.device)
        self.u_b = torch.empty_like(self.u_a)
        self.acc = torch.empty(c.shape, dtype=acc_t, device=c.device)
        self.residual = torch.empty((nt, nrec), dtype=c.dtype, device=c.device)

    def c_struct(self) -> fd_state:
        s = fd_state()
        s.u_a = self.u_a.data_ptr()
        s.u_b = self.u_b.data_ptr()
        s.acc = self.acc.data_ptr()
        s.residual = self.residual.data_ptr()
        return s



class VdSweepState(SweepState):
    """Caller-owned device state between fd_vd_sens_forward and fd_vd_sens_backward:
    the constant-density state plus the stiffness-term accumulator."""

    def __init__(self, m: torch.Tensor, nt: int, nrec: int, acc_dtype=None, nshot: int = 1):
        super().__init__(m, nt, nrec, acc_dtype=acc_dtype, nshot=nshot)
        self.acc_b = torch.empty_like(self.acc)


def fd_vd_sens_forward(m, b, dx, src, wavelet, rec, dt, nt, observed, state: VdSweepState, traces=None,
                       shots=None, **opts) -> float:
    acq = _acq(src, wavelet, rec, shots)
    _check_io(m, nt, acq, observed=observed, traces=traces, extra_fields=[("b", b)])
    _check_state(m, nt, acq, state, acq.nshot)
    g = make_grid(m.shape, dx, 2, _dtype_code(m))
    o = make_opts(**opts)
    J = ctypes.c_double()
    st = state.c_struct()
    _raise(_lib.fd_vd_sens_forward(ctypes.byref(g), _dev(m, "m"), _dev(b, "b"), ctypes.byref(acq.c), float(dt),
                                   int(nt), _dev(observed, "observed"), ctypes.byref(st),
                                   _dev(state.acc_b, "acc_b"), _dev(traces, "traces"), ctypes.byref(J),
                                   ctypes.byref(o), _stream()))
    return J.value


def fd_vd_sens_backward(m, b, dx, src, wavelet, rec, dt, nt, k, state: VdSweepState, grad_scale=1.0,
                        grad_m=None, grad_b=None, shots=None, **opts):
    acq = _acq(src, wavelet, rec, shots)
    grad_m = torch.empty_like(m) if grad_m is None else grad_m
    grad_b = torch.empty_like(m) if grad_b is None else grad_b
    _check_io(m, nt, acq, extra_fields=[("b", b), ("grad_m", grad_m), ("grad_b", grad_b)])
    _check_state(m, nt, acq, state, acq.nshot)
    g = make_grid(m.shape, dx, 2, _dtype_code(m))
    o = make_opts(**opts)
    st = state.c_struct()
    _raise(_lib.fd_vd_sens_backward(ctypes.byref(g), _dev(m, "m"), _dev(b, "b"), ctypes.byref(acq.c), float(dt),
                                    int(nt), float(k), ctypes.byref(st), _dev(state.acc_b, "acc_b"),
                                    float(grad_scale), _dev(grad_m, "grad_m"), _dev(grad_b, "grad_b"),
                                    ctypes.byref(o), _stream()))
    return grad_m, grad_b

def fd_sens_forward(c, dx, order, src, wavelet, rec, dt, nt, observed, state: SweepState,
                    traces=None, shots=None, **opts) -> float:
    acq = _acq(src, wavelet, rec, shots)
    _check_io(c, nt, acq, observed=observed, traces=traces)
    _check_state(c, nt, acq, state, acq.nshot)
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(**opts)
    st = state.c_struct()
    J = ctypes.c_double()
    _raise(_lib.fd_sens_forward(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt),
                                _dev(observed, "observed"), ctypes.byref(st), _dev(traces, "traces"),
                                ctypes.byref(J), ctypes.byref(o), _stream()))
    return J.value


def fd_sens_backward(c, dx, order, src, wavelet, rec, dt, nt, k, state: SweepState, grad_scale=1.0,
                     grad=None, shots=None, **opts):
    acq = _acq(src, wavelet, rec, shots)
    if grad is None:
        grad = torch.empty_like(c)
    _check_io(c, nt, acq, extra_fields=[("grad", grad)])
    _check_state(c, nt, acq, state, acq.nshot)
    g = make_grid(c.shape, dx, order, _dtype_code(c))
    o = make_opts(**opts)
    st = state.c_struct()
    _raise(_lib.fd_sens_backward(ctypes.byref(g), _dev(c, "c"), ctypes.byref(acq.c), float(dt), int(nt),
                                 float(k), ctypes.byref(st), float(grad_scale), _dev(grad, "grad"),
                                 ctypes.byref(o), _stream()))
    return grad


class Problem:
    """One independent problem of a batched call (device tensors stay referenced)."""

    def __init__(self, c, dx, order, src, wavelet, rec, dt, nt, observed, k, grad=None, traces=None):
        self.c, self.observed = c, observed
        self.acq = Acquisition(src, wavelet, rec)
        self.grad = torch.empty_like(c) if grad is None else grad
        self.traces = traces
        _check_io(c, nt, self.acq, observed=observed, traces=traces, extra_fields=[("grad", self.grad)])
        p = fd_problem()
        p.grid = make_grid(c.shape, dx, order, _dtype_code(c))
        p.c = _dev(c, "c")
        p.acq = self.acq.c
        p.dt = float(dt)
        p.nt = int(nt)
        p.observed = _dev(observed, "observed")
        p.k = float(k)
        p.grad_c = _dev(self.grad, "grad")
        p.traces = _dev(traces, "traces")
        self.c_struct = p


def fd_adjoint_sensitivity_batched(problems, **opts):
    """Alg. 1 for a list of ``Problem``s in lock-step launches; returns their J values
    (gradients land in each problem's ``grad``)."""
    arr = (fd_problem * len(problems))(*[p.c_struct for p in problems])
    J = (ctypes.c_double * len(problems))()
    o = make_opts(**opts)
    _raise(_lib.fd_adjoint_sensitivity_batched(arr, len(problems), J, ctypes.byref(o), _stream()))
    return list(J)


class BatchPlan:
    """A batch plan (fd_batch_plan_create) over a list of ``Problem``s.  ``run(J)``
    enqueues one gradient of every problem on the current stream with kernel launches
    only, so it may be captured in a ``torch.cuda.CUDAGraph`` and replayed; ``J`` is a
    float64 device tensor of one value per problem.  The problems' tensors stay
    referenced for the plan's life; ``close()`` releases the plan on the current
    stream."""

    def __init__(self, problems, **opts):
        self.problems = list(problems)
        arr = (fd_problem * len(self.problems))(*[p.c_struct for p in self.problems])
        o = make_opts(**opts)
        h = ctypes.c_void_p()
        _raise(_lib.fd_batch_plan_create(arr, len(self.problems), ctypes.byref(o), _stream(), ctypes.byref(h)))
        self._h = h

    def run(self, J):
        if self._h is None:
            raise FdError(FD_E_ARG, "plan is closed")
        if not (J.is_cuda and J.dtype == torch.float64 and J.is_contiguous() and J.numel() >= len(self.problems)):
            raise FdError(FD_E_ARG, "J must be a contiguous float64 device tensor with one value per problem")
        _raise(_lib.fd_batch_run(self._h, ctypes.c_void_p(J.data_ptr()), _stream()))
        return J

    def timing(self):
        t = fd_timing()
        _raise(_lib.fd_batch_timing(self._h, ctypes.byref(t)))
        return t

    def close(self):
        if self._h is not None:
            _raise(_lib.fd_batch_plan_destroy(self._h, _stream()))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fd_autotune(shape, dx, order, dtype=torch.float32, nshot=1, steps=3, **opts):
    """Time the launch shapes for this grid class; the library remembers the fastest for
    later calls with variant 0.  Returns ({variant, chunk, max_group, variant_plain,
    chunk_plain}, ms per step)."""
    g = make_grid(shape, dx, order, FD_F64 if dtype == torch.float64 else FD_F32)
    o = make_opts(**opts)
    best = fd_opts()
    ms = ctypes.c_double()
    _raise(_lib.fd_autotune(ctypes.byref(g), int(nshot), ctypes.byref(o), int(steps),
                            ctypes.byref(best), ctypes.byref(ms), _stream()))
    return {"variant": best.variant, "chunk": best.chunk, "max_group": best.max_group,
            "variant_plain": best.variant_plain, "chunk_plain": best.chunk_plain}, ms.value


def fd_propagate(coef, u_prev, u_cur, nsteps, dx, order, **opts):
    """In place: (u_prev, u_cur) advance by ``nsteps`` source-free steps."""
    for what, t in (("u_prev", u_prev), ("u_cur", u_cur)):
        _fits(t, coef.numel(), coef, what)
    g = make_grid(coef.shape, dx, order, _dtype_code(coef))
    o = make_opts(**opts)
    _raise(_lib.fd_propagate(ctypes.byref(g), _dev(coef, "coef"), _dev(u_prev, "u_prev"),
                             _dev(u_cur, "u_cur"), int(nsteps), ctypes.byref(o), _stream()))
    return u_prev, u_cur


def fd_workspace_bytes(shape, order, dtype_code, nt, nsrc=0, nrec=0, nshots=1, dx=1.0) -> int:
    """Upper bound of the device bytes one fd_adjoint_sensitivity call takes from the
    stream-ordered pool (see the header)."""
    g = make_grid(shape, dx, order, dtype_code)
    a = fd_acq()
    a.nsrc = int(nsrc)
    a.nrec = int(nrec)
    n = _lib.fd_workspace_bytes(ctypes.byref(g), ctypes.byref(a), int(nt), int(nshots))
    if n == 0:
        raise FdError(FD_E_ARG, _lib.fd_last_error().decode())
    return int(n)


# ---- gradient-based design ---------------------------------------------------------

def make_design(shape, origin, extent, dtype_code, material, filter_radius=0.0, beta=0.0, eta=0.5,
                lo=0.0, hi=1.0) -> fd_design:
    """Description of a design box and its chain (fd_design).  ``material`` is the affine
    map (m0, dm, b0, db); ``rho_scaling`` and ``two_material`` build the paper's two."""
    d = fd_design()
    d.ndim = len(shape)
    for i in range(len(shape)):
        d.shape[i] = int(shape[i])
        d.origin[i] = int(origin[i])
        d.extent[i] = int(extent[i])
    d.dtype = int(dtype_code)
    d.filter_radius = float(filter_radius)
    d.beta = float(beta)
    d.eta = float(eta)
    d.lo = float(lo)
    d.hi = float(hi)
    d.m0, d.dm, d.b0, d.db = (float(v) for v in material)
    return d


def rho_scaling(rho0: float, c0: float):
    """(m0, dm, b0, db) of gamma rho0 u_tt - div(gamma rho0 c0^2 grad u) = f (Eq. scalarwaveequation)."""
    return 0.0, rho0, 0.0, rho0 * c0 * c0


def two_material(rho1: float, rho2: float, kappa1: float, kappa2: float):
    """(m0, dm, b0, db) of the linear inverse bulk modulus and inverse density maps of
    Eq. wavetopopt (gamma = 0: material 1, gamma = 1: material 2)."""
    return 1.0 / kappa1, 1.0 / kappa2 - 1.0 / kappa1, 1.0 / rho1, 1.0 / rho2 - 1.0 / rho1


def _design_sizes(design: fd_design, box_fields, grid_fields):
    nbox = math.prod(int(design.extent[i]) for i in range(design.ndim))
    ngrid = math.prod(int(design.shape[i]) for i in range(design.ndim))
    for name, t in box_fields:
        if t is not None and t.numel() != nbox:
            raise ValueError(f"{name} has {t.numel()} values, the design box {nbox}")
    for name, t in grid_fields:
        if t.numel() != ngrid:
            raise ValueError(f"{name} has {t.numel()} values, the grid {ngrid}")


def fd_design_map(design: fd_design, gamma, m, b, gamma_bar=None):
    """Write the material of the design field into m and b (box cells only)."""
    _design_sizes(design, [("gamma", gamma), ("gamma_bar", gamma_bar)], [("m", m), ("b", b)])
    _raise(_lib.fd_design_map(ctypes.byref(design), _dev(gamma, "gamma"), _dev(m, "m"), _dev(b, "b"),
                              _dev(gamma_bar, "gamma_bar"), _stream()))
    return m, b


def fd_design_adjoint(design: fd_design, gamma, grad_m, grad_b, grad_gamma=None):
    """dC/dgamma from dC/dm and dC/db through the chain of fd_design_map."""
    grad_gamma = torch.empty_like(gamma) if grad_gamma is None else grad_gamma
    _design_sizes(design, [("gamma", gamma), ("grad_gamma", grad_gamma)], [("grad_m", grad_m), ("grad_b", grad_b)])
    _raise(_lib.fd_design_adjoint(ctypes.byref(design), _dev(gamma, "gamma"), _dev(grad_m, "grad_m"),
                                  _dev(grad_b, "grad_b"), _dev(grad_gamma, "grad_gamma"), _stream()))
    return grad_gamma


def fd_adam_step(x, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, lo=-math.inf, hi=math.inf):
    """One Adam update of x in place (moments m1, m2 in place), then x clipped to [lo, hi]."""
    for name, t in (("grad", grad), ("m1", m1), ("m2", m2)):
        if t.numel() != x.numel():
            raise ValueError(f"{name} has {t.numel()} values, x {x.numel()}")
    _raise(_lib.fd_adam_step(x.numel(), _dtype_code(x), _dev(x, "x"), _dev(grad, "grad"), _dev(m1, "m1"),
                             _dev(m2, "m2"), int(step), float(lr), float(beta1), float(beta2), float(eps),
                             float(lo), float(hi), _stream()))
    return x
