"""FP64 CPU oracle for the superposition adjoint method (arXiv:2509.15744).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may load it.  It shares no code with the GPU library; the two
meet only through the seeded input generators, which hold none of the
method's arithmetic.

The arithmetic lives in ``fdoracle.c`` (the constant-density high-order scheme)
and ``vdoracle.c`` (the paper's second-order flux-form scheme with variable mass
and stiffness coefficients), plain double-precision loops; their headers give the
discretisation and the time indexing.  This module

* derives the central second-derivative weights with Fornberg's recursion
  (B. Fornberg, Math. Comp. 51 (1988) 699-706), in exact rationals;
* compiles both C files with gcc on first use (``build()``);
* wraps the C entry points for numpy arrays;
* adds the brute-force central finite-difference gradient.

Readings of the paper taken here:

* stencil: paper Eq. FDstencil2 with rho^-1 = 1, kappa = c^2, generalised
  from 2nd to 2r-th order in space (difference form);
* walls: paper Eq. BC through half-sample mirror ghost cells;
* levels: u^{-1} = u^0 = 0, forward steps n = 0..nt-1 give u^1..u^nt;
* source f^n = wavelet[n] / dx^d at the source cell; adjoint force
  fdag^n = -(u^n(x_r) - obs^n_r) / dt at the receiver, no volume factor;
* J = dt/2 sum_n sum_r (u^n(x_r) - obs^n_r)^2;
* superposed end levels v^nt = u^nt, v^{nt-1} = u^{nt-1} + k coef fdag^nt.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "fdoracle.c"), os.path.join(_HERE, "vdoracle.c")]
_LIB_PATH = os.path.join(_HERE, "_fdoracle.so")
_lib = None


# ---------------------------------------------------------------------------
# stencil weights
# ---------------------------------------------------------------------------

def fornberg_weights(nodes, z, m):
    """Finite-difference weights on ``nodes`` for the derivatives 0..m at ``z``.

    Fornberg's recursion (Math. Comp. 51, 1988), carried out in exact
    rational arithmetic.  Returns ``w[d][i]``: weight of node ``i`` in the
    approximation of the d-th derivative.
    """
    nodes = [Fraction(x) for x in nodes]
    z = Fraction(z)
    npts = len(nodes)
    w = [[Fraction(0)] * npts for _ in range(m + 1)]
    w[0][0] = Fraction(1)
    c1 = Fraction(1)
    c4 = nodes[0] - z
    for i in range(1, npts):
        mn = min(i, m)
        c2 = Fraction(1)
        c5 = c4
        c4 = nodes[i] - z
        for j in range(i):
            c3 = nodes[i] - nodes[j]
            c2 *= c3
            if j == i - 1:
                for d in range(mn, 0, -1):
                    w[d][i] = c1 * (d * w[d - 1][i - 1] - c5 * w[d][i - 1]) / c2
                w[0][i] = -c1 * c5 * w[0][i - 1] / c2
            for d in range(mn, 0, -1):
                w[d][j] = (c4 * w[d][j] - d * w[d - 1][j]) / c3
            w[0][j] = c4 * w[0][j] / c3
        c1 = c2
    return w


def central_weights(order: int):
    """Exact rationals ``[a_0, a_1, ..., a_r]`` of the order-``order`` central
    second derivative: u'' ~ dx^-2 (a_0 u_0 + sum_j a_j (u_j + u_-j))."""
    if order < 2 or order % 2:
        raise ValueError("order must be an even integer >= 2")
    r = order // 2
    nodes = [0]
    for j in range(1, r + 1):
        nodes += [j, -j]
    w = fornberg_weights(nodes, 0, 2)[2]
    a = [w[0]]
    for j in range(1, r + 1):
        if w[2 * j - 1] != w[2 * j]:
            raise AssertionError("central weights must be symmetric")
        a.append(w[2 * j - 1])
    return a


def _a_array(order: int) -> np.ndarray:
    return np.array([float(x) for x in central_weights(order)[1:]], dtype=np.float64)


# ---------------------------------------------------------------------------
# the C library
# ---------------------------------------------------------------------------

def build(force: bool = False) -> str:
    """Compile ``fdoracle.c`` and ``vdoracle.c`` into ``_fdoracle.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or any(
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(src) for src in _SRCS):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        grid = [I, P, D, I, P]
        lib.orc_laplacian.argtypes = grid + [P, P]
        lib.orc_laplacian.restype = None
        lib.orc_propagate.argtypes = grid + [P, P, P, I]
        lib.orc_propagate.restype = I
        lib.orc_forward.argtypes = grid + [P, D, I, I, P, P, I, P, P, P, P]
        lib.orc_forward.restype = I
        lib.orc_misfit.argtypes = [I, I, D, P, P, P]
        lib.orc_misfit.restype = D
        lib.orc_adjoint.argtypes = grid + [P, D, I, I, P, P, P, I, P, P]
        lib.orc_adjoint.restype = I
        lib.orc_exact_gradient.argtypes = grid + [P, D, I, I, P, P, I, P, P, P, P, P, P]
        lib.orc_exact_gradient.restype = I
        lib.orc_superposition.argtypes = grid + [P, D, I, I, P, P, I, P, P, D, P, P, P]
        lib.orc_superposition.restype = I
        lib.orc_exact_gradient_ckpt.argtypes = grid + [P, D, I, I, P, P, I, P, P, I, P, P, P, P]
        lib.orc_exact_gradient_ckpt.restype = I
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = I
        lib.orc_set_threads.argtypes = [I]
        lib.orc_set_threads.restype = I
        vgrid = [I, P, D]
        lib.orc_vd_operator.argtypes = vgrid + [P, P, P]
        lib.orc_vd_operator.restype = None
        lib.orc_vd_forward.argtypes = vgrid + [P, P, D, I, I, P, P, I, P, P, P, P]
        lib.orc_vd_forward.restype = I
        lib.orc_vd_adjoint.argtypes = vgrid + [P, P, D, I, I, P, P, P]
        lib.orc_vd_adjoint.restype = I
        lib.orc_vd_exact_gradient.argtypes = vgrid + [P, P, D, I, I, P, P, I, P, P, P, P, P, P, P, P]
        lib.orc_vd_exact_gradient.restype = I
        lib.orc_vd_superposition.argtypes = vgrid + [P, P, D, I, I, P, P, I, P, P, D, P, P, P, P]
        lib.orc_vd_superposition.restype = I
        _lib = lib
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64).reshape(-1))


def _ptr(a):
    return None if a is None else a.ctypes.data


def _grid_args(shape, dx, order):
    shape = tuple(int(s) for s in shape)
    sh = np.array(list(shape) + [1] * (3 - len(shape)), dtype=np.int64)
    a = _a_array(order)
    return [len(shape), sh.ctypes.data, float(dx), order // 2, a.ctypes.data], (sh, a)


def _check(rc, what):
    if rc == -1:
        raise ValueError(f"oracle {what}: invalid arguments")
    if rc != 0:
        raise MemoryError(f"oracle {what}: allocation failed ({rc})")


def flat_index(shape, coords):
    """C-order flat cell index of integer coordinates ``coords[..., ndim]``."""
    coords = np.asarray(coords, dtype=np.int64)
    return np.ravel_multi_index(tuple(coords.T), tuple(shape)).astype(np.int64)


# ---------------------------------------------------------------------------
# numpy-facing wrappers
# ---------------------------------------------------------------------------

def laplacian(u, dx, order):
    """Order-``order`` Laplacian with mirror walls, ``L u``."""
    u = _f64(u)
    out = np.empty_like(u)
    g, keep = _grid_args(u.shape, dx, order)
    _load().orc_laplacian(*g, u.ctypes.data, out.ctypes.data)
    return out


def propagate(coef, u_prev, u_cur, nsteps, dx, order):
    """Source-free leapfrog steps from (u^{-1}, u^0); returns (u^{n-1}, u^n)."""
    coef = _f64(coef)
    up = _f64(u_prev).copy()
    uc = _f64(u_cur).copy()
    g, keep = _grid_args(coef.shape, dx, order)
    _check(_load().orc_propagate(*g, coef.ctypes.data, up.ctypes.data, uc.ctypes.data,
                                 int(nsteps)), "propagate")
    return up, uc


def forward(c, dx, order, dt, nt, src, wavelet, rec, history=False):
    """Forward solve.  Returns ``(traces [nt, nrec], hist or None, (u^{nt-1}, u^nt))``."""
    c = _f64(c)
    src, rec = _i64(src), _i64(rec)
    wavelet = _f64(np.asarray(wavelet).reshape(nt, len(src)))
    traces = np.zeros((nt, len(rec)))
    hist = np.empty((nt + 1,) + c.shape) if history else None
    last2 = np.empty((2,) + c.shape)
    g, keep = _grid_args(c.shape, dx, order)
    _check(_load().orc_forward(*g, c.ctypes.data, float(dt), int(nt), len(src), _ptr(src),
                               _ptr(wavelet), len(rec), _ptr(rec), traces.ctypes.data,
                               _ptr(hist), last2.ctypes.data), "forward")
    return traces, hist, (last2[0], last2[1])


def misfit(traces, observed, dt):
    """``(J, residual)`` with J = dt/2 sum (traces - observed)^2."""
    traces, observed = _f64(traces), _f64(observed)
    resid = np.empty_like(traces)
    nt, nrec = traces.shape
    J = _load().orc_misfit(nt, nrec, float(dt), traces.ctypes.data, observed.ctypes.data,
                           resid.ctypes.data)
    return J, resid


def adjoint(c, dx, order, dt, nt, rec, fdag, src=None, history=False):
    """Backward sweep driven by ``fdag [nt, nrec]``; returns ``(hist or None, mu at src [nt, nsrc] or None)``."""
    c = _f64(c)
    rec = _i64(rec)
    fdag = _f64(np.asarray(fdag).reshape(nt, len(rec)))
    hist = np.empty((nt + 1,) + c.shape) if history else None
    srcv = _i64(src) if src is not None else None
    mu_src = np.empty((nt, len(srcv))) if srcv is not None else None
    g, keep = _grid_args(c.shape, dx, order)
    _check(_load().orc_adjoint(*g, c.ctypes.data, float(dt), int(nt), len(rec), _ptr(rec),
                               fdag.ctypes.data, _ptr(hist),
                               0 if srcv is None else len(srcv), _ptr(srcv), _ptr(mu_src)),
           "adjoint")
    return hist, mu_src


def exact_gradient(c, dx, order, dt, nt, src, wavelet, rec, observed):
    """Exact discrete adjoint gradient with stored history.

    Returns ``(grad_c, J, sum_dmu2, traces)``; ``sum_dmu2`` is sum_n (mu^{n+1}-mu^n)^2."""
    c = _f64(c)
    src, rec = _i64(src), _i64(rec)
    wavelet = _f64(np.asarray(wavelet).reshape(nt, len(src)))
    observed = _f64(np.asarray(observed).reshape(nt, len(rec)))
    grad = np.empty_like(c)
    s2 = np.empty_like(c)
    traces = np.empty((nt, len(rec)))
    J = ctypes.c_double()
    g, keep = _grid_args(c.shape, dx, order)
    _check(_load().orc_exact_gradient(*g, c.ctypes.data, float(dt), int(nt), len(src),
                                      _ptr(src), wavelet.ctypes.data, len(rec), _ptr(rec),
                                      observed.ctypes.data, grad.ctypes.data,
                                      ctypes.addressof(J), s2.ctypes.data, traces.ctypes.data),
           "exact_gradient")
    return grad, J.value, s2, traces


def exact_gradient_ckpt(c, dx, order, dt, nt, src, wavelet, rec, observed, seg=None):
    """``exact_gradient`` with uniform checkpoints every ``seg`` levels instead of the
    stored history (default seg ~ sqrt(nt)).  Returns ``(grad_c, J, sum_dmu2, traces)``."""
    c = _f64(c)
    src, rec = _i64(src), _i64(rec)
    wavelet = _f64(np.asarray(wavelet).reshape(nt, len(src)))
    observed = _f64(np.asarray(observed).reshape(nt, len(rec)))
    if seg is None:
        seg = max(1, int(round(np.sqrt(nt))))
    grad = np.empty_like(c)
    s2 = np.empty_like(c)
    traces = np.empty((nt, len(rec)))
    J = ctypes.c_double()
    g, keep = _grid_args(c.shape, dx, order)
    _check(_load().orc_exact_gradient_ckpt(*g, c.ctypes.data, float(dt), int(nt), len(src),
                                           _ptr(src), wavelet.ctypes.data, len(rec), _ptr(rec),
                                           observed.ctypes.data, int(seg), grad.ctypes.data,
                                           ctypes.addressof(J), s2.ctypes.data,
                                           traces.ctypes.data),
           "exact_gradient_ckpt")
    return grad, J.value, s2, traces


def superposition_gradient(c, dx, order, dt, nt, src, wavelet, rec, observed, k):
    """Approximate gradient of paper Alg. 1 at factor ``k``; returns ``(grad_c, J, traces)``."""
    c = _f64(c)
    src, rec = _i64(src), _i64(rec)
    wavelet = _f64(np.asarray(wavelet).reshape(nt, len(src)))
    observed = _f64(np.asarray(observed).reshape(nt, len(rec)))
    grad = np.empty_like(c)
    traces = np.empty((nt, len(rec)))
    J = ctypes.c_double()
    g, keep = _grid_args(c.shape, dx, order)
    _check(_load().orc_superposition(*g, c.ctypes.data, float(dt), int(nt), len(src),
                                     _ptr(src), wavelet.ctypes.data, len(rec), _ptr(rec),
                                     observed.ctypes.data, float(k), grad.ctypes.data,
                                     ctypes.addressof(J), traces.ctypes.data),
           "superposition")
    return grad, J.value, traces


def misfit_of_speed(c, dx, order, dt, nt, src, wavelet, rec, observed):
    """J(c) by a forward solve."""
    traces, _, _ = forward(c, dx, order, dt, nt, src, wavelet, rec)
    return misfit(traces, observed, dt)[0]


def fd_gradient(c, dx, order, dt, nt, src, wavelet, rec, observed, cells, eps=1e-6):
    """Central finite differences (J(c + eps e_i) - J(c - eps e_i)) / (2 eps) at ``cells``."""
    c = _f64(c)
    flat = c.reshape(-1)
    out = np.empty(len(cells))
    for q, i in enumerate(cells):
        cp = flat.copy()
        cp[i] += eps
        cm = flat.copy()
        cm[i] -= eps
        jp = misfit_of_speed(cp.reshape(c.shape), dx, order, dt, nt, src, wavelet, rec, observed)
        jm = misfit_of_speed(cm.reshape(c.shape), dx, order, dt, nt, src, wavelet, rec, observed)
        out[q] = (jp - jm) / (2.0 * eps)
    return out


def num_threads() -> int:
    """Threads used by the oracle's parallel cell loops."""
    return int(_load().orc_num_threads())


def set_threads(n: int) -> int:
    """Set the threads of the oracle's parallel loops; returns the previous count."""
    return int(_load().orc_set_threads(int(n)))


def cfl_limit(ndim: int, order: int) -> float:
    """Largest stable c_max dt / dx of the leapfrog scheme: 2 / sqrt(d * |symbol(pi)|)."""
    a = central_weights(order)
    sym_pi = a[0] + 2 * sum(a[j] * (-1) ** j for j in range(1, len(a)))
    return float(2.0 / np.sqrt(ndim * abs(float(sym_pi))))


# ---------------------------------------------------------------------------
# the paper's second-order flux-form scheme with variable material (vdoracle.c)
# ---------------------------------------------------------------------------

def _vgrid_args(shape, dx):
    shape = tuple(int(s) for s in shape)
    sh = np.array(list(shape) + [1] * (3 - len(shape)), dtype=np.int64)
    return [len(shape), sh.ctypes.data, float(dx)], sh


def vd_operator(b, u, dx):
    """(L_b u) with harmonic-mean faces and mirrored walls."""
    b, u = _f64(b), _f64(u)
    out = np.empty_like(u)
    g, keep = _vgrid_args(u.shape, dx)
    _load().orc_vd_operator(*g, b.ctypes.data, u.ctypes.data, out.ctypes.data)
    return out


def vd_forward(m, b, dx, dt, nt, src, wavelet, rec, history=False):
    """Forward solve of m u_tt - div(b grad u) = f; returns ``(traces, hist, last2)``."""
    m, b = _f64(m), _f64(b)
    src, rec = _i64(src), _i64(rec)
    wavelet = _f64(np.asarray(wavelet).reshape(nt, len(src)))
    traces = np.empty((nt, len(rec)))
    hist = np.empty((nt + 1,) + m.shape) if history else None
    last2 = np.empty((2,) + m.shape)
    g, keep = _vgrid_args(m.shape, dx)
    _check(_load().orc_vd_forward(*g, m.ctypes.data, b.ctypes.data, float(dt), int(nt), len(src),
                                  _ptr(src), wavelet.ctypes.data, len(rec), _ptr(rec),
                                  traces.ctypes.data, _ptr(hist), last2.ctypes.data), "vd_forward")
    return traces, hist, last2


def vd_adjoint(m, b, dx, dt, nt, rec, fdag):
    """Adjoint sweep with force ``fdag`` [nt][nrec] at the receivers; returns mu^0..mu^nt."""
    m, b = _f64(m), _f64(b)
    rec = _i64(rec)
    fdag = _f64(np.asarray(fdag).reshape(nt, len(rec)))
    hist = np.empty((nt + 1,) + m.shape)
    g, keep = _vgrid_args(m.shape, dx)
    _check(_load().orc_vd_adjoint(*g, m.ctypes.data, b.ctypes.data, float(dt), int(nt), len(rec),
                                  _ptr(rec), fdag.ctypes.data, hist.ctypes.data), "vd_adjoint")
    return hist


def vd_exact_gradient(m, b, dx, dt, nt, src, wavelet, rec, observed):
    """Exact discrete gradient (stored history).  Returns
    ``(grad_m, grad_b, J, s2_m, s2_b, traces)``; s2_m and s2_b are the k^2 terms of the
    superposition for the two fields."""
    m, b = _f64(m), _f64(b)
    src, rec = _i64(src), _i64(rec)
    wavelet = _f64(np.asarray(wavelet).reshape(nt, len(src)))
    observed = _f64(np.asarray(observed).reshape(nt, len(rec)))
    gm, gb, s2m, s2b = (np.empty_like(m) for _ in range(4))
    traces = np.empty((nt, len(rec)))
    J = ctypes.c_double()
    g, keep = _vgrid_args(m.shape, dx)
    _check(_load().orc_vd_exact_gradient(*g, m.ctypes.data, b.ctypes.data, float(dt), int(nt),
                                         len(src), _ptr(src), wavelet.ctypes.data, len(rec),
                                         _ptr(rec), observed.ctypes.data, gm.ctypes.data,
                                         gb.ctypes.data, ctypes.addressof(J), s2m.ctypes.data,
                                         s2b.ctypes.data, traces.ctypes.data), "vd_exact_gradient")
    return gm, gb, J.value, s2m, s2b, traces


def vd_superposition_gradient(m, b, dx, dt, nt, src, wavelet, rec, observed, k):
    """Alg. 1 for both fields at factor ``k``; returns ``(grad_m, grad_b, J, traces)``."""
    m, b = _f64(m), _f64(b)
    src, rec = _i64(src), _i64(rec)
    wavelet = _f64(np.asarray(wavelet).reshape(nt, len(src)))
    observed = _f64(np.asarray(observed).reshape(nt, len(rec)))
    gm, gb = np.empty_like(m), np.empty_like(m)
    traces = np.empty((nt, len(rec)))
    J = ctypes.c_double()
    g, keep = _vgrid_args(m.shape, dx)
    _check(_load().orc_vd_superposition(*g, m.ctypes.data, b.ctypes.data, float(dt), int(nt),
                                        len(src), _ptr(src), wavelet.ctypes.data, len(rec),
                                        _ptr(rec), observed.ctypes.data, float(k), gm.ctypes.data,
                                        gb.ctypes.data, ctypes.addressof(J), traces.ctypes.data),
           "vd_superposition")
    return gm, gb, J.value, traces


def vd_misfit(m, b, dx, dt, nt, src, wavelet, rec, observed):
    """J(m, b) by a forward solve."""
    traces, _, _ = vd_forward(m, b, dx, dt, nt, src, wavelet, rec)
    return misfit(traces, observed, dt)[0]


def vd_fd_gradient(m, b, which, dx, dt, nt, src, wavelet, rec, observed, cells, eps=1e-6):
    """Central finite differences of J with respect to m (``which="m"``) or b at ``cells``."""
    m, b = _f64(m), _f64(b)
    out = np.empty(len(cells))
    for q, i in enumerate(cells):
        vals = []
        for sgn in (1.0, -1.0):
            mp, bp = m.copy().reshape(-1), b.copy().reshape(-1)
            (mp if which == "m" else bp)[i] += sgn * eps
            vals.append(vd_misfit(mp.reshape(m.shape), bp.reshape(b.shape), dx, dt, nt, src,
                                  wavelet, rec, observed))
        out[q] = (vals[0] - vals[1]) / (2.0 * eps)
    return out
