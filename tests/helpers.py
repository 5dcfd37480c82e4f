"""Shared helpers of the GPU parity tests: oracle references and tensor plumbing."""
import functools
import sys

import numpy as np

import oracle


def say(*args):
    """Name the case before a GPU step (flushed, so it survives a lost box)."""
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_dev(x, dtype):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x), dtype=dtype)
    return t.cuda()


def torch_dtype(code):
    import torch
    return torch.float64 if code == "f64" else torch.float32


class OracleCase:
    """Oracle results for one problem: observed data, traces, J, gradients."""

    def __init__(self, p, k=None, gap=None, exact=True):
        self.p = p
        self.obs, _, _ = oracle.forward(p.c_ref, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec)
        if exact:
            self.g_exact, self.J, self.s2, self.traces = oracle.exact_gradient(
                p.c, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec, self.obs)
            gap1 = np.linalg.norm(self.s2 / p.c ** 3) / np.linalg.norm(self.g_exact)
            if k is None:
                k = gap / gap1
            self.gap_per_k = gap1
        self.k = k
        self.g_approx, self.J_approx, self.traces_approx = oracle.superposition_gradient(
            p.c, p.dx, p.order, p.dt, p.nt, p.src, p.wavelet, p.rec, self.obs, k)
        if not exact:
            self.traces = self.traces_approx
            self.J = self.J_approx


@functools.lru_cache(maxsize=16)
def cached_case(key, builder, k=None, gap=None, exact=True):
    return OracleCase(builder(), k=k, gap=gap, exact=exact)


def shot_problem(shape, nshot, order, nt, dtype, seed):
    """One medium, nshot shots: each shot has 1-2 sources and 3-5 receivers of its own."""
    rng = np.random.default_rng(seed)
    c = 1.0 + rng.random(shape)
    dt = 0.4 * oracle.cfl_limit(len(shape), order) / c.max()
    n = int(np.prod(shape))
    src, src_shot, rec, rec_shot = [], [], [], []
    for s in range(nshot):
        for _ in range(1 + s % 2):
            src.append(rng.integers(n)); src_shot.append(s)
        for _ in range(3 + s % 3):
            rec.append(rng.integers(n)); rec_shot.append(s)
    rec.append(rec[0]); rec_shot.append(rec_shot[0])           # a duplicate receiver
    rec.append(src[-1]); rec_shot.append(src_shot[-1])         # a receiver on a source
    src, rec = np.array(src, np.int64), np.array(rec, np.int64)
    src_shot, rec_shot = np.array(src_shot, np.int32), np.array(rec_shot, np.int32)
    wavelet = rng.standard_normal((nt, len(src)))
    obs = 0.01 * rng.standard_normal((nt, len(rec)))
    return dict(shape=shape, order=order, nt=nt, dtype=dtype, c=c, dt=dt, src=src, rec=rec,
                src_shot=src_shot, rec_shot=rec_shot, wavelet=wavelet, obs=obs, nshot=nshot)


def gershgorin_rows(m, b):
    """Row sums s_i = sum over interior faces of h_f (1/m_i + 1/sqrt(m_i m_j)) of the
    symmetric form M^-1/2 K M^-1/2 (times dx^2), the per-cell stability bound the
    library checks."""
    s = np.zeros(m.shape)
    for ax in range(m.ndim):
        n = m.shape[ax]
        lo = [slice(None)] * m.ndim
        hi = [slice(None)] * m.ndim
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        h = 2 * b[lo] * b[hi] / (b[lo] + b[hi])
        s[lo] += h * (1 / m[lo] + 1 / np.sqrt(m[lo] * m[hi]))
        s[hi] += h * (1 / m[hi] + 1 / np.sqrt(m[lo] * m[hi]))
    return s
