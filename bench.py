"""Throughput of the memory-efficient adjoint sensitivity (forward sweep + superposed
backward sweep) on one MI355X.

One step = one full gradient.  Single-medium workloads run fd_sens_forward (nt fused
steps: propagate, inject, sample, residual, K(u,u)) + fd_sens_backward (terminal
hand-over, nt - 1 fused superposed steps with K(v,v), finalisation); shot batches do
the same for all shots with one shared accumulator; the uneven-problem batch runs
fd_adjoint_sensitivity_batched.  Inputs are resident in HBM before the timed region;
observed data come from a forward solve in the unperturbed medium.  The launch shape
is autotuned in the untimed setup.

    python bench.py [--steps K] [--warmup W] [--workload NAME] ...

Workloads: layered3d (default; 1024^3, order 8, nt 3000, one shot), layered2d (2048^2,
order 8, nt 4000), shots3d (4 shots on 1024^3), shots2d (32 shots on 2048^2),
problems2d (16 independent layered problems, sides 256..2048), vd3d (the paper's own
second-order flux-form scheme with variable mass and stiffness on a layered 1024^3
medium, both sensitivities).  ``--method exact`` times the exact re-simulation gradient
(fd_adjoint_exact) instead of the superposition.

After the timed region (single-medium workloads, superposition): the gap of the
gradient to the exact discrete gradient at full size (fd_adjoint_exact on the device),
and on the 256^3 differentiation workload (order 8, nt 2000) the relative errors of
the device gradients against the FP64 oracle references stored in tests/golden and
against central finite differences of the f64 misfit on sampled cells.

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: the benchmark measures one
GPU (the sweep is not sharded across GPUs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


PARTIAL_CYCLE = 16   # accumulating launches per partial-sum cycle (f32 fields, f64 accumulator)


def acc_terms(l, count):
    """Kernel terms of launch l of a sweep accumulating `count` intervals: 0 (none), 1
    (its own interval, the last launch of an odd count) or 3 (its own and the one before,
    odd l): the accumulator is touched by every other launch."""
    if l < 0 or l >= count:
        return 0
    if l & 1:
        return 3
    return 1 if l == count - 1 else 0


def part_mode(l, count):
    """What accumulating launch l does with its terms when f32 partial sums are kept
    (f32 fields, f64 accumulator): 'start' (write the partial sum), 'add' (read and write
    it), 'flush' (read it, read and write the accumulator) or 'direct' (read and write
    the accumulator only), in cycles of PARTIAL_CYCLE accumulating launches."""
    i, total = l >> 1, (count + 1) >> 1
    j = i % PARTIAL_CYCLE
    if i == total - 1:
        return "direct" if j == 0 else "flush"
    if j == 0:
        return "start"
    return "flush" if j == PARTIAL_CYCLE - 1 else "add"


def launch_bytes(group, acc, mode):
    """Algorithmic HBM bytes per cell of one fused step launch advancing `group` fields:
    read u^n, u^{n-1} per field and c once, write u^{n+1} per field, plus what the launch
    does with the accumulator (mode None: nothing; 'direct': read and write it) or with
    the f32 partial sums (see part_mode)."""
    base = 12 * group + 4
    a = 8 if acc == "f64" else 4
    extra = {None: 0, "direct": 2 * a, "start": 4, "add": 8, "flush": 4 + 2 * a}[mode]
    return base + extra


def sweep_bytes(nt, group, acc, partials, nlaunch):
    """Bytes per cell of the `nlaunch` step launches of one sweep accumulating nt - 1
    intervals (nt launches forward, nt - 1 backward)."""
    total = 0
    for l in range(nlaunch):
        terms = acc_terms(l, nt - 1)
        mode = None if not terms else (part_mode(l, nt - 1) if partials else "direct")
        total += launch_bytes(group, acc, mode)
    return total


def gradient_bytes(nt, group, acc, partials=None):
    """Algorithmic bytes per cell of the step launches of one gradient (forward sweep of
    nt launches, backward of nt - 1).  Partial sums are kept for f32 fields with an f64
    accumulator (every workload of this bench runs f32 fields)."""
    if partials is None:
        partials = acc == "f64"
    return sweep_bytes(nt, group, acc, partials, nt) + sweep_bytes(nt, group, acc, partials, nt - 1)


def pair_gradient_bytes(nt, acc, partials):
    """Algorithmic bytes per cell of the launches of one gradient that runs two steps per
    launch (--pairs): a two-step launch reads u^{n-1}, u^n and c (12 B) and writes two
    levels (8 B) plus the kernel terms of the one-step schedule's accumulating step it
    covers (the later of its two steps adds both intervals, or the earlier one its
    own alone); a last odd step runs as a one-step launch.  Returns (bytes, launches)."""
    total = launches = 0
    for nsteps in (nt, nt - 1):   # forward steps n = 0..nt-1, backward l = 0..nt-2
        l = 0
        while l + 1 < nsteps:
            ta, tb = acc_terms(l, nt - 1), acc_terms(l + 1, nt - 1)
            at = l + 1 if tb == 3 else (l if ta else None)
            mode = None if at is None else (part_mode(at, nt - 1) if partials else "direct")
            total += 20 + acc_extra(acc, mode)
            launches += 1
            l += 2
        if l < nsteps:
            terms = acc_terms(l, nt - 1)
            mode = None if not terms else (part_mode(l, nt - 1) if partials else "direct")
            total += launch_bytes(1, acc, mode)
            launches += 1
    return total, launches


def cycle_mode(i, total):
    """Partial-sum mode of the i-th of `total` accumulating launches of a sweep."""
    j = i % PARTIAL_CYCLE
    if i == total - 1:
        return "direct" if j == 0 else "flush"
    if j == 0:
        return "start"
    return "flush" if j == PARTIAL_CYCLE - 1 else "add"


def acc_extra(acc, mode):
    """Bytes per cell an accumulating launch moves for one accumulator in `mode`."""
    a = 8 if acc == "f64" else 4
    return {None: 0, "direct": 2 * a, "start": 4, "add": 8, "flush": 4 + 2 * a}[mode]


def vd_gradient_bytes(nt, acc, partials=None):
    """Algorithmic bytes per cell of the variable-material step launches of one gradient:
    read u^n, b, m, u^{n-1} and write u^{n+1} (20 B), the mass accumulator on every other
    launch (acc_terms) and the stiffness accumulator on every launch, each directly or
    through f32 partial sums in cycles of PARTIAL_CYCLE (f32 fields, f64 accumulators)."""
    if partials is None:
        partials = acc == "f64"
    total = 0
    for nl in (nt, nt - 1):
        for l in range(nl):
            terms = acc_terms(l, nt - 1)
            mass = None if not terms else (part_mode(l, nt - 1) if partials else "direct")
            stiff = cycle_mode(l, nl) if partials else "direct"
            total += 20 + acc_extra(acc, mass) + acc_extra(acc, stiff)
    return total


def make_single(args, torch, wl):
    if args.workload in ("layered3d", "shots3d"):
        n = args.n or 1024
        nt = args.nt or 3000
        shots = None
        if args.workload == "shots3d":
            q = n // 4
            shots = [(a, b) for a in (q, 3 * q) for b in (q, 3 * q)]
        p = wl.layered_3d(n=n, nt=nt, device="cuda", shots=shots)
        c = p.c.float().contiguous()
        c_ref = p.c_ref.float().contiguous()
        desc = f"{args.workload} {n}^3 f32 order-8 nt={nt}, {len(p.src)} shot(s), {len(p.rec)} receivers each"
    else:
        n = args.n or 2048
        nt = args.nt or 4000
        cols = None
        if args.workload == "shots2d":
            cols = [64 * s + 32 for s in range(32)]
        p = wl.layered_2d(n=n, nt=nt, src_cols=cols)
        c = torch.as_tensor(p.c, dtype=torch.float32, device="cuda")
        c_ref = torch.as_tensor(p.c_ref, dtype=torch.float32, device="cuda")
        desc = f"{args.workload} {n}^2 f32 order-8 nt={nt}, {len(p.src)} shot(s), {len(p.rec)} receivers each"
    return p, c, c_ref, desc


def shot_tags(p, np):
    """Every source is its own shot; every shot records with the whole receiver line."""
    ns = len(p.src)
    if ns == 1:
        return p.src, p.rec, None, p.wavelet
    rec = np.tile(p.rec, ns)
    rec_shot = np.repeat(np.arange(ns, dtype=np.int32), len(p.rec))
    src_shot = np.arange(ns, dtype=np.int32)
    return p.src, rec, (src_shot, rec_shot, ns), p.wavelet


def cpu_baseline(p, c_dev, wl):
    """The FP64 oracle on a bounded sample of the same workload: a crop of the same
    medium around the first source with the receivers that fall inside it, for a few
    time steps (forward + superposed backward sweep)."""
    import numpy as np
    import oracle
    shape = p.shape
    if len(shape) == 3:
        crop = (min(256, shape[0]), min(512, shape[1]), min(512, shape[2]))
        nt_s = 30
    else:
        crop = (min(1024, shape[0]), min(2048, shape[1]))
        nt_s = 400
    sx = [int(s) for s in np.unravel_index(int(p.src[0]), shape)]
    lo = [max(0, min(sx[a] - crop[a] // 2, shape[a] - crop[a])) for a in range(len(shape))]
    sl = tuple(slice(lo[a], lo[a] + crop[a]) for a in range(len(shape)))
    c = c_dev[sl].double().cpu().numpy()
    rc = np.array(np.unravel_index(p.rec, shape)).T
    inside = np.all([(rc[:, a] >= lo[a]) & (rc[:, a] < lo[a] + crop[a]) for a in range(len(shape))], axis=0)
    rec = wl.flat(crop, rc[inside] - np.array(lo))
    src = wl.flat(crop, [[sx[a] - lo[a] for a in range(len(shape))]])
    w = p.wavelet[:nt_s, :1]
    obs = np.zeros((nt_s, len(rec)))
    ncell = int(np.prod(crop))
    oracle.build()
    t0 = time.perf_counter()
    oracle.superposition_gradient(c, p.dx, p.order, p.dt, nt_s, src, w, rec, obs, 1e-3)
    el = time.perf_counter() - t0
    upd = ncell * (2 * nt_s - 1)
    cores = oracle.num_threads()
    # the same crop on one thread, for a few steps
    nt_1 = max(2, nt_s // 10)
    prev = oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.superposition_gradient(c, p.dx, p.order, p.dt, nt_1, src, w[:nt_1], rec, obs[:nt_1], 1e-3)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(prev)
    upd1 = ncell * (2 * nt_1 - 1)
    return {"value": upd / el / 1e9, "unit": "Gcell-updates/s", "cores": cores,
            "kind": "oracle",
            "single_thread_value": upd1 / el1 / 1e9,
            "sample": f"FP64 oracle, crop {'x'.join(map(str, crop))} of the same medium around the "
                      f"first source, {len(rec)} receivers, nt={nt_s}, one shot "
                      f"({upd:.3g} cell-updates in {el:.1f} s on {cores} threads; the same crop for "
                      f"nt={nt_1} on one thread: {upd1:.3g} in {el1:.1f} s)"}


def rel_dev(a, b):
    """||a - b|| / ||b|| of two device tensors, accumulated in f64 slab by slab."""
    num = den = 0.0
    for i in range(0, a.shape[0], 32):
        da, db = a[i:i + 32].double(), b[i:i + 32].double()
        num += float(((da - db) ** 2).sum())
        den += float((db ** 2).sum())
    return math.sqrt(num / den) if den > 0 else float("nan")


def accuracy_full(args, torch, fdw, p, c, acq, obs, grad, ncell):
    """Gap of the superposition gradient `grad` to the exact discrete gradient of the
    same run, both on the device (the exact one by re-simulation)."""
    g_ex = torch.empty_like(c)
    t = fdw.fd_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fdw.fd_adjoint_exact(c, p.dx, p.order, acq, None, None, p.dt, p.nt, obs, grad=g_ex, timing=t,
                         acc_dtype=args.acc)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gap = rel_dev(grad, g_ex)
    del g_ex
    return {"gap_vs_exact_resim": gap,
            "exact_resim_s": round(el, 3),
            "exact_resim_gcell_updates_per_s": round(ncell * (2 * p.nt - 1) / el / 1e9, 3),
            "exact_resim_fwd_ms": round(t.fwd_ms, 2), "exact_resim_bwd_ms": round(t.bwd_ms, 2)}


def accuracy_256(np, torch, fdw, wl, acc, fd_cells=8):
    """Device gradients of the 256^3 differentiation workload (smooth speed in [1, 3],
    order 8, nt 2000, f32) against the oracle's FP64 references in tests/golden (sampled
    on every 8th cell per axis): Alg. 1 at the same k, the exact discrete adjoint; and the
    exact gradient against central differences of the f64 misfit (eps 1e-6) on a few
    sampled cells where |g| >= 1e-3 max |g|."""
    path = os.path.join(ROOT, "tests", "golden", "smooth3d_256_nt2000.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    k = float(ref["k"])
    stride = int(ref["stride"])
    s = (slice(None, None, stride),) * 3
    p = wl.smooth_3d(n=256, nt=2000)

    def dev(x, dt):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=dt).cuda()

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    f32, f64 = torch.float32, torch.float64
    c, w, o = dev(p.c, f32), dev(p.wavelet, f32), dev(p.observed, f32)
    g_ap, J = fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, o, k,
                                         acc_dtype=acc)
    g_ex, _ = fdw.fd_adjoint_exact(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, o, acc_dtype=acc)
    ap = g_ap[s].double().cpu().numpy()
    ex = g_ex[s].double().cpu().numpy()
    ref_ex = ref["exact_sample"]
    out = {"workload": "smooth3d 256^3 f32 order-8 nt=2000 (speed in [1, 3]), oracle sample stride 8",
           "k": k,
           "superposition_vs_oracle_same_k": rel(ap, ref["approx_sample"]),
           "exact_resim_vs_oracle_exact": rel(ex, ref_ex),
           "gap_gpu": rel(ap, ref_ex), "gap_oracle": rel(ref["approx_sample"], ref_ex),
           "J_rel_err": abs(J - float(ref["J"])) / float(ref["J"])}
    cand = np.argwhere(np.abs(ref_ex) >= 1e-3 * np.abs(ref_ex).max())
    pick = cand[np.random.default_rng(64).choice(len(cand), size=min(fd_cells, len(cand)), replace=False)]
    c64, w64, o64 = dev(p.c, f64), dev(p.wavelet, f64), dev(p.observed, f64)
    errs = []
    for cell in pick:
        idx = tuple(int(v) * stride for v in cell)
        jj = []
        for sgn in (1.0, -1.0):
            cp = c64.clone()
            cp[idx] += sgn * 1e-6
            tr = fdw.fd_forward(cp, p.dx, p.order, p.src, w64, p.rec, p.dt, p.nt)
            jj.append(fdw.fd_misfit(tr, o64, p.dt))
        fd = (jj[0] - jj[1]) / 2e-6
        errs.append(abs(ex[tuple(cell)] - fd) / abs(fd))
    out["exact_resim_vs_fd_median"] = float(np.median(errs))
    out["exact_resim_vs_fd_max"] = float(np.max(errs))
    out["fd_cells"] = len(errs)
    return out


def run_single(args, np, torch, fdw, wl):
    from paper_2509_15744_amd import calibrate
    p, c, c_ref, desc = make_single(args, torch, wl)
    src, rec, shots, wav = shot_tags(p, np)
    nshot = shots[2] if shots else 1
    log("workload:", desc, f"dt={p.dt:.5g}")
    w = torch.as_tensor(wav, dtype=torch.float32, device="cuda")
    if args.variant:
        best = {"variant": args.variant, "chunk": args.chunk, "max_group": 0,
                "variant_plain": args.variant_plain, "chunk_plain": args.chunk_plain}
        log("launch shape (given):", best)
    else:
        best, best_ms = fdw.fd_autotune(p.shape, p.dx, p.order, torch.float32, nshot=nshot, steps=4,
                                        acc_dtype=args.acc, no_partials=args.no_partials)
        log("launch shape:", best, f"{best_ms:.3f} ms/step in the tuner")
    obs = fdw.fd_forward(c_ref, p.dx, p.order, src, w, rec, p.dt, p.nt, shots=shots)
    del c_ref
    torch.cuda.synchronize()
    st = fdw.SweepState(c, p.nt, len(rec), acc_dtype=args.acc, nshot=nshot)
    grad = torch.empty_like(c)
    w_norm = float(np.linalg.norm(wav))
    holder, timings = {}, []
    acq = fdw.Acquisition(src, w, rec, *(shots if shots else (None, None, 0)))
    opts = dict(acc_dtype=args.acc, variant=best["variant"], chunk=best["chunk"],
                max_group=best["max_group"], variant_plain=best["variant_plain"],
                chunk_plain=best["chunk_plain"], no_partials=args.no_partials, pairs=args.pairs)

    def exact_step(record):
        t = fdw.fd_timing()
        shape = {"variant": args.variant, "chunk": args.chunk} if args.variant else {}
        _, J = fdw.fd_adjoint_exact(c, p.dx, p.order, acq, None, None, p.dt, p.nt, obs, grad=grad,
                                    timing=t, acc_dtype=args.acc, **shape)
        holder.setdefault("k", None)
        holder.setdefault("J", J)
        if record:
            timings.append((t.fwd_ms, t.fwd_launches, t.bwd_ms, t.bwd_launches))

    def one_step(record):
        tf, tb = fdw.fd_timing(), fdw.fd_timing()
        J = fdw.fd_sens_forward(c, p.dx, p.order, acq, None, None, p.dt, p.nt, obs, st, timing=tf, **opts)
        if "k" not in holder:
            holder["k"] = calibrate.auto_k(J, p.dt, w_norm, p.dx, len(p.shape), args.beta)
            holder["J"] = J
        fdw.fd_sens_backward(c, p.dx, p.order, acq, None, None, p.dt, p.nt, holder["k"], st, grad=grad,
                             timing=tb, **opts)
        if record:
            timings.append((tf.fwd_ms, tf.fwd_launches, tb.bwd_ms, tb.bwd_launches))
            holder["pair_launches"] = tf.fwd_pair_launches + tb.bwd_pair_launches

    exact = args.method == "exact"
    elapsed = timed(args, torch, exact_step if exact else one_step)
    ncell = int(np.prod(p.shape))
    upd = ncell * (2 * p.nt - 1) * nshot
    launches = sum(t[1] + t[3] for t in timings)
    kern_ms = sum(t[0] + t[2] for t in timings)
    if exact:
        # forward: one field per launch, no accumulator; backward: u and mu together with
        # the cross accumulator, one launch per shot and step
        # forward: one field per launch, no accumulator; backward: u and mu together
        per_cell = p.nt * launch_bytes(1, args.acc, None) + sweep_bytes(
            p.nt, 2, args.acc, args.acc == "f64" and not args.no_partials, p.nt - 1)
        bytes_all = ncell * nshot * per_cell * args.steps
        bpu = per_cell / (2 * p.nt - 1)
    else:
        group = best["max_group"] or 1
        ngroups = math.ceil(nshot / group)
        per_cell = gradient_bytes(p.nt, group, args.acc, args.acc == "f64" and not args.no_partials)
        if holder.get("pair_launches"):
            per_cell, _ = pair_gradient_bytes(p.nt, args.acc, args.acc == "f64" and not args.no_partials)
        bytes_all = ncell * ngroups * per_cell * args.steps
        bpu = per_cell / (2 * p.nt - 1) / group
    cfg = {"workload": desc, "grid": list(p.shape), "nt": p.nt, "order": p.order, "shots": nshot,
           "receivers": len(rec), "accumulator": args.acc, "partial_sums": args.acc == "f64" and not args.no_partials,
           "two_step_launches": holder.get("pair_launches", 0),
           "method": args.method, "k": holder["k"],
           "J": holder["J"], "launch_shape": best, "cell_updates_per_step": upd}
    acc_info = None
    if not exact and not args.no_accuracy:
        log("accuracy: exact re-simulation gradient at full size ...")
        acc_info = {"full_size": accuracy_full(args, torch, fdw, p, c, acq, obs, grad, ncell * nshot)}
        log("accuracy:", acc_info["full_size"])
    return upd, elapsed, cfg, (bytes_all / launches, kern_ms / launches, bpu), p, c, acc_info


def cpu_baseline_vd(q, m_dev, b_dev, wl):
    """The FP64 oracle of the variable-material scheme on a bounded sample of the same
    workload: a 128 x 256 x 256 crop around the source with the receivers inside it,
    nt = 20 (forward + superposed backward sweep)."""
    import numpy as np
    import oracle
    shape = q["shape"]
    crop = (min(128, shape[0]), min(256, shape[1]), min(256, shape[2]))
    nt_s = 20
    sx = [int(v) for v in np.unravel_index(int(q["src"][0]), shape)]
    lo = [max(0, min(sx[a] - crop[a] // 2, shape[a] - crop[a])) for a in range(3)]
    sl = tuple(slice(lo[a], lo[a] + crop[a]) for a in range(3))
    m = m_dev[sl].double().cpu().numpy()
    b = b_dev[sl].double().cpu().numpy()
    rc = np.array(np.unravel_index(q["rec"], shape)).T
    inside = np.all([(rc[:, a] >= lo[a]) & (rc[:, a] < lo[a] + crop[a]) for a in range(3)], axis=0)
    rec = wl.flat(crop, rc[inside] - np.array(lo))
    src = wl.flat(crop, [[sx[a] - lo[a] for a in range(3)]])
    obs = np.zeros((nt_s, len(rec)))
    oracle.build()
    t0 = time.perf_counter()
    oracle.vd_superposition_gradient(m, b, q["dx"], q["dt"], nt_s, src, q["wavelet"][:nt_s], rec, obs, 1e-3)
    el = time.perf_counter() - t0
    upd = int(np.prod(crop)) * (2 * nt_s - 1)
    return {"value": upd / el / 1e9, "unit": "Gcell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle (variable material), crop {'x'.join(map(str, crop))} of the same medium "
                      f"around the source, {len(rec)} receivers, nt={nt_s}, one shot "
                      f"({upd:.3g} cell-updates in {el:.1f} s)"}


def run_vd(args, np, torch, fdw, wl):
    """The paper's second-order flux-form scheme with variable mass and stiffness on the
    layered 1024^3 medium: one gradient = fd_vd_adjoint_sensitivity (both sensitivities)."""
    from paper_2509_15744_amd import calibrate
    n = args.n or 1024
    nt = args.nt or 3000
    q = wl.layered_material_3d(n=n, nt=nt, device="cuda")
    desc = (f"vd3d {n}^3 f32 order-2 variable mass and stiffness nt={nt}, 1 shot(s), "
            f"{len(q['rec'])} receivers each")
    log("workload:", desc, f"dt={q['dt']:.5g}")
    w = torch.as_tensor(q["wavelet"], dtype=torch.float32, device="cuda")
    variant = args.variant   # 0: the library's default tile shape
    opts = dict(acc_dtype=args.acc, variant=variant, chunk=args.chunk, no_partials=args.no_partials)
    obs = fdw.fd_vd_forward(q["m_ref"], q["b_ref"], q["dx"], q["src"], w, q["rec"], q["dt"], nt, **opts)
    tr = fdw.fd_vd_forward(q["m"], q["b"], q["dx"], q["src"], w, q["rec"], q["dt"], nt, **opts)
    J0 = fdw.fd_misfit(tr, obs, q["dt"])
    del q["m_ref"], q["b_ref"], tr
    k = calibrate.auto_k(J0, q["dt"], float(np.linalg.norm(q["wavelet"])), q["dx"], 3, args.beta)
    gm, gb = torch.empty_like(q["m"]), torch.empty_like(q["m"])
    torch.cuda.synchronize()
    timings, holder = [], {}

    def one_step(record):
        t = fdw.fd_timing()
        _, _, J = fdw.fd_vd_adjoint_sensitivity(q["m"], q["b"], q["dx"], q["src"], w, q["rec"], q["dt"], nt,
                                                obs, k, grad_m=gm, grad_b=gb, timing=t, **opts)
        holder["J"] = J
        if record:
            timings.append((t.fwd_ms, t.fwd_launches, t.bwd_ms, t.bwd_launches))

    elapsed = timed(args, torch, one_step)
    ncell = n ** 3
    upd = ncell * (2 * nt - 1)
    launches = sum(t[1] + t[3] for t in timings)
    kern_ms = sum(t[0] + t[2] for t in timings)
    per_cell = vd_gradient_bytes(nt, args.acc, args.acc == "f64" and not args.no_partials)
    bytes_all = ncell * per_cell * args.steps
    cfg = {"workload": desc, "grid": [n, n, n], "nt": nt, "order": 2, "shots": 1, "receivers": len(q["rec"]),
           "accumulator": args.acc, "method": "superposition", "k": k, "J": holder["J"],
           "launch_shape": {"variant": variant or "library default (3D: 5)", "chunk": args.chunk}, "cell_updates_per_step": upd}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, variable material) ...")
        cfg["_cpu_baseline"] = cpu_baseline_vd(q, q["m"], q["b"], wl)
    return upd, elapsed, cfg, (bytes_all / launches, kern_ms / launches, per_cell / (2 * nt - 1)), None, None, None


def cpu_baseline_vd2d(q, m_dev, b_dev, wl, crop=(1024, 2048), nt_s=100):
    """The FP64 oracle of the variable-material scheme on a bounded sample of the 2D
    design workload: a crop around the source (design box and region cells inside it
    keep their material and receivers), nt_s steps forward + superposed backward."""
    import numpy as np
    import oracle
    shape = q["shape"]
    crop = (min(crop[0], shape[0]), min(crop[1], shape[1]))
    sx = [int(v) for v in np.unravel_index(int(q["src"][0]), shape)]
    lo = [max(0, min(sx[a] - crop[a] // 2, shape[a] - crop[a])) for a in range(2)]
    sl = tuple(slice(lo[a], lo[a] + crop[a]) for a in range(2))
    m = m_dev[sl].double().cpu().numpy()
    b = b_dev[sl].double().cpu().numpy()
    rc = np.array(np.unravel_index(q["rec"], shape)).T
    inside = np.all([(rc[:, a] >= lo[a]) & (rc[:, a] < lo[a] + crop[a]) for a in range(2)], axis=0)
    rec = wl.flat(crop, rc[inside] - np.array(lo)) if inside.any() else wl.flat(crop, [[0, 0]])
    src = wl.flat(crop, [[sx[a] - lo[a] for a in range(2)]])
    obs = np.zeros((nt_s, len(rec)))
    oracle.build()
    t0 = time.perf_counter()
    oracle.vd_superposition_gradient(m, b, q["dx"], q["dt"], nt_s, src, q["wavelet"][:nt_s], rec, obs, 1e-3)
    el = time.perf_counter() - t0
    upd = int(np.prod(crop)) * (2 * nt_s - 1)
    return {"value": upd / el / 1e9, "unit": "Gcell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle (variable material), crop {'x'.join(map(str, crop))} around the source of "
                      f"the same material, {len(rec)} receivers, nt={nt_s}, the two sweeps only "
                      f"({upd:.3g} cell-updates in {el:.1f} s)"}


def run_tato(args, np, torch, fdw, wl):
    """One iteration of the two-dimensional acoustic black-hole design at the paper's
    size: design map (filter r_f = 1.5, projection beta = 1, eta = 0.5, clip, the
    air/solid map), forward sweep with the region objective, superposed backward sweep,
    chain rule, Adam step (lr 0.1) with clip; everything on the device."""
    from paper_2509_15744_amd import design as dz
    q = wl.tato_2d(nt=args.nt or 17184)
    nt = q["nt"]
    shape = q["shape"]
    mats = q["materials"]
    material = fdw.two_material(mats["rho1"], mats["rho2"], mats["kappa1"], mats["kappa2"])
    d = fdw.make_design(shape, q["design_origin"], q["design_extent"], fdw.FD_F32, material, 1.5, 1.0, 0.5,
                        0.0, 1.0)
    # the paper's dt unless a design could break the per-cell stability bound at it
    q["dt"] = min(q["dt"], dz.stable_dt(material, 0.0, 1.0, q["dx"], 2))
    f32 = torch.float32
    m = torch.full(shape, 1.0 / mats["kappa1"], dtype=f32, device="cuda")
    b = torch.full(shape, 1.0 / mats["rho1"], dtype=f32, device="cuda")
    rec = dz.region_receivers(shape, q["region_origin"], q["region_extent"])
    obs = torch.zeros((nt, len(rec)), dtype=f32, device="cuda")
    w = torch.as_tensor(q["wavelet"], dtype=f32, device="cuda")
    variant = args.variant   # 0: the library's choice
    prob = dz.DesignProblem(design=d, m=m, b=b, dx=q["dx"], src=q["src"], wavelet=w, rec=rec, observed=obs,
                            dt=q["dt"], nt=nt, scale=dz.region_scale(len(rec)), acc_dtype=args.acc,
                            variant=variant, chunk=args.chunk)
    gamma0 = torch.full(q["design_extent"], 0.5, dtype=f32, device="cuda")
    loop = dz.AdamDesign(prob, gamma0, lr=0.1)
    desc = (f"tato2d {shape[0]}x{shape[1]} f32 order-2 air/solid design iteration nt={nt}, "
            f"design box {q['design_extent'][0]}x{q['design_extent'][1]}, {len(rec)} region receivers")
    log("workload:", desc, f"dt={q['dt']:.5g}")
    timings, holder = [], {}

    def one_step(record):
        t = fdw.fd_timing()
        loop.sweep_opts = {"timing": t, "no_partials": args.no_partials}
        holder["C"] = loop.step()
        if record:
            timings.append((t.fwd_ms, t.fwd_launches, t.bwd_ms, t.bwd_launches))

    elapsed = timed(args, torch, one_step)
    ncell = shape[0] * shape[1]
    upd = ncell * (2 * nt - 1)
    launches = sum(t[1] + t[3] for t in timings)
    kern_ms = sum(t[0] + t[2] for t in timings)
    per_cell = vd_gradient_bytes(nt, args.acc, args.acc == "f64" and not args.no_partials)
    bytes_all = ncell * per_cell * args.steps
    cfg = {"workload": desc, "grid": list(shape), "nt": nt, "order": 2, "shots": 1, "receivers": len(rec),
           "design_cells": int(np.prod(q["design_extent"])), "accumulator": args.acc,
           "method": "superposition", "k": loop.k, "objective": holder["C"], "objective_history": loop.history,
           "sweep_kernel_ms_per_step": kern_ms / args.steps,
           "launch_shape": {"variant": variant, "chunk": args.chunk}, "cell_updates_per_step": upd}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, variable material, 2D crop) ...")
        cfg["_cpu_baseline"] = cpu_baseline_vd2d({**q, "rec": rec}, m, b, wl)
    return upd, elapsed, cfg, (bytes_all / launches, kern_ms / launches, per_cell / (2 * nt - 1)), None, None, None


def run_fwi(args, np, torch, fdw, wl):
    """One iteration of the three-dimensional FWI at the paper's size (976 x 503 x 503,
    N = 7200, one source: the paper times FWI per source): the indicator on the whole
    grid through rho-scaling (no filter or projection, clip to [1e-5, 1]), forward
    sweep against traces of the voided specimen, superposed backward sweep, chain rule,
    Adam step (lr 0.2, the paper's alpha)."""
    from paper_2509_15744_amd import design as dz
    q = wl.fwi_3d(nt=args.nt or 7200, device="cuda", **({"n1": args.n, "n2": args.n} if args.n else {}))
    shape, nt = q["shape"], q["nt"]
    material = fdw.rho_scaling(q["rho0"], q["c0"])
    # the paper's dt unless a design could break the per-cell stability bound at it
    q["dt"] = min(q["dt"], dz.stable_dt(material, q["eps"], 1.0, q["dx"], 3))
    d = fdw.make_design(shape, (0, 0, 0), shape, fdw.FD_F32, material, 0.0, 0.0, 0.5, q["eps"], 1.0)
    f32 = torch.float32
    m = torch.empty(shape, dtype=f32, device="cuda")
    b = torch.empty_like(m)
    w = torch.as_tensor(q["wavelet"], dtype=f32, device="cuda")
    fdw.fd_design_map(d, q["gamma_true"], m, b)
    obs = fdw.fd_vd_forward(m, b, q["dx"], q["src"], w, q["rec"], q["dt"], nt, variant=args.variant)
    del q["gamma_true"]
    prob = dz.DesignProblem(design=d, m=m, b=b, dx=q["dx"], src=q["src"], wavelet=w, rec=q["rec"], observed=obs,
                            dt=q["dt"], nt=nt, acc_dtype=args.acc, variant=args.variant, chunk=args.chunk)
    loop = dz.AdamDesign(prob, q["gamma_start"], lr=0.2, lo=q["eps"], hi=1.0)
    del q["gamma_start"]
    desc = (f"fwi3d {shape[0]}x{shape[1]}x{shape[2]} f32 order-2 rho-scaling design iteration nt={nt}, "
            f"1 source, {len(q['rec'])} receivers")
    log("workload:", desc, f"dt={q['dt']:.5g}")
    timings, holder = [], {}

    def one_step(record):
        t = fdw.fd_timing()
        loop.sweep_opts = {"timing": t, "no_partials": args.no_partials}
        holder["C"] = loop.step()
        if record:
            timings.append((t.fwd_ms, t.fwd_launches, t.bwd_ms, t.bwd_launches))

    elapsed = timed(args, torch, one_step)
    ncell = int(np.prod(shape))
    upd = ncell * (2 * nt - 1)
    launches = sum(t[1] + t[3] for t in timings)
    kern_ms = sum(t[0] + t[2] for t in timings)
    per_cell = vd_gradient_bytes(nt, args.acc, args.acc == "f64" and not args.no_partials)
    cfg = {"workload": desc, "grid": list(shape), "nt": nt, "order": 2, "shots": 1, "receivers": len(q["rec"]),
           "design_cells": ncell, "accumulator": args.acc, "method": "superposition", "k": loop.k,
           "objective": holder["C"], "objective_history": loop.history,
           "sweep_kernel_ms_per_step": kern_ms / args.steps,
           "launch_shape": {"variant": args.variant, "chunk": args.chunk}, "cell_updates_per_step": upd}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, variable material) ...")
        cfg["_cpu_baseline"] = cpu_baseline_vd(q, m, b, wl)
    return upd, elapsed, cfg, (ncell * per_cell * args.steps / launches, kern_ms / launches,
                               per_cell / (2 * nt - 1)), None, None, None


def run_autograd(args, np, torch, fdw, wl):
    """The differentiation workload (smooth speed in [1, 3], 256^3, order 8, nt 2000,
    f32): one timed step = J(c) through the autograd Function and .backward() (the
    forward sweep, then the superposed backward sweep as the hand-written backward),
    next to fd_adjoint_sensitivity on the same problem (the plain single-shot call) and
    the two gradients' relative difference."""
    from paper_2509_15744_amd import autograd, calibrate
    n = args.n or 256
    nt = args.nt or 2000
    p = wl.smooth_3d(n=n, nt=nt)
    f32 = torch.float32
    c = torch.as_tensor(p.c, dtype=f32, device="cuda")
    w = torch.as_tensor(p.wavelet, dtype=f32, device="cuda")
    obs = torch.as_tensor(p.observed, dtype=f32, device="cuda")
    tr = fdw.fd_forward(c, p.dx, p.order, p.src, w, p.rec, p.dt, nt)
    J0 = fdw.fd_misfit(tr, obs, p.dt)
    k = calibrate.auto_k(J0, p.dt, float(np.linalg.norm(p.wavelet)), p.dx, 3, args.beta)
    shape = None
    if not args.variant:   # tune once; both paths then take the tuned shape (variant 0)
        shape, _ = fdw.fd_autotune(p.shape, p.dx, p.order, torch.float32, steps=4, acc_dtype=args.acc)
        log("launch shape:", shape)
    prob = autograd.SensProblem(dx=p.dx, order=p.order, src=p.src, rec=p.rec, wavelet=w, observed=obs, dt=p.dt,
                                nt=nt, acc_dtype=args.acc, variant=args.variant, chunk=args.chunk)
    desc = f"autograd3d {n}^3 f32 order-{p.order} nt={nt}, smooth speed in [1, 3], {len(p.rec)} receivers"
    log("workload:", desc, f"dt={p.dt:.5g}")
    holder = {}

    def one_step(record):
        cg = c.clone().requires_grad_(True)
        J = autograd.misfit(cg, prob, k)
        J.backward()
        holder["grad"] = cg.grad
        holder["J"] = float(J.item())

    elapsed = timed(args, torch, one_step)
    ncell = n ** 3
    upd = ncell * (2 * nt - 1)
    # the plain call on the same problem: wall time and the step kernel's launch record
    grad = torch.empty_like(c)
    timings = []
    for rec in (False, True):
        t = fdw.fd_timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fdw.fd_adjoint_sensitivity(c, p.dx, p.order, p.src, w, p.rec, p.dt, nt, obs, k, grad=grad, timing=t,
                                   acc_dtype=args.acc, variant=args.variant, chunk=args.chunk)
        torch.cuda.synchronize()
        if rec:
            plain_s = time.perf_counter() - t0
            timings.append((t.fwd_ms, t.fwd_launches, t.bwd_ms, t.bwd_launches))
    g_ag = holder["grad"].double()
    diff = float(torch.linalg.vector_norm(g_ag - grad.double()) / torch.linalg.vector_norm(grad.double()))
    launches = sum(t[1] + t[3] for t in timings)
    kern_ms = sum(t[0] + t[2] for t in timings)
    per_cell = gradient_bytes(nt, 1, args.acc)
    cfg = {"workload": desc, "grid": [n, n, n], "nt": nt, "order": p.order, "shots": 1, "receivers": len(p.rec),
           "accumulator": args.acc, "k": k, "J": holder["J"],
           "plain_call_gcell_updates_per_s": upd / plain_s / 1e9,
           "autograd_over_plain_time": (elapsed / args.steps) / plain_s,
           "grad_rel_diff_autograd_vs_plain": diff, "launch_shape": shape, "cell_updates_per_step": upd}
    return upd, elapsed, cfg, (ncell * per_cell / launches, kern_ms / launches, per_cell / (2 * nt - 1)), \
        None, None, None


def run_problems(args, np, torch, fdw, wl):
    """16 independent layered problems with sides drawn uniformly from 256..2048 (seeded),
    each with its own medium, dt, source at the top centre and receivers every 4 cells."""
    from paper_2509_15744_amd import calibrate
    rng = np.random.default_rng(33)
    sides = sorted(int(s) for s in rng.integers(256, 2049, size=16))
    nt = args.nt or 4000
    items, ncell_all = [], 0
    probs = []
    for i, n in enumerate(sides):
        p = wl.layered_2d(n=n, nt=nt, seed=100 + i)
        c = torch.as_tensor(p.c, dtype=torch.float32, device="cuda")
        c_ref = torch.as_tensor(p.c_ref, dtype=torch.float32, device="cuda")
        w = torch.as_tensor(p.wavelet, dtype=torch.float32, device="cuda")
        obs = fdw.fd_forward(c_ref, p.dx, p.order, p.src, w, p.rec, p.dt, nt)
        J = fdw.fd_misfit(fdw.fd_forward(c, p.dx, p.order, p.src, w, p.rec, p.dt, nt), obs, p.dt)
        k = calibrate.auto_k(J, p.dt, float(np.linalg.norm(p.wavelet)), p.dx, 2, args.beta)
        items.append(fdw.Problem(c, p.dx, p.order, p.src, w, p.rec, p.dt, nt, obs, k))
        probs.append(p)
        ncell_all += n * n
    desc = f"problems2d: 16 layered problems, sides {sides[0]}..{sides[-1]}, f32 order-8 nt={nt}"
    log("workload:", desc)
    timings, holder = [], {}
    # one batch plan (host work once), run per step on the current stream; with --graph
    # the run is captured once and each step replays the graph
    plan = fdw.BatchPlan(items, persistent=args.persistent, timing=fdw.fd_timing(), variant=args.variant or 1,
                         acc_dtype=args.acc, chunk=args.chunk)
    J = torch.zeros(len(items), dtype=torch.float64, device="cuda")
    graph = None
    if args.graph:
        plan.run(J)   # warm-up outside the capture
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.run(J)

    def one_step(record):
        if graph is not None:
            graph.replay()
        else:
            plan.run(J)
        if record:
            t = plan.timing()
            timings.append((t.fwd_ms, t.fwd_launches, t.bwd_ms, t.bwd_launches))
            holder["persistent_blocks"] = t.persistent_blocks

    elapsed = timed(args, torch, one_step)
    if not bool(torch.isfinite(J).all()):
        raise RuntimeError("problems2d: a misfit is not finite")
    upd = ncell_all * (2 * nt - 1)
    launches = sum(t[1] + t[3] for t in timings)
    kern_ms = sum(t[0] + t[2] for t in timings)
    per_cell = gradient_bytes(nt, 1, args.acc)
    bytes_all = ncell_all * per_cell * args.steps
    cfg = {"workload": desc, "sides": sides, "nt": nt, "order": 8, "problems": 16, "variant": args.variant or 1,
           "chunk": args.chunk or "library",
           "accumulator": args.acc, "graph": bool(args.graph), "persistent": bool(args.persistent),
           "cell_updates_per_step": upd, "persistent_blocks": holder.get("persistent_blocks"),
           "plan": "one fd_batch_plan; steps run it"
           + (" as a captured graph replay" if args.graph else " directly")}
    plan.close()
    return (upd, elapsed, cfg, (bytes_all / launches, kern_ms / launches, per_cell / (2 * nt - 1)),
            probs[0], items[0].c, None)


STEP_KERNEL_SOURCES = ("fdw_internal.h", "fdw_step_body.h", "fdw_step.hip")


def step_kernel_sha():
    """sha256 over the sources of the single-problem step kernel, in this order."""
    import hashlib
    h = hashlib.sha256()
    for name in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_15744_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def gradient_launch_kinds(nt, partials):
    """How many step launches of each kind one gradient (one step per launch) runs:
    None for the launches without kernel terms, else the partial-sum mode
    ('start', 'add', 'flush', 'direct')."""
    kinds = {}
    for nlaunch in (nt, nt - 1):
        for l in range(nlaunch):
            terms = acc_terms(l, nt - 1)
            k = None if not terms else (part_mode(l, nt - 1) if partials else "direct")
            kinds[k] = kinds.get(k, 0) + 1
    return kinds


def measured_traffic(args, shape, nt):
    """HBM bytes per step launch of one gradient from the committed rocprofv3 counter
    record of the default workload (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated,
    per launch kind and shape), averaged over this gradient's launches; None when this
    run is another workload, runs a launch kind or shape the record lacks, or the kernel
    source changed since."""
    if (args.workload != "layered3d" or args.n not in (0, 1024) or args.acc != "f64"
            or args.method != "superposition" or not shape or args.pairs > 0):
        return None
    rec = os.path.join(ROOT, "profiles", "step_kernel_layered3d_1024_traffic.md")
    try:
        lines = open(rec).read().splitlines()
        sha = step_kernel_sha()
    except OSError:
        return None
    recorded_sha = next((ln.split(": ", 1)[1].strip() for ln in lines if ln.startswith("source_sha256: ")), "")
    if recorded_sha != sha:
        return None
    table = {}
    for ln in lines:   # traffic_kind: <kind> <variant> <chunk> <bytes per launch>
        if ln.startswith("traffic_kind: "):
            kind, variant, chunk, nbytes = ln.split(": ", 1)[1].split()
            table[(kind, int(variant), int(chunk))] = float(nbytes)
    total = count = 0.0
    for kind, n in gradient_launch_kinds(nt, True).items():
        key = ("plain", shape["variant_plain"], shape["chunk_plain"]) if kind is None else \
            (kind, shape["variant"], shape["chunk"])
        if key not in table:
            return None
        total += n * table[key]
        count += n
    return total / count


# The paper's own figure for the same workload and metric, where it has one (Tab.
# timings, A100: time per step of a gradient per source; Gcell-updates/s derived as
# 2 dofs / that time), valid at the workload's default size and N only.
PAPER_SAME_WORKLOAD = {
    "tato2d": 19.5,   # 2D TATO 5403 x 2703, N = 17184, one source
    "fwi3d": 3.09,    # 3D FWI 503 x 503 x 976, N = 7200, per source
}


def copy_probe(torch, nbytes=1 << 30, reps=5):
    """HBM rate of a plain device-to-device copy (read + write bytes counted) on the
    current stream, timed with HIP events: what a streaming kernel with no reuse
    reaches on this device, next to the 8 TB/s peak."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    del src, dst
    return round(2.0 * nbytes * reps / (ms * 1e-3) / 1e9, 1)


def timed(args, torch, one_step):
    """Runs the warm-up steps, then times the steps, within wall budgets: warm-up stops
    once its time passes --warmup-budget-s (at least one step runs), and no timed step
    starts once the elapsed time plus the slowest step so far would pass --budget-s (at
    least one step is timed).  args.steps and args.warmup are set to the counts actually
    run (the requested ones stay in args.steps_requested / args.warmup_requested), so
    every figure derived from args.steps counts the steps that were timed."""
    args.steps_requested, args.warmup_requested = args.steps, args.warmup
    w0 = time.perf_counter()
    done = 0
    for i in range(args.warmup):
        one_step(False)
        done += 1
        log(f"warmup step {i + 1}/{args.warmup} done")
        if time.perf_counter() - w0 > args.warmup_budget_s:
            break
    args.warmup = done
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, slowest = 0, 0.0
    for i in range(args.steps):
        s0 = time.perf_counter()
        one_step(True)
        torch.cuda.synchronize()
        slowest = max(slowest, time.perf_counter() - s0)
        done += 1
        log(f"timed step {i + 1}/{args.steps} done")
        if time.perf_counter() - t0 + slowest > args.budget_s:
            break
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if done < args.steps:
        log(f"time budget {args.budget_s:.0f} s reached: {done} of {args.steps} steps timed")
    args.steps = done
    return elapsed


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--budget-s", type=float, default=120.0,
                    help="wall budget of the timed steps: no step starts that would pass it")
    ap.add_argument("--warmup-budget-s", type=float, default=20.0,
                    help="warm-up stops once it has taken this long (at least one step runs)")
    ap.add_argument("--workload", default="layered3d",
                    choices=["layered3d", "layered2d", "shots3d", "shots2d", "problems2d", "vd3d", "tato2d",
                             "autograd3d", "fwi3d"])
    ap.add_argument("--n", type=int, default=0, help="grid side (default: 1024 in 3D, 2048 in 2D)")
    ap.add_argument("--nt", type=int, default=0, help="time steps (default: 3000 in 3D, 4000 in 2D)")
    ap.add_argument("--acc", default="f64", choices=["f64", "f32"])
    ap.add_argument("--variant", type=int, default=0, help="force a tile variant (default: autotuned)")
    ap.add_argument("--chunk", type=int, default=0, help="with --variant: planes per block (0: library)")
    ap.add_argument("--variant-plain", type=int, default=0,
                    help="with --variant: tile variant of the launches without accumulator (0: same)")
    ap.add_argument("--chunk-plain", type=int, default=0, help="with --variant-plain: planes per block")
    ap.add_argument("--graph", type=int, default=1, help="problems2d: replay sweeps as hipGraphs")
    ap.add_argument("--persistent", type=int, default=0, help="problems2d: one cooperative launch per sweep")
    ap.add_argument("--beta", type=float, default=0.005,
                    help="k = beta ||f|| / ||fdag||, fixed from the first step")
    ap.add_argument("--method", default="superposition", choices=["superposition", "exact"],
                    help="single-medium workloads: the gradient that is timed")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the accuracy section")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pairs", type=int, default=0, choices=[-1, 0, 1],
                    help="1: two time steps per launch (3D, one shot); 0: library choice; -1: never")
    ap.add_argument("--no-partials", action="store_true",
                    help="every accumulating step reads and writes the f64 accumulator (no f32 partial sums)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (the sweep is not sharded across GPUs); --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2509_15744_amd import fdwave as fdw
    from paper_2509_15744_amd import workloads as wl

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    runner = {"problems2d": run_problems, "vd3d": run_vd, "tato2d": run_tato,
              "autograd3d": run_autograd, "fwi3d": run_fwi}.get(args.workload, run_single)
    upd, elapsed, cfg, (bytes_launch, avg_ms, bpu), p0, c0, accuracy = runner(args, np, torch, fdw, wl)
    if accuracy is not None:
        log("accuracy: 256^3 gradients against the oracle references ...")
        a256 = accuracy_256(np, torch, fdw, wl, args.acc)
        if a256 is not None:
            accuracy["oracle_256"] = a256
            log("accuracy:", a256)
    log(f"total {time.perf_counter() - t_setup:.1f} s")
    value = upd * args.steps / elapsed / 1e9
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": "Gcell-updates/s fwd+adjoint sweep",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "steps_requested": args.steps_requested,
        "warmup_requested": args.warmup_requested,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args, cfg.get("launch_shape"), cfg.get("nt", 0)),
            "kernel": "fdw::pair_kernel" if cfg.get("two_step_launches") else
                      {"problems2d": "fdw::step_multi_kernel", "vd3d": "fdw::vd_step_kernel",
                       "tato2d": "fdw::vd_step_kernel", "fwi3d": "fdw::vd_step_kernel"}.get(
                args.workload, "fdw::step_kernel"),
            "avg_launch_ms": round(avg_ms, 4),
            "bytes_per_launch": bytes_launch,
            "bytes_per_shot_cell_update": bpu,
            "copy_probe_gbs": copy_probe(torch),
        },
    }
    if args.workload in ("layered3d", "layered2d", "autograd3d") and args.acc == "f64" and args.method == "superposition":
        # the same throughput priced at the 24 B per cell update of the step without partial
        # sums (every other launch reading and writing the f64 accumulator): what the
        # partial sums save shows here, not in `frac`, which uses the bytes actually due
        out["roofline"]["effective_gbs_at_24B"] = round(value * 24.0, 1)
        out["roofline"]["effective_frac_at_24B"] = round(value * 24.0 / HBM_PEAK_GBS, 4)
    if args.workload in PAPER_SAME_WORKLOAD and not args.nt and not args.n:
        out["context"] = {"paper_a100_gcell_updates_per_s": PAPER_SAME_WORKLOAD[args.workload],
                          "note": "another machine and the paper's own code: context, not a baseline"}
    if accuracy is not None:
        out["accuracy"] = accuracy
    if "_cpu_baseline" in cfg:
        out["cpu_baseline"] = cfg.pop("_cpu_baseline")
    elif not args.no_cpu_baseline and p0 is not None:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p0, c0, wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
