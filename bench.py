"""Throughput of the memory-efficient adjoint sensitivity (forward sweep + superposed
backward sweep) on one MI355X.

One step = one full gradient: fd_sens_forward (nt fused steps: propagate, inject,
sample, residual, K(u,u)) + fd_sens_backward (terminal hand-over, nt - 1 fused
superposed steps with K(v,v), finalisation).  Inputs are resident in HBM before the
timed region; the observed data come from a forward solve in the unperturbed medium.

    python bench.py [--steps K] [--warmup W] [--workload layered3d|layered2d] ...

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: this build measures one GPU.
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


def bytes_per_update(dtype, acc):
    """Algorithmic HBM bytes of one fused cell update: read u^n, u^{n-1}, c and the
    accumulator, write u^{n+1} and the accumulator (the last forward step skips the
    accumulator)."""
    f = 8 if dtype == "f64" else 4
    a = 8 if (acc == "f64" or dtype == "f64") else 4
    return 4 * f + 2 * a, 4 * f


def make_problem(args, torch, wl):
    if args.workload == "layered3d":
        n = args.n or 1024
        nt = args.nt or 3000
        p = wl.layered_3d(n=n, nt=nt, device="cuda")
        c = p.c.float().contiguous()
        c_ref = p.c_ref.float().contiguous()
        desc = f"layered3d {n}^3 f32 order-8 nt={nt}, 1 Ricker source, {len(p.rec)} receivers"
    elif args.workload == "layered2d":
        n = args.n or 2048
        nt = args.nt or 4000
        p = wl.layered_2d(n=n, nt=nt)
        c = torch.as_tensor(p.c, dtype=torch.float32, device="cuda")
        c_ref = torch.as_tensor(p.c_ref, dtype=torch.float32, device="cuda")
        desc = f"layered2d {n}^2 f32 order-8 nt={nt}, 1 Ricker source, {len(p.rec)} receivers"
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    return p, c, c_ref, desc


def cpu_baseline(p, c_dev, args, wl, torch):
    """The FP64 oracle on a bounded sample of the same workload: a crop of the same
    medium around the source with the workload's receivers that fall inside it,
    for a few time steps (forward + superposed backward sweep)."""
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
    return {"value": upd / el / 1e9, "unit": "Gcell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle, crop {'x'.join(map(str, crop))} of the same medium around the "
                      f"source, {len(rec)} receivers, nt={nt_s} ({upd:.3g} cell-updates in {el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered3d", choices=["layered3d", "layered2d"])
    ap.add_argument("--n", type=int, default=0, help="grid side (default: 1024 in 3D, 2048 in 2D)")
    ap.add_argument("--nt", type=int, default=0, help="time steps (default: 3000 in 3D, 4000 in 2D)")
    ap.add_argument("--acc", default="f64", choices=["f64", "f32"])
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--beta", type=float, default=0.005,
                    help="k = beta ||f|| / ||f_dagger||, fixed from the first step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2509_15744_amd import fdwave as fdw
    from paper_2509_15744_amd import workloads as wl

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    p, c, c_ref, desc = make_problem(args, torch, wl)
    log("workload:", desc, f"dt={p.dt:.5g}")
    w = torch.as_tensor(p.wavelet, dtype=torch.float32, device="cuda")
    obs = fdw.fd_forward(c_ref, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, variant=args.variant)
    del c_ref
    torch.cuda.synchronize()
    st = fdw.SweepState(c, p.nt, len(p.rec), acc_dtype=args.acc)
    grad = torch.empty_like(c)
    log(f"setup {time.perf_counter() - t_setup:.1f} s; state "
        f"{(st.u_a.numel() * 8 + st.acc.numel() * st.acc.element_size()) / 2**30:.1f} GiB")
    f_norm = float(np.linalg.norm(p.wavelet)) / p.dx ** len(p.shape)
    k_holder = {}
    timings = []

    def one_step(record):
        tf, tb = fdw.fd_timing(), fdw.fd_timing()
        J = fdw.fd_sens_forward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, obs, st,
                                acc_dtype=args.acc, variant=args.variant, timing=tf)
        if "k" not in k_holder:
            fdag_norm = math.sqrt(2.0 * J / p.dt) / p.dt
            k_holder["k"] = args.beta * f_norm / fdag_norm if fdag_norm > 0 else 1.0
            k_holder["J"] = J
        fdw.fd_sens_backward(c, p.dx, p.order, p.src, w, p.rec, p.dt, p.nt, k_holder["k"], st,
                             grad=grad, acc_dtype=args.acc, variant=args.variant, timing=tb)
        if record:
            timings.append((tf.fwd_ms, tf.fwd_launches, tb.bwd_ms, tb.bwd_launches))
        return J

    for i in range(args.warmup):
        one_step(False)
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(True)
        log(f"timed step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ncell = int(np.prod(p.shape))
    upd_per_step = ncell * (2 * p.nt - 1)
    value = upd_per_step * args.steps / elapsed / 1e9
    b_k, b_nok = bytes_per_update("f32", args.acc)
    # dominant kernel: the fused step; average algorithmic bytes per launch over a step
    bytes_step = ncell * (b_k * (p.nt - 1) + b_nok + b_k * (p.nt - 1))
    launches = sum(t[1] + t[3] for t in timings)
    kern_ms = sum(t[0] + t[2] for t in timings)
    avg_ms = kern_ms / launches
    bytes_launch = bytes_step * args.steps / launches
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": "Gcell-updates/s fwd+adjoint sweep",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "grid": list(p.shape),
            "nt": p.nt,
            "order": p.order,
            "shots": len(p.src),
            "receivers": len(p.rec),
            "accumulator": args.acc,
            "k": k_holder["k"],
            "J": k_holder["J"],
            "variant": args.variant,
            "cell_updates_per_step": upd_per_step,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": "fdw::step_kernel",
            "avg_launch_ms": round(avg_ms, 4),
            "bytes_per_launch": bytes_launch,
            "bytes_per_cell_update": b_k,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p, c, args, wl, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
