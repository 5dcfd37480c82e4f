"""Batching: several shots on one medium (shot-tagged acquisition, shared accumulator,
S shots per launch) and independent problems of uneven sizes in lock-step launches
(optionally captured in a hipGraph), against single-shot runs and the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2509_15744_amd import workloads as wl
from helpers import rel, say, shot_problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdw():
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    from paper_2509_15744_amd import fdwave
    return fdwave


def _oracle_sum(P, k):
    """Sum over shots of the oracle's single-shot Alg. 1 (gradients and J add up)."""
    g = np.zeros(P["shape"])
    J = 0.0
    tr = np.zeros((P["nt"], len(P["rec"])))
    for s in range(P["nshot"]):
        si = np.where(P["src_shot"] == s)[0]
        ri = np.where(P["rec_shot"] == s)[0]
        gs, Js, trs = oracle.superposition_gradient(P["c"], 1.0, P["order"], P["dt"], P["nt"],
                                                    P["src"][si], P["wavelet"][:, si], P["rec"][ri],
                                                    P["obs"][:, ri], k)
        g += gs
        J += Js
        tr[:, ri] = trs
    return g, J, tr


@pytest.mark.parametrize("shape,nshot,order,max_group", [
    ((14, 11, 70), 4, 8, 0),
    ((14, 11, 70), 7, 8, 0),      # groups 4 + 2 + 1
    ((14, 11, 70), 3, 4, 2),      # groups 2 + 1
    ((40, 66), 5, 8, 0),
    ((40, 66), 6, 2, 1),          # one shot per launch
])
def test_shots_match_oracle_sum(fdw, shape, nshot, order, max_group):
    """f64: the shot batch equals the sum of per-shot oracle runs (J, traces, gradient)."""
    P = shot_problem(shape, nshot, order, 33, "f64", seed=nshot + len(shape))
    k = 0.05
    g_o, J_o, tr_o = _oracle_sum(P, k)
    f64 = torch.float64
    tr = torch.empty((P["nt"], len(P["rec"])), dtype=f64, device="cuda")
    shots = (P["src_shot"], P["rec_shot"], nshot)
    for variant in [v for v in fdw.variants_for(shape) if v <= 2]:
        say("shots", shape, nshot, order, "variant", variant, "max_group", max_group)
        g, J = fdw.fd_adjoint_sensitivity(to_dev(P["c"], f64), 1.0, order, P["src"],
                                          to_dev(P["wavelet"], f64), P["rec"], P["dt"], P["nt"],
                                          to_dev(P["obs"], f64), k, traces=tr, shots=shots,
                                          variant=variant, max_group=max_group)
        assert rel(tr.cpu().numpy(), tr_o) < 1e-12
        assert abs(J - J_o) < 1e-12 * J_o
        assert rel(g.cpu().numpy(), g_o) < 1e-9


def test_shots_f32_and_split(fdw):
    """f32 shot batch within 1e-4 of the oracle; the split forward/backward pair with
    caller-owned [nshot][ncell] state gives the fused call's result bitwise."""
    P = shot_problem((21, 16, 64), 4, 8, 60, "f32", seed=3)
    k = 0.05
    g_o, J_o, _ = _oracle_sum(P, k)
    f32 = torch.float32
    c, w, obs = to_dev(P["c"], f32), to_dev(P["wavelet"], f32), to_dev(P["obs"], f32)
    shots = (P["src_shot"], P["rec_shot"], 4)
    g, J = fdw.fd_adjoint_sensitivity(c, 1.0, 8, P["src"], w, P["rec"], P["dt"], P["nt"], obs, k,
                                      shots=shots)
    assert rel(g.cpu().numpy(), g_o) < 1e-4
    st = fdw.SweepState(c, P["nt"], len(P["rec"]), nshot=4)
    J2 = fdw.fd_sens_forward(c, 1.0, 8, P["src"], w, P["rec"], P["dt"], P["nt"], obs, st, shots=shots)
    g2 = fdw.fd_sens_backward(c, 1.0, 8, P["src"], w, P["rec"], P["dt"], P["nt"], k, st, shots=shots)
    assert J2 == J and torch.equal(g2, g)


def test_shot_tags_are_validated(fdw):
    P = shot_problem((10, 10, 16), 2, 4, 5, "f32", seed=1)
    bad = P["rec_shot"].copy()
    bad[0] = 2
    f32 = torch.float32
    with pytest.raises(fdw.FdError) as e:
        fdw.fd_forward(to_dev(P["c"], f32), 1.0, 4, P["src"], to_dev(P["wavelet"], f32), P["rec"],
                       P["dt"], 5, shots=(P["src_shot"], bad, 2))
    assert e.value.code == fdw.FD_E_ARG and "shot out of range" in str(e.value)


def _uneven_problems(ndim, nprob, dtype, seed):
    rng = np.random.default_rng(seed)
    probs = []
    for p in range(nprob):
        if ndim == 2:
            shape = (int(rng.integers(20, 90)), int(rng.integers(20, 150)))
        else:
            shape = (int(rng.integers(8, 20)), int(rng.integers(8, 20)), int(rng.integers(8, 80)))
        q = wl.small_random(shape, order=8, nt=int(rng.integers(15, 40)), dtype=dtype,
                            seed=100 * seed + p, nsrc=2, nrec=5)
        q.meta["k"] = float(0.02 * (1 + p))
        probs.append(q)
    return probs


@pytest.mark.parametrize("ndim,graph,persistent", [
    (2, False, False), (2, True, False), (3, False, False), (3, True, False),
    (2, False, True), (3, False, True), (3, True, True)])
def test_batched_problems_match_single_calls(fdw, ndim, graph, persistent):
    """Uneven-size problems (different shapes, dt, nt, k, acquisitions) in one launch per
    step, or one persistent launch per sweep: each result equals its own single-problem
    call bitwise and the oracle to rounding (f64)."""
    probs = _uneven_problems(ndim, 6, "f64", seed=ndim)
    f64 = torch.float64
    items, singles, refs = [], [], []
    for q in probs:
        obs = oracle.forward(q.c_ref, 1.0, 8, q.dt, q.nt, q.src, q.wavelet, q.rec)[0]
        c, w, o = to_dev(q.c, f64), to_dev(q.wavelet, f64), to_dev(obs, f64)
        items.append(fdw.Problem(c, 1.0, 8, q.src, w, q.rec, q.dt, q.nt, o, q.meta["k"]))
        singles.append(fdw.fd_adjoint_sensitivity(c, 1.0, 8, q.src, w, q.rec, q.dt, q.nt, o,
                                                  q.meta["k"]))
        refs.append(oracle.superposition_gradient(q.c, 1.0, 8, q.dt, q.nt, q.src, q.wavelet, q.rec,
                                                  obs, q.meta["k"]))
    say("batched", ndim, "graph", graph, "persistent", persistent, [q.shape for q in probs])
    Js = fdw.fd_adjoint_sensitivity_batched(items, graph=graph, persistent=persistent)
    for it, (g1, J1), (g_o, J_o, _) in zip(items, singles, refs):
        assert torch.equal(it.grad, g1) and Js[items.index(it)] == J1
        assert rel(it.grad.cpu().numpy(), g_o) < 1e-9
        assert abs(J1 - J_o) < 1e-12 * J_o


def test_autotune_picks_a_valid_shape_and_persists(fdw, tmp_path, monkeypatch):
    """The tuner returns a variant that fits the grid, writes a JSON line to the cache
    file, and later calls with variant 0 (which take the tuned shape) still agree with
    the oracle."""
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("FDWAVE_TUNE_CACHE", str(cache))
    shape = (40, 24, 132)
    best, ms = fdw.fd_autotune(shape, 1.0, 8, torch.float32, nshot=4, steps=2)
    say("autotune", best, ms)
    info = fdw.fd_variant_info(3, best["variant"])
    assert shape[-1] % info["cells_per_lane"] == 0
    assert best["max_group"] in (1, 2, 4) and best["chunk"] >= 1 and ms > 0
    plain = fdw.fd_variant_info(3, best["variant_plain"])   # the shape of launches without accumulator
    assert shape[-1] % plain["cells_per_lane"] == 0 and plain["max_fields"] >= best["max_group"]
    assert best["chunk_plain"] >= 1
    lines = cache.read_text().strip().splitlines()
    assert lines and '"variant": %d' % best["variant"] in lines[-1]
    assert '"variant_plain": %d' % best["variant_plain"] in lines[-1]
    P = shot_problem(shape, 4, 8, 20, "f32", seed=5)
    g_o, J_o, _ = _oracle_sum(P, 0.05)
    f32 = torch.float32
    g, J = fdw.fd_adjoint_sensitivity(to_dev(P["c"], f32), 1.0, 8, P["src"], to_dev(P["wavelet"], f32),
                                      P["rec"], P["dt"], P["nt"], to_dev(P["obs"], f32), 0.05,
                                      shots=(P["src_shot"], P["rec_shot"], 4))
    assert rel(g.cpu().numpy(), g_o) < 1e-4


def test_persistent_wait_timeout_is_reported(fdw):
    """A wait limit of 1 microsecond (forced from the host) expires: the 10-row last
    chunk of the 310-row problem finishes its first step long before the 300-row chunk
    next to it and then waits for it.  Every block leaves the launch and the call
    returns FD_E_DEVICE instead of waiting."""
    f32 = torch.float32
    items = []
    for i, shape in enumerate([(300, 260), (280, 300), (310, 290)]):
        q = wl.small_random(shape, order=8, nt=6, dtype="f32", seed=40 + i)
        c, w = to_dev(q.c, f32), to_dev(q.wavelet, f32)
        obs = torch.zeros((q.nt, len(q.rec)), dtype=f32, device="cuda")
        items.append(fdw.Problem(c, 1.0, 8, q.src, w, q.rec, q.dt, q.nt, obs, 0.1))
    say("persistent wait timeout")
    with pytest.raises(fdw.FdError) as e:
        fdw.fd_adjoint_sensitivity_batched(items, persistent=True, barrier_timeout_us=1, chunk=300)
    assert e.value.code == fdw.FD_E_DEVICE and "timed out" in str(e.value)
    # the same batch with the default limit completes and matches the per-step launches
    Js = fdw.fd_adjoint_sensitivity_batched(items, persistent=True, chunk=300)
    grads = [it.grad.clone() for it in items]
    Js2 = fdw.fd_adjoint_sensitivity_batched(items, persistent=False, chunk=300)
    assert Js == Js2 and all(torch.equal(g, it.grad) for g, it in zip(grads, items))


def test_persistent_blocks_take_several_tiles(fdw):
    """With 4-row chunks a 2048 x 2048 problem has far more tiles than the grid has
    blocks, so each group holds many chunks and groups wait for neighbours that other
    blocks (on this XCD or another) reach later in the step; the result equals the
    per-step launches bitwise."""
    f32 = torch.float32
    q = wl.small_random((2048, 2048), order=8, nt=8, dtype="f32", seed=77, nsrc=3, nrec=40)
    c, w = to_dev(q.c, f32), to_dev(q.wavelet, f32)
    obs = torch.zeros((q.nt, len(q.rec)), dtype=f32, device="cuda")
    items = [fdw.Problem(c, 1.0, 8, q.src, w, q.rec, q.dt, q.nt, obs, 0.1)]
    say("persistent several tiles per block")
    Js = fdw.fd_adjoint_sensitivity_batched(items, persistent=True, chunk=4)
    g = items[0].grad.clone()
    Js2 = fdw.fd_adjoint_sensitivity_batched(items, persistent=False, chunk=4)
    assert Js == Js2 and torch.equal(g, items[0].grad)
    assert torch.isfinite(g).all()


def test_persistent_blocks_take_several_groups(fdw):
    """3D problems whose whole tile columns (64 x 8 tiles over a 1024 x 1024 cross-
    section: 2048 of them, plus a small second problem) outnumber the blocks of the
    grid, so even the largest groups leave blocks holding two or more per step; the
    result equals the per-step launches bitwise."""
    f32 = torch.float32
    items = []
    for i, shape in enumerate([(24, 1024, 1024), (40, 70, 130)]):
        q = wl.small_random(shape, order=8, nt=5, dtype="f32", seed=90 + i, nsrc=2, nrec=30)
        c, w = to_dev(q.c, f32), to_dev(q.wavelet, f32)
        obs = torch.zeros((q.nt, len(q.rec)), dtype=f32, device="cuda")
        items.append(fdw.Problem(c, 1.0, 8, q.src, w, q.rec, q.dt, q.nt, obs, 0.1))
    say("persistent several groups per block, 3D")
    t = fdw.fd_timing()
    Js = fdw.fd_adjoint_sensitivity_batched(items, persistent=True, chunk=8, variant=1, timing=t)
    grads = [it.grad.clone() for it in items]
    Js2 = fdw.fd_adjoint_sensitivity_batched(items, persistent=False, chunk=8, variant=1)
    assert 0 < t.persistent_blocks < 2048
    assert Js == Js2 and all(torch.equal(g, it.grad) for g, it in zip(grads, items))
    assert all(torch.isfinite(g).all() for g in grads)


def test_batched_rejects_mixed_orders(fdw):
    a = wl.small_random((20, 20), order=8, nt=5, dtype="f32", seed=1)
    b = wl.small_random((20, 20), order=4, nt=5, dtype="f32", seed=2)
    f32 = torch.float32
    items = []
    for q in (a, b):
        c, w = to_dev(q.c, f32), to_dev(q.wavelet, f32)
        obs = torch.zeros((q.nt, len(q.rec)), dtype=f32, device="cuda")
        items.append(fdw.Problem(c, 1.0, q.order, q.src, w, q.rec, q.dt, q.nt, obs, 0.1))
    with pytest.raises(fdw.FdError) as e:
        fdw.fd_adjoint_sensitivity_batched(items)
    assert "same ndim, order and dtype" in str(e.value)


def test_autotune_2d_keeps_one_shape(fdw):
    """In 2D the tuner gives both launch kinds one shape (chosen by their summed time)."""
    best, ms = fdw.fd_autotune((96, 130), 1.0, 8, torch.float32, nshot=1, steps=2)
    assert best["variant_plain"] == best["variant"] and best["chunk_plain"] == best["chunk"]
    assert ms > 0


def _oracle_refs(probs, cs, obs):
    return [oracle.superposition_gradient(c, 1.0, 8, q.dt, q.nt, q.src, q.wavelet, q.rec, o, q.meta["k"])
            for q, c, o in zip(probs, cs, obs)]


def _check_plan_result(items, J, refs):
    Jh = J.cpu().numpy()
    for p, (it, (g_o, J_o, _)) in enumerate(zip(items, refs)):
        assert rel(it.grad.cpu().numpy(), g_o) < 1e-9, p
        assert abs(Jh[p] - J_o) < 1e-12 * J_o, p


@pytest.mark.parametrize("ndim,persistent", [(2, False), (3, False), (2, True), (3, True)])
def test_batch_plan_graph_replay(fdw, ndim, persistent):
    """A batch plan's run captured once in a graph and replayed three times, with every
    problem's speed field changed in place between replays (and eager runs of the same
    plan in between): each replay equals the oracle's Alg. 1 for the speeds it ran with
    (f64: gradient 1e-9, J 1e-12) and the eager run of the same speeds bitwise.  The
    persistent form (one launch per sweep, its item counter and progress words zeroed
    by kernels) replays the same way."""
    probs = _uneven_problems(ndim, 5, "f64", seed=10 + ndim)
    f64 = torch.float64
    items, obs = [], []
    for q in probs:
        o = oracle.forward(q.c_ref, 1.0, 8, q.dt, q.nt, q.src, q.wavelet, q.rec)[0]
        obs.append(o)
        items.append(fdw.Problem(to_dev(q.c, f64), 1.0, 8, q.src, to_dev(q.wavelet, f64), q.rec, q.dt, q.nt,
                                 to_dev(o, f64), q.meta["k"]))
    say("batch plan", ndim, "persistent", persistent, [q.shape for q in probs])
    plan = fdw.BatchPlan(items, persistent=persistent)
    J = torch.zeros(len(items), dtype=f64, device="cuda")
    plan.run(J)
    torch.cuda.synchronize()
    _check_plan_result(items, J, _oracle_refs(probs, [q.c for q in probs], obs))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(J)
    rng = np.random.default_rng(7)
    for rep in range(3):
        # slower media only: the CFL check of the plan's creation keeps holding
        cs = [q.c * (1.0 - 0.05 * rng.random(q.shape)) for q in probs]
        for it, c in zip(items, cs):
            it.c.copy_(torch.as_tensor(c, dtype=f64))
        J.fill_(-1.0)
        say("batch plan replay", rep)
        graph.replay()
        torch.cuda.synchronize()
        grads = [it.grad.clone() for it in items]
        Jr = J.clone()
        _check_plan_result(items, J, _oracle_refs(probs, cs, obs))
        # the eager run of the same plan and speeds gives the replay's result bitwise
        plan.run(J)
        torch.cuda.synchronize()
        assert torch.equal(J, Jr) and all(torch.equal(g, it.grad) for g, it in zip(grads, items))
    del graph
    plan.close()


def test_batch_plan_persistent_and_timing(fdw):
    """The persistent form of a plan (one launch per sweep) gives the per-step
    form's gradients and J bitwise, run after run with c changed in between; a timed plan
    reports both sweeps."""
    probs = _uneven_problems(2, 4, "f64", seed=21)
    f64 = torch.float64
    items = []
    for q in probs:
        o = oracle.forward(q.c_ref, 1.0, 8, q.dt, q.nt, q.src, q.wavelet, q.rec)[0]
        items.append(fdw.Problem(to_dev(q.c, f64), 1.0, 8, q.src, to_dev(q.wavelet, f64), q.rec, q.dt, q.nt,
                                 to_dev(o, f64), q.meta["k"]))
    t = fdw.fd_timing()
    say("batch plan persistent")
    steps = fdw.BatchPlan(items, timing=t)
    pers = fdw.BatchPlan(items, persistent=True)
    J1 = torch.zeros(len(items), dtype=f64, device="cuda")
    J2 = torch.zeros_like(J1)
    for rep in range(2):
        if rep:
            for it in items:
                it.c.mul_(0.98)
        steps.run(J1)
        tm = steps.timing()
        g1 = [it.grad.clone() for it in items]
        pers.run(J2)
        torch.cuda.synchronize()
        assert torch.equal(J1, J2) and all(torch.equal(g, it.grad) for g, it in zip(g1, items))
        assert torch.isfinite(J1).all()
        assert tm.fwd_ms > 0 and tm.bwd_ms > 0
        assert tm.fwd_launches == max(q.nt for q in probs) and tm.bwd_launches == tm.fwd_launches - 1
    steps.close()
    pers.close()
