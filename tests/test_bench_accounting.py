"""The bench's byte accounting (host logic, no GPU): the launch schedule of a gradient
(which step launches carry kernel terms and what each does with the f32 partial sums),
the algorithmic bytes per cell update derived from it, and the traffic lookup in the
committed rocprofv3 counter record of the default workload."""
import os
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("nt", [2, 3, 17, 60, 3000, 3001])
def test_launch_kinds_cover_the_gradient(nt):
    kinds = bench.gradient_launch_kinds(nt, True)
    assert sum(kinds.values()) == 2 * nt - 1
    # every other launch of each sweep carries kernel terms (the last odd one its own)
    acc = sum(v for k, v in kinds.items() if k is not None)
    assert acc == 2 * ((nt - 1 + 1) // 2)


def test_default_schedule_bytes():
    """nt 3000: 2999 launches without kernel terms (16 B per cell), 188 that start the
    partial sums (20 B), 2624 that add to them (24 B), 188 that fold them into the f64
    accumulator (36 B): 20.25 B per cell update."""
    kinds = bench.gradient_launch_kinds(3000, True)
    assert kinds == {None: 2999, "start": 188, "add": 2624, "flush": 188}
    per_update = bench.gradient_bytes(3000, 1, "f64") / 5999
    assert per_update == pytest.approx((2999 * 16 + 188 * 20 + 2624 * 24 + 188 * 36) / 5999)
    assert per_update == pytest.approx(20.25, abs=0.01)
    # without partial sums every accumulating launch reads and writes the f64 accumulator
    assert bench.gradient_bytes(3000, 1, "f64", partials=False) / 5999 == pytest.approx(24.0, abs=0.01)


def test_pairs_schedule():
    """Two steps per launch: (nt // 2) + ((nt - 1) // 2) two-step launches plus the odd
    steps, fewer bytes per update than one step per launch."""
    for nt in (20, 21, 3000):
        nbytes, launches = bench.pair_gradient_bytes(nt, "f64", True)
        assert launches == (nt + 1) // 2 + nt // 2
        assert nbytes / (2 * nt - 1) < bench.gradient_bytes(nt, 1, "f64") / (2 * nt - 1)


def _args(**kw):
    a = dict(workload="layered3d", n=0, acc="f64", method="superposition", pairs=0)
    a.update(kw)
    return types.SimpleNamespace(**a)


def test_traffic_lookup_matches_the_record():
    """The committed record belongs to the current kernel sources (its sha256 matches),
    and the lookup averages its per-kind figures over the gradient's launches; shapes or
    workloads the record lacks give None."""
    rec = open(os.path.join(ROOT, "profiles", "step_kernel_layered3d_1024_traffic.md")).read()
    assert "source_sha256: " + bench.step_kernel_sha() in rec
    shape = {"variant": 7, "chunk": 64, "variant_plain": 4, "chunk_plain": 1024}
    t = bench.measured_traffic(_args(), shape, 3000)
    assert t is not None and 1.0 < t / (bench.gradient_bytes(3000, 1, "f64") / 5999 * 1024 ** 3) < 1.3
    assert bench.measured_traffic(_args(), dict(shape, variant=2), 3000) is None
    assert bench.measured_traffic(_args(workload="vd3d"), shape, 3000) is None
    assert bench.measured_traffic(_args(pairs=1), shape, 3000) is None
