"""bf16 matrix-core path with certified bounds and plain re-evaluation of
every trial that could be accepted (needs an MI355X).

The mode's decisions are by construction those of the plain evaluation, so
(i) its trajectories follow the CPU oracle like the plain path's, and (ii) at
D=100, where both precisions run the matrix-core kernel, its populations are
bit-identical to the plain mode's.  Traced generations re-evaluate every trial
and check each bf16 value against its bound: no value may lie outside its
bound and no trial the screen alone rejects may be one the plain value
accepts."""
import numpy as np
import pytest

import workloads as W
from paritylib import resync_parity, trajectory_parity

pytestmark = pytest.mark.gpu


def _batch(wl, precision):
    from paper_2502_10470_amd import Batch
    print(f"[case] {wl.name} runs={wl.n_runs} precision={precision}", flush=True)
    return Batch(wl, precision=precision)


def _bound_ok(b, min_checked):
    checked, outside, screened, wrong, ratio = b.bound_check()
    print(f"bound check: {checked} trials, {outside} outside, {screened} screened out "
          f"({screened / max(checked, 1):.3f}), {wrong} wrong, max |dev|/bound {ratio:.3g}",
          flush=True)
    assert checked >= min_checked
    assert outside == 0 and wrong == 0
    return checked, screened, ratio


@pytest.mark.parametrize("kinds,N,D,G", [
    (["elliptic", "rastrigin"], 256, 100, 3),
    (["schwefel", "ackley", "rosenbrock", "elliptic"], 64, 37, 4),
    (["rastrigin", "elliptic"], 100, 20, 4),
])
def test_bf16_follows_oracle(kinds, N, D, G):
    from paper_2502_10470_amd import metade as M
    wl = W.small_batch(N + D, kinds, [N] * 4, [D] * 4, n_cs=3)
    b = _batch(wl, M.BF16_REFINE)
    out = trajectory_parity(b, wl, G)
    print("compared", out["compared"], "near ties", out["near_ties"], "max rel", out["max_fit_rel"])
    assert out["compared"] == 4 * G
    _bound_ok(b, 4 * N * G)


def test_bf16_hybrid_follows_oracle():
    from paper_2502_10470_amd import metade as M
    p = W.make_problem("hybrid", 20, 2, 0)
    wl = W.small_batch(2, ["hybrid"], [100] * 4, [20] * 4, n_cs=2)
    wl.problems = [p] * 4
    wl.problem = np.zeros(4, np.uint32)
    b = _batch(wl, M.BF16_REFINE)
    out = trajectory_parity(b, wl, 4)
    assert out["compared"] == 16
    _bound_ok(b, 1600)


def test_bf16_identical_to_plain_at_d100():
    """C4 shape (reduced run count): both precisions use the matrix-core
    kernel; 60 generations must give bit-identical populations."""
    from paper_2502_10470_amd import metade as M
    wl = W.workload_c4(runs=16, G=60)
    a = _batch(wl, M.FP32)
    b = _batch(wl, M.BF16_REFINE)
    for _ in range(3):
        a.inner_step(20)
        b.inner_step(20)
        pa, fa = a.host_state()
        pb, fb = b.host_state()
        assert np.array_equal(pa, pb) and np.array_equal(fa, fb)
    assert np.array_equal(a.get_best(), b.get_best())
    trials, refined = b.counters()
    print(f"refined {refined} of {trials} trials ({refined / trials:.3f})")
    assert refined < trials


def test_bf16_bound_holds_over_a_c4_run():
    """Every trial of a C4-shaped run (16 runs x N = 256 at D = 100, elliptic
    and Rastrigin, 500 generations) checked: its bf16 fitness lies within its
    bound of the plain value, and the screen never rejects a trial the plain
    value accepts."""
    from paper_2502_10470_amd import metade as M
    wl = W.workload_c4(runs=16, G=500)
    b = _batch(wl, M.BF16_REFINE)
    for g in range(wl.G):
        b.trace_step()
        if g % 100 == 99:
            print(f"generation {g + 1}", flush=True)
    checked, screened, _ = _bound_ok(b, 16 * 256 * 500)
    assert checked == 16 * 256 * 500


def test_bf16_late_generation_resync():
    """Deep inside a full-length launch (499 generations of the C4 shape in the
    untraced, screened mode), one traced generation from the library's own
    state against the oracle: trials, draws and every decision."""
    from paper_2502_10470_amd import metade as M
    wl = W.workload_c4(runs=32, G=500)
    b = _batch(wl, M.BF16_REFINE)
    b.inner_step(499)
    out = resync_parity(b, wl, 499, wl.theta)
    print({k: v for k, v in out.items()}, flush=True)
    assert out["compared"] == 32
    _bound_ok(b, 32 * 256)


def test_checkpoint_across_precisions():
    """A checkpoint carries only populations, fitness, theta and counters; the
    run layout (kernel choice, trial-row area) is the receiving context's.  A
    plain-mode blob (D = 20 runs on the lane kernel, D = 100 on the matrix
    cores) restored into a bf16 context (every run on the matrix cores, each
    with its own trial rows) continues exactly: the D = 100 runs stay
    bit-identical to the plain context's (both evaluate them on the same
    float64 tiles), the D = 20 runs follow the oracle from the restored state."""
    from paper_2502_10470_amd import metade as M
    wl = W.small_batch(77, ["rastrigin", "elliptic", "elliptic", "rastrigin"], [100, 120, 256, 200],
                       [20, 20, 100, 100], n_cs=3)
    a = _batch(wl, M.FP32)
    b = _batch(wl, M.BF16_REFINE)
    a.inner_step(6)
    b.set_state(a.get_state())
    pa, fa = a.host_state()
    pb, fb = b.host_state()
    assert np.array_equal(pa, pb) and np.array_equal(fa, fb)
    a.inner_step(5)
    b.inner_step(4)
    out = resync_parity(b, wl, 10, wl.theta, runs=[0, 1])
    assert out["compared"] == 2
    pa, fa = a.host_state()
    pb, fb = b.host_state()
    for r in (2, 3):
        assert np.array_equal(a.run_pop(pa, r), b.run_pop(pb, r)), f"run {r}"
        assert np.array_equal(a.run_fit(fa, r), b.run_fit(fb, r)), f"run {r}"
    # and back: the bf16 context's state into a fresh plain context
    c = _batch(wl, M.FP32)
    c.set_state(b.get_state())
    b.inner_step(3)
    c.inner_step(3)
    pb, fb = b.host_state()
    pc, fc = c.host_state()
    for r in (2, 3):
        assert np.array_equal(b.run_pop(pb, r), c.run_pop(pc, r)), f"run {r}"
