"""bf16 matrix-core path with certified bounds and plain re-evaluation of
every trial that could be accepted (needs an MI355X).

The mode's decisions are by construction those of the plain evaluation, so
(i) its trajectories follow the CPU oracle like the plain path's, and (ii) at
D=100, where both precisions run the matrix-core kernel, its populations are
bit-identical to the plain mode's.  The refine counter shows how many trials
needed the plain value."""
import numpy as np
import pytest

import workloads as W
from paritylib import state_parity

pytestmark = pytest.mark.gpu


def _batch(wl, precision):
    from paper_2502_10470_amd import Batch, metade
    print(f"[case] {wl.name} runs={wl.n_runs} precision={precision}", flush=True)
    return Batch(wl, precision=precision)


@pytest.mark.parametrize("kinds,N,D,G", [
    (["elliptic", "rastrigin"], 256, 100, 3),
    (["schwefel", "ackley", "rosenbrock", "elliptic"], 64, 37, 4),
    (["rastrigin", "elliptic"], 100, 20, 4),
])
def test_bf16_follows_oracle(kinds, N, D, G):
    from paper_2502_10470_amd import metade as M
    wl = W.small_batch(N + D, kinds, [N] * 4, [D] * 4, n_cs=3)
    b = _batch(wl, M.BF16_REFINE)
    out = state_parity(b, wl, G)
    trials, refined = b.counters()
    print("compared", out["compared"], "diverged", out["diverged"], "refined", refined, "of", trials)
    assert out["compared"] >= 2 * G
    assert 0 < refined <= trials


def test_bf16_hybrid_follows_oracle():
    from paper_2502_10470_amd import metade as M
    p = W.make_problem("hybrid", 20, 2, 0)
    wl = W.small_batch(2, ["hybrid"], [100] * 4, [20] * 4, n_cs=2)
    wl.problems = [p] * 4
    wl.problem = np.zeros(4, np.uint32)
    b = _batch(wl, M.BF16_REFINE)
    out = state_parity(b, wl, 4)
    assert out["compared"] >= 8


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
