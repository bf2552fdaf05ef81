"""Tuning of the generation kernels' launch shapes (needs an MI355X): the
autotuner leaves the context's state unchanged, persists and reuses its
choice, the matrix-core kernel's row-tile count does not change results, and
tuned contexts follow the oracle like any other."""
import numpy as np
import pytest

import workloads as W
from paritylib import trajectory_parity

pytestmark = pytest.mark.gpu


def _batch(wl, **kw):
    from paper_2502_10470_amd import Batch
    print(f"[case] {wl.name} runs={wl.n_runs}", flush=True)
    return Batch(wl, **kw)


def _mixed():
    # lane-kernel runs (D <= 20) and matrix-core runs (D = 100, N = 256)
    return W.small_batch(17, ["rastrigin", "elliptic", "hybrid", "ackley", "elliptic", "rastrigin"],
                         [100, 64, 100, 40, 256, 200], [20, 10, 20, 13, 100, 100], n_cs=3)


def test_autotune_keeps_state_and_persists(tmp_path):
    wl = _mixed()
    b = _batch(wl)
    b.inner_step(3)
    p0, f0 = b.host_state()
    y0 = b.get_best()
    cache = str(tmp_path / "tuning.txt")
    chosen, ms = b.autotune(20, cache)
    print("chosen", chosen, "ms", ms, flush=True)
    assert chosen["mfma_rows"] in (2, 4) and chosen["lane_parts"] in (0, 1, 2, 4)
    assert ms > 0 and b.tuning() == chosen
    p1, f1 = b.host_state()
    assert np.array_equal(p0, p1) and np.array_equal(f0, f1)
    assert np.array_equal(y0, b.get_best())
    lines = open(cache).read().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    # a second context of the same shapes takes the recorded choice
    b2 = _batch(wl)
    chosen2, ms2 = b2.autotune(20, cache)
    assert chosen2 == chosen and ms2 == pytest.approx(ms, rel=1e-5)
    assert len([l for l in open(cache).read().split("\n") if l.strip()]) == 1
    # tuned contexts still follow the oracle on every trial and decision
    b3 = _batch(wl)
    b3.autotune(20, cache)
    out = trajectory_parity(b3, wl, 3)
    assert out["compared"] == wl.n_runs * 3


def test_rotation_rows_do_not_change_results():
    wl = W.workload_c4(runs=8, G=30)
    a, b = _batch(wl), _batch(wl)
    a.set_tuning(mfma_rows=4)
    b.set_tuning(mfma_rows=2)
    a.inner_step(30)
    b.inner_step(30)
    pa, fa = a.host_state()
    pb, fb = b.host_state()
    assert np.array_equal(pa, pb) and np.array_equal(fa, fb)


@pytest.mark.parametrize("parts", [1, 2, 4, 8])
def test_lane_parts_follow_oracle(parts):
    wl = W.small_batch(23 + parts, ["rastrigin", "schwefel", "rosenbrock", "elliptic"],
                       [30, 64, 100, 130], [7, 20, 16, 33], n_cs=3)
    b = _batch(wl)
    b.set_tuning(lane_parts=parts)
    out = trajectory_parity(b, wl, 3)
    assert out["compared"] == 12


def test_tuning_values_are_checked():
    from paper_2502_10470_amd import metade as M
    b = _batch(_mixed())
    with pytest.raises(M.MetadeError, match="mfma_rows"):
        b.set_tuning(mfma_rows=3)
    with pytest.raises(M.MetadeError, match="lane_parts"):
        b.set_tuning(lane_parts=5)
