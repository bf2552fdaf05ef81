"""The no-allocation entry point (metade_inner_step_static) against the
ordinary one, through the C ABI (needs an MI355X): same workload, same
results, bit for bit, on two calls in a row, the second with a smaller
workload (the shared static workspace then still holds the first call's
larger contents)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _pair(wl, precision):
    from paper_2502_10470_amd import Batch
    print(f"[case] {wl.name} runs={wl.n_runs} precision={precision}", flush=True)
    return Batch(wl, precision=precision), Batch(wl, precision=precision)


def _same(a, b):
    pa, fa = a.host_state()
    pb, fb = b.host_state()
    assert np.array_equal(pa, pb)
    assert np.array_equal(fa, fb)
    assert np.array_equal(a.get_best(), b.get_best())
    assert np.array_equal(a.best_x.cpu().numpy(), b.best_x.cpu().numpy())


@pytest.mark.parametrize("precision", [0, 1])
def test_static_entry_matches_inner_step(precision):
    # first call: the D = 100 shape on the matrix-core kernel (32 runs x N = 256)
    wl1 = W.workload_c4(runs=32, G=40)
    a1, b1 = _pair(wl1, precision)
    a1.inner_step(40)
    b1.inner_step_static(40)
    _same(a1, b1)
    # second call, smaller: fewer runs, smaller N and D, a mix of kernels
    wl2 = W.small_batch(93, ["elliptic", "rastrigin", "rosenbrock", "ackley"], [200, 64, 130, 40],
                        [90, 37, 100, 20], n_cs=3)
    a2, b2 = _pair(wl2, precision)
    a2.inner_step(25)
    b2.inner_step_static(25)
    _same(a2, b2)
    # and the first context again, after the smaller one used the workspace
    a1.inner_step(10)
    b1.inner_step_static(10)
    _same(a1, b1)


def test_static_entry_rejects_control_runs():
    from paper_2502_10470_amd import Batch, metade as M
    wl = W.control_batch(5, [16, 20], steps=10)
    b = Batch(wl)
    with pytest.raises(M.MetadeError, match="control"):
        b.inner_step_static(1)
