"""GPU parity of the particle-swarm evolver (the alternative evolver of the
paper's supplement, S.III) against the oracle: positions and velocities bit
for bit, executor scores to float64 rounding, personal-best updates exact."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import metade as ometa
from oracle import pde
from oracle.fitness import evaluate
from paritylib import OracleRun

pytestmark = pytest.mark.gpu


def _batch(wl):
    from paper_2502_10470_amd import Batch, metade as M
    return Batch(wl, evolver=M.EVOLVER_PSO)


def _oracle_scores(wl, U):
    """Executor scores of theta rows U with the oracle, and per executor
    whether a near-tie on the way allows the library to take another path."""
    ys = np.empty(U.shape[0])
    amb = np.zeros(U.shape[0], bool)
    for i in range(U.shape[0]):
        o = OracleRun(wl, i, theta_row=U[i])
        for _ in range(wl.G):
            s = o.step()
            amb[i] |= bool(s["amb_rank"] or np.any(s["amb_sel"]))
        k = int(pde.ranking(o.fit)[0])
        ys[i] = float(evaluate(o.pop[k], o.prob))
    return ys, amb


def test_pso_outer_steps_c1():
    # the small MetaDE config with short executor runs, so that near-ties
    # inside an executor (which end the comparison) stay rare
    wl = dataclasses.replace(W.workload_c1(), G=5)
    b = _batch(wl)
    b.outer_reset()
    X, y, U, _ = b.get_outer()
    st = ometa.pso_init(8, wl.seed, 0, wl.n_cs)
    assert np.array_equal(X, st["p"]) and np.array_equal(U, st["x"]) and np.all(np.isinf(y))
    compared = 0
    for g_o in range(3):
        b.outer_step(wl.G, 1)
        X2, y2, U2, yt = b.get_outer()
        if g_o > 0:
            st = ometa.pso_move(st, g_o, wl.seed, 0, wl.n_cs)
        assert np.array_equal(U2, st["x"]), f"particle positions differ at g_o={g_o}"
        ys, amb = _oracle_scores(wl, st["x"])
        same = np.abs(yt - ys) <= 1e-12 * np.abs(ys)
        assert np.all(same | amb), f"executor scores differ at g_o={g_o}: {np.flatnonzero(~same)}"
        if not np.all(same):
            break  # an executor took the other side of a near-tie: the swarms may now differ
        st, acc = ometa.pso_select(st, ys)
        assert np.array_equal(X2, st["p"])
        assert np.allclose(y2, st["py"], rtol=1e-12, atol=0)
        compared += 1
    print("outer generations compared:", compared)
    assert compared >= 2


def test_pso_run_and_checkpoint():
    wl = W.workload_c1()
    a = _batch(wl)
    a.outer_reset()
    a.outer_step(wl.G, 1)
    a.outer_step(wl.G, 1)
    blob = a.get_state()
    a.outer_step(wl.G, 1)
    Xa, ya, Ua, _ = a.get_outer()
    b = _batch(wl)
    b.outer_reset()
    b.set_state(blob)
    b.outer_step(wl.G, 1)
    Xb, yb, Ub, _ = b.get_outer()
    assert np.array_equal(Xa, Xb) and np.array_equal(ya, yb) and np.array_equal(Ua, Ub)
    by, bt, bx = a.run(3, wl.G, 2)
    X, y, _, _ = a.get_outer()
    k = int(np.lexsort((np.arange(8), y))[0])
    assert by == y[k] and np.array_equal(bt, X[k])
    lo, hi = pde.theta_bounds(wl.n_cs)
    assert np.all(X >= lo) and np.all(X <= hi)


def test_pso_set_outer_needs_reset_and_outer_step_checks_g():
    # host-side checks only: no generation runs
    from paper_2502_10470_amd import metade as M
    wl = W.workload_c1()
    b = _batch(wl)
    X = np.zeros((wl.n_runs, 6), np.float32)
    y = np.zeros(wl.n_runs, np.float64)
    with pytest.raises(M.MetadeError, match=r"status -4: metade_outer_reset must come first"):
        b.set_outer(X, y, 0)
    b.outer_reset()
    b.set_outer(*b.get_outer()[:2], 0)
    with pytest.raises(M.MetadeError, match=r"status -1: G_inner \* power_up exceeds"):
        b.outer_step(1 << 30, 5)
