"""Pins of the oracle's outer loop (Alg. 3): first-generation acceptance,
power-up schedule, evolver trial arithmetic, one-shot determinism."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import metade, pde


def _f32_round(q: Fraction) -> np.float32:
    """Nearest float32 to an exact rational (ties to even)."""
    c = np.float32(float(q))  # float(q) is correctly rounded to f64; refine below
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        e = abs(Fraction(float(cand)) - q)
        if best is None or e < best[0] or (e == best[0] and (int(cand.view(np.uint32)) & 1) == 0):
            best = (e, cand)
    return best[1]


def test_outer_trial_arithmetic_exact():
    """Evolver trial v = x_r1 + 0.5 (x_r2 - x_r3): the halving is exact, so v is
    the correctly rounded value of x_r1 + fl(x_r2 - x_r3) / 2."""
    X, y = metade.outer_init(16, 3, 0, 2)
    U, d = metade.outer_trials(X, y, 0, 3, 0, 2, F=0.5, CR=1.0)
    for i in range(16):
        r1, (r2, r3) = d["r0"][i], d["pairs"][i][0]
        for j in range(6):
            diff = np.float32(X[r2, j] - X[r3, j])
            v = _f32_round(Fraction(float(X[r1, j])) + Fraction(float(diff)) / 2)
            lo, hi = pde.theta_bounds(2)
            v = min(max(v, lo[j]), hi[j])
            assert U[i, j] == v


def test_outer_init_in_box():
    X, y = metade.outer_init(64, 2, 0, 2)
    lo, hi = pde.theta_bounds(2)
    assert np.all(X >= lo) and np.all(X < hi) and np.all(np.isinf(y))


def test_first_generation_accepts_all_and_power_up():
    wl = W.workload_c1()
    calls = []

    def fake_executor(i, th, G):
        calls.append(G)
        return {"y": float(1000 + i), "best_x": np.zeros(10, np.float32)}

    log = []
    res = metade.run_metade(wl, gens=3, executor=fake_executor, log=log)
    assert log[0]["accept"].all()
    assert calls == [50] * 8 + [50] * 8 + [250] * 8
    # later generations: equal scores are accepted (<=), so all accepted again
    assert log[1]["accept"].all() and log[2]["accept"].all()
    assert res["best_index"] == 0 and res["best_y"] == 1000.0


def test_outer_selection_rule():
    X = np.zeros((4, 6), np.float32)
    U = np.ones((4, 6), np.float32)
    y = np.array([1.0, 2.0, np.inf, np.nan])
    yt = np.array([1.0, 3.0, 5.0, 2.0])
    X2, y2, acc = metade.outer_select(X, y, U, yt)
    assert list(acc) == [True, False, True, True]
    _, _, acc = metade.outer_select(X, y, U, np.array([np.nan] * 4))
    assert not acc.any()


def test_c1_metade_deterministic_and_consistent():
    wl = W.workload_c1()
    a = metade.run_metade(wl, gens=2, power_up=1)
    b = metade.run_metade(wl, gens=2, power_up=1)
    assert a["best_y"] == b["best_y"] and np.array_equal(a["X"], b["X"])
    # the reported best equals one executor run at the best theta (one-shot)
    th = pde.decode(a["best_theta"], 2)
    r = pde.run_executor(32, 10, th, 50, wl.seed, 0, -100, 100, wl.problems[0])
    assert r["y"] == a["best_y"]
    assert a["best_y"] >= 100.0
