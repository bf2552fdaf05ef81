"""Pins of the oracle's outer loop (Alg. 3): first-generation acceptance,
power-up schedule, evolver trial arithmetic, one-shot determinism."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import metade, pde
from oracle import metade as ometa


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


# ---------------------------------------------------------------- PSO evolver (Supplement S.III)

def _pso_state(P=6, seed=3, n_cs=2):
    return ometa.pso_init(P, seed, 0, n_cs)


def test_pso_init_matches_de_population_and_is_at_rest():
    st = _pso_state()
    X, y = ometa.outer_init(6, 3, 0, 2)
    assert np.array_equal(st["x"], X) and np.array_equal(st["p"], X)
    assert np.all(st["v"] == 0) and np.all(np.isinf(st["py"]))


def test_pso_fixed_point_when_bests_coincide():
    """p = g = x and v = 0: every term of the velocity update is zero."""
    st = _pso_state()
    x0 = st["x"][2].copy()
    st["x"][:] = x0
    st["p"][:] = x0
    st["py"] = np.arange(6, dtype=np.float64)
    moved = ometa.pso_move(st, 1, 3, 0, 2)
    assert np.array_equal(moved["x"], st["x"]) and np.all(moved["v"] == 0)


def test_pso_inertia_only():
    """p = g = x: the new velocity is w v exactly (one rounding) and the
    position moves by it (clipped to the box)."""
    st = _pso_state()
    x0 = np.array([0.5, 0.5, 2.5, 2.5, 2.5, 2.0], np.float32)
    st["x"][:] = x0
    st["p"][:] = x0
    st["py"] = np.zeros(6)
    st["v"] = np.full((6, 6), 0.25, np.float32)
    moved = ometa.pso_move(st, 4, 3, 0, 2)
    w = np.float32(0.729)
    assert np.all(moved["v"] == w * np.float32(0.25))
    assert np.all(moved["x"] == x0 + w * np.float32(0.25))


def test_pso_attraction_moves_toward_bests_and_stays_in_box():
    """With v = 0 and p, g on the same side of x, each coordinate moves toward
    them by less than c1 |p - x| + c2 |g - x|; positions never leave the box."""
    lo, hi = pde.theta_bounds(2)
    rng = np.random.default_rng(0)
    for trial in range(20):
        st = _pso_state(P=8, seed=trial)
        st["py"] = rng.permutation(8).astype(np.float64)
        st["p"] = (lo + (hi - lo) * rng.random((8, 6))).astype(np.float32)
        gi = int(np.argmin(st["py"]))
        moved = ometa.pso_move(st, 2 + trial, trial, 0, 2)
        assert np.all(moved["x"] >= lo) and np.all(moved["x"] <= hi)
        d = moved["x"] - st["x"]
        dp, dg = st["p"] - st["x"], st["p"][gi][None, :] - st["x"]
        same = (np.sign(dp) == np.sign(dg)) & (dp != 0)
        assert np.all(np.sign(d[same]) * np.sign(dp[same]) >= 0)
        bound = 1.49 * np.abs(dp) + 1.49 * np.abs(dg) + 1e-6
        assert np.all(np.abs(d) <= bound)


def test_pso_selection_rule():
    st = _pso_state(P=4)
    st, acc = ometa.pso_select(st, np.array([1.0, np.nan, 3.0, 2.0]))
    assert acc.tolist() == [True, False, True, True]       # first scores: every finite one
    st["x"] = st["x"] + np.float32(0.01)
    st2, acc = ometa.pso_select(st, np.array([1.0, 0.5, 3.5, np.nan]))
    assert acc.tolist() == [True, True, False, False]      # <= keeps ties, NaN never
    assert np.array_equal(st2["p"][0], st["x"][0]) and np.array_equal(st2["p"][2], st["p"][2])


def test_pso_converges_on_a_quadratic():
    """Personal-best scores never increase, and the swarm finds the minimum of
    a convex function of theta inside the box."""
    lo, hi = pde.theta_bounds(2)
    c = np.array([0.3, 0.7, 2.2, 3.1, 1.7, 1.9], np.float32)
    f = lambda X: np.sum((X.astype(np.float64) - c) ** 2, axis=1)
    st = ometa.pso_init(16, 5, 0, 2)
    best = np.inf
    for g in range(60):
        if g > 0:
            st = ometa.pso_move(st, g, 5, 0, 2)
        prev = st["py"].copy()
        st, _ = ometa.pso_select(st, f(st["x"]))
        assert np.all(st["py"] <= prev)
        best = min(best, st["py"].min())
    assert best < 1e-3


# ---------------------------------------------------------------- CSO evolver (Supplement S.III)

def test_cso_pairs_partition_the_swarm():
    """Every particle is in exactly one pair (even swarm); an odd swarm leaves
    exactly one particle out; pairings change with the generation."""
    for P in (8, 9, 64):
        pairs, _ = ometa.cso_pairs(P, 3, 7, 0)
        flat = [i for pr in pairs for i in pr]
        assert len(pairs) == P // 2 and len(set(flat)) == len(flat) == 2 * (P // 2)
        assert set(flat) <= set(range(P))
    assert ometa.cso_pairs(16, 1, 7, 0)[0] != ometa.cso_pairs(16, 2, 7, 0)[0]


def test_cso_winners_stay_and_losers_learn_from_them():
    """The better particle of each pair keeps position and velocity; a loser
    at rest moves toward its winner by a fraction in [0, 1) of the distance
    per coordinate (before clipping), and stays in the box."""
    lo, hi = pde.theta_bounds(3)
    rng = np.random.default_rng(1)
    for trial in range(10):
        st = ometa.cso_init(10, trial, 0, 3)
        st["y"] = rng.permutation(10).astype(np.float64)
        moved, wl_pairs = ometa.cso_move(st, 1 + trial, trial, 0, 3)
        for wn, ls in wl_pairs:
            assert st["y"][wn] < st["y"][ls]
            assert np.array_equal(moved["x"][wn], st["x"][wn])
            assert np.array_equal(moved["v"][wn], st["v"][wn])
            d, gap = moved["x"][ls] - st["x"][ls], st["x"][wn] - st["x"][ls]
            assert np.all(np.sign(d) * np.sign(gap) >= 0)
            assert np.all(np.abs(d) <= np.abs(gap))
            # from rest, the step is the velocity (up to the rounding of x + v)
            assert np.allclose(moved["v"][ls], d, rtol=0, atol=4e-7 * np.abs(st["x"][ls]).max())
        assert np.all(moved["x"] >= lo) and np.all(moved["x"] <= hi)


def test_cso_ties_go_to_the_lower_index_and_nan_loses():
    st = ometa.cso_init(6, 2, 0, 2)
    st["y"] = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    _, wl_pairs = ometa.cso_move(st, 1, 2, 0, 2)
    assert all(wn < ls for wn, ls in wl_pairs)
    st["y"] = np.full(6, np.nan)
    st["y"][5] = 0.0
    _, wl_pairs = ometa.cso_move(st, 1, 2, 0, 2)
    assert all(ls != 5 for _, ls in wl_pairs)


def test_cso_coincident_pair_is_a_fixed_point():
    """Winner and loser at the same place, loser at rest: nothing moves."""
    st = ometa.cso_init(4, 2, 0, 2)
    st["x"][:] = st["x"][0]
    st["y"] = np.arange(4, dtype=np.float64)
    moved, _ = ometa.cso_move(st, 5, 2, 0, 2)
    assert np.array_equal(moved["x"], st["x"]) and np.all(moved["v"] == 0)


def test_cso_converges_on_a_quadratic():
    """The swarm's best score never increases and reaches the minimum of a
    convex function of theta inside the box."""
    c = np.array([0.3, 0.7, 2.2, 3.1, 1.7, 1.9], np.float32)
    f = lambda X: np.sum((X.astype(np.float64) - c) ** 2, axis=1)
    st = ometa.cso_init(32, 5, 0, 2)
    best = np.inf
    for g in range(150):
        if g > 0:
            st, _ = ometa.cso_move(st, g, 5, 0, 2)
        st, _ = ometa.cso_select(st, f(st["x"]))
        assert st["y"].min() <= best
        best = st["y"].min()
    assert best < 1e-3


# ---------------------------------------------------------------- NES evolver (Supplement S.III)

def test_nes_utilities_are_zero_sum_and_rank_ordered():
    for lam in (4, 5, 8, 64, 100):
        u = ometa.nes_utilities(lam)
        assert abs(u.sum()) < 1e-12
        assert np.all(np.diff(u) <= 1e-15)
        # only ranks below lambda/2 + 1 get weight above the baseline -1/lambda
        r = np.arange(1, lam + 1)
        assert np.all((u > -1.0 / lam + 1e-15) == (r < lam / 2.0 + 1.0))


def test_nes_normals_are_standard_normal():
    """Moments of 30000 x 6 Box-Muller samples: mean 0, variance 1, no
    correlation between the pair of one word pair, kurtosis 3."""
    s = ometa.nes_normals(30000, 1, 3, 0)
    n = s.shape[0]
    assert np.all(np.abs(s.mean(0)) < 5 / np.sqrt(n))
    assert np.all(np.abs(s.var(0) - 1) < 5 * np.sqrt(2 / n))
    for m in range(3):
        c = np.corrcoef(s[:, 2 * m], s[:, 2 * m + 1])[0, 1]
        assert abs(c) < 5 / np.sqrt(n)
    k = (s ** 4).mean(0) / s.var(0) ** 2
    assert np.all(np.abs(k - 3) < 0.15)


def test_nes_samples_follow_the_distribution_and_stay_in_the_box():
    lo, hi = pde.theta_bounds(3)
    st = {"mu": np.array([0.5, 0.5, 3, 3, 3, 2.5], np.float32),
          "sigma": np.array([0.01, 0.02, 0.1, 0.2, 0.3, 0.05], np.float32)}
    z, s = ometa.nes_samples(st, 20000, 2, 4, 0, 3)
    assert np.all(z >= lo) and np.all(z <= hi)
    assert np.all(np.abs(z.mean(0) - st["mu"]) < 5 * st["sigma"] / np.sqrt(20000))
    assert np.allclose(z.std(0), st["sigma"], rtol=0.05)


def test_nes_moves_downhill_and_shrinks_on_a_quadratic():
    """mu reaches the minimum of a convex function of theta inside the box,
    and sigma contracts around it."""
    c = np.array([0.3, 0.7, 2.2, 3.1, 1.7, 1.9], np.float32)
    f = lambda X: np.sum((X.astype(np.float64) - c) ** 2, axis=1)
    st = ometa.nes_init(2)
    s0 = st["sigma"].copy()
    for g in range(150):
        z, _ = ometa.nes_samples(st, 24, g, 5, 0, 2)
        st = ometa.nes_update(st, f(z), g, 5, 0)
    assert np.max(np.abs(st["mu"] - c)) < 0.02
    assert np.all(st["sigma"] < 0.1 * s0)


def test_nes_update_ignores_sample_order_and_equal_scores_rank_by_index():
    """The update depends on the scores only through their ranks."""
    st = ometa.nes_init(2)
    y = np.array([3.0, 1.0, 2.0, 0.5, 7.0, 4.0])
    a = ometa.nes_update(st, y, 1, 2, 0)
    b = ometa.nes_update(st, np.exp(y), 1, 2, 0)       # same ranks, other values
    assert np.array_equal(a["mu"], b["mu"]) and np.array_equal(a["sigma"], b["sigma"])
    c = ometa.nes_update(st, np.where(np.arange(6) == 4, np.nan, y), 1, 2, 0)
    assert np.array_equal(a["mu"], c["mu"])            # the worst sample stays the worst
