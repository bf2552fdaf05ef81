"""Pins of the oracle's executor (Parameterized DE, Alg. 2) against the paper's
equations, closed forms, exhaustive enumeration and distribution laws."""
import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chisquare

import workloads as W
from oracle import pde, philox
from oracle.fitness import evaluate


def _th(F, CR, bl, br, dn, cs):
    return {"F": np.float32(F), "CR": np.float32(CR), "bl": bl, "br": br, "dn": dn, "cs": cs}


# ---------------------------------------------------------------- sampler

@pytest.mark.parametrize("N,m", [(5, 1), (5, 3), (5, 4), (6, 5), (7, 3)])
def test_sampler_is_bijection_onto_distinct_tuples(N, m):
    """Every draw vector t (t_k < N-1-k) maps to an ordered tuple of distinct
    indices != i, and the map is one-to-one and onto all such tuples."""
    ranges = [range(N - 1 - k) for k in range(m)]
    all_t = np.array(list(itertools.product(*ranges)), dtype=np.int64)
    for i in range(N):
        # sample_distinct treats row index as the target, so put target i in row i
        seen = set()
        for t in all_t:
            rows = np.zeros((N, m), np.int64)
            rows[i] = t
            tup = tuple(int(x) for x in pde.sample_distinct(rows, N)[i])
            assert len(set(tup)) == m and i not in tup and all(0 <= x < N for x in tup)
            seen.add(tup)
        expect = {p for p in itertools.permutations([j for j in range(N) if j != i], m)}
        assert seen == expect


def test_sampler_first_draw_uniform():
    N = 12
    w = philox.words(9, np.arange(N), 3, 1, 1)
    counts = np.zeros(N, int)
    for g in range(600):
        w = philox.words(9, np.arange(N), g, 1, 1)
        t = philox.lemire(w[:, :1], N - 1)
        d = pde.sample_distinct(t, N)[:, 0]
        assert np.all(d != np.arange(N))
        counts += np.bincount(d, minlength=N)
    assert chisquare(counts).pvalue > 1e-4


# ---------------------------------------------------------------- ranking

def test_ranking_ties_and_nan():
    f = np.array([3.0, np.nan, 1.0, 3.0, np.inf, 1.0, -2.0], dtype=np.float32)
    ref = sorted(range(len(f)), key=lambda i: (float("inf") if np.isnan(f[i]) else float(f[i]), i))
    assert list(pde.ranking(f)) == ref
    assert list(pde.ranking(f))[:3] == [6, 2, 5]


def test_top_count():
    assert [pde.top_count(n) for n in (1, 9, 10, 11, 20, 32, 100, 101, 256)] == \
        [1, 1, 1, 2, 2, 4, 10, 11, 26]


# ---------------------------------------------------------------- decode

def test_decode_grid():
    """Alg. 3 decode: floor of the categorical parts, the box end mapped to the
    last category, out-of-box values clipped first."""
    for n_cs in (2, 3):
        for u in np.linspace(0.0, 6.0, 241):
            th = np.array([u / 5, u / 5, u, u, u, u], np.float32)
            d = pde.decode(th, n_cs)
            c = min(max(u, 1.0), 5.0)
            assert d["bl"] == d["br"] == d["dn"] == min(int(np.floor(np.float32(c))), 4)
            assert d["cs"] == min(int(np.floor(np.float32(min(max(u, 1.0), 1.0 + n_cs)))), n_cs)
            assert d["F"] == np.float32(min(max(u / 5, 0.0), 1.0))
    d = pde.decode(np.array([np.nan, 0.5, 1, 1, 1, 1], np.float32), 2)
    assert d["bl"] == 1 and d["cs"] == 1


# ---------------------------------------------------------------- mutation (Table I)

def _pop(N, D, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-100, 100, (N, D)).astype(np.float32), rng.uniform(0, 10, N)


TABLE_I = [
    # name, bl, br, dn, textbook mutant from (x, i, draws r, best, pbest, F)
    ("rand/1", 1, 1, 1, lambda x, i, r, b, p, F: x[r[0]] + F * (x[r[1]] - x[r[2]])),
    ("best/1", 2, 2, 1, lambda x, i, r, b, p, F: x[b] + F * (x[r[0]] - x[r[1]])),
    ("current-to-best/1", 4, 2, 1,
     lambda x, i, r, b, p, F: x[i] + F * (x[b] - x[i]) + F * (x[r[0]] - x[r[1]])),
    ("rand/2", 1, 1, 2,
     lambda x, i, r, b, p, F: x[r[0]] + F * (x[r[1]] - x[r[2]]) + F * (x[r[3]] - x[r[4]])),
    ("best/2", 2, 2, 2,
     lambda x, i, r, b, p, F: x[b] + F * (x[r[0]] - x[r[1]]) + F * (x[r[2]] - x[r[3]])),
    ("current-to-pbest/1", 4, 3, 1,
     lambda x, i, r, b, p, F: x[i] + F * (x[p] - x[i]) + F * (x[r[0]] - x[r[1]])),
]


@pytest.mark.parametrize("name,bl,br,dn,formula", TABLE_I, ids=[t[0] for t in TABLE_I])
def test_table_i_mutations(name, bl, br, dn, formula):
    """Each Table I row of (bl, br, dn) with CR = 1 (u = v) reproduces the
    textbook mutation Eqs. (1)-(6), evaluated in float64 from the same indices,
    to within float32 rounding."""
    N, D = 40, 7
    x, f = _pop(N, D, 1)
    F = np.float32(0.7)
    u, desc = pde.make_trials(x, f, _th(F, 1.0, bl, br, dn, pde.BIN), 5, 3, 2, -1e9, 1e9)
    x64 = x.astype(np.float64)
    order = np.lexsort((np.arange(N), f))
    for i in range(N):
        r = []
        if desc["r0"][i] >= 0:
            r.append(desc["r0"][i])
        r += list(desc["pairs"][i].ravel())
        p = order[desc["pbest_rank"][i]]
        assert desc["pbest_rank"][i] < pde.top_count(N)
        ref = formula(x64, i, r, order[0], p, float(F))
        assert np.allclose(u[i], ref, rtol=0, atol=4 * 2.0**-23 * 400)
        assert len(set(r)) == len(r) and i not in r


def test_eq11_rand1_arith_equals_current_to_rand():
    """Eq. (11): DE/rand/1 with arithmetic recombination equals
    x_i + K (x_r1 - x_i) + K F (x_r2 - x_r3) (Eq. (7))."""
    N, D = 30, 6
    x, f = _pop(N, D, 2)
    F = np.float32(0.45)
    u, desc = pde.make_trials(x, f, _th(F, 0.3, 1, 1, 1, pde.ARITH), 2, 4, 0, -1e9, 1e9)
    x64 = x.astype(np.float64)
    for i in range(N):
        K = float(desc["K"][i])
        assert 0.0 < K <= 1.0
        r1, (r2, r3) = desc["r0"][i], desc["pairs"][i][0]
        ref = x64[i] + K * (x64[r1] - x64[i]) + K * float(F) * (x64[r2] - x64[r3])
        assert np.allclose(u[i], ref, rtol=0, atol=8 * 2.0**-23 * 400)


def test_F_zero_gives_base_vector_exactly():
    N, D = 25, 5
    x, f = _pop(N, D, 3)
    for bl, br in [(1, 1), (2, 2), (3, 3), (4, 4), (4, 2), (1, 3), (2, 4)]:
        u, desc = pde.make_trials(x, f, _th(0.0, 1.0, bl, br, 3, pde.BIN), 0, 1, 0, -1e9, 1e9)
        assert np.array_equal(u, x[desc["i_bl"]])


def test_bl_equals_br_has_no_directional_term():
    """With bl == br the mutant is x_bl + F * sum of differences (Sec. III-A2)."""
    N, D = 25, 5
    x, f = _pop(N, D, 4)
    F = np.float32(0.8)
    for code in (1, 2, 3, 4):
        u, d = pde.make_trials(x, f, _th(F, 1.0, code, code, 2, pde.BIN), 1, 2, 0, -1e9, 1e9)
        p = d["pairs"]
        dd = (x[p[:, 0, 0]] - x[p[:, 0, 1]]) + (x[p[:, 1, 0]] - x[p[:, 1, 1]])
        assert np.array_equal(u, x[d["i_bl"]] + F * dd)


def test_mutation_is_linear_in_F_direction():
    """v(F) - x_bl is (numerically) F times the total direction."""
    N, D = 30, 4
    x, f = _pop(N, D, 5)
    th1 = _th(1.0, 1.0, 4, 2, 2, pde.BIN)
    u1, d = pde.make_trials(x, f, th1, 7, 0, 0, -1e9, 1e9)
    u5, _ = pde.make_trials(x, f, _th(0.5, 1.0, 4, 2, 2, pde.BIN), 7, 0, 0, -1e9, 1e9)
    base = x[d["i_bl"]].astype(np.float64)
    assert np.allclose((u5 - base), 0.5 * (u1 - base), atol=1e-3)


# ---------------------------------------------------------------- crossover

def test_binomial_extremes_and_law():
    N, D = 60, 9
    x, f = _pop(N, D, 6)
    th = _th(0.5, 1.0, 1, 1, 1, pde.BIN)
    _, d = pde.make_trials(x, f, th, 0, 0, 0, -1e9, 1e9)
    assert d["mask"].all()
    _, d = pde.make_trials(x, f, _th(0.5, 0.0, 1, 1, 1, pde.BIN), 0, 0, 0, -1e9, 1e9)
    assert np.array_equal(d["mask"], np.arange(D)[None, :] == d["jn"][:, None])
    # count of mutant genes = 1 + Binomial(D - 1, CR)
    CR = 0.35
    counts = np.zeros(D + 1)
    for g in range(150):
        _, d = pde.make_trials(x, f, _th(0.5, CR, 1, 1, 1, pde.BIN), g, 0, 0, -1e9, 1e9)
        counts += np.bincount(d["mask"].sum(1), minlength=D + 1)
    from scipy.stats import binom
    expect = np.array([0] + [binom.pmf(k - 1, D - 1, CR) for k in range(1, D + 1)]) * counts.sum()
    keep = expect > 5
    obs, exp_ = counts[keep], expect[keep]
    assert chisquare(obs, exp_ * obs.sum() / exp_.sum()).pvalue > 1e-4


def test_exponential_extremes_and_censored_geometric_law():
    N, D = 60, 8
    x, f = _pop(N, D, 7)
    _, d = pde.make_trials(x, f, _th(0.5, 0.0, 1, 1, 1, pde.EXP), 0, 0, 0, -1e9, 1e9)
    assert np.all(d["L"] == 1) and np.array_equal(d["mask"], np.arange(D)[None, :] == d["jn"][:, None])
    _, d = pde.make_trials(x, f, _th(0.5, 1.0, 1, 1, 1, pde.EXP), 0, 0, 0, -1e9, 1e9)
    assert np.all(d["L"] == D) and d["mask"].all()
    CR = 0.7
    counts = np.zeros(D + 1)
    for g in range(200):
        _, d = pde.make_trials(x, f, _th(0.5, CR, 1, 1, 1, pde.EXP), g, 0, 0, -1e9, 1e9)
        counts += np.bincount(d["L"], minlength=D + 1)
        # the mask is one contiguous (cyclic) run starting at n
        for i in range(N):
            run = [(d["jn"][i] + k) % D for k in range(d["L"][i])]
            assert set(np.flatnonzero(d["mask"][i])) == set(run)
    pmf = np.array([0] + [CR ** (k - 1) * (1 - CR) for k in range(1, D)] + [CR ** (D - 1)])
    assert abs(pmf.sum() - 1) < 1e-12
    assert chisquare(counts[1:], pmf[1:] * counts.sum()).pvalue > 1e-4


def test_clip_to_box():
    N, D = 30, 6
    x, f = _pop(N, D, 8)
    u, _ = pde.make_trials(x, f, _th(1.0, 1.0, 1, 1, 4, pde.BIN), 0, 0, 0, -100, 100)
    assert u.min() >= -100 and u.max() <= 100
    assert np.any(u == 100) or np.any(u == -100)


# ---------------------------------------------------------------- init

def test_init_single_rounding():
    """x = lb + (ub - lb) u0 rounded once: compare with exact rational rounding."""
    for lb, ub, D in [(-100.0, 100.0, 6), (-1.0, 1.0, 5), (0.1, 0.7, 3)]:
        x = pde.init_population(8, D, 5, 3, lb, ub)
        w = philox.words(5, np.arange(8), philox.INIT_PHASE, 3, D)
        lbq, ubq = Fraction(float(np.float32(lb))), Fraction(float(np.float32(ub)))
        for i in range(8):
            for j in range(D):
                exact = lbq + (ubq - lbq) * Fraction(int(w[i, j]) >> 8, 1 << 24)
                cand = np.float32(x[i, j])
                err = abs(Fraction(float(cand)) - exact)
                up = abs(Fraction(float(np.nextafter(cand, np.float32(np.inf)))) - exact)
                dn = abs(Fraction(float(np.nextafter(cand, np.float32(-np.inf)))) - exact)
                assert err <= up and err <= dn
        assert x.min() >= np.float32(lb) and x.max() <= np.float32(ub)


# ---------------------------------------------------------------- loop invariants

@pytest.mark.parametrize("kind", ["rastrigin", "elliptic", "rosenbrock", "ackley"])
def test_run_invariants(kind):
    prob = W.make_problem(kind, 6, 0, 0)
    th = pde.decode(np.array([0.6, 0.8, 3.5, 2.5, 1.5, 1.2], np.float32), 2)
    N, G = 20, 15
    pop = pde.init_population(N, 6, 0, 0, -100, 100)
    fit = evaluate(pop, prob)
    best = [fit.min()]
    for g in range(G):
        s = pde.step(pop, fit, th, g, 0, 0, -100, 100, prob, decide="f64")
        assert np.all(s["fit"] <= fit)
        acc = s["accept"]
        assert np.array_equal(s["pop"][acc], s["u"][acc]) and np.array_equal(s["pop"][~acc], pop[~acc])
        pop, fit = s["pop"], s["fit"]
        best.append(fit.min())
    assert np.all(np.diff(best) <= 0)
    r = pde.run_executor(N, 6, th, G, 0, 0, -100, 100, prob, decide="f64")
    assert r["y"] == pytest.approx(r["best_seen"], rel=0, abs=0)
    assert r["y"] == pytest.approx(float(fit.min()), rel=0, abs=0)


def test_stationary_population():
    """F = 0 with bl = br = current gives u = x_i, so the population never moves."""
    prob = W.make_problem("rastrigin", 5, 1, 0)
    th = {"F": np.float32(0.0), "CR": np.float32(0.5), "bl": 4, "br": 4, "dn": 2, "cs": 1}
    pop0 = pde.init_population(15, 5, 1, 0, -100, 100)
    r = pde.run_executor(15, 5, th, 6, 1, 0, -100, 100, prob)
    assert np.array_equal(r["pop"], pop0)


def test_one_shot_determinism():
    """The same theta and stream give identical runs; another stream differs."""
    prob = W.make_problem("ackley", 4, 2, 0)
    th = pde.decode(np.array([0.4, 0.6, 1.5, 3.5, 2.2, 2.5], np.float32), 2)
    a = pde.run_executor(16, 4, th, 5, 7, 0, -100, 100, prob)
    b = pde.run_executor(16, 4, th, 5, 7, 0, -100, 100, prob)
    c = pde.run_executor(16, 4, th, 5, 7, 1, -100, 100, prob)
    assert np.array_equal(a["pop"], b["pop"]) and a["y"] == b["y"]
    assert not np.array_equal(a["pop"], c["pop"])


def test_population_too_small_rejected():
    x, f = _pop(8, 3, 0)
    with pytest.raises(ValueError):
        pde.make_trials(x, f, _th(0.5, 0.5, 1, 2, 4, 1), 0, 0, 0, -100, 100)


def test_tiny_population_brute_force():
    """N=10, D=2, 3 generations: recompute every trial of every generation from
    its descriptor with scalar float32 arithmetic and the textbook rules."""
    prob = W.make_problem("rastrigin", 2, 3, 0)
    for vec in ([0.9, 0.3, 1.0, 1.0, 1.0, 1.0], [0.5, 0.7, 4.0, 3.0, 2.0, 2.0],
                [0.2, 0.1, 2.0, 4.0, 4.0, 1.0], [0.7, 0.9, 3.0, 1.0, 1.0, 2.9]):
        th = pde.decode(np.array(vec, np.float32), 3)
        pop = pde.init_population(10, 2, 3, 0, -100, 100)
        fit = evaluate(pop, prob).astype(np.float32)
        for g in range(3):
            s = pde.step(pop, fit, th, g, 3, 0, -100, 100, prob)
            d = s["desc"]
            F = np.float32(th["F"])
            for i in range(10):
                xb = pop[d["i_bl"][i]]
                base = xb if th["bl"] == th["br"] else xb + F * (pop[d["i_br"][i]] - xb)
                diff = np.zeros(2, np.float32)
                for k, (a, b) in enumerate(d["pairs"][i]):
                    diff = (pop[a] - pop[b]) if k == 0 else diff + (pop[a] - pop[b])
                v = base + F * diff
                ui = np.where(d["mask"][i], v, pop[i])
                ui = np.clip(ui, np.float32(-100), np.float32(100))
                assert np.array_equal(ui, s["u"][i])
                better = np.float32(s["fu64"][i]) <= fit[i]
                assert s["accept"][i] == better
            pop, fit = s["pop"], s["fit"]


def test_fitness_override_drives_selection():
    """step(..., fitness_override=fu) applies Alg. 1's selection rule to the given
    values: the trials and draws do not change, ties go to the trial, a NaN trial
    is never taken, and the float64 fitness is still returned for comparison."""
    p = W.make_problem("rastrigin", 6, 5, 0)
    N, D = 12, 6
    pop = pde.init_population(N, D, 5, 0, -100.0, 100.0)
    fit = evaluate(pop, p).astype(np.float32)
    th = pde.decode(np.array([0.5, 0.9, 1.5, 1.5, 1.5, 1.5], np.float32), 2)
    ref = pde.step(pop, fit, th, 0, 5, 0, -100.0, 100.0, p)
    same = pde.step(pop, fit, th, 0, 5, 0, -100.0, 100.0, p, fitness_override=ref["fu"])
    assert np.array_equal(same["u"], ref["u"]) and np.array_equal(same["accept"], ref["accept"])
    fo = fit.copy()                    # every trial ties its target: all taken
    fo[3] = np.nextafter(fit[3], np.float32(np.inf))   # one just above: kept out
    fo[5] = np.nan                     # a NaN trial is never taken
    s = pde.step(pop, fit, th, 0, 5, 0, -100.0, 100.0, p, fitness_override=fo)
    want = np.ones(N, bool)
    want[3] = want[5] = False
    assert np.array_equal(s["accept"], want)
    assert np.array_equal(s["u"], ref["u"])
    assert np.array_equal(s["fu64"], ref["fu64"])
    assert np.array_equal(s["pop"][want], ref["u"][want])
    assert np.array_equal(s["pop"][~want], pop[~want])
    assert np.array_equal(s["fit"][want], fo[want]) and np.array_equal(s["fit"][~want], fit[~want])
