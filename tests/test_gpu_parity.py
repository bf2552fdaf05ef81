"""GPU parity of the HIP path against the CPU oracle (needs an MI355X).

Every test builds its inputs from the seeded generators, runs the library
through the C ABI (via the thin binding) and the oracle independently, and
compares: trial vectors, index draws and masks bit for bit, float32 fitness
to relative 1e-5 of the float64 oracle, and every selection decision exactly
(the oracle applies the selection rule to the library's own fitness values,
so ties and near-ties are checked like any other decision).  Tests that
compare whole runs without tracing (the evolver's scores) still allow a
near-tie to send the two trajectories apart, and say so where they do.
"""
import itertools
import sys

import numpy as np
import pytest

import workloads as W
from oracle import metade as ometa
from oracle import pde
from oracle.fitness import evaluate
from paritylib import FIT_RTOL, OracleRun, rel_err, resync_parity, trajectory_parity

pytestmark = pytest.mark.gpu


def _batch(wl, **kw):
    from paper_2502_10470_amd import Batch
    print(f"[case] {wl.name} runs={wl.n_runs} N={sorted(set(wl.N.tolist()))[:6]} "
          f"D={sorted(set(wl.D_of(r) for r in range(wl.n_runs)))[:6]}", flush=True)
    return Batch(wl, **kw)


def _theta_for(bl, br, dn, cs, F=0.6, CR=0.7):
    return [F, CR, bl + 0.5, br + 0.5, dn + 0.5, cs + 0.5]


def test_every_strategy_small():
    """All 192 strategies DE/bl-to-br/dn/cs (Sec. III-A), one run each, small
    ragged populations and dimensions, 4 traced generations."""
    combos = list(itertools.product([1, 2, 3, 4], [1, 2, 3, 4], [1, 2, 3, 4], [1, 2, 3]))
    assert len(combos) == 192
    rng = np.random.default_rng(0)
    theta = np.array([_theta_for(*c, F=rng.uniform(0, 1), CR=rng.uniform(0, 1)) for c in combos],
                     np.float32)
    Ns = [10 + (k * 7) % 41 for k in range(192)]
    Ds = [1 + (k * 5) % 13 for k in range(192)]
    kinds = ["rastrigin", "rosenbrock", "ackley", "elliptic", "schwefel"]
    wl = W.small_batch(11, kinds, Ns, Ds, n_cs=3, theta=theta)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=4)
    print("compared", out["compared"], "near ties", out["near_ties"], "max rel", out["max_fit_rel"])
    assert out["compared"] == 192 * 4


@pytest.mark.parametrize("N,D", [(10, 2), (33, 7), (64, 20), (100, 20), (200, 37), (256, 64),
                                 (256, 100), (130, 128), (200, 90)])
def test_tiles_and_ragged_tails(N, D):
    """Population and dimension sizes spanning several LDS tiles and chunks,
    with ragged tails (D not a multiple of 4, N not a multiple of a wave).
    The last three run the matrix-core kernel; at N = 200, D = 90 its 42
    (output tile, row-tile pair) items fall unevenly on the eight waves."""
    kinds = ["rastrigin", "elliptic", "ackley", "rosenbrock", "schwefel"]
    wl = W.small_batch(N * 1000 + D, kinds, [N] * 5, [D] * 5, n_cs=3)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=3)
    assert out["compared"] == 15


def test_largest_population_that_fits_and_the_first_that_does_not():
    """N = 256 at D = 124, the largest dimension whose population, draws and
    per-tile partial sums fit the 160 KB of LDS of the matrix-core kernel in
    the plain precision (Rosenbrock, with two more per-tile arrays, and the
    bf16 mode reach 112 and 116), against the oracle; D = 128 at N = 256 is
    rejected at set-up with the LDS message, before any launch."""
    from paper_2502_10470_amd import metade as M
    wl = W.small_batch(256124, ["rastrigin", "elliptic"], [256] * 2, [124] * 2, n_cs=3)
    out = trajectory_parity(_batch(wl), wl, G=2)
    assert out["compared"] == 4
    wl = W.small_batch(256116, ["ackley"], [256], [116], n_cs=3)
    out = trajectory_parity(_batch(wl, precision=M.BF16_REFINE), wl, G=2)
    assert out["compared"] == 2
    for kind, D, kw in (("rastrigin", 128, {}), ("rosenbrock", 116, {}),
                        ("ackley", 120, {"precision": M.BF16_REFINE})):
        wl = W.small_batch(7, [kind], [256], [D], n_cs=3)
        with pytest.raises(M.MetadeError, match="does not fit in LDS"):
            _batch(wl, **kw)


def test_hybrid_function():
    p = W.make_problem("hybrid", 20, 2, 0)
    wl = W.small_batch(2, ["hybrid"], [100] * 6, [20] * 6, n_cs=2)
    wl.problems = [p] * 6
    wl.problem = np.zeros(6, np.uint32)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=5)
    assert out["compared"] == 30


def test_uneven_batch_c2_sample():
    """The uneven batch (256 runs, N 20..200, D 10/20, four kinds) in one
    launch; all runs traced for 3 generations."""
    wl = W.workload_c2()
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=3)
    print("compared", out["compared"], "near ties", out["near_ties"], "max rel", out["max_fit_rel"])
    assert out["compared"] == 256 * 3


def _oracle_final(wl, r, G):
    o = OracleRun(wl, r)
    ambiguous = False
    for _ in range(G):
        s = o.step()
        ambiguous |= bool(s["amb_rank"] or np.any(s["amb_sel"]))
    return o, ambiguous


@pytest.mark.parametrize("name,G,sample,need", [("c4", 2, 40, 6), ("c2", 5, 32, 12)])
def test_full_size_multi_generation_launch(name, G, sample, need):
    """Full-size workloads in the launch shape the benchmark times (all
    generations in one persistent launch): sampled runs must end in exactly the
    oracle's state when the oracle saw no near-tie on the way."""
    wl = W.workload_by_name(name)
    b = _batch(wl)
    b.inner_step(G)
    pop, fit = b.host_state()
    rng = np.random.default_rng(3)
    runs = rng.choice(wl.n_runs, size=sample, replace=False)
    checked = 0
    for r in runs:
        o, amb = _oracle_final(wl, int(r), G)
        if amb:
            continue
        assert np.array_equal(b.run_pop(pop, r), o.pop), f"run {r}: population differs after {G} generations"
        e = rel_err(b.run_fit(fit, r), evaluate(o.pop, o.prob))
        assert e.max() <= FIT_RTOL
        checked += 1
    print(f"{name}: {checked} of {sample} sampled runs free of near-ties, all identical", flush=True)
    assert checked >= need


def test_best_record_float64():
    """y* is the float64 fitness of the float32-best individual; best_x is that
    individual.  Checked on the library's own final state: the best by (f, i)
    of its float32 fitness, and the oracle's float64 value of that vector."""
    wl = W.small_batch(5, ["rastrigin", "elliptic", "ackley", "rosenbrock", "schwefel"],
                       [40] * 10, [10, 20] * 5)
    b = _batch(wl)
    b.inner_step(6)
    y = b.get_best()
    pop, fit = b.host_state()
    bx = b.best_x.cpu().numpy()
    for r in range(wl.n_runs):
        gp = b.run_pop(pop, r)
        k = int(pde.ranking(b.run_fit(fit, r))[0])
        assert np.array_equal(b.run_bx(bx, r), gp[k])
        ref = float(evaluate(gp[k], wl.problems[int(wl.problem[r])]))
        assert abs(y[r] - ref) <= 1e-12 * abs(ref)


def _outer_parity(wl, n_outer):
    P = wl.outer["P"]
    b = _batch(wl)
    b.outer_reset()
    X, y, _, _ = b.get_outer()
    Xo, yo = ometa.outer_init(P, wl.seed, 0, wl.n_cs)
    assert np.array_equal(X, Xo) and np.all(np.isinf(y))
    for g_o in range(n_outer):
        b.outer_step(wl.G, 1)
        X2, y2, U, yt = b.get_outer()
        Uo, _ = ometa.outer_trials(Xo, yo, g_o, wl.seed, 0, wl.n_cs)
        assert np.array_equal(U, Uo), f"outer trial vectors differ at g_o={g_o}"
        ys = np.empty(P)
        diverged = False
        for i in range(P):
            o = OracleRun(wl, i, theta_row=Uo[i])
            amb = False
            for _ in range(wl.G):
                s = o.step()
                amb |= bool(s["amb_rank"] or np.any(s["amb_sel"]))
            k = int(pde.ranking(o.fit)[0])
            ys[i] = float(evaluate(o.pop[k], o.prob))
            same = abs(yt[i] - ys[i]) <= 1e-12 * abs(ys[i])
            # a near-tie on the way allows the other trajectory; otherwise the scores agree
            assert same or amb, f"executor {i} score"
            diverged |= not same
        print("g_o", g_o, "an executor took the other side of a near-tie:", diverged, flush=True)
        if diverged:
            break  # the two evolvers may now legitimately differ
        Xo, yo, acc = ometa.outer_select(Xo, yo, Uo, ys)
        assert np.array_equal(X2, Xo)
        assert np.allclose(y2, yo, rtol=1e-12, atol=0)
        # scores agree to double rounding only; keep the library's exact values
        # out of the oracle: continue from the oracle's own state


def test_outer_step_c1():
    """Evolver (Alg. 3) on the small MetaDE config: initial population,
    trial vectors, decoded theta, executor scores and selection."""
    _outer_parity(W.workload_c1(), 2)


def test_outer_step_paper_meta_space():
    """The paper's own configuration shape: executors N=100 at D=20 and the
    full meta-space with three crossover schemes (192 strategies), on a
    slice of the evolver population and a few inner generations."""
    _outer_parity(W.workload_paper(P=12, gens=2, G=4), 2)


def test_metade_run_c1_consistency():
    wl = W.workload_c1()
    b = _batch(wl)
    by, bt, bx = b.run(2, wl.G, 5)
    X, y, _, _ = b.get_outer()
    k = int(np.lexsort((np.arange(8), y))[0])
    assert by == y[k] and np.array_equal(bt, X[k])
    assert bx.min() >= -100 and bx.max() <= 100
    # one-shot: rerunning the best theta alone reproduces its score (it was
    # scored either by a G-generation run or by the powered-up last one)
    b2 = _batch(wl)
    b2.set_theta(np.repeat(bt[None, :], 8, axis=0))
    b2.inner_step(wl.G)
    y_short = b2.get_best()[0]
    b2.inner_step(wl.G * 4)
    y_long = b2.get_best()[0]
    assert by in (y_short, y_long)


def test_determinism_and_checkpoint():
    wl = W.small_batch(7, ["rastrigin", "ackley"], [50, 60, 70], [10, 20, 15])
    a = _batch(wl)
    a.inner_step(20)
    blob = a.get_state()
    a.inner_step(20)
    pa, fa = a.host_state()
    b = _batch(wl)
    b.set_state(blob)
    b.inner_step(20)
    pb, fb = b.host_state()
    assert np.array_equal(pa, pb) and np.array_equal(fa, fb)
    c = _batch(wl)
    c.inner_step(40)
    pc, fc = c.host_state()
    assert np.array_equal(pa, pc) and np.array_equal(fa, fc)


def test_invariants_long_run():
    """1000 generations: fitness never increases, genes stay in the box, y*
    is consistent with the float32 record."""
    wl = W.small_batch(9, ["rastrigin", "elliptic", "rosenbrock", "ackley"], [100] * 8, [20] * 8)
    b = _batch(wl)
    _, f0 = b.host_state()
    b.inner_step(500)
    _, f1 = b.host_state()
    b.inner_step(500)
    pop, f2 = b.host_state()
    assert np.all(f1 <= f0) and np.all(f2 <= f1)
    assert pop.min() >= -100 and pop.max() <= 100
    y = b.get_best()
    for r in range(wl.n_runs):
        assert abs(y[r] - b.run_fit(f2, r).min()) <= 1e-5 * abs(y[r])


def test_run_order_independence():
    """Runs share a launch but nothing else: the same runs listed in another
    order (each keeping its problem, stream and theta) end bit-identical, on
    both generation kernels."""
    import dataclasses
    kinds = ["rastrigin", "elliptic", "hybrid", "schwefel", "ackley", "rosenbrock"]
    Ns = [40, 100, 64, 256, 33, 120]
    Ds = [10, 20, 20, 100, 7, 64]
    wl = W.small_batch(31, kinds, Ns, Ds, n_cs=3)
    perm = np.array([3, 0, 5, 1, 4, 2])
    wl2 = dataclasses.replace(wl, N=wl.N[perm], problem=wl.problem[perm], stream=wl.stream[perm],
                              theta=wl.theta[perm], name=wl.name + "_perm")
    a, b = _batch(wl), _batch(wl2)
    a.inner_step(12)
    b.inner_step(12)
    pa, fa = a.host_state()
    pb, fb = b.host_state()
    ya, yb = a.get_best(), b.get_best()
    for k, r in enumerate(perm):
        assert np.array_equal(a.run_pop(pa, r), b.run_pop(pb, k)), f"run {r}"
        assert np.array_equal(a.run_fit(fa, r), b.run_fit(fb, k))
        assert ya[r] == yb[k]


def test_nan_targets_rank_last_and_are_replaced():
    """A NaN target fitness counts as +inf: it ranks last and any finite trial
    replaces it (the oracle's step on the same state decides the same way)."""
    wl = W.small_batch(41, ["rastrigin", "elliptic"], [30, 50], [10, 12], n_cs=2,
                       theta=np.array([_theta_for(3, 1, 2, 1, CR=0.8),
                                       _theta_for(2, 3, 1, 2, CR=0.4)], np.float32))
    b = _batch(wl)
    pop0, fit0 = b.host_state()
    fit_nan = fit0.copy()
    nan_idx = [0, 3, 7, 31, 42, 79]
    fit_nan[nan_idx] = np.nan
    b.fit.copy_(b.torch.from_numpy(fit_nan).to(b.fit.device))
    u, fu, desc = b.trace_step()
    pop1, fit1 = b.host_state()
    for r in range(wl.n_runs):
        o = OracleRun(wl, r)
        fr = b.run_fit(fit_nan, r)
        s = pde.step(o.pop, fr.astype(np.float32), o.th, 0, wl.seed, o.stream, wl.lb, wl.ub,
                     o.prob)
        assert np.array_equal(b.run_pop(u, r), s["u"]), f"run {r}: trials (NaN ranks last)"
        acc = desc[b.fit_off[r]:b.fit_off[r + 1], 15].astype(bool)
        nan_here = np.isnan(fr)
        assert nan_here.any() and np.all(acc[nan_here]), f"run {r}: NaN targets kept"
        assert np.all(np.isfinite(b.run_fit(fit1, r)))
        # the selection rule on the library's own values: every decision
        s2 = pde.step(o.pop, fr.astype(np.float32), o.th, 0, wl.seed, o.stream, wl.lb, wl.ub,
                      o.prob, fitness_override=b.run_fit(fu, r))
        assert np.array_equal(acc, s2["accept"])
        assert np.all(rel_err(b.run_fit(fu, r), s["fu64"]) <= FIT_RTOL)


def test_theta_outside_the_box_and_nan():
    """θ components outside the box are clipped and NaN components take the
    lower bound when the library decodes θ (the box's upper end maps to the
    last category); the trajectories follow the oracle run on the clipped θ."""
    import dataclasses
    raw = np.array([[1.7, -0.3, 7.2, 0.1, 5.0, 9.0],
                    [np.nan, 0.6, np.nan, 3.5, np.nan, 2.5],
                    [0.5, np.nan, 2.5, 9.5, -4.0, np.nan],
                    [-2.0, 2.0, 4.999, 1.0, 3.9, 1.0]], np.float32)
    lo, hi = W.theta_box(3)
    clean = np.where(np.isnan(raw), lo, np.minimum(np.maximum(raw, lo), hi)).astype(np.float32)
    wl = W.small_batch(61, ["rastrigin", "elliptic"], [24, 30, 17, 40], [10, 13, 7, 20],
                       theta=clean, n_cs=3)
    b = _batch(wl)
    b.set_theta(raw)
    out = trajectory_parity(b, dataclasses.replace(wl, theta=clean), G=3)
    assert out["compared"] == 12


def _c3_executor_theta(wl):
    """theta of the default workload's first evolver generation (its trial vectors)."""
    X, y = ometa.outer_init(wl.outer["P"], wl.seed, int(wl.stream[0]), wl.n_cs)
    U, _ = ometa.outer_trials(X, y, 0, wl.seed, int(wl.stream[0]), wl.n_cs)
    return U


def test_resync_c3_late_generation():
    """Full MetaDE at D=20 (64 executors, N = 100, hybrid): 999 generations in
    one persistent launch, then one traced generation from the library's own
    state compared with the oracle step on that state -- every trial, draw and
    selection decision of all 64 runs, 1000 generations deep."""
    wl = W.workload_c3()
    U = _c3_executor_theta(wl)
    b = _batch(wl)
    b.set_theta(U)
    b.inner_step(999)
    out = resync_parity(b, wl, 999, U)
    print(out, flush=True)
    assert out["compared"] == 64 and out["trials"] == 6400


@pytest.mark.parametrize("G", [1, 499])
def test_resync_c4_late_generation(G):
    """D = 100 (128 runs x N = 256, elliptic and Rastrigin, matrix-core
    kernel): G generations in one launch, then one traced generation compared
    run by run and decision by decision with the oracle."""
    wl = W.workload_c4()
    b = _batch(wl)
    b.inner_step(G)
    out = resync_parity(b, wl, G, wl.theta)
    print(out, flush=True)
    assert out["compared"] == 128 and out["trials"] == 128 * 256


@pytest.mark.parametrize("seed", [777, 2002])
def test_random_batches(seed):
    """Seeded random batches: 1 to 6 runs each, every kind, N in 10..256,
    D in 1..128 (3.. for the hybrid), two or three crossover schemes, both
    precisions; each batch is checked against the oracle for 3 generations.
    A batch that fits no generation kernel's LDS must be rejected at set-up."""
    from paper_2502_10470_amd import metade as M
    rng = np.random.default_rng(seed)
    kinds_all = ["rastrigin", "rosenbrock", "ackley", "elliptic", "schwefel", "hybrid"]
    compared = 0
    for case in range(30):
        runs = int(rng.integers(1, 7))
        Ns = [int(rng.integers(10, 257)) for _ in range(runs)]
        Ds = [int(rng.integers(1, 129)) for _ in range(runs)]
        kinds = [kinds_all[int(rng.integers(0, 6))] for _ in range(runs)]
        Ds = [max(d, 3) if k == "hybrid" else d for d, k in zip(Ds, kinds)]
        prec = M.BF16_REFINE if rng.random() < 0.3 else M.FP32
        n_cs = int(rng.integers(2, 4))
        wl = W.small_batch(int(rng.integers(0, 2**31)), kinds, Ns, Ds, n_cs=n_cs)
        print(f"[case {case}] precision={prec} runs={list(zip(kinds, Ns, Ds))}", flush=True)
        try:
            b = _batch(wl, precision=prec)
        except M.MetadeError as e:
            assert "does not fit in LDS" in str(e), str(e)
            continue
        out = trajectory_parity(b, wl, G=3)
        assert out["compared"] == 3 * runs
        compared += out["compared"]
        b.close()
    print("run-generations compared:", compared)
    assert compared >= 200


def test_per_kind_kernel_matches_generic_kernel():
    """A batch whose runs all have one kind runs that kind's own generation
    kernel, a batch of several kinds the generic one; both hold the same loop,
    so the same runs must end bit for bit equal after a full-length launch."""
    kinds = ["hybrid", "hybrid", "hybrid", "rastrigin"]
    wl_one = W.small_batch(4242, kinds[:3], [100] * 3, [20] * 3, n_cs=3)
    wl_mix = W.small_batch(4242, kinds, [100] * 4, [20] * 4, n_cs=3)
    assert np.array_equal(wl_one.theta, wl_mix.theta[:3])
    a, b = _batch(wl_one), _batch(wl_mix)
    a.inner_step(300)
    b.inner_step(300)
    pa, fa = a.host_state()
    pb, fb = b.host_state()
    for r in range(3):
        assert np.array_equal(a.run_pop(pa, r), b.run_pop(pb, r)), f"run {r}: populations differ"
        assert np.array_equal(a.run_fit(fa, r), b.run_fit(fb, r)), f"run {r}: fitness differs"
