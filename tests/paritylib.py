"""Helpers of the GPU parity tests: run the oracle on the same seeded inputs
and compare it with the library generation by generation.

Both sides start from the same workload description (seed, streams, instance
data).  The library's trial vectors, index draws and crossover masks must
match the oracle bit for bit, and its float32 fitness must be within the
stated relative tolerance of the oracle's float64 value of the same vector.

Selection is compared literally: the oracle's generation step is given the
library's trial fitness (``fitness_override``) and applies the selection rule
of Alg. 1 to exactly the values the library decided on, so every decision is
checked, ties and near-ties included, and both sides keep identical
populations and fitness values -- the ranking of the next generation then
starts from identical inputs too.  The fitness values themselves are checked
against the float64 oracle separately, trial by trial.
"""
from __future__ import annotations

import numpy as np

from oracle import pde
from oracle.fitness import evaluate, lqr_mlp

FIT_RTOL = 1e-5           # float32 fitness vs float64 oracle, relative
TIE_RTOL = 3e-5           # two values closer than this may be ordered either way
ILL_RTOL = FIT_RTOL / 10  # float64 vs extended precision: beyond this float64 does not fix f


def near(a, b, rtol=TIE_RTOL):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    scale = np.maximum(np.abs(a), np.abs(b))
    return np.abs(a - b) <= rtol * scale


def ranking_ambiguous(fit, kp, th):
    """True when the ranking positions the trials read contain values closer
    than the tie tolerance: positions 0-1 for 'best', 0..kp for 'pbest'
    (pbest maps a drawn rank to an individual, so order inside the top-p set
    matters, and so does its boundary)."""
    uses = {th["bl"], th["br"]}
    if pde.PBEST in uses:
        last = kp
    elif pde.BEST in uses:
        last = 1
    else:
        return False
    f = np.sort(pde.order_key(fit))[: last + 1]
    return bool(np.any(near(f[:-1], f[1:])))


class OracleRun:
    """The oracle's independent trajectory of one executor run."""

    def __init__(self, wl, r, theta_row=None):
        self.wl = wl
        self.r = r
        self.prob = wl.problems[int(wl.problem[r])]
        self.N = int(wl.N[r])
        self.D = self.prob.D
        self.stream = int(wl.stream[r])
        th = wl.theta[r] if theta_row is None else theta_row
        self.th = pde.decode(np.asarray(th, np.float32), wl.n_cs)
        self.th = {k: (v.item() if hasattr(v, "item") else v) for k, v in self.th.items()}
        self.pop = pde.init_population(self.N, self.D, wl.seed, self.stream, wl.lb, wl.ub)
        self.f64 = evaluate(self.pop, self.prob)
        self.fit = self.f64.astype(np.float32)
        self.g = 0
        self.diverged = False
        self.why = ""

    def step(self):
        amb_rank = ranking_ambiguous(self.fit, pde.top_count(self.N), self.th)
        s = pde.step(self.pop, self.fit, self.th, self.g, self.wl.seed, self.stream, self.wl.lb,
                     self.wl.ub, self.prob, decide="f32")
        amb_sel = near(s["fu64"], self.fit) & ~np.isnan(s["fu64"])
        s["amb_rank"] = amb_rank
        s["amb_sel"] = amb_sel
        self.pop, self.fit = s["pop"], s["fit"]
        self.g += 1
        return s


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-300)


def fitness_misses(fg, f64, u, prob):
    """Trials whose float32 fitness misses the oracle's float64 value by more
    than FIT_RTOL, split into (well-determined misses, count of trials whose
    float64 value is itself undetermined).  Only the control workload can
    have the latter: its closed loop may amplify rounding by many orders of
    magnitude, which the oracle measures by re-running in extended precision."""
    e = rel_err(fg, f64)
    bad = np.flatnonzero(e > FIT_RTOL)
    if bad.size == 0 or prob.kind != "lqr_mlp":
        return bad, 0
    fx = lqr_mlp(u[bad], prob, dtype=np.longdouble).astype(np.float64)
    ill = rel_err(f64[bad], fx) > ILL_RTOL
    return bad[~ill], int(ill.sum())


def compare_desc(desc_gpu, s, th):
    """Bit-exact comparison of the per-target draws with the oracle's."""
    d = s["desc"]
    N = desc_gpu.shape[0]
    dn = th["dn"]
    assert np.array_equal(desc_gpu[:, 0], d["i_bl"]), "base-left index"
    assert np.array_equal(desc_gpu[:, 1], d["i_br"]), "base-right index"
    pairs = d["pairs"].reshape(N, 2 * dn)
    assert np.array_equal(desc_gpu[:, 2:2 + 2 * dn], pairs), "difference pairs"
    assert np.all(desc_gpu[:, 2 + 2 * dn:10] == -1)
    assert np.array_equal(desc_gpu[:, 10], d["jn"]), "j_rand / n"
    if th["cs"] == pde.EXP:
        assert np.array_equal(desc_gpu[:, 11], d["L"]), "exponential length"
    assert np.array_equal(desc_gpu[:, 12], d["pbest_rank"]), "pbest rank"
    assert np.array_equal(desc_gpu[:, 13], d["r0"]), "rand index"
    if th["cs"] == pde.ARITH:
        assert np.array_equal(desc_gpu[:, 14].astype(np.int32).view(np.float32), d["K"]), "K"


def _check_step(prob, r, s, ug, fg, dg, pg, fitg, th, g, out):
    """One run-generation of the library (trials ug, fitness fg, descriptors
    dg, population pg and fitness fitg after selection) against the oracle
    step s taken from the same state with the library's fitness."""
    bad = np.argwhere(ug != s["u"])
    assert bad.size == 0, f"run {r} g={g} theta={th}: trial vectors differ at {bad[:5].tolist()}"
    try:
        compare_desc(dg, s, th)
    except AssertionError as exc:
        raise AssertionError(f"run {r} g={g} theta={th}: {exc}") from None
    e = rel_err(fg, s["fu64"])
    miss, n_ill = fitness_misses(fg, s["fu64"], s["u"], prob)
    assert miss.size == 0, f"run {r} g={g} kind={prob.kind}: trial fitness error {e[miss].max():.3g}"
    out["ill"] += n_ill
    ok = rel_err(fg, s["fu64"]) <= FIT_RTOL
    if np.any(ok):
        out["max_fit_rel"] = max(out["max_fit_rel"], float(e[ok].max()))
    acc_g = dg[:, 15].astype(bool)
    mism = np.flatnonzero(acc_g != s["accept"])
    if mism.size:
        i = int(mism[0])
        raise AssertionError(f"run {r} g={g}: selection of {i} differs (gpu {acc_g[i]}, "
                             f"oracle rule on the same values {s['accept'][i]}; "
                             f"f(u)={fg[i]!r} f(x)={s['fx'][i]!r})")
    assert np.array_equal(pg, s["pop"]), f"run {r} g={g}: population after selection differs"
    assert np.array_equal(fitg, s["fit"], equal_nan=True), f"run {r} g={g}: fitness after selection differs"
    out["trials"] += len(fg)
    out["accepted"] += int(acc_g.sum())
    # decisions between values closer than the tie tolerance: the hard cases,
    # checked like every other one
    fx = s["fx"]
    out["near_ties"] += int(np.sum(near(fg, fx) & ~np.isnan(fg) & ~np.isnan(fx)))
    out["exact_ties"] += int(np.sum(fg == fx))
    out["compared"] += 1


def trajectory_parity(batch, wl, G):
    """Compare G generations, one traced launch each, every run and every
    trial.  The oracle's trajectory takes the library's fitness values (after
    checking each against the float64 oracle), so it never leaves the
    library's: nothing is skipped."""
    runs = [OracleRun(wl, r) for r in range(wl.n_runs)]
    pop, fit = batch.host_state()
    out = {"compared": 0, "diverged": 0, "max_fit_rel": 0.0, "trials": 0, "ill": 0,
           "accepted": 0, "near_ties": 0, "exact_ties": 0}
    for o in runs:
        gp = batch.run_pop(pop, o.r)
        assert np.array_equal(gp, o.pop), f"run {o.r}: initial population differs"
        fg = batch.run_fit(fit, o.r)
        bad, n_ill = fitness_misses(fg, o.f64, o.pop, o.prob)
        assert bad.size == 0, f"run {o.r}: initial fitness error {rel_err(fg, o.f64).max():.3g}"
        out["ill"] += n_ill
        e0 = rel_err(fg, o.f64)
        if np.any(e0 <= FIT_RTOL):
            out["max_fit_rel"] = max(out["max_fit_rel"], float(e0[e0 <= FIT_RTOL].max()))
        o.fit = fg.copy()   # identical inputs from here on
    for g in range(G):
        u, fu, desc = batch.trace_step()
        pop, fit = batch.host_state()
        for o in runs:
            r = o.r
            fg = batch.run_fit(fu, r)
            s = pde.step(o.pop, o.fit, o.th, o.g, wl.seed, o.stream, wl.lb, wl.ub, o.prob,
                         decide="f32", fitness_override=fg)
            s["fx"] = o.fit
            _check_step(o.prob, r, s, batch.run_pop(u, r), fg,
                        desc[batch.fit_off[r]:batch.fit_off[r + 1]], batch.run_pop(pop, r),
                        batch.run_fit(fit, r), o.th, g, out)
            o.pop, o.fit = s["pop"], s["fit"]
            o.g += 1
    out["runs"] = runs
    return out


def resync_parity(batch, wl, g, theta, runs=None):
    """One traced generation taken from the library's own state after g
    generations (e.g. deep inside a full-size launch): the oracle steps that
    state with the library's fitness, and every trial, draw and decision is
    compared.  ``theta`` holds the runs' theta rows (continuous encoding)."""
    pop, fit = batch.host_state()
    u, fu, desc = batch.trace_step()
    pop2, fit2 = batch.host_state()
    out = {"compared": 0, "max_fit_rel": 0.0, "trials": 0, "ill": 0, "accepted": 0,
           "near_ties": 0, "exact_ties": 0}
    for r in (range(wl.n_runs) if runs is None else runs):
        r = int(r)
        prob = wl.problems[int(wl.problem[r])]
        th = pde.decode(np.asarray(theta[r], np.float32), wl.n_cs)
        th = {k: (v.item() if hasattr(v, "item") else v) for k, v in th.items()}
        fx = batch.run_fit(fit, r).copy()
        fg = batch.run_fit(fu, r)
        s = pde.step(batch.run_pop(pop, r).copy(), fx, th, g, wl.seed, int(wl.stream[r]), wl.lb,
                     wl.ub, prob, decide="f32", fitness_override=fg)
        s["fx"] = fx
        _check_step(prob, r, s, batch.run_pop(u, r), fg,
                    desc[batch.fit_off[r]:batch.fit_off[r + 1]], batch.run_pop(pop2, r),
                    batch.run_fit(fit2, r), th, g, out)
    return out
