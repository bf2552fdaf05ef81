"""Helpers of the GPU parity tests: run the oracle's own trajectory on the same
seeded inputs and compare it with the library generation by generation.

Both sides start from the same workload description (seed, streams, instance
data).  The library's trial vectors, index draws and crossover masks must
match the oracle bit for bit; its float32 fitness must be within the stated
relative tolerance of the oracle's float64 value of the same vector; its
selection decisions must match.  Selection and ranking are decided in float32
on both sides, but from values that carry different rounding errors, so a
decision between two values closer than the tolerance may legitimately go
either way.  The oracle flags such near-ties; from a flagged generation on
that run's trajectory is no longer compared (and counted as such).
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


def trajectory_parity(batch, wl, G, stats=None, check_desc=True):
    """Compare G generations, one traced launch each.  Returns per-run
    statistics: generations compared, first divergence, max fitness error."""
    runs = [OracleRun(wl, r) for r in range(wl.n_runs)]
    pop, fit = batch.host_state()
    out = {"compared": 0, "diverged": 0, "max_fit_rel": 0.0, "trials": 0, "ill": 0}
    for o in runs:
        gp = batch.run_pop(pop, o.r)
        assert np.array_equal(gp, o.pop), f"run {o.r}: initial population differs"
        fg = batch.run_fit(fit, o.r)
        bad, n_ill = fitness_misses(fg, o.f64, o.pop, o.prob)
        assert bad.size == 0, f"run {o.r}: initial fitness error {rel_err(fg, o.f64).max():.3g}"
        if n_ill:
            o.diverged, o.why = True, "initial fitness undetermined in float64"
            out["diverged"] += 1
            out["ill"] += n_ill
            continue
        out["max_fit_rel"] = max(out["max_fit_rel"], float(rel_err(fg, o.f64).max()))
    for g in range(G):
        u, fu, desc = batch.trace_step()
        pop, fit = batch.host_state()
        for o in runs:
            if o.diverged:
                continue
            s = o.step()
            r = o.r
            ug = batch.run_pop(u, r)
            fg = batch.run_fit(fu, r)
            dg = desc[batch.fit_off[r]:batch.fit_off[r + 1]]
            if s["amb_rank"] and not np.array_equal(ug, s["u"]):
                o.diverged, o.why = True, f"ranking near-tie at g={g}"
                out["diverged"] += 1
                continue
            if check_desc:
                try:
                    compare_desc(dg, s, o.th)
                except AssertionError as exc:
                    raise AssertionError(f"run {r} g={g} theta={o.th}: {exc}") from None
            bad = np.argwhere(ug != s["u"])
            assert bad.size == 0, f"run {r} g={g} theta={o.th}: trial vectors differ at {bad[:5].tolist()}"
            e = rel_err(fg, s["fu64"])
            miss, n_ill = fitness_misses(fg, s["fu64"], s["u"], o.prob)
            assert miss.size == 0, f"run {r} g={g} kind={o.prob.kind}: trial fitness error {e[miss].max():.3g}"
            if n_ill:
                o.diverged, o.why = True, f"trial fitness undetermined in float64 at g={g}"
                out["diverged"] += 1
                out["ill"] += n_ill
                continue
            out["max_fit_rel"] = max(out["max_fit_rel"], float(e.max()))
            out["trials"] += len(fg)
            acc_g = dg[:, 15].astype(bool)
            mism = acc_g != s["accept"]
            if np.any(mism & ~s["amb_sel"]):
                i = int(np.argwhere(mism & ~s["amb_sel"])[0, 0])
                raise AssertionError(f"run {r} g={g}: selection of {i} differs "
                                     f"(gpu {acc_g[i]}, oracle {s['accept'][i]})")
            pg = batch.run_pop(pop, r)
            if np.any(mism):
                o.diverged, o.why = True, f"selection near-tie at g={g}"
                out["diverged"] += 1
                continue
            assert np.array_equal(pg, s["pop"]), f"run {r} g={g}: population after selection differs"
            out["compared"] += 1
    out["runs"] = runs
    return out


def state_parity(batch, wl, G):
    """Compare the populations after each of G generations (one launch each)
    with the oracle's trajectory, without tracing: for paths that do not
    trace (the bf16 mode).  Runs stop being compared at an oracle near-tie."""
    runs = [OracleRun(wl, r) for r in range(wl.n_runs)]
    pop, fit = batch.host_state()
    out = {"compared": 0, "diverged": 0, "max_fit_rel": 0.0}
    for o in runs:
        assert np.array_equal(batch.run_pop(pop, o.r), o.pop), f"run {o.r}: initial population"
    for g in range(G):
        batch.inner_step(1)
        pop, fit = batch.host_state()
        for o in runs:
            if o.diverged:
                continue
            s = o.step()
            if s["amb_rank"] or np.any(s["amb_sel"]):
                o.diverged = True
                out["diverged"] += 1
                continue
            r = o.r
            assert np.array_equal(batch.run_pop(pop, r), o.pop), f"run {r} g={g} theta={o.th}: population differs"
            e = rel_err(batch.run_fit(fit, r), evaluate(o.pop, o.prob))
            assert e.max() <= FIT_RTOL, f"run {r} g={g}: fitness error {e.max():.3g}"
            out["max_fit_rel"] = max(out["max_fit_rel"], float(e.max()))
            out["compared"] += 1
    return out
