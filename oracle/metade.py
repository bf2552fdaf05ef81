"""MetaDE outer loop (the evolver) -- oracle (test infrastructure only).

Restates Alg. 3 and Secs. III-B..III-E of the paper:
  * the evolver is DE/rand/1/bin with F = 0.5, CR = 0.9 (Sec. III-E; the
    experimental setup of Sec. IV-A1) over 6-D vectors in the theta box;
  * the initial fitness of every evolver individual is +inf, so every trial
    of the first outer generation is accepted;
  * each trial is decoded (floor of the categorical parts) and scored by one
    executor run; all executors share the same random stream (one-shot
    evaluation, Sec. III-C), so the score is a deterministic function of theta;
  * the last outer generation runs the executors for 5 G' generations
    (power-up, Sec. III-D);
  * selection keeps the trial iff its score <= the target's.
Particle-swarm, competitive-swarm and natural-evolution-strategy evolvers
(Supplement S.III) are restated below as well.

The evolver draws its random numbers from the executor's Philox layout with
the stream word's top bit set, so the two never share counters.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .pde import (BIN, RAND, clip_theta, decode, init_population, make_trials, order_key,
                  run_executor, theta_bounds)

OUTER_THETA = {"F": np.float32(0.5), "CR": np.float32(0.9), "bl": RAND, "br": RAND, "dn": 1,
               "cs": BIN}


def outer_stream(stream: int) -> int:
    return philox.OUTER_STREAM_BIT | (int(stream) & 0x7FFFFFFF)


def outer_init(P, seed, stream, n_cs):
    lo, hi = theta_bounds(n_cs)
    X = init_population(P, 6, seed, outer_stream(stream), lo, hi)
    y = np.full(P, np.inf)
    return X, y


def outer_trials(X, y, g_o, seed, stream, n_cs, F=0.5, CR=0.9):
    """DE/rand/1/bin trial vectors of the evolver, clipped to the theta box."""
    lo, hi = theta_bounds(n_cs)
    th = dict(OUTER_THETA)
    th["F"], th["CR"] = np.float32(F), np.float32(CR)
    U, desc = make_trials(X, y, th, g_o, seed, outer_stream(stream), lo, hi)
    return clip_theta(U, n_cs), desc


def outer_select(X, y, U, y_trial):
    accept = ~np.isnan(y_trial) & (order_key(y_trial) <= order_key(y))
    return (np.where(accept[:, None], U, X).astype(np.float32), np.where(accept, y_trial, y),
            accept)


# ---------------------------------------------------------------- PSO evolver
#
# The paper's supplement (S.III) compares DE with PSO as the evolver, using
# the recommended inertia w = 0.729 and acceleration c1 = c2 = 1.49.  The
# particle swarm is the textbook one, restated here:
#   * positions start where the DE evolver's population starts, velocities at
#     zero, personal-best scores at +inf;
#   * outer generation 0 scores the initial positions; from generation 1 on,
#     every particle first moves:
#         v <- w v + c1 r1 (p - x) + c2 r2 (g - x),   x <- clip(x + v)
#     with r1, r2 uniform in [0, 1) per coordinate, p the particle's personal
#     best and g the best personal best (first in (score, index) order);
#   * a particle's personal best becomes its position iff the position's score
#     <= the personal-best score (the rule of the DE evolver's selection).
# Readings: float32 arithmetic in the order written, one rounding per
# operation; positions are clipped to the theta box, velocities are not;
# r1 and r2 of coordinate k are Philox words k and 6 + k of (particle, g_o) on
# the evolver's stream, mapped to (w >> 8) 2^-24.

PSO_W, PSO_C1, PSO_C2 = np.float32(0.729), np.float32(1.49), np.float32(1.49)


def pso_init(P, seed, stream, n_cs):
    X, y = outer_init(P, seed, stream, n_cs)
    return {"x": X.copy(), "v": np.zeros_like(X), "p": X.copy(), "py": y}


def pso_move(st, g_o, seed, stream, n_cs):
    """Velocities and positions of outer generation g_o >= 1."""
    lo, hi = theta_bounds(n_cs)
    P = st["x"].shape[0]
    w = philox.words(seed, np.arange(P), g_o, outer_stream(stream), 12)
    r = ((w >> np.uint64(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    r1, r2 = r[:, 0:6], r[:, 6:12]
    gi = int(np.lexsort((np.arange(P), order_key(st["py"])))[0])
    x, v, p = st["x"], st["v"], st["p"]
    g = p[gi][None, :]
    a = (PSO_C1 * r1) * (p - x)
    b = (PSO_C2 * r2) * (g - x)
    v = ((PSO_W * v) + a) + b
    x = np.minimum(np.maximum(x + v, lo), hi)
    st = dict(st)
    st["v"] = v.astype(np.float32)
    st["x"] = x.astype(np.float32)
    return st


def pso_select(st, y_new):
    better = ~np.isnan(y_new) & (order_key(y_new) <= order_key(st["py"]))
    st = dict(st)
    st["p"] = np.where(better[:, None], st["x"], st["p"]).astype(np.float32)
    st["py"] = np.where(better, y_new, st["py"])
    return st, better


# ---------------------------------------------------------------- CSO evolver
#
# The supplement (S.III) also uses the competitive swarm optimiser of Cheng
# and Jin (IEEE Trans. Cybernetics, 2015) as the evolver.  Restated from that
# published definition:
#   * the swarm starts at the DE evolver's initial population, at rest;
#     outer generation 0 scores the initial positions;
#   * from generation 1 on, the particles are split into random pairs; in
#     each pair the particle with the better score (first in (score, index)
#     order) wins and stays where it is; the loser l learns from the winner w:
#         v_l <- r1 v_l + r2 (x_w - x_l),   x_l <- clip(x_l + v_l)
#     with r1, r2 uniform in [0, 1) per coordinate;
#   * every particle then takes the score of its (new or unchanged) position.
# Readings: the social term towards the swarm's mean position is left out
# (its factor is 0, the setting that needs no tuning); all particles are
# scored every generation (one-shot evaluation gives a winner the score it
# already had, except in the powered-up last generation, where every
# particle is scored with the longer run); the pairing sorts the particles
# by Philox word 12 of (particle, g_o) on the evolver's stream (index breaks
# ties) and pairs positions 2k and 2k + 1, an odd last particle sitting out;
# r1, r2 of coordinate k are words k and 6 + k of the loser's (particle,
# g_o), mapped to (w >> 8) 2^-24; float32 arithmetic in the order written;
# velocities are not clipped.


def cso_init(P, seed, stream, n_cs):
    X, y = outer_init(P, seed, stream, n_cs)
    return {"x": X.copy(), "v": np.zeros_like(X), "y": y}


def cso_pairs(P, g_o, seed, stream):
    w = philox.words(seed, np.arange(P), g_o, outer_stream(stream), 13)
    order = np.lexsort((np.arange(P), w[:, 12].astype(np.uint64)))
    return [(int(order[2 * k]), int(order[2 * k + 1])) for k in range(P // 2)], w


def cso_move(st, g_o, seed, stream, n_cs):
    """Positions and velocities of outer generation g_o >= 1; also returns the
    (winner, loser) pairs."""
    lo, hi = theta_bounds(n_cs)
    P = st["x"].shape[0]
    pairs, w = cso_pairs(P, g_o, seed, stream)
    r = ((w[:, :12] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    x, v = st["x"].copy(), st["v"].copy()
    key = order_key(st["y"])
    wl_pairs = []
    for a, b in pairs:
        wn, ls = (a, b) if (key[a], a) < (key[b], b) else (b, a)
        r1, r2 = r[ls, 0:6], r[ls, 6:12]
        vn = (r1 * v[ls]) + (r2 * (x[wn] - x[ls]))
        v[ls] = vn
        x[ls] = np.minimum(np.maximum(x[ls] + vn, lo), hi)
        wl_pairs.append((wn, ls))
    st = dict(st)
    st["x"], st["v"] = x.astype(np.float32), v.astype(np.float32)
    return st, wl_pairs


def cso_select(st, y_new):
    st = dict(st)
    st["y"] = np.asarray(y_new, np.float64).copy()
    return st, np.ones(len(y_new), bool)


# ---------------------------------------------------------------- NES evolver
#
# The supplement (S.III) also uses a natural evolution strategy as the
# evolver.  Restated here is the separable NES (Schaul, Glasmachers and
# Schmidhuber, GECCO 2011): a Gaussian search distribution N(mu, diag sigma^2)
# over theta; every generation draws lambda = P samples z_k = mu + sigma s_k,
# s_k ~ N(0, I), scores them, ranks them (best first) and moves
#     mu    <- mu + eta_mu sigma * sum_r u_r s_(r)
#     sigma <- sigma * exp(eta_sigma / 2 * sum_r u_r (s_(r)^2 - 1))
# with the rank utilities u_r = max(0, ln(lambda/2 + 1) - ln r) / sum_q max(...)
# - 1/lambda, eta_mu = 1 and eta_sigma = (3 + ln d) / (5 sqrt d), d = 6.
# Readings: mu starts at the centre of the theta box and sigma at a quarter
# of its width; samples are clipped to the box before they are decoded and
# scored (the update uses the unclipped s); s comes from the Box-Muller
# transform of Philox words 2m, 2m + 1 of (sample k, g_o) on the evolver's
# stream (u1 = ((w >> 8) + 1) 2^-24, u2 = (w >> 8) 2^-24; s_2m = rho cos(2 pi
# u2), s_2m+1 = rho sin(2 pi u2), rho = sqrt(-2 ln u1)); the sampling, the
# utilities and the update run in float64 with sums in rank order, mu and
# sigma are kept in float32 between generations, and z is rounded once to
# float32; ties in score rank by sample index, NaN last.


def nes_init(n_cs):
    lo, hi = theta_bounds(n_cs)
    return {"mu": ((lo + hi) / np.float32(2)).astype(np.float32),
            "sigma": ((hi - lo) / np.float32(4)).astype(np.float32)}


def nes_normals(P, g_o, seed, stream):
    """s[k][j] for sample k: Box-Muller of Philox words (float64)."""
    w = philox.words(seed, np.arange(P), g_o, outer_stream(stream), 6).astype(np.uint64)
    s = np.empty((P, 6))
    for m in range(3):
        u1 = ((w[:, 2 * m] >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24
        u2 = (w[:, 2 * m + 1] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
        rho = np.sqrt(-2.0 * np.log(u1))
        s[:, 2 * m] = rho * np.cos(2.0 * np.pi * u2)
        s[:, 2 * m + 1] = rho * np.sin(2.0 * np.pi * u2)
    return s


def nes_samples(st, P, g_o, seed, stream, n_cs):
    lo, hi = theta_bounds(n_cs)
    s = nes_normals(P, g_o, seed, stream)
    z = (st["mu"].astype(np.float64)[None, :] + st["sigma"].astype(np.float64)[None, :] * s)
    return np.minimum(np.maximum(z.astype(np.float32), lo), hi), s


def nes_utilities(lam):
    a = np.array([max(0.0, np.log(lam / 2.0 + 1.0) - np.log(r)) for r in range(1, lam + 1)])
    tot = 0.0
    for v in a:
        tot = tot + v
    return a / tot - 1.0 / lam


def nes_update(st, y, g_o, seed, stream):
    P = len(y)
    s = nes_normals(P, g_o, seed, stream)
    order = np.lexsort((np.arange(P), order_key(y)))
    u = nes_utilities(P)
    gmu = np.zeros(6)
    gsig = np.zeros(6)
    for r in range(P):
        sk = s[order[r]]
        gmu = gmu + u[r] * sk
        gsig = gsig + u[r] * (sk * sk - 1.0)
    eta_sigma = (3.0 + np.log(6.0)) / (5.0 * np.sqrt(6.0))
    mu = st["mu"].astype(np.float64)
    sig = st["sigma"].astype(np.float64)
    return {"mu": (mu + sig * gmu).astype(np.float32),
            "sigma": (sig * np.exp((eta_sigma / 2.0) * gsig)).astype(np.float32)}


def run_metade(wl, gens=None, power_up=None, decide="f32", executor=None, log=None,
               evolver="de"):
    """Alg. 3 on a workload with an outer loop (evolver "de"; "pso", "cso" or
    "nes" swaps in the particle swarm, competitive swarm or separable NES of
    the supplement).  Returns the evolver state and the best
    (theta, y, x) found."""
    o = wl.outer
    P = o["P"]
    gens = o["gens"] if gens is None else gens
    pu = o.get("power_up", 5) if power_up is None else power_up
    stream = int(wl.stream[0])
    X, y = outer_init(P, wl.seed, stream, wl.n_cs)
    st = (pso_init(P, wl.seed, stream, wl.n_cs) if evolver == "pso" else
          cso_init(P, wl.seed, stream, wl.n_cs) if evolver == "cso" else
          nes_init(wl.n_cs) if evolver == "nes" else None)
    best_x = np.zeros((P, wl.D_of(0)), np.float32)
    for g_o in range(gens):
        if evolver == "pso":
            if g_o > 0:
                st = pso_move(st, g_o, wl.seed, stream, wl.n_cs)
            U = st["x"]
        elif evolver == "cso":
            if g_o > 0:
                st, _ = cso_move(st, g_o, wl.seed, stream, wl.n_cs)
            U = st["x"]
        elif evolver == "nes":
            U, _ = nes_samples(st, P, g_o, wl.seed, stream, wl.n_cs)
        else:
            U, _ = outer_trials(X, y, g_o, wl.seed, stream, wl.n_cs, o["F"], o["CR"])
        dec = decode(U, wl.n_cs)
        G = wl.G * (pu if g_o == gens - 1 else 1)
        ys = np.empty(P)
        xs = np.zeros_like(best_x)
        for i in range(P):
            th = {k: v[i] for k, v in dec.items()}
            prob = wl.problems[int(wl.problem[i])]
            if executor is not None:
                res = executor(i, th, G)
            else:
                res = run_executor(int(wl.N[i]), prob.D, th, G, wl.seed, int(wl.stream[i]),
                                   wl.lb, wl.ub, prob, decide)
            ys[i] = res["y"]
            xs[i] = res["best_x"]
        if evolver == "pso":
            st, acc = pso_select(st, ys)
            X, y = st["p"], st["py"]
        elif evolver == "cso":
            st, acc = cso_select(st, ys)
            X, y = st["x"], st["y"]
        elif evolver == "nes":
            st = nes_update(st, ys, g_o, wl.seed, stream)
            X, y, acc = U, ys, np.ones(P, bool)
        else:
            X, y, acc = outer_select(X, y, U, ys)
        best_x = np.where(acc[:, None], xs, best_x)
        if log is not None:
            log.append({"g": g_o, "U": U, "y_trial": ys, "accept": acc})
    b = int(np.lexsort((np.arange(P), order_key(y)))[0])
    return {"X": X, "y": y, "best_index": b, "best_theta": X[b], "best_y": float(y[b]),
            "best_x": best_x[b], "best_x_all": best_x}
