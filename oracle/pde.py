"""Parameterized DE (the executor) -- oracle (test infrastructure only).

Restates Sec. III-A (PDE), Alg. 2, Eqs. (1)-(12) and Table I of the paper.
Where the paper is silent or ambiguous the reading taken is stated inline.

One generation, synchronous over the population (the paper tensorises
mutation and crossover, Sec. III-A, so every trial is built from the
generation-g population):
  1. rank the population by (fitness, index), NaN counted as +inf;
     best = first, top-p set = first k_p = max(1, ceil(N/10)) (p = 10%, the
     value the paper gives as typical for current-to-pbest, Eq. (6)).
  2. per target i draw indices from Philox words: the random base (when bl or
     br is 'rand') and dn difference pairs, all mutually distinct and != i;
     a pbest pick from the top-p set; j_rand (or the start n); K_i.
  3. mutation, Eq. (12): v = x_bl + F (x_br - x_bl) + F (D_1 + ... + D_dn);
     the middle term is absent when bl == br.
  4. crossover by cs: binomial Eq. (8), exponential Eq. (9), arithmetic
     Eq. (10); then clip to the search box.
  5. evaluate, then greedy selection: u_i replaces x_i iff f(u_i) <= f(x_i)
     (Alg. 1 selection rule).

Philox word map of one (individual, generation): words 0..8 index draws,
9 pbest pick, 10 j_rand / n, 11 K_i, 12+t the t-th crossover uniform.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .fitness import evaluate

RAND, BEST, PBEST, CURRENT = 1, 2, 3, 4
BIN, EXP, ARITH = 1, 2, 3

W_PBEST, W_JRAND, W_K, W_GENE0 = 9, 10, 11, 12
MAX_DRAWS = 9


def theta_bounds(n_cs: int):
    """Box of the continuous encoding of theta = (F, CR, bl, br, dn, cs).

    F and CR lie in [0, 1] (Sec. III-A1).  The categorical parameters are
    encoded on [1, c_max + 1] and decoded by floor (Alg. 3, decode step), with
    c_max = 4 for bl, br (rand, best, pbest, current) and dn (1..4), and
    c_max = n_cs for cs (bin, exp[, arith]).
    """
    lo = np.array([0, 0, 1, 1, 1, 1], dtype=np.float32)
    hi = np.array([1, 1, 5, 5, 5, 1 + n_cs], dtype=np.float32)
    return lo, hi


def clip_theta(theta, n_cs: int):
    lo, hi = theta_bounds(n_cs)
    return np.minimum(np.maximum(np.asarray(theta, np.float32), lo), hi)


def decode(theta, n_cs: int):
    """Alg. 3 decode: F = u1, CR = u2, bl/br/dn/cs = floor(u3..u6).

    The upper end of the box would floor to c_max + 1; it is mapped to c_max.
    Values are clipped to the box first.
    """
    t = clip_theta(theta, n_cs)
    cmax = np.array([4, 4, 4, n_cs])
    cat = np.minimum(np.floor(t[..., 2:6].astype(np.float64)).astype(np.int64), cmax)
    return {"F": t[..., 0].astype(np.float32), "CR": t[..., 1].astype(np.float32),
            "bl": cat[..., 0], "br": cat[..., 1], "dn": cat[..., 2], "cs": cat[..., 3]}


def top_count(N: int) -> int:
    """k_p = max(1, ceil(N * 10 / 100)) -- the top-p set for pbest."""
    return max(1, (N * 10 + 99) // 100)


def order_key(f):
    f = np.asarray(f, dtype=np.float64)
    return np.where(np.isnan(f), np.inf, f)


def ranking(fit):
    """Indices sorted by (fitness, index) ascending; NaN counts as +inf."""
    idx = np.arange(len(fit))
    return np.lexsort((idx, order_key(fit)))


def sample_distinct(t, N):
    """Index sampling without rejection.

    t: int [n, m] with 0 <= t[i, k] < N - 1 - k.  Row i is target i.  Draw k is
    the t[i, k]-th smallest element (0-based) of {0..N-1} minus {i} minus the
    earlier draws of row i.  Returns int [n, m].
    """
    n, m = t.shape
    rows = np.arange(n)
    taken = np.zeros((n, N), dtype=bool)
    taken[rows, rows] = True
    out = np.empty((n, m), dtype=np.int64)
    for k in range(m):
        rank = np.cumsum(~taken, axis=1)             # free elements in [0..j]
        pick = np.argmax(rank > t[:, k:k + 1], axis=1)
        out[:, k] = pick
        taken[rows, pick] = True
    return out


def n_draws(bl: int, br: int, dn: int) -> int:
    """Random indices one trial needs: the shared 'rand' base (if bl or br is
    rand; one index even when both are) plus two per difference vector."""
    return int(RAND in (bl, br)) + 2 * dn


def init_population(N, D, seed, stream, lb, ub):
    """Uniform initial population in the box (Alg. 2, initialisation).

    x = lb + (ub - lb) * u0 with u0 = (w >> 8) 2^-24 in [0, 1), computed in
    float64 and rounded once to float32.  lb, ub may be scalars or [D] arrays.
    """
    w = philox.words(seed, np.arange(N), philox.INIT_PHASE, stream, D)
    u0 = philox.unit_closed_open64(w)
    lb64 = np.asarray(lb, dtype=np.float32).astype(np.float64)
    ub64 = np.asarray(ub, dtype=np.float32).astype(np.float64)
    return (lb64 + (ub64 - lb64) * u0).astype(np.float32)


def make_trials(pop, fit, th, g, seed, stream, lb, ub):
    """Mutation + crossover + clip for every target of one generation.

    pop: float32 [N, D]; fit: [N]; th: decoded theta of this run (scalars).
    Returns (u float32 [N, D], desc dict of per-target int/float arrays).
    """
    N, D = pop.shape
    F = np.float32(th["F"])
    CR = np.float32(th["CR"])
    bl, br, dn, cs = int(th["bl"]), int(th["br"]), int(th["dn"]), int(th["cs"])
    m = n_draws(bl, br, dn)
    if N < m + 1:
        raise ValueError(f"population {N} too small for {m} distinct indices")
    ids = np.arange(N)
    w = philox.words(seed, ids, g, stream, W_GENE0 + D)

    order = ranking(fit)
    kp = top_count(N)

    bound = np.array([N - 1 - k for k in range(m)])
    t = philox.lemire(w[:, :m], bound[None, :]) if m else np.zeros((N, 0), np.int64)
    draws = sample_distinct(t, N)
    off = 1 if RAND in (bl, br) else 0
    r0 = draws[:, 0] if off else np.full(N, -1)
    pairs = draws[:, off:].reshape(N, dn, 2)

    pb_rank = philox.lemire(w[:, W_PBEST], kp)

    def resolve(code):
        if code == RAND:
            return r0
        if code == BEST:
            return np.full(N, order[0])
        if code == PBEST:
            return order[pb_rank]
        return ids

    i_bl, i_br = resolve(bl), resolve(br)

    # Eq. (12) in float32, one rounding per operation, fixed order.
    x_bl = pop[i_bl]
    if bl != br:
        base = x_bl + F * (pop[i_br] - x_bl)
    else:
        base = x_bl
    d = pop[pairs[:, 0, 0]] - pop[pairs[:, 0, 1]]
    for k in range(1, dn):
        d = d + (pop[pairs[:, k, 0]] - pop[pairs[:, k, 1]])
    v = base + F * d

    jn = philox.lemire(w[:, W_JRAND], D)
    L = np.full(N, -1)
    K = np.full(N, np.nan, dtype=np.float32)
    if cs == ARITH:
        # Eq. (10): u = x + K (v - x), K in (0, 1]; CR is not used.
        K = philox.unit_open_closed(w[:, W_K])
        u = pop + K[:, None] * (v - pop)
        mask = np.ones((N, D), dtype=bool)
    else:
        r = philox.unit_open_closed(w[:, W_GENE0:W_GENE0 + D])
        if cs == BIN:
            # Eq. (8): gene from v iff r_j <= CR or j == j_rand.
            mask = (r <= CR) | (np.arange(D)[None, :] == jn[:, None])
        else:
            # Eq. (9): L ~ censored geometric (P(L >= k) = CR^(k-1), L <= D);
            # the t-th continuation test uses uniform t.  Genes n..n+L-1 mod D.
            mask = np.zeros((N, D), dtype=bool)
            for i in range(N):
                Li = 1
                while Li < D and r[i, Li - 1] <= CR:
                    Li += 1
                L[i] = Li
                mask[i, (jn[i] + np.arange(Li)) % D] = True
        u = np.where(mask, v, pop)
    u = np.minimum(np.maximum(u, np.asarray(lb, np.float32)), np.asarray(ub, np.float32))
    u = u.astype(np.float32)

    desc = {"i_bl": i_bl, "i_br": i_br, "r0": r0, "pairs": pairs, "pbest_rank": pb_rank,
            "jn": jn, "L": L, "K": K, "mask": mask, "best": order[0], "kp": kp}
    return u, desc


def select(pop, fit, u, fu):
    """Greedy selection (Alg. 1): u_i replaces x_i iff f(u_i) <= f(x_i).

    A NaN trial is never accepted; a NaN target counts as +inf.
    """
    fu = np.asarray(fu)
    accept = ~np.isnan(fu) & (order_key(fu) <= order_key(fit))
    new_pop = np.where(accept[:, None], u, pop).astype(np.float32)
    new_fit = np.where(accept, fu, fit)
    return new_pop, new_fit, accept


def as_decision(f64, decide: str):
    """Fitness values in the precision selection decisions are taken in."""
    if decide == "f32":
        return np.asarray(f64, dtype=np.float64).astype(np.float32)
    return np.asarray(f64, dtype=np.float64)


def step(pop, fit, th, g, seed, stream, lb, ub, prob, decide="f32", fitness_override=None):
    """One PDE generation (Alg. 2 loop body).  Returns a dict of everything.

    ``fitness_override`` (one value per trial) replaces the trials' fitness in
    the selection step: given another implementation's state before the
    generation and its trial fitness, the selection rule of Alg. 1 is then
    applied to exactly the values that implementation decided on, so its
    decisions can be compared one by one, ties and near-ties included.  The
    float64 fitness of the trials is still computed and returned as ``fu64``.
    """
    u, desc = make_trials(pop, fit, th, g, seed, stream, lb, ub)
    fu64 = evaluate(u, prob)
    if fitness_override is None:
        fu = as_decision(fu64, decide)
    else:
        fu = np.asarray(fitness_override).reshape(fu64.shape)
        fu = fu.astype(np.float32) if decide == "f32" else fu.astype(np.float64)
    new_pop, new_fit, accept = select(pop, fit, u, fu)
    return {"u": u, "fu64": fu64, "fu": fu, "desc": desc, "pop": new_pop, "fit": new_fit,
            "accept": accept}


def run_executor(N, D, th, G, seed, stream, lb, ub, prob, decide="f32", history=False):
    """One executor run (Alg. 2): init, evaluate, G generations.

    Returns y* = the best fitness seen (float64 value of the best individual
    under the decision ordering), the final population and fitness.
    """
    pop = init_population(N, D, seed, stream, lb, ub)
    f64 = evaluate(pop, prob)
    fit = as_decision(f64, decide)
    best_seen = float(np.min(order_key(fit)))
    hist = []
    for g in range(G):
        s = step(pop, fit, th, g, seed, stream, lb, ub, prob, decide)
        pop, fit = s["pop"], s["fit"]
        best_seen = min(best_seen, float(np.min(order_key(fit))))
        if history:
            hist.append(s)
    b = int(ranking(fit)[0])
    y_star = float(evaluate(pop[b], prob))
    return {"y": y_star, "best_index": b, "best_x": pop[b].copy(), "pop": pop, "fit": fit,
            "best_seen": best_seen, "history": hist}
