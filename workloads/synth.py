"""Seeded synthetic workloads shaped like the paper's experiments.

The paper measures on the CEC2022 suite and on Brax control tasks, neither of
which is available here.  These generators stand in for them with textbook
shifted-rotated functions and a seeded linear control system of the same
dimensions (10-D/20-D, population 100, 1000 inner generations; a 5702-weight
tanh policy).  Every array is produced by ``numpy.random.default_rng`` seeded
from a ``SeedSequence`` so both the oracle and the GPU path see identical
inputs.

Nothing here implements the method: the generators only produce problem data
(o, R, permutations, A, B, x0) and workload shapes (population sizes, streams,
sampled hyperparameter vectors).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

KINDS = ("rastrigin", "rosenbrock", "ackley", "elliptic", "schwefel", "hybrid", "lqr_mlp")

# Integer tags used only to seed per-instance generators.
_KIND_TAG = {k: i + 1 for i, k in enumerate(KINDS)}

LQR_OBS = 17
LQR_ACT = 6
LQR_HIDDEN = (64, 64)
# Policy shapes (obs, act) of the three control tasks of Table VII, hidden 32 x 32
TABLE7_HIDDEN = (32, 32)
TABLE7_TASKS = (("hopper", 11, 3), ("swimmer", 8, 2), ("reacher", 11, 2))
LQR_STEPS = 200
LQR_CTRL_WEIGHT = 0.01
# Weight box of the control workload: 1/sqrt(obs) rounded to 0.25 (the usual
# fan-in scale of a first layer).  With [-1, 1] most random policies make the
# closed loop chaotic, and their cost is then not determined by float64
# arithmetic (it moves by percent against extended precision).
CTRL_BOX = 0.25


def mlp_param_count(n_in: int, hidden, n_out: int) -> int:
    """Number of weights plus biases of a fully connected MLP."""
    sizes = [n_in, *hidden, n_out]
    return sum(sizes[k] * sizes[k + 1] + sizes[k + 1] for k in range(len(sizes) - 1))


@dataclass
class Problem:
    kind: str
    D: int
    bias: float = 100.0
    o: Optional[np.ndarray] = None          # f32[D] shift
    R: Optional[np.ndarray] = None          # f32[D, D] orthogonal rotation (row-major)
    perm: Optional[np.ndarray] = None       # u32[D] hybrid permutation
    split: Optional[tuple] = None           # hybrid block sizes (Schwefel, Rastrigin, elliptic)
    cond: float = 1e6                       # elliptic condition number
    # control-shaped workload
    A: Optional[np.ndarray] = None          # f32[obs, obs]
    B: Optional[np.ndarray] = None          # f32[obs, act]
    x0: Optional[np.ndarray] = None         # f32[E, obs] initial states (E rollouts)
    hidden: tuple = LQR_HIDDEN
    steps: int = LQR_STEPS
    ctrl_weight: float = LQR_CTRL_WEIGHT


@dataclass
class Workload:
    name: str
    seed: int
    lb: float
    ub: float
    n_cs: int
    N: np.ndarray                 # u32[runs] population sizes
    problem: np.ndarray           # u32[runs] index into problems
    stream: np.ndarray            # u32[runs] random stream per run
    problems: List[Problem]
    G: int                        # inner generations per executor run
    theta: Optional[np.ndarray] = None   # f32[runs, 6] when no outer loop drives the runs
    outer: Optional[dict] = None         # {"P", "gens", "power_up", "F", "CR"} for MetaDE runs
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_runs(self) -> int:
        return int(self.N.shape[0])

    def D_of(self, r: int) -> int:
        return int(self.problems[int(self.problem[r])].D)

    def evals_per_pass(self) -> int:
        """Trial evaluations of one full pass (inner generations x populations)."""
        ns = self.N.astype(np.int64)
        if self.outer is None:
            return int(ns.sum() * self.G)
        gens = self.outer["gens"]
        pu = self.outer.get("power_up", 5)
        total_g = (gens - 1) * self.G + pu * self.G if gens > 0 else 0
        return int(ns.sum() * total_g)


def theta_box(n_cs: int):
    """Sampling box of the hyperparameter vector (F, CR, bl, br, dn, cs)."""
    lo = np.array([0.0, 0.0, 1.0, 1.0, 1.0, 1.0], dtype=np.float32)
    hi = np.array([1.0, 1.0, 5.0, 5.0, 5.0, 1.0 + n_cs], dtype=np.float32)
    return lo, hi


def _rng(*words) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(w) & 0xFFFFFFFF for w in words]))


def make_rotation(rng: np.random.Generator, D: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix from the QR factorisation of a Gaussian matrix."""
    g = rng.standard_normal((D, D))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    return np.ascontiguousarray(q.astype(np.float32))


def make_problem(kind: str, D: int, seed: int, run: int, identity_rotation: bool = False,
                 bias: float = 100.0, n_rollouts: int = 1, obs: int = LQR_OBS,
                 act: int = LQR_ACT, steps: int = LQR_STEPS, hidden=LQR_HIDDEN) -> Problem:
    """One seeded instance of a shifted-rotated function (or the control system:
    A = 0.95 G / rho(G) with G Gaussian, B Gaussian / sqrt(obs), x0 ~ N(0, I))."""
    if kind not in KINDS:
        raise ValueError(f"unknown problem kind {kind!r}")
    rng = _rng(seed, run, _KIND_TAG[kind])
    if kind == "lqr_mlp":
        g = rng.standard_normal((obs, obs))
        rho = np.max(np.abs(np.linalg.eigvals(g)))
        A = (0.95 * g / rho).astype(np.float32)
        B = (rng.standard_normal((obs, act)) / np.sqrt(obs)).astype(np.float32)
        x0 = rng.standard_normal((n_rollouts, obs)).astype(np.float32)
        Dm = mlp_param_count(obs, hidden, act)
        if D != Dm:
            raise ValueError(f"control workload has D={Dm}, got {D}")
        return Problem(kind=kind, D=D, bias=0.0, A=A, B=B, x0=x0, steps=steps,
                       hidden=tuple(hidden))
    o = rng.uniform(-80.0, 80.0, size=D).astype(np.float32)
    R = np.eye(D, dtype=np.float32) if identity_rotation else make_rotation(rng, D)
    p = Problem(kind=kind, D=D, bias=bias, o=o, R=R)
    if kind == "hybrid":
        p.perm = rng.permutation(D).astype(np.uint32)
        n1 = int(round(0.3 * D))
        n2 = (D - n1 + 1) // 2
        p.split = (n1, n2, D - n1 - n2)
    return p


def _sample_theta(rng: np.random.Generator, runs: int, n_cs: int) -> np.ndarray:
    lo, hi = theta_box(n_cs)
    u = rng.random((runs, 6))
    return (lo[None, :].astype(np.float64) + (hi - lo)[None, :] * u).astype(np.float32)


def workload_c1() -> Workload:
    """Small MetaDE: outer population 8, 2 outer generations, inner N=32, D=10,
    50 generations, shifted-rotated Rastrigin, random seed 0, one-shot stream 0."""
    seed, P = 0, 8
    prob = make_problem("rastrigin", 10, seed, 0)
    return Workload(name="c1_small_metade", seed=seed, lb=-100.0, ub=100.0, n_cs=2,
                    N=np.full(P, 32, np.uint32), problem=np.zeros(P, np.uint32),
                    stream=np.zeros(P, np.uint32), problems=[prob], G=50,
                    outer={"P": P, "gens": 2, "power_up": 5, "F": 0.5, "CR": 0.9})


def workload_c2(runs: int = 256) -> Workload:
    """Uneven batch: 256 runs, N ~ U{20..200}, D ~ U{10,20}, four function kinds,
    per-run instances, hyperparameters sampled from the meta-space, 200 generations."""
    seed = 1
    rng = _rng(seed, 0xC2)
    N = rng.integers(20, 201, size=runs).astype(np.uint32)
    D = rng.choice(np.array([10, 20]), size=runs)
    kinds = ("rastrigin", "rosenbrock", "ackley", "elliptic")
    kind_idx = rng.integers(0, 4, size=runs)
    theta = _sample_theta(rng, runs, 2)
    problems = [make_problem(kinds[int(kind_idx[r])], int(D[r]), seed, r) for r in range(runs)]
    return Workload(name="c2_uneven_batch", seed=seed, lb=-100.0, ub=100.0, n_cs=2, N=N,
                    problem=np.arange(runs, dtype=np.uint32), stream=np.arange(runs, dtype=np.uint32),
                    problems=problems, G=200, theta=theta)


def workload_c3(P: int = 64, gens: int = 10, G: int = 1000) -> Workload:
    """Full MetaDE at D=20: outer population 64, 10 outer generations (last one
    powered up 5x), inner N=100, 1000 generations, seeded hybrid function."""
    seed = 2
    prob = make_problem("hybrid", 20, seed, 0)
    return Workload(name="c3_metade_d20", seed=seed, lb=-100.0, ub=100.0, n_cs=2,
                    N=np.full(P, 100, np.uint32), problem=np.zeros(P, np.uint32),
                    stream=np.zeros(P, np.uint32), problems=[prob], G=G,
                    outer={"P": P, "gens": gens, "power_up": 5, "F": 0.5, "CR": 0.9})


def workload_paper(D: int = 20, P: int = 100, gens: int = 10, G: int = 1000) -> Workload:
    """MetaDE at the paper's own scale (Sec. IV-A1): evolver population 100,
    executors with N=100 and 1000 generations, the last outer generation
    powered up 5x, and the full meta-space with the three crossover schemes
    (bin, exp, arith: 4 x 4 x 4 x 3 = 192 strategies).  Seeded hybrid
    function at D=20 standing in for the paper's benchmark suite."""
    seed = 5
    prob = make_problem("hybrid", D, seed, 0)
    return Workload(name=f"paper_scale_d{D}", seed=seed, lb=-100.0, ub=100.0, n_cs=3,
                    N=np.full(P, 100, np.uint32), problem=np.zeros(P, np.uint32),
                    stream=np.zeros(P, np.uint32), problems=[prob], G=G,
                    outer={"P": P, "gens": gens, "power_up": 5, "F": 0.5, "CR": 0.9})


def workload_c4(runs: int = 128, N: int = 256, D: int = 100, G: int = 500) -> Workload:
    """Precision stress at D=100: 128 runs x N=256, 500 generations, half elliptic
    (cond 1e6), half Rastrigin, each with its own shift and dense rotation."""
    seed = 3
    rng = _rng(seed, 0xC4)
    theta = _sample_theta(rng, runs, 2)
    half = runs // 2
    problems = [make_problem("elliptic" if r < half else "rastrigin", D, seed, r) for r in range(runs)]
    return Workload(name="c4_precision_d100", seed=seed, lb=-100.0, ub=100.0, n_cs=2,
                    N=np.full(runs, N, np.uint32), problem=np.arange(runs, dtype=np.uint32),
                    stream=np.arange(runs, dtype=np.uint32), problems=problems, G=G, theta=theta)


def workload_c5(runs: int = 16, N: int = 256, G: int = 100, n_rollouts: int = 1) -> Workload:
    """Control-shaped workload: tanh policy 17->64->64->6 (5702 weights) scored by a
    200-step rollout of a seeded stable linear system; 16 runs x N=256, 100 generations."""
    seed = 4
    rng = _rng(seed, 0xC5)
    theta = _sample_theta(rng, runs, 2)
    D = mlp_param_count(LQR_OBS, LQR_HIDDEN, LQR_ACT)
    problems = [make_problem("lqr_mlp", D, seed, r, n_rollouts=n_rollouts) for r in range(runs)]
    return Workload(name="c5_control_mlp", seed=seed, lb=-CTRL_BOX, ub=CTRL_BOX, n_cs=2,
                    N=np.full(runs, N, np.uint32), problem=np.arange(runs, dtype=np.uint32),
                    stream=np.arange(runs, dtype=np.uint32), problems=problems, G=G, theta=theta)


def workload_c5e16(G: int = 10) -> Workload:
    """The control workload with 16 rollouts per policy (16 initial states per
    plant, J averaged): every layer of a step becomes a product with 16 columns.
    16 runs x N=256 policies 17->64->64->6, 10 generations."""
    wl = workload_c5(G=G, n_rollouts=16)
    wl.name = "c5e16_control_mlp_16_rollouts"
    return wl


def workload_t7(runs_per_task: int = 32, N: int = 100, G: int = 50) -> Workload:
    """The policy MLPs of Table VII (hopper 11->32->32->3, 1539 weights; swimmer
    8->32->32->2, 1410; reacher 11->32->32->2, 1506), each scored by a 200-step
    rollout of a seeded stable linear plant of the task's observation / action
    sizes (standing in for the robot simulator).  32 executors per task with the
    control experiment's population 100 and 50 generations (Sec. IV-D)."""
    seed = 7
    rng = _rng(seed, 0x77)
    runs = runs_per_task * len(TABLE7_TASKS)
    theta = _sample_theta(rng, runs, 2)
    problems = []
    for r in range(runs):
        _, obs, act = TABLE7_TASKS[r // runs_per_task]
        D = mlp_param_count(obs, TABLE7_HIDDEN, act)
        problems.append(make_problem("lqr_mlp", D, seed, r, obs=obs, act=act,
                                     hidden=TABLE7_HIDDEN))
    return Workload(name="t7_control_mlp", seed=seed, lb=-CTRL_BOX, ub=CTRL_BOX, n_cs=2,
                    N=np.full(runs, N, np.uint32), problem=np.arange(runs, dtype=np.uint32),
                    stream=np.arange(runs, dtype=np.uint32), problems=problems, G=G, theta=theta)


def small_batch(seed: int, kinds, Ns, Ds, G: int = 3, n_cs: int = 2, theta=None,
                identity_rotation: bool = False, lb: float = -100.0, ub: float = 100.0,
                streams=None) -> Workload:
    """A small batch of independent runs for parity tests: one instance per run."""
    runs = len(Ns)
    rng = _rng(seed, 0x5B)
    if theta is None:
        theta = _sample_theta(rng, runs, n_cs)
    problems = [make_problem(kinds[r % len(kinds)], int(Ds[r]), seed, r,
                             identity_rotation=identity_rotation) for r in range(runs)]
    stream = np.arange(runs, dtype=np.uint32) if streams is None else np.asarray(streams, np.uint32)
    return Workload(name=f"small_{seed}", seed=seed, lb=lb, ub=ub, n_cs=n_cs,
                    N=np.asarray(Ns, np.uint32), problem=np.arange(runs, dtype=np.uint32),
                    stream=stream, problems=problems, G=G, theta=np.asarray(theta, np.float32))


def control_batch(seed: int, Ns, obs: int = LQR_OBS, act: int = LQR_ACT, steps: int = LQR_STEPS,
                  n_rollouts: int = 1, theta=None, n_cs: int = 2, G: int = 3,
                  hidden=LQR_HIDDEN, shapes=None) -> Workload:
    """A small batch of control runs (one plant per run) for parity tests.  ``shapes``
    gives each run's (obs, act) in place of the common obs / act."""
    runs = len(Ns)
    rng = _rng(seed, 0xC7)
    if theta is None:
        theta = _sample_theta(rng, runs, n_cs)
    if shapes is None:
        shapes = [(obs, act)] * runs
    problems = [make_problem("lqr_mlp", mlp_param_count(o, hidden, a), seed, r,
                             n_rollouts=n_rollouts, obs=o, act=a, steps=steps, hidden=hidden)
                for r, (o, a) in enumerate(shapes)]
    return Workload(name=f"control_{seed}", seed=seed, lb=-CTRL_BOX, ub=CTRL_BOX, n_cs=n_cs,
                    N=np.asarray(Ns, np.uint32), problem=np.arange(runs, dtype=np.uint32),
                    stream=np.arange(runs, dtype=np.uint32), problems=problems, G=G,
                    theta=np.asarray(theta, np.float32))


def workload_by_name(name: str) -> Workload:
    table = {"c1": workload_c1, "c2": workload_c2, "c3": workload_c3, "c4": workload_c4,
             "c5": workload_c5, "paper": workload_paper, "t7": workload_t7,
             "c5e16": workload_c5e16}
    return table[name]()
