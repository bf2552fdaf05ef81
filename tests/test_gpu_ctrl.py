"""GPU parity of the control workload: tanh policies scored by a rollout of a
linear system (the paper's neural-control setting, Sec. IV-D, on a synthetic
plant), against the oracle's trajectory on the same seeded inputs.

Trial vectors, draws, crossover and selection are compared bit for bit; the
float32 fitness (a float64 rollout rounded once) within the relative
tolerance of the float64 oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import pde
from oracle.fitness import evaluate
from paritylib import FIT_RTOL, rel_err, resync_parity, trajectory_parity

pytestmark = pytest.mark.gpu


def _batch(wl):
    from paper_2502_10470_amd import Batch
    return Batch(wl)


def _strategy_grid(runs, n_cs, seed):
    """Theta rows covering every base pair, difference count and crossover scheme."""
    rng = np.random.default_rng(seed)
    th = np.empty((runs, 6), np.float32)
    for r in range(runs):
        th[r, 0] = rng.uniform(0.05, 1.0)
        th[r, 1] = rng.uniform(0.0, 1.0)
        th[r, 2] = 1 + (r % 4) + 0.5
        th[r, 3] = 1 + ((r // 4) % 4) + 0.5
        th[r, 4] = 1 + ((r + r // 4) % 4) + 0.5
        th[r, 5] = 1 + (r % n_cs) + 0.5
    return th


@pytest.mark.parametrize("obs,act,steps,n_roll,n_cs", [
    (5, 3, 20, 2, 3),     # odd D (4739): unaligned rows, several rollouts, arithmetic crossover
    (17, 6, 200, 1, 2),   # the policy and horizon of the full workload
    (20, 8, 12, 1, 3),    # largest observation / action sizes
    (1, 1, 30, 3, 2),     # smallest
])
def test_control_follows_oracle(obs, act, steps, n_roll, n_cs):
    Ns = [10, 17, 33, 64, 65, 40, 12, 20]
    th = _strategy_grid(len(Ns), n_cs, seed=obs * 100 + act)
    wl = W.control_batch(11 + obs, Ns, obs=obs, act=act, steps=steps, n_rollouts=n_roll,
                         theta=th, n_cs=n_cs)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=3)
    print(f"obs={obs} act={act}: compared {out['compared']} diverged {out['diverged']} (undetermined {out['ill']}) "
          f"max fitness rel err {out['max_fit_rel']:.3g}")
    assert out["compared"] >= 2 * len(Ns)


def test_control_full_size_two_generations():
    """16 runs x N=256, D=5702, 200-step horizon: two traced generations."""
    wl = W.workload_c5()
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=2)
    print(f"c5: compared {out['compared']} near ties {out['near_ties']} "
          f"max fitness rel err {out['max_fit_rel']:.3g}")
    assert out["compared"] == 32


def test_control_resync_after_50_generations():
    """The full control workload after 50 generations in one untraced sequence
    (graph replays): one traced generation from the library's own state,
    compared with the oracle step on that state for four of the runs --
    trials, draws and every decision."""
    wl = W.workload_c5()
    b = _batch(wl)
    b.inner_step(50)
    out = resync_parity(b, wl, 50, wl.theta, runs=[0, 5, 10, 15])
    print(out, flush=True)
    assert out["compared"] == 4 and out["trials"] == 4 * 256


def test_control_best_record_float64():
    wl = W.control_batch(3, [24, 30, 16], steps=50, G=4)
    b = _batch(wl)
    b.inner_step(4)
    y = b.get_best()
    pop, fit = b.host_state()
    bx = b.best_x.cpu().numpy()
    for r in range(wl.n_runs):
        f = b.run_fit(fit, r)
        i = int(np.lexsort((np.arange(len(f)), pde.order_key(f)))[0])
        x = b.run_pop(pop, r)[i]
        assert np.array_equal(b.run_bx(bx, r), x)
        ref = float(evaluate(x, wl.problems[r]))
        assert abs(y[r] - ref) <= 1e-9 * abs(ref), (r, y[r], ref)
        assert abs(float(f[i]) - ref) <= FIT_RTOL * abs(ref)


def test_control_mixed_with_shifted_runs():
    """Control and shifted-rotated runs in one context, sharing the search box."""
    ctrl = W.control_batch(8, [20, 33], obs=4, act=2, steps=25)
    rast = W.make_problem("rastrigin", 10, 8, 5)
    ell = W.make_problem("elliptic", 100, 8, 6)
    probs = [rast, ctrl.problems[0], ell, ctrl.problems[1]]
    theta = np.concatenate([ctrl.theta, ctrl.theta], 0)
    wl = W.Workload(name="mixed", seed=8, lb=-0.25, ub=0.25, n_cs=2,
                    N=np.array([32, 20, 40, 33], np.uint32), problem=np.arange(4, dtype=np.uint32),
                    stream=np.arange(4, dtype=np.uint32), problems=probs, G=3, theta=theta)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=3)
    assert out["compared"] >= 8


def test_control_deterministic_and_resumable():
    wl = W.control_batch(9, [16, 24], steps=30)
    b1 = _batch(wl)
    b1.inner_step(2)
    blob = b1.get_state()
    b1.inner_step(2)
    p1, f1 = b1.host_state()
    b2 = _batch(wl)
    b2.set_state(blob)
    b2.inner_step(2)
    p2, f2 = b2.host_state()
    assert np.array_equal(p1, p2) and np.array_equal(f1, f2)


def test_control_selection_invariants():
    """Per-individual fitness never increases; trials stay in the box."""
    wl = W.control_batch(10, [32, 48], steps=40)
    b = _batch(wl)
    _, f0 = b.host_state()
    for _ in range(5):
        b.inner_step(1)
        pop, f = b.host_state()
        assert np.all(f <= f0)
        assert pop.min() >= wl.lb and pop.max() <= wl.ub
        f0 = f


@pytest.mark.parametrize("n_roll", [2, 16])
def test_control_graph_replays_match_direct_launches(n_roll):
    """The control generation loop replayed from HIP graphs gives the same
    populations as direct launches, call after call: replays of one graph at
    later starting generations, a second sequence length, host work and
    synchronisations in between, and a checkpoint restored mid-way (vector
    evaluation with 2 rollouts, matrix-core evaluation with 16)."""
    from paper_2502_10470_amd import Batch
    wl = W.control_batch(12, [24, 40, 17], obs=6, act=2, steps=30, n_rollouts=n_roll)
    bg = Batch(wl, graph=True)
    bd = Batch(wl, graph=False)
    blob = None
    for call, n in enumerate([3, 3, 2, 3, 3]):
        bg.inner_step(n)
        bd.inner_step(n)
        pg, fg = bg.host_state()
        pd, fd = bd.host_state()
        assert np.array_equal(pg, pd) and np.array_equal(fg, fd), f"call {call} (n={n})"
        if call == 1:
            blob = bg.get_state()
    # restore the checkpoint taken after two calls into the graph batch and
    # replay: it must follow the direct-launch trajectory from that point
    bg.set_state(blob)
    bd2 = Batch(wl, graph=False)
    bd2.set_state(blob)
    for n in (3, 2):
        bg.inner_step(n)
        bd2.inner_step(n)
        pg, fg = bg.host_state()
        pd, fd = bd2.host_state()
        assert np.array_equal(pg, pd) and np.array_equal(fg, fd)


@pytest.mark.parametrize("shapes,steps,n_roll,n_cs", [
    # the three policies of Table VII (hidden 32 x 32: 1539, 1410, 1506 weights)
    ([(11, 3), (8, 2), (11, 2)] * 3, 200, 1, 2),
    # odd D (1153), several rollouts, arithmetic crossover; largest obs / act
    ([(1, 1), (20, 8), (1, 1), (20, 8)], 15, 2, 3),
])
def test_control_hidden32_follows_oracle(shapes, steps, n_roll, n_cs):
    Ns = [10, 17, 33, 64, 65, 40, 12, 20, 100][:len(shapes)]
    th = _strategy_grid(len(Ns), n_cs, seed=len(shapes) * 10 + steps)
    wl = W.control_batch(21 + steps, Ns, shapes=shapes, steps=steps, n_rollouts=n_roll,
                         theta=th, n_cs=n_cs, hidden=W.TABLE7_HIDDEN)
    assert all(p.hidden == (32, 32) for p in wl.problems)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=3)
    print(f"hidden 32 {shapes[:3]}: compared {out['compared']} diverged {out['diverged']} "
          f"(undetermined {out['ill']}) max fitness rel err {out['max_fit_rel']:.3g}")
    assert out["compared"] >= 2 * len(Ns)


def test_control_table7_workload_two_generations():
    """96 executors (32 per Table VII policy) x N=100, 200-step horizon: two traced
    generations at the full size."""
    wl = W.workload_t7()
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=2)
    print(f"t7: compared {out['compared']} diverged {out['diverged']} "
          f"max fitness rel err {out['max_fit_rel']:.3g}")
    assert out["compared"] >= 96


def test_control_hidden32_best_record_float64():
    wl = W.control_batch(5, [24, 30, 16], shapes=[(11, 3), (8, 2), (11, 2)], steps=50, G=4,
                         hidden=W.TABLE7_HIDDEN)
    b = _batch(wl)
    b.inner_step(4)
    y = b.get_best()
    pop, fit = b.host_state()
    bx = b.best_x.cpu().numpy()
    for r in range(wl.n_runs):
        f = b.run_fit(fit, r)
        i = int(np.lexsort((np.arange(len(f)), pde.order_key(f)))[0])
        x = b.run_pop(pop, r)[i]
        assert np.array_equal(b.run_bx(bx, r), x)
        ref = float(evaluate(x, wl.problems[r]))
        assert abs(y[r] - ref) <= 1e-9 * abs(ref), (r, y[r], ref)
        assert abs(float(f[i]) - ref) <= FIT_RTOL * abs(ref)


@pytest.mark.parametrize("hidden,shapes,steps,n_roll,n_cs", [
    ((64, 64), [(17, 6)] * 4, 30, 16, 2),                 # C5's policy, 16 rollouts
    ((64, 64), [(5, 3)] * 4, 12, 32, 3),                  # odd D, two groups of 16 rollouts
    ((32, 32), [(11, 3), (8, 2), (11, 2), (20, 8)], 25, 16, 2),  # Table VII, largest obs / act
    ((32, 32), [(1, 1)] * 3, 10, 16, 3),                  # smallest
])
def test_control_16_rollouts_matrix_cores_follow_oracle(hidden, shapes, steps, n_roll, n_cs):
    """Policies scored over a multiple of 16 rollouts go to the matrix-core
    evaluation (one policy per wavefront); trajectories follow the oracle."""
    Ns = [10, 17, 33, 24][:len(shapes)]
    th = _strategy_grid(len(Ns), n_cs, seed=steps * 7 + n_roll)
    wl = W.control_batch(31 + steps, Ns, shapes=shapes, steps=steps, n_rollouts=n_roll,
                         theta=th, n_cs=n_cs, hidden=hidden)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=3)
    print(f"E={n_roll} hidden {hidden[0]}: compared {out['compared']} diverged {out['diverged']} "
          f"(undetermined {out['ill']}) max fitness rel err {out['max_fit_rel']:.3g}")
    assert out["compared"] >= 2 * len(Ns)


def test_control_16_rollouts_best_record_and_resume():
    wl = W.control_batch(6, [20, 12], steps=15, n_rollouts=16, G=3)
    b1 = _batch(wl)
    b1.inner_step(2)
    blob = b1.get_state()
    b1.inner_step(2)
    p1, f1 = b1.host_state()
    y = b1.get_best()
    bx = b1.best_x.cpu().numpy()
    for r in range(wl.n_runs):
        f = b1.run_fit(f1, r)
        i = int(np.lexsort((np.arange(len(f)), pde.order_key(f)))[0])
        x = b1.run_pop(p1, r)[i]
        assert np.array_equal(b1.run_bx(bx, r), x)
        ref = float(evaluate(x, wl.problems[r]))
        assert abs(y[r] - ref) <= 1e-9 * abs(ref), (r, y[r], ref)
        assert abs(float(f[i]) - ref) <= FIT_RTOL * abs(ref)
    b2 = _batch(wl)
    b2.set_state(blob)
    b2.inner_step(2)
    p2, f2 = b2.host_state()
    assert np.array_equal(p1, p2) and np.array_equal(f1, f2)


@pytest.mark.parametrize("hidden,n_roll", [((64, 64), 1), ((32, 32), 1), ((64, 64), 16)])
def test_control_largest_population_and_sizes(hidden, n_roll):
    """N = 1024 (the control maximum) with the largest observation / action sizes,
    on the vector evaluation (one rollout) and the matrix-core one (16)."""
    th = _strategy_grid(2, 3, seed=77)
    wl = W.control_batch(71, [1024, 10], shapes=[(20, 8), (20, 8)], steps=4, n_rollouts=n_roll,
                         theta=th, n_cs=3, hidden=hidden)
    b = _batch(wl)
    out = trajectory_parity(b, wl, G=2)
    print(f"N=1024 hidden {hidden[0]} E={n_roll}: compared {out['compared']} "
          f"diverged {out['diverged']} max fitness rel err {out['max_fit_rel']:.3g}")
    assert out["compared"] >= 2
