"""Pins of the oracle's objective functions: closed-form optima, textbook
reductions, rotation orientation, and the control workload's closed form."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fitness
from oracle.fitness import evaluate

KINDS = ["rastrigin", "elliptic", "ackley", "rosenbrock", "schwefel", "hybrid"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("D", [2, 10, 20])
def test_optimum_is_bias_at_shift(kind, D):
    p = W.make_problem(kind, D, 0, 3)
    f = evaluate(p.o[None, :], p)[0]
    assert abs(f - p.bias) < 1e-9 * max(1.0, abs(p.bias))


def _identity(kind, D, seed=1):
    return W.make_problem(kind, D, seed, 0, identity_rotation=True)


def test_rastrigin_textbook_values():
    p = _identity("rastrigin", 3)
    u = p.o.astype(np.float64) + np.array([1.0, 0.5, 0.0])
    u32 = u.astype(np.float32)
    y = u32.astype(np.float64) - p.o
    ref = sum(t * t - 10 * np.cos(2 * np.pi * t) + 10 for t in y) + 100
    assert evaluate(u32, p) == pytest.approx(ref, rel=1e-14)
    # integer offsets: cos term vanishes
    off = np.array([1, -2, 3], np.float64)
    u32 = (p.o + off).astype(np.float32)
    y = u32.astype(np.float64) - p.o
    assert evaluate(u32, p) == pytest.approx(float(np.sum(y * y - 10 * np.cos(2 * np.pi * y) + 10) + 100))


def test_rastrigin_1d_grid_minimum_at_shift():
    p = _identity("rastrigin", 1)
    grid = (p.o[0] + np.linspace(-5, 5, 20001)).astype(np.float32)
    f = evaluate(grid[:, None], p)
    assert abs(float(grid[np.argmin(f)]) - float(p.o[0])) < 1e-3


def test_sphere_rotation_invariance():
    """Elliptic with condition 1 is the sphere, invariant under any orthogonal R."""
    p = W.make_problem("elliptic", 12, 4, 0)
    p.cond = 1.0
    rng = np.random.default_rng(0)
    u = rng.uniform(-100, 100, (50, 12)).astype(np.float32)
    ref = np.sum((u.astype(np.float64) - p.o) ** 2, axis=1) + 100
    assert np.allclose(evaluate(u, p), ref, rtol=1e-6)  # R is orthogonal to float32 accuracy


def test_rotation_orientation():
    """z = R (u - o): with R the cyclic map e0 -> e2, a unit step along e0 lands
    on the last (heaviest) elliptic weight, not the middle one."""
    p = _identity("elliptic", 3)
    p.R = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], np.float32)
    u = (p.o.astype(np.float64) + np.array([1.0, 0, 0])).astype(np.float32)
    y0 = float(u[0]) - float(p.o[0])
    assert evaluate(u, p) == pytest.approx(100 + 1e6 * y0 * y0, rel=1e-12)


def test_elliptic_weights():
    w = fitness.elliptic_weights(7)
    assert w[0] == 1.0 and w[-1] == pytest.approx(1e6) and np.allclose(np.diff(np.log10(w)), 1.0)


def test_ackley_values():
    p = _identity("ackley", 4)
    y = np.array([0.5, 0.5, 0.5, 0.5])
    u = (p.o + y).astype(np.float32)
    y = u.astype(np.float64) - p.o
    ref = -20 * np.exp(-0.2 * np.sqrt(np.mean(y * y))) - np.exp(np.mean(np.cos(2 * np.pi * y))) + 20 + np.e + 100
    assert evaluate(u, p) == pytest.approx(ref, rel=1e-14)
    far = (p.o + 1e3).astype(np.float32)
    assert evaluate(far, p) > 100 + 19


def test_rosenbrock_values():
    p = _identity("rosenbrock", 2)
    # z = u - o + 1 = (0, 0) -> 100*(0-0)^2 + (0-1)^2 = 1
    u = (p.o.astype(np.float64) - 1.0).astype(np.float32)
    z = u.astype(np.float64) - p.o + 1
    assert evaluate(u, p) == pytest.approx(100 * (z[0] ** 2 - z[1]) ** 2 + (z[0] - 1) ** 2 + 100, rel=1e-12)
    assert abs(evaluate(u, p) - 101) < 1e-3


def test_schwefel_textbook_form():
    """g = 418.98... D - sum x sin(sqrt|x|) at x = z + z*, minimised near x = 420.97."""
    p = _identity("schwefel", 3)
    assert fitness.SCHWEFEL_CS == pytest.approx(418.9829, abs=1e-4)
    u = (p.o + np.array([10.0, -20.0, 0.0])).astype(np.float32)
    x = u.astype(np.float64) - p.o + fitness.SCHWEFEL_ZSTAR
    ref = 3 * fitness.SCHWEFEL_CS - np.sum(x * np.sin(np.sqrt(np.abs(x)))) + 100
    assert evaluate(u, p) == pytest.approx(ref, rel=1e-13)
    assert evaluate(u, p) > 100


def test_hybrid_is_sum_of_parts():
    p = W.make_problem("hybrid", 20, 2, 0)
    assert p.split == (6, 7, 7)
    assert sorted(p.perm.tolist()) == list(range(20))
    rng = np.random.default_rng(1)
    u = rng.uniform(-100, 100, 20).astype(np.float32)
    z = p.R.astype(np.float64) @ (u.astype(np.float64) - p.o)
    zp = z[p.perm.astype(int)]
    s = fitness.g_schwefel(zp[:6]) + fitness.g_rastrigin(zp[6:13]) + fitness.g_elliptic(zp[13:])
    assert evaluate(u, p) == pytest.approx(s + 100, rel=1e-13)


def test_rotation_is_orthogonal():
    for D in (2, 10, 20, 100):
        R = W.make_problem("rastrigin", D, 3, 1).R.astype(np.float64)
        assert np.abs(R @ R.T - np.eye(D)).max() < 1e-5


# ---------------------------------------------------------------- control workload

def test_policy_sizes_table_vii():
    """Table VII: in->32->32->out policies of Hopper (11->3), Swimmer (8->2),
    Reacher (11->2) have 1539, 1410 and 1506 parameters; 17->64->64->6 has 5702."""
    assert W.mlp_param_count(11, (32, 32), 3) == 1539
    assert W.mlp_param_count(8, (32, 32), 2) == 1410
    assert W.mlp_param_count(11, (32, 32), 2) == 1506
    assert W.mlp_param_count(17, (64, 64), 6) == 5702


def test_lqr_zero_policy_closed_form():
    """W = 0 gives u = 0, so J = sum_t |A^t x0|^2."""
    p = W.make_problem("lqr_mlp", 5702, 4, 0)
    A = p.A.astype(np.float64)
    x = p.x0[0].astype(np.float64)
    ref = 0.0
    for t in range(p.steps):
        xt = np.linalg.matrix_power(A, t) @ x
        ref += xt @ xt
    assert fitness.lqr_mlp(np.zeros(5702, np.float32), p) == pytest.approx(ref, rel=1e-10)
    rho = np.max(np.abs(np.linalg.eigvals(A)))
    assert rho == pytest.approx(0.95, abs=1e-6)


def test_lqr_constant_action_closed_form():
    """Only the last layer's bias nonzero: u_t = tanh(b3) for every t."""
    p = W.make_problem("lqr_mlp", 5702, 4, 1)
    w = np.zeros(5702, np.float32)
    b3 = np.array([0.5, -0.3, 0.2, 0.0, 1.0, -1.0], np.float32)
    w[-6:] = b3
    ua = np.tanh(b3.astype(np.float64))
    A, B = p.A.astype(np.float64), p.B.astype(np.float64)
    x = p.x0[0].astype(np.float64)
    ref = 0.0
    for t in range(p.steps):
        ref += x @ x + 0.01 * ua @ ua
        x = A @ x + B @ ua
    assert fitness.lqr_mlp(w, p) == pytest.approx(ref, rel=1e-10)


def test_lqr_flatten_order():
    """The first 64*17 weights are W1 row-major: W1[k, j] multiplies x[j] into unit k."""
    layers = fitness.unflatten_policy(np.arange(5702, dtype=np.float64), 17, (64, 64), 6)
    W1, b1 = layers[0]
    assert W1.shape == (64, 17) and W1[1, 0] == 17 and b1[0] == 64 * 17
    W3, b3 = layers[2]
    assert W3.shape == (6, 64) and b3[-1] == 5701


def test_lqr_extended_precision_agrees_when_well_conditioned():
    """The extended-precision rollout reproduces the zero-policy closed form and
    agrees with float64 on policies from the workload's weight box."""
    p = W.make_problem("lqr_mlp", 5702, 4, 0)
    x = p.x0[0].astype(np.float64)
    A = p.A.astype(np.float64)
    ref = 0.0
    for _ in range(p.steps):
        ref += x @ x
        x = A @ x
    J80 = float(fitness.lqr_mlp(np.zeros(5702, np.float32), p, dtype=np.longdouble))
    assert J80 == pytest.approx(ref, rel=1e-12)
    rng = np.random.default_rng(3)
    w = rng.uniform(-0.25, 0.25, (8, 5702)).astype(np.float32)
    J64 = fitness.lqr_mlp(w, p)
    J80 = fitness.lqr_mlp(w, p, dtype=np.longdouble).astype(np.float64)
    assert np.all(np.abs(J64 - J80) <= 1e-12 * J80)


def test_table7_workload_shapes():
    """The T7 workload holds the three policies of Table VII (hidden 32 x 32) with
    their weight counts, 32 executors each, and a plant of each task's sizes."""
    wl = W.workload_t7()
    assert wl.n_runs == 96 and all(int(n) == 100 for n in wl.N) and wl.G == 50
    want = {(11, 3): 1539, (8, 2): 1410, (11, 2): 1506}
    seen = {}
    for p in wl.problems:
        obs, act = p.A.shape[0], p.B.shape[1]
        assert p.hidden == (32, 32) and p.D == want[(obs, act)]
        assert p.B.shape == (obs, act) and p.x0.shape == (1, obs)
        seen[(obs, act)] = seen.get((obs, act), 0) + 1
    assert seen == {k: 32 for k in want}


def test_c5e16_workload_has_16_rollouts():
    wl = W.workload_c5e16()
    assert wl.G == 10 and wl.n_runs == 16
    for p in wl.problems:
        assert p.D == 5702 and p.hidden == (64, 64) and p.x0.shape == (16, 17)


def _sparse_policy_problem(obs, H, act, steps):
    """A hand-made plant for the closed-form pins below (not a workload instance)."""
    rng = np.random.default_rng(11)
    A = np.zeros((obs, obs), np.float32)
    for k in range(obs):
        A[k, k] = 0.9 - 0.05 * (k % 4)
    A[1, 0] = 0.25                     # one off-diagonal coupling, x1 <- x0
    B = np.zeros((obs, act), np.float32)
    B[0, 0] = 1.0                      # action 0 drives x0
    B[obs - 1, act - 1] = 0.5          # the last action drives the last state
    x0 = rng.uniform(-1.5, 1.5, (1, obs)).astype(np.float32)
    return W.Problem(kind="lqr_mlp", D=W.mlp_param_count(obs, (H, H), act), bias=0.0,
                     A=A, B=B, x0=x0, steps=steps, hidden=(H, H))


@pytest.mark.parametrize("obs,H,act,steps", [(3, 4, 2, 2), (17, 64, 6, 3), (11, 32, 3, 2)])
def test_lqr_sparse_policy_closed_form(obs, H, act, steps):
    """A policy whose only weights are one entry of W1, one OFF-diagonal entry of
    W2, one entry of W3, plus nonzero biases on every layer.  The signal path is
    x[q1] -> unit p1 of layer 1 -> unit p2 != p1 of layer 2 -> action m, so J
    follows from scalar tanh values written out unit by unit (no matrix
    products).  A transposed W2 (square, so a product would still run) sends
    h1[p1] to unit p1 of layer 2 instead of p2; a dropped hidden tanh changes
    every downstream value; a wrong flatten offset moves an entry off the path.
    Any of these fails here."""
    p = _sparse_policy_problem(obs, H, act, steps)
    q1, p1, p2, m = obs - 1, 1, H - 2, act - 1          # p1 != p2: off-diagonal W2 entry
    a, b, c = 0.8, -1.3, 0.9                            # W1[p1, q1], W2[p2, p1], W3[m, p2]
    b1 = np.linspace(-0.2, 0.3, H).astype(np.float32)
    b2 = np.linspace(0.15, -0.25, H).astype(np.float32)
    b3 = np.linspace(0.1, -0.1, act).astype(np.float32)
    w = np.zeros(p.D, np.float32)
    o1 = 0                        # W1 [H][obs]
    ob1 = o1 + H * obs            # b1 [H]
    o2 = ob1 + H                  # W2 [H][H]
    ob2 = o2 + H * H              # b2 [H]
    o3 = ob2 + H                  # W3 [act][H]
    ob3 = o3 + act * H            # b3 [act]
    assert ob3 + act == p.D
    w[o1 + p1 * obs + q1] = a
    w[ob1:ob1 + H] = b1
    w[o2 + p2 * H + p1] = b
    w[ob2:ob2 + H] = b2
    w[o3 + m * H + p2] = c
    w[ob3:ob3 + act] = b3
    f = lambda v: float(np.float32(v))                  # the stored float32 weights
    x = [float(v) for v in p.x0[0]]
    J = 0.0
    for _ in range(steps):
        # layer 1: only unit p1 sees the state, every unit has its bias
        h1 = [math.tanh(f(b1[k]) + (f(a) * x[q1] if k == p1 else 0.0)) for k in range(H)]
        # layer 2: only unit p2 sees layer 1, and only through unit p1
        h2 = [math.tanh(f(b2[k]) + (f(b) * h1[p1] if k == p2 else 0.0)) for k in range(H)]
        # layer 3: only action m sees layer 2, through unit p2
        u = [math.tanh(f(b3[j]) + (f(c) * h2[p2] if j == m else 0.0)) for j in range(act)]
        J += sum(v * v for v in x) + p.ctrl_weight * sum(v * v for v in u)
        xn = []
        for r in range(obs):
            s = sum(float(p.A[r, k]) * x[k] for k in range(obs) if p.A[r, k] != 0)
            s += sum(float(p.B[r, j]) * u[j] for j in range(act) if p.B[r, j] != 0)
            xn.append(s)
        x = xn
    assert fitness.lqr_mlp(w, p) == pytest.approx(J, rel=1e-13)
    # the same policy with W2's entry mirrored (the transposed reading) differs
    wt = w.copy()
    wt[o2 + p2 * H + p1] = 0.0
    wt[o2 + p1 * H + p2] = b
    assert abs(fitness.lqr_mlp(wt, p) - J) > 1e-6 * J


def test_lqr_sparse_policy_hand_value():
    """The smallest sparse policy with its cost worked out by hand (to 12 digits):
    obs = 1, hidden 2 x 2, act = 1, one step from x0 = 1 with A = 0.5, B = 1.
    W1 = [[0], [1]], b1 = 0; W2 = [[0, 1], [0, 0]] (row 0 reads unit 1), b2 = 0;
    W3 = [[1, 0]], b3 = 0: u = tanh(tanh(tanh(1))), with tanh(1) = 0.761594155956,
    tanh(0.761594155956) = 0.642014992012, tanh(0.642014992012) = 0.566269975961;
    J = x0^2 + 0.01 u^2 = 1.003206616857."""
    p = W.Problem(kind="lqr_mlp", D=W.mlp_param_count(1, (2, 2), 1), bias=0.0,
                  A=np.array([[0.5]], np.float32), B=np.array([[1.0]], np.float32),
                  x0=np.array([[1.0]], np.float32), steps=1, hidden=(2, 2))
    w = np.zeros(p.D, np.float32)
    w[1] = 1.0            # W1[1, 0]
    w[4 + 1] = 1.0        # W2[0, 1]  (W2 starts after W1 (2) and b1 (2))
    w[4 + 4 + 2] = 1.0    # W3[0, 0]  (after W2 (4) and b2 (2))
    assert fitness.lqr_mlp(w, p) == pytest.approx(1.003206616857, abs=1e-11)
    w2 = np.zeros(p.D, np.float32)
    w2[1] = 1.0
    w2[4 + 2] = 1.0       # W2[1, 0]: the transposed entry leaves unit 0 of layer 2 dark
    w2[4 + 4 + 2] = 1.0
    assert fitness.lqr_mlp(w2, p) == pytest.approx(1.0, abs=1e-12)
