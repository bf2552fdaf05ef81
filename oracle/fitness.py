"""Objective functions in float64 -- oracle (test infrastructure only).

The paper evaluates on CEC2022 (Sec. IV-A), whose data files are not part of
this project.  Its configurations name textbook base functions instead; this
module writes each one out from its standard definition, with the convention
z = R (u - o) [+ c] and f = g(z) + bias, where the float32 values of u, o and
R are promoted to float64 first.  No scaling or penalty conventions of the
CEC suite are used.

    rastrigin   g = sum(z^2 - 10 cos(2 pi z) + 10)
    elliptic    g = sum(cond^(j/(D-1)) z_j^2)
    ackley      g = -20 exp(-0.2 sqrt(mean z^2)) - exp(mean cos(2 pi z)) + 20 + e
    rosenbrock  z += 1; g = sum_{j<D-1} 100 (z_j^2 - z_{j+1})^2 + (z_j - 1)^2
    schwefel    z += z*; g = sum(c_s - z_j sin(sqrt|z_j|)),  c_s = z* sin(sqrt z*)
    hybrid      z permuted, split (n1, n2, n3): schwefel | rastrigin | elliptic

The control-shaped workload scores a flattened tanh policy by a rollout of a
linear system (see ``lqr_mlp``).
"""
from __future__ import annotations

import numpy as np

# Schwefel's shift: the float32-representable point nearest the maximiser
# 420.96874636... of x sin(sqrt x), so both precisions use the same constant.
SCHWEFEL_ZSTAR = 420.96875
SCHWEFEL_CS = SCHWEFEL_ZSTAR * np.sin(np.sqrt(SCHWEFEL_ZSTAR))


def _rotate(u, prob):
    y = np.asarray(u, dtype=np.float32).astype(np.float64) - prob.o.astype(np.float64)
    return y @ prob.R.astype(np.float64).T


def g_rastrigin(z):
    return np.sum(z * z - 10.0 * np.cos(2.0 * np.pi * z) + 10.0, axis=-1)


def elliptic_weights(D, cond=1e6):
    if D == 1:
        return np.ones(1)
    return cond ** (np.arange(D, dtype=np.float64) / (D - 1))


def g_elliptic(z, cond=1e6):
    return np.sum(elliptic_weights(z.shape[-1], cond) * z * z, axis=-1)


def g_ackley(z):
    D = z.shape[-1]
    s1 = np.sum(z * z, axis=-1) / D
    s2 = np.sum(np.cos(2.0 * np.pi * z), axis=-1) / D
    return -20.0 * np.exp(-0.2 * np.sqrt(s1)) - np.exp(s2) + 20.0 + np.e


def g_rosenbrock(z):
    z = z + 1.0
    a = z[..., :-1]
    b = z[..., 1:]
    return np.sum(100.0 * (a * a - b) ** 2 + (a - 1.0) ** 2, axis=-1)


def g_schwefel(z):
    z = z + SCHWEFEL_ZSTAR
    return np.sum(SCHWEFEL_CS - z * np.sin(np.sqrt(np.abs(z))), axis=-1)


def g_hybrid(z, perm, split, cond=1e6):
    zp = z[..., perm.astype(np.int64)]
    n1, n2, _ = split
    return (g_schwefel(zp[..., :n1]) + g_rastrigin(zp[..., n1:n1 + n2])
            + g_elliptic(zp[..., n1 + n2:], cond))


def unflatten_policy(w, n_in, hidden, n_out):
    """Split flat weights [..., D] into [(W, b), ...] with W row-major [out, in]."""
    sizes = [n_in, *hidden, n_out]
    layers = []
    off = 0
    for k in range(len(sizes) - 1):
        fi, fo = sizes[k], sizes[k + 1]
        W = w[..., off:off + fo * fi].reshape(*w.shape[:-1], fo, fi)
        off += fo * fi
        b = w[..., off:off + fo]
        off += fo
        layers.append((W, b))
    assert off == w.shape[-1]
    return layers


def lqr_mlp(w, prob, dtype=np.float64):
    """Mean over rollouts of J = sum_t x_t^T Q x_t + c ||u_t||^2 with Q = I,
    u_t = tanh-MLP(x_t), x_{t+1} = A x_t + B u_t, for t = 0 .. steps-1.

    ``dtype`` is the working precision (float64, or numpy's extended
    longdouble to estimate how well float64 determines J: the closed loop of
    a policy can amplify rounding differences by many orders of magnitude)."""
    w = np.asarray(w, dtype=np.float32).astype(dtype)
    lead = w.shape[:-1]
    A = prob.A.astype(dtype)
    B = prob.B.astype(dtype)
    x0 = prob.x0.astype(dtype)                          # [E, obs]
    cw = dtype(prob.ctrl_weight)
    layers = unflatten_policy(w, A.shape[0], prob.hidden, B.shape[1])
    x = np.broadcast_to(x0, (*lead, *x0.shape)).copy()  # [..., E, obs]
    J = np.zeros((*lead, x0.shape[0]), dtype=dtype)
    for _ in range(prob.steps):
        h = x
        for W, b in layers:
            h = np.tanh(np.einsum("...oi,...ei->...eo", W, h) + b[..., None, :])
        J += np.sum(x * x, axis=-1) + cw * np.sum(h * h, axis=-1)
        x = np.einsum("ji,...ei->...ej", A, x) + np.einsum("ja,...ea->...ej", B, h)
    return J.mean(axis=-1)


def evaluate(u, prob):
    """Fitness of trial vectors u [..., D] (float32 values) in float64."""
    if prob.kind == "lqr_mlp":
        return lqr_mlp(u, prob)
    z = _rotate(u, prob)
    if prob.kind == "rastrigin":
        g = g_rastrigin(z)
    elif prob.kind == "elliptic":
        g = g_elliptic(z, prob.cond)
    elif prob.kind == "ackley":
        g = g_ackley(z)
    elif prob.kind == "rosenbrock":
        g = g_rosenbrock(z)
    elif prob.kind == "schwefel":
        g = g_schwefel(z)
    elif prob.kind == "hybrid":
        g = g_hybrid(z, prob.perm, prob.split, prob.cond)
    else:
        raise ValueError(prob.kind)
    return g + prob.bias
