"""Plain NumPy reference of one step of the trajectory fit.

TEST INFRASTRUCTURE ONLY (imported by tests/ and the benchmark's CPU leg).

Sec. IV-A fits the five IDM parameters per trajectory by gradient descent with
box constraints; Sec. V-B3 uses Adam with a linearly decaying learning rate.
Here the parameters theta are optimised through u = (theta - lo)/(hi - lo):
Adam (Kingma & Ba, 2015) on u, then projection of u onto [0, 1], then
theta = lo + u (hi - lo).
"""
from __future__ import annotations

import numpy as np


def lr_at(t: int, lr0: float, lr1: float, lr_steps: int) -> float:
    """Learning rate of the t-th step (t = 1, 2, ...): linear from lr0 at t = 1
    to lr1 at t = lr_steps + 1, constant afterwards."""
    frac = min((t - 1) / float(lr_steps), 1.0)
    return lr0 + (lr1 - lr0) * frac


def adam_box_step(u, m, v, grad_theta, lo, hi, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on u for the gradient dL/dtheta; returns (u, m, v, theta).
    lo, hi broadcast against u (shape [5, 1] for per-kind boxes)."""
    span = hi - lo
    g = grad_theta * span                      # dL/du by the chain rule
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)                # bias corrections
    vh = v / (1.0 - beta2 ** t)
    u = u - lr * mh / (np.sqrt(vh) + eps)
    u = np.clip(u, 0.0, 1.0)                   # projection onto the box
    return u, m, v, lo + u * span


def adam_raw_step(x, m, v, grad, lo, hi, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step directly on the variables x (the reconstruction fit of
    Sec. IV-A / V-B3), then projection onto [lo, hi] (use -inf / inf for an
    unconstrained variable); returns (x, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    x = np.clip(x - lr * mh / (np.sqrt(vh) + eps), lo, hi)
    return x, m, v
