"""Nonnegative least squares with the matched SRT pair, FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper motivates an exactly matched adjoint by optimisation-based
reconstruction (Sec. 1, Sec. 3.2). An initial pressure cannot be negative,
so a common form of that reconstruction is

    minimise 0.5 ||A f - g||_2^2  subject to  f >= 0,

with A the discrete SRT of Alg. 1 and A^T its transpose, Alg. 2. The
gradient A^T (A f - g) needs only that pair. This module runs the
accelerated projected gradient method FISTA (Beck and Teboulle, SIAM J.
Imaging Sciences 2(1), 2009, Sec. 4, with the indicator function of the
nonnegative orthant as the nonsmooth term, whose proximal map is the
projection max(0, .)):

    y_1 = f_0,  t_1 = 1
    f_k = max(0, y_k - (1/L) A^T (A y_k - g))
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
    y_{k+1} = f_k + ((t_k - 1) / t_{k+1}) (f_k - f_{k-1})     (f_0 as given)

for a step 1/L with L >= ||A||_2^2, the Lipschitz constant of the gradient.
The same paper bounds the objective gap after k steps by
2 L ||f_0 - f*||^2 / (k + 1)^2 (its Theorem 4.4).

||A||_2^2 = lambda_max(A^T A) is estimated by the power method on A^T A from
the all-ones volume: A has no negative entries, so the dominant eigenvector
of A^T A can be taken nonnegative and the start has a component along it.
The Rayleigh quotient ||A v||^2 / ||v||^2 of every iterate is a lower bound
of lambda_max.
"""
from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np


def opnorm2(apply: Callable[[np.ndarray], np.ndarray], apply_t: Callable[[np.ndarray], np.ndarray],
            shape, n_iter: int) -> float:
    """n_iter power steps on A^T A from ones(shape). Returns the Rayleigh
    quotient ||A v||^2 / ||v||^2 of the last iterate v (0 if A v vanishes
    along the way)."""
    v = np.ones(shape, dtype=np.float64)
    lam = 0.0
    for _ in range(n_iter):
        u = apply(v)
        lam = float(np.vdot(u, u)) / float(np.vdot(v, v))
        w = apply_t(u)
        nw = float(np.sqrt(np.vdot(w, w)))
        if nw == 0.0:
            return 0.0
        v = w / nw
    return lam


def momentum(n_iter: int) -> List[float]:
    """The extrapolation weights (t_k - 1) / t_{k+1}, k = 1..n_iter."""
    t, out = 1.0, []
    for _ in range(n_iter):
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        out.append((t - 1.0) / t_next)
        t = t_next
    return out


def fista_nn(apply: Callable[[np.ndarray], np.ndarray], apply_t: Callable[[np.ndarray], np.ndarray],
             g: np.ndarray, f0: np.ndarray, step: float, n_iter: int) -> Tuple[np.ndarray, List[float]]:
    """n_iter FISTA steps with step 1/L = `step` from f0. Returns f_n and the
    misfits ||A y_k - g||_2 at the points y_k where the gradient was taken,
    k = 1..n_iter."""
    f_prev = np.array(f0, dtype=np.float64, copy=True)
    y = f_prev.copy()
    hist = []
    for beta in momentum(n_iter):
        r = apply(y) - g
        hist.append(float(np.sqrt(np.vdot(r, r))))
        f = np.maximum(0.0, y - step * apply_t(r))
        y = f + beta * (f - f_prev)
        f_prev = f
    return f_prev, hist
