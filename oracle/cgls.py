"""Least-squares reconstruction with the matched SRT pair, FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's stated purpose for an exactly matched adjoint (Sec. 1, Sec. 3.2)
is optimisation-based reconstruction: minimise ||A f - g||_2 over volumes f,
with A the discrete SRT of Alg. 1 and A^T its transpose, Alg. 2. This module
runs conjugate gradients on the normal equations A^T A f = A^T g in the CGLS
arrangement (Hestenes and Stiefel; Bjorck, "Numerical Methods for Least
Squares Problems", Sec. 7.4), which only ever applies A and A^T:

    r = g - A f,  s = A^T r,  p = s,  gamma = ||s||^2
    repeat:  q = A p,  alpha = gamma / ||q||^2
             f <- f + alpha p,  r <- r - alpha q
             s = A^T r,  gamma' = ||s||^2,  p <- s + (gamma'/gamma) p

The iterate after k steps minimises ||A f - g|| over f0 plus the Krylov space
span{s0, (A^T A) s0, ..., (A^T A)^(k-1) s0}. `apply` and `apply_t` are any
pair of callables computing A x and A^T y (here: oracle.srt.forward/adjoint).
"""
from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np


def cgls(apply: Callable[[np.ndarray], np.ndarray], apply_t: Callable[[np.ndarray], np.ndarray],
         g: np.ndarray, f0: np.ndarray, n_iter: int) -> Tuple[np.ndarray, List[float]]:
    """n_iter CGLS steps from f0. Returns f_n and the normal-equation
    residual norms ||A^T (g - A f_k)||_2 for k = 0..n_iter."""
    f = np.array(f0, dtype=np.float64, copy=True)
    r = g - apply(f)
    s = apply_t(r)
    p = s.copy()
    gamma = float(np.vdot(s, s))
    hist = [np.sqrt(gamma)]
    for _ in range(n_iter):
        q = apply(p)
        delta = float(np.vdot(q, q))
        alpha = gamma / delta if delta > 0.0 else 0.0
        f += alpha * p
        r -= alpha * q
        s = apply_t(r)
        gamma_new = float(np.vdot(s, s))
        beta = gamma_new / gamma if gamma > 0.0 else 0.0
        p = s + beta * p
        gamma = gamma_new
        hist.append(np.sqrt(gamma))
    return f, hist
