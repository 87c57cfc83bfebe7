"""Time-step sizing (Section 3.1.2 and Section 3.2: a power iteration bounds
the largest eigenvalue and the CFL condition of Section 2.3, tau < 2/omega,
fixes a stable tau).

Power iteration on M^{-1} S: x <- M^{-1} S x, normalised in the M-norm after
every product; the estimate is the Rayleigh quotient x^T S x / x^T M x of the
last iterate.  The workloads use tau = 0.9 * 2 / sqrt(lambda_est) and
L = ceil(2*pi / (omega_min * tau)) nodes per Krylov vector.
"""

from __future__ import annotations

import math

import numpy as np


def power_lambda_max(S, m: np.ndarray, x0: np.ndarray, iters: int) -> float:
    m = np.asarray(m, dtype=np.float64)
    x = np.asarray(x0, dtype=np.float64).copy()
    x /= math.sqrt(float(x @ (m * x)))
    for _ in range(iters):
        x = (S @ x) / m
        x /= math.sqrt(float(x @ (m * x)))
    return float(x @ (S @ x)) / float(x @ (m * x))


def time_step_rule(lambda_est: float, omega_min: float, safety: float = 0.9):
    """tau = safety * 2 / sqrt(lambda_est); L = ceil(2 pi / (omega_min tau))."""
    tau = safety * 2.0 / math.sqrt(lambda_est)
    L = int(math.ceil(2.0 * math.pi / (omega_min * tau)))
    return tau, L
