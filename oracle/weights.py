"""Filter weights (Section 2.2 eq. weightf; Section 2.3 eq. disc_filtercoeff).

The ideal weight is the inverse cosine transform of the indicator of
[omega_min, omega_max] (Section 2.2, eq. filterf); the method truncates it to
[0, T] and gives t = 0 its limit value 2(omega_max - omega_min)/pi.  The
rectangle rule with L nodes and step tau = T/L samples it at t = l*tau,
l = 0..L-1, each node weighted by tau.
"""

from __future__ import annotations

import numpy as np


def alpha(t, omega_min: float, omega_max: float, T: float):
    """Truncated weight function alpha(t) of eq. weightf."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    zero = t == 0.0
    inside = (t > 0.0) & (t <= T)
    out[zero] = 2.0 * (omega_max - omega_min) / np.pi
    ti = t[inside]
    out[inside] = (4.0 / (np.pi * ti)) * np.sin(0.5 * ti * (omega_max - omega_min)) * np.cos(
        0.5 * ti * (omega_max + omega_min)
    )
    return out


def discrete_weights(omega_min: float, omega_max: float, tau: float, L: int) -> np.ndarray:
    """Coefficients w_l = tau * alpha(l*tau), l = 0..L-1, with T = L*tau."""
    if L < 1 or tau <= 0:
        raise ValueError("need L >= 1 and tau > 0")
    T = L * tau
    return tau * alpha(np.arange(L) * tau, omega_min, omega_max, T)
