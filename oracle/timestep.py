"""The operator C of Section 2.3, from its definition (eq. 2stepmethod and
eq. disc_filtercoeff).

For a start vector r (or a block of them, one per column) the explicit
two-step scheme defines the sequence

    y_{-1} = y_0 = r,
    y_{l+1} = -tau^2 M^{-1} S y_l + 2 y_l - y_{l-1},

and the rectangle rule with nodes l*tau, l = 0..L-1, defines

    C r = sum_{l=0}^{L-1} w_l y_l,      w_l = tau*alpha(l*tau).

M is diagonal (lumped), given as the vector m.  Forming y_0 .. y_{L-1}
takes L-1 products with S.
"""

from __future__ import annotations

import numpy as np


def leapfrog_sequence(S, m: np.ndarray, tau: float, r: np.ndarray, count: int):
    """Yield y_0, y_1, ..., y_{count-1} of eq. 2stepmethod started from
    y_{-1} = y_0 = r (float64)."""
    r = np.asarray(r, dtype=np.float64)
    minv = 1.0 / np.asarray(m, dtype=np.float64)
    if r.ndim == 2:
        minv = minv[:, None]
    y_before = r.copy()  # y_{-1}
    y_now = r.copy()  # y_0
    for ell in range(count):
        yield y_now
        if ell + 1 < count:
            y_next = -tau * tau * (minv * (S @ y_now)) + 2.0 * y_now - y_before
            y_before, y_now = y_now, y_next


def apply_filter(S, m: np.ndarray, tau: float, w: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Return C r = sum_l w_l y_l for a vector (N,) or block (N, b), in float64."""
    w = np.asarray(w, dtype=np.float64)
    total = np.zeros(np.shape(r), dtype=np.float64)
    for ell, y in enumerate(leapfrog_sequence(S, m, tau, r, len(w))):
        total = total + w[ell] * y
    return total
