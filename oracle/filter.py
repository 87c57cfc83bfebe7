"""Discrete filter response (Section 2.3: def. scalartimestep, Lemma 2.3).

Diagonalising the two-step scheme splits it into scalar recurrences, one per
eigenvalue omega^2:

    q_{-1} = q_0 = 1,   q_{l+1} = (2 - tau^2 omega^2) q_l - q_{l-1}.

The fully discrete filter is beta~(omega) = sum_{l=0}^{L-1} w_l q_l(omega)
with w_l = tau*alpha(l*tau); Lemma 2.3 states C = beta~(M^{-1} S), so every
eigenvector of the pencil is an eigenvector of C with eigenvalue beta~(omega).
The fourth-order two-step scheme (Remark 2.4, Section 4.2; see
``timestep``) gives the recurrence with factor 2 - x + x^2/12, x = tau^2 omega^2.
"""

from __future__ import annotations

import numpy as np


def q_sequence(omega, tau: float, L: int, order: int = 2) -> np.ndarray:
    """q_l(omega) for l = 0..L-1 by the forward recurrence; shape (L, len(omega))."""
    om = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    q = np.empty((L, om.size))
    q_prev = np.ones(om.size)  # q_{-1}
    q_cur = np.ones(om.size)  # q_0
    x = tau * tau * om * om
    factor = 2.0 - x + (x * x / 12.0 if order == 4 else 0.0)
    for ell in range(L):
        q[ell] = q_cur
        q_prev, q_cur = q_cur, factor * q_cur - q_prev
    return q


def beta_tilde(omega, tau: float, w: np.ndarray, order: int = 2) -> np.ndarray:
    """Fully discrete filter function of Lemma 2.3 at the given omega."""
    w = np.asarray(w, dtype=np.float64)
    q = q_sequence(omega, tau, w.size, order)
    return w @ q
