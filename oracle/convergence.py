"""A model of the Krylov iteration's convergence for a given filter (TEST
INFRASTRUCTURE: the plain form of the library's step predictor).

Section 2.2 asks for |beta(omega)| >> |beta(omega~)| between sought and
unsought frequencies, and Section 3.1.3 shows that the filter alone does not
predict the number of steps.  The model runs the Krylov iteration itself on a
model spectrum: in the eigenbasis of the pencil, C = beta~(M^{-1} S) is the
diagonal matrix D = diag(beta~(omega_j)) (Lemma 2.3) and a start vector has
components of size sqrt(weight_j) (weight_j: how many eigenvalues the model
point stands for).  The Krylov space span{v, D v, D^2 v, ...} is built with an
orthonormal basis Q (Gram-Schmidt twice); the direction e_j of a sought
eigenvalue is resolved once it lies in the space to within eps, i.e. once
1 - |Q[j, :]|^2 <= eps^2.  The predicted number of Krylov steps is the first
dimension at which every model point in [omega_min, omega_max] is resolved.
"""

from __future__ import annotations

import numpy as np

from .filter import beta_tilde


def predict_steps(omega, weight, w, tau, omega_min, omega_max, eps=1e-6, kmax=2000, order=2, beta=None):
    """Predicted Krylov steps (kmax when some sought point is never resolved).
    ``beta`` (optional) gives the filter values directly instead of w."""
    omega = np.asarray(omega, dtype=np.float64)
    d = beta_tilde(omega, tau, w, order) if beta is None else np.asarray(beta, dtype=np.float64)
    v = np.sqrt(np.asarray(weight, dtype=np.float64))
    Q = [v / np.linalg.norm(v)]
    inside = (omega >= omega_min) & (omega <= omega_max)
    if not inside.any():
        return 0
    captured = Q[0] ** 2
    for k in range(1, kmax):
        x = d * Q[-1]
        B = np.column_stack(Q)
        for _ in range(2):
            x = x - B @ (B.T @ x)
        nx = np.linalg.norm(x)
        if nx <= 1e-14:
            # the space is invariant: what is not resolved now never will be
            return k if np.all(1.0 - captured[inside] <= eps * eps) else kmax
        Q.append(x / nx)
        captured = captured + Q[-1] ** 2
        if np.all(1.0 - captured[inside] <= eps * eps):
            return k + 1
    return kmax
