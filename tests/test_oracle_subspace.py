"""Pins of the oracle's fixed-dimension filtered subspace iteration
(Section 4.4, the FEAST-type variant): the closed-form spectrum of the grid
pencil with every multiplicity, an exact invariant start, and a dense
generalized eigensolve on an unstructured mesh."""

import math

import numpy as np
import scipy.linalg as sla

import oracle
from synth import grid_spectrum, power_start, start_block, workload
from synth.grids import grid_problem, jittered_problem


def _grid2d():
    P = workload("grid2d_64")
    lam = oracle.power_lambda_max(P.S, P.m, power_start(P.n, P.seed), 30)
    tau, L = oracle.time_step_rule(lam, P.omega_min)
    return P, tau, oracle.discrete_weights(P.omega_min, P.omega_max, tau, L)


def _inside(vals, lo, hi):
    om = np.sqrt(np.maximum(vals, 0.0))
    return np.sort(vals[(om >= lo) & (om <= hi)])


def test_subspace_finds_every_eigenvalue_with_its_multiplicity():
    # a fixed space of 32 columns holds all 20 eigenvalues of [10, 20] (11
    # distinct, 9 of them double): unlike a single-vector Krylov space it
    # finds every copy of a multiple eigenvalue
    P, tau, w = _grid2d()
    ref = _inside(grid_spectrum(2, 64), P.omega_min, P.omega_max)
    assert ref.size == 20
    r = oracle.subspace_solve(P.S, P.m, tau, w, start_block(P.n, 32, 0), P.omega_min, P.omega_max, tol=1e-9,
                              max_iters=40)
    assert r.omega2.size == 20
    np.testing.assert_allclose(np.sort(r.omega2), ref, rtol=1e-12)
    assert r.residual.max() <= 1e-9
    # the accepted count only grows once pairs start to converge
    counts = [c for _, c in r.history]
    assert counts[-1] == 20 and r.iterations < 40


def test_subspace_from_exact_eigenvectors_is_exact_after_one_iteration():
    # C maps an invariant subspace onto itself (Lemma 2.3), so Rayleigh-Ritz
    # on C X returns the exact pairs at once
    n = 32
    S, m, h = grid_problem(2, n)
    x = np.arange(1, n) * h
    mu = 4.0 / h**2 * np.sin(np.arange(1, n) * np.pi * h / 2) ** 2
    modes, vals = [], []
    for k1 in range(1, 6):
        for k2 in range(1, 6):
            modes.append(np.outer(np.sin(k1 * np.pi * x), np.sin(k2 * np.pi * x)).ravel())
            vals.append(mu[k1 - 1] + mu[k2 - 1])
    X0 = np.column_stack(modes)
    vals = np.array(vals)
    tau = 1.8 / math.sqrt(grid_spectrum(2, n).max())
    lo, hi = math.sqrt(vals.min()) - 1e-9, math.sqrt(vals.max()) + 1e-9
    w = oracle.discrete_weights(lo, hi, tau, 40)
    r = oracle.subspace_solve(S, m, tau, w, X0, lo, hi, tol=1e-12, max_iters=1)
    assert r.iterations == 1 and r.omega2.size == vals.size
    np.testing.assert_allclose(np.sort(r.omega2), np.sort(vals), rtol=1e-13)


def test_subspace_on_unstructured_mesh_matches_dense_eigensolve():
    S, m = jittered_problem(2, 14, 0.15, seed=3)
    lam = sla.eigh(S.toarray(), np.diag(m), eigvals_only=True)
    tau = 0.9 * 2 / math.sqrt(lam.max())
    lo, hi = 6.0, 9.0
    ref = _inside(lam, lo, hi)
    assert 4 <= ref.size <= 12
    L = int(math.ceil(2 * math.pi / (lo * tau)))
    w = oracle.discrete_weights(lo, hi, tau, L)
    r = oracle.subspace_solve(S, m, tau, w, start_block(S.shape[0], 2 * ref.size, 9), lo, hi, tol=1e-10,
                              max_iters=60)
    assert r.omega2.size == ref.size
    np.testing.assert_allclose(np.sort(r.omega2), ref, rtol=1e-11)
