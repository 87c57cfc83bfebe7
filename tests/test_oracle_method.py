"""Pins of the oracle's operator C, power iteration and Krylov solver.

C is pinned by Lemma 2.3 (C = beta~(M^{-1} S)) evaluated through routes that
share nothing with the time loop: discrete sine transforms on tensor grids
(whose eigenvectors are sine modes) and a dense generalized eigendecomposition
on small unstructured meshes.  The Krylov solver is pinned by the closed-form
spectrum of the grid pencils, by dense eigensolves, and by the basis
independence of the projected pencil (Section 2.1, eq. projevp).
"""

import math

import numpy as np
import pytest
import scipy.fft
import scipy.linalg as sla

import oracle
from synth import distinct_target, grid_spectrum, start_block, workload
from synth.grids import grid_problem, jittered_problem


def _sine_eigs(n):
    h = 1.0 / n
    k = np.arange(1, n)
    return 4.0 / h**2 * np.sin(k * np.pi * h / 2) ** 2


def _dst_filter(dim, n, tau, w, r):
    """C r through the sine basis: transform, multiply by beta~(omega_k),
    transform back (DST-I is its own inverse with norm='ortho')."""
    mu = _sine_eigs(n)
    if dim == 2:
        lam = mu[:, None] + mu[None, :]
    else:
        lam = mu[:, None, None] + mu[None, :, None] + mu[None, None, :]
    beta = oracle.beta_tilde(np.sqrt(lam.ravel()), tau, w).reshape(lam.shape)
    shape = (n - 1,) * dim
    coef = scipy.fft.dstn(r.reshape(shape), type=1, norm="ortho")
    return scipy.fft.idstn(coef * beta, type=1, norm="ortho").ravel()


@pytest.mark.parametrize("dim,n,L", [(2, 64, 63), (3, 12, 17), (2, 9, 1), (2, 9, 2)])
def test_filter_matches_sine_transform_route(dim, n, L):
    S, m, h = grid_problem(dim, n)
    lam_max = grid_spectrum(dim, n).max()
    tau = 1.8 / math.sqrt(lam_max)
    w = oracle.discrete_weights(0.3 * math.sqrt(lam_max), 0.5 * math.sqrt(lam_max), tau, L)
    r = np.random.default_rng(7).standard_normal(S.shape[0])
    got = oracle.apply_filter(S, m, tau, w, r)
    ref = _dst_filter(dim, n, tau, w, r)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_filter_on_sine_mode_is_beta_times_mode():
    n, tau = 32, 0.02
    S, m, h = grid_problem(2, n)
    x = np.arange(1, n) * h
    k1, k2 = 3, 5
    v = np.outer(np.sin(k1 * np.pi * x), np.sin(k2 * np.pi * x)).ravel()
    lam = _sine_eigs(n)[k1 - 1] + _sine_eigs(n)[k2 - 1]
    w = oracle.discrete_weights(10.0, 20.0, tau, 50)
    Cv = oracle.apply_filter(S, m, tau, w, v)
    np.testing.assert_allclose(Cv, oracle.beta_tilde(math.sqrt(lam), tau, w)[0] * v, atol=1e-13)


def test_filter_on_unstructured_mesh_matches_dense_spectral_form():
    S, m = jittered_problem(2, 10, 0.2, seed=5)
    lam, V = sla.eigh(S.toarray(), np.diag(m))  # V^T M V = I
    lam = np.maximum(lam, 0.0)
    tau = 1.8 / math.sqrt(lam.max())
    w = oracle.discrete_weights(2.0, 6.0, tau, 40)
    r = np.random.default_rng(1).standard_normal((S.shape[0], 3))
    ref = V @ (oracle.beta_tilde(np.sqrt(lam), tau, w)[:, None] * (V.T @ (m[:, None] * r)))
    np.testing.assert_allclose(oracle.apply_filter(S, m, tau, w, r), ref, atol=1e-11 * np.abs(ref).max())


def test_filter_is_m_self_adjoint_and_columnwise():
    S, m = jittered_problem(3, 4, 0.1, seed=2)
    tau = 0.9 * 2 / math.sqrt(sla.eigh(S.toarray(), np.diag(m), eigvals_only=True).max())
    w = oracle.discrete_weights(1.0, 4.0, tau, 25)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((S.shape[0], 2))
    CX = oracle.apply_filter(S, m, tau, w, X)
    lhs = CX[:, 0] @ (m * X[:, 1])
    rhs = X[:, 0] @ (m * CX[:, 1])
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    np.testing.assert_allclose(CX[:, 1], oracle.apply_filter(S, m, tau, w, X[:, 1]), atol=1e-14)


def test_power_iteration_bounds_and_exact_start():
    S, m, h = grid_problem(2, 20)
    lam = grid_spectrum(2, 20)
    x0 = np.random.default_rng(0).standard_normal(S.shape[0])
    est30 = oracle.power_lambda_max(S, m, x0, 30)
    assert 0.9 * lam.max() < est30 <= lam.max() * (1 + 1e-14)
    est = oracle.power_lambda_max(S, m, x0, 3000)
    assert est == pytest.approx(lam.max(), rel=1e-5)
    x = np.arange(1, 20) * h
    mode = np.outer(np.sin(19 * np.pi * x), np.sin(19 * np.pi * x)).ravel()
    assert oracle.power_lambda_max(S, m, mode, 5) == pytest.approx(lam.max(), rel=1e-13)


def test_time_step_rule_is_stable_and_covers_one_period():
    tau, L = oracle.time_step_rule(32748.264754465545, 10.0)
    assert tau * math.sqrt(32748.264754465545) == pytest.approx(1.8)
    assert L * tau * 10.0 >= 2 * math.pi > (L - 1) * tau * 10.0


@pytest.fixture(scope="module")
def grid2d_run():
    P = workload("grid2d_64")
    from synth import power_start

    lam_est = oracle.power_lambda_max(P.S, P.m, power_start(P.n, P.seed), 30)
    tau, L = oracle.time_step_rule(lam_est, P.omega_min)
    w = oracle.discrete_weights(P.omega_min, P.omega_max, tau, L)
    V0 = start_block(P.n, 1, P.seed)
    res = oracle.krylov_solve(P.S, P.m, tau, w, V0, P.omega_min, P.omega_max, tol=1e-9, m_max=40, keep_basis=True)
    return P, tau, w, V0, res


def test_grid2d_recovers_closed_form_spectrum(grid2d_run):
    P, tau, w, V0, res = grid2d_run
    tgt, vals, mult = distinct_target(grid_spectrum(2, 64), P.omega_min, P.omega_max, 1)
    assert tgt == 11 and res.omega2.size == 11
    np.testing.assert_allclose(res.omega2, vals, rtol=1e-12)
    assert res.residual.max() <= 1e-9
    assert res.basis_size == 40 and res.krylov_steps == 39


def test_basis_is_m_orthonormal(grid2d_run):
    P, tau, w, V0, res = grid2d_run
    B = res.basis
    G = B.T @ (P.m[:, None] * B)
    assert np.abs(G - np.eye(B.shape[1])).max() < 1e-13


def test_projected_pencil_is_basis_independent(grid2d_run):
    # a Euclidean basis (the paper's inner product) spans the same
    # Krylov space; eq. projevp uses both B^T S B and B^T M B, so the Ritz
    # values agree although the bases differ
    P, tau, w, V0, res = grid2d_run
    k = 15
    Bp = oracle.krylov_basis_euclidean(P.S, P.m, tau, w, V0[:, 0], k)
    Bm = res.basis[:, :k]
    th_p = oracle.rayleigh_ritz(P.S, P.m, Bp, 0, 1e9)[0]
    th_m = oracle.rayleigh_ritz(P.S, P.m, Bm, 0, 1e9)[0]
    np.testing.assert_allclose(th_p, th_m, rtol=1e-9)
    assert np.abs(Bp.T @ Bp - np.eye(k)).max() < 1e-12


def test_unstructured_neumann_matches_dense_eigensolve():
    S, m = jittered_problem(2, 14, 0.2, seed=11)
    lam = sla.eigh(S.toarray(), np.diag(m), eigvals_only=True)
    lam_est = oracle.power_lambda_max(S, m, np.random.default_rng(1).standard_normal(S.shape[0]), 30)
    tau, L = oracle.time_step_rule(lam_est, 8.0)
    w = oracle.discrete_weights(8.0, 14.0, tau, L)
    V0 = start_block(S.shape[0], 1, 4)
    tgt, vals, mult = distinct_target(lam, 8.0, 14.0, 1, rtol=1e-8)
    res = oracle.krylov_solve(S, m, tau, w, V0, 8.0, 14.0, tol=1e-9, m_max=120, target=tgt)
    assert res.omega2.size == tgt
    np.testing.assert_allclose(res.omega2, vals, rtol=1e-10)


def test_block_start_recovers_double_eigenvalues():
    # on the square, lambda(k1,k2) = lambda(k2,k1): multiplicity 2 off the
    # diagonal; a single start vector sees one copy, a block of 2 sees both
    S, m, h = grid_problem(2, 24)
    lam = grid_spectrum(2, 24)
    tau, L = oracle.time_step_rule(lam.max(), 15.0)
    w = oracle.discrete_weights(15.0, 24.0, tau, L)
    for b in (1, 2):
        tgt, vals, mult = distinct_target(lam, 15.0, 24.0, b)
        res = oracle.krylov_solve(S, m, tau, w, start_block(S.shape[0], b, 9), 15.0, 24.0, tol=1e-9, m_max=160, target=tgt)
        assert res.omega2.size == tgt
        expect = np.repeat(vals, np.minimum(mult, b))
        np.testing.assert_allclose(res.omega2, expect, rtol=1e-10)
    assert (mult > 1).any()


def test_breakdown_on_exact_eigenvector_start():
    n = 20
    S, m, h = grid_problem(2, n)
    x = np.arange(1, n) * h
    v = np.outer(np.sin(2 * np.pi * x), np.sin(3 * np.pi * x)).ravel()
    lam = _sine_eigs(n)[1] + _sine_eigs(n)[2]
    tau, L = oracle.time_step_rule(grid_spectrum(2, n).max(), 5.0)
    w = oracle.discrete_weights(5.0, 15.0, tau, L)
    res = oracle.krylov_solve(S, m, tau, w, v[:, None], 5.0, 15.0, tol=1e-9, m_max=10)
    assert res.breakdown and res.basis_size == 1 and res.krylov_steps == 1
    assert res.omega2.size == 1 and res.omega2[0] == pytest.approx(lam, rel=1e-13)


def test_residual_of_a_two_mode_mixture_has_closed_form():
    # v = (v1 + v2)/sqrt(2) with M-normalised modes: theta = (l1+l2)/2 and
    # S v - theta M v = ((l1-l2)/2)(M v1 - M v2)/sqrt(2)
    n = 16
    S, m, h = grid_problem(2, n)
    x = np.arange(1, n) * h
    mu = _sine_eigs(n)
    v1 = np.outer(np.sin(np.pi * x), np.sin(2 * np.pi * x)).ravel()
    v2 = np.outer(np.sin(3 * np.pi * x), np.sin(np.pi * x)).ravel()
    v1 /= math.sqrt(v1 @ (m * v1))
    v2 /= math.sqrt(v2 @ (m * v2))
    l1, l2 = mu[0] + mu[1], mu[2] + mu[0]
    B = np.column_stack([(v1 + v2) / math.sqrt(2)])
    theta, th_c, res, V = oracle.rayleigh_ritz(S, m, B, 0.0, 1e9)
    assert theta[0] == pytest.approx(0.5 * (l1 + l2), rel=1e-13)
    num = abs(l1 - l2) / 2 * np.linalg.norm(m * (v1 - v2)) / math.sqrt(2)
    den = np.linalg.norm(m * (l1 * v1 + l2 * v2)) / math.sqrt(2)
    assert res[0] == pytest.approx(num / den, rel=1e-12)
