"""Pins of the FP64 reference of the learned filter network: the untrained
network reproduces the Fourier weights of eq. weightf and the filter of
Lemma 2.3 (computed by the independent oracle routines), backpropagation
agrees with finite differences, and the ridge least-squares teacher is the
optimum of the quadratic loss."""

import numpy as np
import pytest

import oracle
from oracle import mlp
from synth.workloads import filter_samples


def test_untrained_network_returns_fourier_weights_and_filter():
    s = filter_samples(5, stream=1)
    theta = mlp.init_params(0)
    w, J, c = mlp.forward(theta, s)
    for row, (omin, omax, tau, lam) in zip(w, s):
        a, cc, L, xm = mlp.sample_params(omin, omax, tau, lam)
        np.testing.assert_allclose(row[:L], oracle.discrete_weights(omin, omax, tau, L), atol=1e-14)
        assert np.all(row[L:] == 0.0)
        om = 2.0 * mlp.x_grid() / tau
        np.testing.assert_allclose(row @ mlp.q_matrix(), oracle.beta_tilde(om, tau, row[:L]), atol=1e-9)


def test_backpropagation_matches_finite_differences():
    s = filter_samples(6, stream=0)
    rng = np.random.default_rng(1)
    theta = mlp.init_params(2) + 0.05 * rng.standard_normal(mlp.n_params())
    f, g = mlp.loss_and_grad(theta, s)
    idx = rng.choice(mlp.n_params(), 40, replace=False)
    idx = np.concatenate([idx, [mlp.n_params() - 1, 0, 64 * 128 + 5]])
    for i in idx:
        e = np.zeros_like(theta)
        h = 1e-6 * max(1.0, abs(theta[i]))
        e[i] = h
        fd = (mlp.loss_and_grad(theta + e, s)[0] - mlp.loss_and_grad(theta - e, s)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-10)


def test_teacher_is_the_least_squares_optimum():
    for s in filter_samples(3, stream=1):
        wt = mlp.teacher(s, ridge=0.0)
        a, c, L, xm = mlp.sample_params(*s)
        wf = mlp.fourier_weights_normalised(a, c, L)
        assert mlp.loss_of_weights(s, wt) <= mlp.loss_of_weights(s, wf)
        # stationarity: perturbing any free weight increases the loss
        rng = np.random.default_rng(0)
        for _ in range(5):
            d = np.zeros(mlp.LMAX)
            d[:L] = rng.standard_normal(L) * 1e-4
            assert mlp.loss_of_weights(s, wt + d) >= mlp.loss_of_weights(s, wt) - 1e-12


def test_loss_in_frequency_terms():
    """The loss restated in the variable omega: band = [omega_min, omega_max],
    stop band = omega <= sqrt(lambda_max) at more than pi/(tau L) from the
    band (half a main lobe of an L-term filter in omega), beta~ from the
    scalar recurrence of the oracle; grid omega_g = 2 x_g / tau."""
    for s in filter_samples(4, stream=1):
        omin, omax, tau, lam = s
        a, c, L, xm = mlp.sample_params(*s)
        rng = np.random.default_rng(5)
        w = mlp.fourier_weights_normalised(a, c, L)
        w[:L] += 0.01 * rng.standard_normal(L)
        om = 2.0 * mlp.x_grid() / tau
        beta = oracle.beta_tilde(om, tau, w[:L])
        band = (om >= omin) & (om <= omax)
        gap = np.pi / (tau * L)
        stop = (om <= np.sqrt(lam)) & ((om < omin - gap) | (om > omax + gap))
        expect = np.mean((beta[band] - 1.0) ** 2) + np.mean(beta[stop] ** 2)
        assert mlp.loss_of_weights(s, w) == pytest.approx(expect, rel=1e-9)
