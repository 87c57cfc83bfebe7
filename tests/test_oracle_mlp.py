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


def test_bf16_rounding_is_round_to_nearest_even():
    import torch

    one = 1.0
    ulp = 2.0**-7  # spacing of bfloat16 just above 1
    assert mlp.bf16_round(one + ulp / 2)[()] == one  # tie -> even (1.0)
    assert mlp.bf16_round(one + 1.5 * ulp)[()] == one + 2 * ulp  # tie -> even mantissa
    assert mlp.bf16_round(one + 0.49 * ulp)[()] == one
    assert mlp.bf16_round(-3.0)[()] == -3.0
    x = np.random.default_rng(3).standard_normal(10000) * 10.0 ** np.random.default_rng(4).uniform(-6, 6, 10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)
    assert np.max(np.abs(mlp.bf16_round(x) - x) / np.abs(x)) <= 2.0**-8 * (1 + 1e-6)


def test_bf16_gradient_is_the_float64_gradient_to_bfloat16_accuracy():
    # the float64 gradient is pinned by finite differences above; rounding
    # the products' operands to 8 significant bits moves each layer's
    # gradient by a few bfloat16 units relative to the layer's scale
    s = filter_samples(64, stream=0)
    rng = np.random.default_rng(3)
    theta = mlp.init_params(1)
    theta[-(128 * 512 + 512):] = 0.3 * rng.standard_normal(128 * 512 + 512)
    f64, g64 = mlp.loss_and_grad(theta, s)
    f16, g16 = mlp.loss_and_grad(theta, s, bf16=True)
    assert f16 == pytest.approx(f64, rel=2e-2)
    off = 0
    for shape in mlp.SHAPES:
        k = int(np.prod(shape))
        a, b = g16[off:off + k], g64[off:off + k]
        scale = np.abs(b).max()
        if scale > 0:
            assert np.abs(a - b).max() <= 0.02 * scale, shape
        off += k
    # rows of the first layer's slot that no feature feeds get no gradient
    assert np.all(g16[4 * 128:64 * 128] == 0.0)
