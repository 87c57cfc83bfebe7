"""Pins of the oracle's fourth-order two-step scheme (Remark 2.4, Section
4.2: a high-order variant of leapfrog; its iteration is a polynomial in
M^{-1} S, so C stays a function of M^{-1} S as in Lemma 2.3): the scalar
recurrence against its closed form, its stability bound, its order of
accuracy, and the operator against the sine-transform route."""

import math

import numpy as np
import pytest
import scipy.fft

import oracle
from synth import grid_spectrum
from synth.grids import grid_problem


def test_order4_recurrence_equals_closed_form():
    # q_{-1} = q_0 = 1, q_{l+1} = 2c q_l - q_{l-1} with c = 1 - x/2 + x^2/24:
    # q_l = cos((l + 1/2) theta) / cos(theta / 2), cos(theta) = c
    tau, L = 0.01, 60
    om = np.linspace(0.0, 340.0, 41)  # x up to 11.56 < 12
    x = (tau * om) ** 2
    c = 1.0 - x / 2.0 + x * x / 24.0
    th = np.arccos(c)
    ref = np.cos((np.arange(L)[:, None] + 0.5) * th[None, :]) / np.cos(th[None, :] / 2.0)
    np.testing.assert_allclose(oracle.q_sequence(om, tau, L, order=4), ref, atol=1e-9)


def test_order4_is_stable_up_to_sqrt12_and_not_beyond():
    tau, L = 1.0, 200
    for tw in (0.5, 2.0, 3.0, 3.46):
        assert np.abs(oracle.q_sequence([tw], tau, 4000, order=4)).max() < 100.0
    assert np.abs(oracle.q_sequence([3.47], tau, L, order=4)).max() > 1e6
    # the second-order scheme is unstable there already (tau omega > 2)
    assert np.abs(oracle.q_sequence([2.05], tau, L, order=2)).max() > 1e6


def test_order4_phase_error_is_fifth_order():
    # one step advances the phase by theta; the exact solution advances it by
    # tau omega: theta - tau omega = (tau omega)^3/24 + ... for order 2 and
    # O((tau omega)^5) for order 4
    for h in (0.1, 0.05, 0.025):
        x = h * h
        t2 = math.acos(1 - x / 2)
        t4 = math.acos(1 - x / 2 + x * x / 24)
        assert (t2 - h) / h**3 == pytest.approx(1 / 24, rel=0.02)
        assert abs(t4 - h) / h**5 < 0.01


def test_order4_operator_matches_sine_transform_route():
    n = 24
    S, m, h = grid_problem(2, n)
    lam_max = grid_spectrum(2, n).max()
    tau = 3.2 / math.sqrt(lam_max)  # beyond the second-order bound, inside the fourth-order one
    w = oracle.discrete_weights(0.3 * math.sqrt(lam_max), 0.5 * math.sqrt(lam_max), tau, 25)
    r = np.random.default_rng(4).standard_normal(S.shape[0])
    got = oracle.apply_filter(S, m, tau, w, r, order=4)
    k = np.arange(1, n)
    mu = 4.0 / h**2 * np.sin(k * np.pi * h / 2) ** 2
    lam = (mu[:, None] + mu[None, :]).ravel()
    beta = oracle.beta_tilde(np.sqrt(lam), tau, w, order=4).reshape(n - 1, n - 1)
    coef = scipy.fft.dstn(r.reshape(n - 1, n - 1), type=1, norm="ortho")
    ref = scipy.fft.idstn(coef * beta, type=1, norm="ortho").ravel()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
