"""Pins of the oracle's weights and filter response against closed forms.

Weights: Section 2.2 (eq. filterf, eq. weightf), Section 2.3 (eq.
disc_filtercoeff).  Scalar recurrence and filter: Section 2.3 (def.
scalartimestep, Lemma 2.3).
"""

import numpy as np
import pytest

import oracle


def test_alpha_equals_inverse_cosine_transform_of_indicator():
    # (2/pi) * int_{a}^{b} cos(t s) ds = (2/pi) (sin(bt) - sin(at)) / t, an
    # independent route to the product form printed in eq. filterf
    a, b = 10.0, 20.0
    t = np.linspace(1e-3, 5.0, 4001)
    direct = (2.0 / np.pi) * (np.sin(b * t) - np.sin(a * t)) / t
    np.testing.assert_allclose(oracle.alpha(t, a, b, T=10.0), direct, rtol=0, atol=1e-12)


def test_alpha_at_zero_is_the_limit_and_truncates_after_T():
    a, b = 3.0, 7.5
    lim = oracle.alpha(np.array([1e-9]), a, b, T=1.0)[0]
    assert oracle.alpha(np.array([0.0]), a, b, T=1.0)[0] == pytest.approx(2 * (b - a) / np.pi, rel=1e-15)
    assert lim == pytest.approx(2 * (b - a) / np.pi, rel=1e-12)
    assert np.all(oracle.alpha(np.array([1.0 + 1e-12, 2.0, 50.0]), a, b, T=1.0) == 0.0)


def test_discrete_weights_sample_alpha_on_left_rectangle_nodes():
    a, b, tau, L = 10.0, 20.0, 0.01, 63
    w = oracle.discrete_weights(a, b, tau, L)
    assert w.shape == (L,)
    ell = np.arange(L)
    ref = tau * (2.0 / np.pi) * np.where(ell == 0, b - a, (np.sin(b * ell * tau) - np.sin(a * ell * tau)) / np.maximum(ell * tau, 1e-300))
    np.testing.assert_allclose(w, ref, rtol=1e-13, atol=1e-16)


def _q_chebyshev_v(omega, tau, L):
    # third-kind Chebyshev polynomial V_l(x) = cos((l+1/2) th) / cos(th/2),
    # x = cos(th) = 1 - tau^2 omega^2 / 2: the solution of the recurrence with
    # V_{-1} = V_0 = 1 (derived by hand, independent of the recurrence code)
    x = 1.0 - 0.5 * (tau * omega) ** 2
    th = np.arccos(np.clip(x, -1.0, 1.0))
    ell = np.arange(L)[:, None]
    return np.cos((ell + 0.5) * th[None, :]) / np.cos(0.5 * th[None, :])


def test_q_recurrence_matches_chebyshev_v_closed_form():
    tau = 0.01
    om = np.linspace(0.0, 1.9 / tau, 257)
    q = oracle.q_sequence(om, tau, 300)
    np.testing.assert_allclose(q, _q_chebyshev_v(om, tau, 300), rtol=0, atol=5e-10 * 300)
    assert np.all(q[:, 0] == 1.0)  # q_l(0) = 1


def test_printed_closed_form_is_the_previous_index():
    # Reading of Section 2.3: the printed two-term closed form with
    # c = 1 - tau^2 w^2/2 + i sqrt(1 - (1 - tau^2 w^2/2)^2) evaluates to
    # q_{l-1}, not q_l; the recurrence is authoritative.
    tau, om = 0.02, np.array([13.0, 41.0, 77.0])
    x = 1 - 0.5 * (tau * om) ** 2
    c = x + 1j * np.sqrt(1 - x * x)
    L = 40
    q = oracle.q_sequence(om, tau, L)
    ell = np.arange(1, L)[:, None]
    printed = ((1 - np.conj(c)) / (2j * c.imag)) * c ** ell + ((c - 1) / (2j * c.imag)) * np.conj(c) ** ell
    np.testing.assert_allclose(printed.real, q[:-1], atol=1e-10)
    assert np.abs(printed.imag).max() < 1e-10
    assert np.abs(printed.real - q[1:]).max() > 1e-3


def test_q_bounded_under_cfl_and_unbounded_above():
    tau, L = 0.05, 2000
    stable = oracle.q_sequence(np.array([0.5, 1.0, 1.95]) / tau, tau, L)
    th = np.arccos(1 - 0.5 * np.array([0.5, 1.0, 1.95]) ** 2)
    assert np.all(np.abs(stable).max(axis=0) <= 1.0 / np.cos(th / 2) + 1e-9)
    unstable = oracle.q_sequence(np.array([2.05]) / tau, tau, 400)
    assert np.abs(unstable).max() > 1e6


def _beta_clenshaw(omega, tau, w):
    # backward sum: b_k = w_k + a b_{k+1} - b_{k+2} with a = 2 - tau^2 w^2,
    # then sum_k w_k q_k = b_0 - b_1 because q_0 = 1 and q_1 = a - 1
    a = 2.0 - (tau * omega) ** 2
    b1 = np.zeros_like(omega)
    b2 = np.zeros_like(omega)
    for k in range(len(w) - 1, -1, -1):
        b0 = w[k] + a * b1 - b2
        b2, b1 = b1, b0
    return b1 - b2


def test_beta_tilde_forward_equals_clenshaw():
    tau, L = 0.010057834447673006, 63
    w = oracle.discrete_weights(10.0, 20.0, tau, L)
    om = np.linspace(0.0, 1.99 / tau, 1001)
    np.testing.assert_allclose(oracle.beta_tilde(om, tau, w), _beta_clenshaw(om, tau, w), atol=1e-12)


def test_beta_tilde_is_polynomial_of_degree_L_minus_1_in_omega_squared():
    tau, L = 0.02, 12
    w = oracle.discrete_weights(4.0, 9.0, tau, L)
    x = np.linspace(0.0, 3.5 / tau**2, L)  # L nodes in omega^2
    coeff = np.polynomial.polynomial.polyfit(x, oracle.beta_tilde(np.sqrt(x), tau, w), L - 1)
    xt = np.linspace(0.1, 3.4 / tau**2, 37)
    np.testing.assert_allclose(np.polynomial.polynomial.polyval(xt, coeff), oracle.beta_tilde(np.sqrt(xt), tau, w), atol=1e-6)


def test_beta_tilde_tends_to_indicator():
    # tau -> 0 and T -> infinity: the rectangle rule tends to the integral of
    # eq. filterfunc with the untruncated weight, i.e. the indicator of the
    # interval (1/2 at its ends, the Dirichlet integral)
    a, b, tau, L = 2.0, 4.0, 1e-3, 400000
    w = oracle.discrete_weights(a, b, tau, L)
    om = np.array([1.0, 3.0, 5.0, 2.0, 4.0])
    beta = oracle.beta_tilde(om, tau, w)
    np.testing.assert_allclose(beta[:3], [0.0, 1.0, 0.0], atol=2e-3)
    # at the ends the truncated sine integral still oscillates as O(1/(T omega))
    np.testing.assert_allclose(beta[3:], [0.5, 0.5], atol=6e-3)


def test_paper_example_parameters_are_consistent():
    # Section 3.1.2 prints tau ~ 0.0056 and T = 300 tau ~ 1.68; with T = L tau
    # the weights of that run have 300 nodes reaching t = 299 tau < T
    tau, L = 0.0056, 300
    assert L * tau == pytest.approx(1.68, rel=1e-12)
    w = oracle.discrete_weights(0.0, 3.0, tau, L)
    assert w.shape == (300,) and w[0] == pytest.approx(tau * 2 * 3.0 / np.pi)
