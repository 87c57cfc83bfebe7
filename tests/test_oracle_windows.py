"""Pins of the alternative weight functions (Section 4.3): each closed-form
transform against numerical quadrature of its target, the indicator against
eq. weightf, the filter tending to the target for fine steps and long T, and
the spectrum-adapted (notch) weights against the definition of a
minimum-norm constrained change."""

import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from oracle import windows


@pytest.mark.parametrize("kind,width", [("triangle", 2.0), ("triangle", 0.7), ("gaussian", 1.0), ("gaussian", 2.5),
                                        ("indicator", 1.0)])
def test_transform_equals_quadrature_of_the_target(kind, width):
    lo, hi = 3.0, 5.0
    for t in (0.0, 0.37, 1.3, 4.1, 9.9):
        f = lambda om: windows.target(om, kind, lo, hi, width) * math.cos(om * t)  # noqa: E731
        pts = [lo, hi, 4.0 - 2 * width, 4.0 + 2 * width, 4.0 - width, 4.0 + width]
        val = 2.0 / math.pi * quad(f, 0.0, 60.0, points=[p for p in pts if 0 < p < 60], limit=400)[0]
        assert windows.alpha_window(np.array([t]), kind, lo, hi, width)[0] == pytest.approx(val, abs=1e-9)


def test_mirrored_triangle_reaching_zero_is_still_the_transform_of_its_target():
    lo, hi, width = 0.5, 1.5, 3.0  # half-base 1.5 > centre 1.0: the mirrored term is active
    for t in (0.0, 0.8, 2.2):
        f = lambda om: windows.target(om, "triangle", lo, hi, width) * math.cos(om * t)  # noqa: E731
        val = 2.0 / math.pi * quad(f, 0.0, 3.0, points=[0.5, 1.0, 2.5], limit=200)[0]
        assert windows.alpha_window(np.array([t]), "triangle", lo, hi, width)[0] == pytest.approx(val, abs=1e-10)


def test_indicator_window_is_eq_weightf():
    tau, L = 0.01, 300
    np.testing.assert_allclose(windows.window_weights("indicator", 10.0, 20.0, tau, L),
                               oracle.discrete_weights(10.0, 20.0, tau, L), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kind,width,atol", [("triangle", 2.0, 5e-3), ("gaussian", 1.0, 2e-3)])
def test_filter_tends_to_the_target(kind, width, atol):
    # beta~ of the truncated, sampled weights -> g as tau -> 0 and T -> inf
    # (the rectangle rule's unhalved first node and the scheme's start leave
    # an O(tau) offset; the triangle's kinks converge like 1/T)
    lo, hi = 10.0, 20.0
    tau, L = 1e-4, 200000
    w = windows.window_weights(kind, lo, hi, tau, L, width)
    om = np.array([5.0, 10.0, 12.5, 15.0, 17.5, 20.0, 25.0])
    np.testing.assert_allclose(oracle.beta_tilde(om, tau, w), windows.target(om, kind, lo, hi, width), atol=atol)
    # the chosen widths put 1/2 at the interval ends
    assert windows.target(np.array([lo, hi]), kind, lo, hi, width) == pytest.approx([0.5, 0.5], abs=1e-6)


def test_notch_weights_are_the_minimum_norm_change_that_zeroes_the_filter():
    tau, L = 0.01, 80
    w = oracle.discrete_weights(30.0, 40.0, tau, L)
    notches = [0.0, 52.5, 61.0]
    wn = windows.notch_weights(w, tau, notches)
    assert np.abs(oracle.beta_tilde(np.array(notches), tau, wn)).max() <= 1e-12 * np.abs(w).sum()
    # minimum norm: the change is the least-squares solution of Q d = -Q w
    Q = np.array([[oracle.q_sequence([om], tau, L)[ell, 0] for ell in range(L)] for om in notches])
    d = np.linalg.lstsq(Q, -Q @ w, rcond=None)[0]
    np.testing.assert_allclose(wn - w, d, atol=1e-12 * np.abs(w).max())
    # and any other change that zeroes the filter is at least as long
    null = np.linalg.svd(Q)[2][len(notches):]
    rng = np.random.default_rng(0)
    for _ in range(5):
        other = (wn - w) + null.T @ rng.standard_normal(null.shape[0]) * 1e-3
        assert np.linalg.norm(other) >= np.linalg.norm(wn - w)
