"""The library's Krylov convergence model (kf_predict_steps) and the weight
selection built on it (kf_select_weights) against the oracle's model
(oracle.convergence): host arithmetic through the C ABI."""

import math

import numpy as np
import pytest

import oracle
from oracle import windows
from oracle.convergence import predict_steps as oracle_steps
from synth import grid_spectrum


def _kf():
    from paper_2402_08515_amd import kf

    return kf


def _distinct_cube(n, top):
    lam = np.sort(grid_spectrum(3, n))
    om = np.sqrt(lam[np.concatenate([[True], np.diff(lam) > 1e-10 * lam[1:]])])
    om = om[om <= top]
    return om


@pytest.mark.parametrize("factor", [1, 2, 3])
def test_model_matches_oracle_on_a_cube_spectrum(factor):
    kf = _kf()
    om = _distinct_cube(32, 60.0)
    lo, hi = 20.0, 26.0
    tau = 0.9 * 2 / math.sqrt(grid_spectrum(3, 32).max())
    L = int(math.ceil(2 * math.pi / (lo * tau))) * factor
    w = oracle.discrete_weights(lo, hi, tau, L)
    ref = oracle_steps(om, np.ones(om.size), w, tau, lo, hi, eps=1e-6, kmax=400)
    got = kf.predict_steps(om, np.ones(om.size), w, tau, lo, hi, eps=1e-6, kmax=400)
    assert ref < 400 and abs(got - ref) <= 1


def test_model_exact_cases_and_order4():
    kf = _kf()
    omega = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    w = np.array([0.3, 0.2, -0.1])
    assert kf.predict_steps(omega, np.ones(5), w, 0.1, 0.5, 5.5) == oracle_steps(omega, np.ones(5), w, 0.1, 0.5, 5.5)
    dup = np.array([1.0, 2.0, 2.0, 3.0, 6.0])
    w2 = oracle.discrete_weights(1.5, 2.5, 0.1, 20)
    assert kf.predict_steps(dup, np.ones(5), w2, 0.1, 1.5, 2.5, kmax=50) == 50
    om = _distinct_cube(24, 50.0)
    tau = 3.0 / math.sqrt(grid_spectrum(3, 24).max())
    w4 = oracle.discrete_weights(15.0, 20.0, tau, 30)
    assert abs(kf.predict_steps(om, np.ones(om.size), w4, tau, 15.0, 20.0, kmax=400, stepper=4)
               - oracle_steps(om, np.ones(om.size), w4, tau, 15.0, 20.0, kmax=400, order=4)) <= 1


def test_selection_keeps_fourier_unless_another_is_predicted_faster():
    kf = _kf()
    om = _distinct_cube(32, 60.0)
    lo, hi = 20.0, 26.0
    tau = 0.9 * 2 / math.sqrt(grid_spectrum(3, 32).max())
    L = int(math.ceil(2 * math.pi / (lo * tau)))
    four = oracle.discrete_weights(lo, hi, tau, L)
    gauss = windows.window_weights("gaussian", lo, hi, tau, L, 1.0)
    flat = 0.5 * four  # the same filter scaled: the same Krylov space
    idx, steps = kf.select_weights([four, gauss, flat], tau, lo, hi, om, np.ones(om.size), kmax=600)
    assert steps[2] == steps[0]
    if steps[1] < steps[0]:
        assert idx == 1
    else:
        assert idx == 0
    # a margin keeps the Fourier weights unless the gain exceeds it
    idx2, _ = kf.select_weights([four, gauss], tau, lo, hi, om, np.ones(om.size), kmax=600, margin=0.99)
    assert idx2 == 0
