"""Pins of the oracle's Krylov convergence model: exact termination on a
model spectrum with few distinct filter values, no resolution of points that
share a filter value (a Krylov space of C cannot separate them), and the
measured trend of the 3D benchmark cube's Krylov steps against T."""

import math

import numpy as np

import oracle
from oracle.convergence import predict_steps


def test_terminates_when_the_space_is_invariant():
    # 5 model points with distinct filter values: the Krylov space of a 5 x 5
    # diagonal matrix is the whole space after 5 vectors
    omega = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    w = np.array([0.3, 0.2, -0.1])
    tau = 0.1
    k = predict_steps(omega, np.ones(5), w, tau, 0.5, 5.5)
    assert k == 5


def test_points_with_equal_filter_values_are_never_resolved():
    # two sought points with the same beta~ (the same omega, i.e. a double
    # eigenvalue seen through two model points) stay mixed
    omega = np.array([1.0, 2.0, 2.0, 3.0, 6.0])
    w = oracle.discrete_weights(1.5, 2.5, 0.1, 20)
    assert predict_steps(omega, np.ones(5), w, 0.1, 1.5, 2.5, kmax=50) == 50
    # one point per distinct value (one direction per eigenspace) resolves
    assert predict_steps(np.array([1.0, 2.0, 3.0, 6.0]), np.ones(4), w, 0.1, 1.5, 2.5) <= 4


def test_a_filter_that_vanishes_outside_resolves_the_interval_in_count_plus_one_steps():
    # out-of-band filter values exactly 0: one application removes every
    # out-of-band component, so the Krylov space is the start vector plus the
    # Krylov space of the 3 in-band points (distinct values): 4 vectors
    omega = np.concatenate([np.linspace(1.0, 9.0, 20), [10.0, 11.0, 12.0], np.linspace(13.0, 30.0, 25)])
    beta = np.where((omega >= 10.0) & (omega <= 12.0), 0.0, 0.0)
    beta[20:23] = [0.9, 1.0, 1.1]
    assert predict_steps(omega, np.ones(omega.size), None, 0.1, 9.5, 12.5, beta=beta) == 4
