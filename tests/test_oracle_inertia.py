"""Pins of the oracle's inertia count (Sylvester's law on S - sigma M): the
closed-form spectrum of the grid pencils, a dense generalized eigensolve on
small horn meshes, and a diagonal pencil."""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import inertia
from synth import grid_spectrum
from synth.grids import grid_problem
from synth.horn import horn_pencil


def test_diagonal_pencil_counts_entries_below_sigma():
    d = np.array([3.0, -1.0, 7.0, 2.0, 0.5])
    m = np.array([1.0, 2.0, 1.0, 4.0, 1.0])
    S = sp.diags(d).tocsr()
    for sigma in (-1.0, 0.0, 0.6, 1.0, 5.0, 100.0):
        assert inertia.count_below(S, m, sigma) == int(np.sum(d / m < sigma))


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 12)])
def test_grid_counts_match_closed_form(dim, n):
    S, m, h = grid_problem(dim, n)
    lam = grid_spectrum(dim, n)
    rng = np.random.default_rng(dim)
    for sigma in rng.uniform(lam.min(), lam.max(), 6):
        assert inertia.count_below(S, m, sigma) == int(np.sum(lam < sigma))
    # an interval count with eigenvalues of multiplicity on both ends
    om = np.sqrt(lam)
    lo, hi = om[10], om[40]
    assert inertia.count_in_interval(S, m, lo, hi) == int(np.sum((om >= lo * (1 - 1e-12)) & (om <= hi * (1 + 1e-12))))


@pytest.mark.parametrize("n_c,n_z", [(4, 60), (6, 30)])
def test_horn_counts_match_dense_eigensolve(n_c, n_z):
    S, m = horn_pencil(n_c, n_z)
    lam = sla.eigh(S.toarray(), np.diag(m), eigvals_only=True)
    assert inertia.bandwidth(S) <= (n_c + 1) ** 2 + n_c + 2
    for sigma in np.quantile(lam[1:], [0.01, 0.2, 0.5, 0.9]) * 1.0000001:
        assert inertia.count_below(S, m, sigma) == int(np.sum(lam < sigma))
    om = np.sqrt(np.maximum(lam, 0.0))
    assert inertia.count_in_interval(S, m, 200.0, 600.0) == int(np.sum((om >= 200.0) & (om <= 600.0)))
