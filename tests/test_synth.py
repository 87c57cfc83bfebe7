"""The input generators: element assembly equals the stencil form, and the
closed-form spectrum of the grid pencils equals a dense eigensolve."""

import numpy as np
import pytest
import scipy.linalg as sla

from synth import distinct_target, grid_spectrum, start_block, workload
from synth.grids import grid_problem, grid_problem_fem, jittered_problem


@pytest.mark.parametrize("dim,n", [(2, 7), (2, 12), (3, 4), (3, 6)])
def test_fem_assembly_equals_stencil(dim, n):
    S1, m1 = grid_problem_fem(dim, n)
    S2, m2, h = grid_problem(dim, n)
    assert S1.nnz == S2.nnz
    assert abs(S1 - S2).max() <= 1e-13 * abs(S2).max()
    np.testing.assert_allclose(m1, m2, rtol=1e-13)
    assert S2.indices.dtype == np.int32 and S2.has_sorted_indices


@pytest.mark.parametrize("dim,n", [(2, 9), (3, 5)])
def test_grid_spectrum_closed_form(dim, n):
    S, m, h = grid_problem(dim, n)
    ev = sla.eigh(S.toarray(), np.diag(m), eigvals_only=True)
    np.testing.assert_allclose(ev, grid_spectrum(dim, n), rtol=1e-12)


def test_neumann_mesh_is_psd_with_constant_null_space():
    S, m = jittered_problem(2, 8, 0.2, seed=3)
    np.testing.assert_allclose(S @ np.ones(S.shape[0]), 0.0, atol=1e-12)
    assert np.all(m > 0)
    assert m.sum() == pytest.approx(1.0, rel=1e-12)  # area of the unit square
    assert (S - S.T).count_nonzero() == 0 or abs(S - S.T).max() < 1e-14


def test_workload_sizes_and_targets():
    P = workload("grid2d_64")
    assert P.n == 3969 and P.nnz == 19593
    assert distinct_target(grid_spectrum(2, 64), 10, 20, 1)[0] == 11
    assert distinct_target(grid_spectrum(3, 96), 30, 40, 1)[0] == 110


def test_start_block_is_seeded():
    a = start_block(100, 3, 5)
    b = start_block(100, 3, 5)
    assert a.shape == (100, 3) and np.array_equal(a, b)
    assert not np.array_equal(a, start_block(100, 3, 6))
