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


def test_horn_mesh_is_valid_and_matches_the_geometry():
    """Small horn: no tetrahedron turns over under the jitter, the mesh
    volume approaches the solid of revolution (the disk map loses a little
    of the circle), the Neumann stiffness annihilates constants, and every
    neighbour lies within one layer of ids (16-bit offsets fit)."""
    import scipy.integrate as si

    from synth.horn import horn_mesh, horn_pencil, radius, tet_volumes

    v0, t4, b = horn_mesh(8, 80, jitter=0.0)
    v1, _, _ = horn_mesh(8, 80)
    a0, a1 = tet_volumes(v0, t4), tet_volumes(v1, t4)
    assert np.all(np.sign(a0) == np.sign(a1)) and np.all(a0 != 0)
    exact = si.quad(lambda z: np.pi * radius(np.array(z)) ** 2, 0.0, 1.7, points=[1.5])[0]
    assert abs(np.abs(a1).sum() - exact) / exact < 0.01
    S, m = horn_pencil(8, 80)
    assert m.min() > 0 and abs(m.sum() - np.abs(a1).sum()) < 1e-15
    assert np.abs(S @ np.ones(S.shape[0])).max() < 1e-12 * S.diagonal().max()
    assert abs(S - S.T).max() < 1e-15 * S.diagonal().max()
    rows = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
    assert np.abs(S.indices - rows).max() <= 9 * 9 + 9 + 1
    # jittered vertices stay off the wall: the wall and caps are unmoved
    assert np.array_equal(v0[b], v1[b]) and not np.array_equal(v0[~b], v1[~b])
