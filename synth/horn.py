"""The horn workload: a straight tube joined to an exponentially flaring
bell, all walls Neumann (the pencil is positive semi-definite, with the
constants as its null space), P1 tetrahedra with lumped mass.

Geometry (the paper's horn without the surrounding room): tube of radius
0.01 along z in [0, 1.5], bell r(z) = 0.01 * 10^((z - 1.5)/0.2) on
[1.5, 1.7] (outlet radius 0.1).

Mesh: an n_c x n_c square grid mapped onto the disk (elliptical grid map
x = s sqrt(1 - t^2/2), y = t sqrt(1 - s^2/2) for s, t in [-1, 1], then
scaled by r(z)) on n_z + 1 uniformly spaced layers; each hexahedral cell is
cut into the six Kuhn tetrahedra sharing its main diagonal.  Interior
vertices (not on the wall or the end caps) are moved by a uniform random
offset in [-0.05 h, 0.05 h]^3, h the shortest edge at the vertex, drawn from
``numpy.random.default_rng(seed)``.  n_c = 16, n_z = 2604 gives 752,845
vertices and 3,999,744 tetrahedra.
"""

from __future__ import annotations

import itertools

import numpy as np

from .grids import _csr32, assemble_p1

TUBE_LEN, BELL_LEN, R0 = 1.5, 0.2, 0.01


def radius(z: np.ndarray) -> np.ndarray:
    return np.where(z <= TUBE_LEN, R0, R0 * 10.0 ** ((z - TUBE_LEN) / BELL_LEN))


def horn_mesh(n_c: int, n_z: int, jitter: float = 0.05, seed: int = 2):
    """Vertices (nv x 3), tetrahedra (ne x 4, int64) and the wall/cap flag."""
    if n_c < 1 or n_z < 1:
        raise ValueError("n_c and n_z must be positive")
    a = np.arange(n_c + 1)
    i = np.arange(n_z + 1)
    # vertex id = (layer * (n_c + 1) + a) * (n_c + 1) + b: layers slowest, so
    # every neighbour lies within one layer of (n_c + 1)^2 ids
    I, A, Bq = np.meshgrid(i, a, a, indexing="ij")
    s = 2.0 * A.ravel() / n_c - 1.0
    t = 2.0 * Bq.ravel() / n_c - 1.0
    z = (TUBE_LEN + BELL_LEN) * I.ravel() / n_z
    r = radius(z)
    x = s * np.sqrt(1.0 - 0.5 * t * t) * r
    y = t * np.sqrt(1.0 - 0.5 * s * s) * r
    verts = np.stack([x, y, z], 1)
    wall = (A.ravel() == 0) | (A.ravel() == n_c) | (Bq.ravel() == 0) | (Bq.ravel() == n_c)
    cap = (I.ravel() == 0) | (I.ravel() == n_z)
    boundary = wall | cap
    # cells and their six Kuhn tetrahedra
    strides = np.array([n_c + 1, 1, (n_c + 1) ** 2], dtype=np.int64)  # axes (a, b, layer)
    ci, ca, cb = np.meshgrid(np.arange(n_z), np.arange(n_c), np.arange(n_c), indexing="ij")
    base = ca.ravel() * strides[0] + cb.ravel() * strides[1] + ci.ravel() * strides[2]
    tets = []
    for p in itertools.permutations(range(3)):
        path = [base]
        cur = base.copy()
        for ax in p:
            cur = cur + strides[ax]
            path.append(cur)
        tets.append(np.stack(path, 1))
    tets = np.concatenate(tets, 0)
    if jitter > 0:
        # shortest incident edge per vertex
        hmin = np.full(verts.shape[0], np.inf)
        for u, v in itertools.combinations(range(4), 2):
            e = np.linalg.norm(verts[tets[:, u]] - verts[tets[:, v]], axis=1)
            np.minimum.at(hmin, tets[:, u], e)
            np.minimum.at(hmin, tets[:, v], e)
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter, jitter, size=verts.shape) * hmin[:, None]
        verts = verts + np.where(boundary[:, None], 0.0, off)
    return verts, tets, boundary


def tet_volumes(verts: np.ndarray, tets: np.ndarray) -> np.ndarray:
    P = verts[tets]
    E = P[:, 1:, :] - P[:, :1, :]
    return np.linalg.det(E) / 6.0


def horn_pencil(n_c: int, n_z: int, jitter: float = 0.05, seed: int = 2):
    """Neumann P1 pencil (S, m) of the horn mesh (S CSR int32/float64)."""
    verts, tets, _ = horn_mesh(n_c, n_z, jitter, seed)
    S, m = assemble_p1(verts, tets)
    return _csr32(S), m


def horn_problem(n_c: int = 16, n_z: int = 2604, seed: int = 2):
    from .workloads import Problem

    S, m = horn_pencil(n_c, n_z, 0.05, seed)
    return Problem("horn_4m" if (n_c, n_z) == (16, 2604) else f"horn_{n_c}x{n_z}", S, m, 200.0, 600.0, seed,
                   block=16, precision="mixed", meta={"kind": "horn", "n_c": n_c, "n_z": n_z})
