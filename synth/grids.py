"""P1 finite-element pencils ``(S, m)`` on simplicial meshes.

Section 2 defines ``s_ij`` as the integral of grad(phi_i).grad(phi_j) and
``m_ij`` as the integral of phi_i*phi_j over the domain, for a Galerkin space of
piecewise polynomials on simplices; Remark 2.1 replaces ``M`` by a diagonal
matrix through mass lumping.  Here the space is P1 and lumping is the row-sum
rule, which for P1 gives every vertex ``|K|/(d+1)`` from each simplex ``K``
containing it.

Two constructions are provided for the uniform unit square/cube:

* ``grid_problem_fem``: genuine element-by-element assembly on a structured
  simplicial mesh (2D: every cell cut along its (0,0)-(1,1) diagonal; 3D: the
  six Kuhn tetrahedra of every cell sharing its main diagonal), Dirichlet
  vertices removed, exact zeros pruned.
* ``grid_problem``: the same matrices written down directly.  For these meshes
  the assembled stiffness is exactly the 5-point stencil (2D, entries 4/-1) and
  ``h`` times the 7-point stencil (3D, entries 6/-1), and the lumped mass is
  ``h^d`` at every interior vertex; the tests check this identity against the
  assembly, and the fast form is used at large sizes where element assembly
  would need gigabytes of COO triplets.

Vertex numbering is lexicographic with the last axis fastest; matrices are CSR
with int32 indices, sorted columns and float64 values.
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _csr32(A: sp.spmatrix) -> sp.csr_matrix:
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    A.data = A.data.astype(np.float64)
    return A


def structured_mesh(dim: int, n: int):
    """Vertices, simplices and boundary flags of the unit square (dim=2) or
    cube (dim=3) with ``n`` cells per axis."""
    if dim not in (2, 3) or n < 1:
        raise ValueError("dim must be 2 or 3 and n >= 1")
    h = 1.0 / n
    ax = np.arange(n + 1)
    grids = np.meshgrid(*([ax] * dim), indexing="ij")
    ids = np.stack([g.ravel() for g in grids], 1)  # (nv, dim) integer coords
    verts = ids.astype(np.float64) * h
    boundary = np.any((ids == 0) | (ids == n), axis=1)

    strides = np.array([(n + 1) ** (dim - 1 - a) for a in range(dim)])
    cells = np.stack([g.ravel() for g in np.meshgrid(*([np.arange(n)] * dim), indexing="ij")], 1)
    base = cells @ strides
    simplices = []
    # every simplex walks from the cell's lowest corner to its highest corner,
    # one axis at a time, in the order given by a permutation of the axes
    perms = list(itertools.permutations(range(dim)))
    for p in perms:
        path = [base]
        cur = base.copy()
        for a in p:
            cur = cur + strides[a]
            path.append(cur)
        simplices.append(np.stack(path, 1))
    simplices = np.concatenate(simplices, 0).astype(np.int64)
    return verts, simplices, boundary


def assemble_p1(verts: np.ndarray, simplices: np.ndarray):
    """Assemble the P1 stiffness matrix and the row-sum lumped mass vector.

    For a simplex with vertices v_0..v_d put the edge vectors e_k = v_k - v_0
    in the rows of E.  The barycentric coordinates are xi = E^{-T}(x - v_0)
    (plus xi_0 = 1 - sum xi_k), so their gradients are the rows of E^{-T} and
    the element stiffness is |K| * G G^T with G the (d+1) x d gradient table.
    """
    verts = np.asarray(verts, dtype=np.float64)
    simplices = np.asarray(simplices, dtype=np.int64)
    d = verts.shape[1]
    P = verts[simplices]  # (ne, d+1, d)
    E = P[:, 1:, :] - P[:, :1, :]  # (ne, d, d)
    det = np.linalg.det(E)
    vol = np.abs(det) / float(np.prod(np.arange(1, d + 1)))
    Ginv = np.linalg.inv(E)  # columns of E^{-1} are rows of E^{-T}
    G = np.empty((E.shape[0], d + 1, d))
    G[:, 1:, :] = np.transpose(Ginv, (0, 2, 1))
    G[:, 0, :] = -G[:, 1:, :].sum(axis=1)
    Ke = vol[:, None, None] * np.einsum("eid,ejd->eij", G, G)
    rows = np.broadcast_to(simplices[:, :, None], Ke.shape).ravel()
    cols = np.broadcast_to(simplices[:, None, :], Ke.shape).ravel()
    nv = verts.shape[0]
    S = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(nv, nv)).tocsr()
    m = np.zeros(nv)
    np.add.at(m, simplices.ravel(), np.repeat(vol / (d + 1), d + 1))
    return _csr32(S), m


def prune(S: sp.csr_matrix, rel: float = 1e-14) -> sp.csr_matrix:
    """Drop entries with |s_ij| <= rel * max_i |s_ii| (round-off zeros that
    the assembly leaves where element contributions cancel)."""
    S = sp.csr_matrix(S, copy=True)
    thr = rel * np.abs(S.diagonal()).max()
    S.data[np.abs(S.data) <= thr] = 0.0
    S.eliminate_zeros()
    return _csr32(S)


def restrict(S: sp.csr_matrix, m: np.ndarray, keep: np.ndarray):
    """Keep only the rows/columns flagged in ``keep`` (removes Dirichlet
    vertices: their values are fixed to zero)."""
    idx = np.flatnonzero(keep)
    return _csr32(S[idx][:, idx]), np.ascontiguousarray(m[idx])


def grid_problem_fem(dim: int, n: int, dirichlet: bool = True):
    """Element-assembled P1 pencil on the structured unit square/cube mesh."""
    verts, simp, bnd = structured_mesh(dim, n)
    S, m = assemble_p1(verts, simp)
    if dirichlet:
        S, m = restrict(S, m, ~bnd)
    return prune(S), m


def _tridiag(k: int) -> sp.csr_matrix:
    return sp.diags([-np.ones(k - 1), 2.0 * np.ones(k), -np.ones(k - 1)], [-1, 0, 1], format="csr")


def grid_problem(dim: int, n: int):
    """Dirichlet P1 pencil on the unit square/cube with ``n`` cells per axis,
    written directly as the stencil the assembly produces (see module doc).

    Returns ``(S, m, h)`` with N = (n-1)^dim unknowns.
    """
    if dim not in (2, 3) or n < 2:
        raise ValueError("dim must be 2 or 3 and n >= 2")
    h = 1.0 / n
    k = n - 1
    T = _tridiag(k)
    I = sp.identity(k, format="csr")
    if dim == 2:
        S = sp.kron(T, I) + sp.kron(I, T)
        scale = 1.0
    else:
        S = sp.kron(sp.kron(T, I), I) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(I, I), T)
        scale = h
    S = _csr32(S * scale)
    m = np.full(k**dim, h**dim)
    return S, m, h


def jittered_problem(dim: int, n: int, jitter: float, seed: int, dirichlet: bool = False):
    """P1 pencil on a structured mesh whose interior vertices are moved by a
    uniform random offset in [-jitter*h, jitter*h]^dim (seeded).  Used for
    small unstructured test problems (Neumann by default, so S is only
    positive semi-definite with the constants in its null space)."""
    verts, simp, bnd = structured_mesh(dim, n)
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    off = rng.uniform(-jitter * h, jitter * h, size=verts.shape)
    verts = verts + np.where(bnd[:, None], 0.0, off)
    S, m = assemble_p1(verts, simp)
    if dirichlet:
        S, m = restrict(S, m, ~bnd)
    return prune(S), m
