"""Workload recipes: which pencil, which interval, which seeds.

Every workload is a seeded synthetic stand-in for the kind of problem the
paper solves (Section 3: a 2D Neumann dumbbell with about 10^4 unknowns and a
3D horn in a room with about 1.2 million unknowns, both lumped P1/P2 meshes
that are not available here).  The recipes:

``grid2d_64``   2D unit square, Dirichlet, n=64 cells per axis (3,969 DOFs),
                interval omega in [10, 20], one start vector from seed 0,
                40 Krylov iterations.  Small enough for the oracle.
``grid3d_96``   3D unit cube, Dirichlet, Kuhn P1, n=96 (857,375 DOFs),
                omega in [30, 40], one start vector from seed 1.
``horn_4m``     3D tube + exponential bell, Neumann, jittered P1, block of 16
                start vectors from seed 2, omega in [200, 600].
``batch64``     64 independent square/cube problems of uneven size with their
                own intervals, sampled from seed 3, block width 4.
``grid3d_128``  3D unit cube n=128 (2,048,383 DOFs) with 32 intervals sampled
                from seed 4, for the learned-weight comparison.

Start vectors are iid N(0,1) from ``numpy.random.default_rng(seed)``; the
power-iteration start vector for the time-step rule uses seed+1000.  Random
numbers are always drawn here and handed to both sides, never drawn inside the
method.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .grids import grid_problem


@dataclass
class Problem:
    name: str
    S: sp.csr_matrix
    m: np.ndarray
    omega_min: float
    omega_max: float
    seed: int
    block: int = 1
    precision: str = "fp64"
    krylov: int = 0  # fixed number of Krylov iterations for the recipe (0 = run to target)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.S.shape[0]

    @property
    def nnz(self) -> int:
        return self.S.nnz


def start_block(n: int, b: int, seed: int) -> np.ndarray:
    """Start block V0 (n x b, row-major float64): iid N(0,1) from seed."""
    return np.random.default_rng(seed).standard_normal((n, b))


def power_start(n: int, seed: int) -> np.ndarray:
    """Start vector of the power iteration that sizes the time step."""
    return np.random.default_rng(seed + 1000).standard_normal(n)


def grid_spectrum(dim: int, n: int) -> np.ndarray:
    """All eigenvalues (omega^2, with multiplicity, ascending) of the lumped
    Dirichlet P1 pencil of ``grid_problem(dim, n)``.

    The pencil equals the tensor-product finite-difference Laplacian, whose
    eigenvectors are discrete sine modes; the 1D factor has eigenvalues
    (4/h^2) sin^2(k pi h / 2), k = 1..n-1, and the d-dimensional eigenvalues
    are sums of d such terms.
    """
    h = 1.0 / n
    k = np.arange(1, n)
    mu = 4.0 / h**2 * np.sin(k * np.pi * h / 2) ** 2
    if dim == 2:
        lam = (mu[:, None] + mu[None, :]).ravel()
    else:
        lam = (mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).ravel()
    return np.sort(lam)


def distinct_target(lam: np.ndarray, omega_min: float, omega_max: float, b: int, rtol: float = 1e-10):
    """Number of eigenpairs a block-``b`` Krylov space can deliver in the
    closed interval [omega_min, omega_max]: the sum over distinct eigenvalues of
    min(multiplicity, b).  A block of b start vectors sees at most b directions
    of any eigenspace (the block remedy for multiple eigenvalues the paper
    mentions in its outlook).  Returns (target, distinct values, multiplicities)."""
    lam = np.sort(np.asarray(lam, dtype=np.float64))
    lo, hi = omega_min**2, omega_max**2
    sel = lam[(lam >= lo * (1 - 1e-14)) & (lam <= hi * (1 + 1e-14))]
    if sel.size == 0:
        return 0, np.zeros(0), np.zeros(0, dtype=int)
    vals, mult = [sel[0]], [1]
    for v in sel[1:]:
        if v - vals[-1] <= rtol * v:
            mult[-1] += 1
        else:
            vals.append(v)
            mult.append(1)
    mult = np.array(mult)
    return int(np.minimum(mult, b).sum()), np.array(vals), mult


def _grid(name, dim, n, omin, omax, seed, block=1, precision="fp64", krylov=0):
    S, m, h = grid_problem(dim, n)
    return Problem(name, S, m, float(omin), float(omax), seed, block, precision, krylov,
                   meta={"dim": dim, "n": n, "h": h, "kind": "grid"})


def batch64_descriptors(count: int = 64, seed: int = 3):
    """Sizes and intervals of the uneven batch: square or cube with p=1/2,
    n ~ U{32..256} (2D) or U{16..64} (3D), omega_min ~ U[5,50],
    width ~ U[5,20]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        dim = 2 if rng.random() < 0.5 else 3
        n = int(rng.integers(32, 257)) if dim == 2 else int(rng.integers(16, 65))
        omin = float(rng.uniform(5.0, 50.0))
        width = float(rng.uniform(5.0, 20.0))
        out.append((dim, n, omin, omin + width))
    return out


def batch64_problems(count: int = 64, seed: int = 3):
    """The uneven batch as Problem objects (block width 4, float32 stepping);
    start blocks use seed 3 * 1000 + index."""
    out = []
    for i, (dim, n, omin, omax) in enumerate(batch64_descriptors(count, seed)):
        P = _grid(f"batch64[{i}]", dim, n, omin, omax, seed=seed * 1000 + i, block=4, precision="mixed")
        out.append(P)
    return out


def batch64_slices(max_target: int = 150, count: int = 64, seed: int = 3):
    """The uneven batch with every member's interval cut into slices whose
    block-4 target (distinct eigenvalues, each counted up to 4 times) is at
    most ``max_target``; cuts lie halfway (in omega) between consecutive
    distinct eigenvalues of the closed-form spectrum, so no eigenvalue sits on
    a cut.  Returns [(member index, Problem, omega_lo, omega_hi, target)]; a
    member with a small target is one slice, its own interval."""
    import math

    out = []
    for i, P in enumerate(batch64_problems(count, seed)):
        lam = grid_spectrum(P.meta["dim"], P.meta["n"])
        t, vals, mult = distinct_target(lam, P.omega_min, P.omega_max, P.block)
        if t <= max_target:
            out.append((i, P, P.omega_min, P.omega_max, t))
            continue
        w = np.minimum(mult, P.block)
        cum = np.cumsum(w)
        k = int(math.ceil(t / max_target))
        start_i, start_om = 0, P.omega_min
        for s in range(1, k):
            j = max(int(np.searchsorted(cum, s * t / k)), start_i)
            cut = 0.5 * (math.sqrt(vals[j]) + math.sqrt(vals[j + 1]))
            out.append((i, P, start_om, cut, int(w[start_i:j + 1].sum())))
            start_i, start_om = j + 1, cut
        out.append((i, P, start_om, P.omega_max, int(w[start_i:].sum())))
    return out


def grid3d_128_intervals(count: int = 32, seed: int = 4):
    """Evaluation intervals of the learned-weight comparison: stream 1 of
    seed 4 (stream 0 is reserved for training samples)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[1])
    omin = rng.uniform(5.0, 50.0, size=count)
    width = rng.uniform(5.0, 20.0, size=count)
    return [(float(a), float(a + w)) for a, w in zip(omin, width)]


def workload(name: str) -> Problem:
    if name == "grid2d_64":
        return _grid(name, 2, 64, 10.0, 20.0, seed=0, krylov=40)
    if name == "grid3d_96":
        return _grid(name, 3, 96, 30.0, 40.0, seed=1)
    if name == "grid3d_128":
        return _grid(name, 3, 128, 30.0, 40.0, seed=4, precision="mixed")
    if name == "horn_4m":
        from .horn import horn_problem

        return horn_problem()
    raise KeyError(name)


WORKLOADS = ("grid2d_64", "grid3d_96", "horn_4m", "batch64", "grid3d_128")


def filter_samples(count: int, seed: int = 4, stream: int = 0, lam_range=(5e4, 3e5)) -> np.ndarray:
    """(count, 4) rows (omega_min, omega_max, tau, lambda_max) for the learned
    filter weights: lambda_max log-uniform in lam_range (default [5e4, 3e5],
    the spectral bound of the 3D grids of the workloads),
    tau = 0.9*2/sqrt(lambda_max), omega_min ~ U[5, 50], width ~ U[5, 20].
    Stream 0 of the seed trains, stream 1 evaluates."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[stream])
    lam = np.exp(rng.uniform(np.log(lam_range[0]), np.log(lam_range[1]), size=count))
    tau = 0.9 * 2.0 / np.sqrt(lam)
    omin = rng.uniform(5.0, 50.0, size=count)
    width = rng.uniform(5.0, 20.0, size=count)
    return np.stack([omin, omin + width, tau, lam], axis=1)
