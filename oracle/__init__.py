"""CPU FP64 oracle of the filtered time-domain Krylov eigensolver.

TEST INFRASTRUCTURE.  This package is a plain, slow, obviously correct
implementation of what the GPU library computes, written from the paper
(Nannen & Wess, "A Krylov Eigenvalue Solver Based on Filtered Time Domain
Solutions") in FP64 with NumPy/SciPy.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code with the GPU path (the seeded input generators in
``synth`` are the only common dependency, and they hold none of the method's
arithmetic).

Modules and the passages they follow:

* ``weights``   - truncated inverse-Fourier weight (Section 2.2, eq. weightf)
                  and the rectangle-rule coefficients tau*alpha(l*tau)
                  (Section 2.3, eq. disc_filtercoeff).
* ``filter``    - scalar recurrence q_l (Section 2.3, def. scalartimestep) and
                  the fully discrete filter function (Lemma 2.3).
* ``timestep``  - the operator C: explicit two-step scheme (eq. 2stepmethod)
                  with y_{-1} = y_0 = r, weighted by the rectangle rule
                  (eq. disc_filtercoeff).
* ``power``     - power iteration for the largest eigenvalue and the time
                  step / step count rule used by the workloads.
* ``krylov``    - Algorithm 2.5 (Krylov loop), the projected pencil
                  (eq. projevp), residuals (eq. res) and acceptance; a
                  Euclidean basis of the Krylov space (the paper's inner
                  product) and the M-inner CGS2 block form.
* ``subspace``  - the fixed-dimension (FEAST-type) filtered subspace
                  iteration of Section 4.4.
* ``windows``   - the alternative weight functions of Section 4.3.
* ``inertia``   - eigenvalue counts by Sylvester's law of inertia (a banded
                  LDL^T in plain C, ``inertia.c``) for meshes without a closed
                  form spectrum.

Parity status: every function is pinned by CPU tests against closed forms,
invariants or brute force (see ``tests/test_oracle_*.py``); none is
"parity unpinned".
"""

from .weights import alpha, discrete_weights  # noqa: F401
from .filter import q_sequence, beta_tilde  # noqa: F401
from .timestep import apply_filter  # noqa: F401
from .power import power_lambda_max, time_step_rule  # noqa: F401
from .krylov import krylov_basis_euclidean, krylov_solve, rayleigh_ritz, KrylovResult  # noqa: F401
from .subspace import subspace_solve, SubspaceResult  # noqa: F401
