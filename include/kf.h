/*
 * kf.h - filtered time-domain Krylov eigensolver for S v = omega^2 M v on
 * AMD Instinct MI355X (gfx950).
 *
 * Method (Nannen & Wess, "A Krylov Eigenvalue Solver Based on Filtered Time
 * Domain Solutions"):
 *   - Section 2 (eq. def:basisMatrixEVP): S symmetric positive semi-definite,
 *     M symmetric positive definite; Remark 2.1: M is diagonal (mass lumping),
 *     passed here as the vector m_diag.
 *   - Section 2.3 (eq. 2stepmethod, eq. disc_filtercoeff): the operator
 *     C r = sum_{l=0}^{L-1} tau*alpha(l*tau) y_l with y_{-1} = y_0 = r and
 *     y_{l+1} = -tau^2 M^{-1} S y_l + 2 y_l - y_{l-1}.
 *   - Section 2.2 (eq. weightf): the default weights alpha are the truncated
 *     inverse cosine transform of the indicator of [omega_min, omega_max],
 *     with T = L*tau.
 *   - Algorithm 2.5 and Section 2.1 (eq. projevp): Krylov space of C,
 *     projection of the pencil onto it; Section 2.4 (eq. res): residuals and
 *     acceptance.
 *
 * Conventions for every entry point:
 *   - All functions return KF_OK (0) or a positive KF_E* code; on error
 *     kf_last_error() returns a message for the calling thread, and no output
 *     argument is written except where stated.
 *   - Matrices are CSR with int32 row pointers and column indices (sorted,
 *     in range, no duplicates) and float64 values.  Dense blocks are N x b
 *     row-major float64 unless stated.
 *   - Host pointers are read during the call only.  Device pointers (flag
 *     on_device, or where stated) must stay valid for the call; the library
 *     keeps its own device copies of everything it needs afterwards.
 *   - Work is issued on kf_options.stream (a hipStream_t; NULL = the legacy
 *     default stream) and functions return after it has completed, unless
 *     stated otherwise.
 *   - Handles are not thread-safe; distinct handles may be used concurrently
 *     from different threads.
 */
#ifndef KF_H
#define KF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum kf_status {
  KF_OK = 0,
  KF_EINVAL = 1,      /* invalid argument (shape, range, NaN, unsorted CSR, ...) */
  KF_ENOMEM = 2,      /* device or host allocation failed */
  KF_EHIP = 3,        /* a HIP runtime call failed */
  KF_EUNSTABLE = 4,   /* time stepping diverged: tau violates tau < 2/omega_max
                         (Section 2.3, CFL condition), or a non-finite value */
  KF_EBREAKDOWN = 5,  /* informational: the Krylov space became invariant
                         (Algorithm 2.5, zero vector); results are valid */
  KF_ENOTCONV = 6     /* informational: m_max / max_iters reached before the
                         target count was accepted; results are valid */
};

enum kf_precision {
  KF_FP64 = 0,  /* time stepping, accumulation and projection in float64 */
  KF_MIXED = 1  /* time stepping and the filter sum in float32;
                   orthogonalisation, Rayleigh-Ritz and residuals in float64 */
};

typedef struct kf_csr {
  int32_t n;             /* number of rows = columns = DOFs, >= 1 */
  int64_t nnz;           /* number of stored entries, rowptr[n] */
  const int32_t* rowptr; /* n+1 entries, rowptr[0] = 0, non-decreasing */
  const int32_t* col;    /* nnz column indices, strictly increasing per row */
  const double* val;     /* nnz values, finite */
  int32_t on_device;     /* 0: the three arrays (and m_diag) are host memory;
                            1: they are device memory */
} kf_csr;

typedef struct kf_options {
  int32_t precision;     /* kf_precision */
  int32_t check_every;   /* Rayleigh-Ritz every this many Krylov iterations
                            (>= 1); the final state is always checked */
  double check_growth;   /* additionally wait until the basis has grown by
                            this fraction since the last check (0: no wait);
                            once pairs have converged the wait is halved, and
                            it is shortened further when the residuals of the
                            missing pairs predict convergence sooner; checks
                            cost O(k^3) in the basis size k */
  int32_t full_reorth;   /* 1: classical Gram-Schmidt twice against the whole
                            basis; 0: once against the last two blocks (C is
                            M-self-adjoint, so the filtered block is
                            orthogonal to the older ones in exact arithmetic)
                            then once against the whole basis, a second time
                            only when that pass removed over half the norm */
  int32_t target;        /* stop once this many pairs are accepted (0: never);
                            a basis of k columns holds at most k Ritz pairs,
                            so no check runs before it has target columns */
  int32_t max_iters;     /* cap on filter applications (0: none) */
  double drop_tol;       /* a new column whose M-norm after orthogonalisation
                            is <= drop_tol times its M-norm before is dropped
                            (breakdown test of Algorithm 2.5 with a tolerance);
                            0 selects 1e-10 */
  double reorth_tol;     /* full_reorth 0: at a projection onto the whole
                            basis the coefficients are always computed (they
                            are needed for B^T S B), but subtracted only when
                            one exceeds reorth_tol times its column's M-norm; with the pending-column check
                            of proj_every the basis stays M-orthonormal to
                            about 1e-7 (reported as kf_result.orth_error);
                            0 = always subtract */
  int32_t proj_every;    /* float64 stepping, full_reorth 0: the
                            projection onto the whole basis (which forms the
                            new columns of B^T S B and B^T M B and the
                            orthogonalisation coefficients) runs every
                            proj_every steps, and at the latest when 16
                            columns would be pending; in between a step is
                            orthogonalised against the last two columns or
                            blocks only (three-term form; a block is then
                            orthonormalised by Cholesky QR twice).  For a
                            single vector a projection cleans the new column
                            and the last column of the previous interval
                            (both feed the next step).  Columns found
                            more than 1e-7 off M-orthogonal at a projection
                            are orthogonalised
                            again and proj_every is halved from then on (a
                            check repairs such columns without halving).  The
                            Rayleigh-Ritz step corrects to first order for the
                            remaining non-orthogonality (E = B^T M B - I: the
                            eigenvalues of H - (E H + H E)/2); 1 = every step */
  int32_t refine;        /* KF_MIXED only: at most this many iterations of
                            the float64 refinement (0 = none, and no float64
                            operator is kept): the filtered subspace
                            iteration (Section 4.4) in float64 started from
                            the Ritz vectors of the float32 Krylov space near
                            the interval; it stops once the target is met */
  int32_t escalate;      /* KF_MIXED, solves with a target: when the float64
                            refinement misses the target although the float32
                            loop reached it (float32 round-off seeds, at every
                            step, directions of eigenspaces of multiplicity
                            above b that pollute the Ritz vectors of other
                            eigenvalues where the filter cannot tell them
                            apart), or as soon as a check of the float32 loop
                            accepts more than b copies of one eigenvalue (the
                            symptom of that seeding), 1 = the Krylov loop
                            starts again from the start block with float64
                            stepping (kf_result.escalated), so the target is
                            still met; 0 = up to 4 further refinements
                            instead */
  int32_t want_vectors;  /* kf_result.vectors is filled when nonzero */
  int32_t index_bytes;   /* column-index width of the device operator:
                            0 = automatic (2 when every |col - row| < 32768),
                            2 or 4 */
  int32_t xcd_remap;     /* 1: map consecutive row slices to the same XCD */
  int32_t nt_loads;      /* 1: stream the operator with non-temporal loads in
                            the fused time step */
  int32_t autotune;      /* 1: kf_create times the fused step with every
                            combination of xcd_remap, nt_loads and (when both
                            fit) 2- and 4-byte column indices and keeps the
                            fastest, then gather_unroll 2, 3, 4 and 6 when it
                            is 0 (kf_get_tuning reports the choice); blocks of
                            b > 1 vectors also get lanes_per_row and
                            block_band timed on first use */
  int32_t batch_workers; /* batches: host threads that drive the members'
                            Gram-Schmidt and Rayleigh-Ritz between two batched
                            filter launches, each member on a stream of its
                            own (0 = min(8, P); 1 = one after another on the
                            batch stream) */
  int32_t lanes_per_row; /* lanes of a wavefront sharing one row in the fused
                            step for b > 1 (1, 2 or 4, capped at b); 0 =
                            16 bytes of the block row per lane */
  int32_t gather_unroll; /* single vectors: unroll factor (2, 3, 4 or 6) of
                            the fused step's loop over the stored entries of
                            a row slice; 0 = timed by the autotuner (4
                            without it).  Other values: KF_EINVAL */
  int32_t block_band;    /* blocks (b > 1): 1 = each workgroup of the fused
                            step first copies its rows of the current block,
                            and the rows within the operator's largest
                            |col - row| of them, into LDS and gathers from
                            there, whenever that copy fits in 64 KB; -1 =
                            gathers from the caches; 0 = timed with
                            lanes_per_row when autotune is on (else from the
                            caches).  Other values: KF_EINVAL */
  int32_t stepper;       /* time-stepping scheme (Remark 2.4, Section 4.2: any
                            explicit scheme that is a function of M^{-1} S):
                            2 = leapfrog, eq. 2stepmethod (stable for
                            tau omega_max < 2); 4 = its fourth-order variant
                            y+ = 2y - y- - A y + A^2 y / 12, A = tau^2 M^{-1} S
                            (two products with S per step, stable for
                            tau omega_max < sqrt(12)); 0 = 2.  The filter of
                            Lemma 2.3 uses the scheme's scalar recurrence
                            (factor 2 - x + x^2/12, x = tau^2 omega^2, for 4).
                            Batches: 2 only */
  int32_t overlap_checks; /* kf_solve in KF_FP64 with a target: 1 = a
                            Rayleigh-Ritz check that is not expected to be
                            the last one runs on a second stream and host
                            thread while the Krylov loop goes on (its result
                            is taken at a later step; once it meets the
                            target the basis is cut back to the size it
                            checked, and the filter applications made
                            meanwhile are counted in krylov_steps);
                            0 = every check stops the loop until it ends */
  int32_t multistep;     /* single vectors, stepper 2: the time loop as a
                            matrix-powers kernel for banded operators (every
                            stored entry within a band of rows around the
                            diagonal, as a natural grid or axial ordering
                            gives): each workgroup keeps its rows, the rows
                            the next s steps reach and its part of the
                            weighted sum in LDS and advances s steps per
                            launch.  0 = one step per launch (default);
                            s > 0 = s steps per launch; -1 = the whole filter
                            in one launch.  KF_EINVAL from the solve or
                            filter call when the band does not fit;
                            blocks (b > 1) step one step per launch */
  void* stream;          /* hipStream_t */
} kf_options;

typedef struct kf_problem kf_problem; /* opaque */

/* Result of a solve.  The accepted pairs are the Ritz pairs of the projected
 * pencil (Section 2.1, eq. projevp) whose omega lies in [omega_min,
 * omega_max] and whose residual (Section 2.4, eq. res, taken relative to
 * ||S v||_2) is at most tol; the stopping rule after eq. res.  Library-owned
 * until kf_result_free; every array is host memory. */
typedef struct kf_result {
  int64_t n;              /* DOFs */
  int32_t n_pairs;        /* accepted eigenpairs */
  double* omega2;         /* [n_pairs] accepted eigenvalues omega^2, ascending */
  double* omega;          /* [n_pairs] sqrt(omega2) */
  double* residual;       /* [n_pairs] ||S v - omega^2 M v||_2 / ||S v||_2 */
  double* vectors;        /* [n x n_pairs] column-major, M-normalised Ritz
                             vectors, or NULL unless want_vectors */
  int32_t n_ritz;         /* size of the projected pencil at the last check */
  double* ritz;           /* [n_ritz] all Ritz values omega^2, ascending */
  int32_t krylov_steps;   /* filter applications performed */
  int32_t basis_size;     /* columns of the Krylov basis B */
  int32_t breakdown;      /* 1 when the space became invariant */
  int32_t status;         /* KF_OK, KF_EBREAKDOWN or KF_ENOTCONV */
  int64_t leapfrog_vector_steps; /* sum over filter applications of b*(L-1) */
  double t_total;         /* seconds, whole kf_solve */
  double t_leapfrog;      /* seconds in the fused time-stepping kernels */
  double t_gs;            /* seconds in orthogonalisation */
  double t_rr;            /* seconds in projection updates, eigensolves and
                             residuals */
  double t_refine;        /* seconds in the mixed-mode refinement */
  double orth_error;      /* max |B^T M B - I| over the columns checked */
  int32_t full_passes;    /* Gram-Schmidt subtractions over the whole basis */
  int64_t refine_vector_steps; /* vector time steps of the float64 refinement
                                  (KF_MIXED), not in leapfrog_vector_steps for
                                  kf_solve; included in it for
                                  kf_subspace_solve */
  int32_t escalated;      /* 1 when the solve restarted with float64
                             stepping (kf_options.escalate) */
  double t_rr_overlapped; /* device seconds of the Rayleigh-Ritz checks that
                             ran beside the Krylov loop
                             (kf_options.overlap_checks; not in t_rr) */
  int32_t overlapped_checks; /* how many of the checks did */
} kf_result;

/* Fill *opt with defaults: KF_FP64, check_every 1, check_growth 0.3, three-term
 * orthogonalisation (full_reorth 0), no target, no cap,
 * drop_tol 1e-10, reorth_tol 1e-9, proj_every 12, refine 8, escalate 1, stepper 2, no vectors, automatic index width, XCD remap on,
 * cached operator loads, no autotuning, lanes_per_row 0,
 * default stream. */
void kf_default_options(kf_options* opt);

/* Thread-local message describing the last error (never NULL). */
const char* kf_last_error(void);

/* Build a problem for the pencil (S, diag(m_diag)), the interval
 * [omega_min, omega_max] (0 <= omega_min < omega_max), time step tau > 0 and
 * L >= 1 rectangle-rule nodes (T = L*tau).  Copies and validates the inputs,
 * builds the scaled operator A = tau^2 M^{-1} S on the device (float64, plus a
 * float32 copy in KF_MIXED) and sets the default weights of eq. weightf.
 * opt may be NULL (defaults).  *out receives a handle owned by the caller,
 * released with kf_destroy. */
int kf_create(const kf_csr* S, const double* m_diag, double omega_min, double omega_max,
              double tau, int32_t L, const kf_options* opt, kf_problem** out);

/* Release a handle and all its device memory.  NULL is accepted. */
int kf_destroy(kf_problem* p);

/* The dense symmetric eigensolver that kf_solve applies to the projected
 * pencil of eq. projevp (Section 2.1; the basis is M-orthonormal up to
 * E = B^T M B - I, so the pencil is the symmetric matrix
 * B^T S B - (E B^T S B + B^T S B E)/2 to second order): Householder tridiagonalisation,
 * bisection, inverse iteration, back-transformation, all on the GPU.
 * A: host k x k column-major (the two triangles are averaged), 1 <= k <= 2048.
 * theta[k] (host) receives all eigenvalues ascending.  If Y != NULL, the
 * eigenvectors (unit 2-norm) of the eigenvalues in [lo, hi] go to Y (host,
 * k x *n_sel column-major; capacity k*k) and their count to *n_sel.
 * Works on `stream` (hipStream_t, NULL = default); blocks until done.
 * Errors: KF_EINVAL (size, NULL, non-finite entries), KF_ENOMEM, KF_EHIP. */
int kf_sym_eig(int32_t k, const double* A, double lo, double hi, double* theta, int32_t* n_sel, double* Y,
               void* stream);

/* The fused-step variant in use: XCD remap, non-temporal operator loads,
 * column-index bytes, the single-vector unroll factor, and (after
 * autotuning) its time per step in microseconds for one vector (0 when not
 * tuned).  NULL outputs are skipped. */
int kf_get_tuning(const kf_problem* p, int32_t* xcd_remap, int32_t* nt_loads, int32_t* index_bytes,
                  int32_t* gather_unroll, double* us_per_step);

/* Replace the L filter coefficients w_l = tau*alpha(l*tau) (host array of
 * exactly L finite values; Section 2.2 allows any weight function). */
int kf_set_weights(kf_problem* p, const double* w, int32_t L);

/* Copy the current L filter coefficients to the host array w_out[L]. */
int kf_get_weights(const kf_problem* p, double* w_out);

/* Section 3.1.2 and Section 3.2: the stable time step comes from a power
 * iteration and the CFL condition of eq. 2stepmethod.
 * Largest eigenvalue estimate of M^{-1} S by `iters` power iterations from the
 * start vector x0[n] (host, or device when S->on_device), normalised in the
 * M-norm each iteration; *out = Rayleigh quotient x^T S x / x^T M x of the
 * last iterate.  Runs on `stream` (NULL = default).  S is validated as in
 * kf_create; the library allocates and frees its own device copies.
 * Errors: KF_EINVAL (NULL, iters < 0, invalid CSR or mass, a start vector
 * that vanishes or diverges), KF_ENOMEM, KF_EHIP. */
int kf_estimate_lambda_max(const kf_csr* S, const double* m_diag, int32_t iters, const double* x0,
                           void* stream, double* out);

/* The time-step rule used with the estimate: tau = safety*2/sqrt(lambda_est)
 * (CFL condition tau < 2/omega of Section 2.3) and L = ceil(2*pi/(omega_min*tau)),
 * i.e. T covers one period of the lowest sought frequency.  Host arithmetic. */
int kf_time_step_rule(double lambda_est, double omega_min, double safety, double* tau, int32_t* L);

/* ---- alternative weight functions (Section 4.3) --------------------------
 * Section 2.2 builds the weight as the inverse cosine transform of a target
 * function g on the frequency axis, alpha(t) = (2/pi) int_0^inf g(omega)
 * cos(omega t) d omega (eq. filterf, the indicator of the interval), truncated
 * at T = L tau (eq. weightf); Section 4.3 names smoother or more localised
 * targets and weights adapted to the spectrum.  With c = (omega_min +
 * omega_max)/2 and d = (omega_max - omega_min)/2:
 *   KF_WINDOW_INDICATOR: eq. weightf (width unused);
 *   KF_WINDOW_TRIANGLE:  g = max(0, 1 - |omega - c|/h) + the same at -c,
 *                        h = width*d (width 2: g = 1/2 at the interval ends);
 *   KF_WINDOW_GAUSSIAN:  g = exp(-(omega - c)^2/(2 sigma^2)) + the same at -c,
 *                        sigma = width*d/sqrt(2 ln 2) (width 1: g = 1/2 at the
 *                        ends).
 * The mirrored term makes the transform exact in closed form; it only
 * matters when the peak reaches omega = 0.  w_out[l] = tau*alpha(l tau),
 * l < L (eq. disc_filtercoeff), host memory; pass them to kf_set_weights. */
enum kf_window { KF_WINDOW_INDICATOR = 0, KF_WINDOW_TRIANGLE = 1, KF_WINDOW_GAUSSIAN = 2 };
int kf_window_weights(int32_t kind, double omega_min, double omega_max, double tau, int32_t L, double width,
                      double* w_out);

/* Spectrum-adapted weights (Section 4.3: make |beta~| small where unwanted
 * eigenvalues of high multiplicity, or an essential spectrum, are expected):
 * the weights nearest to w[L] in the 2-norm whose discrete filter of
 * Lemma 2.3 vanishes at the k frequencies omega[k] (0 <= k <= min(64, L)),
 * beta~(omega_j) = sum_l w_out[l] q_l(omega_j) = 0.  Host arrays; w_out may
 * equal w.  KF_EINVAL for (nearly) dependent constraints (repeated
 * frequencies). */
int kf_notch_weights(const double* w, int32_t L, double tau, const double* omega, int32_t k, double* w_out);

/* ---- a model of the Krylov iteration's convergence --------------------
 * Section 2.2 asks for |beta~| large on the sought and small on the unsought
 * frequencies; Section 3.1.3 shows that the filter alone does not predict the
 * steps the iteration needs.  In the eigenbasis of the pencil C is the
 * diagonal matrix diag(beta~(omega_j)) (Lemma 2.3); the model runs the Krylov
 * iteration on it for a model spectrum: M points omega[M] (>= 0) standing
 * for weight[M] (> 0) eigenvalues each (a start vector has components
 * sqrt(weight_j)), orthonormal basis by Gram-Schmidt twice.  A sought point
 * (omega in [omega_min, omega_max]) is resolved once its unit direction lies
 * in the space to within eps; *steps receives the first dimension at which
 * all are (kmax when some never are, e.g. two sought points with equal
 * filter values; 0 when none is sought).  Unsought points are merged into
 * 2048 classes of nearly equal filter value (the iteration of a diagonal
 * matrix cannot tell equal values apart), so the cost is O((n_sought +
 * 2048) steps^2) host arithmetic whatever M is.
 * The model spectrum is the caller's: a closed form, a spectral density,
 * the Ritz values of an earlier solve; points standing for a block-b
 * iteration count each eigenvalue's multiplicity up to b.
 * w[L]: filter coefficients, stepper 2 or 4 (kf_options.stepper).
 * Errors: KF_EINVAL (sizes, M x kmax > 2^31, non-positive weight). */
int kf_predict_steps(const double* omega, const double* weight, int32_t M, const double* w, int32_t L, double tau,
                     int32_t stepper, double omega_min, double omega_max, double eps, int32_t kmax, int32_t* steps);

/* The weight set to use among n_cand candidates (candidates[c][L], the same
 * L and tau): candidate 0, by convention the Fourier weights of eq. weightf,
 * unless the model above predicts another to need fewer than (1 - margin)
 * times its steps; then the one with the fewest.  *chosen receives the index,
 * steps[n_cand] (optional) each prediction. */
int kf_select_weights(const double* const* candidates, int32_t n_cand, int32_t L, double tau, int32_t stepper,
                      double omega_min, double omega_max, const double* omega, const double* weight, int32_t M,
                      double eps, int32_t kmax, double margin, int32_t* chosen, int32_t* steps);

/* Discrete filter function of Lemma 2.3, beta~(omega) = sum_l w_l q_l(omega),
 * at n points omega[n] (host) into beta_out[n] (host). */
int kf_filter_response(const kf_problem* p, const double* omega, int32_t n, double* beta_out);

/* y = C x for a block of b columns (1 <= b <= 16): x and y are DEVICE
 * pointers to n x b row-major float64 blocks (they may not overlap).  The time
 * stepping runs in the problem's precision.  Asynchronous on the problem's
 * stream: returns after enqueueing. */
int kf_apply_filter(kf_problem* p, const double* x, double* y, int32_t b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = C x as kf_apply_filter, with its three n x pow2(b) time-stepping blocks
 * taken from a fixed array of 64 MiB that the library holds on every GPU it
 * runs on until the process ends, instead of memory it allocates.  Calls no
 * hipMalloc, hipFree or other allocating routine and does not time block
 * variants (it uses the one kf_create or earlier calls chose).
 * Limit: 3 * n * pow2(b) * value bytes (8 for KF_FP64, 4 for KF_MIXED) must
 * not exceed 64 MiB, else KF_EINVAL (float64, b = 1: n <= 2,796,202).
 * The current device must be the one kf_create ran on (else KF_EINVAL).
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * GPU (other streams, other threads) race.  Every value the kernels read from
 * the array is written first in the same call, so nothing needs clearing.
 * x, y: DEVICE pointers to n x b row-major float64 blocks, 1 <= b <= 16.
 * Asynchronous on the problem's stream. */
int kf_apply_filter_noalloc(kf_problem* p, const double* x, double* y, int32_t b);

/* Algorithm 2.5 with the block remedy of Section 4.4: the Krylov space of C
 * (Section 2.1, def. ArnoldiEWP) grown from the start block, the pencil
 * projected onto it (eq. projevp), residuals and acceptance (Section 2.4,
 * eq. res and the stopping rule after it).
 * Run the eigensolver from the start block start[n x b] (row-major, in host
 * or device memory, 1 <= b <= 16) until opt.target pairs are accepted
 * (residual <= tol), the basis reaches m_max columns, opt.max_iters filter
 * applications, or breakdown.  *out receives a library-owned result released
 * with kf_result_free.  Synchronous.  Errors: KF_EINVAL (NULL, b or m_max
 * out of range (m_max <= 2048), tol <= 0, non-finite or zero start block),
 * KF_EUNSTABLE (the time stepping diverged), KF_ENOMEM, KF_EHIP; the result
 * status KF_EBREAKDOWN / KF_ENOTCONV is informational. */
int kf_solve(kf_problem* p, const double* start, int32_t b, int32_t m_max, double tol,
             kf_result** out);

/* Section 4.4: the fixed-dimension variant of the method, a FEAST-type
 * filtered subspace iteration.  The block X of ncols columns (start: n x ncols
 * row-major, host or device memory, 1 <= ncols <= 2048) is replaced, at each
 * iteration, by an M-orthonormal basis of span(C X) (Section 2.3 operator;
 * directions of relative size below 1e-6 dropped); the pencil is projected
 * onto it (eq. projevp) and the Ritz pairs with omega in [omega_min,
 * omega_max] get residuals (eq. res, relative to ||S v||_2); those <= tol are
 * accepted.  Stops after max_iters iterations, when opt.target pairs are
 * accepted (every copy of a multiple eigenvalue counts: the space holds
 * them all), or (target 0) when every Ritz value inside the interval is
 * accepted and their number did not change since the previous iteration.
 * ncols should exceed the number of eigenvalues in the interval (with
 * multiplicity); the convergence factor of a pair is |beta~| of the first
 * eigenvalue left out of the space over its own |beta~| (Lemma 2.3).
 * KF_MIXED: float32 stepping until the pairs reach the float32 floor, then
 * float64 stepping (when the problem keeps a float64 operator, refine != 0).
 * krylov_steps counts iterations, basis_size the final dimension; status
 * KF_ENOTCONV when the stop test was not met.  Synchronous.
 * Errors: KF_EINVAL (NULL, sizes, tol <= 0, non-finite start), KF_ENOMEM,
 * KF_EUNSTABLE, KF_EHIP. */
int kf_subspace_solve(kf_problem* p, const double* start, int32_t ncols, int32_t max_iters, double tol,
                      kf_result** out);

/* The end time T = L tau by experiment.  Section 3.1.3 shows that a longer
 * T separates the sought eigenvalues better and needs fewer Krylov steps but
 * not always fewer time steps in total, and that the filter alone does not
 * predict which T is cheaper; the conclusion notes that the method's
 * parameters can be optimised experimentally at negligible cost next to
 * repeated solves.  For each of the n_cand step counts L_cand[c] (>= 1) the
 * problem is created with opt (opt->target should be set) and solved from
 * start (as kf_solve: n x b row-major, host or device memory); *L_best
 * receives the L whose solve met the target in the shortest time.
 * seconds[c] and krylov_steps[c] (optional, n_cand entries) receive each
 * solve's time (-1 when the target was missed) and filter applications.
 * Errors: as kf_create and kf_solve; KF_ENOTCONV when no candidate met the
 * target. */
int kf_tune_steps(const kf_csr* S, const double* m_diag, double omega_min, double omega_max, double tau,
                  const int32_t* L_cand, int32_t n_cand, const double* start, int32_t b, int32_t m_max, double tol,
                  const kf_options* opt, int32_t* L_best, double* seconds, int32_t* krylov_steps);

/* Release a result (NULL accepted). */
int kf_result_free(kf_result* r);

/* The basis B_m of Algorithm 2.5 (its output; the span of the Krylov space
 * of Section 2.1) left by the last kf_solve on this handle.
 * Copy up to max_cols columns of the current Krylov basis B (n x k,
 * M-orthonormal to the level reported as kf_result.orth_error) to host memory
 * out[n x max_cols] column-major; *ncols receives the number copied.
 * Errors: KF_EINVAL (NULL, max_cols < 0), KF_EHIP. */
int kf_copy_basis(const kf_problem* p, double* out, int32_t max_cols, int32_t* ncols);

/* ---- batches of independent problems (one batched time-stepping launch) ----
 * Every member is a full problem (kf_create semantics); the time loops of all
 * members advance together: one filter application of the whole batch is a
 * captured graph of max(L)-1 fused-step launches over the stacked
 * (block-diagonal) operator, replayed once per Krylov iteration.
 * Orthogonalisation and Rayleigh-Ritz run per member, on one stream per
 * member driven by kf_options.batch_workers host threads. */
typedef struct kf_problem_desc {
  kf_csr S;
  const double* m_diag;  /* host (or device, with S.on_device) */
  double omega_min, omega_max, tau;
  int32_t L;
  int32_t target;        /* per-member stop count (0: run to m_max) */
  int32_t step_fp64;     /* KF_MIXED batches: 1 = this member steps in
                            float64 from the start (the batch's float64
                            stack), for members whose interval holds
                            eigenvalues of multiplicity above the block width,
                            which float32 stepping cannot resolve (see
                            kf_options.escalate); 0 = the batch's precision */
} kf_problem_desc;

typedef struct kf_batch kf_batch; /* opaque */

/* Create a batch of P (1..256) members from descs[P]; opt applies to every
 * member (its stream and target are ignored: the batch owns one stream).
 * *out is released with kf_destroy_batch. */
int kf_create_batch(int32_t P, const kf_problem_desc* descs, const kf_options* opt, kf_batch** out);

/* Release a batch (NULL accepted). */
int kf_destroy_batch(kf_batch* bt);

/* y_p = C_p x_p for every member p in one batched application: x[p], y[p]
 * are DEVICE pointers to n_p x b COLUMN-major float64 blocks (leading
 * dimension n_p), 1 <= b <= 16.  Synchronous. */
int kf_batch_apply_filter(kf_batch* bt, const double* const* x, double* const* y, int32_t b);

/* Algorithm 2.5 (with the block remedy of Section 4.4) for every member,
 * exactly as kf_solve, with the time loops of all members (eq. 2stepmethod,
 * eq. disc_filtercoeff) advancing in one batched launch sequence.
 * Solve every member from its host start block starts[p] (n_p x b
 * row-major); results[P] receives one library-owned result per member
 * (release each with kf_result_free).  t_leapfrog of every result is the time
 * of the batched time stepping of the whole batch.  Synchronous.  Errors:
 * as kf_solve, prefixed with the failing member's index; on error no result
 * is returned (results[p] = NULL for every p). */
int kf_solve_batch(kf_batch* bt, const double* const* starts, int32_t b, int32_t m_max, double tol,
                   kf_result** results);

/* Replace the filter coefficients of member q (as kf_set_weights; exactly the
 * member's L values, host array) in the batch's device weight table.
 * Errors: KF_EINVAL (index, count, non-finite values), KF_EHIP. */
int kf_batch_set_weights(kf_batch* bt, int32_t q, const double* w, int32_t L);

/* ---- learned filter weights -------------------------------------------------
 * Section 2.2 leaves the weight function free and names the goal |beta|
 * large on the sought omega and small elsewhere.  A small network maps the
 * normalised data (a = tau*omega_min, c = tau*omega_max,
 * x_max = tau*sqrt(lambda_max)/2, L) to the L coefficients as a correction of
 * the Fourier weights of eq. weightf; it is trained to minimise the quadratic
 * leakage of the filter of Lemma 2.3 on a grid of x = tau*omega/2 (band
 * [a/2, c/2] towards 1, outside the band widened by pi/(2L) towards 0).
 * Network products run on the matrix cores in bfloat16 with float32
 * accumulation.  Parameters are float32, count kf_mlp_param_count(), layout
 * W1[64x128] b1[128] W2[128x128] b2 W3[128x128] b3 W4[128x512] b4[512]
 * (row-major, input x output). */
typedef struct kf_mlp kf_mlp; /* opaque */

int32_t kf_mlp_param_count(void);

/* Create a network from host parameters (copied). */
int kf_mlp_create(const float* params, kf_mlp** out);
int kf_mlp_destroy(kf_mlp* net);
/* Copy the current parameters to host out[kf_mlp_param_count()]. */
int kf_mlp_get_params(const kf_mlp* net, float* out);

/* Mean loss over n samples (host, n x 4 rows omega_min, omega_max, tau,
 * lambda_max; n a multiple of 64) and, if grad != NULL, its gradient
 * (host float32 array of the parameter count). */
int kf_mlp_loss_grad(kf_mlp* net, const double* samples, int32_t n, double* loss, float* grad);

/* Adam training (beta1 0.9, beta2 0.999, learning rate lr decayed by a cosine
 * to lr/100) for `epochs` passes over n host samples in the order
 * order[epochs x n] (a permutation per epoch, drawn by the caller), batches
 * of `batch` (multiple of 64, <= n).  epoch_loss[epochs] (optional) receives
 * the mean training loss of each epoch. */
int kf_mlp_train(kf_mlp* net, const double* samples, int32_t n, const int32_t* order, int32_t epochs,
                 int32_t batch, double lr, double* epoch_loss);

/* The network's filter coefficients for n samples (host, n x 4 rows
 * omega_min, omega_max, tau, lambda_max; each needs L = ceil(2 pi /
 * (tau omega_min)) <= 512) without the acceptance gate: w_out (host,
 * n x 512 row-major) receives w_Fourier + 0.01 * network output, zero from
 * l = L on (Section 2.2: any weight function; Lemma 2.3 gives its filter).
 * Errors: KF_EINVAL (NULL, n < 1, invalid sample), KF_ENOMEM, KF_EHIP. */
int kf_mlp_weights(kf_mlp* net, const double* samples, int32_t n, double* w_out);

/* Filter coefficients for one problem: the network's weights when their loss
 * is below that of the Fourier weights (*used_learned = 1), else the Fourier
 * weights (*used_learned = 0; also when L > 512).  w_out[L] host; j_learned and
 * j_fourier (optional) receive both losses. */
int kf_weights_from_mlp(kf_mlp* net, double omega_min, double omega_max, double tau, double lambda_max, int32_t L,
                        double* w_out, int32_t* used_learned, double* j_learned, double* j_fourier);

#ifdef __cplusplus
}
#endif

#endif /* KF_H */
