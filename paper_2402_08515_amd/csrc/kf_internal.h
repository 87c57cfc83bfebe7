// Internal declarations shared by the host driver and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/kf.h"

namespace kf {

// thread-local error text behind kf_last_error()
void set_error(const std::string& msg);

#define KF_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::kf::set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
      return KF_EHIP;                                                                  \
    }                                                                                  \
  } while (0)

#define KF_TRY(call)          \
  do {                        \
    int s_ = (call);          \
    if (s_ != KF_OK) return s_; \
  } while (0)

constexpr int kSlice = 64;  // SELL slice height = wavefront width

// Sliced-ELLPACK operator (slice height 64, one row per lane, entries of a
// slice stored column by column so that lane l reads entry k of its row at
// slice_ptr[s] + 64*k + l).  Column indices are either int32 absolute or
// int16 offsets relative to the row.
struct SellOp {
  int32_t n = 0;
  int32_t nslices = 0;
  int64_t nstored = 0;
  int idx_bytes = 4;
  int val_bytes = 8;
  int64_t* slice_ptr = nullptr;
  void* val = nullptr;
  void* idx = nullptr;
  int32_t max_width = 0;
  int nt_loads = 0;  // 1: stream the matrix with non-temporal loads in the fused step
  int lpr[5] = {0, 0, 0, 0, 0};  // lanes per row of the fused step for blocks 1..16 (0: default)
  int lpr_tuned = 0;             // bit l: lpr[l] was chosen by timing
  int unroll = 0;                // single vectors: unroll of the loop over a slice's entries (2, 3, 4, 6; 0: 4)
  int32_t max_off = 0;           // largest |col - row| of a stored entry
  int band[5] = {0, 0, 0, 0, 0}; // blocks 2..16: 1 = gather from an LDS copy of the workgroup's band of rows
};

// LDS available to the band copy of one workgroup of the fused step.
constexpr size_t kBandLdsBytes = 65536;

// Bytes of the band copy for block width b with lpr lanes per row: the
// workgroup's 4 * 64 / lpr rows and max_off rows on either side.
inline size_t band_lds_bytes(const SellOp& A, int b, int lpr) {
  const int64_t rows = std::min<int64_t>((int64_t)A.n, 4 * (64 / lpr) + 2 * (int64_t)A.max_off);
  return (size_t)rows * b * A.val_bytes;
}

// Whether the fused step for block width b gathers from the LDS band copy.
inline bool use_band(const SellOp& A, int b, int lpr) {
  int lb = 0;
  while ((1 << lb) < b && lb < 4) ++lb;
  return b > 1 && A.band[lb] == 1 && band_lds_bytes(A, b, lpr) <= kBandLdsBytes;
}

// Lanes that share one row in the fused step for block width b.
int lanes_per_row(const SellOp& A, int b);

void free_sell(SellOp& op);

// Build a SELL operator from a device CSR: values scaled per row by
// row_scale[i] (device array, or nullptr for 1), stored as float64
// (val_bytes 8) or float32 (val_bytes 4).  want_idx_bytes 0 chooses 2 when
// every |col - row| < 32768.
int build_sell(int32_t n, int64_t nnz, const int32_t* d_rowptr, const int32_t* d_col, const double* d_val,
               const double* d_row_scale, int val_bytes, int want_idx_bytes, hipStream_t st, SellOp& out);

// ---- fused leapfrog step ----------------------------------------------------
enum StepMode { kMid = 0, kFirst = 1, kLast = 2, kFirstLast = 3, kMidAcc = 4 };

// One step of eq. 2stepmethod fused with the rectangle-rule accumulation:
//   nxt = 2 cur - prev - A cur   (prev ignored in kFirst: prev = cur)
//   kFirst:   acc = wc*cur + wn*nxt
//   kMid:     acc untouched
//   kMidAcc:  acc += wp*prev + wc*cur + wn*nxt
//   kLast:    the value acc + wp*prev + wc*cur + wn*nxt of columns j < bout
//             goes to rout[i*rs + j*cs] (float64) and nxt is not stored
//   kFirstLast: rout gets wc*cur + wn*nxt
// (the step sees three consecutive time levels, so the weighted sum can be
// accumulated once every three steps); otherwise nxt -> out (may alias prev).
// Blocks are n x b row-major in the stepping precision.
int launch_leapfrog(const SellOp& A, int b, int mode, const void* cur, const void* prev, void* out, void* acc,
                    double* rout, int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int xcd_remap,
                    hipStream_t st);

// The fourth-order two-step scheme, same modes and schedule:
//   z = A cur;  nxt = 2 cur - prev - z + (A z)/12
// (two launches; z is an n x b work block in the stepping precision).
int launch_leapfrog4(const SellOp& A, int b, int mode, const void* cur, const void* prev, void* out, void* acc, void* z,
                     double* rout, int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int xcd_remap,
                     hipStream_t st);

// Several leapfrog steps per launch for banded operators (every stored
// entry within A.max_off rows of the diagonal), single vectors: each
// workgroup owns `own` row slices and keeps them, the s*max_off rows on either
// side and its part of the weighted sum in LDS.  plan_multistep picks `own`
// for s steps per launch within lds_bytes (ok = false: the band does not
// fit).  A launch advances y_{l0} to y_{l0+s} and adds w_{l+1} y_{l+1} for
// each step; first: y_{-1} = y_0 = ysrc and the sum starts at w_0 y_0, else
// the levels y_{l0-1}, y_{l0} are read from i0, i1; last: the sum goes to
// rout (float64, row stride rs), else the levels y_{l0+s-1}, y_{l0+s} go to
// o0, o1 (distinct from i0, i1: halo rows are read while their owners write)
// and the sum to acc; vectors are n long in the stepping precision, w holds
// the L weights (float64, device).
struct MultiStepPlan {
  bool ok = false;
  bool reg = false;  // one workgroup, the operator's entries and the sums in registers
  int own = 0;  // owned row slices per workgroup
  int hb = 0;   // the band in slices
  int s = 0;
};
MultiStepPlan plan_multistep(const SellOp& A, int s, size_t lds_bytes);
int launch_leapfrog_mp(const SellOp& A, const MultiStepPlan& pl, int l0, int s, bool first, bool last, const void* ysrc,
                       const void* i0, const void* i1, void* o0, void* o1, void* acc, double* rout, int64_t rs,
                       const double* w, hipStream_t st);

// The accumulation schedule of one filter application (L - 1 steps): for
// step l, the mode and the weights (wp, wc, wn) of prev, cur and nxt.  Every
// y_j enters once: y_0 and y_1 at step 1, then three at a time at steps
// 4, 7, ..., and whatever is pending at the last step.
struct StepPlan {
  int mode;
  int ip, ic, in;  // indices of the weights of prev, cur, nxt (-1: weight 0)
};
StepPlan step_plan(int l, int L);

// Per-problem tables of a batch (device memory, refreshed before every
// batched filter application).  kMaxBatch bounds the number of problems.
constexpr int kMaxBatch = 256;
struct BatchTables {
  int64_t row0[kMaxBatch];  // first stacked row of the problem (multiple of 64)
  int32_t n[kMaxBatch];     // rows of the problem
  int32_t L[kMaxBatch];     // rectangle-rule nodes
  int32_t active[kMaxBatch];
  int32_t bsrc[kMaxBatch];  // source columns (the rest of the block is zero)
  int32_t bout[kMaxBatch];  // destination columns written
  int64_t lds[kMaxBatch];   // source column stride
  int64_t ld[kMaxBatch];    // destination column stride
  const double* src[kMaxBatch];
  double* dst[kMaxBatch];
};

// One batched fused step (step index ell >= 1) over the first nslices row
// slices of the stacked operator (0: all; members are stacked by decreasing
// L, so the members still stepping at ell form a prefix).
int launch_leapfrog_batch(const SellOp& A, int b, const int32_t* slice_problem, const BatchTables* tb,
                          const void* wtab, int lmax, int ell, const void* cur, const void* prev, void* out, void* acc,
                          int nslices, int remap, hipStream_t st);
// Batched load of the filter input into Y1 (and C = w0 I for L_p = 1).
int launch_load_batch(int val_bytes, int64_t rows, int b, const int32_t* slice_problem, const BatchTables* tb,
                      const void* wtab, int lmax, void* Y1, hipStream_t st);

// dst (n x b row-major, stepping precision) = src[i*rs + j*cs] for j < bsrc, 0 beyond.
int launch_load_block(int val_bytes, int32_t n, int b, int bsrc, const double* src, int64_t rs, int64_t cs,
                      void* dst, hipStream_t st);

// rout[i*rs + j*cs] = w0 * src[i*srs + j*scs]   (L = 1: C = w0 I)
int launch_scale_copy(int32_t n, int b, int bsrc, const double* src, int64_t srs, int64_t scs, double w0,
                      double* rout, int64_t rs, int64_t cs, hipStream_t st);

// ---- tall-skinny float64 kernels (column-major blocks) -----------------------
// H[j + c*ldh] = sum_i Bk[i + j*ldb] * wc(i) * X_c[i],  j < k, c < n1 + n2,
// X_c = X1[:, c] (c < n1, weight 1) or X2[:, c - n1] (weight m[i]).
// Two passes (per-chunk partials, then a fixed-order sum): deterministic.
struct GemvTWork {
  double* partial = nullptr;
  size_t cap = 0;  // doubles
};
int gemv_t(int32_t n, int k, const double* Bk, int64_t ldb, const double* X1, int n1, int64_t ldx1,
           const double* X2, int n2, int64_t ldx2, const double* m, double* H, int64_t ldh, GemvTWork& wk,
           hipStream_t st);

// Three-term step of one column x = L[:, lw] (lw <= 2 window columns before
// it, leading dimension ldl), three launches: c_j = L[:, j]^T M x (j < lw),
// x <- (x - sum_j c_j L[:, j]) / sqrt(g) with g the M-norm^2 after the
// subtraction (from x^T M x, c and the window's Gram matrix, no further pass);
// T = [c, x^T M x]; rec (16 doubles of device memory) = {T[0..lw], g, status}
// with status 1 (scaled) or 2 (g < 1e-4 x^T M x: only subtracted, the caller
// normalises explicitly); rec[8..10] is work space.  host_rec (optional):
// device address of pinned host memory that receives the same lw + 3 values
// (visible to the host once the stream has been synchronised).
int window_step(int32_t n, int lw, double* L, int64_t ldl, const double* m, GemvTWork& wk, double* T, double* rec,
                hipStream_t st, double* host_rec = nullptr);

// X[:, c] -= sum_j Bk[:, j] * H[j + c*ldh], c < nrhs; skipped entirely when
// gate (device flag) is given and holds 0
int gemv_n_sub(int32_t n, int k, const double* Bk, int64_t ldb, const double* H, int64_t ldh, double* X,
               int64_t ldx, int nrhs, hipStream_t st, const int32_t* gate = nullptr);

// *flag = 1 if some G[j + c*ldg] (j < k, c < np) differs from the identity
// entry of basis column p0 + c by more than tol (device values)
int block_gate(int k, int p0, int np, const double* G, int64_t ldg, double tol, int32_t* flag, hipStream_t st);

// X <- X R^{-1} with R the Cholesky factor of G = X^T M X (device, nb x nb,
// nb <= 16, leading dimension nb): one pass of Cholesky QR in the M inner
// product; Rinv (nb x nb, device) receives R^{-1}, flags[0..nb) = 1 and
// post[j] = R_jj.  The caller makes sure G is well conditioned.
int chol_orthonormalise(int32_t n, int nb, double* X, int64_t ldx, const double* G, double* Rinv, int32_t* flags,
                        double* post, hipStream_t st);

// *flag = 1 if some x[i] (i < cnt, device) is not finite; the caller clears
// *flag beforehand
int nonfinite_flag(int64_t cnt, const double* x, int32_t* flag, hipStream_t st);

// *gate = 1 if max_j |c[j]| (j < k) > tol * sqrt(*g), else 0 (device values)
int reorth_gate(int k, const double* c, const double* g, double tol, int32_t* gate, hipStream_t st);
// *gate = 1 if some column j < nb of c (rows < k, leading dimension ldc) has
// max_i |c[i, j]| > tol * sqrt(c[k + j, j]), else 0 (device values)
int reorth_gate_block(int k, int nb, const double* c, int64_t ldc, double tol, int32_t* gate, hipStream_t st);

// out[:, 0] = c_last with row kb-1 set to 0, out[:, 1] = cx (rows < kb,
// leading dimension ldo); *gate = 1 if some |c_last[j]| (j < kb-1) > tol,
// left as it is otherwise (gate may be null)
int pair_coef(int kb, const double* c_last, const double* cx, double* out, int64_t ldo, double tol, int32_t* gate,
              hipStream_t st);

// Y[:, c] = S X[:, c] (c < ncols), optional row scaling Y[i,c] *= rscale[i]
int spmv_cols(const SellOp& S, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols,
              const double* rscale, hipStream_t st);

// column j: x = x * scale where scale = 1/sqrt(nrm2) if sqrt(nrm2) > drop*ref
// (ref = sqrt(ref2)), else 0; flags[j] = kept, out_norm[j] = sqrt(nrm2)
int normalize_col(int32_t n, double* x, const double* nrm2, const double* ref2, double drop, int32_t* flag,
                  double* out_norm, hipStream_t st);

// V[:, c] = Bk * Y[:, c], c < nc  (Y is k x nc column-major, ldy)
int gemm_nn(int32_t n, int k, const double* Bk, int64_t ldb, const double* Y, int64_t ldy, double* V,
            int64_t ldv, int nc, hipStream_t st);

// per column c < nc: num[c] = ||SV_c - theta_c m.*V_c||^2, den[c] = ||SV_c||^2
int residual_norms(int32_t n, const double* SV, const double* V, int64_t ld, const double* m,
                   const double* theta, int nc, double* num, double* den, GemvTWork& wk, hipStream_t st);

int copy_cols(int32_t n, const double* src, int64_t lds, double* dst, int64_t ldd, int nc, hipStream_t st);

// H/G scatter: new columns [c0, c0+nc) from T (k x 2nc: first nc columns of
// H, next nc of G) into the symmetric k x k matrices (ld ldh).
int rr_scatter(int k, int c0, int nc, const double* T, int64_t ldt, double* H, double* G, int64_t ldh,
               hipStream_t st);

// Basis M-orthonormal only up to E = G - I: Hc = H - (E H + H E)/2 (k x k,
// leading dimension k; E and EH are k x k work arrays) has the eigenvalues of
// the pencil (H, G) to O(|E|^2); vectors_correct turns eigenvectors y of Hc
// (k x nc, leading dimension k) into (I - E/2) y (tmp: k x nc work).
int pencil_correct(int k, const double* H, const double* G, int64_t ldh, double* E, double* EH, double* Hc,
                   hipStream_t st);
int vectors_correct(int k, int nc, const double* E, double* Y, double* tmp, hipStream_t st);

// A = (A + A^T)/2 for the leading k x k block
int symmetrize(int k, double* A, int64_t lda, hipStream_t st);

// max |G - I| over the leading k x k block -> *out (device scalar)
int orth_error(int k, const double* G, int64_t ldg, double* out, hipStream_t st);

// ---- small dense symmetric eigensolver (projected pencil) ------------------
struct EigWork {
  double* A = nullptr;  // m x m
  double* d = nullptr;
  double* e = nullptr;
  double* e2 = nullptr;      // squared off-diagonal
  double* bounds = nullptr;  // Gershgorin bracket and pivot floor
  double* tau = nullptr;
  double* theta = nullptr;
  double* pv = nullptr;    // 4 x m: two p vectors and two reflectors (multi-workgroup reduction)
  double* Z = nullptr;     // m x nsel (tridiagonal eigenvectors)
  double* Y = nullptr;     // m x nsel (pencil eigenvectors)
  double* scratch = nullptr;
  double* sel = nullptr;   // selected eigenvalues
  int32_t* cl = nullptr;   // cluster starts
  size_t cap_m = 0, cap_sel = 0;
};
void free_eig(EigWork& w);
int eig_reserve(EigWork& w, int m, int nsel);
// Tridiagonalise the k x k symmetric matrix H (ld ldh) and compute all
// eigenvalues ascending into w.theta.
int eig_values(EigWork& w, int k, const double* H, int64_t ldh, hipStream_t st);
// Eigenvectors for nsel selected eigenvalues (host array theta_sel, ascending,
// with cluster ids) into w.Y (k x nsel column-major).
int eig_vectors(EigWork& w, int k, const double* theta_sel, const int32_t* cluster_start, int nclusters,
                int nsel, hipStream_t st);

}  // namespace kf
