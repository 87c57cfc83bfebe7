// Float64 eigensolver for the projected pencil of Section 2.1 (eq. projevp).
//
// The basis is M-orthonormal, so the projected pencil is (H, G) with
// G = I up to rounding; the solver works on the symmetric H (its distance
// from the generalized problem is bounded by |G - I| |theta|, reported as the
// orthogonality error).  Steps:
//   1. Householder reduction of H to tridiagonal form (one workgroup; the
//      reflectors stay in the lower triangle of the work matrix);
//   2. all eigenvalues by Sturm-count bisection, one lane per eigenvalue;
//   3. eigenvectors for the selected eigenvalues only, by inverse iteration
//      on the tridiagonal matrix (LU with partial pivoting), re-orthogonalised
//      inside clusters of nearly equal values;
//   4. back-transformation with the stored reflectors, one wavefront per
//      vector held in registers.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "kf_internal.h"

namespace kf {

namespace {

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// matrices of this order and larger are reduced by k_tri_step
constexpr int kTriMultiFrom = 48;

__device__ __forceinline__ double wave_sum_e(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum over the workgroup, same value and summation order in every thread.
__device__ double block_sum(double v, double* red) {
  v = wave_sum_e(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

__global__ __launch_bounds__(256) void k_copy_square(int k, const double* __restrict__ H, int64_t ldh,
                                                     double* __restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * k) return;
  const int64_t j = t / k, i = t - j * k;
  A[t] = H[i + j * ldh];
}

// Householder reduction to tridiagonal form, one workgroup, full symmetric
// storage in global memory (L2 resident), one row per thread.  Step k uses
// the reflector v_k (v_k[k+1] = 1) with scalar tau_k and w_k = p - (tau/2)(p.v)v,
// p = tau A22 v.  The rank-2 update of step k and the product p of step k+1
// share one pass over the trailing matrix: column k+1 is updated first, v_{k+1}
// is formed from it, then every remaining entry is updated and immediately
// multiplied into p_{k+1}.  Reflector k is stored below the subdiagonal of
// column k.
__global__ __launch_bounds__(1024) void k_tridiag(int m, double* __restrict__ A, double* __restrict__ d,
                                                  double* __restrict__ e, double* __restrict__ tau) {
  extern __shared__ double sh[];
  double* vb[2] = {sh, sh + m};
  double* wb[2] = {sh + 2 * m, sh + 3 * m};
  double* red = sh + 4 * m;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (m == 1) {
    if (tid == 0) d[0] = A[0];
    return;
  }
  if (m == 2) {
    if (tid == 0) {
      d[0] = A[0];
      d[1] = A[3];
      e[0] = A[1];
      tau[0] = 0.0;
    }
    return;
  }
  // reflector from column k (entries k+1..m-1) into v (absolute indexing);
  // returns tau (0 when the column is already reduced) and sets e[k]
  auto make_reflector = [&](int k, double* v) -> double {
    const double* col = A + (int64_t)k * m;
    double s = 0.0;
    for (int i = k + 2 + tid; i < m; i += nt) s = fma(col[i], col[i], s);
    s = block_sum(s, red);
    const double alpha = col[k + 1];
    double beta = alpha, tk = 0.0, v0 = 1.0;
    if (s > 0.0) {
      const double mu = sqrt(alpha * alpha + s);
      beta = alpha <= 0.0 ? mu : -mu;
      v0 = alpha - beta;
      tk = (beta - alpha) / beta;
    }
    for (int i = tid; i < m; i += nt) v[i] = (i <= k) ? 0.0 : (i == k + 1 ? 1.0 : (tk == 0.0 ? 0.0 : col[i] / v0));
    if (tid == 0) {
      e[k] = beta;
      tau[k] = tk;
    }
    __syncthreads();
    return tk;
  };
  // w = p - (tau/2)(p.v) v with p already in w (scaled by tau)
  auto finish_w = [&](int k, double tk, double* v, double* w) {
    double pv = 0.0;
    for (int i = k + 1 + tid; i < m; i += nt) pv = fma(w[i], v[i], pv);
    pv = block_sum(pv, red);
    const double K = 0.5 * tk * pv;
    for (int i = tid; i < m; i += nt) w[i] = (i <= k) ? 0.0 : w[i] - K * v[i];
    __syncthreads();
  };

  // step 0: reflector and the plain product p = tau A22 v
  if (tid == 0) d[0] = A[0];
  double tk = make_reflector(0, vb[0]);
  {
    double* v = vb[0];
    double* w = wb[0];
    for (int i = 1 + tid; i < m; i += nt) {
      double acc = 0.0;
#pragma unroll 8
      for (int j = 1; j < m; ++j) acc = fma(A[i + (int64_t)j * m], v[j], acc);
      w[i] = tk * acc;
    }
    __syncthreads();
    finish_w(0, tk, v, w);
  }
  int cur = 0;
  for (int k = 0; k + 2 < m; ++k) {
    double* v = vb[cur];
    double* w = wb[cur];
    // store reflector k below the subdiagonal of column k
    for (int i = k + 2 + tid; i < m; i += nt) A[i + (int64_t)k * m] = v[i];
    // rank-2 update of column k+1 (rows k+1..m-1)
    const int c = k + 1;
    for (int i = c + tid; i < m; i += nt) A[i + (int64_t)c * m] -= v[i] * w[c] + w[i] * v[c];
    __syncthreads();
    if (tid == 0) d[c] = A[c + (int64_t)c * m];
    if (c + 2 > m - 1) {
      // last 2 x 2 block: update the remaining entry and finish
      if (tid == 0) {
        const int j = c + 1;
        const double a = A[j + (int64_t)j * m] - 2.0 * v[j] * w[j];
        A[j + (int64_t)j * m] = a;
        d[j] = a;
        e[c] = A[j + (int64_t)c * m];
        tau[c] = 0.0;
      }
      break;
    }
    double* vn = vb[cur ^ 1];
    double* wn = wb[cur ^ 1];
    const double tn = make_reflector(c, vn);
    // fused pass: update rows/cols >= c+1 with step k, accumulate p_{k+1}
    for (int i = c + 1 + tid; i < m; i += nt) {
      const double vi = v[i], wi = w[i];
      double acc = 0.0;
      double* __restrict__ ai = A + i;
      int j = c + 1;
      // eight independent loads in flight before the dependent updates
      for (; j + 8 <= m; j += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = ai[(int64_t)(j + u) * m];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a[u] = a[u] - vi * w[j + u] - wi * v[j + u];
          ai[(int64_t)(j + u) * m] = a[u];
          acc = fma(a[u], vn[j + u], acc);
        }
      }
      for (; j < m; ++j) {
        const double a = ai[(int64_t)j * m] - vi * w[j] - wi * v[j];
        ai[(int64_t)j * m] = a;
        acc = fma(a, vn[j], acc);
      }
      wn[i] = tn * acc;
    }
    __syncthreads();
    finish_w(c, tn, vn, wn);
    cur ^= 1;
  }
}

// One step of the same Householder reduction spread over many workgroups
// (one launch per reflector; used for larger matrices, where a single
// workgroup is latency-bound).  Launch k:
//   * every workgroup finishes w_{k-1} = p_{k-1} - (tau_{k-1}/2)(p_{k-1}.v_{k-1}) v_{k-1}
//     from the previous launch's p, applies reflector k-1 to column k on the
//     fly and forms reflector k from it (the same arithmetic in the same
//     order in every workgroup, so all agree bit for bit);
//   * workgroup 0 records d_k, e_k, tau_k and v_k, and stores v_{k-1} below
//     the subdiagonal of column k-1 (no workgroup reads that column here);
//   * each wavefront owns whole columns j > k: it applies reflector k-1 to
//     rows > k of column j (the matrix is symmetric, so a column is a row and
//     the lanes read consecutive addresses) and forms p_k[j] = tau_k (A v_k)_j.
// Column k is only read in launch k; columns > k are only touched by their
// owner, so no two workgroups write the same entry.
__global__ __launch_bounds__(256) void k_tri_step(int m, int k, double* __restrict__ A, double* __restrict__ d,
                                                  double* __restrict__ e, double* __restrict__ tau,
                                                  double* __restrict__ pv) {
  extern __shared__ double sh[];
  double* vp = sh;           // v_{k-1}
  double* w = sh + m;        // w_{k-1}
  double* vk = sh + 2 * m;   // column k after reflector k-1, then v_k
  double* red = sh + 3 * m;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* pprev = pv + (int64_t)((k + 1) & 1) * m;
  double* pcur = pv + (int64_t)(k & 1) * m;
  const double* vprev_g = pv + (int64_t)(2 + ((k + 1) & 1)) * m;
  double* vcur_g = pv + (int64_t)(2 + (k & 1)) * m;
  // w_{k-1}
  if (k == 0) {
    for (int i = tid; i < m; i += nt) {
      vp[i] = 0.0;
      w[i] = 0.0;
    }
    __syncthreads();
  } else {
    double s = 0.0;
    for (int i = tid; i < m; i += nt) {
      const double v = i >= k ? vprev_g[i] : 0.0;
      vp[i] = v;
      if (i >= k) s = fma(pprev[i], v, s);
    }
    s = block_sum(s, red);
    const double K = 0.5 * tau[k - 1] * s;
    for (int i = tid; i < m; i += nt) w[i] = i >= k ? pprev[i] - K * vp[i] : 0.0;
    __syncthreads();
  }
  // column k after reflector k-1, and reflector k
  const double wk = w[k], vpk = vp[k];
  double s = 0.0;
  for (int i = tid; i < m; i += nt) {
    const double a = i >= k ? A[i + (int64_t)k * m] - vp[i] * wk - w[i] * vpk : 0.0;
    vk[i] = a;
    if (i >= k + 2) s = fma(a, a, s);
  }
  s = block_sum(s, red);
  const double dk = vk[k];
  const double alpha = k + 1 < m ? vk[k + 1] : 0.0;
  double beta = alpha, tk = 0.0, v0 = 1.0;
  if (s > 0.0) {
    const double mu = sqrt(alpha * alpha + s);
    beta = alpha <= 0.0 ? mu : -mu;
    v0 = alpha - beta;
    tk = (beta - alpha) / beta;
  }
  __syncthreads();
  for (int i = tid; i < m; i += nt) vk[i] = (i <= k) ? 0.0 : (i == k + 1 ? 1.0 : (tk == 0.0 ? 0.0 : vk[i] / v0));
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid == 0) {
      d[k] = dk;
      e[k] = beta;
      tau[k] = tk;
    }
    for (int i = tid; i < m; i += nt) vcur_g[i] = vk[i];
    if (k >= 1)
      for (int i = k + 1 + tid; i < m; i += nt) A[i + (int64_t)(k - 1) * m] = vp[i];
  }
  // owned columns
  const int lane = tid & 63;
  const int nwaves = gridDim.x * (nt >> 6);
  for (int j = k + 1 + blockIdx.x * (nt >> 6) + (tid >> 6); j < m; j += nwaves) {
    double* __restrict__ col = A + (int64_t)j * m;
    const double wj = w[j], vj = vp[j];
    double dot = 0.0;
    int i = k + 1 + lane;
    for (; i + 192 < m; i += 256) {
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = col[i + 64 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = i + 64 * u;
        a[u] = a[u] - vp[r] * wj - w[r] * vj;
        col[r] = a[u];
        dot = fma(a[u], vk[r], dot);
      }
    }
    for (; i < m; i += 64) {
      const double a = col[i] - vp[i] * wj - w[i] * vj;
      col[i] = a;
      dot = fma(a, vk[i], dot);
      if (k == m - 2 && i == m - 1) d[m - 1] = a;
    }
    dot = wave_sum_e(dot);
    if (lane == 0) pcur[j] = tk * dot;
  }
}

__device__ int sturm_count(int m, const double* __restrict__ d, const double* __restrict__ e2, double x,
                           double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int j = 1; j < m; ++j) {
    q = (d[j] - x) - e2[j - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

__global__ __launch_bounds__(256) void k_tri_prep(int m, const double* __restrict__ d, const double* __restrict__ e,
                                                  double* __restrict__ e2, double* __restrict__ bounds) {
  // e2 = e^2; bounds = {gershgorin lo, hi, pivmin}
  __shared__ double red[3][4];
  double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + (j < m - 1 ? fabs(e[j]) : 0.0);
    lo = fmin(lo, d[j] - r);
    hi = fmax(hi, d[j] + r);
    if (j < m - 1) {
      e2[j] = e[j] * e[j];
      emax2 = fmax(emax2, e2[j]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    emax2 = fmax(emax2, __shfl_xor(emax2, off));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = lo;
    red[1][threadIdx.x >> 6] = hi;
    red[2][threadIdx.x >> 6] = emax2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = fmin(red[0][0], red[0][w]);
      red[0][0] = lo;
      hi = fmax(red[1][0], red[1][w]);
      red[1][0] = hi;
      emax2 = fmax(red[2][0], red[2][w]);
      red[2][0] = emax2;
    }
    lo = red[0][0];
    hi = red[1][0];
    const double pivmin = DBL_MIN * fmax(1.0, red[2][0]);
    const double tn = fmax(fabs(lo), fabs(hi));
    bounds[0] = lo - 2.0 * DBL_EPSILON * tn - pivmin;
    bounds[1] = hi + 2.0 * DBL_EPSILON * tn + pivmin;
    bounds[2] = pivmin;
  }
}

// Eigenvalue i by 65-section: the 64 lanes of a wavefront evaluate Sturm
// counts at 64 interior points of the bracket, which shrinks 65-fold per
// round until it is a few ulps wide.
__global__ __launch_bounds__(256) void k_bisect(int m, const double* __restrict__ d, const double* __restrict__ e2,
                                                const double* __restrict__ bounds, double* __restrict__ theta) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= m) return;
  double lo = bounds[0], hi = bounds[1];
  const double pivmin = bounds[2];
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    const double h = (hi - lo) / 65.0;
    const double x = lo + (lane + 1) * h;
    const bool above = sturm_count(m, d, e2, x, pivmin) > i;
    const unsigned long long mask = __ballot(above);
    double nlo, nhi;
    if (mask == 0ull) {
      nlo = __shfl(x, 63);
      nhi = hi;
    } else {
      const int f = __ffsll((long long)mask) - 1;
      nhi = __shfl(x, f);
      nlo = f > 0 ? __shfl(x, f - 1) : lo;
    }
    if (!(nhi - nlo < hi - lo)) break;  // no progress: bracket is at rounding level
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) theta[i] = 0.5 * (lo + hi);
}

// Inverse iteration, one lane per selected eigenvalue; the recurrences carry
// their running values in registers.  Within a cluster of (nearly) equal
// values the shifts are kept 10 eps apart and each member starts from its own
// vector (its position in the cluster sets the phase), so the members
// converge to different directions of the eigenspace; k_cluster_orth then
// orthonormalises each cluster's vectors.  The lane's work
// arrays (LU factors and the iterate) are interleaved across lanes, element i
// of lane c at [i * ldw + c], so that at every step the lanes of a wavefront
// touch consecutive addresses.  Finished vectors go to Z (m x nsel).
// LDS: the work arrays of the wavefront's first ldw lanes live in LDS (the
// recurrences are chains of dependent steps, and LDS answers in a fraction of
// the time of the cache hierarchy); otherwise in `scratch` (global memory).
constexpr int kIvB = 8;  // rows loaded ahead of the running values
constexpr int kIvLdsBytes = 65536;  // LDS for the work arrays of one wavefront
template <bool LDS>
__global__ __launch_bounds__(64) void k_invit(int m, const double* __restrict__ d, const double* __restrict__ e,
                                              const double* __restrict__ bounds, int ncl,
                                              const int32_t* __restrict__ cstart, const double* __restrict__ sel,
                                              double* __restrict__ Z, double* __restrict__ scratch, int ldw) {
  extern __shared__ double ivs[];
  if (LDS && (int)threadIdx.x >= ldw) return;
  const int s = LDS ? blockIdx.x * ldw + threadIdx.x : blockIdx.x * blockDim.x + threadIdx.x;
  const int nsel = cstart[ncl];
  if (s >= nsel) return;
  const double tn = fmax(fabs(bounds[0]), fabs(bounds[1]));
  const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);
  const int64_t blk = (int64_t)m * ldw;
  double* __restrict__ rinv = LDS ? ivs + threadIdx.x : scratch + s;
  double* __restrict__ u1 = rinv + blk;
  double* __restrict__ u2 = u1 + blk;
  double* __restrict__ lm = u2 + blk;
  double* __restrict__ pv = lm + blk;
  double* __restrict__ z = pv + blk;
  {
    // the cluster holding s (cstart ascending, cstart[0] = 0)
    int lo = 0, hi = ncl;  // cstart[lo] <= s < cstart[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (cstart[mid] <= s) lo = mid;
      else hi = mid;
    }
    const int c0 = cstart[lo];
    // shifts of the cluster's members up to s, each at least 10 eps above the last
    double lam = sel[c0];
    for (int t = c0 + 1; t <= s; ++t) lam = sel[t] - lam < 10.0 * tiny ? lam + 10.0 * tiny : sel[t];
    const int pos = s - c0;
    // LU of T - lam I with partial pivoting; row i is (a, b, c) at columns
    // (i, i+1, i+2) while it is being eliminated.  The recurrences below load
    // kIvB rows ahead of the running values (the loads do not depend on them).
    double a = d[0] - lam;
    double b = m > 1 ? e[0] : 0.0;
    for (int i0 = 0; i0 + 1 < m; i0 += kIvB) {
      double eb[kIvB], dn[kIvB], en[kIvB];
#pragma unroll
      for (int u = 0; u < kIvB; ++u) {
        const int i = i0 + u;
        eb[u] = i + 1 < m ? e[i] : 0.0;
        dn[u] = i + 1 < m ? d[i + 1] : 0.0;
        en[u] = i + 2 < m ? e[i + 1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kIvB; ++u) {
        const int i = i0 + u;
        if (i + 1 >= m) break;
        const int64_t o = (int64_t)i * ldw;
        const double bi = eb[u];
        const double ai1 = dn[u] - lam;
        const double ci1 = en[u];
        double na, nb;
        if (fabs(a) >= fabs(bi)) {
          const double l = (a != 0.0) ? bi / a : 0.0;
          pv[o] = 0.0;
          lm[o] = l;
          u2[o] = 0.0;
          u1[o] = b;
          if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
          rinv[o] = 1.0 / a;
          na = ai1 - l * b;
          nb = ci1;
        } else {
          const double l = a / bi;
          pv[o] = 1.0;
          lm[o] = l;
          u1[o] = ai1;
          u2[o] = ci1;
          rinv[o] = 1.0 / bi;
          na = b - l * ai1;
          nb = -l * ci1;
        }
        a = na;
        b = nb;
      }
    }
    const int64_t ol = (int64_t)(m - 1) * ldw;
    if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
    rinv[ol] = 1.0 / a;
    u1[ol] = 0.0;
    u2[ol] = 0.0;
    if (m >= 2) u2[ol - ldw] = 0.0;
    // start vector: 1 + 0.5 u, u in [-1, 1) from an integer hash of (row,
    // position in the cluster), so that the members of a cluster start from
    // linearly independent vectors
    for (int i = 0; i < m; ++i) {
      uint32_t h = (uint32_t)i * 0x9E3779B1u ^ ((uint32_t)pos + 1u) * 0x85EBCA77u;
      h ^= h >> 16;
      h *= 0x7FEB352Du;
      h ^= h >> 15;
      h *= 0x846CA68Bu;
      h ^= h >> 16;
      z[(int64_t)i * ldw] = 1.0 + 0.5 * ((double)h * (2.0 / 4294967296.0) - 1.0);
    }
    for (int it = 0; it < 3; ++it) {
      // forward: row swaps and elimination, running value in a register
      double y = z[0];
      for (int i0 = 0; i0 + 1 < m; i0 += kIvB) {
        double nxv[kIvB], pvv[kIvB], lmv[kIvB];
#pragma unroll
        for (int u = 0; u < kIvB; ++u) {
          const int i = i0 + u;
          const int64_t o = (int64_t)i * ldw;
          const bool ok = i + 1 < m;
          nxv[u] = ok ? z[o + ldw] : 0.0;
          pvv[u] = ok ? pv[o] : 0.0;
          lmv[u] = ok ? lm[o] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kIvB; ++u) {
          const int i = i0 + u;
          if (i + 1 >= m) break;
          double nx = nxv[u];
          if (pvv[u] != 0.0) {
            const double t = y;
            y = nx;
            nx = t;
          }
          z[(int64_t)i * ldw] = y;
          y = nx - lmv[u] * y;
        }
      }
      z[ol] = y;
      // backward substitution with U (diagonal inverse, two superdiagonals)
      double x1 = 0.0, x2 = 0.0, mx = 0.0;
      for (int i0 = m - 1; i0 >= 0; i0 -= kIvB) {
        double zv[kIvB], u1v[kIvB], u2v[kIvB], rv[kIvB];
#pragma unroll
        for (int u = 0; u < kIvB; ++u) {
          const int i = i0 - u;
          const int64_t o = (int64_t)i * ldw;
          const bool ok = i >= 0;
          zv[u] = ok ? z[o] : 0.0;
          u1v[u] = ok ? u1[o] : 0.0;
          u2v[u] = ok ? u2[o] : 0.0;
          rv[u] = ok ? rinv[o] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kIvB; ++u) {
          const int i = i0 - u;
          if (i < 0) break;
          const double x = (zv[u] - u1v[u] * x1 - u2v[u] * x2) * rv[u];
          z[(int64_t)i * ldw] = x;
          mx = fmax(mx, fabs(x));
          x2 = x1;
          x1 = x;
        }
      }
      const double r = mx > 0.0 ? 1.0 / mx : 0.0;
      for (int i = 0; i < m; ++i) z[(int64_t)i * ldw] *= r;
      double nrm = 0.0;
      for (int i = 0; i < m; ++i) nrm = fma(z[(int64_t)i * ldw], z[(int64_t)i * ldw], nrm);
      const double rn = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = 0; i < m; ++i) z[(int64_t)i * ldw] *= rn;
    }
    double* __restrict__ zs = Z + (int64_t)s * m;
    for (int i = 0; i < m; ++i) zs[i] = z[(int64_t)i * ldw];
  }
}

// The vectors of each cluster with more than one member (Z columns
// cstart[c] .. cstart[c+1]-1): classical Gram-Schmidt twice against the
// cluster's earlier members, then normalisation; one workgroup per cluster.
__device__ __forceinline__ double block_sum256(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_cluster_orth(int m, int ncl, const int32_t* __restrict__ cstart,
                                                      double* __restrict__ Z) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  if (c >= ncl) return;
  const int c0 = cstart[c], c1 = cstart[c + 1];
  if (c1 - c0 < 2) return;
  for (int j = c0; j < c1; ++j) {
    double* zj = Z + (int64_t)j * m;
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = c0; q < j; ++q) {
        const double* zq = Z + (int64_t)q * m;
        double dot = 0.0;
        for (int i = threadIdx.x; i < m; i += 256) dot = fma(zq[i], zj[i], dot);
        dot = block_sum256(dot, red);
        for (int i = threadIdx.x; i < m; i += 256) zj[i] -= dot * zq[i];
        __syncthreads();
      }
    }
    double nrm = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) nrm = fma(zj[i], zj[i], nrm);
    nrm = block_sum256(nrm, red);
    const double rn = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
    for (int i = threadIdx.x; i < m; i += 256) zj[i] *= rn;
    __syncthreads();
  }
}

// y = H_0 H_1 ... H_{m-3} z, H_k = I - tau_k v_k v_k^T acting on rows k+1..m-1,
// v_k = (1, A[k+2.., k]).  One wavefront per vector; lane l keeps rows l+64t.
template <int MT>
__global__ __launch_bounds__(256) void k_backtransform(int m, const double* __restrict__ A,
                                                       const double* __restrict__ tau, int nsel,
                                                       const double* __restrict__ Z, double* __restrict__ Y) {
  const int vec = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (vec >= nsel) return;
  double y[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int i = lane + 64 * t;
    y[t] = i < m ? Z[(int64_t)vec * m + i] : 0.0;
  }
  for (int k = m - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    const double* col = A + (int64_t)k * m;
    double vi[MT];
    double dot = 0.0;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int i = lane + 64 * t;
      vi[t] = (i == k + 1) ? 1.0 : ((i > k + 1 && i < m) ? col[i] : 0.0);
      dot = fma(vi[t], y[t], dot);
    }
    dot = wave_sum_e(dot) * tk;
#pragma unroll
    for (int t = 0; t < MT; ++t) y[t] -= dot * vi[t];
  }
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int i = lane + 64 * t;
    if (i < m) Y[(int64_t)vec * m + i] = y[t];
  }
}

}  // namespace

void free_eig(EigWork& w) {
  double* ptrs[] = {w.A, w.d, w.e, w.e2, w.bounds, w.tau, w.theta, w.pv, w.Z, w.Y, w.scratch, w.sel};
  for (double* p : ptrs)
    if (p) (void)hipFree(p);
  if (w.cl) (void)hipFree(w.cl);
  w = EigWork();
}

int eig_reserve(EigWork& w, int m, int nsel) {
  if ((size_t)m > w.cap_m) {
    double** ps[] = {&w.A, &w.d, &w.e, &w.e2, &w.bounds, &w.tau, &w.theta, &w.pv};
    for (double** p : ps) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    const size_t mm = (size_t)m;
    if (hipMalloc(&w.A, sizeof(double) * mm * mm) != hipSuccess || hipMalloc(&w.d, sizeof(double) * mm) != hipSuccess ||
        hipMalloc(&w.e, sizeof(double) * mm) != hipSuccess || hipMalloc(&w.e2, sizeof(double) * mm) != hipSuccess ||
        hipMalloc(&w.bounds, sizeof(double) * 4) != hipSuccess || hipMalloc(&w.tau, sizeof(double) * mm) != hipSuccess ||
        hipMalloc(&w.theta, sizeof(double) * mm) != hipSuccess || hipMalloc(&w.pv, sizeof(double) * 4 * mm) != hipSuccess) {
      set_error("eig_reserve: allocation failed");
      return KF_ENOMEM;
    }
    w.cap_m = mm;
    w.cap_sel = 0;  // Z/Y/scratch depend on m too
  }
  if ((size_t)nsel > w.cap_sel) {
    double** ps[] = {&w.Z, &w.Y, &w.scratch, &w.sel};
    for (double** p : ps) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    if (w.cl) (void)hipFree(w.cl);
    w.cl = nullptr;
    const size_t ns = std::max<size_t>(nsel, 16);
    if (hipMalloc(&w.Z, sizeof(double) * w.cap_m * ns) != hipSuccess ||
        hipMalloc(&w.Y, sizeof(double) * w.cap_m * ns) != hipSuccess ||
        hipMalloc(&w.scratch, sizeof(double) * 6 * w.cap_m * (ns + 64)) != hipSuccess ||
        hipMalloc(&w.sel, sizeof(double) * ns) != hipSuccess ||
        hipMalloc(&w.cl, sizeof(int32_t) * (ns + 1)) != hipSuccess) {
      set_error("eig_reserve: allocation failed");
      return KF_ENOMEM;
    }
    w.cap_sel = ns;
  }
  return KF_OK;
}

int eig_values(EigWork& w, int k, const double* H, int64_t ldh, hipStream_t st) {
  if (k < 1) return KF_OK;
  if (k > 2048) {
    set_error("eigensolver: projected pencil larger than 2048");
    return KF_EINVAL;
  }
  KF_TRY(eig_reserve(w, k, 1));
  hipLaunchKernelGGL(k_copy_square, dim3(cdiv((int64_t)k * k, 256)), dim3(256), 0, st, k, H, ldh, w.A);
  KF_HIP(hipGetLastError());
  if (k < kTriMultiFrom) {
    const size_t lds = sizeof(double) * (4 * (size_t)k + 32);
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(1024), lds, st, k, w.A, w.d, w.e, w.tau);
    KF_HIP(hipGetLastError());
  } else {
    // one launch per reflector; the grid shrinks with the trailing matrix
    const size_t lds = sizeof(double) * (3 * (size_t)k + 32);
    for (int j = 0; j + 2 <= k; ++j) {
      const int cols = k - j - 1;
      const int grid = std::max(1, std::min(cdiv(cols, 4), 256));
      hipLaunchKernelGGL(k_tri_step, dim3(grid), dim3(256), lds, st, k, j, w.A, w.d, w.e, w.tau, w.pv);
      KF_HIP(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(k_tri_prep, dim3(1), dim3(256), 0, st, k, w.d, w.e, w.e2, w.bounds);
  KF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bisect, dim3(cdiv(k, 4)), dim3(256), 0, st, k, w.d, w.e2, w.bounds, w.theta);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int eig_vectors(EigWork& w, int k, const double* theta_sel, const int32_t* cluster_start, int nclusters, int nsel,
                hipStream_t st) {
  if (nsel <= 0) return KF_OK;
  KF_TRY(eig_reserve(w, k, nsel));
  KF_HIP(hipMemcpyAsync(w.sel, theta_sel, sizeof(double) * nsel, hipMemcpyHostToDevice, st));
  KF_HIP(hipMemcpyAsync(w.cl, cluster_start, sizeof(int32_t) * (nclusters + 1), hipMemcpyHostToDevice, st));
  // six work arrays of k doubles per lane: as many lanes per wavefront as fit
  // in kIvLdsBytes of LDS, else all 64 lanes with the arrays in global memory
  const int lds_lanes = std::min(64, kIvLdsBytes / (6 * 8 * k));
  if (lds_lanes >= 1) {
    const size_t lds = sizeof(double) * 6 * (size_t)k * lds_lanes;
    hipLaunchKernelGGL(k_invit<true>, dim3(cdiv(nsel, lds_lanes)), dim3(64), lds, st, k, w.d, w.e, w.bounds,
                       nclusters, w.cl, w.sel, w.Z, w.scratch, lds_lanes);
  } else {
    const int ldw = cdiv(nsel, 64) * 64;  // <= nsel + 63
    hipLaunchKernelGGL(k_invit<false>, dim3(cdiv(nsel, 64)), dim3(64), 0, st, k, w.d, w.e, w.bounds, nclusters,
                       w.cl, w.sel, w.Z, w.scratch, ldw);
  }
  KF_HIP(hipGetLastError());
  if (nclusters < nsel) {
    hipLaunchKernelGGL(k_cluster_orth, dim3(nclusters), dim3(256), 0, st, k, nclusters, w.cl, w.Z);
    KF_HIP(hipGetLastError());
  }
  const int grid = cdiv(nsel, 4);
  const int mt = cdiv(k, 64);
  if (mt <= 1)
    hipLaunchKernelGGL(k_backtransform<1>, dim3(grid), dim3(256), 0, st, k, w.A, w.tau, nsel, w.Z, w.Y);
  else if (mt <= 2)
    hipLaunchKernelGGL(k_backtransform<2>, dim3(grid), dim3(256), 0, st, k, w.A, w.tau, nsel, w.Z, w.Y);
  else if (mt <= 4)
    hipLaunchKernelGGL(k_backtransform<4>, dim3(grid), dim3(256), 0, st, k, w.A, w.tau, nsel, w.Z, w.Y);
  else if (mt <= 8)
    hipLaunchKernelGGL(k_backtransform<8>, dim3(grid), dim3(256), 0, st, k, w.A, w.tau, nsel, w.Z, w.Y);
  else if (mt <= 16)
    hipLaunchKernelGGL(k_backtransform<16>, dim3(grid), dim3(256), 0, st, k, w.A, w.tau, nsel, w.Z, w.Y);
  else
    hipLaunchKernelGGL(k_backtransform<32>, dim3(grid), dim3(256), 0, st, k, w.A, w.tau, nsel, w.Z, w.Y);
  KF_HIP(hipGetLastError());
  // the host arrays must outlive the asynchronous copies
  KF_HIP(hipStreamSynchronize(st));
  return KF_OK;
}

}  // namespace kf
