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

__global__ __launch_bounds__(1024) void k_tridiag(int m, double* __restrict__ A, double* __restrict__ d,
                                                  double* __restrict__ e, double* __restrict__ tau) {
  extern __shared__ double sh[];
  double* v = sh;
  double* w = sh + m;
  double* red = sh + 2 * m;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k + 2 < m; ++k) {
    const int n2 = m - k - 1;
    const double* col = A + (int64_t)k * m + k + 1;
    double s = 0.0;
    for (int i = 1 + tid; i < n2; i += nt) {
      const double xi = col[i];
      s = fma(xi, xi, s);
    }
    s = block_sum(s, red);
    const double alpha = col[0];
    double beta = alpha, tk = 0.0, v0 = 1.0;
    if (s > 0.0) {
      const double mu = sqrt(alpha * alpha + s);
      beta = alpha <= 0.0 ? mu : -mu;
      v0 = alpha - beta;
      tk = (beta - alpha) / beta;
    }
    for (int i = tid; i < n2; i += nt) v[i] = (i == 0) ? 1.0 : (tk == 0.0 ? 0.0 : col[i] / v0);
    __syncthreads();
    if (tid == 0) {
      e[k] = beta;
      tau[k] = tk;
      d[k] = A[k + (int64_t)k * m];
    }
    for (int i = 1 + tid; i < n2; i += nt) A[(int64_t)k * m + k + 1 + i] = v[i];
    if (tk == 0.0) continue;  // uniform: tk comes from a block-wide sum
    // p = tk * A22 v
    const double* a22 = A + (int64_t)(k + 1) * m + (k + 1);
    for (int i = tid; i < n2; i += nt) {
      double acc = 0.0;
      const double* ai = a22 + i;
      for (int j = 0; j < n2; ++j) acc = fma(ai[(int64_t)j * m], v[j], acc);
      w[i] = tk * acc;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < n2; i += nt) pv = fma(w[i], v[i], pv);
    pv = block_sum(pv, red);
    const double K = 0.5 * tk * pv;
    for (int i = tid; i < n2; i += nt) w[i] -= K * v[i];
    __syncthreads();
    double* b22 = A + (int64_t)(k + 1) * m + (k + 1);
    const int64_t tot = (int64_t)n2 * n2;
    for (int64_t t = tid; t < tot; t += nt) {
      const int j = (int)(t / n2), i = (int)(t - (int64_t)j * n2);
      b22[i + (int64_t)j * m] -= v[i] * w[j] + w[i] * v[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (m >= 2) {
      d[m - 2] = A[(m - 2) + (int64_t)(m - 2) * m];
      e[m - 2] = A[(m - 1) + (int64_t)(m - 2) * m];
      tau[m - 2] = 0.0;
    }
    d[m - 1] = A[(m - 1) + (int64_t)(m - 1) * m];
  }
}

__device__ int sturm_count(int m, const double* __restrict__ d, const double* __restrict__ e, double x,
                           double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int j = 1; j < m; ++j) {
    q = (d[j] - x) - e[j - 1] * e[j - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

__global__ __launch_bounds__(256) void k_bisect(int m, const double* __restrict__ d, const double* __restrict__ e,
                                                double* __restrict__ theta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
  for (int j = 0; j < m; ++j) {
    const double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + (j < m - 1 ? fabs(e[j]) : 0.0);
    lo = fmin(lo, d[j] - r);
    hi = fmax(hi, d[j] + r);
    if (j < m - 1) emax2 = fmax(emax2, e[j] * e[j]);
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double tn = fmax(fabs(lo), fabs(hi));
  lo -= 2.0 * DBL_EPSILON * tn + pivmin;
  hi += 2.0 * DBL_EPSILON * tn + pivmin;
  for (int it = 0; it < 256; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    if (sturm_count(m, d, e, mid, pivmin) > i)
      hi = mid;
    else
      lo = mid;
  }
  theta[i] = 0.5 * (lo + hi);
}

// Inverse iteration, one lane per cluster of selected eigenvalues.
__global__ __launch_bounds__(64) void k_invit(int m, const double* __restrict__ d, const double* __restrict__ e,
                                              int ncl, const int32_t* __restrict__ cstart,
                                              const double* __restrict__ sel, double* __restrict__ Z,
                                              double* __restrict__ scratch) {
  const int cl = blockIdx.x * blockDim.x + threadIdx.x;
  if (cl >= ncl) return;
  double tn = 0.0;
  for (int j = 0; j < m; ++j)
    tn = fmax(tn, fabs(d[j]) + (j > 0 ? fabs(e[j - 1]) : 0.0) + (j < m - 1 ? fabs(e[j]) : 0.0));
  const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);
  double prev_lam = -INFINITY;
  for (int s = cstart[cl]; s < cstart[cl + 1]; ++s) {
    double lam = sel[s];
    if (s > cstart[cl] && lam - prev_lam < 10.0 * tiny) lam = prev_lam + 10.0 * tiny;
    prev_lam = lam;
    double* u0 = scratch + (int64_t)s * 5 * m;
    double* u1 = u0 + m;
    double* u2 = u1 + m;
    double* lm = u2 + m;
    double* pv = lm + m;  // 1.0 where rows i, i+1 were swapped
    double* z = Z + (int64_t)s * m;
    // LU of T - lam I with partial pivoting
    u0[0] = d[0] - lam;
    u1[0] = m > 1 ? e[0] : 0.0;
    for (int i = 0; i + 1 < m; ++i) {
      const double bi = e[i];
      const double ai1 = d[i + 1] - lam;
      const double ci1 = (i + 2 < m) ? e[i + 1] : 0.0;
      if (fabs(u0[i]) >= fabs(bi)) {
        const double l = (u0[i] != 0.0) ? bi / u0[i] : 0.0;
        pv[i] = 0.0;
        lm[i] = l;
        u2[i] = 0.0;
        u0[i + 1] = ai1 - l * u1[i];
        u1[i + 1] = ci1;
      } else {
        const double l = u0[i] / bi;
        const double t = u1[i];
        pv[i] = 1.0;
        lm[i] = l;
        u0[i] = bi;
        u1[i] = ai1;
        u2[i] = ci1;
        u0[i + 1] = t - l * ai1;
        u1[i + 1] = -l * ci1;
      }
    }
    u2[m - 1] = 0.0;
    for (int i = 0; i < m; ++i)
      if (fabs(u0[i]) < tiny) u0[i] = u0[i] < 0.0 ? -tiny : tiny;
    // start vector: fixed, generic (no structure that could hide a component)
    for (int i = 0; i < m; ++i) z[i] = 1.0 + 0.5 * sin(0.7 * i + 1.3 * (s - cstart[cl]) + 0.1);
    for (int it = 0; it < 3; ++it) {
      for (int i = 0; i + 1 < m; ++i) {
        if (pv[i] != 0.0) {
          const double t = z[i];
          z[i] = z[i + 1];
          z[i + 1] = t;
        }
        z[i + 1] -= lm[i] * z[i];
      }
      z[m - 1] = z[m - 1] / u0[m - 1];
      if (m >= 2) z[m - 2] = (z[m - 2] - u1[m - 2] * z[m - 1]) / u0[m - 2];
      for (int i = m - 3; i >= 0; --i) z[i] = (z[i] - u1[i] * z[i + 1] - u2[i] * z[i + 2]) / u0[i];
      // keep clear of overflow before re-orthogonalising
      double mx = 0.0;
      for (int i = 0; i < m; ++i) mx = fmax(mx, fabs(z[i]));
      if (mx > 0.0) {
        const double r = 1.0 / mx;
        for (int i = 0; i < m; ++i) z[i] *= r;
      }
      for (int q = cstart[cl]; q < s; ++q) {
        const double* zq = Z + (int64_t)q * m;
        double dot = 0.0;
        for (int i = 0; i < m; ++i) dot = fma(zq[i], z[i], dot);
        for (int i = 0; i < m; ++i) z[i] -= dot * zq[i];
      }
      double nrm = 0.0;
      for (int i = 0; i < m; ++i) nrm = fma(z[i], z[i], nrm);
      nrm = sqrt(nrm);
      const double r = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int i = 0; i < m; ++i) z[i] *= r;
    }
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
  double* ptrs[] = {w.A, w.d, w.e, w.tau, w.theta, w.Z, w.Y, w.scratch, w.sel};
  for (double* p : ptrs)
    if (p) (void)hipFree(p);
  if (w.cl) (void)hipFree(w.cl);
  w = EigWork();
}

int eig_reserve(EigWork& w, int m, int nsel) {
  if ((size_t)m > w.cap_m) {
    double** ps[] = {&w.A, &w.d, &w.e, &w.tau, &w.theta};
    for (double** p : ps) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    const size_t mm = (size_t)m;
    if (hipMalloc(&w.A, sizeof(double) * mm * mm) != hipSuccess || hipMalloc(&w.d, sizeof(double) * mm) != hipSuccess ||
        hipMalloc(&w.e, sizeof(double) * mm) != hipSuccess || hipMalloc(&w.tau, sizeof(double) * mm) != hipSuccess ||
        hipMalloc(&w.theta, sizeof(double) * mm) != hipSuccess) {
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
        hipMalloc(&w.scratch, sizeof(double) * 5 * w.cap_m * ns) != hipSuccess ||
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
  const size_t lds = sizeof(double) * (2 * (size_t)k + 32);
  hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(1024), lds, st, k, w.A, w.d, w.e, w.tau);
  KF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bisect, dim3(cdiv(k, 256)), dim3(256), 0, st, k, w.d, w.e, w.theta);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int eig_vectors(EigWork& w, int k, const double* theta_sel, const int32_t* cluster_start, int nclusters, int nsel,
                hipStream_t st) {
  if (nsel <= 0) return KF_OK;
  KF_TRY(eig_reserve(w, k, nsel));
  KF_HIP(hipMemcpyAsync(w.sel, theta_sel, sizeof(double) * nsel, hipMemcpyHostToDevice, st));
  KF_HIP(hipMemcpyAsync(w.cl, cluster_start, sizeof(int32_t) * (nclusters + 1), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_invit, dim3(cdiv(nclusters, 64)), dim3(64), 0, st, k, w.d, w.e, nclusters, w.cl, w.sel, w.Z,
                     w.scratch);
  KF_HIP(hipGetLastError());
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
