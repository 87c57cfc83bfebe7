// Float64 kernels around the hot path: tall-skinny products for M-inner
// Gram-Schmidt and the projected pencil (Section 2.1 eq. projevp; the
// orthogonalisation loop of Algorithm 2.5), SpMV with S, and the residuals of
// Section 2.4 (eq. res).  All reductions are two-pass with a fixed summation
// order (bitwise repeatable).

#include <hip/hip_runtime.h>

#include <cfloat>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kf_internal.h"

namespace kf {

namespace {

inline int ceil_div64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Consecutive workgroup ids are dealt round-robin to the 8 XCDs; renumber
// them so that each XCD receives one contiguous range of row slices and its
// L2 keeps the neighbouring rows it gathers.
__device__ __forceinline__ int xcd_map(int i, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = i & 7, t = i >> 3;
  return (x < r) ? x * (q + 1) + t : r * (q + 1) + (x - r) * q + t;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum of p[i * stride], i < count, by one wavefront in a fixed order: lane l
// takes i = l, l + 64, ... into four interleaved sums (four independent loads
// in flight instead of a chain of dependent ones), then the lanes combine.
__device__ __forceinline__ double wave_strided_sum(const double* __restrict__ p, int count, int64_t stride, int lane) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = lane;
  for (; i + 192 < count; i += 256) {
    s0 += p[(int64_t)i * stride];
    s1 += p[(int64_t)(i + 64) * stride];
    s2 += p[(int64_t)(i + 128) * stride];
    s3 += p[(int64_t)(i + 192) * stride];
  }
  for (; i < count; i += 64) s0 += p[(int64_t)i * stride];
  return wave_sum((s0 + s1) + (s2 + s3));
}

// ------------------------------------------------------- tall-skinny float64
// Stage 1 of H = Bk^T diag(w) X: one workgroup per (row chunk, group of 64
// basis columns); the weighted X chunk sits in LDS.  Each wavefront streams
// Q basis columns at once with the row loop unrolled U times, so Q*U
// independent loads per lane are in flight (one column at a time leaves the
// wave waiting on a single load and reaches only about half of HBM
// bandwidth); the X values read from LDS are shared by the Q columns.
template <int NR, int Q, int U>
__global__ __launch_bounds__(256) void k_gemv_t(int32_t n, int k, const double* __restrict__ Bk, int64_t ldb,
                                                const double* __restrict__ X1, int n1, int64_t ldx1,
                                                const double* __restrict__ X2, int n2, int64_t ldx2,
                                                const double* __restrict__ m, double* __restrict__ partial, int CH) {
  extern __shared__ double xs[];
  const int nrhs = n1 + n2;
  // right-hand sides g0 .. g0 + nloc - 1 (groups of NR along the grid's z)
  const int g0 = blockIdx.z * NR;
  const int nloc = min(NR, nrhs - g0);
  const int chunk = blockIdx.x;
  const int64_t r0 = (int64_t)chunk * CH;
  const int rows = (int)std::min<int64_t>(CH, (int64_t)n - r0);
  for (int t = threadIdx.x; t < CH * nloc; t += blockDim.x) {
    const int c = g0 + t / CH, r = t % CH;
    double v = 0.0;
    if (r < rows) {
      const int64_t i = r0 + r;
      v = c < n1 ? X1[i + (int64_t)c * ldx1] : X2[i + (int64_t)(c - n1) * ldx2] * m[i];
    }
    xs[t] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nchunks = gridDim.x;
  const int j0 = blockIdx.y * 64;
  for (int jj = wave * Q; jj < 64; jj += 4 * Q) {
    const int jb = j0 + jj;
    if (jb >= k) break;
    // columns past k repeat column k-1 (in bounds) and are not stored
    const double* bc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) bc[q] = Bk + (int64_t)std::min(jb + q, k - 1) * ldb + r0;
    double s[Q][NR];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int c = 0; c < NR; ++c) s[q][c] = 0.0;
    int r = lane;
    for (; r + 64 * (U - 1) < rows; r += 64 * U) {
      double bv[U][Q];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < Q; ++q) bv[u][q] = bc[q][r + 64 * u];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < NR; ++c)
          if (c < nloc) {
            const double xv = xs[c * CH + r + 64 * u];
#pragma unroll
            for (int q = 0; q < Q; ++q) s[q][c] = fma(bv[u][q], xv, s[q][c]);
          }
    }
    for (; r < rows; r += 64) {
      double bv[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) bv[q] = bc[q][r];
#pragma unroll
      for (int c = 0; c < NR; ++c)
        if (c < nloc) {
          const double xv = xs[c * CH + r];
#pragma unroll
          for (int q = 0; q < Q; ++q) s[q][c] = fma(bv[q], xv, s[q][c]);
        }
    }
    // layout [output (j, c)][chunk]: the second pass reads each output's
    // partials contiguously
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int c = 0; c < NR; ++c)
        if (c < nloc) {
          const double v = wave_sum(s[q][c]);
          if (lane == 0 && jb + q < k) partial[((int64_t)(jb + q) * nrhs + g0 + c) * nchunks + chunk] = v;
        }
  }
}


typedef double f64x4 __attribute__((ext_vector_type(4)));

// H = Bk^T diag(w) X for four or more right-hand sides on the float64 matrix
// cores (v_mfma_f64_16x16x4f64: a 16 x 4 by 4 x 16 product per instruction,
// the sum over rows happening inside the accumulator, so no cross-lane
// reductions).  Workgroup: a chunk of TCH rows and 128 basis columns (eight
// wavefronts, one 16-column tile each), NX right-hand sides of group
// blockIdx.z (NX = 8, 16 or 32; absent ones are zero; 32 = two 16-wide
// accumulators sharing each basis operand).  The weighted X chunk is staged
// in LDS SUB rows at a time as [row/4][c][row%4].  Within each 16-row block,
// lane l (c = l%16, q = l/16) owns rows 4q .. 4q+3: it loads them as one
// 32-byte run of basis column c of its tile and reads the matching four X
// values of right-hand side c (and c + 16) as one 32-byte LDS run each;
// instruction t of the four takes A[j = c][r = q] = Bk[4q+t][c] and
// B[r = q][c] = X[4q+t][c].  Its accumulator register v holds
// D[j = 4v + l/16][c = l%16] (the f64 layout interleaves rows by register).
// `vec`: Bk's columns are 32-byte aligned (else the run is loaded one
// element at a time).
constexpr int kMfmaWaves = 8;
template <int NX, int SUB, int PF>
__global__ __launch_bounds__(64 * kMfmaWaves) void k_gemv_t_mfma(
    int32_t n, int k, const double* __restrict__ Bk, int64_t ldb, const double* __restrict__ X1, int n1, int64_t ldx1,
    const double* __restrict__ X2, int n2, int64_t ldx2, const double* __restrict__ m, double* __restrict__ partial,
    int TCH, int vec) {
  static_assert(SUB % (16 * PF) == 0, "a batch of PF 16-row blocks must divide the staged rows");
  constexpr int NA = NX > 16 ? 2 : 1;  // accumulators per lane
  __shared__ double4 xs[SUB / 4][NX];
  double* xsd = reinterpret_cast<double*>(&xs[0][0]);
  const int nrhs = n1 + n2;
  const int g0 = blockIdx.z * NX;
  const int nloc = min(NX, nrhs - g0);
  const int chunk = blockIdx.x;
  const int64_t r0 = (int64_t)chunk * TCH;
  const int rows = (int)std::min<int64_t>(TCH, (int64_t)n - r0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int jt = (blockIdx.y * kMfmaWaves + wave) * 16;  // first column of this wavefront's tile
  const int q = lane >> 4, cl = lane & 15;
  const bool jok = jt + cl < k;
  bool cok[NA];
  for (int h = 0; h < NA; ++h) cok[h] = cl + 16 * h < nloc;
  const double* __restrict__ bcol = Bk + (int64_t)(jok ? jt + cl : 0) * ldb + r0;
  f64x4 acc[NA];
  for (int h = 0; h < NA; ++h) acc[h] = (f64x4){0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < rows; s0 += SUB) {
    const int srows = min(SUB, rows - s0);
    __syncthreads();
    for (int t = threadIdx.x; t < NX * SUB; t += 64 * kMfmaWaves) {
      const int c = t / SUB, r = t % SUB;
      double v = 0.0;
      if (c < nloc && r < srows) {
        const int64_t i = r0 + s0 + r;
        const int cg = g0 + c;
        v = cg < n1 ? X1[i + (int64_t)cg * ldx1] : X2[i + (int64_t)(cg - n1) * ldx2] * m[i];
      }
      xsd[((r >> 2) * NX + c) * 4 + (r & 3)] = v;
    }
    __syncthreads();
    if (jt >= k) continue;
    for (int rb = 0; rb < srows; rb += 16 * PF) {
      double4 a[PF];
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int r = rb + 16 * p + 4 * q;
        if (vec && jok && r + 3 < srows) {
          a[p] = *reinterpret_cast<const double4*>(bcol + s0 + r);
        } else {
          a[p].x = (jok && r < srows) ? bcol[s0 + r] : 0.0;
          a[p].y = (jok && r + 1 < srows) ? bcol[s0 + r + 1] : 0.0;
          a[p].z = (jok && r + 2 < srows) ? bcol[s0 + r + 2] : 0.0;
          a[p].w = (jok && r + 3 < srows) ? bcol[s0 + r + 3] : 0.0;
        }
      }
#pragma unroll
      for (int p = 0; p < PF; ++p) {
#pragma unroll
        for (int h = 0; h < NA; ++h) {
          // rows past srows hold zeros in LDS
          const double4 x = cok[h] ? xs[(rb >> 2) + 4 * p + q][cl + 16 * h] : (double4){0.0, 0.0, 0.0, 0.0};
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].x, x.x, acc[h], 0, 0, 0);
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].y, x.y, acc[h], 0, 0, 0);
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].z, x.z, acc[h], 0, 0, 0);
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].w, x.w, acc[h], 0, 0, 0);
        }
      }
    }
  }
  if (jt >= k) return;
  const int nchunks = gridDim.x;
  for (int h = 0; h < NA; ++h) {
    if (!cok[h]) continue;
    const int c = g0 + cl + 16 * h;
    for (int v = 0; v < 4; ++v) {
      const int j = jt + 4 * v + q;
      if (j < k) partial[((int64_t)j * nrhs + c) * nchunks + chunk] = acc[h][v];
    }
  }
}

// The same product for 32-byte aligned basis columns (ldb a multiple of 4):
// the staging of the X chunk issues all of a thread's loads at once (thread
// t stages row t % SUB of the right-hand sides t / SUB, t / SUB + G, ..., with
// m[i] read once per row), the basis operand of the next 16*PF rows is loaded
// while the current ones are multiplied, and the basis loads of full blocks
// are unconditional (lanes past column k read column k-1, rows past the
// chunk's last read its last row: both are multiplied by zeros or not
// stored).  About 10 % faster than the general kernel at every width.
template <int NX, int SUB, int PF>
__global__ __launch_bounds__(64 * kMfmaWaves) void k_gemv_t_mfma_a(
    int32_t n, int k, const double* __restrict__ Bk, int64_t ldb, const double* __restrict__ X1, int n1, int64_t ldx1,
    const double* __restrict__ X2, int n2, int64_t ldx2, const double* __restrict__ m, double* __restrict__ partial,
    int TCH) {
  constexpr int NA = (NX + 15) / 16;
  constexpr int G = 64 * kMfmaWaves / SUB;
  constexpr int CPT = NX / G;
  static_assert(G * SUB == 64 * kMfmaWaves && CPT * G == NX, "staging layout");
  static_assert(SUB % (16 * PF) == 0, "a batch of PF 16-row blocks must divide the staged rows");
  __shared__ double4 xs[SUB / 4][NX];
  double* xsd = reinterpret_cast<double*>(&xs[0][0]);
  const int nrhs = n1 + n2;
  const int g0 = blockIdx.z * NX;
  const int nloc = min(NX, nrhs - g0);
  const int chunk = blockIdx.x;
  const int64_t r0 = (int64_t)chunk * TCH;
  const int rows = (int)std::min<int64_t>(TCH, (int64_t)n - r0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int jt = (blockIdx.y * kMfmaWaves + wave) * 16;
  const int q = lane >> 4, cl = lane & 15;
  const bool wok = jt < k;
  bool cok[NA];
  for (int h = 0; h < NA; ++h) cok[h] = cl + 16 * h < nloc;
  const double* __restrict__ bcol = Bk + (int64_t)min(jt + cl, k - 1) * ldb + r0;
  const int sr = threadIdx.x % SUB, sg = threadIdx.x / SUB;
  f64x4 acc[NA];
  for (int h = 0; h < NA; ++h) acc[h] = (f64x4){0.0, 0.0, 0.0, 0.0};
  double4 a[PF], an[PF];
  auto load_full = [&](int r, double4 (&dst)[PF]) {
#pragma unroll
    for (int p = 0; p < PF; ++p) dst[p] = *reinterpret_cast<const double4*>(bcol + r + 16 * p + 4 * q);
  };
  for (int s0 = 0; s0 < rows; s0 += SUB) {
    const int srows = min(SUB, rows - s0);
    double xv[CPT];
    {
      const int row = s0 + sr;
      const bool rok = row < rows;
      const int64_t i = r0 + (rok ? row : rows - 1);
      const double mi = m ? m[i] : 1.0;
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int c = sg + G * u;
        const int cg = g0 + (c < nloc ? c : 0);
        const double* col = cg < n1 ? X1 + (int64_t)cg * ldx1 : X2 + (int64_t)(cg - n1) * ldx2;
        xv[u] = col[i];
      }
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int c = sg + G * u;
        xv[u] = (rok && c < nloc) ? (g0 + c >= n1 ? xv[u] * mi : xv[u]) : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int c = sg + G * u;
      xsd[((sr >> 2) * NX + c) * 4 + (sr & 3)] = xv[u];
    }
    __syncthreads();
    if (!wok) continue;
    const int full = srows / (16 * PF) * (16 * PF);
    if (full > 0) load_full(s0, a);
    int rb = 0;
    for (; rb < full; rb += 16 * PF) {
      if (rb + 16 * PF < full) load_full(s0 + rb + 16 * PF, an);
#pragma unroll
      for (int p = 0; p < PF; ++p) {
#pragma unroll
        for (int h = 0; h < NA; ++h) {
          const double4 x = cok[h] ? xs[(rb >> 2) + 4 * p + q][cl + 16 * h] : (double4){0.0, 0.0, 0.0, 0.0};
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].x, x.x, acc[h], 0, 0, 0);
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].y, x.y, acc[h], 0, 0, 0);
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].z, x.z, acc[h], 0, 0, 0);
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p].w, x.w, acc[h], 0, 0, 0);
        }
      }
#pragma unroll
      for (int p = 0; p < PF; ++p) a[p] = an[p];
    }
    for (; rb < srows; rb += 16) {
      // the last rows of the chunk: LDS holds zeros past srows
      const int r = rb + 4 * q;
      double4 t;
      t.x = bcol[s0 + min(r, srows - 1)];
      t.y = bcol[s0 + min(r + 1, srows - 1)];
      t.z = bcol[s0 + min(r + 2, srows - 1)];
      t.w = bcol[s0 + min(r + 3, srows - 1)];
#pragma unroll
      for (int h = 0; h < NA; ++h) {
        const double4 x = cok[h] ? xs[(rb >> 2) + q][cl + 16 * h] : (double4){0.0, 0.0, 0.0, 0.0};
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(t.x, x.x, acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(t.y, x.y, acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(t.z, x.z, acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(t.w, x.w, acc[h], 0, 0, 0);
      }
    }
  }
  if (!wok) return;
  const int nchunks = gridDim.x;
  for (int h = 0; h < NA; ++h) {
    if (!cok[h]) continue;
    const int c = g0 + cl + 16 * h;
    for (int v = 0; v < 4; ++v) {
      const int j = jt + 4 * v + q;
      if (j < k) partial[((int64_t)j * nrhs + c) * nchunks + chunk] = acc[h][v];
    }
  }
}

// V = Bk Y (n x k times k x nc) on the float64 matrix cores.  A wavefront
// owns 32 rows (two 16-row tiles) and the up to four 16-column tiles of its
// 64-column group that lie below nc; each Y value read from LDS feeds both
// row tiles.  Lane l supplies A[r = l%16][j = l/16] = Bk[r][j] (four 128-byte
// row runs per instruction) and B[j = l/16][c = l%16] = Y[j][c], read from a
// GJ x 64 slice of Y staged in LDS with c contiguous; its accumulator
// register v holds D[r = 4v + l/16][c = l%16].  The basis operand of the next
// slice is loaded while the current one is multiplied.
constexpr int kGemmJ = 16;
constexpr int kGemmRT = 2;
__global__ __launch_bounds__(256) void k_gemm_nn_mfma(int32_t n, int k, const double* __restrict__ Bk, int64_t ldb,
                                                      const double* __restrict__ Y, int64_t ldy, double* __restrict__ V,
                                                      int64_t ldv, int nc) {
  constexpr int S = kGemmJ / 4;
  __shared__ double ys[kGemmJ][64 + 2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t rt = ((int64_t)blockIdx.x * 4 + wave) * 16 * kGemmRT;  // first row of this wavefront
  const bool live = rt < n;
  const int c0 = blockIdx.y * 64;
  const int ntile = std::min(4, (nc - c0 + 15) / 16);
  const int q = lane >> 4, cl = lane & 15;
  f64x4 acc[kGemmRT][4];
#pragma unroll
  for (int r = 0; r < kGemmRT; ++r)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[r][t] = (f64x4){0.0, 0.0, 0.0, 0.0};
  double a[kGemmRT][S], an[kGemmRT][S];
  auto load = [&](int jb, double (&dst)[kGemmRT][S]) {
#pragma unroll
    for (int r = 0; r < kGemmRT; ++r) {
      const int64_t ra = rt + 16 * r + cl;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int j = jb + 4 * s + q;
        dst[r][s] = (ra < n && j < k) ? Bk[ra + (int64_t)j * ldb] : 0.0;
      }
    }
  };
  if (live) load(0, a);
  for (int jb = 0; jb < k; jb += kGemmJ) {
    __syncthreads();
    for (int t = threadIdx.x; t < kGemmJ * 16 * ntile; t += blockDim.x) {
      const int c = t / kGemmJ, j = t % kGemmJ;  // consecutive threads: consecutive j (coalesced)
      ys[j][c] = (jb + j < k && c0 + c < nc) ? Y[(jb + j) + (int64_t)(c0 + c) * ldy] : 0.0;
    }
    __syncthreads();
    if (!live) continue;
    if (jb + kGemmJ < k) load(jb + kGemmJ, an);
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < ntile) {
          const double b = ys[4 * s + q][16 * t + cl];
#pragma unroll
          for (int r = 0; r < kGemmRT; ++r)
            acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][s], b, acc[r][t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kGemmRT; ++r)
#pragma unroll
      for (int s = 0; s < S; ++s) a[r][s] = an[r][s];
  }
  if (!live) return;
  // constant trip counts: the accumulators stay in registers
#pragma unroll
  for (int r = 0; r < kGemmRT; ++r)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = c0 + 16 * t + cl;
      if (t >= ntile || c >= nc) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = rt + 16 * r + 4 * v + q;
        if (row < n) V[row + (int64_t)c * ldv] = acc[r][t][v];
      }
    }
}

__global__ __launch_bounds__(256) void k_reduce_partial(int nchunks, int k, int nrhs,
                                                        const double* __restrict__ partial, double* __restrict__ H,
                                                        int64_t ldh) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= k * nrhs) return;
  const double s = wave_strided_sum(partial + (int64_t)t * nchunks, nchunks, 1, lane);
  if (lane == 0) {
    const int j = t / nrhs, c = t - j * nrhs;
    H[j + (int64_t)c * ldh] = s;
  }
}

// X[:, c] (-)= Bk * H[:, c]   (SUB: subtract from X; else V = Bk H)
template <int NR, bool SUB>
__global__ __launch_bounds__(256) void k_gemv_n(int32_t n, int k, const double* __restrict__ Bk, int64_t ldb,
                                                const double* __restrict__ H, int64_t ldh, double* X, int64_t ldx,
                                                int nrhs, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  constexpr int JT = 128;
  __shared__ double hs[JT * NR];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c0 = blockIdx.y * NR;
  const int nc = std::min(NR, nrhs - c0);
  double acc[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = 0.0;
  for (int j0 = 0; j0 < k; j0 += JT) {
    const int jt = std::min(JT, k - j0);
    __syncthreads();
    for (int t = threadIdx.x; t < jt * NR; t += blockDim.x) {
      const int j = t / NR, c = t - j * NR;
      hs[t] = c < nc ? H[(j0 + j) + (int64_t)(c0 + c) * ldh] : 0.0;
    }
    __syncthreads();
    if (i < n) {
      const double* __restrict__ bp = Bk + i + (int64_t)j0 * ldb;
      for (int j = 0; j < jt; ++j) {
        const double bv = bp[(int64_t)j * ldb];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = fma(bv, hs[j * NR + c], acc[c]);
      }
    }
  }
  if (i < n) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      if (c < nc) {
        double* xp = X + i + (int64_t)(c0 + c) * ldx;
        if (SUB)
          *xp -= acc[c];
        else
          *xp = acc[c];
      }
    }
  }
}

template <typename IT, int NC>
__global__ __launch_bounds__(256) void k_spmv_cols(int32_t n, int32_t nslices, const int64_t* __restrict__ sptr,
                                                   const double* __restrict__ val, const IT* __restrict__ idx,
                                                   const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                                                   int64_t ldy, int ncols, const double* __restrict__ rscale) {
  constexpr bool relative = sizeof(IT) == 2;
  const int slice = xcd_map(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (slice >= nslices) return;
  const int row = slice * 64 + lane;
  if (row >= n) return;
  const int64_t base = sptr[slice];
  const int width = (int)((sptr[slice + 1] - base) >> 6);
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  // every column's gather is issued unconditionally (columns past ncols read
  // column ncols-1 again and are not stored), so all NC loads of an entry are
  // in flight together
  const double* __restrict__ xc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) xc[c] = X + (int64_t)(c < ncols ? c : ncols - 1) * ldx;
  for (int q = 0; q < width; ++q) {
    const double a = val[base + (int64_t)q * 64 + lane];
    const IT ci = idx[base + (int64_t)q * 64 + lane];
    const int64_t col = relative ? row + (int)ci : (int)ci;
    double xv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xv[c] = xc[c][col];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = fma(a, xv[c], acc[c]);
  }
  const double sc = rscale ? rscale[row] : 1.0;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c < ncols) Y[row + (int64_t)c * ldy] = acc[c] * sc;
}

__global__ __launch_bounds__(256) void k_normalize_col(int32_t n, double* __restrict__ x,
                                                       const double* __restrict__ nrm2,
                                                       const double* __restrict__ ref2, double drop,
                                                       int32_t* __restrict__ flag, double* __restrict__ out_norm) {
  const double nr = sqrt(fmax(*nrm2, 0.0));
  const double rf = ref2 ? sqrt(fmax(*ref2, 0.0)) : 0.0;
  const bool keep = isfinite(nr) && nr > 0.0 && nr > drop * rf;
  const double sc = keep ? 1.0 / nr : 0.0;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = keep ? x[i] * sc : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (flag) *flag = keep ? 1 : 0;
    if (out_norm) *out_norm = nr;
  }
}

// partial[(chunk*nc + c)*2 + {0,1}] = sums over the chunk of
// (SV - theta m V)^2 and SV^2 for column c
__global__ __launch_bounds__(256) void k_resid_partial(int32_t n, const double* __restrict__ SV,
                                                       const double* __restrict__ V, int64_t ld,
                                                       const double* __restrict__ m,
                                                       const double* __restrict__ theta, int nc, int CH,
                                                       double* __restrict__ partial) {
  __shared__ double red[2][4];
  const int chunk = blockIdx.x, c = blockIdx.y;
  const int64_t r0 = (int64_t)chunk * CH;
  const int64_t r1 = std::min<int64_t>(r0 + CH, n);
  const double th = theta[c];
  double a = 0.0, b = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double sv = SV[i + (int64_t)c * ld];
    const double t = sv - th * m[i] * V[i + (int64_t)c * ld];
    a = fma(t, t, a);
    b = fma(sv, sv, b);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[((int64_t)chunk * nc + c) * 2 + 0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    partial[((int64_t)chunk * nc + c) * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// one wavefront per column: the sums over chunks of both quantities
__global__ __launch_bounds__(256) void k_resid_reduce(int nchunks, int nc, const double* __restrict__ partial,
                                                      double* __restrict__ num, double* __restrict__ den) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nc) return;
  const double a = wave_strided_sum(partial + (int64_t)c * 2, nchunks, (int64_t)nc * 2, lane);
  const double b = wave_strided_sum(partial + (int64_t)c * 2 + 1, nchunks, (int64_t)nc * 2, lane);
  if (lane == 0) {
    num[c] = a;
    den[c] = b;
  }
}

__global__ __launch_bounds__(256) void k_copy_cols(int32_t n, const double* __restrict__ src, int64_t lds,
                                                   double* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < n) dst[i + (int64_t)c * ldd] = src[i + (int64_t)c * lds];
}

__global__ __launch_bounds__(256) void k_rr_scatter(int k, int c0, int nc, const double* __restrict__ T,
                                                    int64_t ldt, double* __restrict__ H, double* __restrict__ G,
                                                    int64_t ldh) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * nc) return;
  const int c = t / k, j = t - c * k;
  const int col = c0 + c;
  double h, g;
  if (j < c0) {
    h = T[j + (int64_t)c * ldt];
    g = T[j + (int64_t)(nc + c) * ldt];
  } else {
    const int cj = j - c0;  // j is itself a new column
    h = 0.5 * (T[j + (int64_t)c * ldt] + T[col + (int64_t)cj * ldt]);
    g = 0.5 * (T[j + (int64_t)(nc + c) * ldt] + T[col + (int64_t)(nc + cj) * ldt]);
  }
  H[j + (int64_t)col * ldh] = h;
  H[col + (int64_t)j * ldh] = h;
  G[j + (int64_t)col * ldh] = g;
  G[col + (int64_t)j * ldh] = g;
}

__global__ __launch_bounds__(256) void k_symmetrize(int k, double* __restrict__ A, int64_t lda) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * k) return;
  const int64_t j = t / k, i = t - j * k;
  if (i <= j) return;
  const double v = 0.5 * (A[i + j * lda] + A[j + i * lda]);
  A[i + j * lda] = v;
  A[j + i * lda] = v;
}

__global__ __launch_bounds__(1024) void k_orth_error(int k, const double* __restrict__ G, int64_t ldg,
                                                     double* __restrict__ out) {
  __shared__ double red[16];
  double mx = 0.0;
  const int64_t tot = (int64_t)k * k;
  for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
    const int64_t c = t / k, j = t - c * k;
    const double v = fabs(G[j + c * ldg] - (j == c ? 1.0 : 0.0));
    mx = v > mx ? v : mx;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    *out = r;
  }
}


// First-order correction of the projected pencil for a basis that is
// M-orthonormal only up to E = G - I: (H, G) has, to O(|E|^2), the
// eigenvalues of Hc = H - (E H + H E)/2 and the eigenvectors (I - E/2) y.
__global__ __launch_bounds__(256) void k_sub_identity(int k, const double* __restrict__ G, int64_t ldg,
                                                      double* __restrict__ E) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * k) return;
  const int j = (int)(t / k), i = (int)(t - (int64_t)j * k);
  E[t] = G[i + (int64_t)j * ldg] - (i == j ? 1.0 : 0.0);
}

__global__ __launch_bounds__(256) void k_h_correct(int k, const double* __restrict__ H, int64_t ldh,
                                                   const double* __restrict__ EH, double* __restrict__ Hc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * k) return;
  const int j = (int)(t / k), i = (int)(t - (int64_t)j * k);
  Hc[t] = H[i + (int64_t)j * ldh] - 0.5 * (EH[t] + EH[j + (int64_t)i * k]);
}

__global__ __launch_bounds__(256) void k_axpy(int64_t count, double a, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) y[t] = fma(a, x[t], y[t]);
}


// Three-term Gram-Schmidt step of one column in three launches (the window
// pass of Algorithm 2.5 in the M inner product).  k_window_dots writes the
// per-chunk partial sums of the lw window columns' products with x (L's
// column lw is x), x^T M x, and the window's own Gram matrix:
//   D = [L_0^T M x, .., L_{lw-1}^T M x, x^T M x, L_0^T M L_0, L_0^T M L_1, L_1^T M L_1]
// (the last two only for lw = 2).
constexpr int kWinCH = 1024;
__host__ __device__ constexpr int window_dot_count(int lw) { return lw + 1 + lw * (lw + 1) / 2; }
__global__ __launch_bounds__(256) void k_window_dots(int32_t n, int lw, const double* __restrict__ L, int64_t ldl,
                                                     const double* __restrict__ m, double* __restrict__ partial) {
  __shared__ double red[4][6];
  const int chunk = blockIdx.x, nchunks = gridDim.x;
  const int nd = window_dot_count(lw);
  const int64_t r0 = (int64_t)chunk * kWinCH;
  const int rows = (int)std::min<int64_t>(kWinCH, (int64_t)n - r0);
  const double* __restrict__ x = L + (int64_t)lw * ldl;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  auto add = [&](double xi, double mi, double l0, double l1) {
    const double xm = xi * mi;
    if (lw == 2) {
      s[0] = fma(l0, xm, s[0]);
      s[1] = fma(l1, xm, s[1]);
      s[2] = fma(xi, xm, s[2]);
      const double l0m = l0 * mi;
      s[3] = fma(l0, l0m, s[3]);
      s[4] = fma(l1, l0m, s[4]);
      s[5] = fma(l1, l1 * mi, s[5]);
    } else if (lw == 1) {
      s[0] = fma(l0, xm, s[0]);
      s[1] = fma(xi, xm, s[1]);
      s[2] = fma(l0, l0 * mi, s[2]);
    } else {
      s[0] = fma(xi, xm, s[0]);
    }
  };
  if (rows == kWinCH) {
    // a full chunk: every load of the thread's four rows issued before the
    // sums (same order of summation as the loop below)
    constexpr int U = kWinCH / 256;
    double xv[U], mv[U], l0v[U], l1v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = r0 + threadIdx.x + 256 * u;
      xv[u] = x[i];
      mv[u] = m[i];
      l0v[u] = lw > 0 ? L[i] : 0.0;
      l1v[u] = lw > 1 ? L[i + ldl] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) add(xv[u], mv[u], l0v[u], l1v[u]);
  } else {
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
      const int64_t i = r0 + r;
      add(x[i], m[i], lw > 0 ? L[i] : 0.0, lw > 1 ? L[i + ldl] : 0.0);
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = 0; d < 6; ++d) {
    const double v = wave_sum(s[d]);
    if (lane == 0) red[wave][d] = v;
  }
  __syncthreads();
  const int d = (int)threadIdx.x;
  if (d < nd) partial[(int64_t)d * nchunks + chunk] = ((red[0][d] + red[1][d]) + red[2][d]) + red[3][d];
}

// One workgroup sums the partials in chunk order and forms c_j = L_j^T M x
// and g = x^T M x - 2 c^T c + c^T G c (G the window's Gram matrix): the exact
// M-norm^2 after the pass, to rounding of order eps * x^T M x.  When
// g < 1e-4 x^T M x that rounding is no longer small: status 2 tells the caller
// to normalise explicitly (x is then only subtracted).  Writes T = [c, x^T M x],
// coef = {c_0, c_1, scale} for k_window_scale and rec = {T[0..lw], g, status}.
__global__ __launch_bounds__(512) void k_window_reduce(int lw, const double* __restrict__ partial, int nchunks,
                                                       double* __restrict__ T, double* __restrict__ coef,
                                                       double* __restrict__ rec, double* __restrict__ hrec) {
  __shared__ double ds[6];
  const int nd = window_dot_count(lw);
  // (a wavefront per sum: at most six sums, eight wavefronts)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int d = wave; d < nd; d += nw) {
    const double v = wave_strided_sum(partial + (int64_t)d * nchunks, nchunks, 1, lane);
    if (lane == 0) ds[d] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double c0 = lw > 0 ? ds[0] : 0.0, c1 = lw > 1 ? ds[1] : 0.0;
  const double txx = ds[lw];
  double g = txx;
  if (lw == 2) {
    g += c0 * (c0 * ds[3] - 2.0 * c0) + c1 * (c1 * ds[5] - 2.0 * c1) + 2.0 * c0 * c1 * ds[4];
  } else if (lw == 1) {
    g += c0 * (c0 * ds[2] - 2.0 * c0);
  }
  const bool strong = !(g > 0.0 && g >= 1e-4 * txx);
  coef[0] = c0;
  coef[1] = c1;
  coef[2] = strong ? 1.0 : 1.0 / sqrt(g);
  for (int j = 0; j <= lw; ++j) {
    T[j] = ds[j];
    rec[j] = ds[j];
  }
  rec[lw + 1] = g;
  rec[lw + 2] = strong ? 2.0 : 1.0;
  if (hrec) {
    for (int j = 0; j <= lw + 2; ++j) hrec[j] = rec[j];
  }
}

// x <- (x - c_0 L_0 - c_1 L_1) * scale with the coefficients of k_window_reduce
// (four rows per thread, 256 apart: every load issued before the stores)
__global__ __launch_bounds__(256) void k_window_scale(int32_t n, int lw, double* __restrict__ L, int64_t ldl,
                                                      const double* __restrict__ coef) {
  constexpr int U = 4;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x * U + threadIdx.x;
  double* x = L + (int64_t)lw * ldl;
  const double c0 = lw > 0 ? coef[0] : 0.0, c1 = lw > 1 ? coef[1] : 0.0, sc = coef[2];
  double v[U], a[U], b[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = i0 + 256 * u;
    const bool ok = i < n;
    v[u] = ok ? x[i] : 0.0;
    a[u] = ok && lw > 0 ? L[i] : 0.0;
    b[u] = ok && lw > 1 ? L[i + ldl] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = i0 + 256 * u;
    if (i >= n) break;
    double t = v[u];
    if (lw > 0) t = fma(-c0, a[u], t);
    if (lw > 1) t = fma(-c1, b[u], t);
    x[i] = t * sc;
  }
}

}  // namespace

int window_step(int32_t n, int lw, double* L, int64_t ldl, const double* m, GemvTWork& wk, double* T, double* rec,
                hipStream_t st, double* host_rec) {
  if (lw < 0 || lw > 2) {
    set_error("window_step: the window holds at most two columns");
    return KF_EINVAL;
  }
  const int nchunks = ceil_div64(n, kWinCH);
  const size_t need = (size_t)window_dot_count(lw) * nchunks;
  if (wk.cap < need) {
    if (wk.partial) (void)hipFree(wk.partial);
    wk.partial = nullptr;
    wk.cap = 0;
    const size_t cap = std::max(need, (size_t)1 << 20);
    if (hipMalloc(&wk.partial, cap * sizeof(double)) != hipSuccess) {
      set_error("window_step: cannot allocate the partial-sum buffer");
      return KF_ENOMEM;
    }
    wk.cap = cap;
  }
  hipLaunchKernelGGL(k_window_dots, dim3(nchunks), dim3(256), 0, st, n, lw, L, ldl, m, wk.partial);
  KF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_window_reduce, dim3(1), dim3(512), 0, st, lw, wk.partial, nchunks, T, rec + 8, rec, host_rec);
  KF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_window_scale, dim3(ceil_div64(n, 1024)), dim3(256), 0, st, n, lw, L, ldl, rec + 8);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int gemv_t(int32_t n, int k, const double* Bk, int64_t ldb, const double* X1, int n1, int64_t ldx1,
           const double* X2, int n2, int64_t ldx2, const double* m, double* H, int64_t ldh, GemvTWork& wk,
           hipStream_t st) {
  const int nrhs = n1 + n2;
  if (k <= 0 || nrhs <= 0) return KF_OK;
  if (nrhs > 64) {
    set_error("gemv_t: at most 64 right-hand sides");
    return KF_EINVAL;
  }
  if (n2 > 0 && m == nullptr) {
    set_error("gemv_t: weighted columns need the mass vector");
    return KF_EINVAL;
  }
  // up to 3 right-hand sides: vector FMAs, rows of a chunk reduced across
  // lanes; wider sets: the matrix cores, one group of 8 or 16, else groups
  // of 32 along the grid's z, chunks of 2048 rows (the sums over rows stay
  // in the accumulators)
  const bool mfma = nrhs > 3;
  const int vec = ((uintptr_t)Bk % 32 == 0 && ldb % 4 == 0) ? 1 : 0;
  // row chunks of 2048 (1024 on the vector path), halved down to 256 while
  // the grid would leave the chip mostly idle (small problems, few columns)
  const int cols_per_wg = mfma ? 16 * kMfmaWaves : 64;
  const int zgroups = !mfma ? 1 : (nrhs <= 16 || (vec && nrhs <= 48) ? 1 : ceil_div64(nrhs, 32));
  int CH = mfma ? 2048 : 1024;
  while (CH > 256 && (int64_t)ceil_div64(n, CH) * ceil_div64(k, cols_per_wg) * zgroups < 1024) CH /= 2;
  const int nchunks = ceil_div64(n, CH);
  const size_t need = (size_t)nchunks * k * nrhs;
  if (wk.cap < need) {
    if (wk.partial) (void)hipFree(wk.partial);
    wk.partial = nullptr;
    wk.cap = 0;
    const size_t cap = std::max(need, (size_t)1 << 20);
    if (hipMalloc(&wk.partial, cap * sizeof(double)) != hipSuccess) {
      set_error("gemv_t: cannot allocate the partial-sum buffer");
      return KF_ENOMEM;
    }
    wk.cap = cap;
  }
  if (!mfma) {
    const dim3 grid(nchunks, ceil_div64(k, 64), 1);
    const size_t lds = sizeof(double) * CH * nrhs;
    if (nrhs == 1)
      hipLaunchKernelGGL((k_gemv_t<1, 4, 2>), grid, dim3(256), lds, st, n, k, Bk, ldb, X1, n1, ldx1, X2, n2, ldx2, m,
                         wk.partial, CH);
    else if (nrhs == 2)
      hipLaunchKernelGGL((k_gemv_t<2, 4, 2>), grid, dim3(256), lds, st, n, k, Bk, ldb, X1, n1, ldx1, X2, n2, ldx2, m,
                         wk.partial, CH);
    else
      hipLaunchKernelGGL((k_gemv_t<4, 4, 2>), grid, dim3(256), lds, st, n, k, Bk, ldb, X1, n1, ldx1, X2, n2, ldx2, m,
                         wk.partial, CH);
  } else {
    const int vec = ((uintptr_t)Bk % 32 == 0 && ldb % 4 == 0 && CH % 64 == 0) ? 1 : 0;
    const int cols = 16 * kMfmaWaves;
    const dim3 block(64 * kMfmaWaves);
    if (vec && nrhs > 32 && nrhs <= 48)
      // (a block of 16 with its pending block's S- and M-products: one pass
      // over the basis instead of two groups of 32)
      hipLaunchKernelGGL((k_gemv_t_mfma_a<48, 128, 2>), dim3(nchunks, ceil_div64(k, cols), 1), block, 0, st, n, k, Bk,
                         ldb, X1, n1, ldx1, X2, n2, ldx2, m, wk.partial, CH);
    else if (vec && nrhs <= 8)
      hipLaunchKernelGGL((k_gemv_t_mfma_a<8, 256, 2>), dim3(nchunks, ceil_div64(k, cols), 1), block, 0, st, n, k, Bk,
                         ldb, X1, n1, ldx1, X2, n2, ldx2, m, wk.partial, CH);
    else if (vec && nrhs <= 16)
      hipLaunchKernelGGL((k_gemv_t_mfma_a<16, 128, 2>), dim3(nchunks, ceil_div64(k, cols), 1), block, 0, st, n, k, Bk,
                         ldb, X1, n1, ldx1, X2, n2, ldx2, m, wk.partial, CH);
    else if (vec)
      hipLaunchKernelGGL((k_gemv_t_mfma_a<32, 128, 2>), dim3(nchunks, ceil_div64(k, cols), ceil_div64(nrhs, 32)), block,
                         0, st, n, k, Bk, ldb, X1, n1, ldx1, X2, n2, ldx2, m, wk.partial, CH);
    else if (nrhs <= 8)
      hipLaunchKernelGGL((k_gemv_t_mfma<8, 256, 4>), dim3(nchunks, ceil_div64(k, cols), 1), block, 0, st, n, k, Bk,
                         ldb, X1, n1, ldx1, X2, n2, ldx2, m, wk.partial, CH, vec);
    else if (nrhs <= 16)
      hipLaunchKernelGGL((k_gemv_t_mfma<16, 256, 2>), dim3(nchunks, ceil_div64(k, cols), 1), block, 0, st, n, k, Bk,
                         ldb, X1, n1, ldx1, X2, n2, ldx2, m, wk.partial, CH, vec);
    else
      hipLaunchKernelGGL((k_gemv_t_mfma<32, 128, 2>), dim3(nchunks, ceil_div64(k, cols), ceil_div64(nrhs, 32)), block,
                         0, st, n, k, Bk, ldb, X1, n1, ldx1, X2, n2, ldx2, m, wk.partial, CH, vec);
  }
  KF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_partial, dim3(ceil_div64((int64_t)k * nrhs, 4)), dim3(256), 0, st, nchunks, k, nrhs,
                     wk.partial, H, ldh);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

// Cholesky factor R of a block's Gram matrix G = X^T M X (nb x nb, nb <= 16,
// leading dimension nb, upper triangle used) and Rinv = R^{-1} (column-major,
// upper triangular), so that X Rinv is M-orthonormal; flags[j] = 1 and
// post[j] = R_jj.  One thread: order at most 16.
__global__ __launch_bounds__(64) void k_chol_inv(int nb, const double* __restrict__ G, double* __restrict__ Rinv,
                                                 int32_t* __restrict__ flags, double* __restrict__ post) {
  __shared__ double R[16][16], Ri[16][16];
  if (threadIdx.x != 0) return;
  for (int j = 0; j < nb; ++j) {
    double s = G[j + j * nb];
    for (int i = 0; i < j; ++i) s -= R[i][j] * R[i][j];
    const double rjj = sqrt(fmax(s, DBL_MIN));
    R[j][j] = rjj;
    for (int k = j + 1; k < nb; ++k) {
      double t = G[j + k * nb];
      for (int i = 0; i < j; ++i) t -= R[i][j] * R[i][k];
      R[j][k] = t / rjj;
    }
    flags[j] = 1;
    post[j] = rjj;
  }
  for (int k = 0; k < nb; ++k) {
    Ri[k][k] = 1.0 / R[k][k];
    for (int j = k - 1; j >= 0; --j) {
      double t = 0.0;
      for (int i = j + 1; i <= k; ++i) t += R[j][i] * Ri[i][k];
      Ri[j][k] = -t / R[j][j];
    }
  }
  for (int k = 0; k < nb; ++k)
    for (int j = 0; j < nb; ++j) Rinv[j + k * nb] = j <= k ? Ri[j][k] : 0.0;
}

// X <- X Rinv in place (Rinv nb x nb upper triangular, nb <= 16): each thread
// reads its row of the block, then writes the transformed row.
__global__ __launch_bounds__(256) void k_apply_upper(int32_t n, int nb, double* __restrict__ X, int64_t ldx,
                                                     const double* __restrict__ Rinv) {
  __shared__ double ri[256];
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) ri[t] = Rinv[t];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = c < nb ? X[i + c * ldx] : 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k >= nb) break;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c <= k; ++c) s = fma(x[c], ri[c + k * nb], s);
    X[i + k * ldx] = s;
  }
}

// *flag = 1 when some x[i] (i < cnt) is not finite (the caller clears it).
__global__ __launch_bounds__(256) void k_nonfinite_flag(int64_t cnt, const double* __restrict__ x,
                                                        int32_t* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) *flag = 1;
}

// The gate of the selective full subtraction: one workgroup, max |c_j|.
__global__ __launch_bounds__(256) void k_reorth_gate(int k, const double* __restrict__ c, const double* __restrict__ g,
                                                     double tol, int32_t* __restrict__ gate) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) mx = fmax(mx, fabs(c[j]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double nrm = sqrt(fmax(*g, 0.0));
    // a non-finite coefficient or norm always subtracts (and is caught later)
    *gate = (mx <= tol * nrm) ? 0 : 1;
  }
}

// Block form: *gate = 0 when every column j < nb of c (rows < k, leading
// dimension ldc) has max_i |c[i, j]| <= tol * sqrt(c[k + j, j]) (its squared
// M-norm sits in row k + j), else 1.
__global__ __launch_bounds__(256) void k_reorth_gate_block(int k, int nb, const double* __restrict__ c, int64_t ldc,
                                                           double tol, int32_t* __restrict__ gate) {
  __shared__ int red[4];
  int over = 0;
  for (int64_t t = threadIdx.x; t < (int64_t)k * nb; t += blockDim.x) {
    const int j = (int)(t / k), i = (int)(t - (int64_t)j * k);
    const double v = fabs(c[i + (int64_t)j * ldc]);
    const double nrm = sqrt(fmax(c[k + j + (int64_t)j * ldc], 0.0));
    // (a non-finite coefficient or norm always subtracts)
    if (!(v <= tol * nrm)) over = 1;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) over |= __shfl_xor(over, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = over;
  __syncthreads();
  if (threadIdx.x == 0) *gate = (red[0] | red[1] | red[2] | red[3]) ? 1 : 0;
}

// Orthogonality of np basis columns p0.. against the whole basis: G[:, c]
// (c < np, leading dimension ldg, rows < k) against the identity.
__global__ __launch_bounds__(256) void k_block_gate(int k, int p0, int np, const double* __restrict__ G, int64_t ldg,
                                                    double tol, int32_t* __restrict__ flag) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int64_t t = threadIdx.x; t < (int64_t)k * np; t += blockDim.x) {
    const int c = (int)(t / k), j = (int)(t - (int64_t)c * k);
    const double v = G[j + (int64_t)c * ldg] - (j == p0 + c ? 1.0 : 0.0);
    mx = fmax(mx, isfinite(v) ? fabs(v) : INFINITY);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) *flag = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) > tol ? 1 : 0;
}

int block_gate(int k, int p0, int np, const double* G, int64_t ldg, double tol, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_block_gate, dim3(1), dim3(256), 0, st, k, p0, np, G, ldg, tol, flag);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

// Coefficients for one subtraction that cleans two columns: out[:, 0] = c_last
// with its own row (kb - 1) zeroed, out[:, 1] = cx (rows < kb, leading
// dimension ldo).  The gate is raised when an entry of c_last exceeds tol,
// so the subtraction runs whenever either column needs it.
__global__ __launch_bounds__(256) void k_pair_coef(int kb, const double* __restrict__ c_last,
                                                   const double* __restrict__ cx, double* __restrict__ out,
                                                   int64_t ldo, double tol, int32_t* __restrict__ gate) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int j = threadIdx.x; j < kb; j += blockDim.x) {
    const double v = j == kb - 1 ? 0.0 : c_last[j];
    out[j] = v;
    out[ldo + j] = cx[j];
    mx = fmax(mx, isfinite(v) ? fabs(v) : INFINITY);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0 && gate && fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) > tol) *gate = 1;
}

int pair_coef(int kb, const double* c_last, const double* cx, double* out, int64_t ldo, double tol, int32_t* gate,
              hipStream_t st) {
  if (kb <= 0) return KF_OK;
  hipLaunchKernelGGL(k_pair_coef, dim3(1), dim3(256), 0, st, kb, c_last, cx, out, ldo, tol, gate);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int chol_orthonormalise(int32_t n, int nb, double* X, int64_t ldx, const double* G, double* Rinv, int32_t* flags,
                        double* post, hipStream_t st) {
  if (nb < 1 || nb > 16) {
    set_error("chol_orthonormalise: block width must lie in [1, 16]");
    return KF_EINVAL;
  }
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(64), 0, st, nb, G, Rinv, flags, post);
  KF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_apply_upper, dim3(ceil_div64(n, 256)), dim3(256), 0, st, n, nb, X, ldx, Rinv);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int nonfinite_flag(int64_t cnt, const double* x, int32_t* flag, hipStream_t st) {
  if (cnt <= 0) return KF_OK;
  const int grid = (int)std::min<int64_t>(1024, ceil_div64(cnt, 256));
  hipLaunchKernelGGL(k_nonfinite_flag, dim3(grid), dim3(256), 0, st, cnt, x, flag);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int reorth_gate(int k, const double* c, const double* g, double tol, int32_t* gate, hipStream_t st) {
  hipLaunchKernelGGL(k_reorth_gate, dim3(1), dim3(256), 0, st, k, c, g, tol, gate);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int reorth_gate_block(int k, int nb, const double* c, int64_t ldc, double tol, int32_t* gate, hipStream_t st) {
  hipLaunchKernelGGL(k_reorth_gate_block, dim3(1), dim3(256), 0, st, k, nb, c, ldc, tol, gate);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int gemv_n_sub(int32_t n, int k, const double* Bk, int64_t ldb, const double* H, int64_t ldh, double* X,
               int64_t ldx, int nrhs, hipStream_t st, const int32_t* gate) {
  if (k <= 0 || nrhs <= 0) return KF_OK;
  // (up to 16 right-hand sides in one pass over the basis)
  const int NR = nrhs <= 1 ? 1 : (nrhs <= 4 ? 4 : (nrhs <= 8 ? 8 : 16));
  const dim3 grid(ceil_div64(n, 256), ceil_div64(nrhs, NR));
  if (NR == 1)
    hipLaunchKernelGGL((k_gemv_n<1, true>), grid, dim3(256), 0, st, n, k, Bk, ldb, H, ldh, X, ldx, nrhs, gate);
  else if (NR == 4)
    hipLaunchKernelGGL((k_gemv_n<4, true>), grid, dim3(256), 0, st, n, k, Bk, ldb, H, ldh, X, ldx, nrhs, gate);
  else if (NR == 8)
    hipLaunchKernelGGL((k_gemv_n<8, true>), grid, dim3(256), 0, st, n, k, Bk, ldb, H, ldh, X, ldx, nrhs, gate);
  else
    hipLaunchKernelGGL((k_gemv_n<16, true>), grid, dim3(256), 0, st, n, k, Bk, ldb, H, ldh, X, ldx, nrhs, gate);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int gemm_nn(int32_t n, int k, const double* Bk, int64_t ldb, const double* Y, int64_t ldy, double* V, int64_t ldv,
            int nc, hipStream_t st) {
  if (nc <= 0) return KF_OK;
  if (nc <= 8) {
    const dim3 grid(ceil_div64(n, 256), ceil_div64(nc, 8));
    hipLaunchKernelGGL((k_gemv_n<8, false>), grid, dim3(256), 0, st, n, k, Bk, ldb, Y, ldy, V, ldv, nc, nullptr);
  } else {
    // a dense product: on the float64 matrix cores, Bk streamed once per 64 columns
    const dim3 grid(ceil_div64(n, 64 * kGemmRT), ceil_div64(nc, 64));
    hipLaunchKernelGGL(k_gemm_nn_mfma, grid, dim3(256), 0, st, n, k, Bk, ldb, Y, ldy, V, ldv, nc);
  }
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int spmv_cols(const SellOp& S, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols, const double* rscale,
              hipStream_t st) {
  if (S.val_bytes != 8) {
    set_error("spmv_cols: needs the float64 operator");
    return KF_EINVAL;
  }
  const int grid = ceil_div64(S.nslices, 4);
  for (int c0 = 0; c0 < ncols; c0 += 16) {
    const int nc = std::min(16, ncols - c0);
    const double* x = X + (int64_t)c0 * ldx;
    double* y = Y + (int64_t)c0 * ldy;
    if (S.idx_bytes == 2) {
      if (nc == 1)
        hipLaunchKernelGGL((k_spmv_cols<int16_t, 1>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int16_t*)S.idx, x, ldx, y, ldy, nc, rscale);
      else if (nc <= 4)
        hipLaunchKernelGGL((k_spmv_cols<int16_t, 4>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int16_t*)S.idx, x, ldx, y, ldy, nc, rscale);
      else if (nc <= 8)
        hipLaunchKernelGGL((k_spmv_cols<int16_t, 8>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int16_t*)S.idx, x, ldx, y, ldy, nc, rscale);
      else if (nc <= 12)
        hipLaunchKernelGGL((k_spmv_cols<int16_t, 12>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int16_t*)S.idx, x, ldx, y, ldy, nc, rscale);
      else
        hipLaunchKernelGGL((k_spmv_cols<int16_t, 16>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int16_t*)S.idx, x, ldx, y, ldy, nc, rscale);
    } else {
      if (nc == 1)
        hipLaunchKernelGGL((k_spmv_cols<int32_t, 1>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int32_t*)S.idx, x, ldx, y, ldy, nc, rscale);
      else if (nc <= 4)
        hipLaunchKernelGGL((k_spmv_cols<int32_t, 4>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int32_t*)S.idx, x, ldx, y, ldy, nc, rscale);
      else if (nc <= 8)
        hipLaunchKernelGGL((k_spmv_cols<int32_t, 8>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int32_t*)S.idx, x, ldx, y, ldy, nc, rscale);
      else
        hipLaunchKernelGGL((k_spmv_cols<int32_t, 16>), dim3(grid), dim3(256), 0, st, S.n, S.nslices, S.slice_ptr,
                           (const double*)S.val, (const int32_t*)S.idx, x, ldx, y, ldy, nc, rscale);
    }
    KF_HIP(hipGetLastError());
  }
  return KF_OK;
}

int normalize_col(int32_t n, double* x, const double* nrm2, const double* ref2, double drop, int32_t* flag,
                  double* out_norm, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize_col, dim3(ceil_div64(n, 256)), dim3(256), 0, st, n, x, nrm2, ref2, drop, flag,
                     out_norm);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int residual_norms(int32_t n, const double* SV, const double* V, int64_t ld, const double* m, const double* theta,
                   int nc, double* num, double* den, GemvTWork& wk, hipStream_t st) {
  if (nc <= 0) return KF_OK;
  const int CH = 8192;
  const int nchunks = ceil_div64(n, CH);
  const size_t need = (size_t)nchunks * nc * 2;
  if (wk.cap < need) {
    if (wk.partial) (void)hipFree(wk.partial);
    wk.partial = nullptr;
    wk.cap = 0;
    if (hipMalloc(&wk.partial, need * sizeof(double)) != hipSuccess) {
      set_error("residual_norms: allocation failed");
      return KF_ENOMEM;
    }
    wk.cap = need;
  }
  hipLaunchKernelGGL(k_resid_partial, dim3(nchunks, nc), dim3(256), 0, st, n, SV, V, ld, m, theta, nc, CH,
                     wk.partial);
  KF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_resid_reduce, dim3(ceil_div64(nc, 4)), dim3(256), 0, st, nchunks, nc, wk.partial, num, den);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int copy_cols(int32_t n, const double* src, int64_t lds, double* dst, int64_t ldd, int nc, hipStream_t st) {
  if (nc <= 0) return KF_OK;
  hipLaunchKernelGGL(k_copy_cols, dim3(ceil_div64(n, 256), nc), dim3(256), 0, st, n, src, lds, dst, ldd);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int pencil_correct(int k, const double* H, const double* G, int64_t ldh, double* E, double* EH, double* Hc,
                   hipStream_t st) {
  const int grid = ceil_div64((int64_t)k * k, 256);
  hipLaunchKernelGGL(k_sub_identity, dim3(grid), dim3(256), 0, st, k, G, ldh, E);
  KF_HIP(hipGetLastError());
  KF_TRY(gemm_nn(k, k, E, k, H, ldh, EH, k, k, st));
  hipLaunchKernelGGL(k_h_correct, dim3(grid), dim3(256), 0, st, k, H, ldh, EH, Hc);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int vectors_correct(int k, int nc, const double* E, double* Y, double* tmp, hipStream_t st) {
  if (nc <= 0) return KF_OK;
  KF_TRY(gemm_nn(k, k, E, k, Y, k, tmp, k, nc, st));
  hipLaunchKernelGGL(k_axpy, dim3(ceil_div64((int64_t)k * nc, 256)), dim3(256), 0, st, (int64_t)k * nc, -0.5, tmp, Y);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int rr_scatter(int k, int c0, int nc, const double* T, int64_t ldt, double* H, double* G, int64_t ldh,
               hipStream_t st) {
  if (nc <= 0) return KF_OK;
  hipLaunchKernelGGL(k_rr_scatter, dim3(ceil_div64((int64_t)k * nc, 256)), dim3(256), 0, st, k, c0, nc, T, ldt, H, G,
                     ldh);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int symmetrize(int k, double* A, int64_t lda, hipStream_t st) {
  if (k <= 1) return KF_OK;
  hipLaunchKernelGGL(k_symmetrize, dim3(ceil_div64((int64_t)k * k, 256)), dim3(256), 0, st, k, A, lda);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int orth_error(int k, const double* G, int64_t ldg, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_orth_error, dim3(1), dim3(1024), 0, st, k, G, ldg, out);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

}  // namespace kf