// The hot path of the filtered time-domain Krylov eigensolver (gfx950):
// k_leapfrog, one step of the explicit two-step scheme of Section 2.3 (eq.
// 2stepmethod) fused with the rectangle-rule accumulation of eq.
// disc_filtercoeff, over a sliced-ELLPACK copy of A = tau^2 M^{-1} S, for one
// problem or for a stack of independent problems; and the SELL build.  The
// step is bound by HBM bandwidth: per step it streams the matrix once (value +
// column index per stored entry) and five vector streams (cur gather, prev,
// next, accumulator read and write).  A wavefront owns 64 rows of a slice
// (LPR wavefronts for blocks with LPR lanes per row), so every matrix load of
// a wavefront is one contiguous run.

#include <hip/hip_runtime.h>

#include <type_traits>

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

template <typename T, int B>
struct alignas((B * sizeof(T)) >= 16 ? 16 : (B * sizeof(T))) Row {
  T v[B];
};

// ---------------------------------------------------------------- SELL build
__global__ __launch_bounds__(256) void k_sell_stats(int32_t n, int32_t nslices, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col, int32_t* __restrict__ width,
                                                    int32_t* __restrict__ maxoff) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = gid;
  int len = 0, off = 0;
  if (row < n) {
    const int a = rowptr[row], b = rowptr[row + 1];
    len = b - a;
    for (int q = a; q < b; ++q) {
      int d = col[q] - (int)row;
      d = d < 0 ? -d : d;
      off = d > off ? d : off;
    }
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    len = max(len, __shfl_xor(len, s));
    off = max(off, __shfl_xor(off, s));
  }
  const int64_t slice = gid >> 6;
  if ((threadIdx.x & 63) == 0 && slice < nslices) {
    width[slice] = len;
    maxoff[slice] = off;
  }
}

template <typename VT, typename IT>
__global__ __launch_bounds__(256) void k_sell_fill(int32_t n, int32_t nslices, const int64_t* __restrict__ sptr,
                                                   const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, const double* __restrict__ rscale,
                                                   VT* __restrict__ oval, IT* __restrict__ oidx) {
  constexpr bool relative = sizeof(IT) == 2;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slice = gid >> 6;
  const int lane = (int)(gid & 63);
  if (slice >= nslices) return;
  const int64_t row = gid;
  const int64_t base = sptr[slice];
  const int width = (int)((sptr[slice + 1] - base) >> 6);
  int a = 0, len = 0;
  double sc = 1.0;
  if (row < n) {
    a = rowptr[row];
    len = rowptr[row + 1] - a;
    if (rscale) sc = rscale[row];
  }
  for (int q = 0; q < width; ++q) {
    const int64_t pos = base + (int64_t)q * 64 + lane;
    if (q < len) {
      oval[pos] = (VT)(sc * val[a + q]);
      const int c = col[a + q];
      oidx[pos] = relative ? (IT)(c - (int)row) : (IT)c;
    } else {
      // padding: zero value, index of the row itself (a valid gather)
      oval[pos] = (VT)0;
      oidx[pos] = relative ? (IT)0 : (IT)(row < n ? row : 0);
    }
  }
}

// ------------------------------------------------------------ fused leapfrog
// One step for a block of B vectors.  LPR lanes share a row, each owning B/LPR
// consecutive vector columns, so a wavefront covers 64/LPR rows of a slice and
// the gather of a neighbour's block row is LPR adjacent 16-byte pieces (LPR = 1:
// one lane per row with the whole block row in registers).  U: unroll factor
// of the loop over the slice's stored entries.
// BAND (blocks): every column a row gathers lies within moff rows of it, so
// the workgroup first copies the rows [r0 - moff, r0 + 4 RW + moff) of `cur`
// (its own 4 RW rows and their neighbours; one contiguous, coalesced stretch)
// into LDS and gathers from there; the caller checks that the stretch fits.
template <typename T, typename IT, int B, int MODE, bool NT, int LPR, int U, bool BAND>
__global__ __launch_bounds__(256) void k_leapfrog(int32_t n, int32_t nslices, const int64_t* __restrict__ sptr,
                                                  const T* __restrict__ val, const IT* __restrict__ idx,
                                                  const T* __restrict__ cur, const T* prev, T* out,
                                                  T* __restrict__ acc, double* __restrict__ rout, int64_t rs,
                                                  int64_t cs, int bout, T wp, T wc, T wn, int remap, int moff) {
  constexpr bool relative = sizeof(IT) == 2;
  constexpr int BL = B / LPR;   // vector columns per lane
  constexpr int RW = 64 / LPR;  // rows per wavefront
  const int wg = remap ? xcd_map(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int gw = wg * 4 + (threadIdx.x >> 6);  // global wavefront
  const int lane = threadIdx.x & 63;
  extern __shared__ __align__(16) unsigned char band_raw[];
  T* __restrict__ band = reinterpret_cast<T*>(band_raw);
  int clo = 0;
  if constexpr (BAND) {
    // every thread takes part in the copy and the barrier before any returns
    const int rlo = wg * 4 * RW;
    clo = max(0, rlo - moff);
    const int chi = min(n, rlo + 4 * RW + moff);
    constexpr int VB = (B * sizeof(T)) % 16 == 0 ? 16 : ((B * sizeof(T)) % 8 == 0 ? 8 : 4);
    using V = typename std::conditional<VB == 16, int4, typename std::conditional<VB == 8, int2, int>::type>::type;
    const int64_t nv = (int64_t)(chi - clo) * B * sizeof(T) / VB;
    const V* __restrict__ src = reinterpret_cast<const V*>(cur + (int64_t)clo * B);
    V* dst = reinterpret_cast<V*>(band_raw);
    for (int64_t t = threadIdx.x; t < nv; t += blockDim.x) dst[t] = src[t];
    __syncthreads();
  }
  const T* __restrict__ xsrc = BAND ? band : cur;  // gathered rows, indexed from row clo
  const int slice = (gw * RW) >> 6;
  if (slice >= nslices) return;
  const int rin = ((gw * RW) & 63) + lane / LPR;  // row within the slice
  const int part = lane % LPR;
  const int row = slice * 64 + rin;
  if (row >= n) return;
  const int64_t base = sptr[slice];
  const int width = (int)((sptr[slice + 1] - base) >> 6);
  const T* __restrict__ vp = val + base + rin;
  const IT* __restrict__ ip = idx + base + rin;
  const int col0 = part * BL;
  T sum[BL];
#pragma unroll
  for (int j = 0; j < BL; ++j) sum[j] = (T)0;
  const int64_t off = (int64_t)row * B + col0;
  // single vectors: the row's own two levels are loaded before the gathers,
  // so their latency overlaps the product (1 % faster on the 3D grids; the
  // sum's row loaded early as well was slower again); a block row is 16 to
  // 128 bytes, and loading it early costs the product more registers than it
  // saves (7 % slower on the horn's block)
  constexpr bool early = B == 1;
  Row<T, BL> yc, yp;
  if (early) {
    yc = *reinterpret_cast<const Row<T, BL>*>(cur + off);
    if (!(MODE & kFirst)) yp = *reinterpret_cast<const Row<T, BL>*>(prev + off);
  }
#pragma unroll U
  for (int q = 0; q < width; ++q) {
    const T a = NT ? __builtin_nontemporal_load(vp + (int64_t)q * 64) : vp[(int64_t)q * 64];
    const IT ci = NT ? __builtin_nontemporal_load(ip + (int64_t)q * 64) : ip[(int64_t)q * 64];
    const int c = relative ? row + (int)ci : (int)ci;
    const Row<T, BL> x = *reinterpret_cast<const Row<T, BL>*>(xsrc + (int64_t)(c - clo) * B + col0);
#pragma unroll
    for (int j = 0; j < BL; ++j) sum[j] = fma(a, x.v[j], sum[j]);
  }
  if (!early) {
    yc = *reinterpret_cast<const Row<T, BL>*>(xsrc + (int64_t)(row - clo) * B + col0);
    if (!(MODE & kFirst)) yp = *reinterpret_cast<const Row<T, BL>*>(prev + off);
  }
  if (MODE & kFirst) yp = yc;
  Row<T, BL> nx;
#pragma unroll
  for (int j = 0; j < BL; ++j) nx.v[j] = (T)2 * yc.v[j] - yp.v[j] - sum[j];
  if (!(MODE & kLast)) *reinterpret_cast<Row<T, BL>*>(out + off) = nx;
  if (MODE == kMid) return;  // the weighted sum is brought up to date every third step
  Row<T, BL> r;
  if (MODE & kFirst) {
#pragma unroll
    for (int j = 0; j < BL; ++j) r.v[j] = fma(wn, nx.v[j], wc * yc.v[j]);
  } else {
    r = *reinterpret_cast<const Row<T, BL>*>(acc + off);
#pragma unroll
    for (int j = 0; j < BL; ++j) r.v[j] = fma(wn, nx.v[j], fma(wc, yc.v[j], fma(wp, yp.v[j], r.v[j])));
  }
  if (MODE & kLast) {
#pragma unroll
    for (int j = 0; j < BL; ++j)
      if (col0 + j < bout) rout[(int64_t)row * rs + (int64_t)(col0 + j) * cs] = (double)r.v[j];
  } else {
    *reinterpret_cast<Row<T, BL>*>(acc + off) = r;
  }
}

// ------------------------------------------------ fourth-order two-step scheme
// y_{l+1} = 2 y_l - y_{l-1} - A y_l + (1/12) A (A y_l), A = tau^2 M^{-1} S
// (a high-order variant of the leapfrog step; its iteration is a polynomial
// in M^{-1} S).  Two launches per step: k_apply_block forms z = A y_l, then
// k_leapfrog4 gathers A z and does the update and the accumulation with the
// same modes and schedule as k_leapfrog.  One lane per row.
template <typename T, typename IT, int B>
__global__ __launch_bounds__(256) void k_apply_block(int32_t n, int32_t nslices, const int64_t* __restrict__ sptr,
                                                     const T* __restrict__ val, const IT* __restrict__ idx,
                                                     const T* __restrict__ x, T* __restrict__ z, int remap) {
  constexpr bool relative = sizeof(IT) == 2;
  const int wg = remap ? xcd_map(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int slice = wg * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (slice >= nslices) return;
  const int row = slice * 64 + lane;
  if (row >= n) return;
  const int64_t base = sptr[slice];
  const int width = (int)((sptr[slice + 1] - base) >> 6);
  const T* __restrict__ vp = val + base + lane;
  const IT* __restrict__ ip = idx + base + lane;
  T sum[B];
#pragma unroll
  for (int j = 0; j < B; ++j) sum[j] = (T)0;
#pragma unroll 4
  for (int q = 0; q < width; ++q) {
    const T a = vp[(int64_t)q * 64];
    const IT ci = ip[(int64_t)q * 64];
    const int c = relative ? row + (int)ci : (int)ci;
    const Row<T, B> xv = *reinterpret_cast<const Row<T, B>*>(x + (int64_t)c * B);
#pragma unroll
    for (int j = 0; j < B; ++j) sum[j] = fma(a, xv.v[j], sum[j]);
  }
  Row<T, B> o;
#pragma unroll
  for (int j = 0; j < B; ++j) o.v[j] = sum[j];
  *reinterpret_cast<Row<T, B>*>(z + (int64_t)row * B) = o;
}

template <typename T, typename IT, int B, int MODE>
__global__ __launch_bounds__(256) void k_leapfrog4(int32_t n, int32_t nslices, const int64_t* __restrict__ sptr,
                                                   const T* __restrict__ val, const IT* __restrict__ idx,
                                                   const T* __restrict__ cur, const T* prev, T* out,
                                                   T* __restrict__ acc, const T* __restrict__ z,
                                                   double* __restrict__ rout, int64_t rs, int64_t cs, int bout, T wp,
                                                   T wc, T wn, int remap) {
  constexpr bool relative = sizeof(IT) == 2;
  const int wg = remap ? xcd_map(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int slice = wg * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (slice >= nslices) return;
  const int row = slice * 64 + lane;
  if (row >= n) return;
  const int64_t base = sptr[slice];
  const int width = (int)((sptr[slice + 1] - base) >> 6);
  const T* __restrict__ vp = val + base + lane;
  const IT* __restrict__ ip = idx + base + lane;
  T sum[B];
#pragma unroll
  for (int j = 0; j < B; ++j) sum[j] = (T)0;
#pragma unroll 4
  for (int q = 0; q < width; ++q) {
    const T a = vp[(int64_t)q * 64];
    const IT ci = ip[(int64_t)q * 64];
    const int c = relative ? row + (int)ci : (int)ci;
    const Row<T, B> zv = *reinterpret_cast<const Row<T, B>*>(z + (int64_t)c * B);
#pragma unroll
    for (int j = 0; j < B; ++j) sum[j] = fma(a, zv.v[j], sum[j]);
  }
  const int64_t off = (int64_t)row * B;
  const Row<T, B> yc = *reinterpret_cast<const Row<T, B>*>(cur + off);
  const Row<T, B> zc = *reinterpret_cast<const Row<T, B>*>(z + off);
  Row<T, B> yp;
  if (MODE & kFirst)
    yp = yc;
  else
    yp = *reinterpret_cast<const Row<T, B>*>(prev + off);
  constexpr T twelfth = (T)(1.0 / 12.0);
  Row<T, B> nx;
#pragma unroll
  for (int j = 0; j < B; ++j) nx.v[j] = fma(twelfth, sum[j], (T)2 * yc.v[j] - yp.v[j] - zc.v[j]);
  if (!(MODE & kLast)) *reinterpret_cast<Row<T, B>*>(out + off) = nx;
  if (MODE == kMid) return;
  Row<T, B> r;
  if (MODE & kFirst) {
#pragma unroll
    for (int j = 0; j < B; ++j) r.v[j] = fma(wn, nx.v[j], wc * yc.v[j]);
  } else {
    r = *reinterpret_cast<const Row<T, B>*>(acc + off);
#pragma unroll
    for (int j = 0; j < B; ++j) r.v[j] = fma(wn, nx.v[j], fma(wc, yc.v[j], fma(wp, yp.v[j], r.v[j])));
  }
  if (MODE & kLast) {
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (j < bout) rout[(int64_t)row * rs + (int64_t)j * cs] = (double)r.v[j];
  } else {
    *reinterpret_cast<Row<T, B>*>(acc + off) = r;
  }
}

// ------------------------------------------------------- batched leapfrog
// Many independent problems stacked into one block-diagonal operator: every
// problem owns whole 64-row slices (rows padded to a multiple of 64), slice s
// belongs to problem sp[s].  One launch advances every problem whose step
// count L_p - 1 reaches `ell`; first/last modes are decided per problem.  The
// per-problem tables (active flag, column counts, source / destination basis
// columns) live in device memory and are refreshed before each replay, so the
// launch sequence can be captured once in a graph.
template <typename T, typename IT, int B, bool NT>
__global__ __launch_bounds__(256) void k_leapfrog_batch(int32_t nslices, const int64_t* __restrict__ sptr,
                                                        const T* __restrict__ val, const IT* __restrict__ idx,
                                                        const int32_t* __restrict__ sp, const BatchTables* __restrict__ tb,
                                                        const T* __restrict__ wtab, int lmax, int ell,
                                                        const T* __restrict__ cur, const T* prev, T* out,
                                                        T* __restrict__ acc, int remap) {
  constexpr bool relative = sizeof(IT) == 2;
  const int wg = remap ? xcd_map(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int slice = wg * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (slice >= nslices) return;
  const int p = sp[slice];
  const int Lp = tb->L[p];
  if (!tb->active[p] || ell > Lp - 1) return;
  const int row = slice * 64 + lane;
  const int local = row - (int)tb->row0[p];
  if (local >= tb->n[p]) return;
  const bool first = ell == 1, last = ell == Lp - 1;
  const int64_t base = sptr[slice];
  const int width = (int)((sptr[slice + 1] - base) >> 6);
  const T* __restrict__ vp = val + base + lane;
  const IT* __restrict__ ip = idx + base + lane;
  T sum[B];
#pragma unroll
  for (int j = 0; j < B; ++j) sum[j] = (T)0;
  int q = 0;
  if constexpr (B <= 4) {
    // four entries at a time: their values, indices and gathers all in flight
    // before the sums (the same order of summation as the loop below)
    constexpr int U = 8;
    for (; q < width; q += U) {
      // (entries past the row's width: value 0 and the row's own index, whose
      // products add exactly nothing)
      T av[U];
      IT cv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = q + u < width;
        const int64_t o = (int64_t)(ok ? q + u : q) * 64;
        av[u] = ok ? (NT ? __builtin_nontemporal_load(vp + o) : vp[o]) : (T)0;
        cv[u] = ok ? (NT ? __builtin_nontemporal_load(ip + o) : ip[o]) : (IT)(relative ? 0 : row);
      }
      Row<T, B> xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = relative ? row + (int)cv[u] : (int)cv[u];
        xv[u] = *reinterpret_cast<const Row<T, B>*>(cur + (int64_t)c * B);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int j = 0; j < B; ++j) sum[j] = fma(av[u], xv[u].v[j], sum[j]);
      }
    }
  }
  for (; q < width; ++q) {
    const T a = NT ? __builtin_nontemporal_load(vp + (int64_t)q * 64) : vp[(int64_t)q * 64];
    const IT ci = NT ? __builtin_nontemporal_load(ip + (int64_t)q * 64) : ip[(int64_t)q * 64];
    const int c = relative ? row + (int)ci : (int)ci;
    const Row<T, B> x = *reinterpret_cast<const Row<T, B>*>(cur + (int64_t)c * B);
#pragma unroll
    for (int j = 0; j < B; ++j) sum[j] = fma(a, x.v[j], sum[j]);
  }
  const Row<T, B> yc = *reinterpret_cast<const Row<T, B>*>(cur + (int64_t)row * B);
  Row<T, B> yp = first ? yc : *reinterpret_cast<const Row<T, B>*>(prev + (int64_t)row * B);
  Row<T, B> nx, r;
#pragma unroll
  for (int j = 0; j < B; ++j) nx.v[j] = (T)2 * yc.v[j] - yp.v[j] - sum[j];
  if (!last) *reinterpret_cast<Row<T, B>*>(out + (int64_t)row * B) = nx;
  // the same accumulation schedule as the single-problem steps (step_plan):
  // y_0, y_1 at step 1, then three levels at steps 4, 7, ..., the rest at the
  // problem's last step
  const int u = ell >= 2 ? 1 + 3 * ((ell - 2) / 3) : 1;  // latest update before this step
  if (!(first || last || ell - u == 3)) return;
  const T* __restrict__ wq = wtab + (int64_t)p * lmax;
  if (first) {
#pragma unroll
    for (int j = 0; j < B; ++j) r.v[j] = fma(wq[1], nx.v[j], wq[0] * yc.v[j]);
  } else {
    const T wp = ell - 2 > u ? wq[ell - 2] : (T)0, wc = ell - 1 > u ? wq[ell - 1] : (T)0, wn = wq[ell];
    r = *reinterpret_cast<const Row<T, B>*>(acc + (int64_t)row * B);
#pragma unroll
    for (int j = 0; j < B; ++j) r.v[j] = fma(wn, nx.v[j], fma(wc, yc.v[j], fma(wp, yp.v[j], r.v[j])));
  }
  if (last) {
    double* __restrict__ dst = tb->dst[p];
    const int64_t ld = tb->ld[p];
    const int bout = tb->bout[p];
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (j < bout) dst[local + (int64_t)j * ld] = (double)r.v[j];
  } else {
    *reinterpret_cast<Row<T, B>*>(acc + (int64_t)row * B) = r;
  }
}

// Batched start of a filter application: Y1 <- the problem's source columns
// (zero beyond bsrc or for inactive problems); L_p = 1 problems get C = w0 I
// written straight to their destination.
template <typename T>
__global__ __launch_bounds__(256) void k_load_batch(int64_t rows, int b, const int32_t* __restrict__ sp,
                                                    const BatchTables* __restrict__ tb, const T* __restrict__ wtab,
                                                    int lmax, T* __restrict__ Y1) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  const int p = sp[row >> 6];
  const int local = (int)(row - tb->row0[p]);
  const bool on = tb->active[p] && local < tb->n[p];
  const double* __restrict__ src = tb->src[p];
  const int64_t lds = tb->lds[p];
  const int bsrc = tb->bsrc[p];
  for (int j = 0; j < b; ++j) Y1[row * b + j] = (on && j < bsrc) ? (T)src[local + (int64_t)j * lds] : (T)0;
  if (on && tb->L[p] == 1) {
    const double w0 = (double)wtab[(int64_t)p * lmax];
    double* __restrict__ dst = tb->dst[p];
    const int64_t ld = tb->ld[p];
    for (int j = 0; j < tb->bout[p]; ++j) dst[local + (int64_t)j * ld] = j < bsrc ? w0 * src[local + (int64_t)j * lds] : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_load_block(int32_t n, int b, int bsrc, const double* __restrict__ src,
                                                    int64_t rs, int64_t cs, T* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < b; ++j) dst[i * b + j] = j < bsrc ? (T)src[i * rs + (int64_t)j * cs] : (T)0;
}

__global__ __launch_bounds__(256) void k_scale_copy(int32_t n, int b, int bsrc, const double* __restrict__ src,
                                                    int64_t srs, int64_t scs, double w0, double* __restrict__ dst,
                                                    int64_t rs, int64_t cs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < b; ++j) dst[i * rs + (int64_t)j * cs] = j < bsrc ? w0 * src[i * srs + (int64_t)j * scs] : 0.0;
}

// ---- host-side dispatch helpers
template <typename T, typename IT, int B, bool NT, int LPR, int U, bool BAND>
int launch_lf_bn(const SellOp& A, int mode, const void* cur, const void* prev, void* out, void* acc, double* rout,
                 int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap, hipStream_t st) {
  const int grid = ceil_div64((int64_t)A.nslices * LPR, 4);
  const size_t lds = BAND ? band_lds_bytes(A, B, LPR) : 0;
  const T* v = static_cast<const T*>(A.val);
  const IT* ix = static_cast<const IT*>(A.idx);
  const T* c = static_cast<const T*>(cur);
  const T* p = static_cast<const T*>(prev);
  T* o = static_cast<T*>(out);
  T* a = static_cast<T*>(acc);
  switch (mode) {
    case kMid:
      hipLaunchKernelGGL((k_leapfrog<T, IT, B, kMid, NT, LPR, U, BAND>), dim3(grid), dim3(256), lds, st, A.n,
                         A.nslices, A.slice_ptr, v, ix, c, p, o, a, rout, rs, cs, bout, (T)wp, (T)wc, (T)wn, remap,
                         A.max_off);
      break;
    case kFirst:
      hipLaunchKernelGGL((k_leapfrog<T, IT, B, kFirst, NT, LPR, U, BAND>), dim3(grid), dim3(256), lds, st, A.n,
                         A.nslices, A.slice_ptr, v, ix, c, p, o, a, rout, rs, cs, bout, (T)wp, (T)wc, (T)wn, remap,
                         A.max_off);
      break;
    case kMidAcc:
      hipLaunchKernelGGL((k_leapfrog<T, IT, B, kMidAcc, NT, LPR, U, BAND>), dim3(grid), dim3(256), lds, st, A.n,
                         A.nslices, A.slice_ptr, v, ix, c, p, o, a, rout, rs, cs, bout, (T)wp, (T)wc, (T)wn, remap,
                         A.max_off);
      break;
    case kLast:
      hipLaunchKernelGGL((k_leapfrog<T, IT, B, kLast, NT, LPR, U, BAND>), dim3(grid), dim3(256), lds, st, A.n,
                         A.nslices, A.slice_ptr, v, ix, c, p, o, a, rout, rs, cs, bout, (T)wp, (T)wc, (T)wn, remap,
                         A.max_off);
      break;
    default:
      hipLaunchKernelGGL((k_leapfrog<T, IT, B, kFirstLast, NT, LPR, U, BAND>), dim3(grid), dim3(256), lds, st, A.n,
                         A.nslices, A.slice_ptr, v, ix, c, p, o, a, rout, rs, cs, bout, (T)wp, (T)wc, (T)wn, remap,
                         A.max_off);
      break;
  }
  KF_HIP(hipGetLastError());
  return KF_OK;
}

template <typename T, typename IT, int B, int LPR, int U, bool BAND>
int launch_lf_bs(const SellOp& A, int mode, const void* cur, const void* prev, void* out, void* acc, double* rout,
                 int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap, hipStream_t st) {
  if (A.nt_loads)
    return launch_lf_bn<T, IT, B, true, LPR, U, BAND>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn,
                                                      remap, st);
  return launch_lf_bn<T, IT, B, false, LPR, U, BAND>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn,
                                                     remap, st);
}

// Blocks gather from an LDS copy of the workgroup's band of rows when the
// operator chose it for this block width and the band fits.
template <typename T, typename IT, int B, int LPR, int U>
int launch_lf_bu(const SellOp& A, int mode, const void* cur, const void* prev, void* out, void* acc, double* rout,
                 int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap, hipStream_t st) {
  if constexpr (B > 1) {
    if (use_band(A, B, LPR))
      return launch_lf_bs<T, IT, B, LPR, U, true>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap,
                                                  st);
  }
  return launch_lf_bs<T, IT, B, LPR, U, false>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap,
                                               st);
}

// The loop over a slice's entries is unrolled four times for blocks; for
// single vectors the factor (2, 3, 4 or 6) is a tuning choice: the best one
// depends on the slice widths and on how the compiler schedules the loads
// (on the 3D grids, 15 entries per row: 13.9 us per step unrolled six times,
// 14.2 three times, 14.5 five, 14.7 four or two, 15.0 seven, 15.3 eight).
template <typename T, typename IT, int B, int LPR>
int launch_lf_bl(const SellOp& A, int mode, const void* cur, const void* prev, void* out, void* acc, double* rout,
                 int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap, hipStream_t st) {
  if constexpr (B == 1) {
    if (A.unroll == 2)
      return launch_lf_bu<T, IT, B, LPR, 2>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
    if (A.unroll == 3)
      return launch_lf_bu<T, IT, B, LPR, 3>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
    if (A.unroll == 6)
      return launch_lf_bu<T, IT, B, LPR, 6>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
  }
  return launch_lf_bu<T, IT, B, LPR, 4>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
}

template <typename T, typename IT, int B>
int launch_lf_b(const SellOp& A, int mode, const void* cur, const void* prev, void* out, void* acc, double* rout,
                int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap, hipStream_t st) {
  const int lpr = lanes_per_row(A, B);
  if (B >= 4 && lpr == 4)
    return launch_lf_bl<T, IT, B, (B >= 4 ? 4 : 1)>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
  if (B >= 2 && lpr == 2)
    return launch_lf_bl<T, IT, B, (B >= 2 ? 2 : 1)>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
  return launch_lf_bl<T, IT, B, 1>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
}

template <typename T, typename IT>
int launch_lf_t(const SellOp& A, int b, int mode, const void* cur, const void* prev, void* out, void* acc,
                double* rout, int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap, hipStream_t st) {
  switch (b) {
    case 1: return launch_lf_b<T, IT, 1>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 2: return launch_lf_b<T, IT, 2>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 4: return launch_lf_b<T, IT, 4>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 8: return launch_lf_b<T, IT, 8>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 16: return launch_lf_b<T, IT, 16>(A, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, remap, st);
    default: set_error("leapfrog: block width must be 1, 2, 4, 8 or 16"); return KF_EINVAL;
  }
}

template <typename T, typename IT, int B>
int launch_lf4_b(const SellOp& A, int mode, const void* cur, const void* prev, void* out, void* acc, void* z,
                 double* rout, int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap,
                 hipStream_t st) {
  const int grid = ceil_div64(A.nslices, 4);
  const T* v = static_cast<const T*>(A.val);
  const IT* ix = static_cast<const IT*>(A.idx);
  const T* c = static_cast<const T*>(cur);
  const T* p = static_cast<const T*>(prev);
  T* o = static_cast<T*>(out);
  T* a = static_cast<T*>(acc);
  T* zz = static_cast<T*>(z);
  hipLaunchKernelGGL((k_apply_block<T, IT, B>), dim3(grid), dim3(256), 0, st, A.n, A.nslices, A.slice_ptr, v, ix, c, zz,
                     remap);
#define KF_LF4(M)                                                                                                  \
  hipLaunchKernelGGL((k_leapfrog4<T, IT, B, M>), dim3(grid), dim3(256), 0, st, A.n, A.nslices, A.slice_ptr, v, ix, c, \
                     p, o, a, zz, rout, rs, cs, bout, (T)wp, (T)wc, (T)wn, remap)
  switch (mode) {
    case kMid: KF_LF4(kMid); break;
    case kFirst: KF_LF4(kFirst); break;
    case kMidAcc: KF_LF4(kMidAcc); break;
    case kLast: KF_LF4(kLast); break;
    default: KF_LF4(kFirstLast); break;
  }
#undef KF_LF4
  KF_HIP(hipGetLastError());
  return KF_OK;
}

template <typename T, typename IT>
int launch_lf4_t(const SellOp& A, int b, int mode, const void* cur, const void* prev, void* out, void* acc, void* z,
                 double* rout, int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int remap,
                 hipStream_t st) {
  switch (b) {
    case 1: return launch_lf4_b<T, IT, 1>(A, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 2: return launch_lf4_b<T, IT, 2>(A, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 4: return launch_lf4_b<T, IT, 4>(A, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 8: return launch_lf4_b<T, IT, 8>(A, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, remap, st);
    case 16: return launch_lf4_b<T, IT, 16>(A, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, remap, st);
    default: set_error("fourth-order step: block width must be 1, 2, 4, 8 or 16"); return KF_EINVAL;
  }
}

// ------------------------------------------- several steps per launch (bands)
// Communication-avoiding form of the time loop for operators whose stored
// entries lie within max_off rows of the diagonal (banded orderings): a
// workgroup owns a range of row slices and advances y_l -> y_{l+s} for it in
// one launch, keeping y_{l-1}, y_l of its rows and of the s*max_off rows on
// either side in LDS.  Step j updates the rows within (s-1-j)*max_off of the
// owned range (those the later steps still read), each from the previous
// level's values in LDS; the weighted sum of the owned rows stays in LDS for
// the s steps.  HBM traffic per step and row falls from five vector streams
// (plus the operator) to 6/s of a vector (plus the operator, whose band is
// read from the caches at every step); the cost is the halo rows computed
// more than once (s*max_off/own of the work) and the workgroup's LDS.  With
// the whole problem in one workgroup the filter is one launch.
//   first: y_{-1} = y_0 = x (x in ysrc), acc = w_0 x;  else i0, i1 hold
//          y_{l0-1}, y_{l0} and accg the weighted sum so far
//   last:  the weighted sum goes to rout (float64, row stride rs) instead
//          of accg; otherwise y_{l0+s-1}, y_{l0+s} go to o0, o1
// The levels are read from one pair of buffers and written to another (a
// workgroup's halo rows are another workgroup's owned rows, written in the
// same launch); the sum is read and written by its owner only.
// Every step adds w_{l+1} y_{l+1} (one term per step, in step order).
template <typename T, typename IT>
__global__ __launch_bounds__(1024) void k_leapfrog_mp(int32_t n, int32_t nslices, const int64_t* __restrict__ sptr,
                                                      const T* __restrict__ val, const IT* __restrict__ idx,
                                                      const T* __restrict__ ysrc, const T* __restrict__ i0,
                                                      const T* __restrict__ i1, T* __restrict__ o0g,
                                                      T* __restrict__ o1g, T* accg, double* __restrict__ rout,
                                                      int64_t rs, const double* __restrict__ w, int l0, int s, int own,
                                                      int hb, int first, int last) {
  constexpr bool relative = sizeof(IT) == 2;
  extern __shared__ __align__(16) unsigned char mp_raw[];
  const int o0 = blockIdx.x * own;                  // owned slices [o0, o1)
  const int o1 = min(nslices, o0 + own);
  const int w0 = max(0, o0 - s * hb);               // window slices [w0, w1)
  const int w1 = min(nslices, o1 + s * hb);
  const int wrows = (w1 - w0) * 64, orows = (o1 - o0) * 64;
  const int r0 = w0 * 64;                           // first row of the window
  T* Yp = reinterpret_cast<T*>(mp_raw);
  T* Yc = Yp + wrows;
  T* Ra = Yc + wrows;                               // weighted sum of the owned rows
  const int own0 = o0 * 64 - r0;                    // owned rows in window coordinates
  for (int i = threadIdx.x; i < wrows; i += blockDim.x) {
    const int g = r0 + i;
    T a = (T)0, b = (T)0;
    if (g < n) {
      if (first) {
        a = ysrc[g];
        b = a;
      } else {
        a = i0[g];
        b = i1[g];
      }
    }
    Yp[i] = a;
    Yc[i] = b;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < orows; i += blockDim.x) {
    const int g = o0 * 64 + i;
    Ra[i] = g < n ? (first ? (T)w[0] * Yc[own0 + i] : accg[g]) : (T)0;
  }
  for (int j = 0; j < s; ++j) {
    const int l = l0 + j;  // this step forms y_{l+1}
    const T wn = (T)w[l + 1];
    const int a0 = max(w0, o0 - (s - 1 - j) * hb), a1 = min(w1, o1 + (s - 1 - j) * hb);
    const int nrow = (a1 - a0) * 64;
    for (int t = threadIdx.x; t < nrow; t += blockDim.x) {
      const int g = a0 * 64 + t;
      if (g >= n) continue;
      const int slice = g >> 6, lane = g & 63;
      const int64_t base = sptr[slice];
      const int width = (int)((sptr[slice + 1] - base) >> 6);
      const T* __restrict__ vp = val + base + lane;
      const IT* __restrict__ ip = idx + base + lane;
      T sum = (T)0;
      for (int q = 0; q < width; ++q) {
        const T a = vp[(int64_t)q * 64];
        const IT ci = ip[(int64_t)q * 64];
        const int c = relative ? g + (int)ci : (int)ci;
        sum = fma(a, Yc[c - r0], sum);
      }
      const int i = g - r0;
      const T nx = (T)2 * Yc[i] - Yp[i] - sum;
      Yp[i] = nx;  // y_{l+1} replaces y_{l-1}; the other rows read only Yc
      const int oi = i - own0;
      if (oi >= 0 && oi < orows) Ra[oi] = fma(wn, nx, Ra[oi]);
    }
    __syncthreads();
    T* tmp = Yp;
    Yp = Yc;
    Yc = tmp;
  }
  for (int i = threadIdx.x; i < orows; i += blockDim.x) {
    const int g = o0 * 64 + i;
    if (g >= n) continue;
    if (!last) {
      o0g[g] = Yp[own0 + i];
      o1g[g] = Yc[own0 + i];
      accg[g] = Ra[i];
    } else {
      rout[(int64_t)g * rs] = (double)Ra[i];
    }
  }
}

// The same for a whole small problem in one workgroup whose rows and stored
// entries fit in registers (at most MAXR rows per thread, slices at most
// MAXW entries wide): thread t keeps rows t, t + 1024, ... with their entries
// and weighted sums in registers for all s steps, the two levels in LDS, so a
// step reads nothing but LDS.
template <typename T, typename IT, int MAXR, int MAXW>
__global__ __launch_bounds__(1024) void k_leapfrog_mp_reg(int32_t n, int32_t nslices, const int64_t* __restrict__ sptr,
                                                          const T* __restrict__ val, const IT* __restrict__ idx,
                                                          const T* __restrict__ ysrc, const T* __restrict__ i0,
                                                          const T* __restrict__ i1, T* __restrict__ o0g,
                                                          T* __restrict__ o1g, T* accg, double* __restrict__ rout,
                                                          int64_t rs, const double* __restrict__ w, int l0, int s,
                                                          int first, int last) {
  constexpr bool relative = sizeof(IT) == 2;
  extern __shared__ __align__(16) unsigned char mpr_raw[];
  const int rows = nslices * 64;
  T* Yp = reinterpret_cast<T*>(mpr_raw);
  T* Yc = Yp + rows;
  T a[MAXR][MAXW];
  int c[MAXR][MAXW];
  T racc[MAXR];
  int wdt[MAXR];
#pragma unroll
  for (int k = 0; k < MAXR; ++k) {
    const int g = threadIdx.x + 1024 * k;
    wdt[k] = 0;
    racc[k] = (T)0;
    if (g < n) {
      const int slice = g >> 6, lane = g & 63;
      const int64_t base = sptr[slice];
      wdt[k] = min(MAXW, (int)((sptr[slice + 1] - base) >> 6));
#pragma unroll
      for (int q = 0; q < MAXW; ++q) {
        if (q < wdt[k]) {
          a[k][q] = val[base + (int64_t)q * 64 + lane];
          const IT ci = idx[base + (int64_t)q * 64 + lane];
          c[k][q] = relative ? g + (int)ci : (int)ci;
        } else {
          a[k][q] = (T)0;
          c[k][q] = g;
        }
      }
    }
  }
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    T x0 = (T)0, x1 = (T)0;
    if (i < n) {
      if (first) {
        x0 = ysrc[i];
        x1 = x0;
      } else {
        x0 = i0[i];
        x1 = i1[i];
      }
    }
    Yp[i] = x0;
    Yc[i] = x1;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < MAXR; ++k) {
    const int g = threadIdx.x + 1024 * k;
    if (g < n) racc[k] = first ? (T)w[0] * Yc[g] : accg[g];
  }
  for (int j = 0; j < s; ++j) {
    const T wn = (T)w[l0 + j + 1];
#pragma unroll
    for (int k = 0; k < MAXR; ++k) {
      const int g = threadIdx.x + 1024 * k;
      if (g < n) {
        T sum = (T)0;
#pragma unroll
        for (int q = 0; q < MAXW; ++q) sum = fma(a[k][q], Yc[c[k][q]], sum);
        const T nx = (T)2 * Yc[g] - Yp[g] - sum;
        Yp[g] = nx;
        racc[k] = fma(wn, nx, racc[k]);
      }
    }
    __syncthreads();
    T* tmp = Yp;
    Yp = Yc;
    Yc = tmp;
  }
#pragma unroll
  for (int k = 0; k < MAXR; ++k) {
    const int g = threadIdx.x + 1024 * k;
    if (g >= n) continue;
    if (!last) {
      o0g[g] = Yp[g];
      o1g[g] = Yc[g];
      accg[g] = racc[k];
    } else {
      rout[(int64_t)g * rs] = (double)racc[k];
    }
  }
}

}  // namespace


void free_sell(SellOp& op) {
  if (op.slice_ptr) (void)hipFree(op.slice_ptr);
  if (op.val) (void)hipFree(op.val);
  if (op.idx) (void)hipFree(op.idx);
  op = SellOp();
}

int build_sell(int32_t n, int64_t nnz, const int32_t* d_rowptr, const int32_t* d_col, const double* d_val,
               const double* d_row_scale, int val_bytes, int want_idx_bytes, hipStream_t st, SellOp& out) {
  free_sell(out);
  if (n <= 0) {
    set_error("build_sell: empty matrix");
    return KF_EINVAL;
  }
  const int32_t ns = ceil_div64(n, kSlice);
  int32_t* d_stats = nullptr;
  KF_HIP(hipMalloc(&d_stats, sizeof(int32_t) * 2 * (size_t)ns));
  const int grid = ceil_div64((int64_t)ns * kSlice, 256);
  hipLaunchKernelGGL(k_sell_stats, dim3(grid), dim3(256), 0, st, n, ns, d_rowptr, d_col, d_stats, d_stats + ns);
  std::vector<int32_t> h(2 * (size_t)ns);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_stats, sizeof(int32_t) * 2 * ns, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_stats);
  if (e != hipSuccess) {
    set_error(std::string("build_sell: ") + hipGetErrorString(e));
    return KF_EHIP;
  }
  std::vector<int64_t> ptr((size_t)ns + 1);
  ptr[0] = 0;
  int32_t maxw = 0, maxoff = 0;
  for (int32_t s = 0; s < ns; ++s) {
    ptr[s + 1] = ptr[s] + (int64_t)h[s] * kSlice;
    maxw = std::max(maxw, h[s]);
    maxoff = std::max(maxoff, h[ns + s]);
  }
  int ib = want_idx_bytes;
  if (ib == 0) ib = maxoff < 32768 ? 2 : 4;
  if (ib == 2 && maxoff >= 32768) {
    set_error("build_sell: 16-bit relative column offsets requested but |col-row| reaches " +
              std::to_string(maxoff));
    return KF_EINVAL;
  }
  if (ib != 2 && ib != 4) {
    set_error("build_sell: index width must be 0, 2 or 4");
    return KF_EINVAL;
  }
  if (val_bytes != 4 && val_bytes != 8) {
    set_error("build_sell: value width must be 4 or 8");
    return KF_EINVAL;
  }
  const int64_t tot = std::max<int64_t>(ptr[ns], kSlice);
  out.n = n;
  out.nslices = ns;
  out.nstored = ptr[ns];
  out.idx_bytes = ib;
  out.val_bytes = val_bytes;
  out.max_width = maxw;
  out.max_off = maxoff;
  if (hipMalloc(&out.slice_ptr, sizeof(int64_t) * (ns + 1)) != hipSuccess ||
      hipMalloc(&out.val, (size_t)tot * val_bytes) != hipSuccess ||
      hipMalloc(&out.idx, (size_t)tot * ib) != hipSuccess) {
    free_sell(out);
    set_error("build_sell: device allocation failed");
    return KF_ENOMEM;
  }
  KF_HIP(hipMemcpyAsync(out.slice_ptr, ptr.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, st));
  if (val_bytes == 8 && ib == 2)
    hipLaunchKernelGGL((k_sell_fill<double, int16_t>), dim3(grid), dim3(256), 0, st, n, ns, out.slice_ptr, d_rowptr,
                       d_col, d_val, d_row_scale, (double*)out.val, (int16_t*)out.idx);
  else if (val_bytes == 8)
    hipLaunchKernelGGL((k_sell_fill<double, int32_t>), dim3(grid), dim3(256), 0, st, n, ns, out.slice_ptr, d_rowptr,
                       d_col, d_val, d_row_scale, (double*)out.val, (int32_t*)out.idx);
  else if (ib == 2)
    hipLaunchKernelGGL((k_sell_fill<float, int16_t>), dim3(grid), dim3(256), 0, st, n, ns, out.slice_ptr, d_rowptr,
                       d_col, d_val, d_row_scale, (float*)out.val, (int16_t*)out.idx);
  else
    hipLaunchKernelGGL((k_sell_fill<float, int32_t>), dim3(grid), dim3(256), 0, st, n, ns, out.slice_ptr, d_rowptr,
                       d_col, d_val, d_row_scale, (float*)out.val, (int32_t*)out.idx);
  KF_HIP(hipGetLastError());
  KF_HIP(hipStreamSynchronize(st));
  (void)nnz;
  return KF_OK;
}

int lanes_per_row(const SellOp& A, int b) {
  int lb = 0;
  while ((1 << lb) < b && lb < 4) ++lb;
  int l = A.lpr[lb];
  if (l <= 0) {
    // default: 16 bytes of the block row per lane
    l = std::max(1, b * A.val_bytes / 16);
  }
  l = std::min(l, std::min(b, 4));
  return l >= 4 ? 4 : (l >= 2 ? 2 : 1);
}

int launch_leapfrog(const SellOp& A, int b, int mode, const void* cur, const void* prev, void* out, void* acc,
                    double* rout, int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int xcd_remap,
                    hipStream_t st) {
  if (A.val_bytes == 8) {
    if (A.idx_bytes == 2)
      return launch_lf_t<double, int16_t>(A, b, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, xcd_remap,
                                          st);
    return launch_lf_t<double, int32_t>(A, b, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, xcd_remap,
                                        st);
  }
  if (A.idx_bytes == 2)
    return launch_lf_t<float, int16_t>(A, b, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, xcd_remap, st);
  return launch_lf_t<float, int32_t>(A, b, mode, cur, prev, out, acc, rout, rs, cs, bout, wp, wc, wn, xcd_remap, st);
}

MultiStepPlan plan_multistep(const SellOp& A, int s, size_t lds_bytes) {
  MultiStepPlan pl;
  const int vb = A.val_bytes;
  const int hb = (A.max_off + 63) / 64;  // the band in slices
  pl.hb = hb;
  // the whole problem in one workgroup: with its stored entries in registers
  // when every thread holds at most 4 rows of at most 8 entries, else reading
  // them from the caches at every step (no halo either way)
  if ((size_t)A.nslices * 64 <= 4 * 1024 && A.max_width <= 8 && (size_t)A.nslices * 64 * 2 * vb <= lds_bytes) {
    pl.own = A.nslices;
    pl.s = s;
    pl.ok = true;
    pl.reg = true;
    return pl;
  }
  if ((size_t)A.nslices * 64 * 3 * vb <= lds_bytes) {
    pl.own = A.nslices;
    pl.s = s;
    pl.ok = true;
    return pl;
  }
  // largest owned range whose window (own + 2 s hb slices, two levels) and
  // weighted sum fit
  const size_t per_slice = (size_t)64 * vb;
  const size_t halo = (size_t)2 * s * hb;
  const size_t cap = lds_bytes / per_slice;  // slices of one level
  if (2 * halo + 3 > cap) return pl;         // not even one owned slice
  pl.own = (int)std::min<size_t>((cap - 2 * halo) / 3, (size_t)A.nslices);
  pl.s = s;
  pl.ok = pl.own >= 1;
  return pl;
}

int launch_leapfrog_mp(const SellOp& A, const MultiStepPlan& pl, int l0, int s, bool first, bool last, const void* ysrc,
                       const void* i0, const void* i1, void* o0, void* o1, void* acc, double* rout, int64_t rs,
                       const double* w, hipStream_t st) {
  if (!pl.ok || s < 1) {
    set_error("multi-step leapfrog: the band does not fit in LDS");
    return KF_EINVAL;
  }
  if (pl.reg) {
    // the whole problem in one workgroup, operator and sums in registers
    const size_t lds = (size_t)2 * A.nslices * 64 * A.val_bytes;
#define KF_MPR(T, IT)                                                                                              \
  do {                                                                                                             \
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_leapfrog_mp_reg<T, IT, 4, 8>),                       \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                                \
    hipLaunchKernelGGL((k_leapfrog_mp_reg<T, IT, 4, 8>), dim3(1), dim3(1024), lds, st, A.n, A.nslices, A.slice_ptr, \
                       static_cast<const T*>(A.val), static_cast<const IT*>(A.idx), static_cast<const T*>(ysrc),      \
                       static_cast<const T*>(i0), static_cast<const T*>(i1), static_cast<T*>(o0),                      \
                       static_cast<T*>(o1), static_cast<T*>(acc), rout, rs, w, l0, s, first ? 1 : 0, last ? 1 : 0);  \
  } while (0)
    if (A.val_bytes == 8) {
      if (A.idx_bytes == 2)
        KF_MPR(double, int16_t);
      else
        KF_MPR(double, int32_t);
    } else {
      if (A.idx_bytes == 2)
        KF_MPR(float, int16_t);
      else
        KF_MPR(float, int32_t);
    }
#undef KF_MPR
    KF_HIP(hipGetLastError());
    return KF_OK;
  }
  const int grid = ceil_div64(A.nslices, pl.own);
  const int wsl = std::min(A.nslices, pl.own + 2 * s * pl.hb);
  const size_t lds = ((size_t)2 * wsl + pl.own) * 64 * A.val_bytes;
#define KF_MP(T, IT)                                                                                               \
  do {                                                                                                             \
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_leapfrog_mp<T, IT>),                                   \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                                  \
  hipLaunchKernelGGL((k_leapfrog_mp<T, IT>), dim3(grid), dim3(1024), lds, st, A.n, A.nslices, A.slice_ptr,         \
                     static_cast<const T*>(A.val), static_cast<const IT*>(A.idx), static_cast<const T*>(ysrc),        \
                     static_cast<const T*>(i0), static_cast<const T*>(i1), static_cast<T*>(o0), static_cast<T*>(o1), \
                     static_cast<T*>(acc), rout, rs, w, l0, s, pl.own, pl.hb, first ? 1 : 0, last ? 1 : 0);    \
  } while (0)
  if (A.val_bytes == 8) {
    if (A.idx_bytes == 2)
      KF_MP(double, int16_t);
    else
      KF_MP(double, int32_t);
  } else {
    if (A.idx_bytes == 2)
      KF_MP(float, int16_t);
    else
      KF_MP(float, int32_t);
  }
#undef KF_MP
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int launch_leapfrog4(const SellOp& A, int b, int mode, const void* cur, const void* prev, void* out, void* acc, void* z,
                     double* rout, int64_t rs, int64_t cs, int bout, double wp, double wc, double wn, int xcd_remap,
                     hipStream_t st) {
  if (A.val_bytes == 8) {
    if (A.idx_bytes == 2)
      return launch_lf4_t<double, int16_t>(A, b, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn,
                                           xcd_remap, st);
    return launch_lf4_t<double, int32_t>(A, b, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, xcd_remap,
                                         st);
  }
  if (A.idx_bytes == 2)
    return launch_lf4_t<float, int16_t>(A, b, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, xcd_remap,
                                        st);
  return launch_lf4_t<float, int32_t>(A, b, mode, cur, prev, out, acc, z, rout, rs, cs, bout, wp, wc, wn, xcd_remap,
                                      st);
}

StepPlan step_plan(int l, int L) {
  const bool last = l == L - 1;
  if (l == 1) return StepPlan{last ? kFirstLast : kFirst, -1, 0, 1};
  const int u = 1 + 3 * ((l - 2) / 3);  // the latest step that brought the sum up to date
  if (!last && l - u < 3) return StepPlan{kMid, -1, -1, -1};
  return StepPlan{last ? kLast : kMidAcc, l - 2 > u ? l - 2 : -1, l - 1 > u ? l - 1 : -1, l};
}

namespace {
template <typename T, typename IT, bool NT>
int launch_lfb_t(const SellOp& A, int b, const int32_t* sp, const BatchTables* tb, const void* wtab, int lmax, int ell,
                 const void* cur, const void* prev, void* out, void* acc, int nslices, int remap, hipStream_t st) {
  const int grid = ceil_div64(nslices, 4);
  const T* v = static_cast<const T*>(A.val);
  const IT* ix = static_cast<const IT*>(A.idx);
  const T* w = static_cast<const T*>(wtab);
  const T* c = static_cast<const T*>(cur);
  const T* pr = static_cast<const T*>(prev);
  T* o = static_cast<T*>(out);
  T* a = static_cast<T*>(acc);
  switch (b) {
    case 1:
      hipLaunchKernelGGL((k_leapfrog_batch<T, IT, 1, NT>), dim3(grid), dim3(256), 0, st, nslices, A.slice_ptr, v, ix, sp,
                         tb, w, lmax, ell, c, pr, o, a, remap);
      break;
    case 2:
      hipLaunchKernelGGL((k_leapfrog_batch<T, IT, 2, NT>), dim3(grid), dim3(256), 0, st, nslices, A.slice_ptr, v, ix, sp,
                         tb, w, lmax, ell, c, pr, o, a, remap);
      break;
    case 4:
      hipLaunchKernelGGL((k_leapfrog_batch<T, IT, 4, NT>), dim3(grid), dim3(256), 0, st, nslices, A.slice_ptr, v, ix, sp,
                         tb, w, lmax, ell, c, pr, o, a, remap);
      break;
    case 8:
      hipLaunchKernelGGL((k_leapfrog_batch<T, IT, 8, NT>), dim3(grid), dim3(256), 0, st, nslices, A.slice_ptr, v, ix, sp,
                         tb, w, lmax, ell, c, pr, o, a, remap);
      break;
    case 16:
      hipLaunchKernelGGL((k_leapfrog_batch<T, IT, 16, NT>), dim3(grid), dim3(256), 0, st, nslices, A.slice_ptr, v, ix,
                         sp, tb, w, lmax, ell, c, pr, o, a, remap);
      break;
    default:
      set_error("batched leapfrog: block width must be 1, 2, 4, 8 or 16");
      return KF_EINVAL;
  }
  KF_HIP(hipGetLastError());
  return KF_OK;
}
}  // namespace

int launch_leapfrog_batch(const SellOp& A, int b, const int32_t* sp, const BatchTables* tb, const void* wtab, int lmax,
                          int ell, const void* cur, const void* prev, void* out, void* acc, int nslices, int remap,
                          hipStream_t st) {
  if (nslices <= 0 || nslices > A.nslices) nslices = A.nslices;
#define KF_LFB(T, IT)                                                                                               \
  return A.nt_loads ? launch_lfb_t<T, IT, true>(A, b, sp, tb, wtab, lmax, ell, cur, prev, out, acc, nslices, remap, \
                                                st)                                                                 \
                    : launch_lfb_t<T, IT, false>(A, b, sp, tb, wtab, lmax, ell, cur, prev, out, acc, nslices, remap, st)
  if (A.val_bytes == 8) {
    if (A.idx_bytes == 2) KF_LFB(double, int16_t);
    KF_LFB(double, int32_t);
  }
  if (A.idx_bytes == 2) KF_LFB(float, int16_t);
  KF_LFB(float, int32_t);
#undef KF_LFB
}

int launch_load_batch(int val_bytes, int64_t rows, int b, const int32_t* sp, const BatchTables* tb, const void* wtab,
                      int lmax, void* Y1, hipStream_t st) {
  const int grid = ceil_div64(rows, 256);
  if (val_bytes == 8)
    hipLaunchKernelGGL(k_load_batch<double>, dim3(grid), dim3(256), 0, st, rows, b, sp, tb, (const double*)wtab, lmax,
                       (double*)Y1);
  else
    hipLaunchKernelGGL(k_load_batch<float>, dim3(grid), dim3(256), 0, st, rows, b, sp, tb, (const float*)wtab, lmax,
                       (float*)Y1);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int launch_load_block(int val_bytes, int32_t n, int b, int bsrc, const double* src, int64_t rs, int64_t cs,
                      void* dst, hipStream_t st) {
  const int grid = ceil_div64(n, 256);
  if (val_bytes == 8)
    hipLaunchKernelGGL(k_load_block<double>, dim3(grid), dim3(256), 0, st, n, b, bsrc, src, rs, cs, (double*)dst);
  else
    hipLaunchKernelGGL(k_load_block<float>, dim3(grid), dim3(256), 0, st, n, b, bsrc, src, rs, cs, (float*)dst);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

int launch_scale_copy(int32_t n, int b, int bsrc, const double* src, int64_t srs, int64_t scs, double w0,
                      double* rout, int64_t rs, int64_t cs, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3(ceil_div64(n, 256)), dim3(256), 0, st, n, b, bsrc, src, srs, scs, w0, rout,
                     rs, cs);
  KF_HIP(hipGetLastError());
  return KF_OK;
}


}  // namespace kf
