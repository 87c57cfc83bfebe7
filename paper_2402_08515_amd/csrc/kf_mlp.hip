// Learned filter weights: a small network maps the normalised problem data to
// the L filter coefficients.  Section 2.2 leaves the weight function free and
// states the design goal (|beta| large on the sought omega, small elsewhere);
// Lemma 2.3 gives the filter of any weights, beta~(omega) = sum_l w_l q_l.
//
// Normalised variables: a = tau*omega_min, c = tau*omega_max, x = tau*omega/2,
// x_max = tau*sqrt(lambda_max)/2.  In them q_l(x) = cos((l+1/2)phi)/cos(phi/2)
// with phi = 2 arcsin x, and the Fourier weights of eq. weightf are
// w_0 = 2(c-a)/pi, w_l = 4/(pi l) sin(l(c-a)/2) cos(l(c+a)/2), l < L.
//
// Network (features [a/pi, c/pi, x_max, L/512] padded to 64): three GELU
// layers of width 128, a linear layer of 512; w = w_Fourier + 0.01 * out,
// masked to l < L.  Loss on the grid x_g = 0.95 g/511: mean over the band
// [a/2, c/2] of (beta~ - 1)^2 plus the mean over x <= x_max outside the band
// widened by pi/(2L) of beta~^2.
//
// Matrix products of the network run on the matrix cores in bfloat16 with
// float32 accumulation (v_mfma_f32_16x16x16_bf16); the filter-response product
// beta~ = w Q and its adjoint run in float32 on the matrix cores
// (v_mfma_f32_16x16x4_f32), since the leakage being minimised is far below
// bfloat16 resolution.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kf_internal.h"

namespace kf {
namespace {

constexpr int kH = 128;    // hidden width
constexpr int kLM = 512;   // maximum number of weights
constexpr int kG = 512;    // frequency grid
constexpr int kNF = 64;    // padded feature count
constexpr float kOut = 0.01f;
constexpr float kXmaxGrid = 0.95f;
constexpr double kPi = 3.14159265358979323846;

// parameter layout (float32): W1[64x128] b1 W2[128x128] b2 W3[128x128] b3 W4[128x512] b4
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNF * kH;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH * kH;
constexpr int kOffW4 = kOffB3 + kH;
constexpr int kOffB4 = kOffW4 + kH * kLM;
constexpr int kNParams = kOffB4 + kLM;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// C[M x N] (row-major, ldc) (+)= op(A)[M x K] * op(B)[K x N]
//   TA = 0: A[m*lda + k]; TA = 1: A[k*lda + m]
//   TB = 0: B[k*ldb + n]; TB = 1: B[n*ldb + k]
// 64 x 64 tile per workgroup of 4 wavefronts, 32 x 32 per wavefront.
// Requires M % 64 == 0, N % 64 == 0, K % 16 == 0.
template <int TA, int TB, bool BF16>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              int accumulate) {
  __shared__ float As[64][17];
  __shared__ float Bs[16][65];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int t = tid; t < 64 * 16; t += 256) {
      const int mm = t >> 4, kk = t & 15;
      As[mm][kk] = TA ? A[(int64_t)(k0 + kk) * lda + m0 + mm] : A[(int64_t)(m0 + mm) * lda + k0 + kk];
    }
    for (int t = tid; t < 16 * 64; t += 256) {
      const int kk = t >> 6, nn = t & 63;
      Bs[kk][nn] = TB ? B[(int64_t)(n0 + nn) * ldb + k0 + kk] : B[(int64_t)(k0 + kk) * ldb + n0 + nn];
    }
    __syncthreads();
    const int r16 = lane & 15, q4 = lane >> 4;
    for (int i = 0; i < 2; ++i) {
      for (int j = 0; j < 2; ++j) {
        const int r = wm + 16 * i + r16;
        const int cc = wn + 16 * j + r16;
        if (BF16) {
          // lane holds A[r][4*q4 .. 4*q4+3] and B[4*q4 .. 4*q4+3][cc]
          bf16x4 a, b;
          for (int q = 0; q < 4; ++q) {
            a[q] = to_bf16(As[r][4 * q4 + q]);
            b[q] = to_bf16(Bs[4 * q4 + q][cc]);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][j], 0, 0, 0);
        } else {
          // four k-slices of 4: lane holds A[r][4s + q4] and B[4s + q4][cc]
          for (int sl = 0; sl < 4; ++sl)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[r][4 * sl + q4], Bs[4 * sl + q4][cc], acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane holds D[4*q4 + q][r16] of each 16 x 16 tile
  const int r16 = lane & 15, q4 = lane >> 4;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wm + 16 * i + 4 * q4 + q;
        const int col = n0 + wn + 16 * j + r16;
        float* cp = C + (int64_t)row * ldc + col;
        *cp = accumulate ? *cp + acc[i][j][q] : acc[i][j][q];
      }
}

// per sample: features, (a, c, L, x_max), Fourier weights
__global__ void k_prepare(int B, const double* __restrict__ smp, const int32_t* __restrict__ idx,
                          const int32_t* __restrict__ Lover, float* __restrict__ feat, float* __restrict__ prm,
                          float* __restrict__ wF) {
  const int s = blockIdx.x;
  if (s >= B) return;
  const double* r = smp + 4 * (int64_t)(idx ? idx[s] : s);
  const double a = r[2] * r[0], c = r[2] * r[1];
  int L = (int)ceil(2.0 * kPi / a);
  if (Lover) L = Lover[0];
  if (L > kLM) L = kLM;
  if (L < 1) L = 1;
  const double xm = 0.5 * r[2] * sqrt(r[3]);
  if (threadIdx.x == 0) {
    prm[4 * s + 0] = (float)a;
    prm[4 * s + 1] = (float)c;
    prm[4 * s + 2] = (float)L;
    prm[4 * s + 3] = (float)xm;
  }
  if (threadIdx.x < kNF) {
    const int t = threadIdx.x;
    float v = 0.f;
    if (t == 0) v = (float)(a / kPi);
    if (t == 1) v = (float)(c / kPi);
    if (t == 2) v = (float)xm;
    if (t == 3) v = (float)L / kLM;
    feat[(int64_t)s * kNF + t] = v;
  }
  for (int l = threadIdx.x; l < kLM; l += blockDim.x) {
    double w = 0.0;
    if (l == 0)
      w = 2.0 * (c - a) / kPi;
    else if (l < L)
      w = 4.0 / (kPi * l) * sin(0.5 * l * (c - a)) * cos(0.5 * l * (c + a));
    wF[(int64_t)s * kLM + l] = (float)w;
  }
}

__global__ void k_qmat(float* __restrict__ Q) {
  const int l = blockIdx.x;
  for (int g = threadIdx.x; g < kG; g += blockDim.x) {
    const double x = kXmaxGrid * g / (kG - 1);
    const double phi = 2.0 * asin(x);
    Q[(int64_t)l * kG + g] = (float)(cos((l + 0.5) * phi) / cos(0.5 * phi));
  }
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_g(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Z += bias; H = gelu(Z)
__global__ void k_bias_gelu(int M, int N, float* __restrict__ Z, const float* __restrict__ b, float* __restrict__ H) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * N) return;
  const float z = Z[t] + b[t % N];
  Z[t] = z;
  H[t] = gelu_f(z);
}

// w = (wF + s * (out + b4)) * [l < L]
__global__ void k_out_weights(int B, const float* __restrict__ out, const float* __restrict__ b4,
                              const float* __restrict__ wF, const float* __restrict__ prm, float* __restrict__ w,
                              int use_net) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * kLM) return;
  const int s = (int)(t / kLM), l = (int)(t % kLM);
  const int L = (int)prm[4 * s + 2];
  const float d = use_net ? kOut * (out[t] + b4[l]) : 0.f;
  w[t] = l < L ? wF[t] + d : 0.f;
}

// per sample (one workgroup): loss J and dJ/dbeta (scaled by 1/B)
__global__ __launch_bounds__(256) void k_loss(int B, const float* __restrict__ beta, const float* __restrict__ prm,
                                              float* __restrict__ dbeta, float* __restrict__ J, float scale) {
  __shared__ float red[4][4];
  const int s = blockIdx.x;
  const float a = prm[4 * s], c = prm[4 * s + 1], Lf = prm[4 * s + 2], xm = prm[4 * s + 3];
  const float lo = 0.5f * a, hi = 0.5f * c, d = (float)(kPi / (2.0 * Lf));
  float ni = 0.f, no = 0.f, ji = 0.f, jo = 0.f;
  for (int g = threadIdx.x; g < kG; g += blockDim.x) {
    const float x = kXmaxGrid * g / (kG - 1);
    const float bt = beta[(int64_t)s * kG + g];
    if (x >= lo && x <= hi) {
      ni += 1.f;
      ji += (bt - 1.f) * (bt - 1.f);
    } else if (x <= xm && (x < lo - d || x > hi + d)) {
      no += 1.f;
      jo += bt * bt;
    }
  }
  float v[4] = {ni, no, ji, jo};
  for (int q = 0; q < 4; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
  for (int q = 0; q < 4; ++q) v[q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  const float NI = fmaxf(v[0], 1.f), NO = fmaxf(v[1], 1.f);
  if (threadIdx.x == 0 && J) J[s] = v[2] / NI + v[3] / NO;
  if (!dbeta) return;
  for (int g = threadIdx.x; g < kG; g += blockDim.x) {
    const float x = kXmaxGrid * g / (kG - 1);
    const float bt = beta[(int64_t)s * kG + g];
    float gr = 0.f;
    if (x >= lo && x <= hi)
      gr = 2.f * (bt - 1.f) / NI;
    else if (x <= xm && (x < lo - d || x > hi + d))
      gr = 2.f * bt / NO;
    dbeta[(int64_t)s * kG + g] = gr * scale;
  }
}

// dout = s * dw * [l < L]
__global__ void k_mask_scale(int B, const float* __restrict__ dw, const float* __restrict__ prm,
                             float* __restrict__ dout) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * kLM) return;
  const int s = (int)(t / kLM), l = (int)(t % kLM);
  dout[t] = l < (int)prm[4 * s + 2] ? kOut * dw[t] : 0.f;
}

// D = D * gelu'(Z)
__global__ void k_gelu_back(int64_t n, float* __restrict__ D, const float* __restrict__ Z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) D[t] *= gelu_g(Z[t]);
}

// out[n] = sum over rows (fixed order)
__global__ void k_colsum(int M, int N, const float* __restrict__ X, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += X[(int64_t)m * N + n];
  out[n] = s;
}

__global__ void k_adam(int n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gg = g[t];
  const float a = b1 * m1[t] + (1.f - b1) * gg;
  const float b = b2 * m2[t] + (1.f - b2) * gg * gg;
  m1[t] = a;
  m2[t] = b;
  th[t] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ void k_mean(int B, const float* __restrict__ J, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < B; ++i) s += J[i];
    out[0] = (float)(s / B);
  }
}

template <int TA, int TB, bool BF16>
int gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int acc,
         hipStream_t st) {
  if (M % 64 || N % 64 || K % 16) {
    set_error("mlp gemm: shapes must be multiples of 64 / 64 / 16");
    return KF_EINVAL;
  }
  hipLaunchKernelGGL((k_gemm<TA, TB, BF16>), dim3(N / 64, M / 64), dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc,
                     acc);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

inline int nblk(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

}  // namespace
}  // namespace kf

using namespace kf;

struct kf_mlp {
  hipStream_t st = nullptr;
  int cap = 0;  // batch capacity (multiple of 64)
  float* theta = nullptr;
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* Q = nullptr;  // kLM x kG
  // activations (cap rows)
  float *feat = nullptr, *prm = nullptr, *wF = nullptr, *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr,
        *z3 = nullptr, *h3 = nullptr, *out = nullptr, *w = nullptr, *beta = nullptr, *dbeta = nullptr, *dw = nullptr,
        *dh = nullptr, *dz = nullptr, *J = nullptr, *scal = nullptr;
  double* smp = nullptr;  // device samples
  int nsmp_cap = 0;
  int32_t* idx = nullptr;
  int idx_cap = 0;
  int32_t* Lover = nullptr;
  int64_t adam_t = 0;
};

namespace {

int mfail(int code, const std::string& s) {
  set_error(s);
  return code;
}

template <typename T>
int dalloc_m(T** p, size_t n) {
  if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
    *p = nullptr;
    return mfail(KF_ENOMEM, "kf_mlp: device allocation failed");
  }
  return KF_OK;
}

void mfree(void* p) {
  if (p) (void)hipFree(p);
}

int ensure_batch(kf_mlp* net, int B) {
  if (net->cap >= B) return KF_OK;
  float** bufs[] = {&net->feat, &net->prm, &net->wF, &net->z1, &net->h1, &net->z2, &net->h2, &net->z3,
                    &net->h3,   &net->out, &net->w,  &net->beta, &net->dbeta, &net->dw, &net->dh, &net->dz, &net->J};
  for (float** b : bufs) {
    mfree(*b);
    *b = nullptr;
  }
  const size_t Bn = (size_t)B;
  KF_TRY(dalloc_m(&net->feat, Bn * kNF));
  KF_TRY(dalloc_m(&net->prm, Bn * 4));
  KF_TRY(dalloc_m(&net->wF, Bn * kLM));
  KF_TRY(dalloc_m(&net->z1, Bn * kH));
  KF_TRY(dalloc_m(&net->h1, Bn * kH));
  KF_TRY(dalloc_m(&net->z2, Bn * kH));
  KF_TRY(dalloc_m(&net->h2, Bn * kH));
  KF_TRY(dalloc_m(&net->z3, Bn * kH));
  KF_TRY(dalloc_m(&net->h3, Bn * kH));
  KF_TRY(dalloc_m(&net->out, Bn * kLM));
  KF_TRY(dalloc_m(&net->w, Bn * kLM));
  KF_TRY(dalloc_m(&net->beta, Bn * kG));
  KF_TRY(dalloc_m(&net->dbeta, Bn * kG));
  KF_TRY(dalloc_m(&net->dw, Bn * kLM));
  KF_TRY(dalloc_m(&net->dh, Bn * kLM));
  KF_TRY(dalloc_m(&net->dz, Bn * kLM));
  KF_TRY(dalloc_m(&net->J, Bn));
  net->cap = B;
  return KF_OK;
}

int upload_samples(kf_mlp* net, const double* samples, int n) {
  if (n > net->nsmp_cap) {
    mfree(net->smp);
    net->smp = nullptr;
    KF_TRY(dalloc_m(&net->smp, (size_t)n * 4));
    net->nsmp_cap = n;
  }
  for (int i = 0; i < n; ++i) {
    const double* r = samples + 4 * (size_t)i;
    if (!(r[0] > 0) || !(r[1] > r[0]) || !(r[2] > 0) || !(r[3] > 0) || !std::isfinite(r[1]) || !std::isfinite(r[3]))
      return mfail(KF_EINVAL, "kf_mlp: sample " + std::to_string(i) +
                                  " needs 0 < omega_min < omega_max, tau > 0, lambda_max > 0");
    if (2.0 * kPi / (r[2] * r[0]) > kLM) return mfail(KF_EINVAL, "kf_mlp: sample needs more than 512 weights");
  }
  KF_HIP(hipMemcpyAsync(net->smp, samples, sizeof(double) * 4 * n, hipMemcpyHostToDevice, net->st));
  return KF_OK;
}

// forward (use_net: network correction on) and loss; grad: backpropagation
int fwd_bwd(kf_mlp* net, int B, const int32_t* d_idx, bool use_net, bool grad, const int32_t* d_Lover) {
  hipStream_t st = net->st;
  const float* th = net->theta;
  hipLaunchKernelGGL(k_prepare, dim3(B), dim3(256), 0, st, B, net->smp, d_idx, d_Lover, net->feat, net->prm, net->wF);
  KF_HIP(hipGetLastError());
  if (use_net) {
    KF_TRY((gemm<0, 0, true>(B, kH, kNF, net->feat, kNF, th + kOffW1, kH, net->z1, kH, 0, st)));
    hipLaunchKernelGGL(k_bias_gelu, dim3(nblk((int64_t)B * kH)), dim3(256), 0, st, B, kH, net->z1, th + kOffB1, net->h1);
    KF_TRY((gemm<0, 0, true>(B, kH, kH, net->h1, kH, th + kOffW2, kH, net->z2, kH, 0, st)));
    hipLaunchKernelGGL(k_bias_gelu, dim3(nblk((int64_t)B * kH)), dim3(256), 0, st, B, kH, net->z2, th + kOffB2, net->h2);
    KF_TRY((gemm<0, 0, true>(B, kH, kH, net->h2, kH, th + kOffW3, kH, net->z3, kH, 0, st)));
    hipLaunchKernelGGL(k_bias_gelu, dim3(nblk((int64_t)B * kH)), dim3(256), 0, st, B, kH, net->z3, th + kOffB3, net->h3);
    KF_TRY((gemm<0, 0, true>(B, kLM, kH, net->h3, kH, th + kOffW4, kLM, net->out, kLM, 0, st)));
  }
  hipLaunchKernelGGL(k_out_weights, dim3(nblk((int64_t)B * kLM)), dim3(256), 0, st, B, net->out, th + kOffB4, net->wF,
                     net->prm, net->w, use_net ? 1 : 0);
  KF_TRY((gemm<0, 0, false>(B, kG, kLM, net->w, kLM, net->Q, kG, net->beta, kG, 0, st)));
  hipLaunchKernelGGL(k_loss, dim3(B), dim3(256), 0, st, B, net->beta, net->prm, grad ? net->dbeta : nullptr, net->J,
                     1.0f / B);
  KF_HIP(hipGetLastError());
  if (!grad) return KF_OK;
  float* g = net->grad;
  // dw = dbeta Q^T ; dout = s * dw * mask
  KF_TRY((gemm<0, 1, false>(B, kLM, kG, net->dbeta, kG, net->Q, kG, net->dw, kLM, 0, st)));
  hipLaunchKernelGGL(k_mask_scale, dim3(nblk((int64_t)B * kLM)), dim3(256), 0, st, B, net->dw, net->prm, net->dz);
  // layer 4
  KF_TRY((gemm<1, 0, true>(kH, kLM, B, net->h3, kH, net->dz, kLM, g + kOffW4, kLM, 0, st)));
  hipLaunchKernelGGL(k_colsum, dim3(nblk(kLM)), dim3(256), 0, st, B, kLM, net->dz, g + kOffB4);
  KF_TRY((gemm<0, 1, true>(B, kH, kLM, net->dz, kLM, th + kOffW4, kLM, net->dh, kH, 0, st)));
  hipLaunchKernelGGL(k_gelu_back, dim3(nblk((int64_t)B * kH)), dim3(256), 0, st, (int64_t)B * kH, net->dh, net->z3);
  // layer 3
  KF_TRY((gemm<1, 0, true>(kH, kH, B, net->h2, kH, net->dh, kH, g + kOffW3, kH, 0, st)));
  hipLaunchKernelGGL(k_colsum, dim3(nblk(kH)), dim3(256), 0, st, B, kH, net->dh, g + kOffB3);
  KF_TRY((gemm<0, 1, true>(B, kH, kH, net->dh, kH, th + kOffW3, kH, net->dw, kH, 0, st)));
  hipLaunchKernelGGL(k_gelu_back, dim3(nblk((int64_t)B * kH)), dim3(256), 0, st, (int64_t)B * kH, net->dw, net->z2);
  // layer 2
  KF_TRY((gemm<1, 0, true>(kH, kH, B, net->h1, kH, net->dw, kH, g + kOffW2, kH, 0, st)));
  hipLaunchKernelGGL(k_colsum, dim3(nblk(kH)), dim3(256), 0, st, B, kH, net->dw, g + kOffB2);
  KF_TRY((gemm<0, 1, true>(B, kH, kH, net->dw, kH, th + kOffW2, kH, net->dh, kH, 0, st)));
  hipLaunchKernelGGL(k_gelu_back, dim3(nblk((int64_t)B * kH)), dim3(256), 0, st, (int64_t)B * kH, net->dh, net->z1);
  // layer 1
  KF_TRY((gemm<1, 0, true>(kNF, kH, B, net->feat, kNF, net->dh, kH, g + kOffW1, kH, 0, st)));
  hipLaunchKernelGGL(k_colsum, dim3(nblk(kH)), dim3(256), 0, st, B, kH, net->dh, g + kOffB1);
  KF_HIP(hipGetLastError());
  return KF_OK;
}

void free_mlp(kf_mlp* net) {
  if (!net) return;
  if (net->st) (void)hipStreamSynchronize(net->st);
  void* ps[] = {net->theta, net->grad, net->m1, net->m2, net->Q, net->feat, net->prm, net->wF, net->z1, net->h1,
                net->z2, net->h2, net->z3, net->h3, net->out, net->w, net->beta, net->dbeta, net->dw, net->dh, net->dz,
                net->J, net->scal, net->smp, net->idx, net->Lover};
  for (void* p : ps) mfree(p);
  if (net->st) (void)hipStreamDestroy(net->st);
  delete net;
}

}  // namespace

extern "C" {

int32_t kf_mlp_param_count(void) { return kNParams; }

int kf_mlp_create(const float* params, kf_mlp** out) {
  if (!out || !params) return mfail(KF_EINVAL, "kf_mlp_create: NULL argument");
  *out = nullptr;
  for (int i = 0; i < kNParams; ++i)
    if (!std::isfinite(params[i])) return mfail(KF_EINVAL, "kf_mlp_create: non-finite parameter");
  kf_mlp* net = new (std::nothrow) kf_mlp();
  if (!net) return mfail(KF_ENOMEM, "kf_mlp_create: host allocation");
  int rc = KF_OK;
  do {
    if (hipStreamCreate(&net->st) != hipSuccess) {
      rc = mfail(KF_EHIP, "kf_mlp_create: stream");
      break;
    }
    if ((rc = dalloc_m(&net->theta, kNParams)) || (rc = dalloc_m(&net->grad, kNParams)) ||
        (rc = dalloc_m(&net->m1, kNParams)) || (rc = dalloc_m(&net->m2, kNParams)) ||
        (rc = dalloc_m(&net->Q, (size_t)kLM * kG)) || (rc = dalloc_m(&net->scal, 4)) ||
        (rc = dalloc_m(&net->Lover, 1)))
      break;
    if (hipMemcpy(net->theta, params, sizeof(float) * kNParams, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->m1, 0, sizeof(float) * kNParams) != hipSuccess ||
        hipMemset(net->m2, 0, sizeof(float) * kNParams) != hipSuccess) {
      rc = mfail(KF_EHIP, "kf_mlp_create: upload");
      break;
    }
    hipLaunchKernelGGL(k_qmat, dim3(kLM), dim3(256), 0, net->st, net->Q);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(net->st) != hipSuccess) rc = mfail(KF_EHIP, "kf_mlp_create: Q");
  } while (false);
  if (rc) {
    free_mlp(net);
    return rc;
  }
  *out = net;
  return KF_OK;
}

int kf_mlp_destroy(kf_mlp* net) {
  free_mlp(net);
  return KF_OK;
}

int kf_mlp_get_params(const kf_mlp* net, float* out) {
  if (!net || !out) return mfail(KF_EINVAL, "kf_mlp_get_params: NULL argument");
  KF_HIP(hipMemcpy(out, net->theta, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
  return KF_OK;
}

int kf_mlp_loss_grad(kf_mlp* net, const double* samples, int32_t n, double* loss, float* grad) {
  if (!net || !samples || !loss || n < 1) return mfail(KF_EINVAL, "kf_mlp_loss_grad: bad arguments");
  if (n % 64) return mfail(KF_EINVAL, "kf_mlp_loss_grad: n must be a multiple of 64");
  KF_TRY(ensure_batch(net, n));
  KF_TRY(upload_samples(net, samples, n));
  KF_TRY(fwd_bwd(net, n, nullptr, true, grad != nullptr, nullptr));
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, net->st, n, net->J, net->scal);
  float lf = 0.f;
  KF_HIP(hipMemcpyAsync(&lf, net->scal, sizeof(float), hipMemcpyDeviceToHost, net->st));
  if (grad) KF_HIP(hipMemcpyAsync(grad, net->grad, sizeof(float) * kNParams, hipMemcpyDeviceToHost, net->st));
  KF_HIP(hipStreamSynchronize(net->st));
  *loss = lf;
  return KF_OK;
}

int kf_mlp_train(kf_mlp* net, const double* samples, int32_t n, const int32_t* order, int32_t epochs, int32_t batch,
                 double lr, double* epoch_loss) {
  if (!net || !samples || !order || n < 1 || epochs < 1) return mfail(KF_EINVAL, "kf_mlp_train: bad arguments");
  if (batch < 64 || batch % 64 || batch > n) return mfail(KF_EINVAL, "kf_mlp_train: batch must be a multiple of 64, <= n");
  if (!(lr > 0)) return mfail(KF_EINVAL, "kf_mlp_train: lr must be positive");
  for (int64_t i = 0; i < (int64_t)epochs * n; ++i)
    if (order[i] < 0 || order[i] >= n) return mfail(KF_EINVAL, "kf_mlp_train: order out of range");
  KF_TRY(ensure_batch(net, batch));
  KF_TRY(upload_samples(net, samples, n));
  const int64_t total = (int64_t)epochs * n;
  if (total > net->idx_cap) {
    mfree(net->idx);
    net->idx = nullptr;
    KF_TRY(dalloc_m(&net->idx, (size_t)total));
    net->idx_cap = (int)total;
  }
  KF_HIP(hipMemcpyAsync(net->idx, order, sizeof(int32_t) * total, hipMemcpyHostToDevice, net->st));
  const int steps = n / batch;
  std::vector<float> Jh((size_t)batch);
  for (int e = 0; e < epochs; ++e) {
    double acc = 0.0;
    for (int s = 0; s < steps; ++s) {
      const int32_t* d_idx = net->idx + (int64_t)e * n + (int64_t)s * batch;
      KF_TRY(fwd_bwd(net, batch, d_idx, true, true, nullptr));
      ++net->adam_t;
      // cosine decay from lr to lr/100 over the run
      const double prog = (double)(e * steps + s) / std::max(1, epochs * steps - 1);
      const double lrt = lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(kPi * prog)));
      const float c1 = (float)(1.0 - std::pow(0.9, (double)net->adam_t));
      const float c2 = (float)(1.0 - std::pow(0.999, (double)net->adam_t));
      hipLaunchKernelGGL(k_adam, dim3(nblk(kNParams)), dim3(256), 0, net->st, kNParams, net->theta, net->grad, net->m1,
                         net->m2, (float)lrt, 0.9f, 0.999f, 1e-8f, c1, c2);
      KF_HIP(hipGetLastError());
      if (epoch_loss) {
        KF_HIP(hipMemcpyAsync(Jh.data(), net->J, sizeof(float) * batch, hipMemcpyDeviceToHost, net->st));
        KF_HIP(hipStreamSynchronize(net->st));
        for (float v : Jh) acc += v;
      }
    }
    if (epoch_loss) epoch_loss[e] = acc / ((double)steps * batch);
  }
  KF_HIP(hipStreamSynchronize(net->st));
  return KF_OK;
}

int kf_mlp_weights(kf_mlp* net, const double* samples, int32_t n, double* w_out) {
  if (!net || !samples || !w_out || n < 1) return mfail(KF_EINVAL, "kf_mlp_weights: bad arguments");
  // padded to a multiple of 64 rows by repeating the last sample
  const int np = (n + 63) / 64 * 64;
  std::vector<double> rep((size_t)4 * np);
  std::memcpy(rep.data(), samples, sizeof(double) * 4 * (size_t)n);
  for (int i = n; i < np; ++i) std::memcpy(&rep[4 * (size_t)i], samples + 4 * (size_t)(n - 1), sizeof(double) * 4);
  KF_TRY(ensure_batch(net, np));
  KF_TRY(upload_samples(net, rep.data(), np));
  KF_TRY(fwd_bwd(net, np, nullptr, true, false, nullptr));
  std::vector<float> wl((size_t)n * kLM);
  KF_HIP(hipMemcpyAsync(wl.data(), net->w, sizeof(float) * wl.size(), hipMemcpyDeviceToHost, net->st));
  KF_HIP(hipStreamSynchronize(net->st));
  for (size_t i = 0; i < wl.size(); ++i) w_out[i] = wl[i];
  return KF_OK;
}

int kf_weights_from_mlp(kf_mlp* net, double omega_min, double omega_max, double tau, double lambda_max, int32_t L,
                        double* w_out, int32_t* used_learned, double* j_learned, double* j_fourier) {
  if (!net || !w_out || !used_learned) return mfail(KF_EINVAL, "kf_weights_from_mlp: NULL argument");
  if (L < 1) return mfail(KF_EINVAL, "kf_weights_from_mlp: L must be >= 1");
  const double smp[4] = {omega_min, omega_max, tau, lambda_max};
  if (!(omega_min > 0) || !(omega_max > omega_min) || !(tau > 0) || !(lambda_max > 0))
    return mfail(KF_EINVAL, "kf_weights_from_mlp: need 0 < omega_min < omega_max, tau > 0, lambda_max > 0");
  const double a = tau * omega_min, c = tau * omega_max;
  std::vector<double> wf((size_t)L);
  for (int l = 0; l < L; ++l)
    wf[(size_t)l] = l == 0 ? 2.0 * (c - a) / kPi : 4.0 / (kPi * l) * std::sin(0.5 * l * (c - a)) * std::cos(0.5 * l * (c + a));
  *used_learned = 0;
  if (L > kLM) {
    std::memcpy(w_out, wf.data(), sizeof(double) * L);
    return KF_OK;
  }
  // one sample padded to a 64-row batch
  std::vector<double> rep(4 * 64);
  for (int i = 0; i < 64; ++i) std::memcpy(&rep[4 * (size_t)i], smp, sizeof(smp));
  KF_TRY(ensure_batch(net, 64));
  if (net->nsmp_cap < 64) {
    mfree(net->smp);
    net->smp = nullptr;
    KF_TRY(dalloc_m(&net->smp, 4 * 64));
    net->nsmp_cap = 64;
  }
  KF_HIP(hipMemcpyAsync(net->smp, rep.data(), sizeof(double) * 4 * 64, hipMemcpyHostToDevice, net->st));
  KF_HIP(hipMemcpyAsync(net->Lover, &L, sizeof(int32_t), hipMemcpyHostToDevice, net->st));
  float jf = 0.f, jl = 0.f;
  std::vector<float> wl((size_t)kLM);
  // the acceptance gate: Fourier weights (network off), then the network's weights
  KF_TRY(fwd_bwd(net, 64, nullptr, false, false, net->Lover));
  KF_HIP(hipMemcpyAsync(&jf, net->J, sizeof(float), hipMemcpyDeviceToHost, net->st));
  KF_HIP(hipStreamSynchronize(net->st));
  KF_TRY(fwd_bwd(net, 64, nullptr, true, false, net->Lover));
  KF_HIP(hipMemcpyAsync(&jl, net->J, sizeof(float), hipMemcpyDeviceToHost, net->st));
  KF_HIP(hipMemcpyAsync(wl.data(), net->w, sizeof(float) * kLM, hipMemcpyDeviceToHost, net->st));
  KF_HIP(hipStreamSynchronize(net->st));
  if (j_learned) *j_learned = jl;
  if (j_fourier) *j_fourier = jf;
  if (std::isfinite(jl) && jl < jf) {
    *used_learned = 1;
    for (int l = 0; l < L; ++l) w_out[l] = wl[(size_t)l];
  } else {
    std::memcpy(w_out, wf.data(), sizeof(double) * L);
  }
  return KF_OK;
}

}  // extern "C"
