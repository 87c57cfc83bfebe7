// C ABI and host-side control of the filtered time-domain Krylov eigensolver.
//
// The solve follows Algorithm 2.5 (Krylov loop around the time loop) with
// the readings adopted for this library: block of b start vectors, M-inner
// classical Gram-Schmidt applied twice, a relative drop test instead of an
// exact zero (breakdown), and Rayleigh-Ritz on the projected pencil of eq.
// projevp with the residual acceptance of Section 2.4 (eq. res).  Every step
// on vectors of length n runs in the device kernels; the host only decides
// control flow from a few scalars per iteration.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <atomic>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/kf.h"
#include "kf_internal.h"

namespace kf {

static thread_local std::string g_err = "no error";
void set_error(const std::string& msg) { g_err = msg; }

}  // namespace kf

using namespace kf;

// time-stepping buffers (n x cap blocks)
struct StepBufs {
  void* Y0 = nullptr;
  void* Y1 = nullptr;
  void* R = nullptr;
  void* Z = nullptr;  // fourth-order stepper: z = A y
  void* Y2 = nullptr;  // several steps per launch: the second pair of levels
  void* Y3 = nullptr;
  int cap = 0;  // block width held
  int vb = 0;   // value bytes
};

namespace kf {
namespace {
// the stream and pinned staging buffer a Rayleigh-Ritz check runs on (the
// problem's own, or those of the check that overlaps the Krylov loop)
struct Io {
  hipStream_t st;
  char* pin;
  size_t pin_cap;
};
}  // namespace
}  // namespace kf

namespace {
struct AsyncCheck;
}  // namespace

struct kf_problem {
  int32_t n = 0;
  int64_t nnz = 0;
  double omega_min = 0, omega_max = 0, tau = 0;
  int32_t L = 0;
  kf_options opt{};
  hipStream_t st = nullptr;
  std::vector<double> w;  // filter coefficients w_l = tau*alpha(l*tau)

  double* d_m = nullptr;  // lumped mass
  SellOp A;               // tau^2 M^{-1} S in the stepping precision
  SellOp A64;             // float64 copy for the mixed-mode refinement
  SellOp S;               // S in float64 (projection, residuals)

  // time-stepping buffers (n x bk): stepping precision, and float64 for the
  // mixed-mode refinement
  StepBufs sb;    // stepping precision
  StepBufs sb64;  // float64 (mixed-mode refinement)
  // refinement blocks (n x rcap, leading dimension ldb)
  double* Vx = nullptr;
  double* Yy = nullptr;
  double* Ysel = nullptr;  // gathered small vectors (k x rcap)
  double* Gm = nullptr;    // rcap x rcap
  int rcap = 0;
  int rkcap = 0;
  // Krylov basis and projected pencil
  double* B = nullptr;
  int64_t ldb = 0;
  int bcap = 0;       // basis columns allocated
  double* H = nullptr;
  double* G = nullptr;
  int hcap = 0;
  double* T = nullptr;  // (bcap x 64) coefficients
  double* W = nullptr;  // n x 16 scratch (S Q)
  double* V = nullptr;  // n x 64 Ritz vectors
  double* SV = nullptr; // n x 64
  double* small = nullptr;  // device scalars
  int32_t* flags = nullptr;
  GemvTWork gw;
  GemvTWork rw;
  EigWork ew;
  int basis_cols = 0;
  // 0, 1: filter start / end, 2: orthogonalisation end, 3, 4: check start /
  // end; 5, 6: start / end of a filter application queued ahead (swapped
  // with 0, 1 when it is kept)
  hipEvent_t ev[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // phases of the filtered subspace iteration (filter, orthonormalisation,
  // projection and residuals)
  hipEvent_t sev[4] = {nullptr, nullptr, nullptr, nullptr};
  double tuned_us = 0.0;
  // k x k work arrays of the pencil correction (E, E H, corrected H)
  double* rr_work = nullptr;
  size_t rr_cap = 0;
  // batch members with their own stream (concurrent projection work)
  bool own_stream = false;
  hipEvent_t sync_ev = nullptr;
  int device = 0;  // the GPU the problem's memory lives on
  // pinned host staging for the values read back at every Krylov step
  // (copies into it are queued without blocking the host)
  char* pin = nullptr;
  size_t pin_cap = 0;
  // 64 bytes past pin_cap that the window step's kernel writes directly
  // (device address of the same pinned memory), so that no copy is queued
  double* win_rec_host = nullptr;
  double* win_rec_dev = nullptr;
  // a Rayleigh-Ritz check running on its own stream and host thread while
  // the Krylov loop goes on (kf_solve in float64)
  AsyncCheck* ac = nullptr;
  // the weights on the device for the several-steps-per-launch kernel
  double* d_w = nullptr;
  int d_w_cap = 0;
  std::vector<double> d_w_host;
};

// One stacked block-diagonal operator of a batch with its step buffers,
// weight table and captured filter graph.  A batch in KF_MIXED holds two:
// the float32 stack every member starts on, and a float64 stack that the
// members restarted with float64 stepping (kf_options.escalate) continue on
// inside the same batched loop.
struct BatchStack {
  SellOp A;
  void* wtab = nullptr;  // P x lmax weights, in the stack's precision
  StepBufs sb;
  BatchTables h_tb{};    // per-member tables of the next launch (active members of this stack)
  BatchTables* d_tb = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_bk = 0;
  int remap = 1;  // XCD mapping of the batched step (timed with autotune)
  bool tuned = false;
};

struct kf_batch {
  int P = 0;
  int workers = 1;  // host threads driving the members' projection work
  std::vector<kf_problem*> probs;
  hipStream_t st = nullptr;
  BatchStack stk[2];
  int nstk = 1;
  int32_t* d_sp = nullptr;   // slice -> problem
  int lmax = 1;
  int64_t rows = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // members are stacked by decreasing L: at step ell the members still
  // stepping own the first prefix[ell] row slices
  std::vector<int> prefix;
  int autotune = 0;
  // members passed the same operator arrays (slices of one problem's
  // spectrum) share a group: they share the operator's eigenvalue
  // multiplicities, so when float32 stepping fails for one of them the
  // others restart with float64 stepping at once
  std::vector<int> group;
  std::vector<char> fp64_member;  // mixed batches: members that step in float64 from the start
};

namespace {

constexpr size_t kPinBytes = (size_t)64 << 10;  // pinned staging for per-step readbacks
constexpr int kSmall = 4096;
// offsets of the device scalars in kf_problem::small used by the
// orthogonalisation (the Rayleigh-Ritz check uses 1024.. and 2048..)
constexpr int kPost = 256, kNrm2 = 512, kG2 = 768, kT1 = 1100, kRec = 2560, kRinv = 3072, kOne = 4095;
// a block is orthonormalised by Cholesky QR (twice) when every pivot keeps at
// least this fraction of its column's squared M-norm; otherwise column by
// column (classical Gram-Schmidt twice, with the drop test)
constexpr double kCholPivot = 1e-8;
// mixed mode: refinements tried before a solve with a target gives up
constexpr int kMaxRefines = 4;
// columns projected only every proj_every steps must be M-orthogonal to the
// older basis to this level, else they are orthogonalised again and the
// projection interval is halved; the Rayleigh-Ritz step's first-order
// correction leaves an eigenvalue error of order |E|^2 <= 1e-14 relative
constexpr double kPendingTol = 1e-7;

int pow2ceil(int b) {
  int p = 1;
  while (p < b) p <<= 1;
  return p;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

std::vector<double> fourier_weights(double omin, double omax, double tau, int L) {
  // eq. weightf sampled on the left rectangle nodes l*tau, l < L (T = L*tau)
  std::vector<double> w((size_t)L);
  const double pi = 3.14159265358979323846;
  for (int l = 0; l < L; ++l) {
    const double t = l * tau;
    const double a = (l == 0) ? 2.0 * (omax - omin) / pi
                              : 4.0 / (pi * t) * std::sin(0.5 * t * (omax - omin)) * std::cos(0.5 * t * (omax + omin));
    w[(size_t)l] = tau * a;
  }
  return w;
}

int validate_csr_host(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const double* val,
                      const double* m) {
  if (n < 1) return fail(KF_EINVAL, "kf: n must be >= 1");
  if (nnz < 0) return fail(KF_EINVAL, "kf: nnz must be >= 0");
  if (rowptr[0] != 0 || (int64_t)rowptr[n] != nnz) return fail(KF_EINVAL, "kf: rowptr[0] must be 0 and rowptr[n] = nnz");
  for (int32_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return fail(KF_EINVAL, "kf: rowptr must be non-decreasing");
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      if (col[q] < 0 || col[q] >= n) return fail(KF_EINVAL, "kf: column index out of range in row " + std::to_string(i));
      if (q > rowptr[i] && col[q] <= col[q - 1])
        return fail(KF_EINVAL, "kf: column indices must be strictly increasing within row " + std::to_string(i));
      if (!std::isfinite(val[q])) return fail(KF_EINVAL, "kf: non-finite matrix value in row " + std::to_string(i));
    }
  }
  for (int32_t i = 0; i < n; ++i)
    if (!(m[i] > 0.0) || !std::isfinite(m[i])) return fail(KF_EINVAL, "kf: m_diag must be positive and finite");
  return KF_OK;
}

// Host copies of a CSR (pulls device arrays back for validation).
struct HostCsr {
  std::vector<int32_t> rowptr, col;
  std::vector<double> val, m;
};

int fetch_csr(const kf_csr* S, const double* m_diag, HostCsr& h) {
  if (!S || !m_diag) return fail(KF_EINVAL, "kf: NULL matrix or mass");
  if (S->n < 1 || S->nnz < 0) return fail(KF_EINVAL, "kf: n must be >= 1 and nnz >= 0");
  if (!S->rowptr || (S->nnz > 0 && (!S->col || !S->val))) return fail(KF_EINVAL, "kf: NULL CSR array");
  const size_t n = (size_t)S->n, nnz = (size_t)S->nnz;
  try {
    h.rowptr.resize(n + 1);
    h.col.resize(nnz);
    h.val.resize(nnz);
    h.m.resize(n);
  } catch (const std::bad_alloc&) {
    return fail(KF_ENOMEM, "kf: host allocation failed");
  }
  if (S->on_device) {
    KF_HIP(hipMemcpy(h.rowptr.data(), S->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    if (nnz) {
      KF_HIP(hipMemcpy(h.col.data(), S->col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
      KF_HIP(hipMemcpy(h.val.data(), S->val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    }
    KF_HIP(hipMemcpy(h.m.data(), m_diag, sizeof(double) * n, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(h.rowptr.data(), S->rowptr, sizeof(int32_t) * (n + 1));
    if (nnz) {
      std::memcpy(h.col.data(), S->col, sizeof(int32_t) * nnz);
      std::memcpy(h.val.data(), S->val, sizeof(double) * nnz);
    }
    std::memcpy(h.m.data(), m_diag, sizeof(double) * n);
  }
  return validate_csr_host(S->n, S->nnz, h.rowptr.data(), h.col.data(), h.val.data(), h.m.data());
}

struct DevCsr {
  int32_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  ~DevCsr() {
    if (rowptr) (void)hipFree(rowptr);
    if (col) (void)hipFree(col);
    if (val) (void)hipFree(val);
  }
};

int upload_csr(const HostCsr& h, int32_t n, int64_t nnz, hipStream_t st, DevCsr& d) {
  const size_t nz = std::max<int64_t>(nnz, 1);
  if (hipMalloc(&d.rowptr, sizeof(int32_t) * (n + 1)) != hipSuccess || hipMalloc(&d.col, sizeof(int32_t) * nz) != hipSuccess ||
      hipMalloc(&d.val, sizeof(double) * nz) != hipSuccess)
    return fail(KF_ENOMEM, "kf: device allocation for the CSR copy failed");
  KF_HIP(hipMemcpyAsync(d.rowptr, h.rowptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
  if (nnz) {
    KF_HIP(hipMemcpyAsync(d.col, h.col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
    KF_HIP(hipMemcpyAsync(d.val, h.val.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st));
  }
  KF_HIP(hipStreamSynchronize(st));
  return KF_OK;
}

template <typename Tp>
int dalloc(Tp** p, size_t count) {
  *p = nullptr;
  if (hipMalloc((void**)p, sizeof(Tp) * std::max<size_t>(count, 1)) != hipSuccess) {
    *p = nullptr;
    return fail(KF_ENOMEM, "kf: device allocation of " + std::to_string(sizeof(Tp) * count) + " bytes failed");
  }
  return KF_OK;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

int ensure_step_buffers(kf_problem* p, StepBufs& sb, int bk, int vb) {
  const bool needz = p->opt.stepper == 4;
  const bool need23 = p->opt.multistep != 0 && bk == 1;
  if (sb.cap >= bk && sb.vb == vb && (!needz || sb.Z) && (!need23 || sb.Y3)) return KF_OK;
  dfree(sb.Y0);
  dfree(sb.Y1);
  dfree(sb.R);
  dfree(sb.Z);
  dfree(sb.Y2);
  dfree(sb.Y3);
  sb = StepBufs();
  const size_t bytes = (size_t)p->n * bk * vb;
  if (hipMalloc(&sb.Y0, bytes) != hipSuccess || hipMalloc(&sb.Y1, bytes) != hipSuccess ||
      hipMalloc(&sb.R, bytes) != hipSuccess || (needz && hipMalloc(&sb.Z, bytes) != hipSuccess) ||
      (need23 && (hipMalloc(&sb.Y2, bytes) != hipSuccess || hipMalloc(&sb.Y3, bytes) != hipSuccess)))
    return fail(KF_ENOMEM, "kf: time-stepping buffers");
  sb.cap = bk;
  sb.vb = vb;
  return KF_OK;
}

// Fixed device memory for kf_apply_filter_noalloc: one copy per GPU (the
// runtime places the array on every device the library runs on), held until
// the process ends.  Host code never passes the array's name to a kernel:
// that is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  KF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(KF_EINVAL, "kf: device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(KF_EHIP, std::string("kf: no device address for the scratch array: ") + hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return KF_OK;
}

// The n x bk time-stepping blocks (three, four for the fourth-order
// stepper) carved out of the scratch array.
int scratch_step_buffers(int32_t n, int bk, int vb, StepBufs& sb, int nbuf = 3) {
  const size_t one = ((size_t)n * bk * vb + 255) / 256 * 256;
  if (nbuf * one > kScratchBytes)
    return fail(KF_EINVAL, "kf_apply_filter_noalloc: " + std::to_string(nbuf) + " x n x " + std::to_string(bk) +
                               " x " + std::to_string(vb) + " bytes exceed the fixed " +
                               std::to_string(kScratchBytes >> 20) + " MiB");
  void* base = nullptr;
  KF_TRY(scratch_address(&base));
  char* c = static_cast<char*>(base);
  sb.Y0 = c;
  sb.Y1 = c + one;
  sb.R = c + 2 * one;
  sb.Z = nbuf > 3 ? c + 3 * one : nullptr;
  sb.cap = bk;
  sb.vb = vb;
  return KF_OK;
}

void free_step_buffers(StepBufs& sb) {
  dfree(sb.Y0);
  dfree(sb.Y1);
  dfree(sb.R);
  dfree(sb.Z);
  dfree(sb.Y2);
  dfree(sb.Y3);
  sb = StepBufs();
}

// LDS a workgroup may use (device attribute, read once per device).
size_t lds_per_workgroup() {
  static std::mutex mu;
  static int cached[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 65536;
  std::lock_guard<std::mutex> lk(mu);
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    cached[dev] = v;
  }
  return (size_t)cached[dev];
}

// The filter weights on the device (float64), uploaded when they change.
int device_weights(kf_problem* p, const std::vector<double>& w, const double** out) {
  if (p->d_w_host != w) {
    if ((int)w.size() > p->d_w_cap) {
      dfree(p->d_w);
      p->d_w = nullptr;
      p->d_w_cap = 0;
      KF_TRY(dalloc(&p->d_w, w.size()));
      p->d_w_cap = (int)w.size();
    }
    KF_HIP(hipMemcpyAsync(p->d_w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, p->st));
    KF_HIP(hipStreamSynchronize(p->st));
    p->d_w_host = w;
  }
  *out = p->d_w;
  return KF_OK;
}

// C applied to bsrc columns of src (strides srs between rows, scs between
// columns; float64) with kernel block width bk; the first bout columns of the
// result go to dst (strides drs, dcs).  Asynchronous.
int run_filter(kf_problem* p, const SellOp& A, StepBufs& sb, const double* src, int64_t srs, int64_t scs, int bsrc,
               int bk, double* dst, int64_t drs, int64_t dcs, int bout, const std::vector<double>& w,
               bool may_alloc = true) {
  const int L = (int)w.size();
  hipStream_t st = p->st;
  if (L == 1) return launch_scale_copy(p->n, bout, std::min(bsrc, bout), src, srs, scs, w[0], dst, drs, dcs, st);
  if (may_alloc) {
    KF_TRY(ensure_step_buffers(p, sb, bk, A.val_bytes));
  } else if (sb.cap < bk || sb.vb != A.val_bytes || !sb.Y0 || !sb.Y1 || !sb.R || (p->opt.stepper == 4 && !sb.Z)) {
    return fail(KF_EINVAL, "kf: time-stepping buffers too small");
  }
  // a single float64 vector stored contiguously already has the layout of a
  // step buffer: the first two steps read it in place (no load launch);
  // otherwise it is loaded (converted, interleaved) into Y1
  const bool direct = A.val_bytes == 8 && bk == 1 && bsrc == 1 && srs == 1;
  const void* y0 = direct ? static_cast<const void*>(src) : sb.Y1;
  if (!direct) KF_TRY(launch_load_block(A.val_bytes, p->n, bk, bsrc, src, srs, scs, sb.Y1, st));
  if (p->opt.multistep != 0 && bk == 1 && p->opt.stepper != 4 && sb.Y3) {
    // several steps per launch (banded operators): levels alternate between
    // the pairs (Y0, Y1) and (Y2, Y3); the input stays where it was loaded
    const int s = p->opt.multistep > 0 ? std::min(p->opt.multistep, L - 1) : L - 1;
    const MultiStepPlan pl = plan_multistep(A, s, lds_per_workgroup());
    if (!pl.ok)
      return fail(KF_EINVAL, "kf: multistep: " + std::to_string(s) + " steps of a band of " + std::to_string(A.max_off) +
                                 " rows do not fit in a workgroup's LDS");
    const double* dw = nullptr;
    KF_TRY(device_weights(p, w, &dw));
    void* P0[2] = {sb.Y0, sb.Y1};
    void* P1[2] = {sb.Y2, sb.Y3};
    int l = 0, ping = 0;
    while (l < L - 1) {
      const int cnt = std::min(s, L - 1 - l);
      const bool last = l + cnt == L - 1;
      void** in = ping ? P1 : P0;
      void** outp = ping ? P0 : P1;
      KF_TRY(launch_leapfrog_mp(A, pl, l, cnt, l == 0, last, y0, in[0], in[1], outp[0], outp[1], sb.R, dst, drs, dw, st));
      l += cnt;
      ping ^= 1;
    }
    return KF_OK;
  }
  void* Y[2] = {sb.Y0, sb.Y1};
  auto wt = [&](int i) { return i < 0 ? 0.0 : w[(size_t)i]; };
  for (int l = 1; l < L; ++l) {
    const StepPlan sp = step_plan(l, L);
    // step l reads y_l (cur) and y_{l-1} (prev) and writes y_{l+1} over
    // y_{l-1}, except at l = 2 where y_1 is the source itself
    const void* cur = l == 1 ? y0 : Y[l & 1];
    void* nxt = Y[(l + 1) & 1];
    const void* prv = l == 2 ? y0 : nxt;
    if (p->opt.stepper == 4)
      KF_TRY(launch_leapfrog4(A, bk, sp.mode, cur, prv, nxt, sb.R, sb.Z, dst, drs, dcs, bout, wt(sp.ip), wt(sp.ic),
                              wt(sp.in), p->opt.xcd_remap, st));
    else
      KF_TRY(launch_leapfrog(A, bk, sp.mode, cur, prv, nxt, sb.R, dst, drs, dcs, bout, wt(sp.ip), wt(sp.ic),
                             wt(sp.in), p->opt.xcd_remap, st));
  }
  return KF_OK;
}

int ensure_basis(kf_problem* p, int cols) {
  if (p->bcap >= cols) return KF_OK;
  dfree(p->B);
  dfree(p->H);
  dfree(p->G);
  dfree(p->T);
  p->B = p->H = p->G = p->T = nullptr;
  p->bcap = p->hcap = 0;
  p->basis_cols = 0;
  p->ldb = ((int64_t)p->n + 63) / 64 * 64;
  KF_TRY(dalloc(&p->B, (size_t)p->ldb * cols));
  KF_TRY(dalloc(&p->H, (size_t)cols * cols));
  KF_TRY(dalloc(&p->G, (size_t)cols * cols));
  KF_TRY(dalloc(&p->T, (size_t)cols * 64));
  p->bcap = cols;
  p->hcap = cols;
  return KF_OK;
}

// Grow the basis storage to at least `need` columns (B, and H, G and the
// coefficient buffer T with it), keeping the first `keep` basis columns and
// the leading keep x keep blocks of H and G.  The copies are queued behind
// all work on the stream, which is synchronised before the old storage goes.
int async_wait(kf_problem* p);

int grow_basis(kf_problem* p, int need, int keep) {
  if (p->bcap >= need) return KF_OK;
  if (!p->B) return ensure_basis(p, need);
  // a check running on its own stream reads B, H and G
  KF_TRY(async_wait(p));
  hipStream_t st = p->st;
  const int cap = std::max(need, 2 * p->bcap);
  double *nB = nullptr, *nH = nullptr, *nG = nullptr, *nT = nullptr;
  int rc = dalloc(&nB, (size_t)p->ldb * cap);
  if (!rc) rc = dalloc(&nH, (size_t)cap * cap);
  if (!rc) rc = dalloc(&nG, (size_t)cap * cap);
  if (!rc) rc = dalloc(&nT, (size_t)cap * 64);
  if (rc) {
    dfree(nB);
    dfree(nH);
    dfree(nG);
    dfree(nT);
    return rc;
  }
  keep = std::min(keep, p->bcap);
  if (keep > 0) {
    KF_HIP(hipMemcpyAsync(nB, p->B, sizeof(double) * p->ldb * keep, hipMemcpyDeviceToDevice, st));
    KF_HIP(hipMemcpy2DAsync(nH, sizeof(double) * cap, p->H, sizeof(double) * p->hcap, sizeof(double) * keep, keep,
                            hipMemcpyDeviceToDevice, st));
    KF_HIP(hipMemcpy2DAsync(nG, sizeof(double) * cap, p->G, sizeof(double) * p->hcap, sizeof(double) * keep, keep,
                            hipMemcpyDeviceToDevice, st));
  }
  KF_HIP(hipStreamSynchronize(st));
  dfree(p->B);
  dfree(p->H);
  dfree(p->G);
  dfree(p->T);
  p->B = nB;
  p->H = nH;
  p->G = nG;
  p->T = nT;
  p->bcap = p->hcap = cap;
  return KF_OK;
}

int ensure_misc(kf_problem* p) {
  if (p->W) return KF_OK;
  KF_TRY(dalloc(&p->W, (size_t)p->n * 16));
  KF_TRY(dalloc(&p->V, (size_t)p->n * 64));
  KF_TRY(dalloc(&p->SV, (size_t)p->n * 64));
  KF_TRY(dalloc(&p->small, kSmall));
  KF_TRY(dalloc(&p->flags, 64));
  if (hipHostMalloc((void**)&p->pin, kPinBytes + 64, hipHostMallocDefault) != hipSuccess) {
    p->pin = nullptr;
    return fail(KF_ENOMEM, "kf: cannot allocate the pinned staging buffer");
  }
  p->pin_cap = kPinBytes;
  p->win_rec_host = reinterpret_cast<double*>(p->pin + kPinBytes);
  if (hipHostGetDevicePointer((void**)&p->win_rec_dev, p->win_rec_host, 0) != hipSuccess)
    return fail(KF_EHIP, "kf: no device address for the pinned staging buffer");
  const double one = 1.0;
  KF_HIP(hipMemcpy(p->small + kOne, &one, sizeof(double), hipMemcpyHostToDevice));
  return KF_OK;
}

// Orthonormalise columns [c0, c0+nb) of B against B[:, 0:kb) and among
// themselves (M inner product, CGS applied twice at both levels), drop
// columns that lose more than drop_tol of their M-norm, compact the kept
// columns to [c0, c0+kept).  ref_out receives the pre-orthogonalisation
// M-norms.  Synchronises the stream.
// pn > 0: the projected-pencil columns of basis columns [kb - pn, kb) are
// still pending; they are computed in the same pass over B as the first
// Gram-Schmidt coefficients (one pass fewer per Krylov iteration).
//
// loc0 >= 0 selects the three-term form: C is M-self-adjoint (Lemma 2.3,
// C = beta~(M^{-1}S)), so the filtered block is M-orthogonal, in exact
// arithmetic, to every basis block except the last two, [loc0, kb).  The
// block is first orthogonalised against that window, then once against the
// whole basis (the second pass for the window's columns); another full pass
// runs only when the full pass removed more than half of the M-norm of a
// column (the test of Daniel, Gragg, Kaufman and Stewart).  loc0 < 0 runs
// classical Gram-Schmidt twice against the whole basis.
//
// The block's own Gram matrix rides along as extra rows of the first
// projection (the block sits right after its left operand in B: X is column
// kb = c0), so the norms before each pass cost no launch of their own.
//
// monitor = false (three-term form, between the periodic projections): the
// window pass is the only pass over the basis; a single vector is normalised
// from the window's Gram matrix, a block by Cholesky QR twice.  Columns
// formed this way stay pending until the next projection (pn > 0), which
// forms their pencil entries and checks their drift from M-orthogonality with
// the older basis (*pending_loose; drifted columns are repaired).
//
// carried != null (one vector, three-term form, pending columns): the
// periodic projection also cleans the last pending column, column kb - 1,
// against the rest of the basis, in the same subtraction as the new column.
// The recurrence builds each new column from the last two, so their losses of
// orthogonality both pass into the next column: cleaning only the new one
// leaves the next columns near the level the last pending one had reached,
// and the interval between projections shrinks.  Column kb - 1 changes after
// its pencil entries were formed, so *carried = true asks the caller to keep
// it pending (its entries are formed again at the next projection).
int rr_update(kf_problem* p, int c0, int nc);
int repair_block(kf_problem* p, int p0, int pn);

// Device-to-host reads of a few values through the problem's pinned staging
// buffer: `get` queues the copy without blocking the host (a copy into
// pageable memory waits for the stream, so a step's three or four reads
// would cost as many round trips), `land` moves the values to their
// destinations after the caller has synchronised the stream.  Reads that do
// not fit go straight to their destination.
struct Readback {
  hipStream_t st;
  char* pin;
  size_t pin_cap;
  size_t off = 0;
  struct Item {
    void* dst;
    size_t off, bytes;
  };
  Item items[16];
  int nitems = 0;
  explicit Readback(kf_problem* q) : st(q->st), pin(q->pin), pin_cap(q->pin_cap) {}
  explicit Readback(const Io& io) : st(io.st), pin(io.pin), pin_cap(io.pin_cap) {}
  int get(void* dst, const void* src, size_t bytes) {
    off = (off + 15) & ~(size_t)15;
    if (!pin || off + bytes > pin_cap || nitems == 16) {
      KF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
      return KF_OK;
    }
    KF_HIP(hipMemcpyAsync(pin + off, src, bytes, hipMemcpyDeviceToHost, st));
    items[nitems++] = Item{dst, off, bytes};
    off += bytes;
    return KF_OK;
  }
  void land() {
    for (int i = 0; i < nitems; ++i) std::memcpy(items[i].dst, pin + items[i].off, items[i].bytes);
    nitems = 0;
    off = 0;
  }
};

int orth_block(kf_problem* p, int kb, int c0, int nb, int* kept, std::vector<double>& ref_out,
               hipEvent_t done = nullptr, int pn = 0, int loc0 = -1, int* full_passes = nullptr,
               bool monitor = true, bool* pending_loose = nullptr, const std::function<int()>* ahead = nullptr,
               bool* ahead_kept = nullptr, bool* carried = nullptr) {
  if (c0 != kb) return fail(KF_EINVAL, "orth_block: the block must follow the basis");
  hipStream_t st = p->st;
  const int32_t n = p->n;
  const int64_t ldb = p->ldb;
  double* X = p->B + (int64_t)c0 * ldb;
  double* post = p->small + kPost;   // nb post norms
  double* nrm2 = p->small + kNrm2;   // nb squared norms
  double* g2 = p->small + kG2;       // nb x nb Gram after the full pass (blocks)
  double* T1 = p->small + kT1;       // first projection [(w + nb) x nb]
  double* coef = p->T;               // (kb + nb) x (2 pn + nb), 2 more with carried
  const bool local = kb > 0 && loc0 >= 0;
  const int lw = local ? kb - loc0 : 0;
  // first projection: the window [loc0, kb) (none without the three-term
  // form) and the block itself; rows lw.. hold the block's Gram matrix
  const int ld1 = lw + nb;
  double* L1 = p->B + (int64_t)(kb - lw) * ldb;
  const double* Tref = T1 + lw;  // nb x nb, leading dimension ld1
  // one vector between projections: the window pass and the normalisation
  // in three launches and one readback (the norm from the window's Gram
  // matrix and the new column's products with it)
  const bool fused = kb > 0 && nb == 1 && !monitor && local && lw <= 2;
  if (!fused) {
    KF_TRY(gemv_t(n, ld1, L1, ldb, nullptr, 0, 0, X, nb, ldb, p->d_m, T1, ld1, p->gw, st));
    if (lw > 0) KF_TRY(gemv_n_sub(n, lw, L1, ldb, T1, ld1, X, ldb, nb, st));
  }
  // pass over the whole basis; the first one also forms the pending
  // projected-pencil columns [B^T S Q | B^T M Q] with Q = B[:, kb-pn:kb]; the
  // rows below kb give the block's Gram matrix before the pass
  const int ldc = kb + nb;
  // gated: (one vector) subtract only when a coefficient exceeds reorth_tol
  // times the column's M-norm; the decision is taken on the device
  int32_t* gate = p->flags + 32;
  auto full_pass = [&](bool with_pending, bool gated = false) -> int {
    const double* cx = coef;
    if (with_pending && pn > 0) {
      const int p0 = kb - pn;
      const double* Q = p->B + (int64_t)p0 * ldb;
      KF_TRY(spmv_cols(p->S, Q, ldb, p->W, n, pn, nullptr, st));
      KF_TRY(gemv_t(n, ldc, p->B, ldb, p->W, pn, n, Q, pn + nb, ldb, p->d_m, coef, ldc, p->gw, st));
      KF_TRY(rr_scatter(kb, p0, pn, coef, ldc, p->H, p->G, p->hcap, st));
      cx = coef + (int64_t)2 * pn * ldc;
    } else {
      KF_TRY(gemv_t(n, ldc, p->B, ldb, nullptr, 0, 0, X, nb, ldb, p->d_m, coef, ldc, p->gw, st));
    }
    if (gated && nb == 1) KF_TRY(reorth_gate(kb, cx, cx + kb, p->opt.reorth_tol, gate, st));
    if (gated && nb > 1) KF_TRY(reorth_gate_block(kb, nb, cx, ldc, p->opt.reorth_tol, gate, st));
    if (carried && local && with_pending && pn > 0 && nb == 1) {
      // columns kb - 1 and kb in one pass over the basis: the coefficients of
      // column kb - 1 (without its own row) beside those of the new column
      double* pc = coef + (int64_t)(2 * pn + 1) * ldc;
      KF_TRY(pair_coef(kb, coef + (int64_t)(2 * pn - 1) * ldc, cx, pc, ldc, p->opt.reorth_tol, gated ? gate : nullptr,
                       st));
      KF_TRY(gemv_n_sub(n, kb, p->B, ldb, pc, ldc, X - ldb, ldb, 2, st, gated ? gate : nullptr));
      *carried = true;
    } else {
      KF_TRY(gemv_n_sub(n, kb, p->B, ldb, cx, ldc, X, ldb, nb, st, gated ? gate : nullptr));
    }
    if (full_passes && !gated) ++*full_passes;
    return KF_OK;
  };
  const double drop = p->opt.drop_tol > 0 ? p->opt.drop_tol : 1e-10;
  std::vector<double> hv((size_t)ld1 * nb);
  std::vector<int32_t> fl((size_t)nb);
  bool have = false;  // hv and fl hold the final device values
  Readback rb(p);
  auto fetch = [&](const double* src, size_t count, void* dst) -> int { return rb.get(dst, src, sizeof(double) * count); };
  // in-block CGS2 and normalisation of column j against ref2 (device)
  auto finish_cols = [&](const double* ref_base, int64_t ref_ld) -> int {
    for (int j = 0; j < nb; ++j) {
      double* xj = X + (int64_t)j * ldb;
      if (j > 0) {
        for (int pass = 0; pass < 2; ++pass) {
          KF_TRY(gemv_t(n, j, X, ldb, nullptr, 0, 0, xj, 1, ldb, p->d_m, coef, j, p->gw, st));
          KF_TRY(gemv_n_sub(n, j, X, ldb, coef, j, xj, ldb, 1, st));
        }
      }
      KF_TRY(gemv_t(n, 1, xj, ldb, nullptr, 0, 0, xj, 1, ldb, p->d_m, nrm2 + j, 1, p->gw, st));
      KF_TRY(normalize_col(n, xj, nrm2 + j, ref_base + (int64_t)j * ref_ld + j, drop, p->flags + j, post + j, st));
    }
    return KF_OK;
  };
  if (kb > 0 && !local) {
    KF_TRY(full_pass(true));
    KF_TRY(full_pass(false));
    KF_TRY(finish_cols(Tref, ld1));
    if (done) KF_HIP(hipEventRecord(done, st));
  } else if (kb > 0 && nb == 1 && !monitor) {
    // between projections: the window pass only; the coefficients against
    // the older basis are formed at the next projection (every proj_every
    // steps), which also checks how far this column is from orthogonal
    double g2h = 0.0;
    bool explicit_norm = !fused;
    if (fused) {
      double* rec = p->small + kRec;
      // the record {T, g, status} is also written straight to pinned host
      // memory by the kernel (read after the synchronisation below)
      KF_TRY(window_step(n, lw, L1, ldb, p->d_m, p->gw, T1, rec, st, p->win_rec_dev));
      if (ahead && done) {
        // queue the next filter application (on this column) before waiting
        // for the readback: the host's turnaround overlaps the time steps;
        // the caller drops it if this column is changed below
        KF_HIP(hipEventRecord(done, st));
        KF_TRY((*ahead)());
        KF_HIP(hipEventSynchronize(done));
        if (ahead_kept) *ahead_kept = true;
      } else {
        if (done) KF_HIP(hipEventRecord(done, st));
        KF_HIP(hipStreamSynchronize(st));
      }
      rb.land();
      const double* rh = p->win_rec_host;
      for (int j = 0; j <= lw; ++j) hv[(size_t)j] = rh[j];
      g2h = rh[lw + 1];
      fl[0] = 1;
      // status 2: strong cancellation in the window pass, the norm by
      // Pythagoras is not accurate; normalise against the explicit norm
      explicit_norm = rh[lw + 2] != 1.0;
      if (explicit_norm && ahead_kept) *ahead_kept = false;
    }
    if (explicit_norm) {
      KF_TRY(finish_cols(Tref, ld1));
      KF_TRY(fetch(nrm2, 1, &g2h));
      KF_TRY(rb.get(fl.data(), p->flags, sizeof(int32_t)));
      KF_TRY(fetch(T1, (size_t)ld1, hv.data()));
      if (done) KF_HIP(hipEventRecord(done, st));
      KF_HIP(hipStreamSynchronize(st));
      rb.land();
    }
    have = true;
    if (fl[0] && g2h < 1e-4 * hv[(size_t)lw]) {
      if (ahead_kept) *ahead_kept = false;
      have = false;
      // the window pass removed all but 1 % of the norm: its rounding is no
      // longer negligible, so this column gets a pass against the whole basis
      KF_TRY(full_pass(false));
      KF_TRY(gemv_t(n, 1, X, ldb, nullptr, 0, 0, X, 1, ldb, p->d_m, nrm2, 1, p->gw, st));
      KF_TRY(normalize_col(n, X, nrm2, p->small + kOne, drop, p->flags, post, st));
      if (done) KF_HIP(hipEventRecord(done, st));
    }
  } else if (kb > 0 && nb == 1) {
    // one vector: its norm after the full pass is the normalisation norm, so
    // the second-pass test and the drop test share one synchronisation
    const bool gated = p->opt.reorth_tol > 0.0;
    KF_TRY(full_pass(true, gated));
    int32_t* loose = p->flags + 33;
    if (pending_loose && pn > 0) KF_TRY(block_gate(kb, kb - pn, pn, coef + (int64_t)pn * ldc, ldc, kPendingTol, loose, st));
    KF_TRY(finish_cols(Tref, ld1));
    double g1 = 0.0, g2h = 0.0;
    int32_t gh = 1, lh = 0;
    KF_TRY(fetch(coef + kb + (int64_t)(2 * pn) * ldc, 1, &g1));
    KF_TRY(fetch(nrm2, 1, &g2h));
    KF_TRY(rb.get(fl.data(), p->flags, sizeof(int32_t)));
    if (gated) KF_TRY(rb.get(&gh, gate, sizeof(int32_t)));
    if (pending_loose && pn > 0) KF_TRY(rb.get(&lh, loose, sizeof(int32_t)));
    KF_TRY(fetch(T1, (size_t)ld1, hv.data()));
    if (done) KF_HIP(hipEventRecord(done, st));
    KF_HIP(hipStreamSynchronize(st));
    rb.land();
    have = true;
    if (pending_loose) *pending_loose = lh != 0;
    if (full_passes && gated && gh) ++*full_passes;
    if (lh) {
      // the columns formed since the previous projection drifted from
      // M-orthogonality: repair them, then orthogonalise the new column
      // against the repaired ones
      KF_TRY(repair_block(p, kb - pn, pn));
      KF_TRY(full_pass(false));
      KF_TRY(full_pass(false));
      KF_TRY(gemv_t(n, 1, X, ldb, nullptr, 0, 0, X, 1, ldb, p->d_m, nrm2, 1, p->gw, st));
      KF_TRY(normalize_col(n, X, nrm2, p->small + kOne, drop, p->flags, post, st));
      if (done) KF_HIP(hipEventRecord(done, st));
      KF_TRY(rb.get(fl.data(), p->flags, sizeof(int32_t)));
      KF_HIP(hipStreamSynchronize(st));
      rb.land();
    } else if (fl[0] && g2h < 0.25 * g1) {
      // the column is normalised now: one more pass against the whole basis,
      // dropped if it loses all but drop_tol of its unit norm
      have = false;
      KF_TRY(full_pass(false));
      KF_TRY(gemv_t(n, 1, X, ldb, nullptr, 0, 0, X, 1, ldb, p->d_m, nrm2, 1, p->gw, st));
      KF_TRY(normalize_col(n, X, nrm2, p->small + kOne, drop, p->flags, post, st));
      if (done) KF_HIP(hipEventRecord(done, st));
    }
  } else if (kb > 0) {
    std::vector<double> hg1((size_t)ldc * nb), hg2((size_t)nb * nb);
    bool again = false;
    bool between = local && !monitor;
    const bool hv_read = between;  // hv holds T1 (read with the Gram matrix)
    if (between) {
      // a block between projections (three-term form): the window pass above
      // is its only pass over the basis; Cholesky QR within the block when
      // no column lost more than all but 1e-4 of its squared M-norm to the
      // window (else the cancellation calls for the full pass below)
      KF_TRY(gemv_t(n, nb, X, ldb, nullptr, 0, 0, X, nb, ldb, p->d_m, g2, nb, p->gw, st));
      KF_TRY(fetch(g2, (size_t)nb * nb, hg2.data()));
      KF_TRY(fetch(T1, (size_t)ld1 * nb, hv.data()));
      KF_HIP(hipStreamSynchronize(st));
      rb.land();
      for (int j = 0; j < nb; ++j)
        if (!(hg2[(size_t)j * nb + j] >= 1e-4 * hv[(size_t)lw + j + (size_t)j * ld1])) between = false;
      if (!between) {
        // (the columns formed since the last projection stay pending)
        KF_TRY(full_pass(false));
        KF_TRY(full_pass(false));
        KF_TRY(gemv_t(n, nb, X, ldb, nullptr, 0, 0, X, nb, ldb, p->d_m, g2, nb, p->gw, st));
        KF_TRY(fetch(g2, (size_t)nb * nb, hg2.data()));
        KF_HIP(hipStreamSynchronize(st));
        rb.land();
      }
    } else {
      // (the window pass was the first pass: this one subtracts only where a
      // coefficient exceeds reorth_tol times its column's M-norm, as for
      // single vectors)
      const bool gated = p->opt.reorth_tol > 0.0;
      KF_TRY(full_pass(true, gated));
      int32_t* loose = p->flags + 33;
      int32_t lh = 0, gh = 1;
      const bool gate_pending = pending_loose && pn > 0 && local;
      // columns formed since the previous projection were orthogonalised
      // against their window only: their drift from M-orthogonality with the
      // older basis is checked here (as for single vectors)
      if (gate_pending) KF_TRY(block_gate(kb, kb - pn, pn, coef + (int64_t)pn * ldc, ldc, kPendingTol, loose, st));
      KF_TRY(gemv_t(n, nb, X, ldb, nullptr, 0, 0, X, nb, ldb, p->d_m, g2, nb, p->gw, st));
      KF_TRY(fetch(coef + (int64_t)(2 * pn) * ldc, (size_t)ldc * nb, hg1.data()));
      KF_TRY(fetch(g2, (size_t)nb * nb, hg2.data()));
      if (gate_pending) KF_TRY(rb.get(&lh, loose, sizeof(int32_t)));
      if (gated) KF_TRY(rb.get(&gh, gate, sizeof(int32_t)));
      KF_HIP(hipStreamSynchronize(st));
      rb.land();
      if (pending_loose) *pending_loose = lh != 0;
      if (full_passes && gated && gh) ++*full_passes;
      if (lh) {
        // repair the drifted columns, then orthogonalise the block against
        // the repaired basis twice
        KF_TRY(repair_block(p, kb - pn, pn));
        KF_TRY(full_pass(false));
        KF_TRY(full_pass(false));
        KF_TRY(gemv_t(n, nb, X, ldb, nullptr, 0, 0, X, nb, ldb, p->d_m, g2, nb, p->gw, st));
        KF_TRY(fetch(g2, (size_t)nb * nb, hg2.data()));
        KF_HIP(hipStreamSynchronize(st));
        rb.land();
      } else {
        for (int j = 0; j < nb; ++j)
          if (hg2[(size_t)j * nb + j] < 0.25 * hg1[(size_t)kb + j + (size_t)j * ldc]) again = true;
      }
    }
    if (again) KF_TRY(full_pass(false));
    // within the block: Cholesky QR twice (four launches per pass, and no
    // column can be dropped: the full pass kept >= 1/4 of every norm and each
    // pivot keeps >= kCholPivot of its column) when the Gram matrix after the
    // full pass is well conditioned, else column by column; the pivots are
    // checked on the copy of G read back for the second-pass test above
    bool chol = !again;
    std::vector<double> R((size_t)nb * nb, 0.0);  // upper triangle, column-major
    for (int j = 0; chol && j < nb; ++j) {
      double d = hg2[(size_t)j + (size_t)j * nb];
      for (int i = 0; i < j; ++i) {
        double t = hg2[(size_t)i + (size_t)j * nb];
        for (int q = 0; q < i; ++q) t -= R[(size_t)q + (size_t)i * nb] * R[(size_t)q + (size_t)j * nb];
        t /= R[(size_t)i + (size_t)i * nb];
        R[(size_t)i + (size_t)j * nb] = t;
        d -= t * t;
      }
      // (a zero column, e.g. the padding of a block of b < bk filtered
      // columns, has d = 0 and must be dropped: the column path does that)
      if (!std::isfinite(d) || !(d > 0.0) || !(d >= kCholPivot * hg2[(size_t)j + (size_t)j * nb]))
        chol = false;
      else
        R[(size_t)j + (size_t)j * nb] = std::sqrt(d);
    }
    if (chol) {
      double* Rinv = p->small + kRinv;
      KF_TRY(chol_orthonormalise(n, nb, X, ldb, g2, Rinv, p->flags, post, st));
      KF_TRY(gemv_t(n, nb, X, ldb, nullptr, 0, 0, X, nb, ldb, p->d_m, g2, nb, p->gw, st));
      KF_TRY(chol_orthonormalise(n, nb, X, ldb, g2, Rinv, p->flags, post, st));
      if (hv_read) {
        // every column kept: nothing more to read back
        for (int j = 0; j < nb; ++j) fl[(size_t)j] = 1;
        have = true;
      }
    } else {
      KF_TRY(finish_cols(Tref, ld1));
    }
    if (done) KF_HIP(hipEventRecord(done, st));
  } else {
    KF_TRY(finish_cols(Tref, ld1));
    if (done) KF_HIP(hipEventRecord(done, st));
  }
  if (!have) {
    // (single vectors usually have both from their one synchronisation)
    KF_TRY(fetch(T1, (size_t)ld1 * nb, hv.data()));
    KF_TRY(rb.get(fl.data(), p->flags, sizeof(int32_t) * nb));
    KF_HIP(hipStreamSynchronize(st));
    rb.land();
  }
  ref_out.assign((size_t)nb, 0.0);
  for (int j = 0; j < nb; ++j) ref_out[(size_t)j] = std::sqrt(std::max(hv[(size_t)lw + j + (size_t)j * ld1], 0.0));
  int cnt = 0;
  for (int j = 0; j < nb; ++j) {
    if (!fl[(size_t)j]) continue;
    if (j != cnt)
      KF_HIP(hipMemcpyAsync(X + (int64_t)cnt * ldb, X + (int64_t)j * ldb, sizeof(double) * n, hipMemcpyDeviceToDevice,
                            st));
    ++cnt;
  }
  *kept = cnt;
  return KF_OK;
}

// New columns [c0, c0+nc) of the basis: add their rows/columns to
// H = B^T S B and G = B^T M B.
int rr_update(kf_problem* p, int c0, int nc) {
  const int k = c0 + nc;
  hipStream_t st = p->st;
  const double* Q = p->B + (int64_t)c0 * p->ldb;
  KF_TRY(spmv_cols(p->S, Q, p->ldb, p->W, p->n, nc, nullptr, st));
  KF_TRY(gemv_t(p->n, k, p->B, p->ldb, p->W, nc, p->n, Q, nc, p->ldb, p->d_m, p->T, k, p->gw, st));
  KF_TRY(rr_scatter(k, c0, nc, p->T, k, p->H, p->G, p->hcap, st));
  return KF_OK;
}

// Basis columns [p0, p0 + pn) that drifted from M-orthogonality: classical
// Gram-Schmidt twice against the older columns and twice among themselves,
// normalisation, and their projected-pencil columns again.
int repair_block(kf_problem* p, int p0, int pn) {
  hipStream_t st = p->st;
  const int32_t n = p->n;
  const int64_t ldb = p->ldb;
  double* Q = p->B + (int64_t)p0 * ldb;
  double* coef = p->T;
  double* nrm2 = p->small + kNrm2 + 32;
  for (int pass = 0; pass < 2 && p0 > 0; ++pass) {
    KF_TRY(gemv_t(n, p0, p->B, ldb, nullptr, 0, 0, Q, pn, ldb, p->d_m, coef, p0, p->gw, st));
    KF_TRY(gemv_n_sub(n, p0, p->B, ldb, coef, p0, Q, ldb, pn, st));
  }
  for (int j = 0; j < pn; ++j) {
    double* qj = Q + (int64_t)j * ldb;
    for (int pass = 0; pass < 2 && j > 0; ++pass) {
      KF_TRY(gemv_t(n, j, Q, ldb, nullptr, 0, 0, qj, 1, ldb, p->d_m, coef, j, p->gw, st));
      KF_TRY(gemv_n_sub(n, j, Q, ldb, coef, j, qj, ldb, 1, st));
    }
    KF_TRY(gemv_t(n, 1, qj, ldb, nullptr, 0, 0, qj, 1, ldb, p->d_m, nrm2 + j, 1, p->gw, st));
    KF_TRY(normalize_col(n, qj, nrm2 + j, nullptr, 0.0, p->flags + 40, nrm2 + 16 + j, st));
  }
  return rr_update(p, p0, pn);
}

struct CheckOut {
  std::vector<double> ritz;       // all Ritz values
  std::vector<double> acc_theta;  // accepted
  std::vector<double> acc_res;
  std::vector<int> acc_sel;       // index into the candidate list
  std::vector<double> cand_theta; // candidates (interval widened by the margin)
  std::vector<double> cand_res;
  std::vector<double> vectors;    // n x accepted (host), when requested
  double orth = 0.0;
};

// Ritz vectors V = Bk Ysel (chunks of 64), residuals ||S v - theta M v|| /
// ||S v|| and acceptance (theta inside the interval and residual <= tol).
// ew.Y holds the k x nsel eigenvectors for sel.
int ritz_residuals(kf_problem* p, const double* Bk, int64_t ldb, int k, const std::vector<double>& sel_in, double tol,
                   bool want_vectors, CheckOut& out, bool rayleigh = false, const double* Ysel = nullptr,
                   const Io* io = nullptr) {
  // Ysel: the k x sel eigenvectors (default: ew.Y)
  if (!Ysel) Ysel = p->ew.Y;
  std::vector<double> sel = sel_in;
  const Io mio{p->st, p->pin, p->pin_cap};
  if (!io) io = &mio;
  hipStream_t st = io->st;
  const int nsel = (int)sel.size();
  out.cand_theta = sel;
  out.cand_res.assign(sel.size(), 0.0);
  out.acc_theta.clear();
  out.acc_res.clear();
  out.acc_sel.clear();
  out.vectors.clear();
  const double lo2 = p->omega_min * p->omega_min, hi2 = p->omega_max * p->omega_max;
  double* d_theta = p->small + 2048;
  double* d_num = p->small + 2048 + 64;
  double* d_den = p->small + 2048 + 128;
  for (int c0 = 0; c0 < nsel; c0 += 64) {
    const int nc = std::min(64, nsel - c0);
    KF_TRY(gemm_nn(p->n, k, Bk, ldb, Ysel + (int64_t)c0 * k, k, p->V, p->n, nc, st));
    KF_TRY(spmv_cols(p->S, p->V, p->n, p->SV, p->n, nc, nullptr, st));
    if (rayleigh) {
      // theta <- v^T S v / v^T M v for each Ritz vector
      double* q = p->small + 2048 + 192;  // 2 x 64
      for (int c = 0; c < nc; ++c)
        KF_TRY(gemv_t(p->n, 1, p->V + (int64_t)c * p->n, p->n, p->SV + (int64_t)c * p->n, 1, p->n,
                      p->V + (int64_t)c * p->n, 1, p->n, p->d_m, q + 2 * c, 1, p->gw, st));
      std::vector<double> hq((size_t)2 * nc);
      Readback rq(*io);
      KF_TRY(rq.get(hq.data(), q, sizeof(double) * 2 * nc));
      KF_HIP(hipStreamSynchronize(st));
      rq.land();
      for (int c = 0; c < nc; ++c)
        if (hq[(size_t)2 * c + 1] > 0.0) sel[(size_t)c0 + c] = hq[(size_t)2 * c] / hq[(size_t)2 * c + 1];
      out.cand_theta = sel;
    }
    KF_HIP(hipMemcpyAsync(d_theta, sel.data() + c0, sizeof(double) * nc, hipMemcpyHostToDevice, st));
    KF_TRY(residual_norms(p->n, p->SV, p->V, p->n, p->d_m, d_theta, nc, d_num, d_den, p->rw, st));
    std::vector<double> num((size_t)nc), den((size_t)nc);
    Readback rr(*io);
    KF_TRY(rr.get(num.data(), d_num, sizeof(double) * nc));
    KF_TRY(rr.get(den.data(), d_den, sizeof(double) * nc));
    KF_HIP(hipStreamSynchronize(st));
    rr.land();
    for (int c = 0; c < nc; ++c) {
      const double th = sel[(size_t)c0 + c];
      double dn = std::sqrt(den[(size_t)c]);
      if (!(dn > 0.0)) dn = std::max(std::fabs(th), 1e-300);
      const double r = std::sqrt(std::max(num[(size_t)c], 0.0)) / dn;
      out.cand_res[(size_t)c0 + c] = r;
      const double om = std::sqrt(std::max(th, 0.0));
      const bool inside = th >= lo2 && th <= hi2 && om >= p->omega_min && om <= p->omega_max;
      if (inside && r <= tol) {
        out.acc_theta.push_back(th);
        out.acc_res.push_back(r);
        out.acc_sel.push_back(c0 + c);
        if (want_vectors) {
          const size_t off = out.vectors.size();
          out.vectors.resize(off + (size_t)p->n);
          KF_HIP(hipMemcpyAsync(out.vectors.data() + off, p->V + (int64_t)c * p->n, sizeof(double) * p->n,
                                hipMemcpyDeviceToHost, st));
        }
      }
    }
    if (want_vectors) KF_HIP(hipStreamSynchronize(st));
  }
  return KF_OK;
}

// eigenvalues of the k x k symmetric matrix Hm (ld ldh) into out (host), and
// eigenvectors for those selected by keep() into ew.Y; returns the selection
template <class Keep>
int eig_select(EigWork& ew, int k, const double* Hm, int64_t ldh, std::vector<double>& theta, Keep keep,
               std::vector<double>& sel, hipStream_t st) {
  KF_TRY(eig_values(ew, k, Hm, ldh, st));
  theta.assign((size_t)k, 0.0);
  KF_HIP(hipMemcpyAsync(theta.data(), ew.theta, sizeof(double) * k, hipMemcpyDeviceToHost, st));
  KF_HIP(hipStreamSynchronize(st));
  sel.clear();
  for (int i = 0; i < k; ++i)
    if (keep(theta[(size_t)i])) sel.push_back(theta[(size_t)i]);
  const int nsel = (int)sel.size();
  if (nsel == 0) return KF_OK;
  // clusters of (nearly) equal values get mutually orthogonal vectors
  const double tn = std::max(std::fabs(theta.front()), std::fabs(theta.back()));
  std::vector<int32_t> cl{0};
  for (int i = 1; i < nsel; ++i)
    if (sel[(size_t)i] - sel[(size_t)i - 1] > 1e-9 * tn) cl.push_back(i);
  const int ncl = (int)cl.size();
  cl.push_back(nsel);
  return eig_vectors(ew, k, sel.data(), cl.data(), ncl, nsel, st);
}

template <class Keep>
int small_eigen(kf_problem* p, int k, const double* Hm, int64_t ldh, std::vector<double>& theta, Keep keep,
                std::vector<double>& sel, hipStream_t st = nullptr) {
  return eig_select(p->ew, k, Hm, ldh, theta, keep, sel, st ? st : p->st);
}

// Rayleigh-Ritz on the leading k basis columns.  Residuals are formed for the
// Ritz values with omega in the interval widened by `margin` on both sides;
// acceptance needs omega inside the interval and residual <= tol.
int rr_check(kf_problem* p, int k, double tol, CheckOut& out, double margin, bool want_vectors,
             const Io* io = nullptr) {
  const Io mio{p->st, p->pin, p->pin_cap};
  if (!io) io = &mio;
  hipStream_t st = io->st;
  KF_TRY(orth_error(k, p->G, p->hcap, p->small + 1024, st));
  // lands after the eigensolver's own synchronisation
  Readback ro(*io);
  KF_TRY(ro.get(&out.orth, p->small + 1024, sizeof(double)));
  // The pencil is (H, G) with G = I + E, E at the orthogonality level of the
  // basis: its eigenvalues are those of H - (E H + H E)/2 up to O(|E|^2).
  const double* Hm = p->H;
  int64_t ldh = p->hcap;
  double *E = nullptr, *EH = nullptr;
  if (k >= 2) {
    const size_t need = (size_t)3 * k * k;
    if (p->rr_cap < need) {
      dfree(p->rr_work);
      p->rr_work = nullptr;
      p->rr_cap = 0;
      const size_t cap = (size_t)3 * p->hcap * p->hcap;
      KF_TRY(dalloc(&p->rr_work, cap));
      p->rr_cap = cap;
    }
    E = p->rr_work;
    EH = E + (size_t)k * k;
    double* Hc = EH + (size_t)k * k;
    KF_TRY(pencil_correct(k, p->H, p->G, p->hcap, E, EH, Hc, st));
    Hm = Hc;
    ldh = k;
  }
  const double lo = std::max(p->omega_min - margin, 0.0), hi = p->omega_max + margin;
  std::vector<double> sel;
  KF_TRY(small_eigen(
      p, k, Hm, ldh, out.ritz,
      [&](double th) {
        const double om = std::sqrt(std::max(th, 0.0));
        return om >= lo && om <= hi;
      },
      sel, st));
  KF_HIP(hipStreamSynchronize(st));
  ro.land();
  if (E) KF_TRY(vectors_correct(k, (int)sel.size(), E, p->ew.Y, EH, st));
  return ritz_residuals(p, p->B, p->ldb, k, sel, tol, want_vectors, out, false, nullptr, io);
}

// A Rayleigh-Ritz check that overlaps the Krylov loop: it runs on a stream
// and host thread of its own, on the leading k columns of B and the leading
// k x k blocks of H and G, which the loop no longer writes (new columns
// only add rows and columns past k); the loop waits for it before the basis
// storage is reallocated.  Scratch it uses that the loop does not: V, SV,
// the eigensolver's and the residuals' work arrays, the device scalars from
// offset 1024 on, and its own pinned staging buffer.
struct AsyncCheck {
  hipStream_t st = nullptr;
  char* pin = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // basis ready (loop's stream), check start, end
  std::thread th;
  std::atomic<int> state{0};  // 0 idle, 1 running, 2 finished and not yet taken
  int k = 0;
  double tol = 0.0, margin = 0.0;
  CheckOut out;
  int rc = KF_OK;
  std::string err;
};

int async_ensure(kf_problem* p) {
  if (p->ac) return KF_OK;
  AsyncCheck* ac = new (std::nothrow) AsyncCheck();
  if (!ac) return fail(KF_ENOMEM, "kf: host allocation");
  p->ac = ac;
  KF_HIP(hipStreamCreateWithFlags(&ac->st, hipStreamNonBlocking));
  KF_HIP(hipEventCreateWithFlags(&ac->ev[0], hipEventDisableTiming));
  KF_HIP(hipEventCreate(&ac->ev[1]));
  KF_HIP(hipEventCreate(&ac->ev[2]));
  if (hipHostMalloc((void**)&ac->pin, kPinBytes, hipHostMallocDefault) != hipSuccess) {
    ac->pin = nullptr;
    return fail(KF_ENOMEM, "kf: cannot allocate the check's pinned staging buffer");
  }
  return KF_OK;
}

// Starts the check of the leading k columns once the work queued so far on
// the loop's stream (the pending columns' pencil entries) is done.
int async_start(kf_problem* p, int k, double tol, double margin) {
  KF_TRY(async_ensure(p));
  AsyncCheck* ac = p->ac;
  if (ac->state.load() != 0) return fail(KF_EINVAL, "kf: a check is already running");
  ac->k = k;
  ac->tol = tol;
  ac->margin = margin;
  ac->rc = KF_OK;
  ac->err.clear();
  ac->out = CheckOut();
  KF_HIP(hipEventRecord(ac->ev[0], p->st));
  ac->state.store(1);
  try {
    ac->th = std::thread([p, ac]() {
      int rc = KF_OK;
      try {
        rc = hipSetDevice(p->device) == hipSuccess ? KF_OK : fail(KF_EHIP, "kf: check thread cannot select the GPU");
        if (!rc && hipStreamWaitEvent(ac->st, ac->ev[0], 0) != hipSuccess) rc = fail(KF_EHIP, "kf: check stream wait");
        if (!rc && hipEventRecord(ac->ev[1], ac->st) != hipSuccess) rc = fail(KF_EHIP, "kf: check event");
        const Io io{ac->st, ac->pin, kPinBytes};
        if (!rc) rc = rr_check(p, ac->k, ac->tol, ac->out, ac->margin, false, &io);
        if (!rc && hipEventRecord(ac->ev[2], ac->st) != hipSuccess) rc = fail(KF_EHIP, "kf: check event");
        if (!rc && hipEventSynchronize(ac->ev[2]) != hipSuccess) rc = fail(KF_EHIP, "kf: check synchronisation");
      } catch (...) {
        rc = fail(KF_ENOMEM, "kf: host allocation in the check thread");
      }
      // the stream is drained before the result is handed over, also after
      // an error (nothing it queued may still run when the loop continues)
      (void)hipStreamSynchronize(ac->st);
      if (rc) ac->err = g_err;
      ac->rc = rc;
      ac->state.store(2);
    });
  } catch (...) {
    ac->state.store(0);
    return fail(KF_EHIP, "kf: cannot start the check thread");
  }
  return KF_OK;
}

bool async_running(const kf_problem* p) { return p->ac && p->ac->state.load() != 0; }
bool async_ready(const kf_problem* p) { return p->ac && p->ac->state.load() == 2; }

// Waits for a running check (its result stays to be taken).
int async_wait(kf_problem* p) {
  if (p->ac && p->ac->th.joinable()) p->ac->th.join();
  return KF_OK;
}

// The finished check's result, its basis size and its device time.
int async_take(kf_problem* p, CheckOut& out, int* k, double* seconds) {
  AsyncCheck* ac = p->ac;
  if (!ac || ac->state.load() == 0) return fail(KF_EINVAL, "kf: no check to take");
  KF_TRY(async_wait(p));
  ac->state.store(0);
  if (ac->rc) return fail(ac->rc, ac->err);
  float ms = 0.f;
  KF_HIP(hipEventElapsedTime(&ms, ac->ev[1], ac->ev[2]));
  *seconds = ms * 1e-3;
  *k = ac->k;
  out = std::move(ac->out);
  return KF_OK;
}

void async_free(kf_problem* p) {
  AsyncCheck* ac = p->ac;
  if (!ac) return;
  if (ac->th.joinable()) ac->th.join();
  if (ac->st) (void)hipStreamSynchronize(ac->st);
  for (hipEvent_t e : ac->ev)
    if (e) (void)hipEventDestroy(e);
  if (ac->st) (void)hipStreamDestroy(ac->st);
  if (ac->pin) (void)hipHostFree(ac->pin);
  delete ac;
  p->ac = nullptr;
}

// Mixed-precision refinement.  The near-interval Ritz vectors X of the
// float32 Krylov space (residual <= 0.1, omega within the interval widened by
// the margin) get one float64 application of the filter, Y = C X, which
// damps the high-frequency round-off of the float32 steps; the pencil is
// projected onto span(Y) in float64.  span(Y) is M-orthonormalised through the
// eigen-decomposition of G = Y^T M Y (twice; directions with eigenvalue below
// 1e-12 of the largest are dropped), and each Ritz value is replaced by the
// Rayleigh quotient of its Ritz vector before the residual is taken.
// Limitation: float32 round-off also seeds the copies of a multiple
// eigenvalue that a block of b start vectors cannot see in exact arithmetic
// (multiplicity > b); those half-converged copies contaminate the pairs near
// them, so such spectra need b >= the multiplicity in this mode.
int eig_orthonormalise(kf_problem* p, double* Z, int nz, double* out, int* r_out) {
  // out = Z * U diag(g)^{-1/2} over the kept eigenpairs (g, U) of Z^T M Z
  hipStream_t st = p->st;
  const int n = p->n;
  const int64_t ld = p->ldb;
  for (int c0 = 0; c0 < nz; c0 += 32) {
    const int nb = std::min(32, nz - c0);
    KF_TRY(gemv_t(n, nz, Z, ld, nullptr, 0, 0, Z + (int64_t)c0 * ld, nb, ld, p->d_m, p->Gm + (int64_t)c0 * nz, nz,
                  p->gw, st));
  }
  KF_TRY(symmetrize(nz, p->Gm, nz, st));
  {
    // already M-orthonormal up to E = Z^T M Z - I with |E| <= 1e-8: the
    // inverse square root is I - E/2 to O(|E|^2) (below rounding), and an
    // eigen-decomposition of the all-ones spectrum would be one large cluster
    std::vector<double> Gh((size_t)nz * nz);
    KF_HIP(hipMemcpyAsync(Gh.data(), p->Gm, sizeof(double) * nz * nz, hipMemcpyDeviceToHost, st));
    KF_HIP(hipStreamSynchronize(st));
    double emax = 0.0;
    for (int j = 0; j < nz; ++j)
      for (int i = 0; i < nz; ++i) emax = std::max(emax, std::fabs(Gh[(size_t)j * nz + i] - (i == j ? 1.0 : 0.0)));
    if (emax <= 1e-8) {
      for (int j = 0; j < nz; ++j)
        for (int i = 0; i < nz; ++i) {
          double& g = Gh[(size_t)j * nz + i];
          g = (i == j ? 1.0 : 0.0) - 0.5 * (g - (i == j ? 1.0 : 0.0));
        }
      KF_HIP(hipMemcpyAsync(p->Ysel, Gh.data(), sizeof(double) * nz * nz, hipMemcpyHostToDevice, st));
      KF_TRY(gemm_nn(n, nz, Z, ld, p->Ysel, nz, out, ld, nz, st));
      KF_HIP(hipStreamSynchronize(st));
      *r_out = nz;
      return KF_OK;
    }
  }
  std::vector<double> g, gsel;
  KF_TRY(small_eigen(p, nz, p->Gm, nz, g, [](double) { return true; }, gsel));
  const double gmax = g.empty() ? 0.0 : g.back();
  std::vector<int> keep;
  for (int i = 0; i < nz; ++i)
    if (g[(size_t)i] > 1e-12 * gmax) keep.push_back(i);
  const int r = (int)keep.size();
  *r_out = r;
  if (r == 0) return KF_OK;
  std::vector<double> U((size_t)nz * nz), Th((size_t)nz * r);
  KF_HIP(hipMemcpyAsync(U.data(), p->ew.Y, sizeof(double) * nz * nz, hipMemcpyDeviceToHost, st));
  KF_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < r; ++j) {
    const double sc = 1.0 / std::sqrt(g[(size_t)keep[(size_t)j]]);
    for (int i = 0; i < nz; ++i) Th[(size_t)j * nz + i] = U[(size_t)keep[(size_t)j] * nz + i] * sc;
  }
  KF_HIP(hipMemcpyAsync(p->Ysel, Th.data(), sizeof(double) * nz * r, hipMemcpyHostToDevice, st));
  KF_TRY(gemm_nn(n, nz, Z, ld, p->Ysel, nz, out, ld, r, st));
  KF_HIP(hipStreamSynchronize(st));
  return KF_OK;
}

int distinct_count(const std::vector<double>& acc, int b);

// Two n x cap blocks (Vx, Yy, leading dimension ldb), a cap x cap Gram and a
// kc x cap block of small vectors for the subspace iteration.
int ensure_refine(kf_problem* p, int nc, int k) {
  if (nc <= p->rcap && k <= p->rkcap) return KF_OK;
  dfree(p->Vx);
  dfree(p->Yy);
  dfree(p->Ysel);
  dfree(p->Gm);
  const int cap = std::max({nc, 64, p->rcap});
  const int kc = std::max({k, cap, p->rkcap});
  p->Vx = p->Yy = p->Ysel = p->Gm = nullptr;
  p->rcap = p->rkcap = 0;
  KF_TRY(dalloc(&p->Vx, (size_t)p->ldb * cap));
  KF_TRY(dalloc(&p->Yy, (size_t)p->ldb * cap));
  KF_TRY(dalloc(&p->Ysel, (size_t)kc * cap));
  KF_TRY(dalloc(&p->Gm, (size_t)cap * cap));
  p->rcap = cap;
  p->rkcap = kc;
  return KF_OK;
}

struct SubspaceStats {
  int iters = 0;
  int dim = 0;
  int64_t lf_steps = 0;  // vector time steps
  double t_lf = 0, t_orth = 0, t_rr = 0;
};

// Fixed-dimension filtered subspace iteration (Section 4.4: a space of fixed
// dimension instead of a growing Krylov space, i.e. a FEAST-type method with
// the time-domain filter).  X holds nc columns (device, column-major,
// leading dimension ldb; X and Q are p->Vx and p->Yy in either order, the
// other one is work space).  One iteration:
//   Q = C X with the operator A (float64 or float32 stepping), 16 columns at a
//   time; Q M-orthonormalised twice through the eigen-decomposition of
//   Q^T M Q (directions below 1e-12 of the largest dropped); H = Q^T S Q;
//   the Ritz values with omega in the interval widened by `margin` get Ritz
//   vectors, Rayleigh quotients and residuals (eq. projevp, eq. res);
//   X <- Q for the next iteration (the Ritz vectors span the same space).
// Stops after max_iters iterations, when `target` pairs (counted as
// distinct_count with cnt_b) are accepted, or (target 0) when every Ritz
// value inside the interval is accepted and their number did not change.
// On return X points at the last M-orthonormal block, st.dim its columns.
int subspace_iterate(kf_problem* p, const SellOp& A, StepBufs& sb, double*& X, double*& Q, int nc, int max_iters,
                     double tol, int target, int cnt_b, double margin, bool want_vectors, CheckOut& out,
                     SubspaceStats& stats, int stall_limit = 0) {
  hipStream_t st = p->st;
  const int n = p->n;
  const int64_t ld = p->ldb;
  const double lo = std::max(p->omega_min - margin, 0.0), hi = p->omega_max + margin;
  const double lo2 = p->omega_min * p->omega_min, hi2 = p->omega_max * p->omega_max;
  int prev_inside = -1;
  int best = -1, stalled = 0;
  int cur = nc;
  auto lap = [&](hipEvent_t a, hipEvent_t b, double& acc) -> int {
    KF_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    KF_HIP(hipEventElapsedTime(&ms, a, b));
    acc += 1e-3 * ms;
    return KF_OK;
  };
  for (int it = 0; it < max_iters && cur > 0; ++it) {
    KF_HIP(hipEventRecord(p->sev[0], st));
    for (int c0 = 0; c0 < cur; c0 += 16) {
      const int nb = std::min(16, cur - c0);
      KF_TRY(run_filter(p, A, sb, X + (int64_t)c0 * ld, 1, ld, nb, pow2ceil(nb), Q + (int64_t)c0 * ld, 1, ld, nb,
                        p->w));
    }
    {
      // a time step beyond the CFL bound (or non-finite input) shows as
      // non-finite filtered columns
      int32_t* bad = p->flags + 49;
      int32_t hb = 0;
      KF_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
      for (int c = 0; c < cur; ++c) KF_TRY(nonfinite_flag(n, Q + (int64_t)c * ld, bad, st));
      KF_HIP(hipEventRecord(p->sev[1], st));
      KF_HIP(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      KF_HIP(hipStreamSynchronize(st));
      if (hb) return fail(KF_EUNSTABLE, "kf: filtered subspace not finite (tau too large for the spectrum?)");
    }
    stats.lf_steps += (int64_t)cur * ((int64_t)p->w.size() - 1);
    KF_TRY(lap(p->sev[0], p->sev[1], stats.t_lf));
    ++stats.iters;
    int r = 0, r2 = 0;
    KF_TRY(eig_orthonormalise(p, Q, cur, X, &r));
    if (r > 0) KF_TRY(eig_orthonormalise(p, X, r, Q, &r2));
    KF_HIP(hipEventRecord(p->sev[2], st));
    KF_TRY(lap(p->sev[1], p->sev[2], stats.t_orth));
    if (r2 == 0) {
      cur = 0;
      break;
    }
    std::swap(X, Q);  // X: the M-orthonormal block; Q: work space
    cur = r2;
    // projected pencil X^T S X, S X into Q
    for (int c0 = 0; c0 < cur; c0 += 16) {
      const int nb = std::min(16, cur - c0);
      KF_TRY(spmv_cols(p->S, X + (int64_t)c0 * ld, ld, Q + (int64_t)c0 * ld, ld, nb, nullptr, st));
    }
    for (int c0 = 0; c0 < cur; c0 += 32) {
      const int nb = std::min(32, cur - c0);
      KF_TRY(gemv_t(n, cur, X, ld, Q + (int64_t)c0 * ld, nb, ld, nullptr, 0, 0, nullptr, p->Gm + (int64_t)c0 * cur,
                    cur, p->gw, st));
    }
    KF_TRY(symmetrize(cur, p->Gm, cur, st));
    std::vector<double> th, sel;
    KF_TRY(small_eigen(
        p, cur, p->Gm, cur, th,
        [&](double t) {
          const double om = std::sqrt(std::max(t, 0.0));
          return om >= lo && om <= hi;
        },
        sel));
    KF_TRY(ritz_residuals(p, X, ld, cur, sel, tol, want_vectors, out, true));
    out.ritz = th;
    KF_HIP(hipEventRecord(p->sev[3], st));
    KF_TRY(lap(p->sev[2], p->sev[3], stats.t_rr));
    int inside = 0;
    bool all = true;
    for (size_t q = 0; q < out.cand_theta.size(); ++q) {
      const double t = out.cand_theta[q];
      if (t >= lo2 && t <= hi2) {
        ++inside;
        if (!(out.cand_res[q] <= tol)) all = false;
      }
    }
    const int cnt = distinct_count(out.acc_theta, cnt_b);
    if (target > 0 && cnt >= target) break;
    if (target <= 0 && inside > 0 && all && inside == prev_inside) break;
    prev_inside = inside;
    // stall_limit > 0: stop once the accepted count has not grown for that
    // many iterations
    if (cnt > best) {
      best = cnt;
      stalled = 0;
    } else if (stall_limit > 0 && ++stalled >= stall_limit) {
      break;
    }
  }
  stats.dim = cur;
  return KF_OK;
}

// The subspace iteration with locking (the mixed-precision refinement): Ritz
// pairs accepted at tol (inside the interval) are kept in the space but no
// longer filtered; every other Ritz vector of the space stays active, so the
// dimension is kept.  X holds [locked | active] (nl + na columns, leading
// dimension ldb) on entry (nl = 0) and between iterations.  One iteration:
//   Q = [locked | C active], the filtered part made M-orthogonal to the
//   locked columns (classical Gram-Schmidt twice) and M-orthonormalised;
//   Rayleigh-Ritz on span(Q) (all Ritz vectors), residuals for the Ritz
//   values in the interval widened by `margin`;
//   X = [accepted Ritz vectors | all other Ritz vectors].
int subspace_iterate_locked(kf_problem* p, const SellOp& A, StepBufs& sb, int nc, int max_iters, double tol,
                            int target, int cnt_b, double margin, bool want_vectors, CheckOut& out,
                            SubspaceStats& stats, int stall_limit) {
  hipStream_t st = p->st;
  const int n = p->n;
  const int64_t ld = p->ldb;
  double* X = p->Vx;
  double* Q = p->Yy;
  const double lo = std::max(p->omega_min - margin, 0.0), hi = p->omega_max + margin;
  const double lo2 = p->omega_min * p->omega_min, hi2 = p->omega_max * p->omega_max;
  int nl = 0, na = nc, best = -1, stalled = 0;
  auto lap = [&](hipEvent_t a, hipEvent_t b, double& acc) -> int {
    KF_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    KF_HIP(hipEventElapsedTime(&ms, a, b));
    acc += 1e-3 * ms;
    return KF_OK;
  };
  for (int it = 0; it < max_iters && na > 0; ++it) {
    KF_HIP(hipEventRecord(p->sev[0], st));
    for (int c0 = 0; c0 < na; c0 += 16) {
      const int nb = std::min(16, na - c0);
      KF_TRY(run_filter(p, A, sb, X + (int64_t)(nl + c0) * ld, 1, ld, nb, pow2ceil(nb), Q + (int64_t)(nl + c0) * ld, 1,
                        ld, nb, p->w));
    }
    KF_HIP(hipEventRecord(p->sev[1], st));
    stats.lf_steps += (int64_t)na * ((int64_t)p->w.size() - 1);
    KF_TRY(lap(p->sev[0], p->sev[1], stats.t_lf));
    ++stats.iters;
    if (nl > 0) {
      KF_TRY(copy_cols(n, X, ld, Q, ld, nl, st));
      // the filtered columns against the locked ones, twice
      for (int pass = 0; pass < 2; ++pass)
        for (int c0 = 0; c0 < na; c0 += 32) {
          const int nb = std::min(32, na - c0);
          double* Qc = Q + (int64_t)(nl + c0) * ld;
          KF_TRY(gemv_t(n, nl, Q, ld, nullptr, 0, 0, Qc, nb, ld, p->d_m, p->Ysel, nl, p->gw, st));
          KF_TRY(gemv_n_sub(n, nl, Q, ld, p->Ysel, nl, Qc, ld, nb, st));
        }
    }
    int r = 0, r2 = 0;
    KF_TRY(eig_orthonormalise(p, Q + (int64_t)nl * ld, na, X + (int64_t)nl * ld, &r));
    if (r > 0) KF_TRY(eig_orthonormalise(p, X + (int64_t)nl * ld, r, Q + (int64_t)nl * ld, &r2));
    KF_HIP(hipEventRecord(p->sev[2], st));
    KF_TRY(lap(p->sev[1], p->sev[2], stats.t_orth));
    const int k = nl + r2;
    if (k == 0) break;
    // projected pencil on span(Q): S Q into X, H = Q^T S Q
    for (int c0 = 0; c0 < k; c0 += 16) {
      const int nb = std::min(16, k - c0);
      KF_TRY(spmv_cols(p->S, Q + (int64_t)c0 * ld, ld, X + (int64_t)c0 * ld, ld, nb, nullptr, st));
    }
    for (int c0 = 0; c0 < k; c0 += 32) {
      const int nb = std::min(32, k - c0);
      KF_TRY(gemv_t(n, k, Q, ld, X + (int64_t)c0 * ld, nb, ld, nullptr, 0, 0, nullptr, p->Gm + (int64_t)c0 * k, k,
                    p->gw, st));
    }
    KF_TRY(symmetrize(k, p->Gm, k, st));
    std::vector<double> th, all;
    KF_TRY(small_eigen(p, k, p->Gm, k, th, [](double) { return true; }, all));
    // the Ritz values in the widened interval form a contiguous range
    int i0 = 0, i1 = 0;
    while (i0 < k && std::sqrt(std::max(th[(size_t)i0], 0.0)) < lo) ++i0;
    i1 = i0;
    while (i1 < k && std::sqrt(std::max(th[(size_t)i1], 0.0)) <= hi) ++i1;
    std::vector<double> sel(th.begin() + i0, th.begin() + i1);
    KF_TRY(ritz_residuals(p, Q, ld, k, sel, tol, want_vectors, out, true, p->ew.Y + (int64_t)i0 * k));
    out.ritz = th;
    KF_HIP(hipEventRecord(p->sev[3], st));
    KF_TRY(lap(p->sev[2], p->sev[3], stats.t_rr));
    const int cnt = distinct_count(out.acc_theta, cnt_b);
    if (target > 0 && cnt >= target) break;
    if (cnt > best) {
      best = cnt;
      stalled = 0;
    } else if (stall_limit > 0 && ++stalled >= stall_limit) {
      break;
    }
    // next block: accepted Ritz vectors first (locked), then all others
    std::vector<char> acc((size_t)k, 0);
    for (int a : out.acc_sel) {
      const double t = out.cand_theta[(size_t)a];
      if (t >= lo2 && t <= hi2) acc[(size_t)(i0 + a)] = 1;
    }
    std::vector<int> order;
    for (int i = 0; i < k; ++i)
      if (acc[(size_t)i]) order.push_back(i);
    const int nl_new = (int)order.size();
    for (int i = 0; i < k; ++i)
      if (!acc[(size_t)i]) order.push_back(i);
    for (int j = 0; j < k; ++j)
      KF_HIP(hipMemcpyAsync(p->Ysel + (int64_t)j * k, p->ew.Y + (int64_t)order[(size_t)j] * k, sizeof(double) * k,
                            hipMemcpyDeviceToDevice, st));
    KF_TRY(gemm_nn(n, k, Q, ld, p->Ysel, k, X, ld, k, st));
    nl = nl_new;
    na = k - nl;
  }
  stats.dim = nl + na;
  return KF_OK;
}

// Mixed-precision refinement: the float64 filtered subspace iteration started
// from the Ritz vectors of the float32 Krylov space whose omega lies in the
// interval widened by the margin.  At most opt.refine iterations; it stops
// once `target` pairs (distinct_count with block width b) are accepted, or
// when two iterations in a row accepted no more pairs (pollution along
// directions with the same filter value as the pairs' own does not decay).
int refine_mixed(kf_problem* p, int k, double tol, const CheckOut& in, bool want_vectors, CheckOut& out,
                 int64_t* lf_steps, int target = 0, int b = 1, double margin = 0.0) {
  hipStream_t st = p->st;
  const int n = p->n;
  const int64_t ld = p->ldb;
  const int nc = (int)in.cand_theta.size();
  out = in;
  if (nc == 0 || !p->A64.val) return KF_OK;
  if (nc > 2048) return fail(KF_EINVAL, "kf_solve: refinement block larger than 2048 columns");
  KF_TRY(ensure_refine(p, nc, k));
  // X = B * (eigenvectors of the last check's candidates, ew.Y), into Vx
  KF_TRY(gemm_nn(n, k, p->B, p->ldb, p->ew.Y, k, p->Vx, ld, nc, st));
  SubspaceStats stats;
  KF_TRY(subspace_iterate_locked(p, p->A64, p->sb64, nc, std::max(1, p->opt.refine), tol, target, b, margin,
                                 want_vectors, out, stats, 2));
  *lf_steps += stats.lf_steps;
  out.ritz = in.ritz;
  out.orth = in.orth;
  return KF_OK;
}

// Pairs that count towards the target: accepted values within 1e-8
// (relative) of each other form one eigenvalue, which counts at most b times
// (a block of b start vectors sees at most b directions of an eigenspace).
int distinct_count(const std::vector<double>& acc, int b) {
  int cnt = 0;
  size_t i = 0;
  while (i < acc.size()) {
    size_t j = i + 1;
    while (j < acc.size() && acc[j] - acc[j - 1] <= 1e-8 * std::fabs(acc[j])) ++j;
    cnt += (int)std::min<size_t>(j - i, (size_t)b);
    i = j;
  }
  return cnt;
}

// More than b accepted Ritz values within 1e-8 of each other (ascending acc):
// a block of b start vectors reaches at most b directions of an eigenspace in
// exact arithmetic, so the extra copies were seeded by round-off.
bool copies_beyond_block(const std::vector<double>& acc, int b) {
  size_t i = 0;
  while (i < acc.size()) {
    size_t j = i + 1;
    while (j < acc.size() && acc[j] - acc[j - 1] <= 1e-8 * std::fabs(acc[j])) ++j;
    if (j - i > (size_t)b) return true;
    i = j;
  }
  return false;
}

// Time `reps` fused steps of operator A for a block of bk vectors with the
// given XCD mapping; returns microseconds per step.
int time_variant(kf_problem* p, const SellOp& A, StepBufs& sb, int remap, int reps, double* us, int bk = 1) {
  hipStream_t st = p->st;
  KF_TRY(ensure_step_buffers(p, sb, bk, A.val_bytes));
  const size_t bytes = (size_t)p->n * bk * A.val_bytes;
  KF_HIP(hipMemsetAsync(sb.Y0, 0, bytes, st));
  KF_HIP(hipMemsetAsync(sb.Y1, 0, bytes, st));
  KF_HIP(hipMemsetAsync(sb.R, 0, bytes, st));
  for (int w = 0; w < 3; ++w)
    KF_TRY(launch_leapfrog(A, bk, kMid, sb.Y1, sb.Y0, sb.Y0, sb.R, nullptr, 0, 0, 0, 0.0, 0.0, 0.0, remap, st));
  KF_HIP(hipEventRecord(p->ev[0], st));
  // the mix of a filter application: the weighted sum is updated every third step
  for (int r = 0; r < reps; ++r) {
    void* a = (r & 1) ? sb.Y0 : sb.Y1;
    void* b = (r & 1) ? sb.Y1 : sb.Y0;
    KF_TRY(launch_leapfrog(A, bk, r % 3 == 2 ? kMidAcc : kMid, a, b, b, sb.R, nullptr, 0, 0, 0, 0.0, 0.0, 0.0, remap,
                           st));
  }
  KF_HIP(hipEventRecord(p->ev[1], st));
  KF_HIP(hipEventSynchronize(p->ev[1]));
  float ms = 0.f;
  KF_HIP(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
  *us = 1e3 * ms / reps;
  return KF_OK;
}

// The fastest of three timings of a variant: one timing can be thrown off by
// other work on the GPU (a profiler, another process), and a wrong choice of
// index width or lanes per row costs up to a quarter of every later step.
int time_variant_min(kf_problem* p, const SellOp& A, StepBufs& sb, int remap, int reps, double* us, int bk = 1) {
  double best = 1e300;
  for (int t = 0; t < 3; ++t) {
    double u = 0.0;
    KF_TRY(time_variant(p, A, sb, remap, reps, &u, bk));
    best = std::min(best, u);
  }
  *us = best;
  return KF_OK;
}

// Block widths above 1: the lanes sharing a row (1, 2 or 4) are timed on
// the problem's operator the first time a width is used (autotune on).
// Called outside the timed regions of a solve (it records ev[0], ev[1]).
int tune_block(kf_problem* p, SellOp& A, StepBufs& sb, int bk) {
  if (!p->opt.autotune || bk < 2) return KF_OK;
  int lb = 0;
  while ((1 << lb) < bk && lb < 4) ++lb;
  if (A.lpr_tuned & (1 << lb)) return KF_OK;
  double best = 1e300;
  int best_l = 1, best_b = 0;
  // lanes per row, each with the gathers from the caches and (unless the
  // caller fixed it, and where the band copy fits) from LDS
  const bool try_band = p->opt.block_band == 0;
  for (int l = 1; l <= std::min(bk, 4); l *= 2) {
    for (int band = 0; band <= 1; ++band) {
      if (band && (!try_band || band_lds_bytes(A, bk, l) > kBandLdsBytes)) continue;
      A.lpr[lb] = l;
      A.band[lb] = try_band ? band : A.band[lb];
      double us = 0.0;
      KF_TRY(time_variant_min(p, A, sb, p->opt.xcd_remap, 10, &us, bk));
      if (us < best) {
        best = us;
        best_l = l;
        best_b = A.band[lb];
      }
    }
  }
  A.lpr[lb] = best_l;
  A.band[lb] = best_b;
  A.lpr_tuned |= 1 << lb;
  return KF_OK;
}

// The autotuner: every combination of XCD mapping, non-temporal loads and
// index width (2 and 4 bytes when 2 fits) of the fused step, timed on this
// operator; the fastest is kept.
int autotune(kf_problem* p, DevCsr& dc, const double* d_scale) {
  SellOp alt;
  const bool try_alt = p->A.idx_bytes == 2;
  if (try_alt) {
    KF_TRY(build_sell(p->n, p->nnz, dc.rowptr, dc.col, dc.val, d_scale, p->A.val_bytes, 4, p->st, alt));
    // the alternative is timed, and kept, with the caller's fixed choices
    // (unroll factor, lanes per row, band copy)
    alt.unroll = p->A.unroll;
    for (int l = 0; l < 5; ++l) {
      alt.lpr[l] = p->A.lpr[l];
      alt.band[l] = p->A.band[l];
    }
  }
  double best = 1e300;
  int best_remap = p->opt.xcd_remap, best_nt = p->A.nt_loads, best_alt = 0;
  for (int use_alt = 0; use_alt <= (try_alt ? 1 : 0); ++use_alt) {
    SellOp& A = use_alt ? alt : p->A;
    for (int nt = 0; nt <= 1; ++nt) {
      for (int remap = 0; remap <= 1; ++remap) {
        A.nt_loads = nt;
        double us = 0;
        int rc = time_variant_min(p, A, p->sb, remap, 20, &us);
        if (rc) {
          free_sell(alt);
          return rc;
        }
        if (us < best) {
          best = us;
          best_remap = remap;
          best_nt = nt;
          best_alt = use_alt;
        }
      }
    }
  }
  if (best_alt) {
    std::swap(p->A, alt);
  }
  free_sell(alt);
  p->A.nt_loads = best_nt;
  p->A64.nt_loads = best_nt;
  p->opt.xcd_remap = best_remap;
  // then the unroll factor of the single-vector step's loop over a slice's
  // entries (unless the caller fixed it); the float64 copy of the operator
  // used by the refinement has the same slices and takes the same factor
  if (p->opt.gather_unroll == 0) {
    int best_u = 4;
    for (int u : {2, 3, 4, 6}) {
      p->A.unroll = u;
      double us = 0;
      KF_TRY(time_variant_min(p, p->A, p->sb, best_remap, 20, &us));
      if (us < best) {
        best = us;
        best_u = u;
      }
    }
    p->A.unroll = p->A64.unroll = best_u;
  }
  p->tuned_us = best;
  return KF_OK;
}

void free_problem(kf_problem* p) {
  if (!p) return;
  free_sell(p->A);
  free_sell(p->A64);
  free_sell(p->S);
  void* ptrs[] = {p->d_m, p->B,  p->H,  p->G,  p->T,  p->W,    p->V,      p->SV,
                  p->small, p->flags, p->Vx, p->Yy, p->Ysel, p->Gm, p->rr_work, p->d_w};
  for (void* q : ptrs) dfree(q);
  free_step_buffers(p->sb);
  free_step_buffers(p->sb64);
  if (p->gw.partial) (void)hipFree(p->gw.partial);
  if (p->rw.partial) (void)hipFree(p->rw.partial);
  free_eig(p->ew);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->sev)
    if (e) (void)hipEventDestroy(e);
  if (p->sync_ev) (void)hipEventDestroy(p->sync_ev);
  if (p->own_stream && p->st) {
    (void)hipStreamSynchronize(p->st);
    (void)hipStreamDestroy(p->st);
  }
  if (p->pin) (void)hipHostFree(p->pin);
  delete p;
}

}  // namespace

extern "C" {

void kf_default_options(kf_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = KF_FP64;
  o->check_every = 1;
  o->check_growth = 0.3;
  o->full_reorth = 0;
  o->target = 0;
  o->max_iters = 0;
  o->drop_tol = 1e-10;
  o->reorth_tol = 1e-9;
  o->proj_every = 12;
  o->refine = 8;
  o->escalate = 1;
  o->stepper = 2;
  o->want_vectors = 0;
  o->index_bytes = 0;
  o->xcd_remap = 1;
  o->nt_loads = 0;
  o->autotune = 0;
  o->lanes_per_row = 0;
  o->gather_unroll = 0;
  o->block_band = 0;
  o->batch_workers = 0;
  o->overlap_checks = 1;
  o->multistep = 0;
  o->stream = nullptr;
}

const char* kf_last_error(void) { return g_err.c_str(); }

int kf_time_step_rule(double lambda_est, double omega_min, double safety, double* tau, int32_t* L) {
  if (!tau || !L) return fail(KF_EINVAL, "kf_time_step_rule: NULL output");
  if (!(lambda_est > 0) || !std::isfinite(lambda_est)) return fail(KF_EINVAL, "kf_time_step_rule: lambda_est must be > 0");
  if (!(omega_min > 0) || !std::isfinite(omega_min)) return fail(KF_EINVAL, "kf_time_step_rule: omega_min must be > 0");
  if (!(safety > 0 && safety < 1)) return fail(KF_EINVAL, "kf_time_step_rule: safety must lie in (0, 1)");
  const double t = safety * 2.0 / std::sqrt(lambda_est);
  const double pi = 3.14159265358979323846;
  const double Ld = std::ceil(2.0 * pi / (omega_min * t));
  if (Ld > 1e9) return fail(KF_EINVAL, "kf_time_step_rule: step count overflows");
  *tau = t;
  *L = (int32_t)Ld;
  return KF_OK;
}

int kf_create(const kf_csr* S, const double* m_diag, double omega_min, double omega_max, double tau, int32_t L,
              const kf_options* opt, kf_problem** out) {
  if (!out) return fail(KF_EINVAL, "kf_create: NULL output handle");
  *out = nullptr;
  if (!(omega_min >= 0) || !(omega_max > omega_min) || !std::isfinite(omega_max))
    return fail(KF_EINVAL, "kf_create: need 0 <= omega_min < omega_max (finite)");
  if (!(tau > 0) || !std::isfinite(tau)) return fail(KF_EINVAL, "kf_create: tau must be positive and finite");
  if (L < 1) return fail(KF_EINVAL, "kf_create: L must be >= 1");
  kf_options o;
  kf_default_options(&o);
  if (opt) o = *opt;
  if (o.precision != KF_FP64 && o.precision != KF_MIXED) return fail(KF_EINVAL, "kf_create: unknown precision");
  if (o.index_bytes != 0 && o.index_bytes != 2 && o.index_bytes != 4)
    return fail(KF_EINVAL, "kf_create: index_bytes must be 0, 2 or 4");
  if (o.check_every < 1) o.check_every = 1;
  if (!(o.check_growth >= 0.0) || !std::isfinite(o.check_growth)) o.check_growth = 0.0;
  if (!(o.drop_tol > 0)) o.drop_tol = 1e-10;
  if (!(o.reorth_tol >= 0.0) || !std::isfinite(o.reorth_tol))
    return fail(KF_EINVAL, "kf_create: reorth_tol must be finite and >= 0");
  if (o.batch_workers < 0) return fail(KF_EINVAL, "kf_create: batch_workers must be >= 0");
  if (o.proj_every < 1) o.proj_every = 1;
  if (o.lanes_per_row != 0 && o.lanes_per_row != 1 && o.lanes_per_row != 2 && o.lanes_per_row != 4)
    return fail(KF_EINVAL, "kf_create: lanes_per_row must be 0, 1, 2 or 4");
  if (o.gather_unroll != 0 && o.gather_unroll != 2 && o.gather_unroll != 3 && o.gather_unroll != 4 &&
      o.gather_unroll != 6)
    return fail(KF_EINVAL, "kf_create: gather_unroll must be 0, 2, 3, 4 or 6");
  if (o.block_band < -1 || o.block_band > 1) return fail(KF_EINVAL, "kf_create: block_band must be -1, 0 or 1");
  if (o.stepper == 0) o.stepper = 2;
  if (o.stepper != 2 && o.stepper != 4) return fail(KF_EINVAL, "kf_create: stepper must be 2 or 4");
  if (o.multistep < -1) return fail(KF_EINVAL, "kf_create: multistep must be -1, 0 or a step count");
  if (o.multistep != 0 && o.stepper == 4)
    return fail(KF_EINVAL, "kf_create: several steps per launch need the second-order scheme (stepper 2)");
  HostCsr h;
  KF_TRY(fetch_csr(S, m_diag, h));

  kf_problem* p = new (std::nothrow) kf_problem();
  if (!p) return fail(KF_ENOMEM, "kf_create: host allocation failed");
  p->n = S->n;
  p->nnz = S->nnz;
  p->omega_min = omega_min;
  p->omega_max = omega_max;
  p->tau = tau;
  p->L = L;
  p->opt = o;
  p->st = (hipStream_t)o.stream;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(KF_EHIP, "kf_create: no current device");
  }
  p->w = fourier_weights(omega_min, omega_max, tau, L);
  int rc = KF_OK;
  do {
    DevCsr dc;
    rc = upload_csr(h, p->n, p->nnz, p->st, dc);
    if (rc) break;
    rc = dalloc(&p->d_m, (size_t)p->n);
    if (rc) break;
    if (hipMemcpy(p->d_m, h.m.data(), sizeof(double) * p->n, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(KF_EHIP, "kf_create: copy of m_diag failed");
      break;
    }
    std::vector<double> scale((size_t)p->n);
    for (int32_t i = 0; i < p->n; ++i) scale[(size_t)i] = tau * tau / h.m[(size_t)i];
    double* d_scale = nullptr;
    rc = dalloc(&d_scale, (size_t)p->n);
    if (rc) break;
    if (hipMemcpy(d_scale, scale.data(), sizeof(double) * p->n, hipMemcpyHostToDevice) != hipSuccess) {
      dfree(d_scale);
      rc = fail(KF_EHIP, "kf_create: copy of the row scaling failed");
      break;
    }
    const int vb = o.precision == KF_MIXED ? 4 : 8;
    rc = build_sell(p->n, p->nnz, dc.rowptr, dc.col, dc.val, d_scale, vb, o.index_bytes, p->st, p->A);
    if (!rc && o.precision == KF_MIXED && o.refine)
      rc = build_sell(p->n, p->nnz, dc.rowptr, dc.col, dc.val, d_scale, 8, o.index_bytes, p->st, p->A64);
    if (!rc) rc = build_sell(p->n, p->nnz, dc.rowptr, dc.col, dc.val, nullptr, 8, o.index_bytes, p->st, p->S);
    if (rc) {
      dfree(d_scale);
      break;
    }
    p->A.nt_loads = o.nt_loads ? 1 : 0;
    p->A64.nt_loads = p->A.nt_loads;
    p->A.unroll = p->A64.unroll = o.gather_unroll;
    for (int l = 0; l < 5; ++l) p->A.band[l] = p->A64.band[l] = o.block_band == 1 ? 1 : 0;
    for (hipEvent_t& e : p->ev)
      if (!rc && hipEventCreate(&e) != hipSuccess) rc = fail(KF_EHIP, "kf_create: event creation failed");
    for (hipEvent_t& e : p->sev)
      if (!rc && hipEventCreate(&e) != hipSuccess) rc = fail(KF_EHIP, "kf_create: event creation failed");
    if (!rc && o.autotune) rc = autotune(p, dc, d_scale);
    for (int l = 0; l < 5; ++l) p->A.lpr[l] = p->A64.lpr[l] = o.lanes_per_row;
    dfree(d_scale);
    if (rc) break;
  } while (false);
  if (rc) {
    free_problem(p);
    return rc;
  }
  *out = p;
  return KF_OK;
}

int kf_sym_eig(int32_t k, const double* A, double lo, double hi, double* theta, int32_t* n_sel, double* Y,
               void* stream) {
  if (k < 1 || k > 2048) return fail(KF_EINVAL, "kf_sym_eig: k must be in [1, 2048]");
  if (!A || !theta) return fail(KF_EINVAL, "kf_sym_eig: NULL argument");
  if (Y && !n_sel) return fail(KF_EINVAL, "kf_sym_eig: n_sel is needed with Y");
  for (int64_t i = 0; i < (int64_t)k * k; ++i)
    if (!std::isfinite(A[i])) return fail(KF_EINVAL, "kf_sym_eig: non-finite entry");
  hipStream_t st = static_cast<hipStream_t>(stream);
  EigWork ew;
  double* dA = nullptr;
  int rc = KF_OK;
  do {
    if ((rc = dalloc(&dA, (size_t)k * k))) break;
    if (hipMemcpyAsync(dA, A, sizeof(double) * k * k, hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = fail(KF_EHIP, "kf_sym_eig: copy failed");
      break;
    }
    if ((rc = symmetrize(k, dA, k, st))) break;
    std::vector<double> th, sel;
    auto keep = [&](double t) { return Y != nullptr && t >= lo && t <= hi; };
    if ((rc = eig_select(ew, k, dA, k, th, keep, sel, st))) break;
    std::copy(th.begin(), th.end(), theta);
    if (Y) {
      *n_sel = (int32_t)sel.size();
      if (!sel.empty() && hipMemcpyAsync(Y, ew.Y, sizeof(double) * k * sel.size(), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = fail(KF_EHIP, "kf_sym_eig: copy failed");
      if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(KF_EHIP, "kf_sym_eig: synchronisation failed");
    }
  } while (false);
  dfree(dA);
  free_eig(ew);
  return rc;
}

int kf_get_tuning(const kf_problem* p, int32_t* xcd_remap, int32_t* nt_loads, int32_t* index_bytes,
                  int32_t* gather_unroll, double* us_per_step) {
  if (!p) return fail(KF_EINVAL, "kf_get_tuning: NULL handle");
  if (xcd_remap) *xcd_remap = p->opt.xcd_remap;
  if (nt_loads) *nt_loads = p->A.nt_loads;
  if (index_bytes) *index_bytes = p->A.idx_bytes;
  if (gather_unroll) *gather_unroll = p->A.unroll ? p->A.unroll : 4;
  if (us_per_step) *us_per_step = p->tuned_us;
  return KF_OK;
}

int kf_destroy(kf_problem* p) {
  if (!p) return KF_OK;
  async_free(p);
  (void)hipStreamSynchronize(p->st);
  free_problem(p);
  return KF_OK;
}

int kf_set_weights(kf_problem* p, const double* w, int32_t L) {
  if (!p || !w) return fail(KF_EINVAL, "kf_set_weights: NULL argument");
  if (L != p->L) return fail(KF_EINVAL, "kf_set_weights: expected exactly L coefficients");
  for (int32_t l = 0; l < L; ++l)
    if (!std::isfinite(w[l])) return fail(KF_EINVAL, "kf_set_weights: non-finite coefficient");
  p->w.assign(w, w + L);
  return KF_OK;
}

int kf_get_weights(const kf_problem* p, double* w_out) {
  if (!p || !w_out) return fail(KF_EINVAL, "kf_get_weights: NULL argument");
  std::memcpy(w_out, p->w.data(), sizeof(double) * p->w.size());
  return KF_OK;
}

int kf_window_weights(int32_t kind, double omega_min, double omega_max, double tau, int32_t L, double width,
                      double* w_out) {
  if (!w_out) return fail(KF_EINVAL, "kf_window_weights: NULL output");
  if (!(omega_min >= 0) || !(omega_max > omega_min) || !std::isfinite(omega_max))
    return fail(KF_EINVAL, "kf_window_weights: need 0 <= omega_min < omega_max (finite)");
  if (!(tau > 0) || !std::isfinite(tau) || L < 1) return fail(KF_EINVAL, "kf_window_weights: need tau > 0, L >= 1");
  if (kind != KF_WINDOW_INDICATOR && !(width > 0 && std::isfinite(width)))
    return fail(KF_EINVAL, "kf_window_weights: width must be positive");
  const double pi = 3.14159265358979323846;
  const double c = 0.5 * (omega_min + omega_max), d = 0.5 * (omega_max - omega_min);
  for (int32_t l = 0; l < L; ++l) {
    const double t = l * tau;
    double a = 0.0;
    switch (kind) {
      case KF_WINDOW_INDICATOR:
        // eq. weightf
        a = l == 0 ? 2.0 * (omega_max - omega_min) / pi
                   : 4.0 / (pi * t) * std::sin(0.5 * t * (omega_max - omega_min)) * std::cos(0.5 * t * (omega_max + omega_min));
        break;
      case KF_WINDOW_TRIANGLE: {
        // transform of max(0, 1 - |omega - c| / h) (+ its mirror image)
        const double h = width * d;
        const double x = 0.5 * h * t;
        const double sn = x == 0.0 ? 1.0 : std::sin(x) / x;
        a = 2.0 / pi * h * std::cos(c * t) * sn * sn;
        break;
      }
      case KF_WINDOW_GAUSSIAN: {
        // transform of exp(-(omega - c)^2 / (2 sigma^2)) (+ its mirror image)
        const double sigma = width * d / std::sqrt(2.0 * std::log(2.0));
        a = 2.0 / pi * sigma * std::sqrt(2.0 * pi) * std::exp(-0.5 * sigma * sigma * t * t) * std::cos(c * t);
        break;
      }
      default:
        return fail(KF_EINVAL, "kf_window_weights: unknown kind");
    }
    w_out[l] = tau * a;
  }
  return KF_OK;
}

int kf_notch_weights(const double* w, int32_t L, double tau, const double* omega, int32_t k, double* w_out) {
  if (!w || !w_out || (k > 0 && !omega)) return fail(KF_EINVAL, "kf_notch_weights: NULL argument");
  if (L < 1 || k < 0 || k > 64 || k > L) return fail(KF_EINVAL, "kf_notch_weights: need L >= 1 and 0 <= k <= min(64, L)");
  if (!(tau > 0) || !std::isfinite(tau)) return fail(KF_EINVAL, "kf_notch_weights: tau must be positive");
  for (int32_t l = 0; l < L; ++l)
    if (!std::isfinite(w[l])) return fail(KF_EINVAL, "kf_notch_weights: non-finite weight");
  // Q[j][l] = q_l(omega_j) by the scalar recurrence (Section 2.3), so that
  // beta~(omega_j) = (Q w)_j (Lemma 2.3)
  std::vector<double> Q((size_t)k * L);
  for (int32_t j = 0; j < k; ++j) {
    if (!std::isfinite(omega[j])) return fail(KF_EINVAL, "kf_notch_weights: non-finite frequency");
    const double f = 2.0 - tau * tau * omega[j] * omega[j];
    double qm = 1.0, q = 1.0;
    for (int32_t l = 0; l < L; ++l) {
      Q[(size_t)j * L + l] = q;
      const double qn = f * q - qm;
      qm = q;
      q = qn;
    }
  }
  // w_out = w - Q^T (Q Q^T)^{-1} Q w: the nearest weights (2-norm) with
  // beta~(omega_j) = 0; Q Q^T solved by Cholesky
  std::vector<double> G((size_t)k * k), r((size_t)k);
  for (int32_t i = 0; i < k; ++i) {
    double acc = 0.0;
    for (int32_t l = 0; l < L; ++l) acc += Q[(size_t)i * L + l] * w[l];
    r[(size_t)i] = acc;
    for (int32_t j = 0; j <= i; ++j) {
      double g = 0.0;
      for (int32_t l = 0; l < L; ++l) g += Q[(size_t)i * L + l] * Q[(size_t)j * L + l];
      G[(size_t)i * k + j] = G[(size_t)j * k + i] = g;
    }
  }
  for (int32_t j = 0; j < k; ++j) {
    double dj = G[(size_t)j * k + j];
    for (int32_t q = 0; q < j; ++q) dj -= G[(size_t)j * k + q] * G[(size_t)j * k + q];
    if (!(dj > 1e-13 * G[(size_t)j * k + j]))
      return fail(KF_EINVAL, "kf_notch_weights: the notch constraints are (nearly) dependent");
    dj = std::sqrt(dj);
    G[(size_t)j * k + j] = dj;
    for (int32_t i = j + 1; i < k; ++i) {
      double v = G[(size_t)i * k + j];
      for (int32_t q = 0; q < j; ++q) v -= G[(size_t)i * k + q] * G[(size_t)j * k + q];
      G[(size_t)i * k + j] = v / dj;
    }
  }
  for (int32_t i = 0; i < k; ++i) {  // forward: L y = r
    double v = r[(size_t)i];
    for (int32_t q = 0; q < i; ++q) v -= G[(size_t)i * k + q] * r[(size_t)q];
    r[(size_t)i] = v / G[(size_t)i * k + i];
  }
  for (int32_t i = k - 1; i >= 0; --i) {  // backward: L^T c = y
    double v = r[(size_t)i];
    for (int32_t q = i + 1; q < k; ++q) v -= G[(size_t)q * k + i] * r[(size_t)q];
    r[(size_t)i] = v / G[(size_t)i * k + i];
  }
  for (int32_t l = 0; l < L; ++l) {
    double v = w[l];
    for (int32_t j = 0; j < k; ++j) v -= Q[(size_t)j * L + l] * r[(size_t)j];
    w_out[l] = v;
  }
  return KF_OK;
}

namespace {

// beta~(omega_j) for the weights w[L] (scalar recurrence of the stepper)
void filter_values(const double* w, int L, double tau, int stepper, const double* omega, int M, double* beta) {
  for (int j = 0; j < M; ++j) {
    const double x = tau * tau * omega[j] * omega[j];
    const double f = 2.0 - x + (stepper == 4 ? x * x / 12.0 : 0.0);
    double qm = 1.0, q = 1.0, acc = 0.0;
    for (int l = 0; l < L; ++l) {
      acc += w[l] * q;
      const double qn = f * q - qm;
      qm = q;
      q = qn;
    }
    beta[j] = acc;
  }
}

// The Krylov iteration of D = diag(beta) from the start vector sqrt(weight)
// (Gram-Schmidt twice); the first dimension at which every sought point j
// has 1 - |Q[j, :]|^2 <= eps^2, or kmax.
int krylov_model_steps(const std::vector<double>& beta, const double* weight, const std::vector<char>& inside, int M,
                       double eps, int kmax) {
  bool any = false;
  for (int j = 0; j < M; ++j) any = any || inside[(size_t)j];
  if (!any) return 0;
  std::vector<double> Q((size_t)M * std::max(kmax, 1)), x((size_t)M), cap((size_t)M), h((size_t)kmax);
  double nv = 0.0;
  for (int j = 0; j < M; ++j) nv += weight[j];
  nv = std::sqrt(nv);
  for (int j = 0; j < M; ++j) {
    Q[(size_t)j] = std::sqrt(weight[j]) / nv;
    cap[(size_t)j] = Q[(size_t)j] * Q[(size_t)j];
  }
  const double e2 = eps * eps;
  auto resolved = [&]() {
    for (int j = 0; j < M; ++j)
      if (inside[(size_t)j] && 1.0 - cap[(size_t)j] > e2) return false;
    return true;
  };
  for (int k = 1; k < kmax; ++k) {
    const double* qp = &Q[(size_t)(k - 1) * M];
    for (int j = 0; j < M; ++j) x[(size_t)j] = beta[(size_t)j] * qp[j];
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < k; ++i) {
        const double* qi = &Q[(size_t)i * M];
        double c = 0.0;
        for (int j = 0; j < M; ++j) c += qi[j] * x[(size_t)j];
        h[(size_t)i] = c;
      }
      for (int i = 0; i < k; ++i) {
        const double* qi = &Q[(size_t)i * M];
        const double c = h[(size_t)i];
        for (int j = 0; j < M; ++j) x[(size_t)j] -= c * qi[j];
      }
    }
    double nx = 0.0;
    for (int j = 0; j < M; ++j) nx += x[(size_t)j] * x[(size_t)j];
    nx = std::sqrt(nx);
    if (!(nx > 1e-14)) return resolved() ? k : kmax;  // invariant space
    double* qk = &Q[(size_t)k * M];
    for (int j = 0; j < M; ++j) {
      qk[j] = x[(size_t)j] / nx;
      cap[(size_t)j] += qk[j] * qk[j];
    }
    if (resolved()) return k + 1;
  }
  return kmax;
}

}  // namespace

int kf_predict_steps(const double* omega, const double* weight, int32_t M, const double* w, int32_t L, double tau,
                     int32_t stepper, double omega_min, double omega_max, double eps, int32_t kmax, int32_t* steps) {
  if (!omega || !weight || !w || !steps || M < 1 || L < 1 || kmax < 1)
    return fail(KF_EINVAL, "kf_predict_steps: bad arguments");
  if (!(tau > 0) || !(eps > 0) || (stepper != 2 && stepper != 4))
    return fail(KF_EINVAL, "kf_predict_steps: need tau > 0, eps > 0, stepper 2 or 4");
  if ((size_t)M * (size_t)kmax > ((size_t)1 << 31)) return fail(KF_EINVAL, "kf_predict_steps: M x kmax too large");
  for (int32_t j = 0; j < M; ++j)
    if (!(weight[j] > 0) || !std::isfinite(omega[j])) return fail(KF_EINVAL, "kf_predict_steps: bad model point");
  std::vector<double> beta((size_t)M);
  filter_values(w, L, tau, stepper, omega, M, beta.data());
  // The Krylov iteration of a diagonal matrix cannot tell points with equal
  // values apart: the unsought points are merged into kBins classes of
  // nearly equal filter value (weights summed, value the weighted mean);
  // sought points stay apart.
  constexpr int kBins = 2048;
  std::vector<double> bw, bv, bwt;
  std::vector<char> inside;
  double blo = 1e300, bhi = -1e300;
  for (int32_t j = 0; j < M; ++j) {
    const bool in = omega[j] >= omega_min && omega[j] <= omega_max;
    if (in) {
      bv.push_back(beta[(size_t)j]);
      bwt.push_back(weight[j]);
      inside.push_back(1);
    } else {
      blo = std::min(blo, beta[(size_t)j]);
      bhi = std::max(bhi, beta[(size_t)j]);
    }
  }
  if (blo <= bhi) {
    std::vector<double> W((size_t)kBins, 0.0), V((size_t)kBins, 0.0);
    const double width = (bhi - blo) / kBins;
    for (int32_t j = 0; j < M; ++j) {
      if (omega[j] >= omega_min && omega[j] <= omega_max) continue;
      int c = width > 0 ? (int)((beta[(size_t)j] - blo) / width) : 0;
      c = std::min(std::max(c, 0), kBins - 1);
      W[(size_t)c] += weight[j];
      V[(size_t)c] += weight[j] * beta[(size_t)j];
    }
    for (int c = 0; c < kBins; ++c)
      if (W[(size_t)c] > 0) {
        bv.push_back(V[(size_t)c] / W[(size_t)c]);
        bwt.push_back(W[(size_t)c]);
        inside.push_back(0);
      }
  }
  const int Mb = (int)bv.size();
  *steps = krylov_model_steps(bv, bwt.data(), inside, Mb, eps, std::min<int32_t>(kmax, Mb + 1));
  if (*steps == std::min<int32_t>(kmax, Mb + 1) && kmax > Mb + 1) *steps = kmax;
  return KF_OK;
}

int kf_select_weights(const double* const* candidates, int32_t n_cand, int32_t L, double tau, int32_t stepper,
                      double omega_min, double omega_max, const double* omega, const double* weight, int32_t M,
                      double eps, int32_t kmax, double margin, int32_t* chosen, int32_t* steps) {
  if (!candidates || n_cand < 1 || !chosen) return fail(KF_EINVAL, "kf_select_weights: bad arguments");
  if (!(margin >= 0.0) || margin >= 1.0) return fail(KF_EINVAL, "kf_select_weights: margin must lie in [0, 1)");
  std::vector<int32_t> st((size_t)n_cand);
  for (int32_t c = 0; c < n_cand; ++c) {
    if (!candidates[c]) return fail(KF_EINVAL, "kf_select_weights: NULL candidate");
    KF_TRY(kf_predict_steps(omega, weight, M, candidates[c], L, tau, stepper, omega_min, omega_max, eps, kmax,
                            &st[(size_t)c]));
    if (steps) steps[c] = st[(size_t)c];
  }
  // candidate 0 (the Fourier weights) unless another is predicted to need
  // fewer than (1 - margin) of its steps
  int32_t best = 0;
  for (int32_t c = 1; c < n_cand; ++c)
    if (st[(size_t)c] < st[(size_t)best] && st[(size_t)c] < (1.0 - margin) * st[0]) best = c;
  *chosen = best;
  return KF_OK;
}

int kf_filter_response(const kf_problem* p, const double* omega, int32_t n, double* beta_out) {
  if (!p || (n > 0 && (!omega || !beta_out)) || n < 0) return fail(KF_EINVAL, "kf_filter_response: bad arguments");
  // Lemma 2.3: beta~(omega) = sum_l w_l q_l(omega), q by the scalar recurrence
  for (int32_t i = 0; i < n; ++i) {
    const double x = p->tau * p->tau * omega[i] * omega[i];
    const double f = 2.0 - x + (p->opt.stepper == 4 ? x * x / 12.0 : 0.0);
    double qm = 1.0, q = 1.0, s = 0.0;
    for (size_t l = 0; l < p->w.size(); ++l) {
      s += p->w[l] * q;
      const double qn = f * q - qm;
      qm = q;
      q = qn;
    }
    beta_out[i] = s;
  }
  return KF_OK;
}

int kf_estimate_lambda_max(const kf_csr* S, const double* m_diag, int32_t iters, const double* x0, void* stream,
                           double* out) {
  if (!out || !x0) return fail(KF_EINVAL, "kf_estimate_lambda_max: NULL argument");
  if (iters < 0) return fail(KF_EINVAL, "kf_estimate_lambda_max: iters must be >= 0");
  HostCsr h;
  KF_TRY(fetch_csr(S, m_diag, h));
  hipStream_t st = (hipStream_t)stream;
  const int32_t n = S->n;
  DevCsr dc;
  KF_TRY(upload_csr(h, n, S->nnz, st, dc));
  SellOp op;
  double *dm = nullptr, *dminv = nullptr, *x = nullptr, *y = nullptr, *sc = nullptr;
  GemvTWork gw;
  int rc = KF_OK;
  do {
    rc = build_sell(n, S->nnz, dc.rowptr, dc.col, dc.val, nullptr, 8, 0, st, op);
    if (rc) break;
    if ((rc = dalloc(&dm, n)) || (rc = dalloc(&dminv, n)) || (rc = dalloc(&x, n)) || (rc = dalloc(&y, n)) ||
        (rc = dalloc(&sc, 8)))
      break;
    std::vector<double> minv((size_t)n);
    for (int32_t i = 0; i < n; ++i) minv[(size_t)i] = 1.0 / h.m[(size_t)i];
    if (hipMemcpy(dm, h.m.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dminv, minv.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(x, x0, sizeof(double) * n, S->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice) !=
            hipSuccess) {
      rc = fail(KF_EHIP, "kf_estimate_lambda_max: copy failed");
      break;
    }
    // x /= ||x||_M, then iters times x <- M^{-1} S x / ||.||_M
    if ((rc = gemv_t(n, 1, x, n, nullptr, 0, 0, x, 1, n, dm, sc, 1, gw, st))) break;
    if ((rc = normalize_col(n, x, sc, nullptr, 0.0, nullptr, nullptr, st))) break;
    for (int32_t it = 0; it < iters && !rc; ++it) {
      if ((rc = spmv_cols(op, x, n, y, n, 1, dminv, st))) break;
      if ((rc = gemv_t(n, 1, y, n, nullptr, 0, 0, y, 1, n, dm, sc, 1, gw, st))) break;
      if ((rc = normalize_col(n, y, sc, nullptr, 0.0, nullptr, nullptr, st))) break;
      std::swap(x, y);
    }
    if (rc) break;
    // Rayleigh quotient x^T S x / x^T M x
    if ((rc = spmv_cols(op, x, n, y, n, 1, nullptr, st))) break;
    if ((rc = gemv_t(n, 1, x, n, y, 1, n, x, 1, n, dm, sc, 1, gw, st))) break;
    double hs[2] = {0, 0};
    if (hipMemcpyAsync(hs, sc, sizeof(double) * 2, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(KF_EHIP, "kf_estimate_lambda_max: readback failed");
      break;
    }
    if (!(hs[1] > 0) || !std::isfinite(hs[0])) {
      rc = fail(KF_EINVAL, "kf_estimate_lambda_max: start vector vanished or diverged");
      break;
    }
    *out = hs[0] / hs[1];
  } while (false);
  free_sell(op);
  dfree(dm);
  dfree(dminv);
  dfree(x);
  dfree(y);
  dfree(sc);
  if (gw.partial) (void)hipFree(gw.partial);
  return rc;
}

int kf_apply_filter(kf_problem* p, const double* x, double* y, int32_t b) {
  if (!p || !x || !y) return fail(KF_EINVAL, "kf_apply_filter: NULL argument");
  if (b < 1 || b > 16) return fail(KF_EINVAL, "kf_apply_filter: b must lie in [1, 16]");
  const int bk = pow2ceil(b);
  KF_TRY(tune_block(p, p->A, p->sb, bk));
  return run_filter(p, p->A, p->sb, x, b, 1, b, bk, y, b, 1, b, p->w);
}

int kf_apply_filter_noalloc(kf_problem* p, const double* x, double* y, int32_t b) {
  if (!p || !x || !y) return fail(KF_EINVAL, "kf_apply_filter_noalloc: NULL argument");
  if (b < 1 || b > 16) return fail(KF_EINVAL, "kf_apply_filter_noalloc: b must lie in [1, 16]");
  int dev = -1;
  KF_HIP(hipGetDevice(&dev));
  if (dev != p->device)
    return fail(KF_EINVAL, "kf_apply_filter_noalloc: the problem lives on device " + std::to_string(p->device) +
                               ", the current device is " + std::to_string(dev));
  const int bk = pow2ceil(b);
  StepBufs sb;
  KF_TRY(scratch_step_buffers(p->n, bk, p->A.val_bytes, sb, p->opt.stepper == 4 ? 4 : 3));
  return run_filter(p, p->A, sb, x, b, 1, b, bk, y, b, 1, b, p->w, false);
}

int kf_result_free(kf_result* r) {
  if (!r) return KF_OK;
  std::free(r->omega2);
  std::free(r->omega);
  std::free(r->residual);
  std::free(r->vectors);
  std::free(r->ritz);
  std::free(r);
  return KF_OK;
}

}  // extern "C"

namespace {

// State of one eigensolve between filter applications (Algorithm 2.5's Krylov
// loop unrolled into begin / after-filter / finish so that a batch driver can
// interleave many problems around one batched time-stepping launch).
struct SolveState {
  int b = 1, bk = 1, m_max = 0;
  double tol = 0, tol_loop = 0, margin = 0;
  bool refine = false;
  int cur = 0, q0 = 0, qn = 0, prev0 = 0, pending = 0;
  int iters = 0, full_passes = 0, checked_at = -1, next_check = 0, target = 0;
  int64_t lf_steps = 0;
  int64_t ref_lf_steps = 0;  // vector time steps of the mixed-mode refinement
  bool breakdown = false, done = false, rr_pending = false, timed_filter = false;
  double wsum = 0, t0 = 0, t_lf = 0, t_gs = 0, t_rr = 0, t_ref = 0;
  CheckOut chk;
  std::vector<double> ref;
  // mixed mode: refinement already run at basis size fin_at
  CheckOut fin;
  int fin_at = -1, refines = 0, next_refine = 0;
  int proj_every = 1, since_proj = 0;
  int pred_k = -1;  // basis size and unconverged candidates at the previous check
  std::vector<double> pred_theta, pred_res;
  // kf_solve: the next filter application may be queued before the host
  // has read this step's orthogonalisation (ahead_ok), and was (ahead_ready)
  bool ahead_ok = false, ahead_ready = false;
  // operator and step buffers of the Krylov loop's filter (the stepping
  // precision; float64 after an escalation)
  const SellOp* Aop = nullptr;
  StepBufs* sbop = nullptr;
  const double* start = nullptr;  // the caller's start block (valid for the call)
  bool escalated = false;
  bool may_escalate = true;  // false: a batch without a float64 stack escalates members after its loop
  bool in_batch = false;     // the filter is the batch's stacked launch
  bool fp64_from_start = false;  // a batch member the caller put on the float64 stack
  bool wants_escalation = false;
  double t_lf_own = 0.0;  // a batch member's own stepping time after an escalation
  // checks beside the Krylov loop (kf_options.overlap_checks)
  bool async_ok = false;
  bool async_all = false;  // batch members: every check beside the loop
  int async_checks = 0;
  double t_rr_async = 0.0;
  // host wall seconds (batch progress report): orthogonalisation, checks and
  // refinement (taken results included)
  double h_orth = 0.0, h_check = 0.0;
};

int elapsed_acc(hipEvent_t a, hipEvent_t b, double& acc) {
  KF_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  KF_HIP(hipEventElapsedTime(&ms, a, b));
  acc += ms * 1e-3;
  return KF_OK;
}

// Basis size of the next Rayleigh-Ritz check: after growth by check_growth,
// or sooner when the residuals of the pairs still missing from the target
// predict convergence sooner.  Each unconverged candidate in the interval is
// matched with the nearest Ritz value of the previous check; from the
// geometric decrease of its residual per basis column it gets a predicted
// number of columns to the tolerance, and the check is placed where the
// missing-th fastest of them arrives (with 10 % to spare).
int next_check_at(const kf_problem* p, SolveState& s, int k) {
  int next = (int)std::ceil(k * (1.0 + p->opt.check_growth));
  if (s.target <= 0 || p->opt.check_growth <= 0.0) return next;
  const int missing = s.target - distinct_count(s.chk.acc_theta, s.b);
  const double lo2 = p->omega_min * p->omega_min, hi2 = p->omega_max * p->omega_max;
  std::vector<double> th_now, res_now;
  for (size_t i = 0; i < s.chk.cand_theta.size(); ++i) {
    const double th = s.chk.cand_theta[i], res = s.chk.cand_res[i];
    if (th >= lo2 && th <= hi2 && res > s.tol_loop && std::isfinite(res)) {
      th_now.push_back(th);
      res_now.push_back(res);
    }
  }
  if (missing > 0 && s.pred_k >= 0 && k > s.pred_k && !s.pred_theta.empty()) {
    std::vector<double> cols;
    size_t q = 0;
    for (size_t i = 0; i < th_now.size(); ++i) {
      while (q + 1 < s.pred_theta.size() &&
             std::fabs(s.pred_theta[q + 1] - th_now[i]) <= std::fabs(s.pred_theta[q] - th_now[i]))
        ++q;
      if (std::fabs(s.pred_theta[q] - th_now[i]) > 1e-2 * th_now[i] || !(res_now[i] < s.pred_res[q])) continue;
      const double rate = std::log(res_now[i] / s.pred_res[q]) / (k - s.pred_k);  // per column, < 0
      const double c = std::log(s.tol_loop / res_now[i]) / rate;
      if (std::isfinite(c) && c > 0.0) cols.push_back(c);
    }
    if (!cols.empty()) {
      // (pairs without a Ritz value in the interval yet are not predictable:
      // then the slowest predictable one sets an early check, which is cheap
      // next to overshooting by a growth step)
      std::sort(cols.begin(), cols.end());
      const size_t r = (size_t)std::min<int>(missing, (int)cols.size()) - 1;
      next = std::min(next, k + (int)std::ceil(1.1 * cols[r]));
    }
  }
  // once pairs converge, a growth step is halved: the rest typically follow
  // within a fraction of the basis, Krylov convergence accelerates (so the
  // geometric prediction above runs late), and an early check costs less
  // than an overshoot
  if (missing > 0 && missing < s.target) next = k + std::max(1, (next - k + 1) / 2);
  s.pred_k = k;
  s.pred_theta = th_now;
  s.pred_res = res_now;
  return next;
}

// Mixed mode with a target: the float64 refinement of the current Ritz block.
int solve_refine_now(kf_problem* p, SolveState& s) {
  hipStream_t st = p->st;
  KF_HIP(hipEventSynchronize(p->ev[4]));
  if (s.rr_pending) KF_TRY(elapsed_acc(p->ev[3], p->ev[4], s.t_rr));
  s.rr_pending = false;
  KF_HIP(hipEventRecord(p->ev[3], st));
  KF_TRY(refine_mixed(p, s.cur, s.tol, s.chk, p->opt.want_vectors != 0, s.fin, &s.ref_lf_steps, s.target, s.b,
                      s.margin));
  KF_HIP(hipEventRecord(p->ev[4], st));
  KF_HIP(hipEventSynchronize(p->ev[4]));
  KF_TRY(elapsed_acc(p->ev[3], p->ev[4], s.t_ref));
  s.fin_at = s.cur;
  ++s.refines;
  return KF_OK;
}

int load_start(kf_problem* p, SolveState& s, int* kept_out);

int solve_begin(kf_problem* p, const double* start, int32_t b, int32_t m_max, double tol, SolveState& s) {
  s = SolveState();
  s.t0 = now_s();
  if (!p || !start) return fail(KF_EINVAL, "kf_solve: NULL argument");
  if (b < 1 || b > 16) return fail(KF_EINVAL, "kf_solve: b must lie in [1, 16]");
  if (m_max < b) return fail(KF_EINVAL, "kf_solve: m_max must be >= b");
  if (m_max > 2048) return fail(KF_EINVAL, "kf_solve: m_max must be <= 2048");
  if (!(tol > 0)) return fail(KF_EINVAL, "kf_solve: tol must be positive");
  s.b = b;
  s.bk = pow2ceil(b);
  s.m_max = m_max;
  // float32 steps leave components of relative size ~1e-7 along the whole
  // basis in every new column: those are removed at every step
  s.proj_every = p->opt.precision == KF_MIXED ? 1 : std::min(p->opt.proj_every, 15);
  KF_TRY(tune_block(p, p->A, p->sb, s.bk));
  s.tol = tol;
  // the basis storage starts at a few times the target and grows on demand
  // (up to m_max + bk columns)
  {
    const int full = m_max + s.bk;
    const int first = std::min(full, std::max(256, 4 * std::max(p->opt.target, 0)) + 3 * s.bk);
    if (p->bcap < first || p->ldb != ((int64_t)p->n + 63) / 64 * 64) {
      if (p->bcap < first) KF_TRY(ensure_basis(p, first));
    }
  }
  KF_TRY(ensure_misc(p));
  s.Aop = &p->A;
  s.sbop = &p->sb;
  s.start = start;
  int kept = 0;
  KF_TRY(load_start(p, s, &kept));
  // Mixed precision: float32 time stepping leaves a residual floor of about
  // eps32 * lambda_max / omega^2 (lambda_max <= 4/tau^2 by the CFL bound); the
  // Krylov loop accepts at ten times that floor and the float64 refinement
  // takes the pairs to tol.  Candidates are taken from the interval widened
  // by 5% of its width.
  s.refine = p->opt.precision == KF_MIXED && p->opt.refine && p->A64.val;
  const double floor32 = 5.96e-8 * 4.0 / (p->tau * p->tau) / std::max(p->omega_min * p->omega_min, 1e-300);
  s.tol_loop = s.refine ? std::max(tol, std::min(1e-3, 10.0 * floor32)) : tol;
  s.margin = s.refine ? 0.05 * (p->omega_max - p->omega_min) : 0.0;
  s.cur = kept;
  s.q0 = 0;
  s.qn = kept;
  s.prev0 = 0;
  s.pending = kept;
  s.target = p->opt.target;
  // k columns hold at most k Ritz pairs: no check can meet the target earlier
  s.next_check = std::max(s.target, 0);
  for (double v : p->w) s.wsum += std::fabs(v);
  return KF_OK;
}

// The caller's start block (row-major in host or device memory; the runtime
// tells them apart) -> V (scratch), checked there for non-finite entries (on
// the device, so a device block is never read by the host) -> B[:, 0:b],
// M-orthonormalised; *kept receives the columns kept.
int load_start(kf_problem* p, SolveState& s, int* kept_out) {
  hipStream_t st = p->st;
  const int32_t n = p->n;
  const int b = s.b;
  const double* start = s.start;
  KF_HIP(hipMemcpyAsync(p->V, start, sizeof(double) * n * b, hipMemcpyDefault, st));
  {
    int32_t* fin = p->flags + 48;
    int32_t hf = 0;
    KF_HIP(hipMemsetAsync(fin, 0, sizeof(int32_t), st));
    KF_TRY(nonfinite_flag((int64_t)n * b, p->V, fin, st));
    Readback rb(p);
    KF_TRY(rb.get(&hf, fin, sizeof(int32_t)));
    KF_HIP(hipStreamSynchronize(st));
    rb.land();
    if (hf) return fail(KF_EINVAL, "kf_solve: non-finite start block");
  }
  KF_TRY(launch_scale_copy(n, b, b, p->V, b, 1, 1.0, p->B, 1, p->ldb, st));
  int kept = 0;
  KF_HIP(hipEventRecord(p->ev[1], st));
  KF_TRY(orth_block(p, 0, 0, b, &kept, s.ref, p->ev[2]));
  KF_TRY(elapsed_acc(p->ev[1], p->ev[2], s.t_gs));
  if (kept == 0) return fail(KF_EINVAL, "kf_solve: start block is zero");
  *kept_out = kept;
  return KF_OK;
}

// Mixed precision, when the float64 refinement misses the target although
// the float32 loop had reached it at its own tolerance: float32 round-off
// seeds, at every step, the directions of an eigenspace of multiplicity
// above b that the start block cannot reach; their partial copies pollute
// the Ritz vectors of the other eigenvalues along directions with the same
// filter value, so neither more float64 filtering nor a float64 continuation
// of this basis removes them.  The loop starts again from the start block
// with float64 stepping (no further refinement).
int escalate_restart(kf_problem* p, SolveState& s) {
  if (async_running(p)) {
    // a check of the float32 basis still running: its result is not needed
    KF_TRY(async_wait(p));
    p->ac->state.store(0);
  }
  s.escalated = true;
  s.Aop = &p->A64;
  s.sbop = &p->sb64;
  s.refine = false;
  // from here on a float64 solve: its early checks may run beside the loop
  if (!s.in_batch && p->opt.overlap_checks != 0 && s.target > 0) s.async_ok = true;
  s.tol_loop = s.tol;
  s.margin = 0.0;
  s.proj_every = std::min(p->opt.proj_every, 15);
  s.since_proj = 0;
  s.ahead_ready = false;
  // (a batch member steps in the batch's float64 stack instead)
  if (!s.in_batch) KF_TRY(tune_block(p, p->A64, p->sb64, s.bk));
  int kept = 0;
  KF_TRY(load_start(p, s, &kept));
  s.cur = kept;
  s.q0 = 0;
  s.qn = kept;
  s.prev0 = 0;
  s.pending = kept;
  s.checked_at = -1;
  s.next_check = std::max(s.target, 0);
  s.pred_k = -1;
  s.pred_theta.clear();
  s.pred_res.clear();
  s.chk = CheckOut();
  s.fin = CheckOut();
  s.fin_at = -1;
  s.next_refine = 0;
  s.done = false;
  return KF_OK;
}

bool solve_wants_filter(const kf_problem* p, const SolveState& s) {
  if (s.done) return false;
  if (p->opt.max_iters > 0 && s.iters >= p->opt.max_iters) return false;
  return s.cur < s.m_max;
}

// The pending columns' pencil entries (and a repair of those that drifted
// from M-orthogonality), queued on the loop's stream before a check.
int solve_check_prepare(kf_problem* p, SolveState& s) {
  hipStream_t st = p->st;
  if (s.pending > 0) {
    const int c0 = s.cur - s.pending, nc = s.pending;
    KF_TRY(rr_update(p, c0, nc));
    if (s.proj_every > 1) {
      // columns never projected since they were formed: check them too
      int32_t lh = 0;
      KF_TRY(block_gate(s.cur, c0, nc, p->T + (int64_t)nc * s.cur, s.cur, kPendingTol, p->flags + 33, st));
      Readback rl(p);
      KF_TRY(rl.get(&lh, p->flags + 33, sizeof(int32_t)));
      KF_HIP(hipStreamSynchronize(st));
      rl.land();
      // drifted columns are orthogonalised again; the interval is left to
      // the periodic projection's own check (halving here as well shortened
      // it more than needed: slower solves on the 96- and 128-cell cubes)
      if (lh) KF_TRY(repair_block(p, c0, nc));
    }
  }
  // the check formed the pending columns' projections and checked their
  // orthogonality: the projection interval starts again from here
  s.pending = 0;
  s.since_proj = 0;
  return KF_OK;
}

int solve_check_now(kf_problem* p, SolveState& s) {
  hipStream_t st = p->st;
  if (!s.rr_pending) KF_HIP(hipEventRecord(p->ev[3], st));
  KF_TRY(solve_check_prepare(p, s));
  KF_TRY(rr_check(p, s.cur, s.tol_loop, s.chk, s.margin, false));
  KF_HIP(hipEventRecord(p->ev[4], st));
  s.rr_pending = true;
  s.checked_at = s.cur;
  return KF_OK;
}

// A check beside the loop is used while more than an eighth of the target
// (at least 3 pairs) was still missing at the previous check; closer to the
// end the check runs in line, so that no filter application is spent past
// the basis that meets the target.
bool check_overlaps(const kf_problem* p, const SolveState& s) {
  if (!(s.async_ok || s.async_all) || async_running(p)) return false;
  // batch members: every check (the batched filter does not wait for it)
  if (s.async_all) return true;
  const int missing = s.checked_at < 0 ? s.target : s.target - distinct_count(s.chk.acc_theta, s.b);
  return missing > std::max(3, s.target / 8);
}

int escalate_restart(kf_problem* p, SolveState& s);

// After a check at the current basis size: the target reached at the loop's
// tolerance ends the solve (float64 stepping) or starts the float64
// refinement (mixed), which ends it, restarts with float64 stepping
// (escalate), or lets the loop go on.  A float32 loop whose check accepted
// more copies of one eigenvalue than the block width restarts with float64
// stepping at once (escalate): those copies come from float32 round-off along
// an eigenspace of multiplicity above b, the case no refinement of this basis
// resolves, and every further float32 step would be lost work.
int decide_after_check(kf_problem* p, SolveState& s) {
  if (s.refine && p->opt.escalate && !s.escalated && s.target > 0 && copies_beyond_block(s.chk.acc_theta, s.b)) {
    if (s.may_escalate) {
      KF_TRY(escalate_restart(p, s));
    } else {
      s.wants_escalation = true;
      s.done = true;
    }
    return KF_OK;
  }
  if (!(s.target > 0 && distinct_count(s.chk.acc_theta, s.b) >= s.target)) return KF_OK;
  if (!s.refine) {
    s.done = true;
  } else if (s.cur >= s.next_refine) {
    // the loop reached the target at its own tolerance: refine now, and
    // keep iterating (up to kMaxRefines refinements) if some pairs
    // still miss the requested tolerance
    KF_TRY(solve_refine_now(p, s));
    s.next_refine = (int)std::ceil(s.cur * 1.1);
    const bool met = distinct_count(s.fin.acc_theta, s.b) >= s.target;
    if (met) {
      s.done = true;
    } else if (p->opt.escalate) {
      // missed: float32 round-off left pollution no refinement of this
      // basis removes (see escalate_restart); a batch without a float64
      // stack defers it
      if (s.may_escalate) {
        KF_TRY(escalate_restart(p, s));
      } else {
        s.wants_escalation = true;
        s.done = true;
      }
    } else if (s.refines >= kMaxRefines) {
      s.done = true;
    }
  }
  return KF_OK;
}

// Takes the result of a check that ran beside the loop.  When it meets the
// target the basis is cut back to the columns it checked (the columns added
// meanwhile are dropped) and the decision is taken there: the solve ends,
// or in mixed mode the refinement runs on that basis and either ends the
// solve or restarts it with float64 stepping (overlapped checks in mixed
// mode are used only with escalate, so the loop never continues from a cut
// basis).
int solve_take_overlapped(kf_problem* p, SolveState& s) {
  CheckOut c;
  int k = 0;
  double secs = 0.0;
  KF_TRY(async_take(p, c, &k, &secs));
  s.t_rr_async += secs;
  s.chk = std::move(c);
  s.next_check = next_check_at(p, s, k);
  if (s.refine && p->opt.escalate && s.target > 0 && copies_beyond_block(s.chk.acc_theta, s.b)) {
    // (see decide_after_check: float32 round-off copies, restart now)
    return decide_after_check(p, s);
  }
  if (s.target > 0 && distinct_count(s.chk.acc_theta, s.b) >= s.target) {
    s.cur = k;
    s.checked_at = k;
    s.next_refine = 0;
    KF_TRY(decide_after_check(p, s));
    if (!s.done && !s.escalated && s.refine) {
      // (refinement missed without escalation: end with what was refined)
      s.done = true;
    }
  }
  return KF_OK;
}

// The filtered block C Q (Q = B[:, q0:q0+qn]) is in B[:, cur:cur+bk).
int solve_after_filter(kf_problem* p, SolveState& s) {
  hipStream_t st = p->st;
  // room for this block, the next one and one queued ahead
  KF_TRY(grow_basis(p, std::min(s.cur + 3 * s.bk, s.m_max + s.bk), s.cur + s.bk));
  ++s.iters;
  s.lf_steps += (int64_t)s.qn * (p->L - 1);
  if (async_ready(p)) {
    const bool was_escalated = s.escalated;
    KF_TRY(solve_take_overlapped(p, s));
    if (s.done || s.escalated != was_escalated) {
      // the filtered block just formed is not needed (the solve ended, or
      // restarted from the start block with float64 stepping)
      s.ahead_ready = false;
      if (s.timed_filter) {
        KF_HIP(hipEventSynchronize(p->ev[1]));
        KF_TRY(elapsed_acc(p->ev[0], p->ev[1], s.t_lf));
      }
      return KF_OK;
    }
  }
  int kept = 0;
  // in the three-term form the projection onto the whole basis runs every
  // proj_every steps (single vectors: the new column and the last pending one
  // are cleaned; blocks: the new block), and at most 15 columns are pending;
  // columns that drifted beyond kPendingTol are repaired and the interval
  // halved
  const bool three = !p->opt.full_reorth && s.cur > 0;
  const bool monitor = !three || s.proj_every <= 1 || s.since_proj + 1 >= s.proj_every ||
                       s.pending + s.bk > 15;
  bool loose = false;
  // between projections and checks the step's column is final once the
  // window pass is done (unless the pass cancels strongly): the next filter
  // application can then be queued before the host reads it back
  const int it1 = s.iters, cur1 = s.cur + s.bk;
  const bool check_next = it1 % p->opt.check_every == 0 && cur1 >= s.next_check;
  const bool go_on = !(p->opt.max_iters > 0 && it1 >= p->opt.max_iters) && cur1 < s.m_max;
  const bool ahead_ok = s.ahead_ok && three && s.bk == 1 && !monitor && !check_next && go_on;
  const int64_t ldb = p->ldb;
  const std::function<int()> ahead = [&]() -> int {
    KF_HIP(hipEventRecord(p->ev[5], st));
    KF_TRY(run_filter(p, *s.Aop, *s.sbop, p->B + (int64_t)s.cur * ldb, 1, ldb, s.bk, s.bk, p->B + (int64_t)cur1 * ldb, 1,
                      ldb, s.bk, p->w));
    KF_HIP(hipEventRecord(p->ev[6], st));
    return KF_OK;
  };
  bool ahead_kept = false, carried = false;
  const double h0 = now_s();
  KF_TRY(orth_block(p, s.cur, s.cur, s.bk, &kept, s.ref, p->ev[2], monitor ? s.pending : 0,
                    p->opt.full_reorth ? -1 : s.prev0, &s.full_passes, monitor, &loose, ahead_ok ? &ahead : nullptr,
                    &ahead_kept, s.proj_every > 1 ? &carried : nullptr));  // synchronises with the step's readback
  const double h1 = now_s();
  s.h_orth += h1 - h0;
  if (loose) s.proj_every = std::max(1, s.proj_every / 2);
  if (monitor) {
    // the last pending column, cleaned with the new one, stays pending (with
    // a projection at every step each column was cleaned at its own step)
    s.pending = carried ? 1 : 0;
    s.since_proj = 0;
  } else {
    ++s.since_proj;
  }
  if (s.rr_pending) {
    KF_TRY(elapsed_acc(p->ev[3], p->ev[4], s.t_rr));
    s.rr_pending = false;
  }
  if (s.timed_filter) {
    KF_TRY(elapsed_acc(p->ev[0], p->ev[1], s.t_lf));
    KF_TRY(elapsed_acc(p->ev[1], p->ev[2], s.t_gs));
  }
  // a filter queued ahead is kept when the column it read stayed as it was
  // (it is recomputed otherwise); its events become the next step's
  s.ahead_ready = ahead_kept && kept == s.bk;
  if (s.ahead_ready) {
    std::swap(p->ev[0], p->ev[5]);
    std::swap(p->ev[1], p->ev[6]);
  }
  for (int j = 0; j < s.bk; ++j) {
    // a stable step keeps |C x|_M <= sum|w_l| max|q_l| for |x|_M = 1
    if (!std::isfinite(s.ref[(size_t)j]) || s.ref[(size_t)j] > 1e6 * std::max(s.wsum, 1e-300))
      return fail(KF_EUNSTABLE, "kf_solve: time stepping diverged (tau too large for the spectrum?)");
  }
  kept = std::min(kept, s.m_max - s.cur);
  if (kept == 0) {
    s.breakdown = true;
    s.done = true;
    return KF_OK;
  }
  s.prev0 = s.q0;
  s.q0 = s.cur;
  s.qn = kept;
  s.cur += kept;
  s.pending += kept;
  if (s.iters % p->opt.check_every == 0 && s.cur >= s.next_check && check_overlaps(p, s)) {
    KF_TRY(solve_check_prepare(p, s));
    KF_TRY(async_start(p, s.cur, s.tol_loop, s.margin));
    ++s.async_checks;
    s.checked_at = s.cur;
    // no further check until this one's result is taken
    s.next_check = INT32_MAX;
  } else if (s.iters % p->opt.check_every == 0 && s.cur >= s.next_check) {
    KF_TRY(solve_check_now(p, s));
    s.next_check = next_check_at(p, s, s.cur);
    KF_TRY(decide_after_check(p, s));
  }
  if (!s.done && async_running(p) && s.cur + s.bk > s.m_max) KF_TRY(solve_take_overlapped(p, s));
  // mixed precision: the float32 loop ran out of basis before it reached
  // the target at its own tolerance; refine what it has, and when pairs are
  // still missing restart with float64 stepping (the same budget)
  if (!s.done && s.refine && s.target > 0 && s.cur + s.bk > s.m_max && p->opt.escalate) {
    if (s.checked_at != s.cur) KF_TRY(solve_check_now(p, s));
    KF_TRY(solve_refine_now(p, s));
    if (distinct_count(s.fin.acc_theta, s.b) >= s.target) {
      s.done = true;
    } else if (s.may_escalate) {
      KF_TRY(escalate_restart(p, s));
    } else {
      s.wants_escalation = true;
      s.done = true;
    }
  }
  s.h_check += now_s() - h1;
  (void)st;
  return KF_OK;
}

// A library-owned result holding the accepted pairs of `fin` (host arrays).
int new_result(kf_problem* p, const CheckOut& fin, kf_result** out) {
  const int32_t n = p->n;
  kf_result* r = (kf_result*)std::calloc(1, sizeof(kf_result));
  if (!r) return fail(KF_ENOMEM, "kf: result allocation");
  const int na = (int)fin.acc_theta.size();
  r->n = n;
  r->n_pairs = na;
  r->omega2 = (double*)std::malloc(sizeof(double) * std::max(na, 1));
  r->omega = (double*)std::malloc(sizeof(double) * std::max(na, 1));
  r->residual = (double*)std::malloc(sizeof(double) * std::max(na, 1));
  r->n_ritz = (int)fin.ritz.size();
  r->ritz = (double*)std::malloc(sizeof(double) * std::max(r->n_ritz, 1));
  if (!r->omega2 || !r->omega || !r->residual || !r->ritz) {
    kf_result_free(r);
    return fail(KF_ENOMEM, "kf: result allocation");
  }
  for (int i = 0; i < na; ++i) {
    r->omega2[i] = fin.acc_theta[(size_t)i];
    r->omega[i] = std::sqrt(std::max(fin.acc_theta[(size_t)i], 0.0));
    r->residual[i] = fin.acc_res[(size_t)i];
  }
  if (r->n_ritz) std::memcpy(r->ritz, fin.ritz.data(), sizeof(double) * r->n_ritz);
  if (p->opt.want_vectors && na > 0) {
    r->vectors = (double*)std::malloc(sizeof(double) * (size_t)n * na);
    if (!r->vectors) {
      kf_result_free(r);
      return fail(KF_ENOMEM, "kf: vector allocation");
    }
    std::memcpy(r->vectors, fin.vectors.data(), sizeof(double) * (size_t)n * na);
  }
  *out = r;
  return KF_OK;
}

// The Krylov loop of one problem on its own stream (kf_solve, and members
// of a batch solved on their own after an escalation).
int solve_loop(kf_problem* p, SolveState& s) {
  s.timed_filter = true;
  s.ahead_ok = true;
  const int64_t ldb = p->ldb;
  while (solve_wants_filter(p, s)) {
    if (s.ahead_ready) {
      // queued during the previous step's orthogonalisation (same input
      // column q0, same output column cur)
      s.ahead_ready = false;
    } else {
      KF_HIP(hipEventRecord(p->ev[0], p->st));
      KF_TRY(run_filter(p, *s.Aop, *s.sbop, p->B + (int64_t)s.q0 * ldb, 1, ldb, s.qn, s.bk,
                        p->B + (int64_t)s.cur * ldb, 1, ldb, s.bk, p->w));
      KF_HIP(hipEventRecord(p->ev[1], p->st));
    }
    KF_TRY(solve_after_filter(p, s));
  }
  return KF_OK;
}

int solve_finish(kf_problem* p, SolveState& s, kf_result** out) {
  hipStream_t st = p->st;
  const int b = s.b;
  CheckOut& chk = s.chk;
  if (async_running(p)) KF_TRY(solve_take_overlapped(p, s));
  if (s.checked_at != s.cur) KF_TRY(solve_check_now(p, s));
  KF_HIP(hipEventSynchronize(p->ev[4]));
  if (s.rr_pending) KF_TRY(elapsed_acc(p->ev[3], p->ev[4], s.t_rr));
  s.rr_pending = false;
  p->basis_cols = s.cur;
  CheckOut fin;
  if (s.refine) {
    if (s.fin_at != s.cur) KF_TRY(solve_refine_now(p, s));
    fin = s.fin;
  } else if (p->opt.want_vectors) {
    KF_TRY(rr_check(p, s.cur, s.tol, fin, s.margin, true));
  } else {
    fin = chk;
  }
  const int target = s.target;
  int status = KF_OK;
  if (s.breakdown)
    status = KF_EBREAKDOWN;
  else if (target > 0 && distinct_count(fin.acc_theta, b) < target)
    status = KF_ENOTCONV;
  const int iters = s.iters;
  const int cur = s.cur;
  const bool breakdown = s.breakdown;
  const int64_t lf_steps = s.lf_steps;
  const double t_lf = s.t_lf, t_gs = s.t_gs, t_rr = s.t_rr, t_ref = s.t_ref, t0 = s.t0;
  const int full_passes = s.full_passes;
  kf_result* r = nullptr;
  KF_TRY(new_result(p, fin, &r));
  r->krylov_steps = iters;
  r->basis_size = cur;
  r->breakdown = breakdown ? 1 : 0;
  r->status = status;
  r->leapfrog_vector_steps = lf_steps;
  r->t_leapfrog = t_lf;
  r->t_gs = t_gs;
  r->t_rr = t_rr;
  r->t_refine = t_ref;
  r->orth_error = chk.orth;
  r->full_passes = full_passes;
  r->refine_vector_steps = s.ref_lf_steps;
  r->escalated = (s.escalated && !s.fp64_from_start) ? 1 : 0;
  r->t_rr_overlapped = s.t_rr_async;
  r->overlapped_checks = s.async_checks;
  KF_HIP(hipStreamSynchronize(st));
  r->t_total = now_s() - t0;
  *out = r;
  return KF_OK;
}


}  // namespace

extern "C" {

int kf_solve(kf_problem* p, const double* start, int32_t b, int32_t m_max, double tol, kf_result** out) {
  if (!out) return fail(KF_EINVAL, "kf_solve: NULL argument");
  *out = nullptr;
  if (!p) return fail(KF_EINVAL, "kf_solve: NULL argument");
  SolveState s;
  KF_TRY(solve_begin(p, start, b, m_max, tol, s));
  s.async_ok = p->opt.overlap_checks != 0 && p->opt.precision == KF_FP64 && s.target > 0 && !s.refine;
  int rc = solve_loop(p, s);
  if (rc) {
    // nothing may still read the basis when the caller continues
    (void)async_wait(p);
    if (async_running(p)) p->ac->state.store(0);
    return rc;
  }
  return solve_finish(p, s, out);
}

int kf_subspace_solve(kf_problem* p, const double* start, int32_t ncols, int32_t max_iters, double tol,
                      kf_result** out) {
  if (!out) return fail(KF_EINVAL, "kf_subspace_solve: NULL argument");
  *out = nullptr;
  if (!p || !start) return fail(KF_EINVAL, "kf_subspace_solve: NULL argument");
  if (ncols < 1 || ncols > 2048) return fail(KF_EINVAL, "kf_subspace_solve: ncols must lie in [1, 2048]");
  if (max_iters < 1) return fail(KF_EINVAL, "kf_subspace_solve: max_iters must be >= 1");
  if (!(tol > 0)) return fail(KF_EINVAL, "kf_subspace_solve: tol must be positive");
  const double t0 = now_s();
  hipStream_t st = p->st;
  const int32_t n = p->n;
  KF_TRY(ensure_basis(p, 16));
  KF_TRY(ensure_misc(p));
  KF_TRY(ensure_refine(p, ncols, ncols));
  // start block: row-major in host or device memory -> Yy (contiguous),
  // checked for non-finite entries, then into Vx column by column
  KF_HIP(hipMemcpyAsync(p->Yy, start, sizeof(double) * (size_t)n * ncols, hipMemcpyDefault, st));
  {
    int32_t* fin = p->flags + 48;
    int32_t hf = 0;
    KF_HIP(hipMemsetAsync(fin, 0, sizeof(int32_t), st));
    KF_TRY(nonfinite_flag((int64_t)n * ncols, p->Yy, fin, st));
    KF_HIP(hipMemcpyAsync(&hf, fin, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    KF_HIP(hipStreamSynchronize(st));
    if (hf) return fail(KF_EINVAL, "kf_subspace_solve: non-finite start block");
  }
  KF_TRY(launch_scale_copy(n, ncols, ncols, p->Yy, ncols, 1, 1.0, p->Vx, 1, p->ldb, st));
  double* X = p->Vx;
  double* Q = p->Yy;
  const bool mixed = p->opt.precision == KF_MIXED;
  const bool has64 = p->A64.val != nullptr;
  const int target = p->opt.target;
  SubspaceStats s32, s64;
  CheckOut chk;
  int used = 0;
  if (mixed) {
    // float32 stepping until the pairs reach the float32 floor
    // (eps32 * lambda_max / omega^2, lambda_max <= 4/tau^2), then, when a
    // float64 operator is kept (refine != 0), float64 stepping to tol
    const double floor32 = 5.96e-8 * 4.0 / (p->tau * p->tau) / std::max(p->omega_min * p->omega_min, 1e-300);
    const double tol32 = has64 ? std::max(tol, std::min(1e-3, 10.0 * floor32)) : tol;
    KF_TRY(subspace_iterate(p, p->A, p->sb, X, Q, ncols, max_iters, tol32, target, ncols, 0.0,
                            has64 ? false : p->opt.want_vectors != 0, chk, s32));
    used = s32.iters;
    if (has64 && used < max_iters && s32.dim > 0)
      KF_TRY(subspace_iterate(p, p->A64, p->sb64, X, Q, s32.dim, max_iters - used, tol, target, ncols, 0.0,
                              p->opt.want_vectors != 0, chk, s64));
  } else {
    KF_TRY(subspace_iterate(p, p->A, p->sb, X, Q, ncols, max_iters, tol, target, ncols, 0.0,
                            p->opt.want_vectors != 0, chk, s64));
  }
  const int iters = s32.iters + s64.iters;
  int inside = 0, accepted = (int)chk.acc_theta.size();
  const double lo2 = p->omega_min * p->omega_min, hi2 = p->omega_max * p->omega_max;
  for (double t : chk.cand_theta) inside += (t >= lo2 && t <= hi2) ? 1 : 0;
  kf_result* r = nullptr;
  KF_TRY(new_result(p, chk, &r));
  r->krylov_steps = iters;
  r->basis_size = (s64.iters ? s64.dim : s32.dim);
  r->status = (target > 0 ? accepted < target : accepted < inside || inside == 0) ? KF_ENOTCONV : KF_OK;
  r->leapfrog_vector_steps = s32.lf_steps + s64.lf_steps;
  r->refine_vector_steps = mixed ? s64.lf_steps : 0;
  r->t_leapfrog = s32.t_lf + s64.t_lf;
  r->t_gs = s32.t_orth + s64.t_orth;
  r->t_rr = s32.t_rr + s64.t_rr;
  r->t_refine = mixed ? s64.t_lf + s64.t_orth + s64.t_rr : 0.0;
  KF_HIP(hipStreamSynchronize(st));
  r->t_total = now_s() - t0;
  *out = r;
  return KF_OK;
}

int kf_tune_steps(const kf_csr* S, const double* m_diag, double omega_min, double omega_max, double tau,
                  const int32_t* L_cand, int32_t n_cand, const double* start, int32_t b, int32_t m_max, double tol,
                  const kf_options* opt, int32_t* L_best, double* seconds, int32_t* krylov_steps) {
  if (!L_best || !L_cand || n_cand < 1 || !start) return fail(KF_EINVAL, "kf_tune_steps: bad arguments");
  *L_best = 0;
  double best = 1e300;
  for (int32_t c = 0; c < n_cand; ++c) {
    if (L_cand[c] < 1) return fail(KF_EINVAL, "kf_tune_steps: every candidate L must be >= 1");
    kf_problem* p = nullptr;
    KF_TRY(kf_create(S, m_diag, omega_min, omega_max, tau, L_cand[c], opt, &p));
    kf_result* r = nullptr;
    // the problem's first solve of this width also times the block step
    // variant when autotuning is on: it is set up before the timed solve
    int rc = tune_block(p, p->A, p->sb, pow2ceil(b));
    if (!rc) rc = kf_solve(p, start, b, m_max, tol, &r);
    if (rc) {
      kf_destroy(p);
      return rc;
    }
    const bool met = r->status == KF_OK;
    if (seconds) seconds[c] = met ? r->t_total : -1.0;
    if (krylov_steps) krylov_steps[c] = r->krylov_steps;
    if (met && r->t_total < best) {
      best = r->t_total;
      *L_best = L_cand[c];
    }
    kf_result_free(r);
    kf_destroy(p);
  }
  if (*L_best == 0) return fail(KF_ENOTCONV, "kf_tune_steps: no candidate reached the target");
  return KF_OK;
}

int kf_copy_basis(const kf_problem* p, double* out, int32_t max_cols, int32_t* ncols) {
  if (!p || !out || !ncols || max_cols < 0) return fail(KF_EINVAL, "kf_copy_basis: bad arguments");
  const int k = std::min(max_cols, (int32_t)p->basis_cols);
  for (int c = 0; c < k; ++c)
    KF_HIP(hipMemcpy(out + (size_t)c * p->n, p->B + (int64_t)c * p->ldb, sizeof(double) * p->n, hipMemcpyDeviceToHost));
  *ncols = k;
  return KF_OK;
}


}  // extern "C"

namespace {

void free_stack(BatchStack& k) {
  if (k.exec) (void)hipGraphExecDestroy(k.exec);
  if (k.graph) (void)hipGraphDestroy(k.graph);
  k.exec = nullptr;
  k.graph = nullptr;
  free_sell(k.A);
  dfree(k.d_tb);
  k.d_tb = nullptr;
  dfree(k.wtab);
  k.wtab = nullptr;
  free_step_buffers(k.sb);
}

void free_batch(kf_batch* bt) {
  if (!bt) return;
  if (bt->st) (void)hipStreamSynchronize(bt->st);
  for (BatchStack& k : bt->stk) free_stack(k);
  for (kf_problem* p : bt->probs) kf_destroy(p);
  dfree(bt->d_sp);
  for (hipEvent_t e : bt->ev)
    if (e) (void)hipEventDestroy(e);
  if (bt->st) (void)hipStreamDestroy(bt->st);
  delete bt;
}

// Record the batched filter application of a stack (load + lmax-1 fused
// steps) for block width bk once; replays read the per-problem tables from
// device memory.
int ensure_batch_graph(kf_batch* bt, BatchStack& k, int bk) {
  if (k.exec && k.graph_bk == bk) return KF_OK;
  if (k.exec) (void)hipGraphExecDestroy(k.exec);
  if (k.graph) (void)hipGraphDestroy(k.graph);
  k.exec = nullptr;
  k.graph = nullptr;
  // stacked time-stepping buffers (rows x bk)
  if (k.sb.cap < bk || k.sb.vb != k.A.val_bytes) {
    free_step_buffers(k.sb);
    const size_t bytes = (size_t)bt->rows * bk * k.A.val_bytes;
    if (hipMalloc(&k.sb.Y0, bytes) != hipSuccess || hipMalloc(&k.sb.Y1, bytes) != hipSuccess ||
        hipMalloc(&k.sb.R, bytes) != hipSuccess)
      return fail(KF_ENOMEM, "kf_batch: time-stepping buffers");
    k.sb.cap = bk;
    k.sb.vb = k.A.val_bytes;
  }
  hipStream_t st = bt->st;
  if (bt->autotune && !k.tuned) {
    // the batched step's variant (XCD mapping, operator loads), timed on a
    // middle step of every member before the graph is captured
    BatchTables tt = k.h_tb;
    for (int q = 0; q < bt->P; ++q) tt.active[q] = 1;
    KF_HIP(hipMemcpyAsync(k.d_tb, &tt, sizeof(BatchTables), hipMemcpyHostToDevice, st));
    const size_t bytes = (size_t)bt->rows * bk * k.A.val_bytes;
    KF_HIP(hipMemsetAsync(k.sb.Y0, 0, bytes, st));
    KF_HIP(hipMemsetAsync(k.sb.Y1, 0, bytes, st));
    double best = 1e300;
    int best_remap = k.remap, best_nt = k.A.nt_loads;
    for (int nt = 0; nt <= 1; ++nt)
      for (int remap = 0; remap <= 1; ++remap) {
        k.A.nt_loads = nt;
        for (int rep = 0; rep < 2; ++rep) {  // warm-up, then the timing
          KF_HIP(hipEventRecord(bt->ev[0], st));
          for (int t = 0; t < 10; ++t)
            KF_TRY(launch_leapfrog_batch(k.A, bk, bt->d_sp, k.d_tb, k.wtab, bt->lmax, 2, k.sb.Y1, k.sb.Y0, k.sb.Y0,
                                         k.sb.R, 0, remap, st));
          KF_HIP(hipEventRecord(bt->ev[1], st));
        }
        KF_HIP(hipEventSynchronize(bt->ev[1]));
        float ms = 0.f;
        KF_HIP(hipEventElapsedTime(&ms, bt->ev[0], bt->ev[1]));
        if (ms < best) {
          best = ms;
          best_remap = remap;
          best_nt = nt;
        }
      }
    k.remap = best_remap;
    k.A.nt_loads = best_nt;
    k.tuned = true;
  }
  KF_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int rc = launch_load_batch(k.A.val_bytes, bt->rows, bk, bt->d_sp, k.d_tb, k.wtab, bt->lmax, k.sb.Y1, st);
  void* Y[2] = {k.sb.Y0, k.sb.Y1};
  for (int l = 1; l < bt->lmax && rc == KF_OK; ++l)
    rc = launch_leapfrog_batch(k.A, bk, bt->d_sp, k.d_tb, k.wtab, bt->lmax, l, Y[l & 1], Y[(l + 1) & 1],
                               Y[(l + 1) & 1], k.sb.R, bt->prefix[(size_t)l], k.remap, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc != KF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(KF_EHIP, std::string("kf_batch: graph capture failed: ") + hipGetErrorString(e));
  k.graph = g;
  KF_HIP(hipGraphInstantiate(&k.exec, k.graph, nullptr, nullptr, 0));
  k.graph_bk = bk;
  return KF_OK;
}

int run_batch_filter(kf_batch* bt, BatchStack& k, int bk) {
  KF_TRY(ensure_batch_graph(bt, k, bk));
  KF_HIP(hipMemcpyAsync(k.d_tb, &k.h_tb, sizeof(BatchTables), hipMemcpyHostToDevice, bt->st));
  KF_HIP(hipGraphLaunch(k.exec, bt->st));
  return KF_OK;
}

// Weights of member q in a stack's table (its precision).
int upload_weights(kf_batch* bt, BatchStack& k, int q, const double* w, int L) {
  const int vb = k.A.val_bytes;
  char* row = static_cast<char*>(k.wtab) + (size_t)q * bt->lmax * vb;
  if (vb == 8) {
    KF_HIP(hipMemcpy(row, w, sizeof(double) * L, hipMemcpyHostToDevice));
  } else {
    std::vector<float> w32(w, w + L);
    KF_HIP(hipMemcpy(row, w32.data(), sizeof(float) * L, hipMemcpyHostToDevice));
  }
  return KF_OK;
}

}  // namespace

extern "C" {

int kf_create_batch(int32_t P, const kf_problem_desc* descs, const kf_options* opt, kf_batch** out) {
  if (!out) return fail(KF_EINVAL, "kf_create_batch: NULL output");
  *out = nullptr;
  if (P < 1 || P > kMaxBatch || !descs)
    return fail(KF_EINVAL, "kf_create_batch: need 1 <= P <= " + std::to_string(kMaxBatch) + " descriptors");
  kf_options o;
  kf_default_options(&o);
  if (opt) o = *opt;
  kf_batch* bt = new (std::nothrow) kf_batch();
  if (!bt) return fail(KF_ENOMEM, "kf_create_batch: host allocation");
  bt->P = P;
  if (o.batch_workers < 0) {
    delete bt;
    return fail(KF_EINVAL, "kf_create_batch: batch_workers must be >= 0");
  }
  bt->workers = o.batch_workers > 0 ? std::min<int>(o.batch_workers, P) : std::min<int>(8, P);
  if (o.stepper != 0 && o.stepper != 2) {
    delete bt;
    return fail(KF_EINVAL, "kf_create_batch: batches step with the second-order scheme (stepper 2)");
  }
  int rc = KF_OK;
  do {
    if (hipStreamCreate(&bt->st) != hipSuccess) {
      rc = fail(KF_EHIP, "kf_create_batch: stream creation failed");
      break;
    }
    o.stream = bt->st;
    // stacked operator: problem p occupies rows [row0_p, row0_p + n_p), padded to 64
    std::vector<int32_t> rowptr{0}, col;
    std::vector<double> val;
    std::vector<int32_t> sp;
    int64_t row0 = 0;
    bt->autotune = o.autotune;
    for (int32_t q = 0; q < P && rc == KF_OK; ++q) {
      const kf_problem_desc& d = descs[q];
      kf_options oq = o;
      oq.target = d.target;
      kf_problem* pq = nullptr;
      rc = kf_create(&d.S, d.m_diag, d.omega_min, d.omega_max, d.tau, d.L, &oq, &pq);
      if (rc) {
        set_error("kf_create_batch: problem " + std::to_string(q) + ": " + kf_last_error());
        break;
      }
      bt->probs.push_back(pq);
      if (bt->workers > 1) {
        // the member's Gram-Schmidt and Rayleigh-Ritz run on a stream of its
        // own so that members proceed concurrently between filter launches
        hipStream_t ms = nullptr;
        if (hipStreamCreateWithFlags(&ms, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&pq->sync_ev, hipEventDisableTiming) != hipSuccess) {
          if (ms) (void)hipStreamDestroy(ms);
          rc = fail(KF_EHIP, "kf_create_batch: member stream creation failed");
          break;
        }
        (void)hipStreamSynchronize(bt->st);  // set-up work of the member was queued on the batch stream
        pq->st = ms;
        pq->own_stream = true;
      }
    }
    if (rc) break;
    bt->fp64_member.assign((size_t)P, 0);
    for (int q = 0; q < P; ++q) bt->fp64_member[(size_t)q] = descs[q].step_fp64 ? 1 : 0;
    bt->group.assign((size_t)P, 0);
    for (int q = 0; q < P; ++q) {
      bt->group[(size_t)q] = q;
      for (int r = 0; r < q; ++r) {
        const kf_csr &a = descs[q].S, &c = descs[r].S;
        if (a.n == c.n && a.nnz == c.nnz && a.rowptr == c.rowptr && a.col == c.col && a.val == c.val &&
            descs[q].m_diag == descs[r].m_diag) {
          bt->group[(size_t)q] = bt->group[(size_t)r];
          break;
        }
      }
    }
    // members stacked by decreasing L (stable): the members still stepping
    // at step ell own a prefix of the stacked rows
    std::vector<int> ord((size_t)P);
    for (int q = 0; q < P; ++q) ord[(size_t)q] = q;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return descs[a].L > descs[b].L; });
    std::vector<int64_t> slices_of((size_t)P, 0);
    BatchTables& tb0 = bt->stk[0].h_tb;
    for (int32_t oi = 0; oi < P && rc == KF_OK; ++oi) {
      const int q = ord[(size_t)oi];
      const kf_problem_desc& d = descs[q];
      HostCsr h;
      rc = fetch_csr(&d.S, d.m_diag, h);
      if (rc) break;
      const int32_t n = d.S.n;
      const int64_t padded = ((int64_t)n + 63) / 64 * 64;
      if (row0 + padded > INT32_MAX / 2) {
        rc = fail(KF_EINVAL, "kf_create_batch: stacked problems exceed 2^30 rows");
        break;
      }
      for (int32_t i = 0; i < n; ++i) {
        const double sc = d.tau * d.tau / h.m[(size_t)i];
        for (int32_t k = h.rowptr[(size_t)i]; k < h.rowptr[(size_t)i + 1]; ++k) {
          col.push_back((int32_t)(row0 + h.col[(size_t)k]));
          val.push_back(sc * h.val[(size_t)k]);
        }
        rowptr.push_back((int32_t)col.size());
      }
      for (int64_t i = n; i < padded; ++i) rowptr.push_back((int32_t)col.size());
      for (int64_t s = 0; s < padded / 64; ++s) sp.push_back(q);
      slices_of[(size_t)q] = padded / 64;
      tb0.row0[q] = row0;
      tb0.n[q] = n;
      tb0.L[q] = d.L;
      bt->lmax = std::max(bt->lmax, (int)d.L);
      row0 += padded;
    }
    if (rc) break;
    bt->rows = row0;
    bt->prefix.assign((size_t)bt->lmax + 1, 0);
    for (int ell = 0; ell <= bt->lmax; ++ell) {
      int64_t cnt = 0;
      for (int oi = 0; oi < P && descs[ord[(size_t)oi]].L - 1 >= ell; ++oi) cnt += slices_of[(size_t)ord[(size_t)oi]];
      bt->prefix[(size_t)ell] = (int)std::max<int64_t>(cnt, 1);
    }
    HostCsr hs;
    hs.rowptr = std::move(rowptr);
    hs.col = std::move(col);
    hs.val = std::move(val);
    DevCsr dc;
    rc = upload_csr(hs, (int32_t)bt->rows, (int64_t)hs.col.size(), bt->st, dc);
    if (rc) break;
    // the stepping precision's stack, and in KF_MIXED the float64 stack of
    // the members that restart with float64 stepping
    const bool mixed = o.precision == KF_MIXED;
    bt->nstk = mixed ? 2 : 1;
    if ((rc = dalloc(&bt->d_sp, sp.size()))) break;
    std::vector<double> w64((size_t)P * bt->lmax, 0.0);
    for (int32_t q = 0; q < P; ++q)
      for (size_t l = 0; l < bt->probs[(size_t)q]->w.size(); ++l) w64[(size_t)q * bt->lmax + l] = bt->probs[(size_t)q]->w[l];
    for (int ks = 0; ks < bt->nstk && rc == KF_OK; ++ks) {
      BatchStack& k = bt->stk[ks];
      const int vb = (mixed && ks == 0) ? 4 : 8;
      rc = build_sell((int32_t)bt->rows, (int64_t)hs.col.size(), dc.rowptr, dc.col, dc.val, nullptr, vb, o.index_bytes,
                      bt->st, k.A);
      if (rc) break;
      k.A.nt_loads = o.nt_loads ? 1 : 0;
      if ((rc = dalloc(&k.d_tb, 1))) break;
      if (ks > 0) {
        // the same member layout; no member is active here before it restarts
        k.h_tb = tb0;
        for (int q = 0; q < P; ++q) k.h_tb.active[q] = 0;
      }
      if (hipMalloc(&k.wtab, w64.size() * vb) != hipSuccess) {
        rc = fail(KF_ENOMEM, "kf_create_batch: weight table");
        break;
      }
      if (vb == 8) {
        if (hipMemcpy(k.wtab, w64.data(), w64.size() * 8, hipMemcpyHostToDevice) != hipSuccess) rc = KF_EHIP;
      } else {
        std::vector<float> w32(w64.begin(), w64.end());
        if (hipMemcpy(k.wtab, w32.data(), w32.size() * 4, hipMemcpyHostToDevice) != hipSuccess) rc = KF_EHIP;
      }
      if (rc) set_error("kf_create_batch: weight table upload failed");
    }
    if (rc) break;
    if (hipMemcpy(bt->d_sp, sp.data(), sizeof(int32_t) * sp.size(), hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(KF_EHIP, "kf_create_batch: table upload failed");
      break;
    }
    for (hipEvent_t& e : bt->ev)
      if (!rc && hipEventCreate(&e) != hipSuccess) rc = fail(KF_EHIP, "kf_create_batch: event creation failed");
  } while (false);
  if (rc) {
    free_batch(bt);
    return rc;
  }
  *out = bt;
  return KF_OK;
}

int kf_batch_set_weights(kf_batch* bt, int32_t q, const double* w, int32_t L) {
  if (!bt || q < 0 || q >= bt->P) return fail(KF_EINVAL, "kf_batch_set_weights: bad handle or member index");
  KF_TRY(kf_set_weights(bt->probs[(size_t)q], w, L));
  KF_HIP(hipStreamSynchronize(bt->st));
  for (int ks = 0; ks < bt->nstk; ++ks) KF_TRY(upload_weights(bt, bt->stk[ks], q, w, L));
  return KF_OK;
}

int kf_destroy_batch(kf_batch* bt) {
  free_batch(bt);
  return KF_OK;
}

int kf_batch_apply_filter(kf_batch* bt, const double* const* x, double* const* y, int32_t b) {
  if (!bt || !x || !y) return fail(KF_EINVAL, "kf_batch_apply_filter: NULL argument");
  if (b < 1 || b > 16) return fail(KF_EINVAL, "kf_batch_apply_filter: b must lie in [1, 16]");
  BatchTables& tb = bt->stk[0].h_tb;
  for (int q = 0; q < bt->P; ++q) {
    if (!x[q] || !y[q]) return fail(KF_EINVAL, "kf_batch_apply_filter: NULL block");
    tb.active[q] = 1;
    tb.src[q] = x[q];
    tb.lds[q] = tb.n[q];
    tb.bsrc[q] = b;
    tb.dst[q] = y[q];
    tb.ld[q] = tb.n[q];
    tb.bout[q] = b;
  }
  KF_TRY(run_batch_filter(bt, bt->stk[0], pow2ceil(b)));
  KF_HIP(hipStreamSynchronize(bt->st));
  return KF_OK;
}

int kf_solve_batch(kf_batch* bt, const double* const* starts, int32_t b, int32_t m_max, double tol,
                   kf_result** results) {
  if (!bt || !starts || !results) return fail(KF_EINVAL, "kf_solve_batch: NULL argument");
  for (int q = 0; q < bt->P; ++q) results[q] = nullptr;
  std::vector<SolveState> S((size_t)bt->P);
  // with a float64 stack, members restart with float64 stepping inside the
  // batched loop; otherwise after it, one after another
  const bool in_loop = bt->nstk > 1;
  for (int q = 0; q < bt->P; ++q) {
    S[(size_t)q].in_batch = true;
    int rc = solve_begin(bt->probs[(size_t)q], starts[q], b, m_max, tol, S[(size_t)q]);
    if (rc) {
      set_error("kf_solve_batch: problem " + std::to_string(q) + ": " + kf_last_error());
      return rc;
    }
    S[(size_t)q].may_escalate = in_loop;
    // checks beside the batched loop (the next batched filter does not wait
    // for them); in mixed mode only where a missed refinement restarts
    kf_problem* pq = bt->probs[(size_t)q];
    if (in_loop && bt->fp64_member[(size_t)q]) {
      // the caller's choice: float64 stepping from the start (the float64 stack)
      rc = escalate_restart(pq, S[(size_t)q]);
      if (rc) {
        set_error("kf_solve_batch: problem " + std::to_string(q) + ": " + kf_last_error());
        return rc;
      }
      S[(size_t)q].fp64_from_start = true;
    }
    S[(size_t)q].async_all = pq->opt.overlap_checks != 0 && S[(size_t)q].target > 0 &&
                             (!S[(size_t)q].refine || (pq->opt.escalate && in_loop));
  }
  const int bk = pow2ceil(b);
  double t_lf = 0.0;
  // KF_PROGRESS set: one line on stderr every 100 batched filter launches
  const bool progress = std::getenv("KF_PROGRESS") != nullptr;
  int round = 0;
  double host_filter = 0.0, host_members = 0.0;  // wall seconds: launching and waiting for the filter, member work
  while (true) {
    bool any[2] = {false, false};
    for (int q = 0; q < bt->P; ++q) {
      kf_problem* p = bt->probs[(size_t)q];
      SolveState& s = S[(size_t)q];
      const bool act = solve_wants_filter(p, s);
      const int ks = (in_loop && s.escalated) ? 1 : 0;
      for (int j = 0; j < bt->nstk; ++j) bt->stk[j].h_tb.active[q] = 0;
      if (!act) continue;
      any[ks] = true;
      BatchTables& tb = bt->stk[ks].h_tb;
      tb.active[q] = 1;
      tb.src[q] = p->B + (int64_t)s.q0 * p->ldb;
      tb.lds[q] = p->ldb;
      tb.bsrc[q] = s.qn;
      tb.dst[q] = p->B + (int64_t)s.cur * p->ldb;
      tb.ld[q] = p->ldb;
      tb.bout[q] = bk;
    }
    if (!any[0] && !any[1]) break;
    if (progress && ++round % 100 == 0) {
      int na = 0, ne = 0;
      double ho = 0.0, hc = 0.0;
      for (int q = 0; q < bt->P; ++q) {
        na += (bt->stk[0].h_tb.active[q] || (bt->nstk > 1 && bt->stk[1].h_tb.active[q])) ? 1 : 0;
        ne += S[(size_t)q].escalated ? 1 : 0;
        ho += S[(size_t)q].h_orth;
        hc += S[(size_t)q].h_check;
      }
      std::fprintf(stderr,
                   "[kf] batch: %d filter launches, %d of %d members stepping, %d restarted in float64; "
                   "%.2f s batched filter, %.2f s member Gram-Schmidt/Rayleigh-Ritz (summed over members: "
                   "%.2f s orthogonalisation, %.2f s checks and refinement)\n",
                   round, na, bt->P, ne, host_filter, host_members, ho, hc);
      std::fflush(stderr);
    }
    const bool par = bt->workers > 1;
    if (par) {
      // the filter reads the members' newest basis columns
      for (int q = 0; q < bt->P; ++q) {
        if (!bt->stk[0].h_tb.active[q] && !(bt->nstk > 1 && bt->stk[1].h_tb.active[q])) continue;
        kf_problem* p = bt->probs[(size_t)q];
        KF_HIP(hipEventRecord(p->sync_ev, p->st));
        KF_HIP(hipStreamWaitEvent(bt->st, p->sync_ev, 0));
      }
    }
    const double th0 = now_s();
    KF_HIP(hipEventRecord(bt->ev[0], bt->st));
    for (int ks = 0; ks < bt->nstk; ++ks)
      if (any[ks]) KF_TRY(run_batch_filter(bt, bt->stk[ks], bk));
    KF_HIP(hipEventRecord(bt->ev[1], bt->st));
    if (progress) {
      KF_HIP(hipEventSynchronize(bt->ev[1]));
      host_filter += now_s() - th0;
    }
    const double th1 = now_s();
    std::vector<int> act;
    for (int q = 0; q < bt->P; ++q)
      if (bt->stk[0].h_tb.active[q] || (bt->nstk > 1 && bt->stk[1].h_tb.active[q])) act.push_back(q);
    if (!par) {
      for (int q : act) {
        int rc = solve_after_filter(bt->probs[(size_t)q], S[(size_t)q]);
        if (rc) {
          set_error("kf_solve_batch: problem " + std::to_string(q) + ": " + kf_last_error());
          return rc;
        }
      }
    } else {
      for (int q : act) KF_HIP(hipStreamWaitEvent(bt->probs[(size_t)q]->st, bt->ev[1], 0));
      std::atomic<int> next{0};
      std::vector<int> rcs(act.size(), KF_OK);
      std::vector<std::string> msgs(act.size());
      auto work = [&]() {
        for (int i = next.fetch_add(1); i < (int)act.size(); i = next.fetch_add(1)) {
          const int q = act[(size_t)i];
          rcs[(size_t)i] = solve_after_filter(bt->probs[(size_t)q], S[(size_t)q]);
          if (rcs[(size_t)i]) msgs[(size_t)i] = kf_last_error();
        }
      };
      const int nt = std::min<int>(bt->workers, (int)act.size());
      std::vector<std::thread> pool;
      for (int t = 1; t < nt; ++t) pool.emplace_back(work);
      work();
      for (std::thread& th : pool) th.join();
      for (size_t i = 0; i < act.size(); ++i)
        if (rcs[i]) {
          set_error("kf_solve_batch: problem " + std::to_string(act[i]) + ": " + msgs[i]);
          return rcs[i];
        }
    }
    host_members += now_s() - th1;
    if (in_loop) {
      // a member that restarted with float64 stepping: its siblings on the
      // same operator follow now (their float32 refinement would miss too)
      for (int q : act) {
        if (!S[(size_t)q].escalated) continue;
        for (int r = 0; r < bt->P; ++r) {
          SolveState& sr = S[(size_t)r];
          if (r == q || bt->group[(size_t)r] != bt->group[(size_t)q] || sr.escalated || sr.done || !sr.refine)
            continue;
          int rc = escalate_restart(bt->probs[(size_t)r], sr);
          if (rc) {
            set_error("kf_solve_batch: problem " + std::to_string(r) + " (float64 restart): " + kf_last_error());
            return rc;
          }
        }
      }
    }
    // (members whose solve ended at this step did not wait for the filter)
    KF_HIP(hipEventSynchronize(bt->ev[1]));
    KF_TRY(elapsed_acc(bt->ev[0], bt->ev[1], t_lf));
  }
  // (batches without a float64 stack) members whose float64 refinement
  // missed the target: their own float64 Krylov loop from the start block
  // (see escalate_restart), one member after another on its own stream
  for (int q = 0; q < bt->P; ++q) {
    SolveState& s = S[(size_t)q];
    if (!s.wants_escalation) continue;
    kf_problem* p = bt->probs[(size_t)q];
    s.may_escalate = true;
    s.in_batch = false;
    s.t_lf = 0.0;
    int rc = escalate_restart(p, s);
    if (!rc) rc = solve_loop(p, s);
    if (rc) {
      set_error("kf_solve_batch: problem " + std::to_string(q) + " (float64 restart): " + kf_last_error());
      return rc;
    }
    s.t_lf_own = s.t_lf;
  }
  for (int q = 0; q < bt->P; ++q) {
    S[(size_t)q].t_lf = t_lf + S[(size_t)q].t_lf_own;  // the batched stepping time, shared by all members
    int rc = solve_finish(bt->probs[(size_t)q], S[(size_t)q], &results[q]);
    if (rc) {
      for (int r = 0; r < q; ++r) {
        kf_result_free(results[r]);
        results[r] = nullptr;
      }
      return rc;
    }
  }
  return KF_OK;
}

}  // extern "C"
