// wc_pc_apply_noalloc: the preconditioner apply of wc_pc_apply without a plan and without
// any device allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops).  The FP64/FP32 tables of the three-step apply and the spectral
// workspace live in one file-scope device array `scratch`; the tables are computed on the
// device by a small kernel at every call (so the call is capture-safe: no host-to-device
// copies), then the same pass kernels as wc_pc_apply run on a plan descriptor whose device
// pointers point into the array.
//
// The array is shared by every call on a device: calls that overlap on one GPU (on
// different streams, or from different host threads without ordering) race on it.

#include <cmath>
#include <cstring>
#include <mutex>

#include "wc_internal.h"

using namespace wc;

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

// Address of this device's copy of `scratch`, looked up once per device with that device
// current (hipGetSymbolAddress).  In host code the array's name is only a stand-in.
hipError_t scratch_ptr(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the tables and the spectral array inside the scratch array.
struct Layout {
  size_t lam64, lam32, dtw, twt64, twt32, tws64, tws32, sin64, sin32, mu64, mu32, spec, total;
};

Layout layout_of(int n, int N1, int M, size_t m, int precision) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  L.lam64 = take((size_t)n * 8);        // n/2 complex
  L.lam32 = take((size_t)n * 4);
  L.dtw = take((size_t)n * 16);         // n complex: omega^{k/n}
  L.twt64 = take((size_t)n * 16);       // n complex: e^{-2 pi i p/n}
  L.twt32 = take((size_t)n * 8);
  L.tws64 = take((size_t)N1 * 16);      // N1 complex: e^{-2 pi i p/N1}
  L.tws32 = take((size_t)N1 * 8);
  L.sin64 = take((size_t)N1 * 8);       // sin(pi i/N1)
  L.sin32 = take((size_t)N1 * 4);
  L.mu64 = take((size_t)M * 8);         // eigenvalues of the 1D -L_h
  L.mu32 = take((size_t)M * 4);
  L.spec = take((size_t)n * m * (precision == WC_MIXED ? 8 : 16));
  L.total = o;
  return L;
}

// The tables of set_tables (Section 3.4, remark on the singular S^(2)) in FP64 and FP32,
// one thread per entry index.
__global__ __launch_bounds__(kThreads) void k_noalloc_tables(unsigned char *base, Layout L, int n,
                                                             int N1, int M, double zeta,
                                                             double theta, double s2_remedy,
                                                             double inv_h2, double h) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  double s, c;
  if (i < n / 2) {  // kept frequency l = i + 1
    const int l = i + 1;
    sincos((zeta - 2.0 * M_PI * l) / n, &s, &c);
    const double l1x = 1.0 - c, l1y = -s;
    double l2x = theta + (1.0 - theta) * c, l2y = (1.0 - theta) * s;
    if (sqrt(l2x * l2x + l2y * l2y) < 1e-13) { l2x = s2_remedy; l2y = 0.0; }
    const double d = l2x * l2x + l2y * l2y;
    const double lx = (l1x * l2x + l1y * l2y) / d, ly = (l1y * l2x - l1x * l2y) / d;
    ((double *)(base + L.lam64))[2 * i] = lx;
    ((double *)(base + L.lam64))[2 * i + 1] = ly;
    ((float *)(base + L.lam32))[2 * i] = (float)lx;
    ((float *)(base + L.lam32))[2 * i + 1] = (float)ly;
  }
  if (i < n) {
    sincos(zeta * i / n, &s, &c);
    ((double *)(base + L.dtw))[2 * i] = c;
    ((double *)(base + L.dtw))[2 * i + 1] = s;
    sincos(2.0 * M_PI * i / n, &s, &c);
    ((double *)(base + L.twt64))[2 * i] = c;
    ((double *)(base + L.twt64))[2 * i + 1] = -s;
    ((float *)(base + L.twt32))[2 * i] = (float)c;
    ((float *)(base + L.twt32))[2 * i + 1] = (float)-s;
  }
  if (i < N1) {
    sincos(2.0 * M_PI * i / N1, &s, &c);
    ((double *)(base + L.tws64))[2 * i] = c;
    ((double *)(base + L.tws64))[2 * i + 1] = -s;
    ((float *)(base + L.tws32))[2 * i] = (float)c;
    ((float *)(base + L.tws32))[2 * i + 1] = (float)-s;
    const double sn = sin(M_PI * i / N1);
    ((double *)(base + L.sin64))[i] = sn;
    ((float *)(base + L.sin32))[i] = (float)sn;
  }
  if (i < M) {
    const double sv = sin((i + 1) * M_PI * h / 2.0);
    const double mu = 4.0 * inv_h2 * sv * sv;
    ((double *)(base + L.mu64))[i] = mu;
    ((float *)(base + L.mu32))[i] = (float)mu;
  }
}

bool pow2_in(int x, int lo, int hi) { return x >= lo && x <= hi && (x & (x - 1)) == 0; }

}  // namespace

extern "C" {

size_t wc_pc_apply_noalloc_limit(void) { return kScratchBytes; }

wc_status wc_pc_apply_noalloc(const wc_problem *prob, int method, int precision,
                              const double *v, double *w, void *stream) {
  if (!prob || !v || !w) return WC_E_ARG;
  if (prob->dims != 1 && prob->dims != 2) return WC_E_ARG;
  if (prob->M < 1 || prob->n < 2) return WC_E_ARG;
  if (!(prob->T > 0) || !std::isfinite(prob->T)) return WC_E_ARG;
  if (!(prob->theta >= 0.5 && prob->theta <= 1.0)) return WC_E_ARG;
  if (!(prob->gamma > 0) || !std::isfinite(prob->gamma)) return WC_E_ARG;
  if (!std::isfinite(prob->zeta) || !std::isfinite(prob->s2_remedy)) return WC_E_ARG;
  if (method < WC_MINRES_ABS_PS || method > WC_GMRES_PS) return WC_E_ARG;
  if (precision != WC_FP64 && precision != WC_MIXED) return WC_E_ARG;
  if (prob->disc != WC_FD && prob->disc != WC_FEM) return WC_E_ARG;
  if (prob->bc != WC_DIRICHLET && prob->bc != WC_NEUMANN) return WC_E_ARG;
  if (!(prob->kappa >= 0) || !std::isfinite(prob->kappa)) return WC_E_ARG;
  // the same coverage as wc_pc_apply for finite differences, Dirichlet data, constant a
  if (prob->a_face_host || prob->disc != WC_FD || prob->bc != WC_DIRICHLET)
    return WC_E_UNSUPPORTED;
  if (std::fabs(prob->zeta - M_PI) > 1e-12 || !pow2_in(prob->n, 4, 1024) ||
      !pow2_in(prob->M + 1, 4, 1024))
    return WC_E_UNSUPPORTED;
  if (prob->s2_remedy == 0.0) {  // a zero eigenvalue of S^(2) needs a remedy value
    for (int l = 0; l < prob->n; ++l) {
      const double a = (prob->zeta - 2.0 * M_PI * l) / prob->n;
      const double re = prob->theta + (1.0 - prob->theta) * std::cos(a);
      const double im = (1.0 - prob->theta) * std::sin(a);
      if (std::sqrt(re * re + im * im) < 1e-13) return WC_E_SINGULAR_S2;
    }
  }
  const int M = prob->M, n = prob->n, N1 = M + 1;
  const size_t m = prob->dims == 1 ? (size_t)M : (size_t)M * M;
  const Layout L = layout_of(n, N1, M, m, precision);
  if (L.total > kScratchBytes) return WC_E_ARG;  // beyond the scratch array's capacity

  void *base = nullptr;
  if (scratch_ptr(&base) != hipSuccess) {
    (void)hipGetLastError();
    return WC_E_HIP;
  }
  unsigned char *b = (unsigned char *)base;
  // plan descriptor over the scratch array (no allocation: its vectors stay empty)
  wc_plan p;
  p.dims = prob->dims;
  p.M = M;
  p.n = n;
  p.m = (int)m;
  p.N1 = N1;
  p.T = prob->T;
  p.theta = prob->theta;
  p.gamma = prob->gamma;
  p.zeta = prob->zeta;
  p.s2_remedy = prob->s2_remedy;
  p.h = 1.0 / N1;
  p.kappa = prob->kappa == 0.0 ? 1.0 : prob->kappa;
  p.inv_h2 = p.kappa * N1 * N1;
  p.tau = prob->T / n;
  p.alpha = p.tau / std::sqrt(prob->gamma);
  p.var_coeff = false;
  p.pc_ok = true;
  wc_opts_default(&p.opts);
  p.opts.method = method;
  p.opts.precision = precision;
  p.stream = (hipStream_t)stream;
  p.nvec = 2 * (size_t)n * m;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      p.num_cu = cus;
  }
  p.d_lam64 = (double *)(b + L.lam64);
  p.d_lam32 = (float *)(b + L.lam32);
  p.d_dtw = (double *)(b + L.dtw);
  p.d_twt64 = (double *)(b + L.twt64);
  p.d_twt32 = (float *)(b + L.twt32);
  p.d_tws64 = (double *)(b + L.tws64);
  p.d_tws32 = (float *)(b + L.tws32);
  p.d_sin64 = (double *)(b + L.sin64);
  p.d_sin32 = (float *)(b + L.sin32);
  p.d_mu64 = (double *)(b + L.mu64);
  p.d_mu32 = (float *)(b + L.mu32);
  p.d_specA = (void *)(b + L.spec);

  const int ntab = std::max(n, std::max(N1, M));
  hipLaunchKernelGGL(k_noalloc_tables, dim3((ntab + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     p.stream, b, L, n, N1, M, prob->zeta, prob->theta, prob->s2_remedy,
                     p.inv_h2, p.h);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_pc_apply(p, v, w, false, nullptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return WC_E_HIP;
  }
  return WC_OK;
}

}  // extern "C"
