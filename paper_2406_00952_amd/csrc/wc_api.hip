// C ABI of libwcirc: plan construction (FP64 tables, workspaces), the asynchronous
// building blocks (rhs, matvec, pc apply, recovery) and the Krylov drivers.
//
// Krylov drivers keep every vector on the device.  MINRES advances its scalar
// recurrences in one-block device kernels between the vector passes; the host reads
// back a status word once per iteration.  GMRES(k) computes Hessenberg entries on the
// device (classical Gram-Schmidt applied twice), copies the new column to the host once
// per iteration and does the Givens QR of the small (k+1) x k matrix there.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <new>

#include "wc_internal.h"

using namespace wc;

namespace wc {

const char *kernel_name(int id) {
  static const char *names[K_COUNT] = {
      "tfft_fwd", "dst_x1_fwd", "pair_mode", "dst_x1_inv", "tfft_inv", "matvec", "rhs",
      "recover", "lincomb3", "dot", "finalize", "minres_update", "minres_scalar", "multidot",
      "multiaxpy", "scale", "fill", "multidot_re", "multiaxpy_re", "mg_smooth", "mg_restrict",
      "mg_lds", "mg_norm", "mg_mix", "lr_setup", "contract", "pair_contract", "dst_x2_fwd"};
  return (id >= 0 && id < K_COUNT) ? names[id] : "?";
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace wc

namespace {

bool pow2_in(int x, int lo, int hi) { return x >= lo && x <= hi && (x & (x - 1)) == 0; }

wc_status validate(const wc_problem *pr, const wc_opts *op) {
  if (!pr || !op) return WC_E_ARG;
  if (pr->dims != 1 && pr->dims != 2) return WC_E_ARG;
  if (pr->M < 1 || pr->n < 2) return WC_E_ARG;
  if (!(pr->T > 0) || !std::isfinite(pr->T)) return WC_E_ARG;
  if (!(pr->theta >= 0.5 && pr->theta <= 1.0)) return WC_E_ARG;
  if (!(pr->gamma > 0) || !std::isfinite(pr->gamma)) return WC_E_ARG;
  if (!std::isfinite(pr->zeta) || !std::isfinite(pr->s2_remedy)) return WC_E_ARG;
  if (op->method < WC_MINRES_ABS_PS || op->method > WC_GMRES_PS) return WC_E_ARG;
  if (op->precision != WC_FP64 && op->precision != WC_MIXED) return WC_E_ARG;
  if (!(op->tol > 0) || op->maxit < 1) return WC_E_ARG;
  if (op->method == WC_GMRES_PS && (op->restart < 1 || op->restart > kMaxRestart)) return WC_E_ARG;
  if (op->method == WC_MINRES_ABS_PS && pr->a_face_host) return WC_E_ARG;  // |P_S| needs a == 1
  if (pr->disc != WC_FD && pr->disc != WC_FEM) return WC_E_ARG;
  if (pr->disc == WC_FEM && (pr->a_face_host || op->lowrank)) return WC_E_ARG;
  if (pr->bc != WC_DIRICHLET && pr->bc != WC_NEUMANN) return WC_E_ARG;
  if (!(pr->kappa >= 0) || !std::isfinite(pr->kappa)) return WC_E_ARG;
  if (pr->a_face_host && pr->kappa != 0.0 && pr->kappa != 1.0) return WC_E_ARG;
  // Neumann data: finite differences, constant a, the nonsymmetric system (GMRES-P_S)
  if (pr->bc == WC_NEUMANN && (pr->disc != WC_FD || pr->a_face_host || pr->M < 2 ||
                               op->method != WC_GMRES_PS || op->lowrank))
    return WC_E_ARG;
  // low-rank GMRES: a == 1; the FP32 preconditioner (restarts on the FP64 true residual
  // correct what FP32 leaves, like iterative refinement) in 2D only
  if (op->lowrank && (op->method != WC_GMRES_PS || pr->a_face_host ||
                      (op->precision == WC_MIXED && pr->dims != 2)))
    return WC_E_ARG;
  const double m = std::pow((double)pr->M, pr->dims);
  if (m * pr->n * 2.0 > 4.0e9) return WC_E_ARG;  // 32-bit spatial indexing inside kernels
  if (pr->a_face_host) {
    if (op->mg_max_cycles < 1 || !(op->mg_tol >= 0) || !std::isfinite(op->mg_tol)) return WC_E_ARG;
    const size_t nf = pr->dims == 1 ? (size_t)pr->M + 1 : 2 * (size_t)pr->M * (pr->M + 1);
    for (size_t i = 0; i < nf; ++i)
      if (!(pr->a_face_host[i] > 0) || !std::isfinite(pr->a_face_host[i])) return WC_E_ARG;
  }
  return WC_OK;
}

// A zero eigenvalue of S_n^(2) (remark on the singular S_n^(2), Section 1: theta = 1/2 with
// omega^{1/n} e^{-2 pi i l/n} = -1 for some l, e.g. zeta = pi and n odd) with no remedy
// value.  Host arithmetic only, so plan creation refuses it before touching the device.
bool singular_s2_unremedied(const wc_problem *pr) {
  if (pr->s2_remedy != 0.0) return false;
  for (int l = 0; l < pr->n; ++l) {
    const std::complex<double> e = std::polar(1.0, (pr->zeta - 2.0 * M_PI * l) / pr->n);
    if (std::abs(pr->theta + (1.0 - pr->theta) * e) < 1e-13) return true;
  }
  return false;
}

// Whether the GPU preconditioner covers this problem: zeta == pi (real arithmetic, half
// spectrum), n and M+1 powers of two in [4, 1024] (sine transforms for a == 1, a
// multigrid hierarchy down to one point otherwise).
bool pc_path_ok(const wc_problem *pr) {
  if (std::fabs(pr->zeta - M_PI) > 1e-12) return false;
  if (pr->bc == WC_NEUMANN)  // dense cosine steps: any M up to 1024
    return pow2_in(pr->n, 4, 1024) && pr->M >= 2 && pr->M <= 1024;
  return pow2_in(pr->n, 4, 1024) && pow2_in(pr->M + 1, 4, 1024);
}

// Sizes or zeta outside the FFT path, constant coefficient finite differences: the general
// path (dense time transform over all n frequencies, dense spatial steps).  Its tables
// grow with n^2 and M^2, so n and M stay at most 1024.
bool general_ok(const wc_problem *pr) {
  if (pr->a_face_host || pr->disc != WC_FD) return false;
  if (pr->n < 2 || pr->n > 1024 || pr->M > 1024) return false;
  return pr->bc == WC_NEUMANN ? pr->M >= 2 : pr->M >= 1;
}
bool uses_general(const wc_problem *pr) { return !pc_path_ok(pr) && general_ok(pr); }

int krylov_vectors(const wc_problem *pr, const wc_opts *op) {
  (void)pr;
  if (op->lowrank) return 2 + 2;  // r0, P^{-1} update; B, X
  if (op->method == WC_GMRES_PS) {
    const bool flex = op->flexible || op->precision == WC_MIXED;
    return (op->restart + 1) + (flex ? op->restart : 1) + 1 + 2;  // V, Z, T, B, X
  }
  return 8 + 2;  // R V0 V1 Z ZN W0 W1 AZ, B, X
}

struct Sizes {
  size_t nvec, spec_bytes, spec_t_bytes, fem_bytes, neu_bytes, gen_bytes, partials, tables, vecs,
      mg, total;
};

bool uses_spec_t(const wc_problem *pr, const wc_opts *op) {
  return pr->dims == 2 && !pr->a_face_host && !op->lowrank && pr->disc == WC_FD &&
         pr->bc == WC_DIRICHLET && pr->M + 1 >= 128 && pc_path_ok(pr);
}

// The general path at power-of-two sizes (2D Dirichlet, a constant, any zeta): FFTs over all
// n frequencies and the transposed sine passes, whose copy holds 2n slabs of M rows of M + 1.
bool uses_full_fft(const wc_problem *pr) {
  auto p2 = [](int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; };
  return uses_general(pr) && pr->dims == 2 && pr->bc == WC_DIRICHLET && !pr->a_face_host &&
         pr->disc == WC_FD && p2(pr->n, 4, 1024) && p2(pr->M + 1, 128, 1024);
}

// Multigrid levels M_0 = M, M_{l+1} = (M_l - 1)/2, ..., 1; the first level whose remaining
// pyramid fits the LDS budget of one workgroup; bytes of u and f of levels 1..ltop.
struct MgShape {
  int nlev = 0, ltop = 0;
  int M[kMgMaxLevels] = {};
  size_t work = 0, faces = 0;
};

MgShape mg_shape(int dims, int M, int n, int precision) {
  MgShape g;
  const size_t es = precision == WC_MIXED ? 8 : 16;
  for (int Ml = M; g.nlev < kMgMaxLevels; Ml = (Ml - 1) / 2) {
    g.M[g.nlev++] = Ml;
    if (Ml <= 1) break;
  }
  g.ltop = g.nlev - 1;
  for (int l = 0; l < g.nlev; ++l)
    if (mg_lds_bytes(dims, g.M[l], precision) <= kMgLdsBytes) { g.ltop = l; break; }
  for (int l = 1; l <= g.ltop; ++l)
    g.work += (dims == 2 ? 3 : 2) * (size_t)n * (dims == 2 ? (size_t)g.M[l] * g.M[l] : (size_t)g.M[l]) * es;
  for (int l = 1; l < g.nlev; ++l)
    g.faces += dims == 2 ? 2 * (size_t)g.M[l] * (g.M[l] + 1) : (size_t)g.M[l] + 1;
  return g;
}

Sizes sizes_of(const wc_problem *pr, const wc_opts *op) {
  Sizes s{};
  const size_t m = (size_t)std::llround(std::pow((double)pr->M, pr->dims));
  s.nvec = 2 * (size_t)pr->n * m;
  const size_t es = op->precision == WC_MIXED ? 8 : 16;
  const bool gen = uses_general(pr);
  // n/2 frequencies x 2 halves x m complex; the general path keeps all n frequencies
  s.spec_bytes = (gen ? 2 : 1) * (size_t)pr->n * m * es;
  // 2D a == 1 (standard form), N1 >= 128: the transposed copy of the x2 pass, rows of N1
  s.spec_t_bytes = uses_spec_t(pr, op) ? (size_t)pr->n * pr->M * (pr->M + 1) * es
                  : uses_full_fft(pr)   ? 2 * (size_t)pr->n * pr->M * (pr->M + 1) * es
                                        : 0;
  // finite elements: the FP64 complex sine transforms of the data and the solution
  s.fem_bytes = pr->disc == WC_FEM ? (size_t)pr->n * m * 16 : 0;
  // Neumann: the second spectral array of the out-of-place dense steps, C and C^{-1}
  s.neu_bytes = pr->bc == WC_NEUMANN || gen
                    ? s.spec_bytes + 2 * (size_t)pr->M * pr->M * (sizeof(double) + sizeof(float))
                    : 0;
  // general path: Phi and its inverse, the full eigenvalue table (FP64 and FP32)
  s.gen_bytes = gen ? (2 * (size_t)pr->n * pr->n + pr->n) * 3 * sizeof(double) : 0;
  // the Gram-Schmidt reduction of GMRES step j writes (j + 2) rows of kRedBlocks partials
  // (j + 1 projections and the norm), j < kMaxRestart
  size_t parts = std::max<size_t>(2 * ((m + kThreads - 1) / kThreads),
                                  (size_t)(kMaxRestart + 2) * kRedBlocks);
  parts = std::max<size_t>(parts, (size_t)pc_partials_needed(pr->n, (int)m, op->precision));
  s.partials = parts + 64;
  s.tables = 1 << 20;
  s.vecs = (size_t)krylov_vectors(pr, op) * s.nvec * sizeof(double);
  if (op->lowrank)  // compact basis (restart + 2 vectors of 1 + 2m), s0, g, r, rho, partials
    s.vecs += ((size_t)(op->restart + 2) * (1 + 2 * m) + 2 * m + 4 * (size_t)pr->n +
               (size_t)std::max(kContractChunks, kColChunks) * 2 * m) * sizeof(double);
  if (op->lowrank && pr->dims == 2)  // rank-term spectra, a1 and a2 (r0's spectrum: d_specA)
    s.vecs += (4 * (size_t)pr->n + 2 * m) * sizeof(double);
  s.mg = 0;
  if (pr->a_face_host) {  // fine solution, coarse levels, face pyramid, shifts, rotations
    const MgShape g = mg_shape(pr->dims, pr->M, pr->n, op->precision);
    s.mg = s.spec_bytes * (pr->dims == 2 && g.ltop > 0 ? 2 : 1) + g.work +
           (g.faces + 2 * (size_t)(pr->M + 1) * pr->M) * sizeof(double) +
           (size_t)pr->n * 6 * sizeof(double);
  }
  s.total = s.spec_bytes + s.spec_t_bytes + s.fem_bytes + s.neu_bytes + s.gen_bytes +
            s.partials * sizeof(double) + s.tables + s.vecs + S_COUNT * sizeof(double) + s.mg;
  return s;
}

// Copies a host table to the device on the plan's stream, allocating the buffer on first
// use.  The caller keeps src alive until the stream has been synchronised.  (A copy on
// the legacy default stream would wait for every other blocking stream of the device.)
template <typename T>
hipError_t upload(hipStream_t st, T **dst, const std::vector<T> &src) {
  if (!*dst) {
    hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
    if (e != hipSuccess) return e;
  }
  return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

void drop_graphs(wc_plan *p) {
  for (int i = 0; i < wc_plan::kGraphSlots; ++i) {
    if (p->gexec[i]) (void)hipGraphExecDestroy(p->gexec[i]);
    p->gexec[i] = nullptr;
    p->gkey[i] = nullptr;
  }
}

bool graphs_usable(const wc_plan *p) {
  return p->opts.graphs && !p->prof.on && !p->graphs_failed &&
         (!p->var_coeff || p->opts.mg_tol == 0.0);  // the multigrid test reads the host
}

// Enqueues `body` (work on p->stream) directly, or replays the graph cached in `slot`,
// capturing it on a private stream the first time (and again when `key` changed).
// A capture that fails turns graphs off for the plan; the work is then enqueued directly.
template <typename F>
hipError_t run_captured(wc_plan *p, int slot, const void *key, F body) {
  if (!graphs_usable(p)) return body();
  if (p->gexec[slot] && p->gkey[slot] != key) {
    (void)hipGraphExecDestroy(p->gexec[slot]);
    p->gexec[slot] = nullptr;
  }
  if (!p->gexec[slot]) {
    // non-blocking: work that other threads put on the legacy stream must not take an
    // implicit dependency on a stream while it captures (an error under capture)
    if (!p->cap_stream &&
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      p->graphs_failed = true;
      return body();
    }
    hipStream_t saved = p->stream;
    p->stream = p->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t eb = body();
      const hipError_t ee = hipStreamEndCapture(p->cap_stream, &g);
      e = eb != hipSuccess ? eb : ee;
    }
    p->stream = saved;
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess && g) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess || !ex) {
      (void)hipGetLastError();
      p->graphs_failed = true;
      return body();
    }
    p->gexec[slot] = ex;
    p->gkey[slot] = key;
  }
  return hipGraphLaunch(p->gexec[slot], p->stream);
}

void free_plan(wc_plan *p) {
  if (!p) return;
  for (auto &r : p->prof.recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  for (auto e : p->prof.pool) (void)hipEventDestroy(e);
  dfree(p->d_aface);
  dfree(p->d_lam64); dfree(p->d_lam32); dfree(p->d_dtw);
  dfree(p->d_twt64); dfree(p->d_twt32); dfree(p->d_tws64); dfree(p->d_tws32);
  dfree(p->d_sin64); dfree(p->d_sin32); dfree(p->d_mu64); dfree(p->d_mu32);
  dfree(p->d_mass64); dfree(p->d_femW); dfree(p->d_cos64); dfree(p->d_cos32);
  dfree(p->d_phi64); dfree(p->d_phi32); dfree(p->d_lamf64); dfree(p->d_lamf32);
  dfree(p->d_specA); dfree(p->d_specB); dfree(p->d_specT); dfree(p->d_partials); dfree(p->d_scal);
  dfree(p->d_mg_a); dfree(p->d_mg_work); dfree(p->d_mg_shift); dfree(p->d_mg_mix);
  dfree(p->d_mg_u2);
  dfree(p->d_lr_gr); dfree(p->d_lr_s0); dfree(p->d_lr_hat); dfree(p->d_lr_rho);
  dfree(p->d_lr_part);
  dfree(p->d_lr_rank); dfree(p->d_lr_a);
  drop_graphs(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  dfree(p->d_mg_fn2);
  dfree(p->d_vecs);
  if (p->h_scal) (void)hipHostFree(p->h_scal);
  p->h_scal = nullptr;
  delete p;
}

std::vector<float> to_f32(const std::vector<double> &v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
  return o;
}

hipError_t sync_read(wc_plan *p, int slot, int count) {
  hipError_t e = hipMemcpyAsync(p->h_scal + slot, p->d_scal + slot, count * sizeof(double),
                                hipMemcpyDeviceToHost, p->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(p->stream);
}

hipError_t write_scalar(wc_plan *p, int slot, const double *vals, int count) {
  std::memcpy(p->h_scal + slot, vals, count * sizeof(double));
  return hipMemcpyAsync(p->d_scal + slot, p->h_scal + slot, count * sizeof(double),
                        hipMemcpyHostToDevice, p->stream);
}

// ---------------------------------------------------------------------------------
// MINRES (preconditioned, Lanczos in the P^{-1} inner product).  The residual
// r_j = b - A x_j is carried by the recurrence r_j = s^2 r_{j-1} + c eta_j v~_{j+1}
// that follows from the Givens QR of the Lanczos tridiagonal, and is confirmed by an
// explicit FP64 matvec when the recurrence reports convergence; a mismatch restarts
// MINRES from the current iterate.
// ---------------------------------------------------------------------------------
wc_status run_minres(wc_plan *p, const double *b, double *x, wc_info *info) {
  double *R = p->vec(0), *V0 = p->vec(1), *V1 = p->vec(2), *Z = p->vec(3), *ZN = p->vec(4);
  double *W0 = p->vec(5), *W1 = p->vec(6), *AZ = p->vec(7);
  const double tol = p->opts.tol;
  WC_TRY(launch_dot(*p, b, b, S_DOT));
  WC_TRY(sync_read(p, S_DOT, 1));
  const double bnorm = std::sqrt(p->h_scal[S_DOT]);
  WC_TRY(launch_fill(*p, x, 0.0, p->nvec));
  if (!std::isfinite(bnorm)) return WC_E_NONFINITE;
  if (bnorm == 0.0) {
    if (info) { info->status = WC_OK; info->relres = 0; info->relres_est = 0; }
    return WC_OK;
  }
  {
    const double v[1] = {bnorm};
    WC_TRY(write_scalar(p, S_BNORM, v, 1));
  }
  WC_TRY(launch_lincomb3(*p, R, b, nullptr, nullptr, -1, 1.0, 0.0, 0.0));
  int iters = 0, restarts = 0;
  wc_status st = WC_E_MAXIT;
  double relres = 1.0, relres_est = 1.0;
  for (;;) {
    {
      const double zero[2] = {0.0, 0.0};
      WC_TRY(write_scalar(p, S_STATUS, zero, 2));  // status, iteration count
    }
    WC_TRY(launch_lincomb3(*p, V1, R, nullptr, nullptr, -1, 1.0, 0.0, 0.0));
    WC_TRY(launch_fill(*p, V0, 0.0, p->nvec));
    WC_TRY(launch_fill(*p, W0, 0.0, p->nvec));
    WC_TRY(launch_fill(*p, W1, 0.0, p->nvec));
    int np = 0;
    WC_TRY(launch_pc_apply(*p, V1, Z, true, &np));
    WC_TRY(launch_minres_scalar(*p, 0, np, tol));
    WC_TRY(sync_read(p, 0, 16));
    int code = (int)p->h_scal[S_STATUS];
    if (code == ST_NONFINITE) return WC_E_NONFINITE;
    if (code == ST_BREAKDOWN) { st = WC_E_BREAKDOWN; break; }
    while (code == ST_RUNNING && iters < p->opts.maxit) {
      auto body = [&]() -> hipError_t {
        hipError_t e;
        int nq = 0;
        if ((e = launch_matvec(*p, Z, AZ, p->d_partials, &nq)) != hipSuccess) return e;
        if ((e = launch_minres_scalar(*p, 1, nq, tol)) != hipSuccess) return e;
        if ((e = launch_lincomb3(*p, V0, AZ, V1, V0, S_CV0, 0, 0, 0)) != hipSuccess) return e;
        if ((e = launch_pc_apply(*p, V0, ZN, true, &nq)) != hipSuccess) return e;
        if ((e = launch_minres_scalar(*p, 2, nq, tol)) != hipSuccess) return e;
        if ((e = launch_minres_update(*p, W0, W1, Z, x, R, V0)) != hipSuccess) return e;
        if ((e = launch_minres_scalar(*p, 3, red_blocks(p->nvec), tol)) != hipSuccess) return e;
        return hipMemcpyAsync(p->h_scal, p->d_scal, 16 * sizeof(double), hipMemcpyDeviceToHost,
                              p->stream);
      };
      WC_TRY(run_captured(p, wc_plan::kGraphSlots - 2 + (V0 == p->vec(1) ? 0 : 1), x, body));
      WC_TRY(hipStreamSynchronize(p->stream));
      ++iters;
      std::swap(V0, V1);
      std::swap(W0, W1);
      std::swap(Z, ZN);
      code = (int)p->h_scal[S_STATUS];
      relres_est = std::sqrt(p->h_scal[S_RNORM2]) / bnorm;
    }
    if (code == ST_NONFINITE) { st = WC_E_NONFINITE; break; }
    // explicit FP64 true residual
    int mv_blocks = 0;  // R = b - A x and its squared norm in one pass
    WC_TRY(launch_matvec(*p, x, R, p->d_partials, &mv_blocks, b, true));
    WC_TRY(launch_finalize(*p, p->d_partials, mv_blocks, 1, S_DOT));
    WC_TRY(sync_read(p, S_DOT, 1));
    relres = std::sqrt(p->h_scal[S_DOT]) / bnorm;
    if (relres <= tol) { st = WC_OK; break; }
    if (code == ST_BREAKDOWN && restarts > 0) { st = WC_E_BREAKDOWN; break; }
    if (iters >= p->opts.maxit) { st = WC_E_MAXIT; break; }
    if (++restarts > 20) { st = WC_E_MAXIT; break; }
  }
  if (info) {
    info->iters = iters;
    info->restarts = restarts;
    info->relres = relres;
    info->relres_est = relres_est;
    info->status = st;
  }
  return st;
}

// ---------------------------------------------------------------------------------
// GMRES(k), right preconditioned: solve A P^{-1} u = b, x = P^{-1} u.  Flexible form
// (stores z_j = P^{-1} v_j) when requested or when the preconditioner runs in FP32.
//
// Arnoldi with classical Gram-Schmidt and a second projection only when the first one
// removed more than half of the norm (decided on the device; the second pass launches
// are no-ops otherwise).  Basis vectors are stored unnormalised (V_j = nu_j v_j, nu_j
// kept as a device scalar): the matvec writes straight into the next basis slot and no
// scaling pass is needed; all coefficients are rescaled on the host.
// ---------------------------------------------------------------------------------
//
// Low-rank form (opts.lowrank): by the GMRES proposition Ahat = P_S + (Ahat - P_S) with
// Ahat - P_S = omega diag(g r^T, r g^T) (x) I, so E v = (Ahat - P_S) P^{-1} v lies in
// {[g (x) a; r (x) b]} and the Krylov space of r0 is span{r0_perp} + that range, r0_perp
// being r0's part orthogonal to it (N0 = ||r0_perp||^2).  A basis vector
// v = c r0_perp + [g (x) s1; r (x) s2] is kept as its coordinates [sqrt(N0) c; |g| s1; |r| s2],
// whose Euclidean inner products equal those of the full vectors (the three parts are
// mutually orthogonal), so the Gram-Schmidt kernels run unchanged on 1 + 2m numbers; E v_j is one preconditioner apply on the generated
// v_j whose inverse time transform contracts over time.  The update x += P^{-1} sum y_j v_j
// is one more apply.
// ---------------------------------------------------------------------------------
wc_status run_gmres(wc_plan *p, const double *b, double *x, wc_info *info) {
  const int k = p->opts.restart;
  const bool lr = p->opts.lowrank != 0;
  if (lr && !p->lr_ok) return WC_E_UNSUPPORTED;
  const bool flex = !lr && (p->opts.flexible || p->opts.precision == WC_MIXED);
  const size_t nv = p->nvec;
  const size_t len = lr ? p->lr_len : nv;  // basis vector length (and stride)
  double *V = lr ? p->d_lr_hat : p->vec(0);
  double *const R0buf = lr ? p->vec(0) : nullptr;  // full residual of later cycles (low-rank)
  double *Zb = lr ? nullptr : p->vec(k + 1);
  double *T = lr ? p->vec(1) : p->vec(k + 1 + (flex ? k : 1));
  const double tol = p->opts.tol;
  const double *gate = p->d_scal + S_REORTH;
  WC_TRY(launch_dot(*p, b, b, S_DOT));
  WC_TRY(sync_read(p, S_DOT, 1));
  const double bnorm = std::sqrt(p->h_scal[S_DOT]);
  // x0 = 0 (the low-rank form writes its first update straight into x instead)
  if (!lr || bnorm == 0.0 || !std::isfinite(bnorm)) WC_TRY(launch_fill(*p, x, 0.0, nv));
  if (!std::isfinite(bnorm)) return WC_E_NONFINITE;
  if (bnorm == 0.0) {
    if (info) { info->status = WC_OK; info->relres = 0; info->relres_est = 0; }
    return WC_OK;
  }
  std::vector<double> H((size_t)(k + 1) * k), cs(k), sn(k), g(k + 1), y(k), nu(k + 1);
  int total = 0, cycles = 0, reorth = 0;
  bool first = true;
  wc_status st = WC_E_MAXIT;
  double relres = 1.0, relres_est = 1.0;
  for (;;) {
    // the cycle's full residual r0 = b - Ahat x (x = 0 in the first cycle: b itself)
    const double *R0 = lr ? (first ? b : R0buf) : nullptr;
    double *Rf = lr ? R0buf : V;
    int mv_blocks = 0;
    if (first) {
      if (!lr) WC_TRY(launch_lincomb3(*p, Rf, b, nullptr, nullptr, -1, 1.0, 0.0, 0.0));
    } else {
      WC_TRY(launch_matvec(*p, x, Rf, p->d_partials, &mv_blocks, b, true));
    }
    double beta;
    if (lr) {
      // ||r0||^2: the matvec's partial sums (first cycle: r0 = b, whose norm is in S_DOT)
      if (!first) WC_TRY(launch_finalize(*p, p->d_partials, mv_blocks, 1, S_DOT));
      WC_TRY(sync_read(p, S_DOT, 1));
      relres = std::sqrt(p->h_scal[S_DOT]) / bnorm;
    } else {
      if (first) WC_TRY(launch_dot(*p, V, V, S_NU2));
      else WC_TRY(launch_finalize(*p, p->d_partials, mv_blocks, 1, S_NU2));
      WC_TRY(sync_read(p, S_NU2, 1));
      beta = std::sqrt(p->h_scal[S_NU2]);
      relres = beta / bnorm;
    }
    if (!std::isfinite(relres)) { st = WC_E_NONFINITE; break; }
    if (relres <= tol) { st = WC_OK; break; }
    if (total >= p->opts.maxit) { st = WC_E_MAXIT; break; }
    // low-rank form with the FP32 preconditioner: a cycle cannot take the true residual
    // much below the FP32 level of its start, so it stops there and the next cycle
    // restarts from the FP64 true residual (iterative refinement)
    const double cycle_tol =
        lr && p->opts.precision == WC_MIXED ? std::max(tol, kMixedCycleDrop * relres) : tol;
    if (lr) {  // compact coordinates of r0 (its range part and the rest)
      WC_TRY(launch_lr_setup(*p, R0, V));
      if (p->lr_2d) WC_TRY(launch_lr_spectrum(*p, R0));
      WC_TRY(launch_dot(*p, V, V, S_NU2, len));
      WC_TRY(sync_read(p, S_NU2, 1));
      beta = std::sqrt(p->h_scal[S_NU2]);
    }
    nu[0] = beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jd = 0;
    bool stop = false;
    for (int j = 0; j < k && !stop; ++j) {
      double *Vj = V + (size_t)j * len;
      double *Vn = V + (size_t)(j + 1) * len;
      double *Zj = lr ? nullptr : (flex ? Zb + (size_t)j * nv : Zb);
      int np = 0;
      auto body = [&]() -> hipError_t {
        hipError_t e;
        if (lr) {  // E v_j in compact coordinates
          if ((e = launch_pc_lowrank(*p, R0, Vj, Vn, nullptr)) != hipSuccess) return e;
        } else {
          if ((e = launch_pc_apply(*p, Vj, Zj, false, nullptr)) != hipSuccess) return e;
          // Arnoldi on E = Ahat P^{-1} - I (same Krylov space, H = H_E + I): Ahat z - v is
          // not dominated by v, so one classical Gram-Schmidt pass normally suffices
          if ((e = launch_matvec(*p, Zj, Vn, p->d_partials, nullptr, Vj)) != hipSuccess) return e;
        }
        // the second (DGKS) pass is rare: the host launches it below when the flag is set
        if ((e = launch_gram_schmidt(*p, V, j, Vn, len, 1)) != hipSuccess) return e;
        return hipMemcpyAsync(p->h_scal + S_WN2, p->d_scal + S_WN2,
                              (S_D2 + j + 1 - S_WN2) * sizeof(double), hipMemcpyDeviceToHost,
                              p->stream);
      };
      WC_TRY(run_captured(p, first ? j : kMaxRestart + j, R0, body));
      WC_TRY(hipStreamSynchronize(p->stream));
      const bool two = p->h_scal[S_REORTH] != 0.0;
      reorth += two ? 1 : 0;
      if (two) {
        WC_TRY(launch_gs_second_pass(*p, V, j, Vn, len));
        WC_TRY(hipMemcpyAsync(p->h_scal + S_WN2, p->d_scal + S_WN2,
                              (S_D2 + j + 1 - S_WN2) * sizeof(double), hipMemcpyDeviceToHost,
                              p->stream));
        WC_TRY(hipStreamSynchronize(p->stream));
      }
      const double nn = std::sqrt(std::max(p->h_scal[S_NU2 + j + 1], 0.0));
      nu[j + 1] = nn;
      double *h = &H[(size_t)j * (k + 1)];  // column j of the Hessenberg matrix
      for (int i = 0; i <= j; ++i)
        h[i] = (p->h_scal[S_D1 + i] + (two ? p->h_scal[S_D2 + i] : 0.0)) / (nu[i] * nu[j]);
      h[j] += 1.0;
      const double hn = nn / nu[j];
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double r = std::hypot(h[j], hn);
      cs[j] = r > 0 ? h[j] / r : 1.0;
      sn[j] = r > 0 ? hn / r : 0.0;
      h[j] = r;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      jd = j + 1;
      relres_est = std::fabs(g[j + 1]) / bnorm;
      if (!std::isfinite(relres_est) || r == 0.0) { stop = true; break; }
      if (relres_est <= cycle_tol || hn == 0.0 || total >= p->opts.maxit) stop = true;
    }
    // back substitution R y = g; the update uses the unnormalised vectors, so y_i / nu_i
    for (int i = jd - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < jd; ++l) s -= H[(size_t)l * (k + 1) + i] * y[l];
      const double d = H[(size_t)i * (k + 1) + i];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
    for (int i = 0; i < jd; ++i) y[i] /= nu[i];
    WC_TRY(write_scalar(p, S_Y, y.data(), jd));
    if (lr) {
      double *U = V + (size_t)(k + 1) * len;
      WC_TRY(launch_fill(*p, U, 0.0, len));
      WC_TRY(launch_multiaxpy(*p, U, V, jd, S_Y, 1.0, false, nullptr, nullptr, len));
      if (first) {  // x is still zero
        WC_TRY(launch_pc_lowrank(*p, R0, U, nullptr, x));
      } else {
        WC_TRY(launch_pc_lowrank(*p, R0, U, nullptr, T));
        WC_TRY(launch_lincomb3(*p, x, x, T, nullptr, -1, 1.0, 1.0, 0.0));
      }
    } else if (flex) {
      WC_TRY(launch_multiaxpy(*p, x, Zb, jd, S_Y, 1.0, false, nullptr, nullptr));
    } else {
      WC_TRY(launch_fill(*p, T, 0.0, nv));
      WC_TRY(launch_multiaxpy(*p, T, V, jd, S_Y, 1.0, false, nullptr, nullptr));
      WC_TRY(launch_pc_apply(*p, T, Zb, false, nullptr));
      WC_TRY(launch_lincomb3(*p, x, x, Zb, nullptr, -1, 1.0, 1.0, 0.0));
    }
    first = false;
    ++cycles;
  }
  if (info) {
    info->iters = total;
    info->restarts = cycles;
    info->relres = relres;
    info->relres_est = relres_est;
    info->reorth = reorth;
    info->status = st;
  }
  return st;
}

// Coarse face coefficients: the coarse face between two coarse nodes sits on a fine node,
// between two fine faces of the same line; its coefficient is their mean.
std::vector<double> coarsen_faces(int dims, int Mf, const std::vector<double> &af) {
  const int Mc = (Mf - 1) / 2;
  if (dims == 1) {
    std::vector<double> ac(Mc + 1);
    for (int I = 0; I <= Mc; ++I) ac[I] = 0.5 * (af[2 * I] + af[2 * I + 1]);
    return ac;
  }
  const double *axf = af.data();                            // (Mf, Mf+1)
  const double *ayf = af.data() + (size_t)Mf * (Mf + 1);    // (Mf+1, Mf)
  std::vector<double> ac(2 * (size_t)Mc * (Mc + 1));
  double *axc = ac.data(), *ayc = ac.data() + (size_t)Mc * (Mc + 1);
  for (int J = 0; J < Mc; ++J)
    for (int I = 0; I <= Mc; ++I)
      axc[(size_t)J * (Mc + 1) + I] =
          0.5 * (axf[(size_t)(2 * J + 1) * (Mf + 1) + 2 * I] + axf[(size_t)(2 * J + 1) * (Mf + 1) + 2 * I + 1]);
  for (int J = 0; J <= Mc; ++J)
    for (int I = 0; I < Mc; ++I)
      ayc[(size_t)J * Mc + I] =
          0.5 * (ayf[(size_t)(2 * J) * Mf + 2 * I + 1] + ayf[(size_t)(2 * J + 1) * Mf + 2 * I + 1]);
  return ac;
}

// Multigrid hierarchy, per-system shifts and the block-row rotation of P_S (see the
// multigrid source for the algebra).
wc_status build_multigrid(wc_plan *p, const double *a_face_host) {
  const MgShape g = mg_shape(p->dims, p->M, p->n, p->opts.precision);
  p->mg_nlev = g.nlev;
  p->mg_ltop = g.ltop;
  const size_t es = p->opts.precision == WC_MIXED ? 8 : 16;
  std::vector<double> faces;
  const size_t nf0 = p->dims == 1 ? (size_t)p->M + 1 : 2 * (size_t)p->M * (p->M + 1);
  std::vector<double> cur(a_face_host, a_face_host + nf0);
  size_t woff = 0;
  for (int l = 0; l < g.nlev; ++l) {
    p->mg_M[l] = g.M[l];
    p->mg_inv_h2[l] = (double)(g.M[l] + 1) * (g.M[l] + 1);
    if (l > 0) {
      cur = coarsen_faces(p->dims, g.M[l - 1], cur);
      p->mg_aoff[l] = faces.size();
      faces.insert(faces.end(), cur.begin(), cur.end());
    }
    if (l >= 1 && l <= g.ltop) {
      p->mg_woff[l] = woff;
      woff += (p->dims == 2 ? 3 : 2) * (size_t)p->n *
              (p->dims == 2 ? (size_t)g.M[l] * g.M[l] : (size_t)g.M[l]) * es;
    }
  }
  const int nq = p->n / 2;
  std::vector<double> shift(2 * (size_t)p->n), mix(6 * (size_t)nq);
  const double a = p->alpha;
  for (int q = 0; q < nq; ++q) {
    const int l = q + 1;
    const std::complex<double> e = std::polar(1.0, (p->zeta - 2.0 * M_PI * l) / p->n);
    std::complex<double> l2 = p->theta + (1.0 - p->theta) * e;
    if (std::abs(l2) < 1e-13) l2 = p->s2_remedy;
    const std::complex<double> lam = (1.0 - e) / l2;
    if (p->opts.method == WC_GMRES_PS) {
      const double im = lam.imag(), s = std::hypot(im, a);
      // mu_1 = i (Im - s)/alpha, mu_2 = i (Im + s)/alpha, cancellation-free
      const double m1 = im >= 0 ? -a / (im + s) : (im - s) / a;
      const double m2 = im <= 0 ? a / (s - im) : (im + s) / a;
      const double c1 = 1.0 / std::sqrt(1.0 + m1 * m1), c2 = 1.0 / std::sqrt(1.0 + m2 * m2);
      shift[4 * q + 0] = lam.real();
      shift[4 * q + 1] = s;
      shift[4 * q + 2] = lam.real();
      shift[4 * q + 3] = -s;
      double *t = &mix[6 * (size_t)q];
      t[0] = c1; t[1] = 0.0; t[2] = c1 * m1;  // c1 mu1 = i c1 m1
      t[3] = c2; t[4] = 0.0; t[5] = c2 * m2;
    } else {
      const double sg = std::sqrt(std::norm(lam) + a * a);
      shift[4 * q + 0] = sg; shift[4 * q + 1] = 0.0;
      shift[4 * q + 2] = sg; shift[4 * q + 3] = 0.0;
    }
  }
  hipError_t e = hipSuccess;
  if (!faces.empty()) e = upload(p->stream, &p->d_mg_a, faces);
  if (e == hipSuccess) e = upload(p->stream, &p->d_mg_shift, shift);
  if (e == hipSuccess) e = upload(p->stream, &p->d_mg_mix, mix);
  if (e == hipSuccess && !p->d_mg_fn2)
    e = hipMalloc((void **)&p->d_mg_fn2, (size_t)p->n * sizeof(double));
  if (e == hipSuccess && woff > 0 && !p->d_mg_work) e = hipMalloc(&p->d_mg_work, woff);
  if (e == hipSuccess && p->dims == 2 && g.ltop > 0 && !p->d_mg_u2)
    e = hipMalloc(&p->d_mg_u2, (size_t)p->n * p->m * es);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? WC_E_NOMEM : WC_E_HIP;
  }
  return WC_OK;
}

// Problem scalars and options (everything but the sizes).
void set_scalars(wc_plan *p, const wc_problem *prob, const wc_opts *opts) {
  p->T = prob->T;
  p->theta = prob->theta;
  p->gamma = prob->gamma;
  p->zeta = prob->zeta;
  p->s2_remedy = prob->s2_remedy;
  p->tau = prob->T / prob->n;
  p->alpha = p->tau / std::sqrt(prob->gamma);
  p->kappa = prob->kappa == 0.0 ? 1.0 : prob->kappa;
  p->inv_h2 = p->kappa / (p->h * p->h);  // K_m scaled by the constant a
  p->pc_ok = pc_path_ok(prob) || p->general;
  p->opts = *opts;
}

// FP64 (and FP32 copies of the) eigenvalue, twiddle and sine tables of Section 3.4 and
// the face coefficients; device buffers are allocated on first use and overwritten after.
wc_status set_tables(wc_plan *p, const wc_problem *prob) {
  // ---- FP64 tables ----
  const int n = p->n, N1 = p->N1, M = p->M;
  std::vector<double> lam(n), dtw(2 * n), twt(2 * n), tws(2 * N1), sn(N1), mu(M), mass(M), cs;
  for (int l = 0; l < n; ++l) {  // check every frequency of S^(2) for a zero eigenvalue
    const std::complex<double> e = std::polar(1.0, (p->zeta - 2.0 * M_PI * l) / n);
    const std::complex<double> l2 = p->theta + (1.0 - p->theta) * e;
    if (std::abs(l2) < 1e-13 && p->s2_remedy == 0.0) return WC_E_SINGULAR_S2;
  }
  for (int q = 0; q < n / 2; ++q) {  // kept frequencies l = q + 1
    const int l = q + 1;
    const std::complex<double> e = std::polar(1.0, (p->zeta - 2.0 * M_PI * l) / n);
    const std::complex<double> l1 = 1.0 - e;
    std::complex<double> l2 = p->theta + (1.0 - p->theta) * e;
    if (std::abs(l2) < 1e-13) l2 = p->s2_remedy;
    const std::complex<double> lv = l1 / l2;
    lam[2 * q] = lv.real();
    lam[2 * q + 1] = lv.imag();
  }
  for (int k = 0; k < n; ++k) {
    dtw[2 * k] = std::cos(p->zeta * k / n);
    dtw[2 * k + 1] = std::sin(p->zeta * k / n);
    twt[2 * k] = std::cos(2.0 * M_PI * k / n);
    twt[2 * k + 1] = -std::sin(2.0 * M_PI * k / n);
  }
  for (int k = 0; k < N1; ++k) {
    tws[2 * k] = std::cos(2.0 * M_PI * k / N1);
    tws[2 * k + 1] = -std::sin(2.0 * M_PI * k / N1);
    sn[k] = std::sin(M_PI * k / N1);
  }
  for (int j = 0; j < M; ++j) {
    if (p->fem) {  // linear elements: U M1 U and U K1 U diagonal; mu = their ratio
      const double c = std::cos((j + 1) * M_PI * p->h);
      mass[j] = p->h / 3.0 * (2.0 + c);
      mu[j] = p->kappa * (2.0 / p->h * (1.0 - c)) / mass[j];
    } else if (p->neumann) {  // cosine k = j: 4 kappa h^-2 sin^2(k pi h/2), k = 0..M-1
      const double sv = std::sin(j * M_PI * p->h / 2.0);
      mu[j] = 4.0 * p->inv_h2 * sv * sv;
    } else {
      const double sv = std::sin((j + 1) * M_PI * p->h / 2.0);
      mu[j] = 4.0 * p->inv_h2 * sv * sv;
    }
  }
  hipError_t e = hipSuccess;
  const std::vector<float> lam32 = to_f32(lam), twt32 = to_f32(twt), tws32 = to_f32(tws),
                           sn32 = to_f32(sn), mu32 = to_f32(mu);
#define WC_UP(dst, src)                 \
  if (e == hipSuccess) e = upload(p->stream, &p->dst, src);
  WC_UP(d_lam64, lam) WC_UP(d_dtw, dtw) WC_UP(d_twt64, twt) WC_UP(d_tws64, tws)
  WC_UP(d_sin64, sn) WC_UP(d_mu64, mu)
  WC_UP(d_lam32, lam32) WC_UP(d_twt32, twt32) WC_UP(d_tws32, tws32)
  WC_UP(d_sin32, sn32) WC_UP(d_mu32, mu32)
  if (p->fem) WC_UP(d_mass64, mass)
  std::vector<float> cs32, phi32, lamf32;
  std::vector<double> phi, lamf;
  if (p->general) {
    // Phi[l][k] = e^{i zeta k/n} e^{-2 pi i k l/n}; its inverse (1/n) e^{-i zeta k/n}
    // e^{2 pi i k l/n}; lambda_l = lambda^(1)_l / lambda^(2)_l of every frequency (remedy)
    phi.resize(4 * (size_t)n * n);
    for (int l = 0; l < n; ++l)
      for (int k = 0; k < n; ++k) {
        const double a = p->zeta * k / n - 2.0 * M_PI * (double)(((long)k * l) % n) / n;
        const size_t f = 2 * ((size_t)l * n + k), b = 2 * ((size_t)n * n + (size_t)k * n + l);
        phi[f] = std::cos(a);
        phi[f + 1] = std::sin(a);
        phi[b] = std::cos(a) / n;
        phi[b + 1] = -std::sin(a) / n;
      }
    lamf.resize(2 * (size_t)n);
    for (int l = 0; l < n; ++l) {
      const std::complex<double> e1 = std::polar(1.0, (p->zeta - 2.0 * M_PI * l) / n);
      std::complex<double> l2 = p->theta + (1.0 - p->theta) * e1;
      if (std::abs(l2) < 1e-13) l2 = p->s2_remedy;
      const std::complex<double> lv = (1.0 - e1) / l2;
      lamf[2 * l] = lv.real();
      lamf[2 * l + 1] = lv.imag();
    }
    phi32 = to_f32(phi);
    lamf32 = to_f32(lamf);
    WC_UP(d_phi64, phi) WC_UP(d_phi32, phi32) WC_UP(d_lamf64, lamf) WC_UP(d_lamf32, lamf32)
    if (!p->neumann) {  // Dirichlet: the orthonormal sine matrix U = U^{-1} both ways
      cs.resize(2 * (size_t)M * M);
      for (int j = 0; j < M; ++j)
        for (int k = 0; k < M; ++k) {
          const long r = ((long)(j + 1) * (k + 1)) % (2L * (M + 1));
          const double u = std::sqrt(2.0 / (M + 1)) * std::sin(M_PI * (double)r / (M + 1));
          cs[(size_t)j * M + k] = cs[(size_t)M * M + (size_t)j * M + k] = u;
        }
      cs32 = to_f32(cs);
      WC_UP(d_cos64, cs) WC_UP(d_cos32, cs32)
    }
  }
  if (p->neumann) {  // C[j][k] = cos(j k pi/(M-1)), then C^{-1} = (2/(M-1)) W C W
    const int L = M - 1;
    cs.resize(2 * (size_t)M * M);
    for (int j = 0; j < M; ++j)
      for (int k = 0; k < M; ++k) {
        const long r = ((long)j * k) % (2L * L);  // exact angle reduction
        const double c = std::cos(M_PI * (double)r / L);
        const double w = (j == 0 || j == L ? 0.5 : 1.0) * (k == 0 || k == L ? 0.5 : 1.0);
        cs[(size_t)j * M + k] = c;
        cs[(size_t)M * M + (size_t)j * M + k] = 2.0 / L * w * c;
      }
    cs32 = to_f32(cs);
    WC_UP(d_cos64, cs) WC_UP(d_cos32, cs32)
  }
#undef WC_UP
  // low-rank GMRES: S_n - B_n = -omega g r^T with omega = e^{i zeta} = -1 (zeta = pi):
  // g = e_1 + (1 - theta) B_n e_1, r_k = q^{n-k} / (theta + omega (1 - theta) q^{n-1}),
  // q = -(1 - theta)/theta (k = 1..n; the wrap-around corners of S^(1), S^(2))
  std::vector<double> gr, rho, rk;  // alive until the uploads below are synchronised
  p->lr_ok = false;
  if (p->opts.lowrank) {
    const double th = p->theta, q = -(1.0 - th) / th;
    gr.assign(2 * (size_t)n, 0.0);
    std::vector<double> z(n, 0.0);  // B_n e_1 = (B^(2))^{-1} (e_1 - e_2)
    for (int k = 0; k < n; ++k) {
      const double rhs = k == 0 ? 1.0 : (k == 1 ? -1.0 : 0.0);
      z[k] = (rhs - (k > 0 ? (1.0 - th) * z[k - 1] : 0.0)) / th;
    }
    for (int k = 0; k < n; ++k) gr[k] = (k == 0 ? 1.0 : 0.0) + (1.0 - th) * z[k];
    const double den = th - (1.0 - th) * std::pow(q, n - 1);
    double g2 = 0.0, r2 = 0.0;
    for (int k = 0; k < n; ++k) {
      gr[n + k] = std::pow(q, n - 1 - k) / den;
      g2 += gr[k] * gr[k];
      r2 += gr[n + k] * gr[n + k];
    }
    // the remedied singular S^(2) (theta = 1/2, n odd) breaks the rank-one form
    p->lr_ok = std::fabs(den) > 1e-12 && std::isfinite(g2) && std::isfinite(r2) && p->pc_ok;
    p->lr_gn = std::sqrt(g2);
    p->lr_rn = std::sqrt(r2);
    if (e == hipSuccess) e = upload(p->stream, &p->d_lr_gr, gr);
    // contraction weights on the kept frequencies l = q + 1:
    //   rho_r[q] = sum_k r_k e^{-i zeta k/n} e^{2 pi i k l/n}, rho_g likewise with g
    rho.assign(2 * (size_t)n, 0.0);
    for (int q = 0; q < n / 2; ++q) {
      std::complex<double> ar = 0.0, ag = 0.0;
      for (int k = 0; k < n; ++k) {
        const std::complex<double> ph =
            std::polar(1.0, -p->zeta * k / n + 2.0 * M_PI * k * (q + 1) / n);
        ar += gr[n + k] * ph;
        ag += gr[k] * ph;
      }
      rho[2 * q] = ar.real();
      rho[2 * q + 1] = ar.imag();
      rho[n + 2 * q] = ag.real();
      rho[n + 2 * q + 1] = ag.imag();
    }
    if (e == hipSuccess) e = upload(p->stream, &p->d_lr_rho, rho);
    if (p->dims == 2) {
      // spectra of the rank-one terms as the time transform stores them: with
      // G_l = sum_k e^{i zeta k/n} g_k e^{-2 pi i k l/n} (R_l likewise with r), the input
      // [g (x) a1; r (x) a2] packs to Z_l = G_l a1 + i R_l a2, and the kept frequency
      // l = q + 1 with its partner -q stores A = (Z_{q+1} + conj Z_{-q})/2 and
      // -i D, D = (Z_{q+1} - conj Z_{-q})/2; a1, a2 are real, so per half two complex
      // factors multiply a1 and a2
      using C = std::complex<double>;
      std::vector<C> G(n), R(n);
      for (int l = 0; l < n; ++l) {
        C sg = 0.0, sr = 0.0;
        for (int k = 0; k < n; ++k) {
          const C ph = std::polar(1.0, p->zeta * k / n - 2.0 * M_PI * (double)((long)k * l % n) / n);
          sg += gr[k] * ph;
          sr += gr[n + k] * ph;
        }
        G[l] = sg;
        R[l] = sr;
      }
      const C I(0.0, 1.0);
      rk.assign(4 * (size_t)n, 0.0);
      for (int q = 0; q < n / 2; ++q) {
        const int lp = q + 1, lm = (n - q) % n;
        const C f[4] = {(G[lp] + std::conj(G[lm])) * 0.5,        // half A, times a1
                        I * (R[lp] - std::conj(R[lm])) * 0.5,     // half A, times a2
                        -I * (G[lp] - std::conj(G[lm])) * 0.5,    // half -iD, times a1
                        (R[lp] + std::conj(R[lm])) * 0.5};        // half -iD, times a2
        for (int t = 0; t < 4; ++t) {
          rk[8 * (size_t)q + 2 * t] = f[t].real();
          rk[8 * (size_t)q + 2 * t + 1] = f[t].imag();
        }
      }
      if (e == hipSuccess) e = upload(p->stream, &p->d_lr_rank, rk);
    }
  }
  std::vector<double> af;
  if (e == hipSuccess && prob->a_face_host) {
    const size_t nf = p->dims == 1 ? (size_t)M + 1 : 2 * (size_t)M * (M + 1);
    af.assign(prob->a_face_host, prob->a_face_host + nf);
    e = upload(p->stream, &p->d_aface, af);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? WC_E_NOMEM : WC_E_HIP;
  }
  return WC_OK;
}

}  // namespace

extern "C" {

const char *wc_version(void) { return "libwcirc 0.1 gfx950"; }

wc_status wc_profile(wc_plan *plan, int enable) {
  if (!plan) return WC_E_ARG;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return WC_E_HIP;
  if (enable) {  // recycle the previous recording's events, start a new one
    for (auto &r : plan->prof.recs) {
      if (r.a) plan->prof.pool.push_back(r.a);
      if (r.b) plan->prof.pool.push_back(r.b);
    }
    plan->prof.recs.clear();
  }
  plan->prof.on = enable != 0;
  return WC_OK;
}

int wc_profile_read(wc_plan *plan, wc_kernel_stat *out, int max) {
  if (!plan || (!out && max > 0)) return -1;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return -1;
  int launches[K_COUNT] = {0};
  double ms[K_COUNT] = {0};
  double bytes[K_COUNT] = {0};
  for (const auto &r : plan->prof.recs) {
    float t = 0.f;
    if (r.a && r.b && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess && r.kid >= 0 &&
        r.kid < K_COUNT) {
      launches[r.kid] += 1;
      ms[r.kid] += t;
      bytes[r.kid] += r.bytes;
    }
  }
  int cnt = 0;
  for (int k = 0; k < K_COUNT; ++k) {
    if (!launches[k]) continue;
    if (cnt < max) {
      std::memset(&out[cnt], 0, sizeof(wc_kernel_stat));
      std::strncpy(out[cnt].name, kernel_name(k), sizeof(out[cnt].name) - 1);
      out[cnt].launches = launches[k];
      out[cnt].total_ms = ms[k];
      out[cnt].bytes = bytes[k];
    }
    ++cnt;
  }
  return cnt < max ? cnt : max;
}

const char *wc_status_str(int s) {
  switch (s) {
    case WC_OK: return "ok";
    case WC_E_ARG: return "invalid argument";
    case WC_E_SINGULAR_S2: return "S_n^(2) singular and no remedy value";
    case WC_E_NOMEM: return "device allocation failed";
    case WC_E_MAXIT: return "maximum iterations reached";
    case WC_E_BREAKDOWN: return "Krylov breakdown";
    case WC_E_NONFINITE: return "non-finite value";
    case WC_E_CANCELLED: return "cancelled";
    case WC_E_ADMISSION: return "admission refused";
    case WC_E_UNSUPPORTED: return "unsupported by the GPU path";
    case WC_E_HIP: return "HIP runtime error";
    default: return "internal error";
  }
}

void wc_opts_default(wc_opts *o) {
  if (!o) return;
  o->method = WC_GMRES_PS;
  o->precision = WC_FP64;
  o->tol = 1e-8;
  o->maxit = 500;
  o->restart = 30;
  o->flexible = 0;
  o->mg_max_cycles = 30;
  o->mg_tol = 1e-10;
  o->graphs = 1;
  o->lowrank = 0;
}

size_t wc_plan_footprint_bytes(const wc_problem *prob, const wc_opts *opts) {
  if (validate(prob, opts) != WC_OK) return 0;
  return sizes_of(prob, opts).total;
}

wc_status wc_plan_create(const wc_problem *prob, const wc_opts *opts, void *stream,
                         wc_plan **out) {
  if (!out) return WC_E_ARG;
  *out = nullptr;
  wc_status vs = validate(prob, opts);
  if (vs != WC_OK) return vs;
  if (singular_s2_unremedied(prob)) return WC_E_SINGULAR_S2;
  // finite elements work in sine coordinates: the data transforms need the sine sizes
  if (prob->disc == WC_FEM && !pc_path_ok(prob)) return WC_E_UNSUPPORTED;
  // the low-rank form runs on the FFT path only
  if (opts->lowrank && uses_general(prob)) return WC_E_UNSUPPORTED;
  wc_plan *p = new (std::nothrow) wc_plan();
  if (!p) return WC_E_NOMEM;
  p->dims = prob->dims;
  p->M = prob->M;
  p->n = prob->n;
  p->m = prob->dims == 1 ? prob->M : prob->M * prob->M;
  p->N1 = prob->M + 1;
  p->h = 1.0 / (prob->M + 1);
  p->var_coeff = prob->a_face_host != nullptr;
  p->fem = prob->disc == WC_FEM;
  p->neumann = prob->bc == WC_NEUMANN;
  if (p->neumann) p->h = 1.0 / (prob->M - 1);  // M nodes including both boundary nodes
  p->general = uses_general(prob);
  p->stream = (hipStream_t)stream;
  p->nvec = 2 * (size_t)p->n * p->m;
  set_scalars(p, prob, opts);
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      p->num_cu = cus;
  }
  const Sizes sz = sizes_of(prob, opts);
  {
    const wc_status ts = set_tables(p, prob);
    if (ts != WC_OK) {
      free_plan(p);
      return ts;
    }
  }
  // ---- workspaces ----
  bool oom = false;
  auto alloc = [&](void **ptr, size_t bytes) {
    if (oom) return;
    if (hipMalloc(ptr, bytes) != hipSuccess) oom = true;
  };
  alloc(&p->d_specA, sz.spec_bytes);
  if (sz.spec_t_bytes && p->pc_ok) alloc(&p->d_specT, sz.spec_t_bytes);
  if (p->var_coeff) alloc(&p->d_specB, sz.spec_bytes);
  if (sz.fem_bytes) alloc((void **)&p->d_femW, sz.fem_bytes);
  if (p->neumann || p->general) alloc(&p->d_specB, sz.spec_bytes);
  alloc((void **)&p->d_partials, sz.partials * sizeof(double));
  alloc((void **)&p->d_scal, S_COUNT * sizeof(double));
  p->nkvec = krylov_vectors(prob, opts);
  alloc((void **)&p->d_vecs, (size_t)p->nkvec * p->nvec * sizeof(double));
  if (opts->lowrank) {
    p->lr_len = 1 + 2 * (size_t)p->m;
    alloc((void **)&p->d_lr_s0, 2 * (size_t)p->m * sizeof(double));
    alloc((void **)&p->d_lr_hat, (size_t)(opts->restart + 2) * p->lr_len * sizeof(double));
    alloc((void **)&p->d_lr_part,
          (size_t)std::max(kContractChunks, kColChunks) * 2 * p->m * sizeof(double));
    if (p->dims == 2) {  // (the rank-term spectra were uploaded with the tables)
      p->lr_2d = true;
      alloc((void **)&p->d_lr_a, 2 * (size_t)p->m * sizeof(double));
    }
  }
  if (!oom && hipHostMalloc((void **)&p->h_scal, S_COUNT * sizeof(double), 0) != hipSuccess)
    oom = true;
  if (oom) {
    (void)hipGetLastError();
    free_plan(p);
    return WC_E_NOMEM;
  }
  std::memset(p->h_scal, 0, S_COUNT * sizeof(double));
  if (hipMemcpyAsync(p->d_scal, p->h_scal, S_COUNT * sizeof(double), hipMemcpyHostToDevice,
                     p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess) {
    free_plan(p);
    return WC_E_HIP;
  }
  if (p->var_coeff && p->pc_ok) {
    const wc_status ms = build_multigrid(p, prob->a_face_host);
    if (ms != WC_OK) {
      free_plan(p);
      return ms;
    }
  }
  p->footprint = sz.total;
  *out = p;
  return WC_OK;
}

wc_status wc_plan_destroy(wc_plan *plan) {
  if (!plan) return WC_E_ARG;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) {
    free_plan(plan);
    return WC_E_HIP;
  }
  free_plan(plan);
  return WC_OK;
}

wc_status wc_plan_retarget(wc_plan *p, const wc_problem *prob, const wc_opts *opts) {
  if (!p) return WC_E_ARG;
  wc_status vs = validate(prob, opts);
  if (vs != WC_OK) return vs;
  const wc_opts &o = p->opts;
  if (prob->dims != p->dims || prob->M != p->M || prob->n != p->n ||
      (prob->a_face_host != nullptr) != p->var_coeff || (prob->disc == WC_FEM) != p->fem ||
      (prob->bc == WC_NEUMANN) != p->neumann || uses_general(prob) != p->general ||
      opts->method != o.method ||
      opts->precision != o.precision || opts->restart != o.restart ||
      opts->flexible != o.flexible || opts->lowrank != o.lowrank)
    return WC_E_ARG;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return WC_E_HIP;
  drop_graphs(p);  // captured launches hold the old scalars
  set_scalars(p, prob, opts);
  wc_status st = set_tables(p, prob);
  if (st == WC_OK && p->var_coeff && p->pc_ok) st = build_multigrid(p, prob->a_face_host);
  if (st != WC_OK) p->pc_ok = false;  // tables may be half written: refuse solves
  return st;
}

wc_status wc_plan_autotune(wc_plan *p, int reps, int *ts_out, int *tx_out) {
  if (!p || reps < 1) return WC_E_ARG;
  if (!p->pc_ok) return WC_E_UNSUPPORTED;
  double *v = p->vec(0), *w = p->vec(1);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return WC_E_HIP;
  const bool prof = p->prof.on;
  p->prof.on = false;
  WC_TRY(launch_fill(*p, v, 1.0, p->nvec));
  // time-FFT tile widths; x2 pass: column tiles of 4, 8, 16, or the transposed rows in
  // x1 tiles of 4 or 8 rows (tx < 0, when the plan holds the transposed copy)
  // time passes: packed tiles of 4, 8, 16 columns, or per-block-row tiles of 8, 16, 32 (< 0)
  const int tss[6] = {4, 8, 16, -8, -16, -32}, txs[5] = {4, 8, 16, -4, -8};
  const int nts = p->general ? 1 : (p->n >= 64 ? 6 : 3);
  // (finite elements: no sine passes in the preconditioner, only the time tiles matter)
  const int ntx = (p->dims == 2 && !p->var_coeff && !p->fem && !p->neumann) ? (p->d_specT ? 5 : 3) : 1;
  float best = -1.f;
  int bts = p->ts_time, btx = p->tx_cols;
  hipError_t e = hipSuccess;
  for (int it = 0; it < nts && e == hipSuccess; ++it)
    for (int ix = 0; ix < ntx && e == hipSuccess; ++ix) {
      p->ts_time = tss[it];
      p->tx_cols = ntx > 1 ? txs[ix] : 0;
      e = launch_pc_apply(*p, v, w, false, nullptr);
      if (e == hipSuccess) e = hipEventRecord(a, p->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_pc_apply(*p, v, w, false, nullptr);
      if (e == hipSuccess) e = hipEventRecord(b, p->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e == hipSuccess && (best < 0.f || ms < best)) {
        best = ms;
        bts = p->ts_time;
        btx = p->tx_cols;
      }
    }
  p->ts_time = bts;
  p->tx_cols = btx;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  p->prof.on = prof;
  drop_graphs(p);  // captured launches hold the previous kernel choice
  if (e != hipSuccess) return WC_E_HIP;
  if (ts_out) *ts_out = bts;
  if (tx_out) *tx_out = btx;
  return WC_OK;
}

wc_status wc_plan_set_tiles(wc_plan *p, int ts, int tx) {
  if (!p) return WC_E_ARG;
  const bool ts_ok =
      ts == 0 || ts == 4 || ts == 8 || ts == 16 || ts == -8 || ts == -16 || ts == -32;
  const bool tx_ok = tx == 0 || tx == 4 || tx == 8 || tx == 16 ||
                     ((tx == -4 || tx == -8) && p->d_specT);
  if (!ts_ok || !tx_ok) return WC_E_ARG;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return WC_E_HIP;
  p->ts_time = ts;
  p->tx_cols = tx;
  drop_graphs(p);  // captured launches hold the previous kernel choice
  return WC_OK;
}

wc_status wc_plan_set_stream(wc_plan *plan, void *stream) {
  if (!plan) return WC_E_ARG;
  // the plan's work so far is ordered on the old stream: finish it before switching
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return WC_E_HIP;
  plan->stream = (hipStream_t)stream;
  return WC_OK;
}

wc_status wc_rhs(wc_plan *plan, const double *f, const double *g, const double *y0, double *b) {
  if (!plan || !f || !g || !y0 || !b) return WC_E_ARG;
  WC_TRY(launch_rhs(*plan, f, g, y0, b));
  return WC_OK;
}

wc_status wc_matvec(wc_plan *plan, const double *x, double *y) {
  if (!plan || !x || !y || x == y) return WC_E_ARG;
  WC_TRY(launch_matvec(*plan, x, y, plan->d_partials, nullptr));
  return WC_OK;
}

wc_status wc_pc_apply(wc_plan *plan, const double *v, double *w) {
  if (!plan || !v || !w) return WC_E_ARG;
  if (!plan->pc_ok) return WC_E_UNSUPPORTED;
  WC_TRY(launch_pc_apply(*plan, v, w, false, nullptr));
  return WC_OK;
}

wc_status wc_recover(wc_plan *plan, const double *x, double *y, double *p, double *u) {
  if (!plan || !x || !y || !p) return WC_E_ARG;
  WC_TRY(launch_recover(*plan, x, y, p, u));
  return WC_OK;
}

wc_status wc_krylov(wc_plan *plan, const double *b, double *x, wc_info *info) {
  if (!plan || !b || !x || b == x) return WC_E_ARG;
  if (!plan->pc_ok) return WC_E_UNSUPPORTED;
  wc_info local{};
  wc_info *inf = info ? info : &local;
  std::memset(inf, 0, sizeof(*inf));
  const auto t0 = std::chrono::steady_clock::now();
  plan->mg_cycles_max = 0;
  wc_status st = plan->opts.method == WC_GMRES_PS ? run_gmres(plan, b, x, inf)
                                                  : run_minres(plan, b, x, inf);
  if (hipStreamSynchronize(plan->stream) != hipSuccess) st = WC_E_HIP;
  const auto t1 = std::chrono::steady_clock::now();
  inf->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  inf->mg_cycles_max = plan->mg_cycles_max;
  if (plan->var_coeff && plan->opts.mg_tol == 0.0) inf->mg_cycles_max = plan->opts.mg_max_cycles;
  inf->status = st;
  return st;
}

wc_status wc_solve(wc_plan *plan, const double *f, const double *g, const double *y0, double *y,
                   double *p, double *u, wc_info *info) {
  if (!plan || !f || !g || !y0 || !y || !p) return WC_E_ARG;
  if (!plan->pc_ok) return WC_E_UNSUPPORTED;
  double *B = plan->vec(plan->nkvec - 2);
  double *X = plan->vec(plan->nkvec - 1);
  WC_TRY(launch_rhs(*plan, f, g, y0, B));
  wc_status st = wc_krylov(plan, B, X, info);
  if (st != WC_OK && st != WC_E_MAXIT) return st;
  WC_TRY(launch_recover(*plan, X, y, p, u));
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return WC_E_HIP;
  return st;
}

}  // extern "C"
