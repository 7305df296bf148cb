// Internal declarations shared by the HIP translation units of libwcirc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/wc.h"

// in a function returning wc_status: a failed HIP call returns WC_E_HIP
#define WC_TRY(expr)                                          \
  do {                                                        \
    hipError_t _e = (expr);                                   \
    if (_e != hipSuccess) return WC_E_HIP;                    \
  } while (0)

namespace wc {

constexpr int kThreads = 256;        // threads per workgroup for every kernel
constexpr int kRedBlocks = 1024;     // max workgroups of the streaming reductions
constexpr int kMaxRestart = 32;
// GMRES second Gram-Schmidt pass when the first pass leaves less than this
// fraction of the squared norm of E v_j (E = Ahat P^{-1} - I).  With the shift
// the drop reflects the convergence rate, not the preconditioner's quality; a
// hundredfold drop in norm costs about two digits of orthogonality.
constexpr double kReorthEta2 = 1e-4;
// Low-rank GMRES with the FP32 preconditioner: relative reduction a restart cycle aims for
// (about twenty FP32 unit roundoffs: below it the FP32 apply's own error dominates)
constexpr double kMixedCycleDrop = 1e-6;
// multigrid (variable a): LDS budget of the single-workgroup coarse cycle, capacity of
// the per-system norm partials, and the floor of the cycle tolerance in FP32
constexpr size_t kMgLdsBytes = 60 * 1024;
constexpr int kMgPartials = 32768;
constexpr double kMgTolFp32 = 1e-5;
constexpr int kMgMaxLevels = 12;
constexpr int kMaxPartials = 1 << 16;

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

// ---- device-side scalar state of the Krylov solvers ------------------------
// A small FP64 array in device memory; kernels read their coefficients from it
// so no host round trip is needed between the steps of one iteration.
enum ScalarSlot : int {
  // MINRES state
  S_GAMMA_PREV = 0, S_GAMMA, S_DELTA, S_ETA, S_C_PREV, S_C, S_S_PREV, S_S,
  S_BNORM, S_RNORM2, S_STATUS, S_ITER,
  // v update:  v_new = c0*Az + c1*v + c2*v_prev
  S_CV0 = 16, S_CV1, S_CV2,
  // w/x/r update
  S_CWZ = 20, S_CW0, S_CW1, S_CX, S_CRR, S_CRV,
  // GMRES: classical Gram-Schmidt with a DGKS-triggered second pass; basis vectors are
  // stored unnormalised and their squared norms kept here
  S_WN2 = 32,    // ||w||^2 before projection
  S_WP2,         // ||w'||^2 after the first projection
  S_WPP2,        // ||w''||^2 after the second projection (when taken)
  S_REORTH,      // 1 when the second projection is needed
  S_NU2 = 64,    // kMaxRestart+1 squared norms of the stored basis vectors
  S_D1 = 104,    // kMaxRestart+1 raw dots <V_i, w>, first pass
  S_D2 = 144,    // second pass
  S_GSC = 184,   // kMaxRestart+1 projection coefficients of the current pass
  S_Y = 224,     // kMaxRestart update coefficients
  S_DOT = 300,   // scratch dot results
  S_MG_RELRES = 310,  // largest relative residual over the multigrid systems
  S_LR_N0 = 320,      // low-rank GMRES: squared norm of r0's part outside the correction's range
  S_LR_SQN0,          //   its square root (0 when that part vanishes)
  S_GS_COUNT = 330,   // Gram-Schmidt reductions: workgroups done (an unsigned counter, 0 at rest)
  S_COUNT = 512
};

enum SolveStatusCode : int { ST_RUNNING = 0, ST_CONVERGED = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3 };

// kernel families for the optional event timing
enum KernelId : int {
  K_TFFT_FWD = 0, K_DST_X1_FWD, K_PAIR_MODE, K_DST_X1_INV, K_TFFT_INV, K_MATVEC, K_RHS,
  K_RECOVER, K_LINCOMB, K_DOT, K_FINALIZE, K_MINRES_UPDATE, K_MINRES_SCALAR, K_MULTIDOT,
  K_MULTIAXPY, K_SCALE, K_FILL, K_MULTIDOT_RE, K_MULTIAXPY_RE, K_MG_SMOOTH, K_MG_RESTRICT,
  K_MG_LDS, K_MG_NORM, K_MG_MIX, K_LR_SETUP, K_CONTRACT, K_PAIR_CONTRACT, K_DST_X2_FWD, K_COUNT
};
const char *kernel_name(int id);

struct ProfRec {
  int kid;
  double bytes;  // algorithmic HBM bytes the launch must move
  hipEvent_t a, b;
};

struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  // the launch ran but did no work (a device-gated pass): it moved no bytes
  void void_last(int kid) {
    for (auto it = recs.rbegin(); it != recs.rend(); ++it)
      if (it->kid == kid) { it->bytes = 0.0; return; }
  }
};

}  // namespace wc

struct wc_plan {
  // problem
  int dims = 1, M = 0, n = 0, m = 0, N1 = 0;
  double T = 1, theta = 1, gamma = 1, zeta = 0, s2_remedy = 1;
  double tau = 0, alpha = 0, h = 0, inv_h2 = 0;
  bool var_coeff = false;
  bool fem = false;              // finite elements (a == 1): the system in sine coordinates
  bool neumann = false;          // Neumann data: M nodes incl. the boundary, dense cosine steps
  bool general = false;          // sizes / zeta outside the FFT path: dense steps throughout
  double kappa = 1;              // constant a (folded into inv_h2 and the eigenvalue tables)
  bool pc_ok = false;            // the GPU preconditioner covers this problem
  int num_cu = 256;              // compute units of the plan's device
  int ts_time = 0;               // time passes: > 0 packed tile width, < 0 per-block-row
                                 // tile width (n >= 64), 0: default
  int tx_cols = 0;               // x2 pass: > 0 column tile width, < 0 transposed rows with
                                 // -tx_cols rows per x1 tile (0: default)
  wc_opts opts{};
  hipStream_t stream = nullptr;
  size_t nvec = 0;          // 2*n*m
  // device tables
  double *d_aface = nullptr;     // face coefficients (variable a) or null
  double *d_lam64 = nullptr;     // n/2 complex: eigenvalues of S_n at kept frequencies
  float *d_lam32 = nullptr;
  double *d_dtw = nullptr;       // n complex: omega^{k/n} = e^{i zeta k/n}
  double *d_twt64 = nullptr;     // n complex: e^{-2 pi i p/n}
  float *d_twt32 = nullptr;
  double *d_tws64 = nullptr;     // N1 complex: e^{-2 pi i p/N1}
  float *d_tws32 = nullptr;
  double *d_sin64 = nullptr;     // N1 reals: sin(pi i/N1)
  float *d_sin32 = nullptr;
  double *d_mu64 = nullptr;      // M reals: eigenvalues of the 1D -L_h (a == 1), or of
  float *d_mu32 = nullptr;       //   M1^{-1/2} K1 M1^{-1/2} (finite elements)
  double *d_mass64 = nullptr;    // finite elements: M eigenvalues of the 1D mass matrix
  double *d_femW = nullptr;      // finite elements: n*m complex FP64, the sine transforms
                                 // of the data and of the solution
  double *d_cos64 = nullptr;     // dense spatial steps: 2 M*M reals, the basis matrix then its
  float *d_cos32 = nullptr;      //   inverse (row-major [j][k]): C, C^{-1} or U, U
  double *d_phi64 = nullptr;     // general path: 2 n*n complex, Phi = F diag(omega^{k/n}) then
  float *d_phi32 = nullptr;      //   its inverse (row-major)
  double *d_lamf64 = nullptr;    // general path: n complex, lambda_l of every frequency
  float *d_lamf32 = nullptr;
  // workspaces
  void *d_specA = nullptr;       // n*m complex (P): spectral array, layout [q][half][x2][x1]
  void *d_specB = nullptr;       // n*m complex (P): multigrid fine solution (variable a)
  void *d_specT = nullptr;       // 2D, a == 1, N1 >= 128: the spectrum after the x1 pass,
                                 // transposed, [q][half][j1][x2] with row stride N1
  double *d_partials = nullptr;  // reduction partials
  double *d_scal = nullptr;      // Krylov scalars (wc::S_COUNT)
  double *h_scal = nullptr;      // pinned host mirror
  // Krylov vectors: one allocation of nvecs * nvec doubles
  double *d_vecs = nullptr;
  int nkvec = 0;
  size_t footprint = 0;
  // multigrid hierarchy (variable a); level 0 is the fine grid, the last has M = 1
  int mg_nlev = 0;
  int mg_ltop = 0;                        // first level cycled inside LDS
  int mg_M[wc::kMgMaxLevels] = {};
  double mg_inv_h2[wc::kMgMaxLevels] = {};
  size_t mg_aoff[wc::kMgMaxLevels] = {};  // level l's faces at d_mg_a + mg_aoff[l] (l >= 1)
  // level l >= 1 at d_mg_work + mg_woff[l] bytes: u, then (2D) a second u, then f
  size_t mg_woff[wc::kMgMaxLevels] = {};
  void *d_mg_u2 = nullptr;                // 2D: second fine solution buffer
  mutable int mg_cur[wc::kMgMaxLevels] = {};  // 2D: which u buffer holds the current values
  double *d_mg_a = nullptr;
  void *d_mg_work = nullptr;
  double *d_mg_shift = nullptr;           // n complex: shift of each system
  double *d_mg_mix = nullptr;             // n/2 x 6: rotation of the two block rows (P_S)
  double *d_mg_fn2 = nullptr;             // n: squared right-hand side norms
  mutable int mg_cycles_last = 0, mg_cycles_max = 0;
  // low-rank GMRES (a = 1, FP64, GMRES-P_S): Ahat - P_S = -diag(D, D^T) (x) I with
  // D = S_n - B_n = -omega g r^T; the Krylov basis lives in compact coordinates
  bool lr_ok = false;
  double lr_gn = 0, lr_rn = 0;      // |g|, |r|
  size_t lr_len = 0;                // 1 + 2m
  double *d_lr_gr = nullptr;        // 2n: g then r
  double *d_lr_s0 = nullptr;        // 2m
  double *d_lr_hat = nullptr;       // (restart + 2) compact vectors of lr_len
  double *d_lr_rho = nullptr;       // n complex: contraction weights per kept frequency
  double *d_lr_part = nullptr;      // max(kContractChunks, kColChunks) x 2m
  // 2D: the time and sine transforms are linear and r0 is fixed within a cycle, so the
  // Arnoldi steps take the spectrum of c r0 + [g (x) a1; r (x) a2] from these instead of
  // transforming (the time, x1 and x2 transforms of r0 sit in d_specA for the cycle)
  bool lr_2d = false;               // 2D low-rank GMRES
  double *d_lr_rank = nullptr;      // n/2 x 2 halves x 2 complex: spectra of g and of r
  double *d_lr_a = nullptr;         // m complex: a1 + i a2 of the current vector, sine-transformed

  mutable wc::Profiler prof;
  // captured Krylov iterations: GMRES step j in slot j (first restart cycle) or
  // kMaxRestart + j (later cycles), the two MINRES buffer arrangements in the last two;
  // key = the caller pointer the work also depends on
  static constexpr int kGraphSlots = 2 * wc::kMaxRestart + 2;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[kGraphSlots] = {};
  const void *gkey[kGraphSlots] = {};
  bool graphs_failed = false;

  double *vec(int i) const { return d_vecs + (size_t)i * nvec; }
};

namespace wc {
// Records an event pair around the launches in its scope when profiling is on.
struct ProfScope {
  const wc_plan &p;
  int kid;
  double bytes;
  hipEvent_t a = nullptr;
  ProfScope(const wc_plan &pl, int k, double nbytes) : p(pl), kid(k), bytes(nbytes) {
    if (p.prof.on) {
      a = p.prof.get();
      (void)hipEventRecord(a, p.stream);
    }
  }
  ~ProfScope() {
    if (p.prof.on && a) {
      hipEvent_t b = p.prof.get();
      (void)hipEventRecord(b, p.stream);
      p.prof.recs.push_back({kid, bytes, a, b});
    }
  }
};
}  // namespace wc

namespace wc {

// ---- low-rank GMRES ---------------------------------------------------------
// Compact input (low-rank GMRES): the system vector is generated on the fly from the
// compact coordinates h = [sqrt(N0) c; |g| s1; |r| s2] of c r0_perp + [g (x) s1; r (x) s2],
// r0_perp = r0 - [g (x) s0_1; r (x) s0_2]:
//   v1[k][s] = c r0_1[k][s] + g_k (s1[s] - c s0_1[s]),  v2 likewise with r_k and s2.
struct GenIn {
  const double *hat;    // compact coordinates (1 + 2m)
  const double *s0;     // 2m: projection coefficients of r0 on the range of the correction
  const double *gr;     // 2n: g_k then r_k
  const double *sqn0;   // device scalar: sqrt(N0) (0 when r0 lies in that range)
  double inv_gn, inv_rn;
};

// Contracted output (low-rank GMRES): instead of z, the compact coordinates of
// (Ahat - P_S) z = omega [g (x) sum_k r_k z1_k; r (x) sum_k g_k z2_k]:
//   hat[0] = 0, hat[1+s] = |g| omega sum_k r_k z1[k][s], hat[1+m+s] = |r| omega sum_k g_k z2[k][s].
// The time sums are taken on the spectrum, before the inverse time transform: for real z
// with the half spectrum Z_q (frequency l = q + 1; its partner 1 - l carries conj(Z_q)),
//   sum_k r_k z_k = sum_q 2 Re(rho_q Z_q),  rho_q = sum_k r_k conj(omega^{k/n}) e^{2 pi i k (q+1)/n}.
struct ContractOut {
  double *hat;
  double gn_omega, rn_omega;
  const double *rho;   // n complex: rho_r[q] then rho_g[q], q < n/2 (frequency l = q + 1)
  double *part;        // chunks x 2m partial sums (1D: kContractChunks, 2D: kColChunks)
};
// frequency chunks of the contraction kernels (deterministic two-stage sums): 1D, and the
// 2D pointwise step (its grid is chunks x m / 256 workgroups; 8 measured faster than 16)
constexpr int kContractChunks = 8;
constexpr int kColChunks = 8;


// ---- launchers (wc_ops.hip) -------------------------------------------------
// Step 2 for variable a: batched multigrid on d_specA (in/out), d_specB = fine solution.
hipError_t mg_space_apply(const wc_plan &p);
// LDS bytes of a cycle over the pyramid from an M-point level down to M = 1
size_t mg_lds_bytes(int dims, int M, int precision);
// y = Ahat x (GMRES layout) or A x (MINRES layout); with sub, y = (.) x - sub, or
// sub - (.) x with negate (a residual in one pass).
hipError_t launch_matvec(const wc_plan &p, const double *x, double *y, double *partials,
                         int *nblocks_out, const double *sub = nullptr, bool negate = false);
hipError_t launch_rhs(const wc_plan &p, const double *f, const double *g, const double *y0,
                      double *b);
hipError_t launch_recover(const wc_plan &p, const double *x, double *y, double *pp, double *u);
// finite elements: b holds the right-hand side combinations of the two block rows without
// the y0 terms (physical); into sine coordinates with M^{-1/2} M = M^{1/2}, plus the y0 terms
hipError_t launch_fem_rhs_finish(const wc_plan &p, const double *y0, double *b);
// finite elements: y, p hold the recovered solution in sine coordinates without the
// M^{-1/2} scaling; into physical nodal values (and u = p/gamma when u is not null)
hipError_t launch_fem_recover_finish(const wc_plan &p, double *y, double *pp, double *u);

int red_blocks(size_t n);
// dst[i] = c0*a + c1*b + c2*c, coefficient k read from d_scal[slot + k] (slot < 0: host c*)
hipError_t launch_lincomb3(const wc_plan &p, double *dst, const double *a, const double *b,
                           const double *c, int slot, double h0, double h1, double h2);
// partials of <a, b> (one per block) -> finalize into d_scal[slot]
// sum_i a_i b_i over the system vector as partial sums in d_partials (count in *nparts)
hipError_t launch_dot_partials(const wc_plan &p, const double *a, const double *b, int *nparts);
hipError_t launch_dot(const wc_plan &p, const double *a, const double *b, int slot,
                      size_t len = 0);
hipError_t launch_finalize(const wc_plan &p, const double *partials, int count, int nsum,
                           int slot);
hipError_t launch_minres_update(const wc_plan &p, double *w0, const double *w1,
                                const double *z, double *x, double *r, const double *vnew);
hipError_t launch_minres_scalar(const wc_plan &p, int stage, int nparts, double tol);
// <basis_i, w> for i < nb (plus <w, w> when self) -> partials [sum][block]; *nblocks out.
// gate (device pointer or null): the launch does nothing when *gate == 0.
// len: vector length and basis stride (0: a system vector)
hipError_t launch_multidot(const wc_plan &p, const double *basis, int nb, const double *w,
                           bool self, const double *gate, int *nblocks, size_t len = 0);
// w += sign * sum_i scal[slot+i] basis_i; partials of ||w||^2 when norm.
hipError_t launch_multiaxpy(const wc_plan &p, double *w, const double *basis, int nb,
                            int slot, double sign, bool norm, const double *gate,
                            int *nblocks, size_t len = 0);
// Gram-Schmidt bookkeeping of GMRES iteration j (one block): stage 1 first-pass dots,
// 2 first-pass norm and DGKS test, 3 second-pass dots, 4 second-pass norm.
hipError_t launch_gs_finalize(const wc_plan &p, int stage, int j, int count);
// Classical Gram-Schmidt passes of GMRES iteration j on Vn against V_0..V_j (vectors of
// length len, 0: a system vector), the second gated on the device by the DGKS test; the
// bookkeeping of each reduction (the four gs_finalize stages) is done by the last
// workgroup of that reduction, so the passes are four launches.
// passes = 1 launches the first pass only (a caller that reads the DGKS flag on the host
// then runs launch_gs_second_pass itself when it is set).
hipError_t launch_gram_schmidt(const wc_plan &p, const double *V, int j, double *Vn,
                               size_t len = 0, int passes = 2);
hipError_t launch_gs_second_pass(const wc_plan &p, const double *V, int j, double *Vn,
                                 size_t len = 0);
hipError_t launch_fill(const wc_plan &p, double *dst, double val, size_t count);
hipError_t launch_copy(const wc_plan &p, double *dst, const double *src, size_t count);

// ---- preconditioner (wc_pc.hip) --------------------------------------------
// w = P^{-1} v.  With dot = true the last pass also writes per-block partial sums of
// <w, v> to p.d_partials[0..*nparts) (v must then not alias w).
hipError_t launch_pc_apply(const wc_plan &p, const double *v, double *w, bool dot, int *nparts);
// P^{-1} applied to the vector generated from compact coordinates hat_in (low-rank GMRES);
// hat_out != nullptr: write the compact coordinates of (Ahat - P_S) P^{-1} v there,
// else write P^{-1} v to w.
hipError_t launch_pc_lowrank(const wc_plan &p, const double *r0, const double *hat_in,
                             double *hat_out, double *w);
// s0 = projection coefficients of r0 on the correction's range; N0 = ||r0 - [g s0_1; r s0_2]||^2
// and sqrt(N0) into the scalar slots; hat = [sqrt(N0), |g| s0_1, |r| s0_2] (2D: s0 and the
// compact vectors in orthonormal sine coordinates).  Expects
// ||r0||^2 in d_scal[S_DOT] (launch_dot before).
hipError_t launch_lr_setup(const wc_plan &p, const double *r0, double *hat);
// 2D low-rank GMRES: time transform and x1 sine transform of the cycle's r0 into
// d_specA, then its x2 sine transform in place (once per cycle)
hipError_t launch_lr_spectrum(const wc_plan &p, const double *r0);
// 2D low-rank GMRES: s0 into orthonormal sine coordinates (the compact vectors of a 2D
// plan are held in them)
hipError_t launch_lr_sine_s0(const wc_plan &p);
bool pc_supported(int n, int N1);

// ---- many instances in one launch per pass (2D, a = 1) ------------------------------
// Per-instance data that stays fixed for the life of a batch (device resident): sizes,
// step-2 parameters, the instance's spectral workspace and its tables in its precision.
constexpr int kBatchMax = 32;
struct BatchInst {
  int n, N1, m, kind;
  double tau, alpha, cnorm;
  void *W;
  const void *dtw, *twt, *tws, *sin, *lam, *mu;
};
bool batch_sizes_ok(int n, int N1);
// P^{-1} v_i -> w_i for the instances idx[0..cnt) of the table, all of one precision
// (FP64 or FP32 transforms): five launches, each over every instance's work units.
hipError_t launch_pc_batch(hipStream_t st, const BatchInst *d_tab, const BatchInst *h_tab,
                           int cnt, const int *idx, const double *const *v, double *const *w,
                           bool fp32);
int pc_partials_needed(int n, int m, int precision);

}  // namespace wc

// ---- continuous batching (wc_batch.hip) -------------------------------------------------
struct LockstepEngine;
namespace wc {
// GMRES(k)-P_S solves that can join a lockstep engine: 2D, a == 1, zeta == pi, standard
// form, n and M + 1 in {64, 128, 256, 512}
bool lockstep_eligible(const wc_problem *pr, const wc_opts *op);
LockstepEngine *lockstep_create(hipStream_t st);
void lockstep_destroy(LockstepEngine *eng);
int lockstep_active(const LockstepEngine *eng);
// a solve joins (its plan's stream must be the engine's); asynchronous
hipError_t lockstep_add(LockstepEngine *eng, wc_plan *p, const double *f, const double *g,
                        const double *y0, double *y, double *pout, double *u, uint64_t tag);
struct LockstepDone {
  uint64_t tag;
  wc_plan *plan;
  wc_info info;
};
// one round; the solves that finished in it (y, p, u written) are appended to done
hipError_t lockstep_round(LockstepEngine *eng, std::vector<LockstepDone> &done);
}  // namespace wc
