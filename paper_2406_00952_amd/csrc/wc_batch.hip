// Batches: many right-hand sides and many instances of uneven (n, M) whose preconditioner
// passes run as one launch per pass over all of them, and a GMRES(k)-P_S driver that
// advances every instance of a batch in lockstep (one batched preconditioner apply and one
// host synchronisation per Arnoldi step for the whole batch).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "wc_internal.h"

using namespace wc;

struct wc_batch {
  std::vector<wc_plan *> plans;
  std::vector<BatchInst> h_tab;
  BatchInst *d_tab = nullptr;
};

namespace {

int pc_kind(const wc_plan &p) {
  return p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
}

// P^{-1} v_i -> w_i for the listed instances: one launch per pass and precision.
hipError_t batch_pc(const wc_batch &b, const std::vector<int> &idx,
                    const std::vector<const double *> &v, const std::vector<double *> &w) {
  hipStream_t st = b.plans[0]->stream;
  for (int fp32 = 0; fp32 < 2; ++fp32) {
    std::vector<int> gi;
    std::vector<const double *> gv;
    std::vector<double *> gw;
    for (size_t i = 0; i < idx.size(); ++i) {
      if ((b.plans[idx[i]]->opts.precision == WC_MIXED) != (fp32 == 1)) continue;
      gi.push_back(idx[i]);
      gv.push_back(v[i]);
      gw.push_back(w[i]);
    }
    if (gi.empty()) continue;
    hipError_t e = launch_pc_batch(st, b.d_tab, b.h_tab.data(), (int)gi.size(), gi.data(),
                                   gv.data(), gw.data(), fp32 == 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

bool same_stream(const wc_batch &b) {
  for (const wc_plan *p : b.plans)
    if (p->stream != b.plans[0]->stream) return false;
  return true;
}

// One GMRES(k)-P_S instance of a lockstep batch solve: right preconditioning on
// E = Ahat P^{-1} - I with classical Gram-Schmidt and a DGKS-gated second pass, the
// restart test on the true residual b - Ahat x; the same steps as the single solve.
struct Lane {
  enum Phase { INIT, BETA, ARNOLDI, DONE };
  wc_plan *p = nullptr;
  uint64_t tag = 0;                       // caller's identifier (continuous batching)
  double *yo = nullptr, *po = nullptr, *uo = nullptr;
  double *B = nullptr, *X = nullptr, *V = nullptr, *Zb = nullptr, *T = nullptr;
  int k = 0, total = 0, cycles = 0, reorth = 0, j = 0;
  bool flex = false;
  double bnorm = 0.0, relres = 1.0, relres_est = 1.0;
  std::vector<double> H, cs, sn, g, y, nu;
  Phase ph = BETA;
  wc_status st = WC_E_MAXIT;

  double *Zj() const { return flex ? Zb + (size_t)j * p->nvec : Zb; }
};

hipError_t read_async(wc_plan *p, int slot, int count) {
  return hipMemcpyAsync(p->h_scal + slot, p->d_scal + slot, count * sizeof(double),
                        hipMemcpyDeviceToHost, p->stream);
}

// r0 = b - Ahat x into V_0 and its squared norm toward the host (x = 0: r0 = b).
hipError_t start_cycle(Lane &L, bool x_zero) {
  wc_plan &p = *L.p;
  hipError_t e;
  if (x_zero) {
    e = launch_lincomb3(p, L.V, L.B, nullptr, nullptr, -1, 1.0, 0.0, 0.0);
  } else {
    e = launch_matvec(p, L.X, L.V, p.d_partials, nullptr, L.B, true);
  }
  if (e != hipSuccess) return e;
  if ((e = launch_dot(p, L.V, L.V, S_NU2)) != hipSuccess) return e;
  return read_async(L.p, S_NU2, 1);
}

// Arnoldi step j after the preconditioner: V_{j+1} = Ahat Z_j - V_j, two Gram-Schmidt
// passes (the second gated on the device), the projection scalars toward the host.
hipError_t arnoldi_tail(Lane &L) {
  wc_plan &p = *L.p;
  const size_t nv = p.nvec;
  double *Vj = L.V + (size_t)L.j * nv, *Vn = L.V + (size_t)(L.j + 1) * nv;
  hipError_t e;
  if ((e = launch_matvec(p, L.Zj(), Vn, p.d_partials, nullptr, Vj)) != hipSuccess) return e;
  if ((e = launch_gram_schmidt(p, L.V, L.j, Vn)) != hipSuccess) return e;
  return read_async(L.p, S_WN2, S_D2 + L.j + 1 - S_WN2);
}

// Host side of Arnoldi step j: the Hessenberg column, its Givens rotation and the
// residual estimate.  Returns true when the cycle ends here.
bool arnoldi_host(Lane &L, double tol, int maxit) {
  const double *hs = L.p->h_scal;
  const int k = L.k, j = L.j;
  const bool two = hs[S_REORTH] != 0.0;
  L.reorth += two ? 1 : 0;
  const double nn = std::sqrt(std::max(hs[S_NU2 + j + 1], 0.0));
  L.nu[j + 1] = nn;
  double *h = &L.H[(size_t)j * (k + 1)];
  for (int i = 0; i <= j; ++i)
    h[i] = (hs[S_D1 + i] + (two ? hs[S_D2 + i] : 0.0)) / (L.nu[i] * L.nu[j]);
  h[j] += 1.0;  // H = H_E + I
  const double hn = nn / L.nu[j];
  for (int i = 0; i < j; ++i) {
    const double t = L.cs[i] * h[i] + L.sn[i] * h[i + 1];
    h[i + 1] = -L.sn[i] * h[i] + L.cs[i] * h[i + 1];
    h[i] = t;
  }
  const double r = std::hypot(h[j], hn);
  L.cs[j] = r > 0 ? h[j] / r : 1.0;
  L.sn[j] = r > 0 ? hn / r : 0.0;
  h[j] = r;
  L.g[j + 1] = -L.sn[j] * L.g[j];
  L.g[j] = L.cs[j] * L.g[j];
  ++L.total;
  L.relres_est = std::fabs(L.g[j + 1]) / L.bnorm;
  return !std::isfinite(L.relres_est) || r == 0.0 || L.relres_est <= tol || hn == 0.0 ||
         L.total >= maxit || j + 1 == k;
}

// End of a cycle after jd steps: x += Z y (flexible) or x += P^{-1} V y.
hipError_t cycle_update(Lane &L, int jd) {
  wc_plan &p = *L.p;
  const int k = L.k;
  for (int i = jd - 1; i >= 0; --i) {
    double s = L.g[i];
    for (int l = i + 1; l < jd; ++l) s -= L.H[(size_t)l * (k + 1) + i] * L.y[l];
    const double d = L.H[(size_t)i * (k + 1) + i];
    L.y[i] = d != 0.0 ? s / d : 0.0;
  }
  for (int i = 0; i < jd; ++i) L.y[i] /= L.nu[i];
  std::memcpy(p.h_scal + S_Y, L.y.data(), jd * sizeof(double));
  hipError_t e = hipMemcpyAsync(p.d_scal + S_Y, p.h_scal + S_Y, jd * sizeof(double),
                                hipMemcpyHostToDevice, p.stream);
  if (e != hipSuccess) return e;
  if (L.flex) return launch_multiaxpy(p, L.X, L.Zb, jd, S_Y, 1.0, false, nullptr, nullptr);
  if ((e = launch_fill(p, L.T, 0.0, p.nvec)) != hipSuccess) return e;
  if ((e = launch_multiaxpy(p, L.T, L.V, jd, S_Y, 1.0, false, nullptr, nullptr)) != hipSuccess)
    return e;
  if ((e = launch_pc_apply(p, L.T, L.Zb, false, nullptr)) != hipSuccess) return e;
  return launch_lincomb3(p, L.X, L.X, L.Zb, nullptr, -1, 1.0, 1.0, 0.0);
}

// Lane set-up shared by the lockstep batch and the continuous engine: buffers from the
// plan's Krylov vectors, the right-hand side and the request of ||b|| to the host.
hipError_t lane_setup(Lane &L, wc_plan &p, const double *f, const double *g, const double *y0) {
  L.p = &p;
  L.k = p.opts.restart;
  L.flex = p.opts.flexible || p.opts.precision == WC_MIXED;
  L.V = p.vec(0);
  L.Zb = p.vec(L.k + 1);
  L.T = p.vec(L.k + 1 + (L.flex ? L.k : 1));
  L.B = p.vec(p.nkvec - 2);
  L.X = p.vec(p.nkvec - 1);
  L.H.assign((size_t)(L.k + 1) * L.k, 0.0);
  L.cs.assign(L.k, 0.0);
  L.sn.assign(L.k, 0.0);
  L.g.assign(L.k + 1, 0.0);
  L.y.assign(L.k, 0.0);
  L.nu.assign(L.k + 1, 0.0);
  hipError_t e = launch_rhs(p, f, g, y0, L.B);
  if (e == hipSuccess) e = launch_dot(p, L.B, L.B, S_DOT);
  if (e == hipSuccess) e = read_async(&p, S_DOT, 1);
  return e;
}

// After the synchronisation that follows lane_setup: ||b||, x = 0 and the first cycle.
hipError_t lane_start(Lane &L) {
  L.bnorm = std::sqrt(L.p->h_scal[S_DOT]);
  hipError_t e = launch_fill(*L.p, L.X, 0.0, L.p->nvec);
  if (e != hipSuccess) return e;
  if (!std::isfinite(L.bnorm)) {
    L.ph = Lane::DONE;
    L.st = WC_E_NONFINITE;
  } else if (L.bnorm == 0.0) {
    L.ph = Lane::DONE;
    L.st = WC_OK;
    L.relres = L.relres_est = 0.0;
  } else {
    e = start_cycle(L, true);
    L.ph = Lane::BETA;
  }
  return e;
}

// Host side of one round for a lane that was in phase `was` when the round's work was
// enqueued (the restart test, or the Arnoldi step and possibly the cycle's end).
hipError_t lane_advance(Lane &L, Lane::Phase was) {
  wc_plan &p = *L.p;
  if (was == Lane::INIT) return lane_start(L);
  if (was == Lane::BETA) {
    const double beta = std::sqrt(p.h_scal[S_NU2]);
    L.relres = beta / L.bnorm;
    if (!std::isfinite(L.relres)) {
      L.ph = Lane::DONE;
      L.st = WC_E_NONFINITE;
    } else if (L.relres <= p.opts.tol) {
      L.ph = Lane::DONE;
      L.st = WC_OK;
    } else if (L.total >= p.opts.maxit) {
      L.ph = Lane::DONE;
      L.st = WC_E_MAXIT;
    } else {
      L.nu[0] = beta;
      std::fill(L.g.begin(), L.g.end(), 0.0);
      L.g[0] = beta;
      L.j = 0;
      L.ph = Lane::ARNOLDI;
    }
    return hipSuccess;
  }
  if (was == Lane::ARNOLDI) {
    if (!arnoldi_host(L, p.opts.tol, p.opts.maxit)) {
      ++L.j;
      return hipSuccess;
    }
    hipError_t e = cycle_update(L, L.j + 1);
    if (e != hipSuccess) return e;
    ++L.cycles;
    e = start_cycle(L, false);
    L.ph = Lane::BETA;
    return e;
  }
  return hipSuccess;
}

wc_info lane_info(const Lane &L) {
  wc_info in;
  std::memset(&in, 0, sizeof(in));
  in.status = L.st;
  in.iters = L.total;
  in.restarts = L.cycles;
  in.relres = L.relres;
  in.relres_est = L.relres_est;
  in.reorth = L.reorth;
  return in;
}

BatchInst batch_inst(const wc_plan &p) {
  const bool f32 = p.opts.precision == WC_MIXED;
  BatchInst I{};
  I.n = p.n;
  I.N1 = p.N1;
  I.m = p.m;
  I.kind = pc_kind(p);
  I.tau = p.tau;
  I.alpha = p.alpha;
  I.cnorm = (1.0 / p.n) * (2.0 / p.N1) * (2.0 / p.N1);
  I.W = p.d_specA;
  I.dtw = p.d_dtw;
  I.twt = f32 ? (const void *)p.d_twt32 : (const void *)p.d_twt64;
  I.tws = f32 ? (const void *)p.d_tws32 : (const void *)p.d_tws64;
  I.sin = f32 ? (const void *)p.d_sin32 : (const void *)p.d_sin64;
  I.lam = f32 ? (const void *)p.d_lam32 : (const void *)p.d_lam64;
  I.mu = f32 ? (const void *)p.d_mu32 : (const void *)p.d_mu64;
  return I;
}

}  // namespace

// ---- continuous batching ------------------------------------------------------------
// The lanes of a lockstep GMRES(k)-P_S whose membership changes between rounds: a solve
// joins (its right-hand side and ||b|| are enqueued at once and it starts its first cycle
// after the next synchronisation) and leaves (its solution recovered) at any round
// boundary, while the others keep iterating.  Each round applies the preconditioner of
// every lane inside an Arnoldi cycle in one batched launch per pass and precision, then
// each lane's matvec and Gram-Schmidt passes, and synchronises the host once.
struct LockstepEngine {
  hipStream_t st = nullptr;
  std::vector<Lane> lanes;
  BatchInst *d_tab = nullptr;  // kBatchMax entries, rebuilt when the lanes change
  BatchInst *h_tab = nullptr;  // pinned staging of the table
  bool dirty = true;
};

namespace wc {

bool lockstep_eligible(const wc_problem *pr, const wc_opts *op) {
  const auto p2 = [](int x) { return x == 64 || x == 128 || x == 256 || x == 512; };
  return pr->dims == 2 && !pr->a_face_host && pr->disc == WC_FD && pr->bc == WC_DIRICHLET &&
         op->method == WC_GMRES_PS &&
         !op->lowrank &&
         std::fabs(pr->zeta - M_PI) <= 1e-12 && p2(pr->n) && p2(pr->M + 1);
}

LockstepEngine *lockstep_create(hipStream_t st) {
  auto *eng = new (std::nothrow) LockstepEngine;
  if (!eng) return nullptr;
  eng->st = st;
  if (hipMalloc((void **)&eng->d_tab, kBatchMax * sizeof(BatchInst)) != hipSuccess ||
      hipHostMalloc((void **)&eng->h_tab, kBatchMax * sizeof(BatchInst), 0) != hipSuccess) {
    (void)hipGetLastError();
    lockstep_destroy(eng);
    return nullptr;
  }
  return eng;
}

void lockstep_destroy(LockstepEngine *eng) {
  if (!eng) return;
  if (eng->st) (void)hipStreamSynchronize(eng->st);
  if (eng->d_tab) (void)hipFree(eng->d_tab);
  if (eng->h_tab) (void)hipHostFree(eng->h_tab);
  delete eng;
}

int lockstep_active(const LockstepEngine *eng) { return (int)eng->lanes.size(); }

hipError_t lockstep_add(LockstepEngine *eng, wc_plan *p, const double *f, const double *g,
                        const double *y0, double *y, double *pout, double *u, uint64_t tag) {
  if ((int)eng->lanes.size() >= kBatchMax || p->stream != eng->st || !p->pc_ok ||
      p->dims != 2 || p->var_coeff || !batch_sizes_ok(p->n, p->N1))
    return hipErrorInvalidValue;
  Lane L;
  L.tag = tag;
  L.yo = y;
  L.po = pout;
  L.uo = u;
  L.ph = Lane::INIT;
  hipError_t e = lane_setup(L, *p, f, g, y0);
  if (e != hipSuccess) return e;
  eng->lanes.push_back(std::move(L));
  eng->dirty = true;
  return hipSuccess;
}

hipError_t lockstep_round(LockstepEngine *eng, std::vector<LockstepDone> &done) {
  std::vector<Lane> &lanes = eng->lanes;
  const int cnt = (int)lanes.size();
  if (cnt == 0) return hipSuccess;
  hipError_t e;
  if (eng->dirty) {  // the previous round synchronised: the staging buffer is free
    for (int i = 0; i < cnt; ++i) eng->h_tab[i] = batch_inst(*lanes[i].p);
    e = hipMemcpyAsync(eng->d_tab, eng->h_tab, cnt * sizeof(BatchInst), hipMemcpyHostToDevice,
                       eng->st);
    if (e != hipSuccess) return e;
    eng->dirty = false;
  }
  for (int fp32 = 0; fp32 < 2; ++fp32) {  // one batched apply per precision
    std::vector<int> idx;
    std::vector<const double *> vin;
    std::vector<double *> wout;
    for (int i = 0; i < cnt; ++i) {
      const Lane &L = lanes[i];
      if (L.ph != Lane::ARNOLDI || (L.p->opts.precision == WC_MIXED) != (fp32 == 1)) continue;
      idx.push_back(i);
      vin.push_back(L.V + (size_t)L.j * L.p->nvec);
      wout.push_back(L.Zj());
    }
    if (idx.empty()) continue;
    e = launch_pc_batch(eng->st, eng->d_tab, eng->h_tab, (int)idx.size(), idx.data(), vin.data(),
                        wout.data(), fp32 == 1);
    if (e != hipSuccess) return e;
  }
  for (Lane &L : lanes)
    if (L.ph == Lane::ARNOLDI && (e = arnoldi_tail(L)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(eng->st)) != hipSuccess) return e;
  std::vector<Lane::Phase> was(cnt);
  for (int i = 0; i < cnt; ++i) was[i] = lanes[i].ph;
  for (int i = 0; i < cnt; ++i)
    if ((e = lane_advance(lanes[i], was[i])) != hipSuccess) return e;
  bool any = false;
  for (Lane &L : lanes) {
    if (L.ph != Lane::DONE) continue;
    any = true;
    if (L.st == WC_OK || L.st == WC_E_MAXIT)
      if ((e = launch_recover(*L.p, L.X, L.yo, L.po, L.uo)) != hipSuccess) return e;
  }
  if (!any) return hipSuccess;
  if ((e = hipStreamSynchronize(eng->st)) != hipSuccess) return e;
  std::vector<Lane> keep;
  for (Lane &L : lanes) {
    if (L.ph == Lane::DONE) done.push_back({L.tag, L.p, lane_info(L)});
    else keep.push_back(std::move(L));
  }
  lanes.swap(keep);
  eng->dirty = true;
  return hipSuccess;
}

}  // namespace wc

namespace {

wc_status run_batch_gmres(wc_batch &b, const double *const *f, const double *const *g,
                          const double *const *y0, double *const *y, double *const *pout,
                          wc_info *infos) {
  const int cnt = (int)b.plans.size();
  hipStream_t st = b.plans[0]->stream;
  std::vector<Lane> lanes(cnt);
  for (int i = 0; i < cnt; ++i) {
    lanes[i].ph = Lane::INIT;
    WC_TRY(lane_setup(lanes[i], *b.plans[i], f[i], g[i], y0[i]));
  }
  if (hipStreamSynchronize(st) != hipSuccess) return WC_E_HIP;
  for (Lane &L : lanes) WC_TRY(lane_start(L));
  std::vector<Lane::Phase> was(cnt);
  for (;;) {
    // every lane in an Arnoldi cycle advances one step: one batched preconditioner apply
    std::vector<int> idx;
    std::vector<const double *> vin;
    std::vector<double *> wout;
    for (int i = 0; i < cnt; ++i) {
      if (lanes[i].ph != Lane::ARNOLDI) continue;
      idx.push_back(i);
      vin.push_back(lanes[i].V + (size_t)lanes[i].j * lanes[i].p->nvec);
      wout.push_back(lanes[i].Zj());
    }
    bool pending = !idx.empty();
    for (const Lane &L : lanes) pending = pending || L.ph == Lane::BETA;
    if (!pending) break;
    if (!idx.empty()) WC_TRY(batch_pc(b, idx, vin, wout));
    for (int i : idx) WC_TRY(arnoldi_tail(lanes[i]));
    if (hipStreamSynchronize(st) != hipSuccess) return WC_E_HIP;
    for (int i = 0; i < cnt; ++i) was[i] = lanes[i].ph;
    for (int i = 0; i < cnt; ++i) WC_TRY(lane_advance(lanes[i], was[i]));
  }
  for (int i = 0; i < cnt; ++i) {
    Lane &L = lanes[i];
    if (L.st == WC_OK || L.st == WC_E_MAXIT)
      WC_TRY(launch_recover(*L.p, L.X, y[i], pout[i], nullptr));
    if (infos) infos[i] = lane_info(L);
  }
  if (hipStreamSynchronize(st) != hipSuccess) return WC_E_HIP;
  wc_status worst = WC_OK;
  for (const Lane &L : lanes)
    if (L.st != WC_OK && (worst == WC_OK || worst == WC_E_MAXIT)) worst = L.st;
  return worst;
}

}  // namespace

extern "C" {

wc_status wc_batch_create(wc_plan *const *plans, int count, wc_batch **out) {
  if (!plans || !out || count < 1 || count > kBatchMax) return WC_E_ARG;
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return WC_E_ARG;
    for (int k = 0; k < i; ++k)
      if (plans[k] == plans[i]) return WC_E_ARG;  // each instance needs its own workspace
    const wc_plan &p = *plans[i];
    if (p.dims != 2 || p.var_coeff || p.fem || p.neumann || p.general || !p.pc_ok ||
        !batch_sizes_ok(p.n, p.N1))
      return WC_E_UNSUPPORTED;
  }
  auto *b = new (std::nothrow) wc_batch;
  if (!b) return WC_E_NOMEM;
  b->plans.assign(plans, plans + count);
  for (wc_plan *pp : b->plans) b->h_tab.push_back(batch_inst(*pp));
  const size_t bytes = b->h_tab.size() * sizeof(BatchInst);
  if (hipMalloc((void **)&b->d_tab, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return WC_E_NOMEM;
  }
  if (hipMemcpy(b->d_tab, b->h_tab.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(b->d_tab);
    delete b;
    return WC_E_HIP;
  }
  *out = b;
  return WC_OK;
}

wc_status wc_batch_destroy(wc_batch *b) {
  if (!b) return WC_E_ARG;
  for (wc_plan *p : b->plans) (void)hipStreamSynchronize(p->stream);
  if (b->d_tab) (void)hipFree(b->d_tab);
  delete b;
  return WC_OK;
}

wc_status wc_batch_pc_apply(wc_batch *b, const double *const *v, double *const *w) {
  if (!b || !v || !w) return WC_E_ARG;
  if (!same_stream(*b)) return WC_E_ARG;
  const int cnt = (int)b->plans.size();
  std::vector<int> idx(cnt);
  std::vector<const double *> vv(cnt);
  std::vector<double *> ww(cnt);
  for (int i = 0; i < cnt; ++i) {
    if (!v[i] || !w[i]) return WC_E_ARG;
    idx[i] = i;
    vv[i] = v[i];
    ww[i] = w[i];
  }
  WC_TRY(batch_pc(*b, idx, vv, ww));
  return WC_OK;
}

wc_status wc_batch_solve(wc_batch *b, const double *const *f, const double *const *g,
                         const double *const *y0, double *const *y, double *const *p,
                         wc_info *infos) {
  if (!b || !f || !g || !y0 || !y || !p) return WC_E_ARG;
  if (!same_stream(*b)) return WC_E_ARG;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    if (!f[i] || !g[i] || !y0[i] || !y[i] || !p[i]) return WC_E_ARG;
    const wc_plan &pl = *b->plans[i];
    if (pl.opts.method != WC_GMRES_PS || pl.opts.lowrank) return WC_E_UNSUPPORTED;
  }
  const auto t0 = std::chrono::steady_clock::now();
  const wc_status st = run_batch_gmres(*b, f, g, y0, y, p, infos);
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (infos)
    for (size_t i = 0; i < b->plans.size(); ++i) infos[i].ms = ms;
  return st;
}

}  // extern "C"
