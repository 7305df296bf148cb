// Step 2 of the preconditioner apply for a variable diffusion coefficient a(x): the
// spatial problems of every kept frequency are solved by batched multigrid.
//
// After the omega-scaled time transform, frequency l (lambda = lambda_l) couples the two
// block rows through
//   P_S  (GMRES):  [[lambda I + tau K, -alpha I], [alpha I, conj(lambda) I + tau K]]
//   P_MS (MINRES): sigma_l I + tau K on each block row, sigma_l = sqrt(|lambda_l|^2 + alpha^2)
// (Section 3.4, Lemma 2.3).  The 2x2 scalar matrix E = [[lambda, -alpha], [alpha,
// conj(lambda)]] is normal (E E^* = (|lambda|^2 + alpha^2) I), so it has orthonormal
// eigenvectors u_k = c_k [1; mu_k] with eigenvalues D_1,2 = Re lambda +- i s,
// s = sqrt(Im(lambda)^2 + alpha^2), mu_k = (lambda - D_k)/alpha.  Rotating the two block
// rows by U = [u_1 u_2] (unitary, so nothing is amplified) leaves two independent
// complex-shifted problems (D_k I + tau K) w_k = r_k.  Each is solved by V(2,2) cycles of
// red-black Gauss-Seidel (red sweeps first before the coarse correction, black first
// after it, so the cycle is symmetric), full-weighting restriction, bilinear
// prolongation and coarse operators rediscretised with face coefficients averaged from
// the finer level, down to one interior point, where the solve is exact.  Cycles repeat
// until every system's relative residual is at most mg_tol (or mg_max_cycles).
//
// Layout: systems sys = 2q + k (q = 0..n/2-1 <-> l = q+1, k = rotated block row), each
// an M^dims complex grid [x2][x1], i.e. the spectral array of the time transform.  The
// fine solution lives in d_specB; coarse levels in d_mg_work.  Levels whose whole
// remaining pyramid fits in one workgroup's LDS are cycled by a single kernel with one
// workgroup per system.

#include "wc_internal.h"

namespace wc {
namespace {

struct MgLev {
  int M;
  double inv_h2;
  const double *ax;  // 1D: M+1 faces; 2D: faces normal to x1, (M, M+1)
  const double *ay;  // 2D: faces normal to x2, (M+1, M)
};

constexpr int kMgMaxLds = 12;
struct MgLdsLevels {
  int nl;
  MgLev lev[kMgMaxLds];
};

// tau * (stencil coefficients) of the shifted operator at (i, j): the four neighbour
// weights and the diagonal sum (Dirichlet neighbours keep their face in the diagonal).
struct Coef {
  double w, e, s, n, d;
};

template <int D>
__device__ __forceinline__ Coef coef_at(const MgLev &L, int i, int j, double tau) {
  const double t = tau * L.inv_h2;
  Coef c;
  if constexpr (D == 1) {
    const double aw = L.ax[i], ae = L.ax[i + 1];
    c.w = t * aw;
    c.e = t * ae;
    c.s = c.n = 0.0;
    c.d = c.w + c.e;
  } else {
    const int M = L.M;
    const double aw = L.ax[(size_t)j * (M + 1) + i], ae = L.ax[(size_t)j * (M + 1) + i + 1];
    const double as = L.ay[(size_t)j * M + i], an = L.ay[(size_t)(j + 1) * M + i];
    c.w = t * aw;
    c.e = t * ae;
    c.s = t * as;
    c.n = t * an;
    c.d = c.w + c.e + c.s + c.n;
  }
  return c;
}

// sum of the neighbour terms  w u_W + e u_E + s u_S + n u_N  (outside the grid u = 0)
template <typename P, int D>
__device__ __forceinline__ cx<P> nb_sum(const cx<P> *u, const Coef &c, int M, int i, int j) {
  cx<P> r{(P)0, (P)0};
  if (i > 0) { const cx<P> v = u[(size_t)j * M + i - 1]; r.x += (P)c.w * v.x; r.y += (P)c.w * v.y; }
  if (i < M - 1) { const cx<P> v = u[(size_t)j * M + i + 1]; r.x += (P)c.e * v.x; r.y += (P)c.e * v.y; }
  if constexpr (D == 2) {
    if (j > 0) { const cx<P> v = u[(size_t)(j - 1) * M + i]; r.x += (P)c.s * v.x; r.y += (P)c.s * v.y; }
    if (j < M - 1) { const cx<P> v = u[(size_t)(j + 1) * M + i]; r.x += (P)c.n * v.x; r.y += (P)c.n * v.y; }
  }
  return r;
}

// x / (shift + d)
template <typename P>
__device__ __forceinline__ cx<P> div_shift(cx<P> x, cx<double> shift, double d) {
  const double dr = shift.x + d, di = shift.y;
  const double inv = 1.0 / (dr * dr + di * di);
  const P ar = (P)(dr * inv), ai = (P)(-di * inv);  // 1/(dr + i di)
  return cx<P>{x.x * ar - x.y * ai, x.x * ai + x.y * ar};
}

// residual f - (shift + d) u_P + neighbours
template <typename P, int D>
__device__ __forceinline__ cx<P> resid(const cx<P> *u, const cx<P> *f, const MgLev &L,
                                       cx<double> shift, double tau, int i, int j) {
  const Coef c = coef_at<D>(L, i, j, tau);
  const size_t o = (size_t)j * L.M + i;
  const cx<P> up = u[o], fp = f[o];
  const cx<P> nb = nb_sum<P, D>(u, c, L.M, i, j);
  const double dr = shift.x + c.d, di = shift.y;
  return cx<P>{fp.x + nb.x - (P)dr * up.x + (P)di * up.y, fp.y + nb.y - (P)dr * up.y - (P)di * up.x};
}

// bilinear interpolation of the coarse grid (Mc points per direction) at fine (i, j)
__device__ __forceinline__ void interp_1d(int i, int Mc, int &I0, int &I1, double &w0) {
  if (i & 1) { I0 = (i - 1) >> 1; I1 = -1; w0 = 1.0; }
  else { I0 = (i >> 1) - 1; I1 = i >> 1; w0 = 0.5; }
  if (I0 >= Mc) I0 = -1;
  if (I1 >= Mc) I1 = -1;
}

template <typename P, int D>
__device__ __forceinline__ cx<P> interp(const cx<P> *uc, int Mc, int i, int j) {
  int I0, I1;
  double wi;
  interp_1d(i, Mc, I0, I1, wi);
  cx<P> r{(P)0, (P)0};
  if constexpr (D == 1) {
    if (I0 >= 0) { r.x += (P)wi * uc[I0].x; r.y += (P)wi * uc[I0].y; }
    if (I1 >= 0) { r.x += (P)wi * uc[I1].x; r.y += (P)wi * uc[I1].y; }
  } else {
    int J0, J1;
    double wj;
    interp_1d(j, Mc, J0, J1, wj);
    const int Is[2] = {I0, I1}, Js[2] = {J0, J1};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (Js[b] < 0) continue;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (Is[a] < 0) continue;
        const P w = (P)(wi * wj);
        const cx<P> v = uc[(size_t)Js[b] * Mc + Is[a]];
        r.x += w * v.x;
        r.y += w * v.y;
      }
    }
  }
  return r;
}

// Gauss-Seidel value of point (i, j).  zero: all neighbours are taken as 0 (first sweep
// from a zero guess).  uc != nullptr: neighbours are corrected by the prolongated
// coarse solution on the fly (first sweep after the coarse correction).
template <typename P, int D>
__device__ __forceinline__ cx<P> gs_value(const cx<P> *u, const cx<P> *f, const MgLev &L,
                                          cx<double> shift, double tau, int i, int j, bool zero,
                                          const cx<P> *uc, int Mc) {
  const Coef c = coef_at<D>(L, i, j, tau);
  const int M = L.M;
  cx<P> acc = f[(size_t)j * M + i];
  if (!zero) {
    const cx<P> nb = nb_sum<P, D>(u, c, M, i, j);
    acc.x += nb.x;
    acc.y += nb.y;
    if (uc) {
      cx<P> e{(P)0, (P)0};
      if (i > 0) { const cx<P> v = interp<P, D>(uc, Mc, i - 1, j); e.x += (P)c.w * v.x; e.y += (P)c.w * v.y; }
      if (i < M - 1) { const cx<P> v = interp<P, D>(uc, Mc, i + 1, j); e.x += (P)c.e * v.x; e.y += (P)c.e * v.y; }
      if constexpr (D == 2) {
        if (j > 0) { const cx<P> v = interp<P, D>(uc, Mc, i, j - 1); e.x += (P)c.s * v.x; e.y += (P)c.s * v.y; }
        if (j < M - 1) { const cx<P> v = interp<P, D>(uc, Mc, i, j + 1); e.x += (P)c.n * v.x; e.y += (P)c.n * v.y; }
      }
      acc.x += e.x;
      acc.y += e.y;
    }
  }
  return div_shift(acc, shift, c.d);
}

// Full-weighting restriction of the residual at coarse point (I, J).  Called right after
// a black sweep, when the residual vanishes at black points: only the red fine points of
// the stencil (the centre and, in 2D, the four corners) contribute.
template <typename P, int D>
__device__ __forceinline__ cx<P> restrict_val(const cx<P> *u, const cx<P> *f, const MgLev &L,
                                              cx<double> shift, double tau, int I, int J) {
  const int i = 2 * I + 1, j = D == 2 ? 2 * J + 1 : 0;
  const cx<P> rc = resid<P, D>(u, f, L, shift, tau, i, j);
  if constexpr (D == 1) {
    return cx<P>{rc.x * (P)0.5, rc.y * (P)0.5};
  } else {
    cx<P> r{rc.x * (P)4, rc.y * (P)4};
#pragma unroll
    for (int dj = -1; dj <= 1; dj += 2)
#pragma unroll
      for (int di = -1; di <= 1; di += 2) {
        const cx<P> v = resid<P, D>(u, f, L, shift, tau, i + di, j + dj);
        r.x += v.x;
        r.y += v.y;
      }
    return cx<P>{r.x * (P)0.0625, r.y * (P)0.0625};
  }
}

// red points: the colour holding the coarse-grid points ((odd, odd) in 2D, odd in 1D)
template <int D> __device__ __forceinline__ int color_i(int t, int j, int color) {
  return 2 * t + ((j + (D == 1 ? 1 : 0) + color) & 1);
}

__device__ __forceinline__ cx<double> sys_shift(const double *sh, int sys) {
  return cx<double>{sh[2 * sys], sh[2 * sys + 1]};
}

// ---- kernels on levels held in global memory ------------------------------------
template <typename P, int D>
__global__ __launch_bounds__(kThreads) void k_mg_smooth(cx<P> *__restrict__ u,
                                                        const cx<P> *__restrict__ f, MgLev L,
                                                        const double *__restrict__ shifts,
                                                        double tau, int color, int zero,
                                                        const cx<P> *__restrict__ uc, int nsys) {
  const int M = L.M, half = (M + 1) / 2, rows = D == 2 ? M : 1;
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (size_t)nsys * rows * half) return;
  // index arithmetic in 32 bits (every level holds fewer than 2^32 points)
  const unsigned ui = (unsigned)idx, r = ui / (unsigned)half;
  const int t = (int)(ui - r * (unsigned)half);
  const int j = (int)(r % (unsigned)rows), sys = (int)(r / (unsigned)rows);
  const int i = color_i<D>(t, j, color);
  if (i >= M) return;
  const size_t np = (size_t)rows * M;
  const int Mc = (M - 1) / 2;
  const cx<P> *ucs = uc ? uc + (size_t)sys * (D == 2 ? (size_t)Mc * Mc : Mc) : nullptr;
  u[sys * np + (size_t)j * M + i] = gs_value<P, D>(u + sys * np, f + sys * np, L,
                                                   sys_shift(shifts, sys), tau, i, j, zero != 0,
                                                   ucs, Mc);
}

template <typename P, int D>
__global__ __launch_bounds__(kThreads) void k_mg_restrict(const cx<P> *__restrict__ u,
                                                          const cx<P> *__restrict__ f, MgLev L,
                                                          cx<P> *__restrict__ fc,
                                                          const double *__restrict__ shifts,
                                                          double tau, int nsys) {
  const int M = L.M, Mc = (M - 1) / 2, rows = D == 2 ? Mc : 1;
  const size_t npc = (size_t)rows * Mc, np = (size_t)(D == 2 ? M : 1) * M;
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (size_t)nsys * npc) return;
  const unsigned ui = (unsigned)idx, un = (unsigned)npc;  // 32-bit index arithmetic
  const int sys = (int)(ui / un);
  const int o = (int)(ui - (unsigned)sys * un), I = o % Mc, J = o / Mc;
  fc[idx] = restrict_val<P, D>(u + sys * np, f + sys * np, L, sys_shift(shifts, sys), tau, I, J);
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// partials[sys * gridDim.x + b]: squared residual norm at black points (the cycle ended
// with a red sweep, so red residuals vanish), or with resid == 0 the squared norm of f.
template <typename P, int D>
__global__ __launch_bounds__(kThreads) void k_mg_norms(const cx<P> *__restrict__ u,
                                                       const cx<P> *__restrict__ f, MgLev L,
                                                       const double *__restrict__ shifts,
                                                       double tau, int resid_mode,
                                                       double *__restrict__ partials) {
  __shared__ double red[kThreads / 64];
  const int sys = blockIdx.y, M = L.M, rows = D == 2 ? M : 1, half = (M + 1) / 2;
  const size_t np = (size_t)rows * M;
  const cx<P> *us = u + sys * np, *fs = f + sys * np;
  const cx<double> sh = sys_shift(shifts, sys);
  double acc = 0.0;
  if (resid_mode) {
    const int cnt = rows * half;
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < cnt; t += gridDim.x * kThreads) {
      const int j = t / half, i = color_i<D>(t % half, j, 1);
      if (i >= M) continue;
      const cx<P> r = resid<P, D>(us, fs, L, sh, tau, i, j);
      acc += (double)r.x * r.x + (double)r.y * r.y;
    }
  } else {
    for (size_t t = (size_t)blockIdx.x * kThreads + threadIdx.x; t < np;
         t += (size_t)gridDim.x * kThreads) {
      const cx<P> v = fs[t];
      acc += (double)v.x * v.x + (double)v.y * v.y;
    }
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(size_t)sys * gridDim.x + blockIdx.x] = r;
}

// mode 0: fn2[sys] = sum of partials;  mode 1: S[slot] = max_sys sqrt(res2 / fn2)
__global__ __launch_bounds__(kThreads) void k_mg_reduce(const double *__restrict__ partials,
                                                        int gx, int nsys, double *fn2,
                                                        double *S, int slot, int mode) {
  __shared__ double red[kThreads / 64];
  double mx = 0.0;
  for (int sys = threadIdx.x; sys < nsys; sys += kThreads) {
    double a = 0.0;
    for (int b = 0; b < gx; ++b) a += partials[(size_t)sys * gx + b];
    if (mode == 0) {
      fn2[sys] = a;
    } else {
      const double rr = fn2[sys] > 0.0 ? sqrt(a / fn2[sys]) : 0.0;
      mx = rr > mx ? rr : mx;
    }
  }
  if (mode == 0) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_down(mx, o, 64);
    mx = v > mx ? v : mx;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) r = red[i] > r ? red[i] : r;
    S[slot] = r;
  }
}

// Rotation into / out of the decoupled systems, with the 1/n of the inverse time
// transform.  mix[q] = {c1, Re c1 mu1, Im c1 mu1, c2, Re c2 mu2, Im c2 mu2}.
//   in : r_k = (c_k/n) (A + conj(mu_k) B)       out: a = c1 w1 + c2 w2, b = c1 mu1 w1 + c2 mu2 w2
// P_MS (mix == nullptr): r = (A, B)/n in, identity out.
template <typename P>
__global__ __launch_bounds__(kThreads) void k_mg_mix(const cx<P> *__restrict__ src,
                                                     cx<P> *__restrict__ dst,
                                                     const double *__restrict__ mix, int m,
                                                     int nq, double inv_n, int out) {
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (size_t)nq * m) return;
  const unsigned ui = (unsigned)idx;  // 32-bit index arithmetic
  const int q = (int)(ui / (unsigned)m), s = (int)(ui - (unsigned)q * (unsigned)m);
  const size_t o0 = ((size_t)q * 2) * m + s, o1 = o0 + m;
  const cx<P> x0 = src[o0], x1 = src[o1];
  if (!mix) {
    if (out) { dst[o0] = x0; dst[o1] = x1; }
    else {
      dst[o0] = cx<P>{x0.x * (P)inv_n, x0.y * (P)inv_n};
      dst[o1] = cx<P>{x1.x * (P)inv_n, x1.y * (P)inv_n};
    }
    return;
  }
  const double *t = mix + 6 * (size_t)q;
  const P c1 = (P)t[0], c2 = (P)t[3];
  const cx<P> g1{(P)t[1], (P)t[2]}, g2{(P)t[4], (P)t[5]};  // c_k mu_k
  if (!out) {
    const P sc = (P)inv_n;
    // c_k conj(mu_k) B = conj(g_k) B
    const cx<P> r1{(c1 * x0.x + g1.x * x1.x + g1.y * x1.y) * sc, (c1 * x0.y + g1.x * x1.y - g1.y * x1.x) * sc};
    const cx<P> r2{(c2 * x0.x + g2.x * x1.x + g2.y * x1.y) * sc, (c2 * x0.y + g2.x * x1.y - g2.y * x1.x) * sc};
    dst[o0] = r1;
    dst[o1] = r2;
  } else {
    const cx<P> a{c1 * x0.x + c2 * x1.x, c1 * x0.y + c2 * x1.y};
    const cx<P> b{g1.x * x0.x - g1.y * x0.y + g2.x * x1.x - g2.y * x1.y,
                  g1.x * x0.y + g1.y * x0.x + g2.x * x1.y + g2.y * x1.x};
    dst[o0] = a;
    dst[o1] = b;
  }
}


// ---- 2D levels in global memory: four colour sweeps per pass over LDS tiles ------
// A workgroup owns a kTile x kTile block of one system and holds it with a halo of H
// points in LDS; it reads uin and writes uout (halos overlap other workgroups' tiles).
// Each sweep updates its colour on a region one point narrower than the previous one,
// so after NS sweeps the values at distance >= NS from the halo edge are
// exactly those of NS global sweeps (the halo points are recomputed redundantly); with
// H = NS the tile itself is exact, with H = NS + 1 also the residual on it.
//   uc != nullptr: the loaded values are corrected by the prolongated coarse solution
//   (the first sweep after the coarse correction then reads corrected neighbours).
//   partials != nullptr: after the sweeps, the squared residual of the colour not swept
//   last (the other one vanishes) is summed per tile: partials[sys * tiles + tile].
constexpr int kTile = 32;
constexpr int kTileThreads = 512;

// Every thread owns the region points q = tid + kTileThreads*k for the whole pass: their
// stencil weights, right-hand side and 1/(shift + diagonal) stay in registers, so the
// sweeps only exchange values through LDS.
//   RST: also restrict (full weighting) the residual left by the sweeps to the coarse
//   grid: fc[sys][J][I] for the coarse points of this tile (needs H = NS + 2: the corner
//   residuals reach one point beyond the tile).
template <typename P, int H, int NS, bool RST>
__global__ __launch_bounds__(kTileThreads) void k_mg_tile(const cx<P> *__restrict__ uin,
                                                          cx<P> *__restrict__ uout,
                                                          const cx<P> *__restrict__ f, MgLev L,
                                                          const double *__restrict__ shifts,
                                                          double tau, int c0, int zero,
                                                          const cx<P> *__restrict__ uc,
                                                          int tiles_x,
                                                          double *__restrict__ partials,
                                                          cx<P> *__restrict__ fc) {
  constexpr int R = kTile + 2 * H, NPT = R * R;
  constexpr int PPT = (NPT + kTileThreads - 1) / kTileThreads;
  static_assert(!RST || H >= NS + 2, "restriction needs residuals one point outside the tile");
  __shared__ cx<P> U[NPT];
  __shared__ cx<P> RS[RST ? NPT : 1];
  __shared__ double red[kTileThreads / 64];
  const int M = L.M, Mc = (M - 1) / 2, sys = blockIdx.y;
  const int tile = blockIdx.x, i0 = (tile % tiles_x) * kTile, j0 = (tile / tiles_x) * kTile;
  const int gi0 = i0 - H, gj0 = j0 - H;  // global index of region point (0, 0)
  const size_t np = (size_t)M * M;
  const cx<P> *us = uin + sys * np;
  cx<P> *uo = uout + sys * np;
  const cx<P> *fs = f + sys * np;
  const cx<P> *ucs = uc ? uc + (size_t)sys * Mc * Mc : nullptr;
  const cx<double> sh = sys_shift(shifts, sys);
  P cw[PPT], ce[PPT], cs[PPT], cn[PPT];
  cx<P> fv[PPT], iv[PPT];
  bool in[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int q = threadIdx.x + kTileThreads * k;
    const int gi = gi0 + q % R, gj = gj0 + q / R;
    in[k] = q < NPT && gi >= 0 && gi < M && gj >= 0 && gj < M;
    cx<P> uv{(P)0, (P)0};
    fv[k] = uv;
    iv[k] = uv;
    cw[k] = ce[k] = cs[k] = cn[k] = (P)0;
    if (in[k]) {
      const size_t o = (size_t)gj * M + gi;
      fv[k] = fs[o];
      if (!zero) uv = us[o];
      if (ucs) {
        const cx<P> e = interp<P, 2>(ucs, Mc, gi, gj);
        uv.x += e.x;
        uv.y += e.y;
      }
      const Coef c = coef_at<2>(L, gi, gj, tau);
      cw[k] = (P)c.w; ce[k] = (P)c.e; cs[k] = (P)c.s; cn[k] = (P)c.n;
      const double dr = sh.x + c.d, di = sh.y, inv = 1.0 / (dr * dr + di * di);
      iv[k] = cx<P>{(P)(dr * inv), (P)(-di * inv)};
    }
    if (q < NPT) U[q] = uv;
  }
  __syncthreads();
  for (int sw = 0; sw < NS; ++sw) {
    const int color = (c0 + sw) & 1, d = sw + 1;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int q = threadIdx.x + kTileThreads * k, r = q / R, c = q % R;
      if (!in[k] || ((gi0 + c + gj0 + r) & 1) != color || r < d || r >= R - d || c < d ||
          c >= R - d)
        continue;
      const cx<P> a = U[q - 1], b = U[q + 1], s = U[q - R], n = U[q + R];
      const P x = fv[k].x + cw[k] * a.x + ce[k] * b.x + cs[k] * s.x + cn[k] * n.x;
      const P y = fv[k].y + cw[k] * a.y + ce[k] * b.y + cs[k] * s.y + cn[k] * n.y;
      U[q] = cx<P>{x * iv[k].x - y * iv[k].y, x * iv[k].y + y * iv[k].x};
    }
    __syncthreads();
  }
  double acc2 = 0.0;
  const int rc = (c0 + NS) & 1;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int q = threadIdx.x + kTileThreads * k, r = q / R, c = q % R;
    if (!in[k] || r < H || r >= H + kTile || c < H || c >= H + kTile) continue;
    const int gi = gi0 + c, gj = gj0 + r;
    const cx<P> up = U[q];
    uo[(size_t)gj * M + gi] = up;
    if (partials && ((gi + gj) & 1) == rc) {
      const cx<P> a = U[q - 1], b = U[q + 1], s = U[q - R], n = U[q + R];
      const double dd = (double)cw[k] + ce[k] + cs[k] + cn[k];
      const double dr = sh.x + dd, di = sh.y;
      const double rx = (double)fv[k].x + cw[k] * a.x + ce[k] * b.x + cs[k] * s.x +
                        cn[k] * n.x - dr * up.x + di * up.y;
      const double ry = (double)fv[k].y + cw[k] * a.y + ce[k] * b.y + cs[k] * s.y +
                        cn[k] * n.y - dr * up.y - di * up.x;
      acc2 += rx * rx + ry * ry;
    }
  }
  if constexpr (RST) {
    // residual at the points of colour rc on the tile and one point beyond it
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int q = threadIdx.x + kTileThreads * k, r = q / R, c = q % R;
      if (!in[k] || r < H - 1 || r > H + kTile || c < H - 1 || c > H + kTile ||
          ((gi0 + c + gj0 + r) & 1) != rc)
        continue;
      const cx<P> up = U[q], a = U[q - 1], b = U[q + 1], s = U[q - R], n = U[q + R];
      const double dd = (double)cw[k] + ce[k] + cs[k] + cn[k];
      const P dr = (P)(sh.x + dd), di = (P)sh.y;
      RS[q] = cx<P>{fv[k].x + cw[k] * a.x + ce[k] * b.x + cs[k] * s.x + cn[k] * n.x -
                        dr * up.x + di * up.y,
                    fv[k].y + cw[k] * a.y + ce[k] * b.y + cs[k] * s.y + cn[k] * n.y -
                        dr * up.y - di * up.x};
    }
    __syncthreads();
    // coarse point (I, J) sits on fine (2I+1, 2J+1): 4/16 of the centre residual plus 1/16 of
    // each corner; the edge neighbours have the other colour, whose residual vanishes
    constexpr int KC = kTile / 2;
    for (int t = threadIdx.x; t < KC * KC; t += kTileThreads) {
      const int I = i0 / 2 + t % KC, J = j0 / 2 + t / KC;
      if (I >= Mc || J >= Mc) continue;
      const int q = (2 * J + 1 - gj0) * R + (2 * I + 1 - gi0);
      const cx<P> c0v = RS[q], c1 = RS[q - R - 1], c2 = RS[q - R + 1], c3 = RS[q + R - 1],
                  c4 = RS[q + R + 1];
      fc[(size_t)sys * Mc * Mc + (size_t)J * Mc + I] =
          cx<P>{(P)0.0625 * ((P)4 * c0v.x + c1.x + c2.x + c3.x + c4.x),
                (P)0.0625 * ((P)4 * c0v.y + c1.y + c2.y + c3.y + c4.y)};
    }
  }
  if (partials) {
    double v = acc2;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < kTileThreads / 64; ++i) t += red[i];
      partials[(size_t)sys * gridDim.x + tile] = t;
    }
  }
}

// ---- the small levels: one workgroup cycles one system entirely in LDS ----------
template <int D> __device__ __forceinline__ int npts_of(int M) { return D == 2 ? M * M : M; }

template <typename P, int D>
__device__ void lds_sweep(cx<P> *u, const cx<P> *f, const MgLev &L, cx<double> sh, double tau,
                          int color, bool zero, const cx<P> *uc) {
  const int M = L.M, half = (M + 1) / 2, rows = D == 2 ? M : 1, Mc = (M - 1) / 2;
  for (int t = threadIdx.x; t < rows * half; t += blockDim.x) {
    const int j = t / half, i = color_i<D>(t % half, j, color);
    if (i < M) u[(size_t)j * M + i] = gs_value<P, D>(u, f, L, sh, tau, i, j, zero, uc, Mc);
  }
  __syncthreads();
}

template <typename P, int D>
__global__ __launch_bounds__(kThreads) void k_mg_lds(cx<P> *__restrict__ utop,
                                                     const cx<P> *__restrict__ ftop,
                                                     MgLdsLevels lv,
                                                     const double *__restrict__ shifts,
                                                     double tau, int zero) {
  extern __shared__ unsigned char smem_raw[];
  cx<P> *smem = reinterpret_cast<cx<P> *>(smem_raw);
  const int sys = blockIdx.x;
  const cx<double> sh = sys_shift(shifts, sys);
  cx<P> *U[kMgMaxLds];
  cx<P> *F[kMgMaxLds];
  {
    size_t off = 0;
    for (int k = 0; k < lv.nl; ++k) {
      const int np = npts_of<D>(lv.lev[k].M);
      U[k] = smem + off;
      F[k] = smem + off + np;
      off += 2 * (size_t)np;
    }
  }
  const int np0 = npts_of<D>(lv.lev[0].M);
  for (int t = threadIdx.x; t < np0; t += blockDim.x) {
    F[0][t] = ftop[(size_t)sys * np0 + t];
    if (!zero) U[0][t] = utop[(size_t)sys * np0 + t];
  }
  __syncthreads();
  for (int k = 0; k + 1 < lv.nl; ++k) {  // down: pre-smooth, restrict
    const MgLev &L = lv.lev[k];
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 0, k > 0 || zero, nullptr);
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 1, false, nullptr);
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 0, false, nullptr);
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 1, false, nullptr);
    const int Mc = lv.lev[k + 1].M, rows = D == 2 ? Mc : 1;
    for (int t = threadIdx.x; t < rows * Mc; t += blockDim.x)
      F[k + 1][t] = restrict_val<P, D>(U[k], F[k], L, sh, tau, t % Mc, t / Mc);
    __syncthreads();
  }
  {  // coarsest level: one interior point (M + 1 is a power of two), solved exactly
    const int k = lv.nl - 1;
    if (threadIdx.x == 0)
      U[k][0] = gs_value<P, D>(U[k], F[k], lv.lev[k], sh, tau, 0, 0, true, nullptr, 0);
    __syncthreads();
  }
  for (int k = lv.nl - 2; k >= 0; --k) {  // up: correct and post-smooth
    const MgLev &L = lv.lev[k];
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 1, false, U[k + 1]);
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 0, false, nullptr);
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 1, false, nullptr);
    lds_sweep<P, D>(U[k], F[k], L, sh, tau, 0, false, nullptr);
  }
  for (int t = threadIdx.x; t < np0; t += blockDim.x) utop[(size_t)sys * np0 + t] = U[0][t];
}

// ---- host side --------------------------------------------------------------------
MgLev level(const wc_plan &p, int l) {
  MgLev L;
  L.M = p.mg_M[l];
  L.inv_h2 = p.mg_inv_h2[l];
  const double *a = l == 0 ? p.d_aface : p.d_mg_a + p.mg_aoff[l];
  L.ax = a;
  L.ay = p.dims == 2 ? a + (size_t)L.M * (L.M + 1) : nullptr;
  return L;
}

size_t level_pts(const wc_plan &p, int l) {
  return p.dims == 2 ? (size_t)p.mg_M[l] * p.mg_M[l] : (size_t)p.mg_M[l];
}

// 2D levels keep two u buffers: a tile pass reads one and writes the other (a workgroup's
// halo overlaps its neighbours' tiles), then mg_cur flips.
template <typename P> cx<P> *level_u_buf(const wc_plan &p, int l, int which) {
  if (l == 0) return (cx<P> *)(which ? p.d_mg_u2 : p.d_specB);
  return (cx<P> *)((char *)p.d_mg_work + p.mg_woff[l]) + (size_t)which * p.n * level_pts(p, l);
}
template <typename P> cx<P> *level_u(const wc_plan &p, int l) {
  return level_u_buf<P>(p, l, p.dims == 2 ? p.mg_cur[l] : 0);
}
template <typename P> cx<P> *level_f(const wc_plan &p, int l) {
  if (l == 0) return (cx<P> *)p.d_specA;
  return (cx<P> *)((char *)p.d_mg_work + p.mg_woff[l]) +
         (size_t)(p.dims == 2 ? 2 : 1) * p.n * level_pts(p, l);
}

unsigned blocks_for(size_t threads) { return (unsigned)((threads + kThreads - 1) / kThreads); }

template <typename P, int D>
hipError_t smooth(const wc_plan &p, int l, int color, bool zero, const cx<P> *uc) {
  const int M = p.mg_M[l], nsys = p.n;
  const size_t thr = (size_t)nsys * (D == 2 ? M : 1) * ((M + 1) / 2);
  ProfScope ps(p, K_MG_SMOOTH, 2.0 * nsys * level_pts(p, l) * sizeof(cx<P>) * (zero ? 0.5 : 1.5));
  hipLaunchKernelGGL((k_mg_smooth<P, D>), dim3(blocks_for(thr)), dim3(kThreads), 0, p.stream,
                     level_u<P>(p, l), level_f<P>(p, l), level(p, l), p.d_mg_shift, p.tau, color,
                     zero ? 1 : 0, uc, nsys);
  return hipGetLastError();
}


int tiles_x(int M) { return (M + kTile - 1) / kTile; }

// pre-smoothing (red first) with the restriction of its residual to level l+1, or
// post-smoothing (black first, coarse correction folded into the load; H = 5 when the
// residual partials are wanted)
template <typename P>
hipError_t tile_sweeps(const wc_plan &p, int l, bool post, bool zero, double *partials) {
  const int M = p.mg_M[l], tx = tiles_x(M);
  dim3 grid(tx * tx, p.n);
  const double arr = (double)p.n * level_pts(p, l) * sizeof(cx<P>);
  ProfScope ps(p, post ? K_MG_SMOOTH : K_MG_RESTRICT,
               arr * (zero ? 2.0 : 3.0) + arr / 4);
  const int cur = p.mg_cur[l];
  const cx<P> *uin = level_u_buf<P>(p, l, cur);
  cx<P> *uout = level_u_buf<P>(p, l, cur ^ 1);
  const cx<P> *f = level_f<P>(p, l);
  const MgLev L = level(p, l);
  if (!post)
    hipLaunchKernelGGL((k_mg_tile<P, 6, 4, true>), grid, dim3(kTileThreads), 0, p.stream, uin,
                       uout, f, L, p.d_mg_shift, p.tau, 0, zero ? 1 : 0, nullptr, tx, nullptr,
                       level_f<P>(p, l + 1));
  else if (partials)
    hipLaunchKernelGGL((k_mg_tile<P, 5, 4, false>), grid, dim3(kTileThreads), 0, p.stream, uin,
                       uout, f, L, p.d_mg_shift, p.tau, 1, 0, level_u<P>(p, l + 1), tx, partials,
                       nullptr);
  else
    hipLaunchKernelGGL((k_mg_tile<P, 4, 4, false>), grid, dim3(kTileThreads), 0, p.stream, uin,
                       uout, f, L, p.d_mg_shift, p.tau, 1, 0, level_u<P>(p, l + 1), tx, nullptr,
                       nullptr);
  p.mg_cur[l] = cur ^ 1;
  return hipGetLastError();
}

// whether the fine level's post-smoothing pass can also produce the residual partials
bool fused_norm(const wc_plan &p) {
  if (p.dims != 2 || p.mg_ltop == 0) return false;
  const size_t t = (size_t)tiles_x(p.mg_M[0]);
  return t * t * (size_t)p.n <= (size_t)kMgPartials;
}

template <typename P, int D>
hipError_t vcycle(const wc_plan &p, int l, bool zero, double *partials = nullptr) {
  hipError_t e;
  if (l == p.mg_ltop) {
    MgLdsLevels lv{};
    lv.nl = p.mg_nlev - l;
    size_t bytes = 0;
    for (int k = 0; k < lv.nl; ++k) {
      lv.lev[k] = level(p, l + k);
      bytes += 2 * level_pts(p, l + k) * sizeof(cx<P>);
    }
    ProfScope ps(p, K_MG_LDS, (double)p.n * level_pts(p, l) * sizeof(cx<P>) * (zero ? 2 : 3));
    hipLaunchKernelGGL((k_mg_lds<P, D>), dim3(p.n), dim3(kThreads), bytes, p.stream,
                       level_u<P>(p, l), level_f<P>(p, l), lv, p.d_mg_shift, p.tau, zero ? 1 : 0);
    return hipGetLastError();
  }
#define WC_E(x) if ((e = (x)) != hipSuccess) return e
  if constexpr (D == 2) {
    WC_E((tile_sweeps<P>(p, l, false, zero, nullptr)));  // also restricts to level l+1
  } else {
    WC_E((smooth<P, D>(p, l, 0, zero, nullptr)));
    WC_E((smooth<P, D>(p, l, 1, false, nullptr)));
    WC_E((smooth<P, D>(p, l, 0, false, nullptr)));
    WC_E((smooth<P, D>(p, l, 1, false, nullptr)));
    const size_t thr = (size_t)p.n * level_pts(p, l + 1);
    ProfScope ps(p, K_MG_RESTRICT,
                 (double)p.n * (2.0 * level_pts(p, l) + level_pts(p, l + 1)) * sizeof(cx<P>));
    hipLaunchKernelGGL((k_mg_restrict<P, D>), dim3(blocks_for(thr)), dim3(kThreads), 0,
                       p.stream, level_u<P>(p, l), level_f<P>(p, l), level(p, l),
                       level_f<P>(p, l + 1), p.d_mg_shift, p.tau, p.n);
    WC_E(hipGetLastError());
  }
  WC_E((vcycle<P, D>(p, l + 1, true)));
  if constexpr (D == 2) {
    WC_E((tile_sweeps<P>(p, l, true, false, partials)));
  } else {
    WC_E((smooth<P, D>(p, l, 1, false, level_u<P>(p, l + 1))));
    WC_E((smooth<P, D>(p, l, 0, false, nullptr)));
    WC_E((smooth<P, D>(p, l, 1, false, nullptr)));
    WC_E((smooth<P, D>(p, l, 0, false, nullptr)));
  }
#undef WC_E
  return hipSuccess;
}

int norm_blocks(const wc_plan &p) {
  const size_t np = level_pts(p, 0);
  size_t g = (np + 2 * kThreads - 1) / (2 * kThreads);
  const size_t cap = (size_t)kMgPartials / p.n;
  if (g > 64) g = 64;
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

template <typename P, int D> hipError_t norms(const wc_plan &p, bool resid_mode) {
  const int gx = norm_blocks(p);
  {
    ProfScope ps(p, K_MG_NORM, (double)p.n * level_pts(p, 0) * sizeof(cx<P>) * (resid_mode ? 1.5 : 1.0));
    hipLaunchKernelGGL((k_mg_norms<P, D>), dim3(gx, p.n), dim3(kThreads), 0, p.stream,
                       level_u<P>(p, 0), level_f<P>(p, 0), level(p, 0), p.d_mg_shift, p.tau,
                       resid_mode ? 1 : 0, p.d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  ProfScope ps(p, K_FINALIZE, 8.0 * p.n * gx);
  hipLaunchKernelGGL(k_mg_reduce, dim3(1), dim3(kThreads), 0, p.stream, p.d_partials, gx, p.n,
                     p.d_mg_fn2, p.d_scal, S_MG_RELRES, resid_mode ? 1 : 0);
  return hipGetLastError();
}

template <typename P> hipError_t mix(const wc_plan &p, bool out) {
  const size_t cnt = (size_t)(p.n / 2) * p.m;
  const double *mx = p.opts.method == WC_GMRES_PS ? p.d_mg_mix : nullptr;
  const cx<P> *src = out ? (const cx<P> *)level_u<P>(p, 0) : (const cx<P> *)p.d_specA;
  ProfScope ps(p, K_MG_MIX, 2.0 * p.n * p.m * sizeof(cx<P>));
  hipLaunchKernelGGL((k_mg_mix<P>), dim3(blocks_for(cnt)), dim3(kThreads), 0, p.stream, src,
                     (cx<P> *)p.d_specA, mx, p.m, p.n / 2, 1.0 / p.n, out ? 1 : 0);
  return hipGetLastError();
}

template <typename P, int D> hipError_t mg_apply_t(const wc_plan &p) {
  hipError_t e;
  if ((e = mix<P>(p, false)) != hipSuccess) return e;
  const bool fp32 = sizeof(P) == 4;
  double tol = p.opts.mg_tol;
  if (fp32 && tol > 0.0 && tol < kMgTolFp32) tol = kMgTolFp32;
  const bool check = tol > 0.0;
  if (check && (e = norms<P, D>(p, false)) != hipSuccess) return e;
  int c = 0;
  const bool fused = check && fused_norm(p);
  for (; c < p.opts.mg_max_cycles;) {
    if ((e = vcycle<P, D>(p, 0, c == 0, fused ? p.d_partials : nullptr)) != hipSuccess) return e;
    ++c;
    if (!check) continue;
    if (fused) {
      const int t = tiles_x(p.mg_M[0]);
      ProfScope ps(p, K_FINALIZE, 8.0 * p.n * t * t);
      hipLaunchKernelGGL(k_mg_reduce, dim3(1), dim3(kThreads), 0, p.stream, p.d_partials, t * t,
                         p.n, p.d_mg_fn2, p.d_scal, S_MG_RELRES, 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if ((e = norms<P, D>(p, true)) != hipSuccess) {
      return e;
    }
    if ((e = hipMemcpyAsync(p.h_scal + S_MG_RELRES, p.d_scal + S_MG_RELRES, sizeof(double),
                            hipMemcpyDeviceToHost, p.stream)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(p.stream)) != hipSuccess) return e;
    const double rr = p.h_scal[S_MG_RELRES];
    if (!(rr > tol)) break;  // converged (a NaN surfaces in the Krylov scalars)
  }
  p.mg_cycles_last = c;
  if (c > p.mg_cycles_max) p.mg_cycles_max = c;
  return mix<P>(p, true);
}

}  // namespace

hipError_t mg_space_apply(const wc_plan &p) {
  const bool f32 = p.opts.precision == WC_MIXED;
  if (p.dims == 1) return f32 ? mg_apply_t<float, 1>(p) : mg_apply_t<double, 1>(p);
  return f32 ? mg_apply_t<float, 2>(p) : mg_apply_t<double, 2>(p);
}

size_t mg_lds_bytes(int dims, int M, int precision) {
  const size_t es = precision == WC_MIXED ? 8 : 16;
  size_t b = 0;
  for (int Ml = M; Ml >= 1; Ml = (Ml - 1) / 2) {
    b += 2 * (dims == 2 ? (size_t)Ml * Ml : (size_t)Ml) * es;
    if (Ml == 1) break;
  }
  return b;
}

}  // namespace wc
