// FP64 kernels of the solve around the preconditioner: the all-at-once operator,
// right-hand side assembly, recovery of y and p, deterministic reductions and the
// device-side scalar steps of MINRES.
//
// Operator (eqn:matrix_A, eqn:matrix_T): T = B_n kron I + tau I kron K with
// B_n = (B^(2))^{-1} B^(1) (Section 1).  B_n x is the forward recurrence
//   z_k = (x_k - x_{k-1} - (1-theta) z_{k-1}) / theta,
// B_n^T x the backward recurrence
//   u_k = (x_k - (1-theta) u_{k+1}) / theta,  z_k = u_k - u_{k+1},
// so one thread per spatial point marches through time, O(nm) for every theta.
// K = -L_h is the conservative five-point (three-point) stencil with face
// coefficients; Dirichlet neighbours are zero.

#include "wc_internal.h"

namespace wc {
namespace {

typedef double d2v __attribute__((ext_vector_type(2)));

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
  return r;  // valid in thread 0
}

struct Stencil {
  double cc, cw, ce, cs, cn;   // K x = cc x_P - cw x_W - ce x_E - cs x_S - cn x_N
  int ow, oe, os, on;          // neighbour offsets (0 when absent: coefficient is 0)
};

// K_m for finite differences (the 3/5-point stencil), or, with diag (finite elements in
// sine coordinates), the diagonal operator M^{-1/2} K M^{-1/2}: diag[j1] (+ diag[j2]).
// neumann: M nodes per dimension including the boundary nodes, the missing neighbour of
// a boundary node mirrored onto the inner one (its weight doubles); constant a.
__device__ __forceinline__ Stencil make_stencil(int s, int M, int dims, double inv_h2,
                                                const double *__restrict__ aface,
                                                const double *__restrict__ diag = nullptr,
                                                bool neumann = false) {
  Stencil st;
  if (neumann) {
    const int i = dims == 1 ? s : s % M, j = dims == 1 ? 0 : s / M;
    st.cw = i > 0 ? inv_h2 * (i == M - 1 ? 2.0 : 1.0) : 0.0;
    st.ce = i < M - 1 ? inv_h2 * (i == 0 ? 2.0 : 1.0) : 0.0;
    st.ow = i > 0 ? -1 : 0;
    st.oe = i < M - 1 ? 1 : 0;
    st.cc = 2.0 * inv_h2;
    st.cs = st.cn = 0.0;
    st.os = st.on = 0;
    if (dims == 2) {
      st.cs = j > 0 ? inv_h2 * (j == M - 1 ? 2.0 : 1.0) : 0.0;
      st.cn = j < M - 1 ? inv_h2 * (j == 0 ? 2.0 : 1.0) : 0.0;
      st.os = j > 0 ? -M : 0;
      st.on = j < M - 1 ? M : 0;
      st.cc = 4.0 * inv_h2;
    }
    return st;
  }
  if (diag) {
    st.cc = dims == 1 ? diag[s] : diag[s % M] + diag[s / M];
    st.cw = st.ce = st.cs = st.cn = 0.0;
    st.ow = st.oe = st.os = st.on = 0;
    return st;
  }
  if (dims == 1) {
    const double aw = aface ? aface[s] : 1.0;
    const double ae = aface ? aface[s + 1] : 1.0;
    st.cc = inv_h2 * (aw + ae);
    st.cw = s > 0 ? inv_h2 * aw : 0.0;
    st.ce = s < M - 1 ? inv_h2 * ae : 0.0;
    st.ow = s > 0 ? -1 : 0;
    st.oe = s < M - 1 ? 1 : 0;
    st.cs = st.cn = 0.0;
    st.os = st.on = 0;
    return st;
  }
  const int i = s % M, j = s / M;
  double aw = 1.0, ae = 1.0, as = 1.0, an = 1.0;
  if (aface) {
    const double *ax = aface;                      // (M, M+1)
    const double *ay = aface + (size_t)M * (M + 1);  // (M+1, M)
    aw = ax[(size_t)j * (M + 1) + i];
    ae = ax[(size_t)j * (M + 1) + i + 1];
    as = ay[(size_t)j * M + i];
    an = ay[(size_t)(j + 1) * M + i];
  }
  st.cc = inv_h2 * (aw + ae + as + an);
  st.cw = i > 0 ? inv_h2 * aw : 0.0;
  st.ce = i < M - 1 ? inv_h2 * ae : 0.0;
  st.cs = j > 0 ? inv_h2 * as : 0.0;
  st.cn = j < M - 1 ? inv_h2 * an : 0.0;
  st.ow = i > 0 ? -1 : 0;
  st.oe = i < M - 1 ? 1 : 0;
  st.os = j > 0 ? -M : 0;
  st.on = j < M - 1 ? M : 0;
  return st;
}

__device__ __forceinline__ double apply_stencil(const Stencil &st, const double *__restrict__ xk,
                                                int s) {
  return st.cc * xk[s] - st.cw * xk[s + st.ow] - st.ce * xk[s + st.oe] - st.cs * xk[s + st.os] -
         st.cn * xk[s + st.on];
}

struct MvArgs {
  int n, M, dims, m, sym;
  double theta, tau, alpha, inv_h2;
  const double *aface;
  const double *diag;  // finite elements: the 1D eigenvalues of M^{-1/2} K M^{-1/2}
  double ssign;  // with sub: y = ssign * (A x - sub)
  int neumann;   // Neumann data (nodes including the boundary)
};

// blockIdx.y == 0: T x1 - alpha x2 (forward in time); 1: T^T x2 + alpha x1 (backward).
// Output block rows: A (sym) = [alpha x1 + T^T x2; T x1 - alpha x2],
//                    A_hat   = [T x1 - alpha x2; alpha x1 + T^T x2].
// partials[dir*gridDim.x + block] = this block's share of <y, x>.
// With sub != nullptr the kernel writes ssign * (y - sub) (same layout as y) and the
// partial sums are this block's share of the squared norm of what it wrote (a residual's
// norm without another pass over it).
// Each thread marches kMvPts spatial points (kThreads apart, so every load of a wave stays
// one contiguous 512-byte run) through time, with the loads of kMvKb time levels issued
// before the recurrences consume them: 2 points x 4 levels measured 7% faster than
// 1 point x 8 levels at M = 511, n = 512, and 1 x 16 or 1 x 4 slower.
// DG (diagonal operator) and SUB (subtracted vector) are template arguments: a run-time
// branch around the loads splits the batch, and every batch then waits for its loads one
// branch at a time.
constexpr int kMvPts = 2, kMvKb = 4;
template <bool DG, bool SUB>
__global__ __launch_bounds__(kThreads) void k_matvec(const double *__restrict__ x,
                                                     double *__restrict__ y,
                                                     const double *__restrict__ sub, MvArgs a,
                                                     double *__restrict__ partials) {
  __shared__ double red[kThreads / 64];
  constexpr int PP = kMvPts, KB = kMvKb;
  const int dir = blockIdx.y;
  const size_t nm = (size_t)a.n * a.m;
  const double *xs = dir == 0 ? x : x + nm;
  const double *xo = dir == 0 ? x + nm : x;
  const size_t ooff = a.sym ? (dir == 0 ? nm : 0) : (dir == 0 ? 0 : nm);
  double *yo = y + ooff;
  const double *so = SUB ? sub + ooff : nullptr;
  const double omt = 1.0 - a.theta, ith = 1.0 / a.theta;
  int sp[PP];
  bool live[PP];
  Stencil st[PP];
  double zprev[PP], xprev[PP];
#pragma unroll
  for (int p = 0; p < PP; ++p) {
    const int s = blockIdx.x * (kThreads * PP) + p * kThreads + threadIdx.x;
    live[p] = s < a.m;
    sp[p] = live[p] ? s : a.m - 1;  // a point past the end repeats the last one, stores nothing
    st[p] = make_stencil(sp[p], a.M, a.dims, a.inv_h2, a.aface, a.diag, a.neumann);
    zprev[p] = 0.0;
    xprev[p] = 0.0;
  }
  double acc = 0.0;
  for (int kk0 = 0; kk0 < a.n; kk0 += KB) {
    double xc[KB][PP], kx[KB][PP], xok[KB][PP], sk[KB][PP];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int kk = kk0 + u < a.n ? kk0 + u : a.n - 1;
      const int k = dir == 0 ? kk : a.n - 1 - kk;
      const double *xk = xs + (size_t)k * a.m;
#pragma unroll
      for (int p = 0; p < PP; ++p) {
        const int s = sp[p];
        xc[u][p] = xk[s];
        kx[u][p] = DG ? st[p].cc * xc[u][p] : apply_stencil(st[p], xk, s);
        xok[u][p] = xo[(size_t)k * a.m + s];
        sk[u][p] = SUB ? so[(size_t)k * a.m + s] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int kk = kk0 + u;
      if (kk >= a.n) break;
      const int k = dir == 0 ? kk : a.n - 1 - kk;
#pragma unroll
      for (int p = 0; p < PP; ++p) {
        double out;
        if (dir == 0) {
          const double z = (xc[u][p] - xprev[p] - omt * zprev[p]) * ith;
          out = z + a.tau * kx[u][p] - a.alpha * xok[u][p];
          zprev[p] = z;
          xprev[p] = xc[u][p];
        } else {
          const double uu = (xc[u][p] - omt * zprev[p]) * ith;
          out = (uu - zprev[p]) + a.tau * kx[u][p] + a.alpha * xok[u][p];
          zprev[p] = uu;
        }
        if (!live[p]) continue;
        const size_t g = (size_t)k * a.m + sp[p];
        if (SUB) {
          const double v = a.ssign * (out - sk[u][p]);
          yo[g] = v;
          acc += v * v;
        } else {
          yo[g] = out;
          acc += out * (a.sym ? xok[u][p] : xc[u][p]);
        }
      }
    }
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) partials[dir * gridDim.x + blockIdx.x] = r;
}

struct RhsArgs {
  int n, M, dims, m, sym;
  double theta, tau, sqrt_gamma, inv_h2;
  const double *aface;
  int y0_terms;  // 0: leave out the y0 terms (finite elements add them in sine coordinates)
  int neumann;   // Neumann data (nodes including the boundary)
};

// f_tilde, g_tilde of Section 1 with M = I, then b = [g; sqrt(gamma) f] (sym) or
// [sqrt(gamma) f; g].  One thread per (time slice k+1, point s).
__global__ __launch_bounds__(kThreads) void k_rhs(const double *__restrict__ f,
                                                  const double *__restrict__ g,
                                                  const double *__restrict__ y0,
                                                  double *__restrict__ b, RhsArgs a) {
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const size_t nm = (size_t)a.n * a.m;
  if (idx >= nm) return;
  const unsigned ui = (unsigned)idx;  // n m < 2^32
  const int k = (int)(ui / (unsigned)a.m), s = (int)(ui - (unsigned)k * (unsigned)a.m);
  const double th = a.theta, omt = 1.0 - th;
  double ft = a.tau * (th * f[(size_t)(k + 1) * a.m + s] + omt * f[(size_t)k * a.m + s]);
  double gt = a.tau * (th * g[(size_t)k * a.m + s] + omt * g[(size_t)(k + 1) * a.m + s]);
  if (k == 0 && a.y0_terms) {
    const Stencil st = make_stencil(s, a.M, a.dims, a.inv_h2, a.aface, nullptr, a.neumann);
    ft += y0[s] - omt * a.tau * apply_stencil(st, y0, s);
    gt -= a.tau * omt * y0[s];
  }
  if (a.sym) {
    b[idx] = gt;
    b[nm + idx] = a.sqrt_gamma * ft;
  } else {
    b[idx] = a.sqrt_gamma * ft;
    b[nm + idx] = gt;
  }
}

// y from theta y_1 = yt_1, theta y_k + (1-theta) y_{k-1} = yt_k (yt = x1/sqrt(gamma));
// p from theta p^{(n-1)} = pt_n, theta p^{(k-1)} + (1-theta) p^{(k)} = pt_k.
__global__ __launch_bounds__(kThreads) void k_recover(const double *__restrict__ x,
                                                      double *__restrict__ y,
                                                      double *__restrict__ p,
                                                      double *__restrict__ u, int n, int m,
                                                      double theta, double inv_sqrt_gamma,
                                                      double inv_gamma) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= m) return;
  const size_t nm = (size_t)n * m;
  const double omt = 1.0 - theta, ith = 1.0 / theta;
  // the loads of KB time levels are issued before the recurrence consumes them
  constexpr int KB = 8;
  if (blockIdx.y == 0) {
    double prev = 0.0;
    for (int k0 = 0; k0 < n; k0 += KB) {
      double xv[KB];
#pragma unroll
      for (int u2 = 0; u2 < KB; ++u2)
        xv[u2] = k0 + u2 < n ? x[(size_t)(k0 + u2) * m + s] : 0.0;
#pragma unroll
      for (int u2 = 0; u2 < KB; ++u2) {
        if (k0 + u2 >= n) break;
        const double v = (xv[u2] * inv_sqrt_gamma - omt * prev) * ith;
        y[(size_t)(k0 + u2) * m + s] = v;
        prev = v;
      }
    }
  } else {
    double next = 0.0;
    for (int k0 = n - 1; k0 >= 0; k0 -= KB) {
      double xv[KB];
#pragma unroll
      for (int u2 = 0; u2 < KB; ++u2)
        xv[u2] = k0 - u2 >= 0 ? x[nm + (size_t)(k0 - u2) * m + s] : 0.0;
#pragma unroll
      for (int u2 = 0; u2 < KB; ++u2) {
        const int k = k0 - u2;
        if (k < 0) break;
        const double v = (xv[u2] - omt * next) * ith;
        p[(size_t)k * m + s] = v;
        if (u) u[(size_t)k * m + s] = v * inv_gamma;
        next = v;
      }
    }
  }
}

// ---- streaming BLAS-1 with deterministic reductions ---------------------------

// 16-byte accesses (pairs of elements) when every vector is 16-byte aligned and the length
// even (system vectors have 2 n m elements); the streams present are template arguments, so
// no run-time branch splits a thread's loads.
__device__ __forceinline__ bool pairs_ok(size_t nv, const void *a, const void *b = nullptr,
                                         const void *c = nullptr, const void *d = nullptr,
                                         const void *e = nullptr, const void *f = nullptr) {
  const uintptr_t m = (uintptr_t)a | (uintptr_t)b | (uintptr_t)c | (uintptr_t)d |
                      (uintptr_t)e | (uintptr_t)f;
  return (nv & 1) == 0 && (m & 15) == 0;
}

template <bool HB, bool HC>
__global__ __launch_bounds__(kThreads) void k_lincomb3(double *__restrict__ dst,
                                                       const double *__restrict__ a,
                                                       const double *__restrict__ b,
                                                       const double *__restrict__ c, size_t nv,
                                                       const double *__restrict__ scal,
                                                       int slot, double h0, double h1,
                                                       double h2) {
  const double c0 = slot >= 0 ? scal[slot] : h0;
  const double c1 = slot >= 0 ? scal[slot + 1] : h1;
  const double c2 = slot >= 0 ? scal[slot + 2] : h2;
  if (pairs_ok(nv, dst, a, b, c)) {
    const size_t np = nv >> 1;
    const d2v *a2 = reinterpret_cast<const d2v *>(a);
    const d2v *b2 = reinterpret_cast<const d2v *>(b);
    const d2v *c2v = reinterpret_cast<const d2v *>(c);
    d2v *o2 = reinterpret_cast<d2v *>(dst);
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < np;
         i += (size_t)gridDim.x * kThreads) {
      d2v v = c0 * a2[i];
      if (HB) v += c1 * b2[i];
      if (HC) v += c2 * c2v[i];
      o2[i] = v;
    }
    return;
  }
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nv;
       i += (size_t)gridDim.x * kThreads) {
    double v = c0 * a[i];
    if (HB) v += c1 * b[i];
    if (HC) v += c2 * c[i];
    dst[i] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_dot(const double *__restrict__ a,
                                                  const double *__restrict__ b, size_t nv,
                                                  double *__restrict__ partials) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  if (pairs_ok(nv, a, b)) {
    const size_t np = nv >> 1;
    const d2v *a2 = reinterpret_cast<const d2v *>(a);
    const d2v *b2 = reinterpret_cast<const d2v *>(b);
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < np;
         i += (size_t)gridDim.x * kThreads) {
      const d2v x = a2[i], y = b2[i];
      acc += x.x * y.x + x.y * y.y;
    }
  } else {
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nv;
         i += (size_t)gridDim.x * kThreads)
      acc += a[i] * b[i];
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// scal[slot + j] = sum_{i < count} partials[j*count + i], fixed order.
__global__ __launch_bounds__(kThreads) void k_finalize(const double *__restrict__ partials,
                                                       int count, int nsum,
                                                       double *__restrict__ scal, int slot) {
  __shared__ double red[kThreads / 64];
  for (int j = 0; j < nsum; ++j) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kThreads) acc += partials[(size_t)j * count + i];
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) scal[slot + j] = r;
  }
}

// MINRES direction / iterate / residual update (coefficients in scal):
//   w0 <- CWZ z + CW0 w0 + CW1 w1   (the new direction overwrites w_{j-1})
//   x  <- x + CX w0
//   r  <- CRR r + CRV vnew,   partial sums of ||r||^2
__global__ __launch_bounds__(kThreads) void k_minres_update(double *__restrict__ w0,
                                                            const double *__restrict__ w1,
                                                            const double *__restrict__ z,
                                                            double *__restrict__ x,
                                                            double *__restrict__ r,
                                                            const double *__restrict__ vnew,
                                                            size_t nv,
                                                            const double *__restrict__ scal,
                                                            double *__restrict__ partials) {
  __shared__ double red[kThreads / 64];
  const double cwz = scal[S_CWZ], cw0 = scal[S_CW0], cw1 = scal[S_CW1];
  const double cxx = scal[S_CX], crr = scal[S_CRR], crv = scal[S_CRV];
  double acc = 0.0;
  if (pairs_ok(nv, w0, w1, z, x, r, vnew)) {
    const size_t np = nv >> 1;
    d2v *w02 = reinterpret_cast<d2v *>(w0);
    const d2v *w12 = reinterpret_cast<const d2v *>(w1);
    const d2v *z2 = reinterpret_cast<const d2v *>(z);
    d2v *x2 = reinterpret_cast<d2v *>(x);
    d2v *r2 = reinterpret_cast<d2v *>(r);
    const d2v *v2 = reinterpret_cast<const d2v *>(vnew);
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < np;
         i += (size_t)gridDim.x * kThreads) {
      const d2v zi = z2[i], a0 = w02[i], a1 = w12[i], xi = x2[i], ri = r2[i], vi = v2[i];
      const d2v wn = cwz * zi + cw0 * a0 + cw1 * a1;
      w02[i] = wn;
      x2[i] = xi + cxx * wn;
      const d2v rn = crr * ri + crv * vi;
      r2[i] = rn;
      acc += rn.x * rn.x + rn.y * rn.y;
    }
  } else {
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nv;
         i += (size_t)gridDim.x * kThreads) {
      const double wn = cwz * z[i] + cw0 * w0[i] + cw1 * w1[i];
      w0[i] = wn;
      x[i] += cxx * wn;
      const double rn = crr * r[i] + crv * vnew[i];
      r[i] = rn;
      acc += rn * rn;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// One block: reduce `nparts` partials and advance the MINRES scalar recurrences.
// stage 0: init from <z1, v1>; 1: after A z (delta); 2: after P^{-1} v_new (gamma_new,
// Givens rotation, update coefficients); 3: after the update (true residual norm).
__global__ __launch_bounds__(kThreads) void k_minres_scalar(const double *__restrict__ partials,
                                                            int nparts, double *__restrict__ S,
                                                            int stage, double tol) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) acc += partials[i];
  const double dot = block_sum(acc, red);
  if (threadIdx.x != 0) return;
  if (stage == 0) {
    if (!(dot >= 0.0) || !isfinite(dot)) {
      S[S_STATUS] = isfinite(dot) ? ST_BREAKDOWN : ST_NONFINITE;
      return;
    }
    const double g = sqrt(dot);
    S[S_GAMMA_PREV] = 1.0;
    S[S_GAMMA] = g;
    S[S_ETA] = g;
    S[S_C_PREV] = 1.0;
    S[S_C] = 1.0;
    S[S_S_PREV] = 0.0;
    S[S_S] = 0.0;
    S[S_STATUS] = g == 0.0 ? ST_CONVERGED : ST_RUNNING;
  } else if (stage == 1) {
    const double g = S[S_GAMMA];
    const double delta = dot / (g * g);
    S[S_DELTA] = delta;
    S[S_CV0] = 1.0 / g;
    S[S_CV1] = -delta / g;
    S[S_CV2] = -g / S[S_GAMMA_PREV];
    if (!isfinite(delta)) S[S_STATUS] = ST_NONFINITE;
  } else if (stage == 2) {
    if (!isfinite(dot)) {
      S[S_STATUS] = ST_NONFINITE;
      return;
    }
    if (dot < 0.0) S[S_STATUS] = ST_BREAKDOWN;
    const double gn = dot > 0.0 ? sqrt(dot) : 0.0;
    const double g = S[S_GAMMA], delta = S[S_DELTA];
    const double c = S[S_C], cp = S[S_C_PREV], s = S[S_S], sp = S[S_S_PREV], eta = S[S_ETA];
    const double a0 = c * delta - cp * s * g;
    const double a1 = hypot(a0, gn);
    const double a2 = s * delta + cp * c * g;
    const double a3 = sp * g;
    const double cn = a0 / a1, sn = gn / a1;
    const double eta_n = -sn * eta;
    S[S_CWZ] = 1.0 / (g * a1);
    S[S_CW0] = -a3 / a1;
    S[S_CW1] = -a2 / a1;
    S[S_CX] = cn * eta;
    S[S_CRR] = sn * sn;
    S[S_CRV] = gn > 0.0 ? cn * eta_n / gn : 0.0;
    S[S_GAMMA_PREV] = g;
    S[S_GAMMA] = gn;
    S[S_C_PREV] = c;
    S[S_C] = cn;
    S[S_S_PREV] = s;
    S[S_S] = sn;
    S[S_ETA] = eta_n;
    if (!isfinite(a1) || a1 == 0.0) S[S_STATUS] = ST_BREAKDOWN;
  } else {
    S[S_RNORM2] = dot;
    S[S_ITER] += 1.0;
    const double rel = sqrt(dot) / S[S_BNORM];
    if (!isfinite(rel)) {
      S[S_STATUS] = ST_NONFINITE;
    } else if (S[S_STATUS] == ST_RUNNING && (rel <= tol || S[S_GAMMA] == 0.0)) {
      S[S_STATUS] = ST_CONVERGED;
    }
  }
}

// Gram-Schmidt bookkeeping for GMRES iteration j (basis V_0..V_j, new vector w).
//  stage 1: D1_i = <V_i, w>, WN2 = ||w||^2, GSC_i = D1_i / NU2_i
//  stage 2: WP2 = ||w'||^2; REORTH = WP2 < kReorthEta2 * WN2 (the projection cancelled
//           most of the norm: orthogonality may be lost, project again); else NU2_{j+1} = WP2
//  stage 3 (when REORTH): D2_i = <V_i, w'>, GSC_i = D2_i / NU2_i
//  stage 4 (when REORTH): WPP2 = ||w''||^2, NU2_{j+1} = WPP2
__device__ void gs_finalize_block(const double *__restrict__ partials, int count,
                                  double *__restrict__ S, int stage, int j, double *red) {
  if ((stage == 3 || stage == 4) && S[S_REORTH] == 0.0) return;
  const int nsum = stage == 1 ? j + 2 : (stage == 3 ? j + 1 : 1);
  for (int t = 0; t < nsum; ++t) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kThreads) acc += partials[(size_t)t * count + i];
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) {
      if (stage == 1) {
        if (t <= j) {
          S[S_D1 + t] = r;
          S[S_GSC + t] = r / S[S_NU2 + t];
        } else {
          S[S_WN2] = r;
        }
      } else if (stage == 2) {
        S[S_WP2] = r;
        const bool again = r < kReorthEta2 * S[S_WN2];
        S[S_REORTH] = again ? 1.0 : 0.0;
        S[S_WPP2] = r;
        if (!again) S[S_NU2 + j + 1] = r;
      } else if (stage == 3) {
        S[S_D2 + t] = r;
        S[S_GSC + t] = r / S[S_NU2 + t];
      } else {
        S[S_WPP2] = r;
        S[S_NU2 + j + 1] = r;
      }
    }
  }
}

// End of a reduction kernel whose thread 0 has written this workgroup's partials: the
// workgroup that finishes last (device-scope counter in the scalar array) folds all
// partials into the Gram-Schmidt scalars and resets the counter for the next launch.
__device__ void finalize_if_last(const double *__restrict__ partials, double *__restrict__ S,
                                 int stage, int j, double *red) {
  __shared__ bool last;
  unsigned int *cnt = reinterpret_cast<unsigned int *>(S + S_GS_COUNT);
  if (threadIdx.x == 0) {
    __threadfence();  // this workgroup's partials before its count
    last = atomicAdd(cnt, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();  // every other workgroup's partials are visible after its count
  gs_finalize_block(partials, gridDim.x, S, stage, j, red);
  if (threadIdx.x == 0) atomicExch(cnt, 0u);
}

// <basis_i, w> for i < NB (and <w, w> when SELF), basis vectors contiguous with stride nv.
// partials[j * gridDim.x + block].  Does nothing when gate && *gate == 0.
template <int NB, bool SELF>
__global__ __launch_bounds__(kThreads) void k_multidot(const double *__restrict__ basis,
                                                       const double *__restrict__ w, size_t nv,
                                                       double *__restrict__ partials,
                                                       const double *__restrict__ gate,
                                                       double *__restrict__ S, int stage, int jj) {
  if (gate && *gate == 0.0) return;
  __shared__ double red[kThreads / 64];
  constexpr int NS = NB + (SELF ? 1 : 0);
  double acc[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) acc[j] = 0.0;
  if ((nv & 1) == 0) {  // pairs of elements: 16-byte loads (every vector starts 16-aligned)
    const size_t np = nv >> 1;
    const d2v *w2 = reinterpret_cast<const d2v *>(w);
    const d2v *b2 = reinterpret_cast<const d2v *>(basis);
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < np;
         i += (size_t)gridDim.x * kThreads) {
      const d2v wi = w2[i];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const d2v b = __builtin_nontemporal_load(b2 + (size_t)j * np + i);
        acc[j] += b.x * wi.x + b.y * wi.y;
      }
      if (SELF) acc[NS - 1] += wi.x * wi.x + wi.y * wi.y;
    }
  } else {
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nv;
         i += (size_t)gridDim.x * kThreads) {
      const double wi = w[i];
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[j] += basis[(size_t)j * nv + i] * wi;
      if (SELF) acc[NS - 1] += wi * wi;
    }
  }
  // every sum's wave reductions first, then thread 0 adds the waves' sums (block_sum's order)
  // and writes the partials: one barrier instead of two per sum
  __shared__ double wsum[NS * (kThreads / 64)];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    double v = acc[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) wsum[j * (kThreads / 64) + wv] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < NS; ++j) {
      double r = 0.0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) r += wsum[j * (kThreads / 64) + w];
      partials[(size_t)j * gridDim.x + blockIdx.x] = r;
    }
  }
  if (stage) finalize_if_last(partials, S, stage, jj, red);
}

// w += sign * sum_i scal[slot+i] basis_i  (optional partials of ||w||^2); gated like above
template <int NB>
__global__ __launch_bounds__(kThreads) void k_multiaxpy(double *__restrict__ w,
                                                        const double *__restrict__ basis,
                                                        size_t nv, const double *__restrict__ scal,
                                                        int slot, double sign,
                                                        double *__restrict__ partials,
                                                        const double *__restrict__ gate,
                                                        double *__restrict__ S, int stage,
                                                        int jj) {
  if (gate && *gate == 0.0) return;
  __shared__ double red[kThreads / 64];
  double c[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) c[j] = sign * scal[slot + j];
  double acc = 0.0;
  if ((nv & 1) == 0) {  // pairs of elements: 16-byte loads and stores
    const size_t np = nv >> 1;
    d2v *w2 = reinterpret_cast<d2v *>(w);
    const d2v *b2 = reinterpret_cast<const d2v *>(basis);
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < np;
         i += (size_t)gridDim.x * kThreads) {
      d2v v = w2[i];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const d2v b = __builtin_nontemporal_load(b2 + (size_t)j * np + i);
        v.x += c[j] * b.x;
        v.y += c[j] * b.y;
      }
      __builtin_nontemporal_store(v, w2 + i);
      acc += v.x * v.x + v.y * v.y;
    }
  } else {
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nv;
         i += (size_t)gridDim.x * kThreads) {
      double v = w[i];
#pragma unroll
      for (int j = 0; j < NB; ++j) v += c[j] * basis[(size_t)j * nv + i];
      w[i] = v;
      acc += v * v;
    }
  }
  if (partials) {
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
    if (stage) finalize_if_last(partials, S, stage, jj, red);
  }
}

__global__ __launch_bounds__(kThreads) void k_gs_finalize(const double *__restrict__ partials,
                                                          int count, double *__restrict__ S,
                                                          int stage, int j) {
  __shared__ double red[kThreads / 64];
  gs_finalize_block(partials, count, S, stage, j, red);
}

__global__ __launch_bounds__(kThreads) void k_fill(double *__restrict__ dst, double val,
                                                   size_t count) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kThreads)
    dst[i] = val;
}


// ---- low-rank GMRES setup -------------------------------------------------------
// s0_1[s] = sum_k g_k r0_1[k][s] / |g|^2, s0_2[s] = sum_k r_k r0_2[k][s] / |r|^2: the
// coefficients of the orthogonal projection of r0 on {[g (x) a; r (x) b]}.
__global__ __launch_bounds__(kThreads) void k_lr_project(const double *__restrict__ r0,
                                                         const double *__restrict__ gr,
                                                         double *__restrict__ s0, int n, int m,
                                                         double inv_g2, double inv_r2) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= m) return;
  const double *a = r0, *b = r0 + (size_t)n * m;
  double sa = 0.0, sb = 0.0;
  constexpr int KB = 8;  // loads of KB time levels issued together; the sums keep their order
  for (int k0 = 0; k0 < n; k0 += KB) {
    double va[KB], vb[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = k0 + u < n ? k0 + u : n - 1;
      va[u] = a[(size_t)k * m + s];
      vb[u] = b[(size_t)k * m + s];
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      if (k0 + u < n) {
        sa += gr[k0 + u] * va[u];
        sb += gr[n + k0 + u] * vb[u];
      }
    }
  }
  s0[s] = sa * inv_g2;
  s0[m + s] = sb * inv_r2;
}

// partials of ||r0 - [g (x) s0_1; r (x) s0_2]||^2
__global__ __launch_bounds__(kThreads) void k_lr_perp(const double *__restrict__ r0,
                                                      const double *__restrict__ gr,
                                                      const double *__restrict__ s0, int n,
                                                      int m, double *__restrict__ partials) {
  __shared__ double red[kThreads / 64];
  const size_t nm = (size_t)n * m;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nm;
       i += (size_t)gridDim.x * kThreads) {
    const unsigned ui = (unsigned)i;  // n m < 2^32
    const int k = (int)(ui / (unsigned)m), s = (int)(ui - (unsigned)k * (unsigned)m);
    const double d1 = r0[i] - gr[k] * s0[s];
    const double d2 = r0[nm + i] - gr[n + k] * s0[m + s];
    acc += d1 * d1 + d2 * d2;
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// S[slot] = N0 (sum of the partials), S[slot + 1] = sqrt(N0) or 0 when N0 <= tiny * ||r0||^2;
// hat = [S[slot + 1], |g| s0_1, |r| s0_2]
__global__ __launch_bounds__(kThreads) void k_lr_hat0(const double *__restrict__ partials,
                                                      int count, double *__restrict__ S,
                                                      int slot,
                                                      const double *__restrict__ r0n2p,
                                                      const double *__restrict__ s0, int m,
                                                      double gn, double rn,
                                                      double *__restrict__ hat) {
  __shared__ double red[kThreads / 64];
  if (blockIdx.x == 0) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kThreads) acc += partials[i];
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) {
      const double n0 = r > 1e-28 * *r0n2p ? r : 0.0;
      S[slot] = n0;
      S[slot + 1] = sqrt(n0);
      hat[0] = sqrt(n0);
    }
  }
  for (int s = blockIdx.x * kThreads + threadIdx.x; s < m; s += gridDim.x * kThreads) {
    hat[1 + s] = gn * s0[s];
    hat[1 + m + s] = rn * s0[m + s];
  }
}

__global__ __launch_bounds__(kThreads) void k_copy(double *__restrict__ dst,
                                                   const double *__restrict__ src, size_t count) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

}  // namespace

int red_blocks(size_t n) {
  size_t b = (n + (size_t)kThreads * 4 - 1) / ((size_t)kThreads * 4);
  if (b < 1) b = 1;
  if (b > (size_t)kRedBlocks) b = kRedBlocks;
  return (int)b;
}

hipError_t launch_matvec(const wc_plan &p, const double *x, double *y, double *partials,
                         int *nblocks_out, const double *sub, bool negate) {
  MvArgs a{p.n, p.M, p.dims, p.m, p.opts.method == WC_GMRES_PS ? 0 : 1,
           p.theta, p.tau, p.alpha, p.inv_h2, p.d_aface, p.fem ? p.d_mu64 : nullptr,
           negate ? -1.0 : 1.0, p.neumann ? 1 : 0};
  dim3 grid((p.m + kThreads * kMvPts - 1) / (kThreads * kMvPts), 2);
  ProfScope ps(p, K_MATVEC, (sub ? 24.0 : 16.0) * p.nvec);
  const bool dg = a.diag != nullptr;
  if (dg && sub)
    hipLaunchKernelGGL((k_matvec<true, true>), grid, dim3(kThreads), 0, p.stream, x, y, sub, a, partials);
  else if (dg)
    hipLaunchKernelGGL((k_matvec<true, false>), grid, dim3(kThreads), 0, p.stream, x, y, sub, a, partials);
  else if (sub)
    hipLaunchKernelGGL((k_matvec<false, true>), grid, dim3(kThreads), 0, p.stream, x, y, sub, a, partials);
  else
    hipLaunchKernelGGL((k_matvec<false, false>), grid, dim3(kThreads), 0, p.stream, x, y, sub, a, partials);
  if (nblocks_out) *nblocks_out = 2 * grid.x;
  return hipGetLastError();
}

hipError_t launch_rhs(const wc_plan &p, const double *f, const double *g, const double *y0,
                      double *b) {
  RhsArgs a{p.n, p.M, p.dims, p.m, p.opts.method == WC_GMRES_PS ? 0 : 1,
            p.theta, p.tau, sqrt(p.gamma), p.inv_h2, p.d_aface, p.fem ? 0 : 1, p.neumann ? 1 : 0};
  const size_t nm = (size_t)p.n * p.m;
  dim3 grid((unsigned)((nm + kThreads - 1) / kThreads));
  {
    ProfScope ps(p, K_RHS, 8.0 * (2.0 * (p.n + 1) * p.m + p.m + p.nvec));
    hipLaunchKernelGGL(k_rhs, grid, dim3(kThreads), 0, p.stream, f, g, y0, b, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !p.fem) return e;
  }
  return launch_fem_rhs_finish(p, y0, b);
}

hipError_t launch_recover(const wc_plan &p, const double *x, double *y, double *pp, double *u) {
  dim3 grid((p.m + kThreads - 1) / kThreads, 2);
  ProfScope ps(p, K_RECOVER, 8.0 * (p.nvec + p.nvec + (u ? p.nvec / 2 : 0)));
  hipLaunchKernelGGL(k_recover, grid, dim3(kThreads), 0, p.stream, x, y, pp,
                     p.fem ? nullptr : u, p.n, p.m, p.theta, 1.0 / sqrt(p.gamma), 1.0 / p.gamma);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess || !p.fem) return e;
  return launch_fem_recover_finish(p, y, pp, u);
}

hipError_t launch_lincomb3(const wc_plan &p, double *dst, const double *a, const double *b,
                           const double *c, int slot, double h0, double h1, double h2) {
  ProfScope ps(p, K_LINCOMB, 8.0 * p.nvec * (2 + (b ? 1 : 0) + (c ? 1 : 0)));
  const dim3 grid(red_blocks(p.nvec)), block(kThreads);
  if (b && c)
    hipLaunchKernelGGL((k_lincomb3<true, true>), grid, block, 0, p.stream, dst, a, b, c, p.nvec,
                       p.d_scal, slot, h0, h1, h2);
  else if (b)
    hipLaunchKernelGGL((k_lincomb3<true, false>), grid, block, 0, p.stream, dst, a, b, c,
                       p.nvec, p.d_scal, slot, h0, h1, h2);
  else if (c)
    hipLaunchKernelGGL((k_lincomb3<false, true>), grid, block, 0, p.stream, dst, a, b, c,
                       p.nvec, p.d_scal, slot, h0, h1, h2);
  else
    hipLaunchKernelGGL((k_lincomb3<false, false>), grid, block, 0, p.stream, dst, a, b, c,
                       p.nvec, p.d_scal, slot, h0, h1, h2);
  return hipGetLastError();
}

hipError_t launch_finalize(const wc_plan &p, const double *partials, int count, int nsum,
                           int slot) {
  ProfScope ps(p, K_FINALIZE, 8.0 * count * nsum);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, p.stream, partials, count, nsum,
                     p.d_scal, slot);
  return hipGetLastError();
}

hipError_t launch_dot_partials(const wc_plan &p, const double *a, const double *b,
                               int *nparts) {
  const int nb = red_blocks(p.nvec);
  ProfScope ps(p, K_DOT, 16.0 * p.nvec);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kThreads), 0, p.stream, a, b, p.nvec, p.d_partials);
  if (nparts) *nparts = nb;
  return hipGetLastError();
}

hipError_t launch_dot(const wc_plan &p, const double *a, const double *b, int slot,
                      size_t len) {
  const size_t nv = len ? len : p.nvec;
  const int nb = red_blocks(nv);
  hipError_t e;
  {
    ProfScope ps(p, K_DOT, 8.0 * nv * (a == b ? 1 : 2));
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kThreads), 0, p.stream, a, b, nv, p.d_partials);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  return launch_finalize(p, p.d_partials, nb, 1, slot);
}

hipError_t launch_minres_update(const wc_plan &p, double *w0, const double *w1,
                                const double *z, double *x, double *r, const double *vnew) {
  const int nb = red_blocks(p.nvec);
  ProfScope ps(p, K_MINRES_UPDATE, 9.0 * 8.0 * p.nvec);
  hipLaunchKernelGGL(k_minres_update, dim3(nb), dim3(kThreads), 0, p.stream, w0, w1, z, x, r,
                     vnew, p.nvec, p.d_scal, p.d_partials);
  return hipGetLastError();
}

hipError_t launch_minres_scalar(const wc_plan &p, int stage, int nparts, double tol) {
  ProfScope ps(p, K_MINRES_SCALAR, 8.0 * nparts);
  hipLaunchKernelGGL(k_minres_scalar, dim3(1), dim3(kThreads), 0, p.stream, p.d_partials,
                     nparts, p.d_scal, stage, tol);
  return hipGetLastError();
}

#define WC_NB_CASES(X)                                                                         \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)      \
  X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31)  \
  X(32)

namespace {
hipError_t multidot_fin(const wc_plan &p, const double *basis, int nb, const double *w,
                        bool self, const double *gate, int *nblocks, size_t len, int stage,
                        int jj) {
  const size_t nv = len ? len : p.nvec;
  const int g = red_blocks(nv);
  if (nblocks) *nblocks = g;
  ProfScope ps(p, gate ? K_MULTIDOT_RE : K_MULTIDOT, 8.0 * nv * (nb + 1));
  switch (nb) {
#define CASE_NB(K)                                                                           \
  case K:                                                                                    \
    if (self)                                                                                \
      hipLaunchKernelGGL((k_multidot<K, true>), dim3(g), dim3(kThreads), 0, p.stream, basis, \
                         w, nv, p.d_partials, gate, p.d_scal, stage, jj);                    \
    else                                                                                     \
      hipLaunchKernelGGL((k_multidot<K, false>), dim3(g), dim3(kThreads), 0, p.stream,       \
                         basis, w, nv, p.d_partials, gate, p.d_scal, stage, jj);             \
    break;
    WC_NB_CASES(CASE_NB)
#undef CASE_NB
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t multiaxpy_fin(const wc_plan &p, double *w, const double *basis, int nb, int slot,
                         double sign, bool norm, const double *gate, int *nblocks, size_t len,
                         int stage, int jj) {
  const size_t nv = len ? len : p.nvec;
  const int g = red_blocks(nv);
  if (nblocks) *nblocks = g;
  double *parts = norm ? p.d_partials : nullptr;
  ProfScope ps(p, gate ? K_MULTIAXPY_RE : K_MULTIAXPY, 8.0 * nv * (nb + 2));
  switch (nb) {
#define CASE_NB(K)                                                                            \
  case K:                                                                                     \
    hipLaunchKernelGGL(k_multiaxpy<K>, dim3(g), dim3(kThreads), 0, p.stream, w, basis, nv,      \
                       p.d_scal, slot, sign, parts, gate, p.d_scal, stage, jj);               \
    break;
    WC_NB_CASES(CASE_NB)
#undef CASE_NB
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_multidot(const wc_plan &p, const double *basis, int nb, const double *w,
                           bool self, const double *gate, int *nblocks, size_t len) {
  return multidot_fin(p, basis, nb, w, self, gate, nblocks, len, 0, 0);
}

hipError_t launch_multiaxpy(const wc_plan &p, double *w, const double *basis, int nb, int slot,
                            double sign, bool norm, const double *gate, int *nblocks,
                            size_t len) {
  return multiaxpy_fin(p, w, basis, nb, slot, sign, norm, gate, nblocks, len, 0, 0);
}

hipError_t launch_gram_schmidt(const wc_plan &p, const double *V, int j, double *Vn,
                               size_t len, int passes) {
  hipError_t e;
  if ((e = multidot_fin(p, V, j + 1, Vn, true, nullptr, nullptr, len, 1, j)) != hipSuccess)
    return e;
  if ((e = multiaxpy_fin(p, Vn, V, j + 1, S_GSC, -1.0, true, nullptr, nullptr, len, 2, j)) !=
      hipSuccess)
    return e;
  return passes > 1 ? launch_gs_second_pass(p, V, j, Vn, len) : hipSuccess;
}

hipError_t launch_gs_second_pass(const wc_plan &p, const double *V, int j, double *Vn,
                                 size_t len) {
  const double *gate = p.d_scal + S_REORTH;
  hipError_t e;
  if ((e = multidot_fin(p, V, j + 1, Vn, false, gate, nullptr, len, 3, j)) != hipSuccess)
    return e;
  return multiaxpy_fin(p, Vn, V, j + 1, S_GSC, -1.0, true, gate, nullptr, len, 4, j);
}

hipError_t launch_gs_finalize(const wc_plan &p, int stage, int j, int count) {
  ProfScope ps(p, K_FINALIZE, 8.0 * count * (j + 2));
  hipLaunchKernelGGL(k_gs_finalize, dim3(1), dim3(kThreads), 0, p.stream, p.d_partials, count,
                     p.d_scal, stage, j);
  return hipGetLastError();
}

hipError_t launch_copy(const wc_plan &p, double *dst, const double *src, size_t count) {
  size_t b = (count + kThreads * 4 - 1) / (kThreads * 4);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  ProfScope ps(p, K_FILL, 16.0 * count);
  hipLaunchKernelGGL(k_copy, dim3((unsigned)b), dim3(kThreads), 0, p.stream, dst, src, count);
  return hipGetLastError();
}

hipError_t launch_lr_setup(const wc_plan &p, const double *r0, double *hat) {
  hipError_t e;
  {
    ProfScope ps(p, K_LR_SETUP, 8.0 * p.nvec + 16.0 * p.m);
    hipLaunchKernelGGL(k_lr_project, dim3((p.m + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       p.stream, r0, p.d_lr_gr, p.d_lr_s0, p.n, p.m,
                       1.0 / (p.lr_gn * p.lr_gn), 1.0 / (p.lr_rn * p.lr_rn));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int nb = red_blocks(p.nvec / 2);
  {
    ProfScope ps(p, K_LR_SETUP, 8.0 * p.nvec + 16.0 * p.m);
    hipLaunchKernelGGL(k_lr_perp, dim3(nb), dim3(kThreads), 0, p.stream, r0, p.d_lr_gr,
                       p.d_lr_s0, p.n, p.m, p.d_partials);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // 2D: s0, and with it every compact vector, in orthonormal sine coordinates
  if (p.lr_2d && (e = launch_lr_sine_s0(p)) != hipSuccess) return e;
  ProfScope ps(p, K_LR_SETUP, 8.0 * p.lr_len);
  hipLaunchKernelGGL(k_lr_hat0, dim3((p.m + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     p.stream, p.d_partials, nb, p.d_scal, (int)S_LR_N0, p.d_scal + S_DOT,
                     p.d_lr_s0, p.m, p.lr_gn, p.lr_rn, hat);
  return hipGetLastError();
}

hipError_t launch_fill(const wc_plan &p, double *dst, double val, size_t count) {
  size_t b = (count + kThreads * 4 - 1) / (kThreads * 4);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  ProfScope ps(p, K_FILL, 8.0 * count);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)b), dim3(kThreads), 0, p.stream, dst, val, count);
  return hipGetLastError();
}

}  // namespace wc
