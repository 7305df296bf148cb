// Preconditioner apply for a == 1: three-step procedure of Section 3.4.
//
//  step 1  omega-scaled time transform  v_hat_l = sum_k e^{i zeta k/n} e^{-2 pi i k l/n} v_k
//          (the printed eigendecomposition of S_n^(j) does not reproduce S_n^(1); the
//          transform used here is Phi = F diag(omega^{k/n}) with eigenvalues
//          lambda_l = f_1(psi_l)/f_2(psi_l), psi_l = (zeta - 2 pi l)/n, read off
//          Phi S Phi^{-1}), then the orthonormal sine transform in each space direction;
//  step 2  per (frequency, sine mode) scaling (|P_S|, P_MS) or 2x2 solve coupling the two
//          block rows (P_S), with Lambda = lambda_l + tau (mu_j1 + mu_j2);
//  step 3  inverse sine transforms and inverse time transform.
//
// zeta = pi keeps everything real: for a real sequence v_hat_{(1-l) mod n} = conj(v_hat_l),
// so only the n/2 frequencies l = 1..n/2 are stored.  The two block rows are transformed
// together as one complex sequence z = v1 + i v2 and separated afterwards with that
// symmetry.  The sine transform (DST-I of length N1-1, N1 = M+1) runs as one N1-point
// complex FFT with O(N1) pre/post-processing (even outputs directly, odd outputs as a
// running sum).  All normalisations (1/n and (2/N1)^dims) are folded into step 2.
//
// Passes over HBM (2D): time FFT, x1-DST (written x2-contiguous), fused [x2-DST, step 2,
// x2-iDST], x1-iDST (written back x1-contiguous), inverse time FFT.  1D: three passes.
// Every FFT is a Stockham radix-8/4/2 transform staged in LDS.

#include "wc_internal.h"

namespace wc {
namespace {

template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
template <typename T> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }

// ---- small DFTs in registers, natural order in and out ---------------------
template <typename T, bool INV> __device__ __forceinline__ void dft2(cx<T> *v) {
  cx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(cx<T> *v) {
  cx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  cx<T> s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
  cx<T> t = INV ? mul_i(d13) : mul_mi(d13);
  v[0] = cadd(s02, s13);
  v[2] = csub(s02, s13);
  v[1] = cadd(d02, t);
  v[3] = csub(d02, t);
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(cx<T> *v) {
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const T r = (T)0.70710678118654752440;
  o[1] = cmul(o[1], cx<T>{r, INV ? r : -r});
  o[2] = INV ? mul_i(o[2]) : mul_mi(o[2]);
  o[3] = cmul(o[3], cx<T>{-r, INV ? r : -r});
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dftR(cx<T> *v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else dft8<T, INV>(v);
}

// One Stockham stage on B batched sequences of length N stored as buf[k*B + b].
// tw[p] = e^{-2 pi i p/N}.  All reads of the stage complete before any write.
template <typename T, int N, int R, int NS, int B, bool INV>
__device__ __forceinline__ void fft_stage(cx<T> *buf, const cx<T> *__restrict__ tw, int tid) {
  constexpr int NB = N / R;
  constexpr int TOTAL = NB * B;
  constexpr int IT = (TOTAL + kThreads - 1) / kThreads;
  cx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = tid + it * kThreads;
    if (TOTAL % kThreads == 0 || idx < TOTAL) {
      const int b = idx % B, j = idx / B;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[(j + r * NB) * B + b];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[k * r * (N / (NS * R))];
          if (INV) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
      }
      dftR<T, R, INV>(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = tid + it * kThreads;
    if (TOTAL % kThreads == 0 || idx < TOTAL) {
      const int b = idx % B, j = idx / B;
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(base + r * NS) * B + b] = v[it][r];
    }
  }
  __syncthreads();
}

// Complete length-N FFT (forward e^{-2 pi i}, inverse unnormalised e^{+2 pi i}).
template <typename T, int N, int NS, int B, bool INV>
__device__ __forceinline__ void fft_lds(cx<T> *buf, const cx<T> *__restrict__ tw, int tid) {
  if constexpr (NS < N) {
    constexpr int REM = N / NS;
    constexpr int R = REM >= 8 ? 8 : REM;
    fft_stage<T, N, R, NS, B, INV>(buf, tw, tid);
    fft_lds<T, N, NS * R, B, INV>(buf, tw, tid);
  }
}

// Unnormalised DST-I, Y_j = sum_{i=1}^{N1-1} x_i sin(pi i j/N1), of B complex lines held
// in buf[i*B + b] (i = 1..N1-1; slot 0 is scratch).  Result in the same slots.
//   y_i = sin(pi i/N1)(x_i + x_{N1-i}) + (x_i - x_{N1-i})/2,  F = FFT_N1(y)
//   C_k = (F_k + F_{N1-k})/2,  S_k = i (F_k - F_{N1-k})/2
//   Y_{2k} = S_k,  Y_{2k+1} = C_0/2 + C_1 + ... + C_k
template <typename T, int N1, int B>
__device__ __forceinline__ void dst_lds(cx<T> *buf, const cx<T> *__restrict__ tw,
                                        const T *__restrict__ sintab, int tid) {
  constexpr int H = N1 / 2;
  constexpr int ITEMS = H * B;
  constexpr int IT = (ITEMS + kThreads - 1) / kThreads;
  for (int idx = tid; idx < ITEMS; idx += kThreads) {
    const int b = idx % B, i = idx / B + 1;
    const cx<T> xa = buf[i * B + b];
    const cx<T> xb = buf[(N1 - i) * B + b];
    const T s = sintab[i];
    const cx<T> sum = cadd(xa, xb);
    const cx<T> dif = cscale(csub(xa, xb), (T)0.5);
    buf[i * B + b] = cadd(cscale(sum, s), dif);
    if (i != H) buf[(N1 - i) * B + b] = csub(cscale(sum, s), dif);
    if (i == 1) buf[b] = cx<T>{(T)0, (T)0};
  }
  __syncthreads();
  fft_lds<T, N1, 1, B, false>(buf, tw, tid);
  cx<T> cc[IT], ss[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = tid + it * kThreads;
    if (ITEMS % kThreads == 0 || idx < ITEMS) {
      const int b = idx % B, k = idx / B;
      const cx<T> Fk = buf[k * B + b];
      const cx<T> Fm = buf[((N1 - k) & (N1 - 1)) * B + b];
      cx<T> C = cscale(cadd(Fk, Fm), (T)0.5);
      if (k == 0) C = cscale(C, (T)0.5);
      cc[it] = C;
      ss[it] = mul_i(cscale(csub(Fk, Fm), (T)0.5));
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = tid + it * kThreads;
    if (ITEMS % kThreads == 0 || idx < ITEMS) {
      const int b = idx % B, k = idx / B;
      buf[(2 * k + 1) * B + b] = cc[it];
      if (k > 0) buf[(2 * k) * B + b] = ss[it];
    }
  }
  __syncthreads();
  // inclusive running sum over the odd slots 2k+1, k = 0..H-1 (Hillis-Steele)
#pragma unroll 1
  for (int off = 1; off < H; off <<= 1) {
    cx<T> val[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + it * kThreads;
      if (ITEMS % kThreads == 0 || idx < ITEMS) {
        const int b = idx % B, k = idx / B;
        cx<T> v = buf[(2 * k + 1) * B + b];
        if (k >= off) v = cadd(v, buf[(2 * (k - off) + 1) * B + b]);
        val[it] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + it * kThreads;
      if (ITEMS % kThreads == 0 || idx < ITEMS) {
        const int b = idx % B, k = idx / B;
        buf[(2 * k + 1) * B + b] = val[it];
      }
    }
    __syncthreads();
  }
}

constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
template <typename P, int N> struct TileCfg {
  static constexpr int kLds = 65536;
  static constexpr int TS = clampi(kLds / (N * 2 * (int)sizeof(P)), 1, 16);    // time FFT columns
  static constexpr int L = clampi(kLds / (N * 2 * (int)sizeof(P)), 1, 16);     // DST lines
  static constexpr int U = clampi(kLds / (N * 4 * (int)sizeof(P)), 1, 8);      // paired line units
};

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
  return r;
}

// ---- step 1a: time transform of both block rows ------------------------------
// v: 2 x (n, m) FP64.  W: [q][half][s] complex, q = 0..n/2-1 <-> frequency l = q+1.
template <typename P, int N, int TS>
__global__ __launch_bounds__(kThreads) void k_tfft_fwd(const double *__restrict__ v,
                                                       cx<P> *__restrict__ W,
                                                       const cx<double> *__restrict__ dtw,
                                                       const cx<P> *__restrict__ tw, int m) {
  __shared__ cx<P> buf[N * TS];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * TS;
  const double *v1 = v;
  const double *v2 = v + (size_t)N * m;
  for (int idx = tid; idx < N * TS; idx += kThreads) {
    const int k = idx / TS, s = idx % TS, gs = s0 + s;
    double a = 0.0, b = 0.0;
    if (gs < m) {
      a = v1[(size_t)k * m + gs];
      b = v2[(size_t)k * m + gs];
    }
    const cx<double> d = dtw[k];
    buf[idx] = cx<P>{(P)(a * d.x - b * d.y), (P)(a * d.y + b * d.x)};
  }
  __syncthreads();
  fft_lds<P, N, 1, TS, false>(buf, tw, tid);
  for (int idx = tid; idx < (N / 2) * TS; idx += kThreads) {
    const int q = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs >= m) continue;
    const cx<P> Zl = buf[(q + 1) * TS + s];
    const cx<P> Zp = buf[((N - q) & (N - 1)) * TS + s];  // frequency (1-l) mod n
    const cx<P> A = {(Zl.x + Zp.x) * (P)0.5, (Zl.y - Zp.y) * (P)0.5};
    const cx<P> D = {(Zl.x - Zp.x) * (P)0.5, (Zl.y + Zp.y) * (P)0.5};
    W[((size_t)q * 2 + 0) * m + gs] = A;
    W[((size_t)q * 2 + 1) * m + gs] = mul_mi(D);
  }
}

// ---- step 3b: inverse time transform, real output, optional fused <w, dotv> ----
template <typename P, int N, int TS>
__global__ __launch_bounds__(kThreads) void k_tfft_inv(const cx<P> *__restrict__ W,
                                                       double *__restrict__ out,
                                                       const cx<double> *__restrict__ dtw,
                                                       const cx<P> *__restrict__ tw, int m,
                                                       const double *__restrict__ dotv,
                                                       double *__restrict__ partials) {
  __shared__ cx<P> buf[N * TS];
  __shared__ double red[kThreads / 64];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * TS;
  for (int idx = tid; idx < (N / 2) * TS; idx += kThreads) {
    const int q = idx / TS, s = idx % TS, gs = s0 + s;
    cx<P> A = {(P)0, (P)0}, Bv = {(P)0, (P)0};
    if (gs < m) {
      A = W[((size_t)q * 2 + 0) * m + gs];
      Bv = W[((size_t)q * 2 + 1) * m + gs];
    }
    buf[(q + 1) * TS + s] = cx<P>{A.x - Bv.y, A.y + Bv.x};                  // A + iB
    buf[((N - q) & (N - 1)) * TS + s] = cx<P>{A.x + Bv.y, Bv.x - A.y};      // conj(A) + i conj(B)
  }
  __syncthreads();
  fft_lds<P, N, 1, TS, true>(buf, tw, tid);
  double acc = 0.0;
  double *o1 = out;
  double *o2 = out + (size_t)N * m;
  for (int idx = tid; idx < N * TS; idx += kThreads) {
    const int k = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs >= m) continue;
    const cx<P> z = buf[idx];
    const cx<double> d = dtw[k];  // multiply by conj(d)
    const double zx = (double)z.x, zy = (double)z.y;
    const double r1 = zx * d.x + zy * d.y;
    const double r2 = zy * d.x - zx * d.y;
    const size_t g = (size_t)k * m + gs;
    o1[g] = r1;
    o2[g] = r2;
    if (dotv) acc += r1 * dotv[g] + r2 * dotv[(size_t)N * m + g];
  }
  if (dotv) {
    const double r = block_sum(acc, red);
    if (tid == 0) partials[blockIdx.x] = r;
  }
}

// ---- x1 sine transform of (n) slabs of M x M, with a transposing store/load -----
// ROWS_IN: src rows [x2][x1] -> dst [j1][x2];  otherwise src [j1][x2] -> dst rows [x2][x1].
template <typename P, int N1, int L, bool ROWS_IN>
__global__ __launch_bounds__(kThreads) void k_dst_x1(const cx<P> *__restrict__ src,
                                                     cx<P> *__restrict__ dst,
                                                     const cx<P> *__restrict__ tw,
                                                     const P *__restrict__ sintab) {
  constexpr int M = N1 - 1;
  __shared__ cx<P> buf[N1 * L];
  const int tid = threadIdx.x;
  const size_t slab = blockIdx.y;
  const int r0 = blockIdx.x * L;
  const cx<P> *S = src + slab * (size_t)M * M;
  cx<P> *D = dst + slab * (size_t)M * M;
  if (ROWS_IN) {
    for (int idx = tid; idx < L * M; idx += kThreads) {
      const int x1 = idx % M, r = idx / M;
      cx<P> val = {(P)0, (P)0};
      if (r0 + r < M) val = S[(size_t)(r0 + r) * M + x1];
      buf[(x1 + 1) * L + r] = val;
    }
  } else {
    for (int idx = tid; idx < L * M; idx += kThreads) {
      const int r = idx % L, j1 = idx / L;
      cx<P> val = {(P)0, (P)0};
      if (r0 + r < M) val = S[(size_t)j1 * M + r0 + r];
      buf[(j1 + 1) * L + r] = val;
    }
  }
  __syncthreads();
  dst_lds<P, N1, L>(buf, tw, sintab, tid);
  if (ROWS_IN) {
    for (int idx = tid; idx < L * M; idx += kThreads) {
      const int r = idx % L, j1 = idx / L;
      if (r0 + r < M) D[(size_t)j1 * M + r0 + r] = buf[(j1 + 1) * L + r];
    }
  } else {
    for (int idx = tid; idx < L * M; idx += kThreads) {
      const int x1 = idx % M, r = idx / M;
      if (r0 + r < M) D[(size_t)(r0 + r) * M + x1] = buf[(x1 + 1) * L + r];
    }
  }
}

// ---- last space direction: DST, step 2, inverse DST, on both block rows --------
// Lines are contiguous.  A "unit" is (q) in 1D or (q, j1) in 2D and owns the two half
// lines at ((q*2 + h) * M [+ j1]) * M.  kind: 0 P_S (2x2), 1 |P_S|, 2 P_MS.
template <typename P, int N1, int U, int DIMS>
__global__ __launch_bounds__(kThreads) void k_pair_mode(cx<P> *__restrict__ Wd,
                                                        const cx<P> *__restrict__ tw,
                                                        const P *__restrict__ sintab,
                                                        const cx<P> *__restrict__ lam,
                                                        const P *__restrict__ mu, int nunits,
                                                        int kind, P tau, P alpha, P cnorm) {
  constexpr int M = N1 - 1;
  constexpr int B = 2 * U;
  __shared__ cx<P> buf[N1 * B];
  const int tid = threadIdx.x;
  const int unit0 = blockIdx.x * U;
  auto line_off = [&](int unit, int h) -> size_t {
    if (DIMS == 1) return ((size_t)unit * 2 + h) * M;
    const int q = unit / M, j1 = unit % M;
    return (((size_t)q * 2 + h) * M + j1) * M;
  };
  for (int idx = tid; idx < B * M; idx += kThreads) {
    const int x = idx % M, bh = idx / M;
    const int unit = unit0 + (bh >> 1);
    cx<P> val = {(P)0, (P)0};
    if (unit < nunits) val = Wd[line_off(unit, bh & 1) + x];
    buf[(x + 1) * B + bh] = val;
  }
  __syncthreads();
  dst_lds<P, N1, B>(buf, tw, sintab, tid);
  for (int idx = tid; idx < U * M; idx += kThreads) {
    const int u = idx % U, j = idx / U;
    const int unit = unit0 + u;
    if (unit >= nunits) continue;
    int q;
    P musum;
    if (DIMS == 1) {
      q = unit;
      musum = mu[j];
    } else {
      q = unit / M;
      musum = mu[unit % M] + mu[j];
    }
    const cx<P> l = lam[q];
    const cx<P> a = buf[(j + 1) * B + 2 * u];
    const cx<P> b = buf[(j + 1) * B + 2 * u + 1];
    cx<P> na, nb;
    if (kind == 0) {
      const cx<P> Lm = {l.x + tau * musum, l.y};
      const P det = Lm.x * Lm.x + Lm.y * Lm.y + alpha * alpha;
      const P c = cnorm / det;
      // [a; b] <- c [[conj(Lm), alpha], [-alpha, Lm]] [a; b]
      const cx<P> ca = {Lm.x * a.x + Lm.y * a.y, Lm.x * a.y - Lm.y * a.x};
      const cx<P> lb = cmul(Lm, b);
      na = cscale(cx<P>{ca.x + alpha * b.x, ca.y + alpha * b.y}, c);
      nb = cscale(cx<P>{lb.x - alpha * a.x, lb.y - alpha * a.y}, c);
    } else {
      P s;
      if (kind == 1) {
        const P re = l.x + tau * musum;
        s = cnorm / sqrt(re * re + l.y * l.y + alpha * alpha);
      } else {
        s = cnorm / (sqrt(l.x * l.x + l.y * l.y + alpha * alpha) + tau * musum);
      }
      na = cscale(a, s);
      nb = cscale(b, s);
    }
    buf[(j + 1) * B + 2 * u] = na;
    buf[(j + 1) * B + 2 * u + 1] = nb;
  }
  __syncthreads();
  dst_lds<P, N1, B>(buf, tw, sintab, tid);
  for (int idx = tid; idx < B * M; idx += kThreads) {
    const int x = idx % M, bh = idx / M;
    const int unit = unit0 + (bh >> 1);
    if (unit < nunits) Wd[line_off(unit, bh & 1) + x] = buf[(x + 1) * B + bh];
  }
}

// ---- host dispatch -------------------------------------------------------------
struct PcArgs {
  const wc_plan *p;
  const double *v;
  double *w;
  double *partials;
};

template <typename P> struct Tabs;
template <> struct Tabs<double> {
  static const cx<double> *twt(const wc_plan &p) { return (const cx<double> *)p.d_twt64; }
  static const cx<double> *tws(const wc_plan &p) { return (const cx<double> *)p.d_tws64; }
  static const double *sin(const wc_plan &p) { return p.d_sin64; }
  static const cx<double> *lam(const wc_plan &p) { return (const cx<double> *)p.d_lam64; }
  static const double *mu(const wc_plan &p) { return p.d_mu64; }
};
template <> struct Tabs<float> {
  static const cx<float> *twt(const wc_plan &p) { return (const cx<float> *)p.d_twt32; }
  static const cx<float> *tws(const wc_plan &p) { return (const cx<float> *)p.d_tws32; }
  static const float *sin(const wc_plan &p) { return p.d_sin32; }
  static const cx<float> *lam(const wc_plan &p) { return (const cx<float> *)p.d_lam32; }
  static const float *mu(const wc_plan &p) { return p.d_mu32; }
};

template <typename P, int N>
hipError_t run_tfft_fwd(const wc_plan &p, const double *v) {
  constexpr int TS = TileCfg<P, N>::TS;
  dim3 grid((p.m + TS - 1) / TS);
  ProfScope ps(p, K_TFFT_FWD, (double)p.nvec * (8.0 + sizeof(P)));
  hipLaunchKernelGGL((k_tfft_fwd<P, N, TS>), grid, dim3(kThreads), 0, p.stream, v,
                     (cx<P> *)p.d_specA, (const cx<double> *)p.d_dtw, Tabs<P>::twt(p), p.m);
  return hipGetLastError();
}

template <typename P, int N>
hipError_t run_tfft_inv(const wc_plan &p, double *w, const double *dotv, int *nparts) {
  constexpr int TS = TileCfg<P, N>::TS;
  dim3 grid((p.m + TS - 1) / TS);
  *nparts = grid.x;
  ProfScope ps(p, K_TFFT_INV, (double)p.nvec * (sizeof(P) + (dotv ? 16.0 : 8.0)));
  hipLaunchKernelGGL((k_tfft_inv<P, N, TS>), grid, dim3(kThreads), 0, p.stream,
                     (const cx<P> *)p.d_specA, w, (const cx<double> *)p.d_dtw, Tabs<P>::twt(p),
                     p.m, dotv, p.d_partials);
  return hipGetLastError();
}

template <typename P, int N1>
hipError_t run_space(const wc_plan &p) {
  constexpr int L = TileCfg<P, N1>::L;
  constexpr int U = TileCfg<P, N1>::U;
  constexpr int M = N1 - 1;
  const int kind = p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
  const double c = (1.0 / p.n) * (p.dims == 2 ? (2.0 / N1) * (2.0 / N1) : (2.0 / N1));
  if (p.dims == 1) {
    const int nunits = p.n / 2;
    dim3 grid((nunits + U - 1) / U);
    ProfScope ps(p, K_PAIR_MODE, 2.0 * p.nvec * sizeof(P));
    hipLaunchKernelGGL((k_pair_mode<P, N1, U, 1>), grid, dim3(kThreads), 0, p.stream,
                       (cx<P> *)p.d_specA, Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lam(p),
                       Tabs<P>::mu(p), nunits, kind, (P)p.tau, (P)p.alpha, (P)c);
    return hipGetLastError();
  }
  dim3 g1((M + L - 1) / L, p.n);
  hipError_t e;
  {
    ProfScope ps(p, K_DST_X1_FWD, 2.0 * p.nvec * sizeof(P));
    hipLaunchKernelGGL((k_dst_x1<P, N1, L, true>), g1, dim3(kThreads), 0, p.stream,
                       (const cx<P> *)p.d_specA, (cx<P> *)p.d_specB, Tabs<P>::tws(p),
                       Tabs<P>::sin(p));
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  const int nunits = (p.n / 2) * M;
  dim3 g2((nunits + U - 1) / U);
  {
    ProfScope ps(p, K_PAIR_MODE, 2.0 * p.nvec * sizeof(P));
    hipLaunchKernelGGL((k_pair_mode<P, N1, U, 2>), g2, dim3(kThreads), 0, p.stream,
                       (cx<P> *)p.d_specB, Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lam(p),
                       Tabs<P>::mu(p), nunits, kind, (P)p.tau, (P)p.alpha, (P)c);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  ProfScope ps(p, K_DST_X1_INV, 2.0 * p.nvec * sizeof(P));
  hipLaunchKernelGGL((k_dst_x1<P, N1, L, false>), g1, dim3(kThreads), 0, p.stream,
                     (const cx<P> *)p.d_specB, (cx<P> *)p.d_specA, Tabs<P>::tws(p),
                     Tabs<P>::sin(p));
  return hipGetLastError();
}

#define WC_POW2_CASES(X) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

template <typename P>
hipError_t pc_apply_t(const wc_plan &p, const double *v, double *w, const double *dotv,
                      int *nparts) {
  hipError_t e = hipErrorInvalidValue;
  switch (p.n) {
#define CASE_N(NN) case NN: e = run_tfft_fwd<P, NN>(p, v); break;
    WC_POW2_CASES(CASE_N)
#undef CASE_N
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (p.N1) {
#define CASE_S(NN) case NN: e = run_space<P, NN>(p); break;
    WC_POW2_CASES(CASE_S)
#undef CASE_S
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (p.n) {
#define CASE_N(NN) case NN: e = run_tfft_inv<P, NN>(p, w, dotv, nparts); break;
    WC_POW2_CASES(CASE_N)
#undef CASE_N
    default: return hipErrorInvalidValue;
  }
  return e;
}

}  // namespace

bool pc_supported(int n, int N1) {
  auto pow2 = [](int x) { return x >= 4 && x <= 1024 && (x & (x - 1)) == 0; };
  return pow2(n) && pow2(N1);
}

hipError_t launch_pc_apply(const wc_plan &p, const double *v, double *w, bool dot,
                           int *nparts) {
  int np = 0;
  const double *dotv = dot ? v : nullptr;
  hipError_t e = p.opts.precision == WC_MIXED ? pc_apply_t<float>(p, v, w, dotv, &np)
                                              : pc_apply_t<double>(p, v, w, dotv, &np);
  if (nparts) *nparts = np;
  return e;
}

int pc_partials_needed(int n, int m, int precision) {
  int ts = 1;
  const int es = precision == WC_MIXED ? 8 : 16;
  ts = 65536 / (n * es);
  if (ts < 1) ts = 1;
  if (ts > 16) ts = 16;
  return (m + ts - 1) / ts;
}

}  // namespace wc
