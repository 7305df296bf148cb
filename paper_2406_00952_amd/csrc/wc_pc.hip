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
// Passes over HBM (2D): [time FFT], [x1-DST, rows in place], [x2-DST, step 2, x2-iDST on
// column tiles in place], [x1-iDST, rows in place], [inverse time FFT].  1D: [time FFT],
// [DST, step 2, iDST on rows], [inverse time FFT].
//
// Every FFT is a Stockham radix-8/4/2 transform executed by ONE wavefront on lines it owns
// in LDS; waves synchronise only themselves, so the four waves of a workgroup never wait
// on each other between stages.  The DST running sum is a segmented wave-shuffle scan.

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

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

// one complex value loaded past the caches (non-temporal)
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cx<double> load_stream(const cx<double> *p) {
  const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
  return {v.x, v.y};
}
__device__ __forceinline__ cx<float> load_stream(const cx<float> *p) {
  const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
  return {v.x, v.y};
}

// Orders the LDS accesses of one wavefront (LDS operations of a wave complete in order;
// this stops the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS position of FFT index k: one pad slot every 2^PS elements breaks the power-of-two
// strides of the Stockham writes so the lanes of a wave hit distinct banks.
template <int PS> __device__ __forceinline__ int pk(int k) { return k + (k >> PS); }
template <int PS> constexpr int padded(int n) { return n + (n >> PS) + 1; }

template <typename T> __device__ __forceinline__ cx<T> shfl_up_cx(cx<T> v, int d) {
  return cx<T>{__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64)};
}
template <typename T> __device__ __forceinline__ cx<T> shfl_cx(cx<T> v, int src) {
  return cx<T>{__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) round robin by linear id.
// Tiles adjacent in memory share cache lines, so give each XCD a contiguous run of
// tiles: tile = first tile of XCD (b mod 8) + b div 8.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int X = 8;
  const int q = nb / X, r = nb % X, x = b % X;
  return x * q + (x < r ? x : r) + b / X;
}

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

// 16 points as 4 x 4: index n = 4 n1 + n2, output k = k1 + 4 k2:
//   A[n2][k1] = DFT4 over n1 of v[4 n1 + n2];  A[n2][k1] *= w16^(n2 k1);
//   X[k1 + 4 k2] = DFT4 over n2 of A[n2][k1].
template <typename T, bool INV> __device__ __forceinline__ void dft16(cx<T> *v) {
  cx<T> a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
    dft4<T, INV>(a[n2]);
  }
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;  // cos, sin pi/8
  const T h = (T)0.70710678118654752440;
  const T sg = INV ? (T)1 : (T)-1;  // w16 = e^{sg i 2 pi / 16}
  // w16^1, w16^2, w16^3 and w16^4, w16^6, w16^9
  const cx<T> w1{c1, sg * s1}, w2{h, sg * h}, w3{s1, sg * c1};
  a[1][1] = cmul(a[1][1], w1);
  a[1][2] = cmul(a[1][2], w2);
  a[1][3] = cmul(a[1][3], w3);
  a[2][1] = cmul(a[2][1], w2);
  a[2][2] = INV ? mul_i(a[2][2]) : mul_mi(a[2][2]);                 // w16^4
  a[2][3] = cmul(a[2][3], cx<T>{-h, sg * h});                        // w16^6
  a[3][1] = cmul(a[3][1], w3);
  a[3][2] = cmul(a[3][2], cx<T>{-h, sg * h});                        // w16^6
  a[3][3] = cmul(a[3][3], cx<T>{-c1, -sg * s1});                     // w16^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4<T, INV>(b);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
  }
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dftR(cx<T> *v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else dft16<T, INV>(v);
}

// One Stockham stage executed by one wave on B lines of length N stored at
// buf[pk(k)*S + b].  tw[p] = e^{-2 pi i p/N} (LDS or global).  Butterfly index j runs
// fastest across lanes.  For radix 8 only w^1 and w^2 are looked up; w^3..w^7 are
// products of those.
template <typename T, int N, int R, int NS, int B, int S, int PS, bool INV>
__device__ __forceinline__ void wstage(cx<T> *buf, const cx<T> *__restrict__ tw, int lane) {
  constexpr int NB = N / R;
  constexpr int TOTAL = NB * B;
  constexpr int IT = (TOTAL + 63) / 64;
  cx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = lane + 64 * it;
    if (TOTAL % 64 == 0 || idx < TOTAL) {
      const int j = idx % NB, b = idx / NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[pk<PS>(j + r * NB) * S + b];
      if constexpr (NS > 1) {
        const int k = j % NS;
        constexpr int STEP = N / (NS * R);
        cx<T> w[R];
        w[1] = tw[k * STEP];
        if constexpr (R >= 4) w[2] = tw[2 * k * STEP];
        if constexpr (R >= 4) w[3] = cmul(w[1], w[2]);
        if constexpr (R == 8) {
          w[4] = cmul(w[2], w[2]);
          w[5] = cmul(w[1], w[4]);
          w[6] = cmul(w[2], w[4]);
          w[7] = cmul(w[3], w[4]);
        }
        if constexpr (R == 16) {  // w^4 and w^8 looked up, the rest as short products
          w[4] = tw[4 * k * STEP];
          w[8] = tw[8 * k * STEP];
          w[5] = cmul(w[1], w[4]);
          w[6] = cmul(w[2], w[4]);
          w[7] = cmul(w[3], w[4]);
#pragma unroll
          for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> ww = w[r];
          if (INV) ww.y = -ww.y;
          v[it][r] = cmul(v[it][r], ww);
        }
      }
      dftR<T, R, INV>(v[it]);
    }
  }
  wave_sync();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = lane + 64 * it;
    if (TOTAL % 64 == 0 || idx < TOTAL) {
      const int j = idx % NB, b = idx / NB;
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pk<PS>(base + r * NS) * S + b] = v[it][r];
    }
  }
  wave_sync();
}

// Radix 16 (R16) when the remaining length allows it and its butterflies still fill the
// wave (N/16 * B >= 64), else radix 8, 4, 2.
template <typename T, int N, int NS, int B, int S, int PS, bool INV, bool R16 = false>
__device__ __forceinline__ void wfft(cx<T> *buf, const cx<T> *__restrict__ tw, int lane) {
  if constexpr (NS < N) {
    constexpr int REM = N / NS;
    constexpr bool use16 = R16 && REM >= 16 && (N / 16) * B >= 64;
    constexpr int R = use16 ? 16 : (REM >= 8 ? 8 : REM);
    wstage<T, N, R, NS, B, S, PS, INV>(buf, tw, lane);
    wfft<T, N, NS * R, B, S, PS, INV, R16>(buf, tw, lane);
  }
}

// Unnormalised DST-I, Y_j = sum_{i=1}^{N1-1} x_i sin(pi i j/N1), of B complex lines held
// by one wave at buf[i*S + b] (i = 1..N1-1; slot 0 is scratch).  Result in the same slots.
//   y_i = sin(pi i/N1)(x_i + x_{N1-i}) + (x_i - x_{N1-i})/2,  F = FFT_N1(y)
//   C_k = (F_k + F_{N1-k})/2,  S_k = i (F_k - F_{N1-k})/2
//   Y_{2k} = S_k,  Y_{2k+1} = C_0/2 + C_1 + ... + C_k
template <typename T, int N1, int B, int S, int PS>
__device__ __forceinline__ void wdst_core(cx<T> *buf, const cx<T> *__restrict__ tw, int lane);

template <typename T, int N1, int B, int S, int PS>
__device__ __forceinline__ void wdst(cx<T> *buf, const cx<T> *__restrict__ tw,
                                     const T *__restrict__ sintab, int lane) {
  constexpr int H = N1 / 2;
  constexpr int ITEMS = H * B;
  for (int idx = lane; idx < ITEMS; idx += 64) {
    const int i = 1 + idx % H, b = idx / H;
    const cx<T> xa = buf[pk<PS>(i) * S + b];
    const cx<T> xb = buf[pk<PS>(N1 - i) * S + b];
    const T s = sintab[i];
    const cx<T> sum = cadd(xa, xb);
    const cx<T> dif = cscale(csub(xa, xb), (T)0.5);
    buf[pk<PS>(i) * S + b] = cadd(cscale(sum, s), dif);
    if (i != H) buf[pk<PS>(N1 - i) * S + b] = csub(cscale(sum, s), dif);
    if (i == 1) buf[b] = cx<T>{(T)0, (T)0};
  }
  wave_sync();
  wdst_core<T, N1, B, S, PS>(buf, tw, lane);
}

// FFT and post-processing of wdst, on the pre-processed sequence already in buf.
template <typename T, int N1, int B, int S, int PS>
__device__ __forceinline__ void wdst_core(cx<T> *buf, const cx<T> *__restrict__ tw, int lane) {
  constexpr int H = N1 / 2;
  constexpr int ITEMS = H * B;
  wfft<T, N1, 1, B, S, PS, false, true>(buf, tw, lane);
  // post-processing: every lane owns CH consecutive k of one line; the running sum is a
  // sequential scan inside the chunk plus a shuffle scan of the chunk totals.
  constexpr int CH = ITEMS >= 64 ? ITEMS / 64 : 1;
  constexpr int G = H / CH;  // lanes per line
  const int b = lane / G, g = lane % G, k0 = g * CH;
  const bool valid = b < B;
  cx<T> cc[CH], ss[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    cc[c] = cx<T>{(T)0, (T)0};
    ss[c] = cx<T>{(T)0, (T)0};
    if (valid) {
      const int k = k0 + c;
      const cx<T> Fk = buf[pk<PS>(k) * S + b];
      const cx<T> Fm = buf[pk<PS>((N1 - k) & (N1 - 1)) * S + b];
      cx<T> C = cscale(cadd(Fk, Fm), (T)0.5);
      if (k == 0) C = cscale(C, (T)0.5);
      cc[c] = C;
      ss[c] = mul_i(cscale(csub(Fk, Fm), (T)0.5));
    }
  }
#pragma unroll
  for (int c = 1; c < CH; ++c) cc[c] = cadd(cc[c], cc[c - 1]);
  const cx<T> tot = cc[CH - 1];
  cx<T> inc = tot;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const cx<T> y = shfl_up_cx(inc, off);
    if (g >= off) inc = cadd(inc, y);
  }
  const cx<T> excl = csub(inc, tot);
  wave_sync();
  if (valid) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = k0 + c;
      buf[pk<PS>(2 * k + 1) * S + b] = cadd(cc[c], excl);
      if (k > 0) buf[pk<PS>(2 * k) * S + b] = ss[c];
    }
  }
  wave_sync();
}

// The DST of B lines as above, for callers that write the pre-processed sequence
// (y_i, slot 0 = 0) themselves and take the outputs from registers: lane (b, g) gets
// k = k0 + c, c < CH, with odd[c] = Y_{2k+1} and even[c] = Y_{2k} (k >= 1); valid is false
// for lanes without a line.  buf may be rewritten once the wave has synchronised.
template <typename T, int N1, int B> struct DstLanes {
  static constexpr int H = N1 / 2, ITEMS = H * B;
  static constexpr int CH = ITEMS >= 64 ? ITEMS / 64 : 1;
  static constexpr int G = H / CH;  // lanes per line
};

template <typename T, int N1, int B, int S, int PS>
__device__ __forceinline__ void wdst_regs(cx<T> *buf, const cx<T> *__restrict__ tw, int lane,
                                          cx<T> *odd, cx<T> *even, int &b, int &k0,
                                          bool &valid) {
  using L = DstLanes<T, N1, B>;
  constexpr int CH = L::CH, G = L::G;
  wfft<T, N1, 1, B, S, PS, false, true>(buf, tw, lane);
  b = lane / G;
  const int g = lane % G;
  k0 = g * CH;
  valid = b < B;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    odd[c] = cx<T>{(T)0, (T)0};
    even[c] = cx<T>{(T)0, (T)0};
    if (valid) {
      const int k = k0 + c;
      const cx<T> Fk = buf[pk<PS>(k) * S + b];
      const cx<T> Fm = buf[pk<PS>((N1 - k) & (N1 - 1)) * S + b];
      cx<T> C = cscale(cadd(Fk, Fm), (T)0.5);
      if (k == 0) C = cscale(C, (T)0.5);
      odd[c] = C;
      even[c] = mul_i(cscale(csub(Fk, Fm), (T)0.5));
    }
  }
#pragma unroll
  for (int c = 1; c < CH; ++c) odd[c] = cadd(odd[c], odd[c - 1]);
  const cx<T> tot = odd[CH - 1];
  cx<T> inc = tot;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const cx<T> y = shfl_up_cx(inc, off);
    if (g >= off) inc = cadd(inc, y);
  }
  const cx<T> excl = csub(inc, tot);
#pragma unroll
  for (int c = 0; c < CH; ++c) odd[c] = cadd(odd[c], excl);
}

// Pre-processing straight from global memory: line b's x_i (i = 1..N1-1) is src(b, i-1);
// writes y_i = sin(pi i/N1)(x_i + x_{N1-i}) + (x_i - x_{N1-i})/2 and y_0 = 0 into buf.
template <typename T, int N1, int B, int S, int PS, typename Src>
__device__ __forceinline__ void dst_pre_global(cx<T> *buf, const T *__restrict__ sintab,
                                               int lane, Src src) {
  constexpr int H = N1 / 2, IT = (H * B + 63) / 64;
  cx<T> xa[IT], xb[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {  // every load is issued before any is consumed
    const int idx = lane + 64 * it, i = 1 + idx % H, b = idx / H;
    xa[it] = cx<T>{(T)0, (T)0};
    xb[it] = cx<T>{(T)0, (T)0};
    if ((H * B) % 64 == 0 || idx < H * B) {
      xa[it] = src(b, i - 1);
      xb[it] = src(b, N1 - i - 1);
    }
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = lane + 64 * it, i = 1 + idx % H, b = idx / H;
    if ((H * B) % 64 != 0 && idx >= H * B) continue;
    const T s = sintab[i];
    const cx<T> sum = cadd(xa[it], xb[it]);
    const cx<T> dif = cscale(csub(xa[it], xb[it]), (T)0.5);
    buf[pk<PS>(i) * S + b] = cadd(cscale(sum, s), dif);
    if (i != H) buf[pk<PS>(N1 - i) * S + b] = csub(cscale(sum, s), dif);
    if (i == 1) buf[b] = cx<T>{(T)0, (T)0};
  }
}

constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
constexpr int oddize(int b) { return b <= 2 ? b : (b | 1); }

// LDS budget of a tile workgroup: two such workgroups fit in the 160 KiB of a gfx950 CU.
constexpr int kTileLds = 81920;
constexpr int kCuLds = 163840;
constexpr int blocks_per_cu(int lds) { return lds > 0 ? kCuLds / lds : 0; }

// Time FFT tile: TS spatial columns x N time levels (4 waves, TS/4 columns each).
// Waves per workgroup (TS / WAVES columns each): the inverse transform runs 8 (its input
// loads are complex, half as many per column; measured 12% faster than 4 at n = 256),
// the forward transform 4 (8 gave no gain there).
constexpr int kTimeWavesFwd = 4, kTimeWavesInv = 8;
template <typename P, int N, int TS, int WV = kTimeWavesFwd> struct TimeCfg {
  static constexpr int WAVES = TS < WV ? TS : WV;
  static constexpr int NT = 64 * WAVES;
  static constexpr int CXB = 2 * (int)sizeof(P);
  static constexpr int PS = 4;
  static constexpr int PN = padded<PS>(N);
  static constexpr int S = TS + 1;  // odd column stride
  static constexpr int TILE = PN * S * CXB;
  static constexpr bool FITS = TILE <= kCuLds - 1024;
  // twiddles in LDS when that does not cost a resident workgroup
  static constexpr bool TW_LDS = blocks_per_cu(TILE + N * CXB) == blocks_per_cu(TILE);
};

template <typename P, int N1> struct RowCfg {
  static constexpr int CXB = 2 * (int)sizeof(P);
  static constexpr int PS = 3;
  static constexpr int PN = padded<PS>(N1);
  static constexpr int B = clampi(512 / N1, 1, 64);     // lines per wave
  static constexpr int S = oddize(B);
  static constexpr int UNITS = clampi(256 / N1, 1, 32);  // paired units per wave (1D)
  static constexpr int SU = oddize(2 * UNITS);
  static constexpr int TAB = N1 * CXB + N1 * (int)sizeof(P);  // twiddles + sine table
  static constexpr int WPB = clampi((kTileLds - TAB) / (PN * S * CXB), 1, 4);   // waves/block
  static constexpr int WPBU = clampi((kTileLds - TAB) / (PN * SU * CXB), 1, 4);
};

// x2 pass tile: TX x1-columns of both block rows (4 waves, TX/4 columns each).
// x2 pass: 4 waves per workgroup, TX / 4 columns (both block rows) each (8 waves measured
// no faster in FP64 and 20% slower in FP32)
constexpr int kColWaves = 4;
template <typename P, int N1, int TX> struct ColCfg {
  static constexpr int WAVES = TX < kColWaves ? TX : kColWaves;
  static constexpr int NT = 64 * WAVES;
  static constexpr int CXB = 2 * (int)sizeof(P);
  static constexpr int PS = 4;
  static constexpr int PN = padded<PS>(N1);
  static constexpr int TAB = N1 * CXB + N1 * (int)sizeof(P);
  static constexpr int S = 2 * TX + 1;
  static constexpr int CPW = TX / WAVES;                    // columns per wave
  static constexpr int MIT = (CPW * (N1 - 1) + 63) / 64;    // lane items of a wave's columns
  static constexpr int TILE = PN * S * CXB;
  static constexpr bool FITS = TILE <= kCuLds - 1024;
  static constexpr bool TAB_LDS = blocks_per_cu(TILE + TAB) == blocks_per_cu(TILE);
};

template <int NT = kThreads>
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
  }
  return r;
}

// ---- per-mode operation of step 2 ---------------------------------------------
// kind 0: P_S, [a; b] <- c [[conj(L), alpha], [-alpha, L]] [a; b] / (|L|^2 + alpha^2)
// kind 1: |P_S|, scale c / sqrt(|L|^2 + alpha^2);  kind 2: P_MS, c / (sigma_l + tau mu)
template <typename P>
__device__ __forceinline__ void mode_op(cx<P> &a, cx<P> &b, cx<P> l, P musum, int kind, P tau,
                                        P alpha, P cnorm) {
  if (kind == 0) {
    const cx<P> Lm = {l.x + tau * musum, l.y};
    const P c = cnorm / (Lm.x * Lm.x + Lm.y * Lm.y + alpha * alpha);
    const cx<P> ca = {Lm.x * a.x + Lm.y * a.y, Lm.x * a.y - Lm.y * a.x};
    const cx<P> lb = cmul(Lm, b);
    const cx<P> na = cscale(cx<P>{ca.x + alpha * b.x, ca.y + alpha * b.y}, c);
    const cx<P> nb = cscale(cx<P>{lb.x - alpha * a.x, lb.y - alpha * a.y}, c);
    a = na;
    b = nb;
  } else {
    P s;
    if (kind == 1) {
      const P re = l.x + tau * musum;
      s = cnorm / sqrt(re * re + l.y * l.y + alpha * alpha);
    } else {
      s = cnorm / (sqrt(l.x * l.x + l.y * l.y + alpha * alpha) + tau * musum);
    }
    a = cscale(a, s);
    b = cscale(b, s);
  }
}

// The same per-mode operation with the method and the block row fixed at compile time, as
// the x2 row pass uses it: own is this row's mode, other the partner row's (read for P_S
// only; the other two preconditioners scale each row by itself).
template <typename P, int KIND, int H>
__device__ __forceinline__ cx<P> mode_op_fixed(cx<P> own, cx<P> other, cx<P> l, P musum, P tau,
                                               P alpha, P cnorm) {
  if constexpr (KIND == 0) {
    const cx<P> Lm = {l.x + tau * musum, l.y};
    const P c = cnorm / (Lm.x * Lm.x + Lm.y * Lm.y + alpha * alpha);
    if constexpr (H == 0)  // (conj(L) a + alpha b) c with a = own, b = other
      return cscale(cx<P>{Lm.x * own.x + Lm.y * own.y + alpha * other.x,
                          Lm.x * own.y - Lm.y * own.x + alpha * other.y}, c);
    const cx<P> lb = cmul(Lm, own);  // (L b - alpha a) c with b = own, a = other
    return cscale(cx<P>{lb.x - alpha * other.x, lb.y - alpha * other.y}, c);
  } else if constexpr (KIND == 1) {
    const P re = l.x + tau * musum;
    return cscale(own, cnorm / sqrt(re * re + l.y * l.y + alpha * alpha));
  } else {
    return cscale(own, cnorm / (sqrt(l.x * l.x + l.y * l.y + alpha * alpha) + tau * musum));
  }
}

// ---- step 1a: time transform of both block rows ------------------------------
// v: 2 x (n, m) FP64.  W: [q][half][s] complex, q = 0..n/2-1 <-> frequency l = q+1.
template <typename P, int N, int TS, bool GEN, bool TWL>
__device__ __forceinline__ void tfft_fwd_tile(const double *__restrict__ v, cx<P> *__restrict__ W,
                                              const cx<double> *__restrict__ dtw,
                                              const cx<P> *__restrict__ twg, int m, GenIn gi,
                                              int tile, cx<P> *buf, cx<P> *stw) {
  using C = TimeCfg<P, N, TS>;
  constexpr int S = C::S, PS = C::PS, NT = C::NT, CPW = TS / C::WAVES;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int s0 = tile * TS;
  const double *v1 = v;
  const double *v2 = v + (size_t)N * m;
  // all global loads of the tile are issued before any is consumed
  constexpr int LIT = (N * TS + NT - 1) / NT;
  double ra[LIT], rb[LIT];
  // generated input: this thread's column is fixed (NT is a multiple of TS), so its
  // coefficients of the two range terms are formed once
  double gc = 0.0, a1 = 0.0, a2 = 0.0;
  if constexpr (GEN) {
    static_assert(NT % TS == 0, "a thread's column must not change");
    const int gs = s0 + tid % TS;
    gc = *gi.sqn0 > 0.0 ? gi.hat[0] / *gi.sqn0 : 0.0;
    if (gs < m) {
      a1 = gi.hat[1 + gs] * gi.inv_gn - gc * gi.s0[gs];
      a2 = gi.hat[1 + m + gs] * gi.inv_rn - gc * gi.s0[m + gs];
    }
  }
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    const int k = idx / TS, s = idx % TS, gs = s0 + s;
    ra[it] = 0.0;
    rb[it] = 0.0;
    if ((N * TS % NT == 0 || idx < N * TS) && gs < m) {
      if constexpr (std::is_same<P, double>::value) {
        // FP64: the input is streamed past the caches, the spectral array this pass writes
        // (as large as the memory-side cache) keeps it (measured 159 -> 147 us at n = 256,
        // M = 255; in FP32 the whole spectral array fits and streaming the input loses)
        ra[it] = __builtin_nontemporal_load(v1 + (size_t)k * m + gs);
        rb[it] = __builtin_nontemporal_load(v2 + (size_t)k * m + gs);
      } else {
        ra[it] = v1[(size_t)k * m + gs];
        rb[it] = v2[(size_t)k * m + gs];
      }
    }
  }
  // twiddles are staged while the tile's loads are in flight
  if constexpr (TWL)
    for (int i = tid; i < N; i += NT) stw[i] = twg[i];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (N * TS % NT == 0 || idx < N * TS) {
      const int k = idx / TS, s = idx % TS;
      const cx<double> d = dtw[k];
      double a = ra[it], b = rb[it];
      if constexpr (GEN) {
        // columns past m hold zeros there and get zero coefficients a1 = a2 = 0
        a = gc * a + gi.gr[k] * a1;
        b = gc * b + gi.gr[N + k] * a2;
      }
      buf[pk<PS>(k) * S + s] = cx<P>{(P)(a * d.x - b * d.y), (P)(a * d.y + b * d.x)};
    }
  }
  __syncthreads();
  wfft<P, N, 1, CPW, S, PS, false, true>(buf + wv * CPW, TWL ? stw : twg, lane);
  __syncthreads();
  for (int idx = tid; idx < (N / 2) * TS; idx += NT) {
    const int q = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs >= m) continue;
    const cx<P> Zl = buf[pk<PS>(q + 1) * S + s];
    const cx<P> Zp = buf[pk<PS>((N - q) & (N - 1)) * S + s];  // frequency (1-l) mod n
    const cx<P> A = {(Zl.x + Zp.x) * (P)0.5, (Zl.y - Zp.y) * (P)0.5};
    const cx<P> D = {(Zl.x - Zp.x) * (P)0.5, (Zl.y + Zp.y) * (P)0.5};
    W[((size_t)q * 2 + 0) * m + gs] = A;
    W[((size_t)q * 2 + 1) * m + gs] = mul_mi(D);
  }
}
template <typename P, int N, int TS, bool GEN>
__global__ __launch_bounds__((TimeCfg<P, N, TS>::NT)) void k_tfft_fwd(const double *__restrict__ v,
                                                       cx<P> *__restrict__ W,
                                                       const cx<double> *__restrict__ dtw,
                                                       const cx<P> *__restrict__ twg, int m,
                                                       GenIn gi) {
  using C = TimeCfg<P, N, TS>;
  __shared__ cx<P> buf[C::PN * C::S];
  __shared__ cx<P> stw[C::TW_LDS ? N : 1];
  tfft_fwd_tile<P, N, TS, GEN, C::TW_LDS>(v, W, dtw, twg, m, gi, xcd_tile(blockIdx.x, gridDim.x),
                                          buf, stw);
}

// ---- step 3b: inverse time transform, real output, optional fused <w, dotv> ----
template <typename P, int N, int TS, bool TWL>
__device__ __forceinline__ void tfft_inv_tile(const cx<P> *__restrict__ W, double *__restrict__ out,
                                              const cx<double> *__restrict__ dtw,
                                              const cx<P> *__restrict__ twg, int m,
                                              const double *__restrict__ dotv,
                                              double *__restrict__ partials, int tile, cx<P> *buf,
                                              cx<P> *stw, double *red) {
  using C = TimeCfg<P, N, TS, kTimeWavesInv>;
  constexpr int S = C::S, PS = C::PS, NT = C::NT, CPW = TS / C::WAVES;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int s0 = tile * TS;
  constexpr int HT = (N / 2) * TS;
  constexpr int LIT = (HT + NT - 1) / NT;
  cx<P> ra[LIT], rb[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    const int q = idx / TS, s = idx % TS, gs = s0 + s;
    ra[it] = cx<P>{(P)0, (P)0};
    rb[it] = cx<P>{(P)0, (P)0};
    if ((HT % NT == 0 || idx < HT) && gs < m) {
      ra[it] = W[((size_t)q * 2 + 0) * m + gs];
      rb[it] = W[((size_t)q * 2 + 1) * m + gs];
    }
  }
  if constexpr (TWL)
    for (int i = tid; i < N; i += NT) stw[i] = twg[i];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (HT % NT == 0 || idx < HT) {
      const int q = idx / TS, s = idx % TS;
      const cx<P> A = ra[it], Bv = rb[it];
      buf[pk<PS>(q + 1) * S + s] = cx<P>{A.x - Bv.y, A.y + Bv.x};              // A + iB
      buf[pk<PS>((N - q) & (N - 1)) * S + s] = cx<P>{A.x + Bv.y, Bv.x - A.y};  // conj(A) + i conj(B)
    }
  }
  __syncthreads();
  wfft<P, N, 1, CPW, S, PS, true, true>(buf + wv * CPW, TWL ? stw : twg, lane);
  __syncthreads();
  double acc = 0.0;
  double *o1 = out;
  double *o2 = out + (size_t)N * m;
  for (int idx = tid; idx < N * TS; idx += NT) {
    const int k = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs >= m) continue;
    const cx<P> z = buf[pk<PS>(k) * S + s];
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
    const double r = block_sum<NT>(acc, red);
    if (tid == 0) partials[tile] = r;
  }
}

template <typename P, int N, int TS>
__global__ __launch_bounds__((TimeCfg<P, N, TS, kTimeWavesInv>::NT)) void k_tfft_inv(const cx<P> *__restrict__ W,
                                                       double *__restrict__ out,
                                                       const cx<double> *__restrict__ dtw,
                                                       const cx<P> *__restrict__ twg, int m,
                                                       const double *__restrict__ dotv,
                                                       double *__restrict__ partials) {
  using C = TimeCfg<P, N, TS, kTimeWavesInv>;
  __shared__ cx<P> buf[C::PN * C::S];
  __shared__ cx<P> stw[C::TW_LDS ? N : 1];
  __shared__ double red[C::NT / 64];
  tfft_inv_tile<P, N, TS, C::TW_LDS>(W, out, dtw, twg, m, dotv, partials,
                                     xcd_tile(blockIdx.x, gridDim.x), buf, stw, red);
}

// ---- step 1a / 3b per block row: the time transform as an n/2-point FFT -----------------
// At zeta = pi the kept coefficients are a real sequence's DFT at half-integer frequencies,
// Y_p = sum_k v_k e^{-2 pi i k (p + 1/2)/n}, p < n/2 (frequency l = p + 1).  With
// z_j = e^{-2 pi i j/n} (v_{2j} + i v_{2j+1}) and Z its n/2-point DFT,
//   E_p = (Z_p + conj Z_{p'})/2,  O_p = (Z_p - conj Z_{p'})/(2i),  p' = n/2 - 1 - p,
//   Y_p = E_p + c_p O_p,  Y_{p'} = conj(E_p - c_p O_p),  c_p = e^{-i pi (2p+1)/n}
// (E and O are the DFTs of the twiddled even and odd samples, each conjugate symmetric
// under p <-> p').  The inverse runs the same steps backwards:
//   E_p = (Y_p + conj Y_{p'})/2,  O_p = conj(c_p) (Y_p - conj Y_{p'})/2,  Z_p = E_p + i O_p,
//   Z_{p'} = conj E_p + i conj O_p,  v_{2j} + i v_{2j+1} = 2 e^{2 pi i j/n} IDFT(Z)_j
// (unnormalised like the one-sequence form: the 1/n sits in step 2).  Each block row is
// transformed on its own, so a tile of TS columns holds n/2 complex values per column: half
// the LDS of the packed form at the same tile width, or twice the width (the real input
// rows read TS * 8 bytes at a time) at the same LDS.
// Waves per workgroup: 8 for the inverse transform and for FP32, 4 for the FP64 forward
// transform (measured at M = 511, n = 512: the FP64 inverse 5% faster with 8, the FP64
// forward 1% slower; FP32 with 32-column tiles 6% and 3% faster with 8).
template <typename P, bool INV> constexpr int time_waves_h() {
  return INV || sizeof(P) == 4 ? 8 : 4;
}
template <typename P, int N, int TS, int WV> struct TimeCfgH {
  static constexpr int N2 = N / 2;
  static constexpr int WAVES = TS < WV ? TS : WV;
  static constexpr int NT = 64 * WAVES;
  static constexpr int CXB = 2 * (int)sizeof(P);
  static constexpr int PS = 4;
  static constexpr int PN = padded<PS>(N2);
  static constexpr int S = TS + 1;
  static constexpr int TILE = PN * S * CXB + N2 * CXB;
};

template <typename P, int N, int TS>
__global__ __launch_bounds__((TimeCfgH<P, N, TS, time_waves_h<P, false>()>::NT)) void k_tfft_fwd_h(
    const double *__restrict__ v, cx<P> *__restrict__ W, const cx<double> *__restrict__ dtw,
    const cx<double> *__restrict__ twt, int m, int ntile) {
  using C = TimeCfgH<P, N, TS, time_waves_h<P, false>()>;
  constexpr int N2 = C::N2, S = C::S, PS = C::PS, NT = C::NT, CPW = TS / C::WAVES;
  constexpr int LIT = (N2 * TS + NT - 1) / NT;
  __shared__ cx<P> buf[C::PN * S];
  __shared__ cx<P> stw[N2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int h = t / ntile, s0 = (t % ntile) * TS;
  const double *src = v + (size_t)h * N * m;
  double ra[LIT], rb[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {  // every load issued before any is consumed
    const int idx = tid + it * NT, j = idx / TS, gs = s0 + idx % TS;
    ra[it] = 0.0;
    rb[it] = 0.0;
    if ((N2 * TS % NT == 0 || idx < N2 * TS) && gs < m) {
      ra[it] = __builtin_nontemporal_load(src + (size_t)(2 * j) * m + gs);
      rb[it] = __builtin_nontemporal_load(src + (size_t)(2 * j + 1) * m + gs);
    }
  }
  for (int i = tid; i < N2; i += NT) {  // e^{-2 pi i p/(n/2)}
    const cx<double> w = twt[2 * i];
    stw[i] = cx<P>{(P)w.x, (P)w.y};
  }
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (N2 * TS % NT == 0 || idx < N2 * TS) {
      const int j = idx / TS, s = idx % TS;
      const cx<double> w = twt[j];
      buf[pk<PS>(j) * S + s] = cx<P>{(P)(ra[it] * w.x - rb[it] * w.y), (P)(ra[it] * w.y + rb[it] * w.x)};
    }
  }
  __syncthreads();
  wfft<P, N2, 1, CPW, S, PS, false, true>(buf + wv * CPW, stw, lane);
  __syncthreads();
  for (int idx = tid; idx < (N2 / 2) * TS; idx += NT) {
    const int p = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs >= m) continue;
    const int pp = N2 - 1 - p;
    const cx<P> Zp = buf[pk<PS>(p) * S + s], Zq = buf[pk<PS>(pp) * S + s];
    const cx<P> E = {(Zp.x + Zq.x) * (P)0.5, (Zp.y - Zq.y) * (P)0.5};
    const cx<P> O = {(Zp.y + Zq.y) * (P)0.5, (Zq.x - Zp.x) * (P)0.5};  // (Zp - conj Zq)/(2i)
    const cx<double> d = dtw[2 * p + 1];                                // c_p = conj(d)
    const cx<P> cO = cmul(cx<P>{(P)d.x, (P)-d.y}, O);
    W[((size_t)p * 2 + h) * m + gs] = cadd(E, cO);
    W[((size_t)pp * 2 + h) * m + gs] = cx<P>{E.x - cO.x, cO.y - E.y};
  }
}

template <typename P, int N, int TS>
__global__ __launch_bounds__((TimeCfgH<P, N, TS, time_waves_h<P, true>()>::NT)) void k_tfft_inv_h(
    const cx<P> *__restrict__ W, double *__restrict__ out, const cx<double> *__restrict__ dtw,
    const cx<double> *__restrict__ twt, int m, int ntile, const double *__restrict__ dotv,
    double *__restrict__ partials) {
  using C = TimeCfgH<P, N, TS, time_waves_h<P, true>()>;
  constexpr int N2 = C::N2, S = C::S, PS = C::PS, NT = C::NT, CPW = TS / C::WAVES;
  constexpr int HT = (N2 / 2) * TS, LIT = (HT + NT - 1) / NT;
  __shared__ cx<P> buf[C::PN * S];
  __shared__ cx<P> stw[N2];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int h = t / ntile, s0 = (t % ntile) * TS;
  cx<P> ya[LIT], yb[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT, p = idx / TS, gs = s0 + idx % TS;
    ya[it] = cx<P>{(P)0, (P)0};
    yb[it] = cx<P>{(P)0, (P)0};
    if ((HT % NT == 0 || idx < HT) && gs < m) {
      ya[it] = W[((size_t)p * 2 + h) * m + gs];
      yb[it] = W[((size_t)(N2 - 1 - p) * 2 + h) * m + gs];
    }
  }
  for (int i = tid; i < N2; i += NT) {
    const cx<double> w = twt[2 * i];
    stw[i] = cx<P>{(P)w.x, (P)w.y};
  }
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (HT % NT == 0 || idx < HT) {
      const int p = idx / TS, s = idx % TS;
      const cx<P> Yp = ya[it], Yq = yb[it];
      const cx<P> E = {(Yp.x + Yq.x) * (P)0.5, (Yp.y - Yq.y) * (P)0.5};
      const cx<P> Dh = {(Yp.x - Yq.x) * (P)0.5, (Yp.y + Yq.y) * (P)0.5};  // (Yp - conj Yq)/2
      const cx<double> d = dtw[2 * p + 1];                                  // conj(c_p) = d
      const cx<P> O = cmul(cx<P>{(P)d.x, (P)d.y}, Dh);
      buf[pk<PS>(p) * S + s] = cx<P>{E.x - O.y, E.y + O.x};                  // E + i O
      buf[pk<PS>(N2 - 1 - p) * S + s] = cx<P>{E.x + O.y, O.x - E.y};         // conj E + i conj O
    }
  }
  __syncthreads();
  wfft<P, N2, 1, CPW, S, PS, true, true>(buf + wv * CPW, stw, lane);
  __syncthreads();
  double acc = 0.0;
  double *o = out + (size_t)h * N * m;
  const double *dv = dotv ? dotv + (size_t)h * N * m : nullptr;
  for (int idx = tid; idx < N2 * TS; idx += NT) {
    const int j = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs >= m) continue;
    const cx<P> z = buf[pk<PS>(j) * S + s];
    const cx<double> w = twt[j];  // times 2 conj(w) = 2 e^{2 pi i j/n}
    const double zx = (double)z.x, zy = (double)z.y;
    const double r0 = 2.0 * (zx * w.x + zy * w.y), r1 = 2.0 * (zy * w.x - zx * w.y);
    const size_t g = (size_t)(2 * j) * m + gs;
    o[g] = r0;
    o[g + m] = r1;
    if (dv) acc += r0 * dv[g] + r1 * dv[g + m];
  }
  if (dotv) {
    const double r = block_sum<NT>(acc, red);
    if (tid == 0) partials[t] = r;
  }
}

// ---- sine transform of contiguous rows, in place (2D x1 passes) ------------------
// nlines rows of M complex each; every wave owns B rows at a time.
template <typename P, int N1>
__device__ __forceinline__ void dst_rows_group(cx<P> *__restrict__ W, int nlines, int grp,
                                               const cx<P> *tw, const P *sn, cx<P> *buf,
                                               int lane) {
  using R = RowCfg<P, N1>;
  constexpr int M = N1 - 1, B = R::B, S = R::S, PS = R::PS;
  const int l0 = grp * B;
  dst_pre_global<P, N1, B, S, PS>(buf, sn, lane, [&](int b, int x) {
    return l0 + b < nlines ? W[(size_t)(l0 + b) * M + x] : cx<P>{(P)0, (P)0};
  });
  wave_sync();
  wdst_core<P, N1, B, S, PS>(buf, tw, lane);
  for (int idx = lane; idx < B * M; idx += 64) {  // coalesced store of the B lines
    const int b = idx / M, x = idx % M;
    if (l0 + b < nlines) W[(size_t)(l0 + b) * M + x] = buf[pk<PS>(x + 1) * S + b];
  }
  wave_sync();
}

template <typename P, int N1>
__global__ __launch_bounds__(kThreads) void k_dst_rows(cx<P> *__restrict__ W, int nlines,
                                                       const cx<P> *__restrict__ twg,
                                                       const P *__restrict__ sing) {
  using R = RowCfg<P, N1>;
  constexpr int B = R::B, S = R::S;
  __shared__ cx<P> lds[R::WPB][R::PN * S];
  __shared__ cx<P> stw[N1];
  __shared__ P ssin[N1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < N1; i += blockDim.x) {
    stw[i] = twg[i];
    ssin[i] = sing[i];
  }
  __syncthreads();
  const int ngroups = (nlines + B - 1) / B;
  for (int grp = blockIdx.x * R::WPB + wv; grp < ngroups; grp += gridDim.x * R::WPB)
    dst_rows_group<P, N1>(W, nlines, grp, stw, ssin, lds[wv], lane);
}

// ---- x1 sine transform of lines read and written through functors (the m-point work of
// a low-rank step: its input is formed as it loads and its output finished as it stores)
template <typename P, int N1, typename Src, typename Dst>
__global__ __launch_bounds__(kThreads) void k_dst_rows_fn(int nlines, const cx<P> *__restrict__ twg,
                                                          const P *__restrict__ sing, Src src,
                                                          Dst dst) {
  using R = RowCfg<P, N1>;
  constexpr int M = N1 - 1, B = R::B, S = R::S, PS = R::PS;
  __shared__ cx<P> lds[R::WPB][R::PN * S];
  __shared__ cx<P> stw[N1];
  __shared__ P ssin[N1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < N1; i += blockDim.x) {
    stw[i] = twg[i];
    ssin[i] = sing[i];
  }
  __syncthreads();
  cx<P> *buf = lds[wv];
  const int ngroups = (nlines + B - 1) / B;
  for (int grp = blockIdx.x * R::WPB + wv; grp < ngroups; grp += gridDim.x * R::WPB) {
    const int l0 = grp * B;
    dst_pre_global<P, N1, B, S, PS>(buf, ssin, lane, [&](int b, int x) {
      return l0 + b < nlines ? src(l0 + b, x) : cx<P>{(P)0, (P)0};
    });
    wave_sync();
    wdst_core<P, N1, B, S, PS>(buf, stw, lane);
    for (int idx = lane; idx < B * M; idx += 64) {
      const int b = idx / M, x = idx % M;
      if (l0 + b < nlines) dst(l0 + b, x, buf[pk<PS>(x + 1) * S + b]);
    }
    wave_sync();
  }
}

// 2D low-rank GMRES keeps the compact vectors and s0 in orthonormal sine coordinates
// (Q = (2/N1) DST_x1 DST_x2, symmetric and orthogonal, so Euclidean inner products are
// unchanged).
// s0_1 + i s0_2 in physical coordinates, line x2, and the same written back (scaled) as
// line j1 of the x2 pass
struct PairSrc {
  const double *s0;
  int m, M;
  __device__ cx<double> operator()(int x2, int x) const {
    const int s = x2 * M + x;
    return cx<double>{s0[s], s0[m + s]};
  }
};
struct PairStore {
  double *s0;
  int m, M;
  double scale;
  __device__ void operator()(int j1, int j2, cx<double> v) const {
    const int s = j2 * M + j1;
    s0[s] = scale * v.x;
    s0[m + s] = scale * v.y;
  }
};
// ... stored as A[x2][j1]
template <typename P> struct StoreA {
  cx<P> *A;
  int M;
  __device__ void operator()(int x2, int x, cx<P> v) const { A[x2 * M + x] = v; }
};
// x2 lines (one per x1 index j1) of an m-point field [x2][j1], read and written
template <typename T> struct ColLine {
  cx<T> *f;
  int M;
  __device__ cx<T> operator()(int j1, int x2) const { return f[x2 * M + j1]; }
  __device__ void operator()(int j1, int x2, cx<T> v) const { f[x2 * M + j1] = v; }
};

// ---- 1D: DST, step 2, inverse DST on both block rows of each frequency, in place ----
// W layout [q][half][x]; every wave owns UNITS frequencies (2*UNITS lines) at a time.
template <typename P, int N1>
__global__ __launch_bounds__(kThreads) void k_pair_rows(cx<P> *__restrict__ W, int nunits,
                                                        const cx<P> *__restrict__ twg,
                                                        const P *__restrict__ sing,
                                                        const cx<P> *__restrict__ lam,
                                                        const P *__restrict__ mu, int kind,
                                                        P tau, P alpha, P cnorm) {
  using R = RowCfg<P, N1>;
  constexpr int M = N1 - 1, UNITS = R::UNITS, B = 2 * UNITS, S = R::SU, PS = R::PS;
  __shared__ cx<P> lds[R::WPBU][R::PN * S];
  __shared__ cx<P> stw[N1];
  __shared__ P ssin[N1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < N1; i += blockDim.x) {
    stw[i] = twg[i];
    ssin[i] = sing[i];
  }
  __syncthreads();
  cx<P> *buf = lds[wv];
  const int ngroups = (nunits + UNITS - 1) / UNITS;
  for (int grp = blockIdx.x * R::WPBU + wv; grp < ngroups; grp += gridDim.x * R::WPBU) {
    const int u0 = grp * UNITS;
    const int nl = 2 * nunits;
    constexpr int LIT = (B * M + 63) / 64;
    cx<P> r[LIT];
#pragma unroll
    for (int it = 0; it < LIT; ++it) {
      const int idx = lane + 64 * it;
      const int b = idx / M, x = idx % M;
      r[it] = cx<P>{(P)0, (P)0};
      if (idx < B * M && 2 * u0 + b < nl) r[it] = W[(size_t)(2 * u0 + b) * M + x];
    }
#pragma unroll
    for (int it = 0; it < LIT; ++it) {
      const int idx = lane + 64 * it;
      if (idx < B * M) buf[pk<PS>(idx % M + 1) * S + idx / M] = r[it];
    }
    wave_sync();
    wdst<P, N1, B, S, PS>(buf, stw, ssin, lane);
    for (int idx = lane; idx < UNITS * M; idx += 64) {
      const int u = idx / M, j = idx % M;
      if (u0 + u >= nunits) continue;
      cx<P> a = buf[pk<PS>(j + 1) * S + 2 * u];
      cx<P> bb = buf[pk<PS>(j + 1) * S + 2 * u + 1];
      mode_op<P>(a, bb, lam[u0 + u], mu[j], kind, tau, alpha, cnorm);
      buf[pk<PS>(j + 1) * S + 2 * u] = a;
      buf[pk<PS>(j + 1) * S + 2 * u + 1] = bb;
    }
    wave_sync();
    wdst<P, N1, B, S, PS>(buf, stw, ssin, lane);
    for (int idx = lane; idx < B * M; idx += 64) {
      const int b = idx / M, x = idx % M;
      if (2 * u0 + b < nl) W[(size_t)(2 * u0 + b) * M + x] = buf[pk<PS>(x + 1) * S + b];
    }
    wave_sync();
  }
}

// ---- 2D spatial step on a transposed copy (large N1) --------------------------------
// The x2 transforms read columns of [q][h][x2][x1]; at N1 >= 128 a tile of columns of both
// block rows takes so much LDS that one or two workgroups fit per CU.  Instead the
// forward x1 pass writes its result transposed, T = [q][h][j1][x2] with row stride N1
// (x2 contiguous, rows aligned), the x2 pass works on contiguous rows of T, one
// (frequency, j1) unit per wave with its two block rows transformed one after the other
// (one LDS line per wave), and the inverse x1 pass reads T and writes [q][h][x2][x1] rows
// again.  The x1 passes use tiles of R consecutive rows (one per wave), so the transposed
// accesses move R consecutive elements at a time.
// Pad spacing of the LDS lines: every 8 elements in the forward pass, every 32 in the
// inverse pass (measured at N1 = 512: the inverse pass 5% faster in FP64 and 13% in FP32
// than with 8; the forward pass 8% slower in FP32 with 32).
template <typename P, int N1, int R, bool INV = false> struct TrCfg {
  static constexpr int CXB = 2 * (int)sizeof(P);
  static constexpr int PS = INV ? 5 : 3;
  static constexpr int PN = padded<PS>(N1);
  static constexpr int NT = 64 * R;
  static constexpr int TAB = N1 * CXB + N1 * (int)sizeof(P);
  static constexpr int BUF = R * PN * CXB;
  // tables in LDS only where that does not cost a resident workgroup
  static constexpr bool TAB_LDS = blocks_per_cu(BUF + TAB) == blocks_per_cu(BUF);
};
constexpr int kPairWaves = 4;  // waves per workgroup of the x2 row pass (two per unit)
template <typename P, int N1> struct PairCfg {
  static constexpr int CXB = 2 * (int)sizeof(P);
  static constexpr int PS = 3;
  static constexpr int PN = padded<PS>(N1);
  static constexpr int TAB = N1 * CXB + N1 * (int)sizeof(P);
  static constexpr int BUF = kPairWaves * PN * CXB;
  // the pass holds about 160 VGPRs per lane in FP64 at N1 = 512 (three waves per SIMD,
  // three workgroups per CU), so the tables go to LDS whenever three workgroups still fit
  static constexpr bool TAB_LDS = 3 * (BUF + TAB) <= kCuLds;
  // FP64 at N1 = 512: the P_S form is held to three waves per SIMD (168 VGPRs; left to the
  // compiler it takes 184 and two waves, measured 1416 us against 1268 us at M = 511,
  // n = 512); elsewhere the compiler's choice
  static constexpr int WAVES_PER_SIMD = sizeof(P) == 8 && N1 == 512 ? 3 : 1;
};

template <typename P, int N1, bool TWL>
__device__ __forceinline__ void stage_tables(const cx<P> *__restrict__ twg, const P *__restrict__ sing,
                                             cx<P> *stw, P *ssin, int nt) {
  if constexpr (TWL) {
    for (int i = threadIdx.x; i < N1; i += nt) {
      stw[i] = twg[i];
      ssin[i] = sing[i];
    }
  }
}

// forward x1 sine transform of R rows of a slab (q, h) of A, written to the slab of T
template <typename P, int N1, int R>
__global__ __launch_bounds__(64 * R) void k_rows_fwd_t(const cx<P> *__restrict__ A,
                                                       cx<P> *__restrict__ T,
                                                       const cx<P> *__restrict__ twg,
                                                       const P *__restrict__ sing) {
  using C = TrCfg<P, N1, R>;
  constexpr int M = N1 - 1, PS = C::PS, PN = C::PN, NT = C::NT, NRB = (M + R - 1) / R;
  __shared__ cx<P> lds[R * PN];
  __shared__ cx<P> stw[C::TAB_LDS ? N1 : 1];
  __shared__ P ssin[C::TAB_LDS ? N1 : 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int slab = t / NRB, rb = t % NRB, x2 = rb * R + wv;
  const cx<P> *src = A + (size_t)slab * M * M;
  cx<P> *buf = lds + wv * PN;
  stage_tables<P, N1, C::TAB_LDS>(twg, sing, stw, ssin, NT);
  if constexpr (C::TAB_LDS) __syncthreads();
  const cx<P> *tw = C::TAB_LDS ? stw : twg;
  const P *sn = C::TAB_LDS ? ssin : sing;
  dst_pre_global<P, N1, 1, 1, PS>(buf, sn, lane, [&](int, int x) {
    return x2 < M ? src[(size_t)x2 * M + x] : cx<P>{(P)0, (P)0};
  });
  wave_sync();
  wdst_core<P, N1, 1, 1, PS>(buf, tw, lane);
  __syncthreads();
  cx<P> *dst = T + (size_t)slab * M * N1;
  for (int idx = tid; idx < M * R; idx += NT) {
    const int r = idx % R, j1 = idx / R, xx = rb * R + r;
    if (xx < M) dst[(size_t)j1 * N1 + xx] = lds[r * PN + pk<PS>(j1 + 1)];
  }
}

// inverse x1 sine transform: R consecutive x2 of every j1 row of a slab of T, written as R
// rows of the slab of A
template <typename P, int N1, int R>
__global__ __launch_bounds__(64 * R) void k_rows_inv_t(const cx<P> *__restrict__ T,
                                                       cx<P> *__restrict__ A,
                                                       const cx<P> *__restrict__ twg,
                                                       const P *__restrict__ sing) {
  using C = TrCfg<P, N1, R, true>;
  constexpr int M = N1 - 1, PS = C::PS, PN = C::PN, NT = C::NT, NRB = (M + R - 1) / R;
  constexpr int LIT = (M * R + NT - 1) / NT;
  __shared__ cx<P> lds[R * PN];
  __shared__ cx<P> stw[C::TAB_LDS ? N1 : 1];
  __shared__ P ssin[C::TAB_LDS ? N1 : 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int slab = t / NRB, rb = t % NRB, x2 = rb * R + wv;
  const cx<P> *src = T + (size_t)slab * M * N1;
  cx<P> v[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {  // every load issued before any is consumed
    const int idx = tid + it * NT, r = idx % R, j1 = idx / R, xx = rb * R + r;
    v[it] = cx<P>{(P)0, (P)0};
    if (idx < M * R && xx < M) v[it] = src[(size_t)j1 * N1 + xx];
  }
  stage_tables<P, N1, C::TAB_LDS>(twg, sing, stw, ssin, NT);
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (idx < M * R) lds[(idx % R) * PN + pk<PS>(idx / R + 1)] = v[it];
  }
  __syncthreads();
  cx<P> *buf = lds + wv * PN;
  wdst<P, N1, 1, 1, PS>(buf, C::TAB_LDS ? stw : twg, C::TAB_LDS ? ssin : sing, lane);
  if (x2 < M) {
    cx<P> *dst = A + (size_t)slab * M * M + (size_t)x2 * M;
    for (int x = lane; x < M; x += 64) dst[x] = buf[pk<PS>(x + 1)];
  }
}

// x2 sine transform, step 2 and inverse x2 sine transform on T, in place.  A (q, j1) unit
// is two waves, one per block row, each transforming its line with the result in
// registers; for P_S (KIND 0) the per-mode operation couples the two through their LDS
// lines (each wave publishes its modes in natural order, reads its partner's, keeps its
// own block row of the 2x2 result), |P_S| (1) and P_MS (2) scale each row by itself; then
// each wave runs the inverse transform on its own line.  The method is a template
// argument and the block row a scalar, so neither costs per-lane selects.
template <typename P, int N1, int KIND>
__global__ __launch_bounds__(64 * kPairWaves) __attribute__((
    amdgpu_waves_per_eu(PairCfg<P, N1>::WAVES_PER_SIMD))) void k_pair_cols_t(
    cx<P> *__restrict__ T, int nunits, const cx<P> *__restrict__ twg, const P *__restrict__ sing,
    const cx<P> *__restrict__ lam, const P *__restrict__ mu, P tau, P alpha, P cnorm) {
  using C = PairCfg<P, N1>;
  using L = DstLanes<P, N1, 1>;
  constexpr int M = N1 - 1, PS = C::PS, PN = C::PN, CH = L::CH, UPB = kPairWaves / 2;
  static_assert(L::G == 64, "one line per wave: every lane holds modes of it");
  __shared__ cx<P> lds[kPairWaves * PN];
  __shared__ cx<P> stw[C::TAB_LDS ? N1 : 1];
  __shared__ P ssin[C::TAB_LDS ? N1 : 1];
  // the wave index is uniform across the wave: read it into a scalar register, so the
  // block row h selects code paths by scalar branches rather than per-lane selects
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), h = wv & 1;
  stage_tables<P, N1, C::TAB_LDS>(twg, sing, stw, ssin, 64 * kPairWaves);
  if constexpr (C::TAB_LDS) __syncthreads();
  const cx<P> *tw = C::TAB_LDS ? stw : twg;
  const P *sn = C::TAB_LDS ? ssin : sing;
  // units in XCD order (workgroups, then the workgroup's units)
  // a unit past the end (the last workgroup when nunits is odd) repeats the last unit and
  // stores nothing
  const int u0 = xcd_tile(blockIdx.x, gridDim.x) * UPB + (wv >> 1);
  const bool live = u0 < nunits;
  const int unit = live ? u0 : nunits - 1;
  const int q = unit / M, j1 = unit % M;
  cx<P> *row = T + ((size_t)(2 * q + h) * M + j1) * N1;
  cx<P> *buf = lds + wv * PN;
  const cx<P> *pbuf = lds + (wv ^ 1) * PN;  // the other block row's line
  cx<P> o[CH], e[CH];
  int b, k0;
  bool valid;
  dst_pre_global<P, N1, 1, 1, PS>(buf, sn, lane, [&](int, int x) { return row[x]; });
  wave_sync();
  wdst_regs<P, N1, 1, 1, PS>(buf, tw, lane, o, e, b, k0, valid);
  wave_sync();
  // modes j2 = 2k (odd outputs) and 2k - 1 (even outputs, k >= 1): k0 > 0 except on lane 0
  const cx<P> l = lam[q];
  const P muj1 = mu[j1];
  if constexpr (KIND == 0) {  // P_S couples the two block rows: exchange through LDS
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = k0 + c;
      buf[pk<PS>(2 * k + 1)] = o[c];
      if (k > 0) buf[pk<PS>(2 * k)] = e[c];
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = k0 + c;
        const cx<P> po = pbuf[pk<PS>(2 * k + 1)];
        const cx<P> pe = pbuf[pk<PS>(k > 0 ? 2 * k : 2 * k + 1)];
        o[c] = mode_op_fixed<P, 0, 0>(o[c], po, l, muj1 + mu[2 * k], tau, alpha, cnorm);
        e[c] = mode_op_fixed<P, 0, 0>(e[c], pe, l, muj1 + mu[k > 0 ? 2 * k - 1 : 0], tau,
                                      alpha, cnorm);
      }
    } else {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = k0 + c;
        const cx<P> po = pbuf[pk<PS>(2 * k + 1)];
        const cx<P> pe = pbuf[pk<PS>(k > 0 ? 2 * k : 2 * k + 1)];
        o[c] = mode_op_fixed<P, 0, 1>(o[c], po, l, muj1 + mu[2 * k], tau, alpha, cnorm);
        e[c] = mode_op_fixed<P, 0, 1>(e[c], pe, l, muj1 + mu[k > 0 ? 2 * k - 1 : 0], tau,
                                      alpha, cnorm);
      }
    }
    __syncthreads();
  } else {  // |P_S| and P_MS scale each row by itself
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int k = k0 + c;
      o[c] = mode_op_fixed<P, KIND, 0>(o[c], o[c], l, muj1 + mu[2 * k], tau, alpha, cnorm);
      e[c] = mode_op_fixed<P, KIND, 0>(e[c], e[c], l, muj1 + mu[k > 0 ? 2 * k - 1 : 0], tau,
                                       alpha, cnorm);
    }
  }
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int k = k0 + c;
    buf[pk<PS>(2 * k + 1)] = o[c];
    if (k > 0) buf[pk<PS>(2 * k)] = e[c];
  }
  wave_sync();
  wdst<P, N1, 1, 1, PS>(buf, tw, sn, lane);
  if (live)
    for (int x = lane; x < M; x += 64) row[x] = buf[pk<PS>(x + 1)];
}

// ---- 2D: x2-DST, step 2, x2-iDST on tiles of TX x1-columns (both block rows) -------
// W layout [q][half][x2][x1], x1 already sine transformed (index j1).
//
// 2D low-rank GMRES: the time and sine transforms are linear and r0 is fixed within a
// cycle, so the fully transformed spectrum of c r0 + [g (x) a1; r (x) a2] is
// c Yhat0 + F[q][h][0] Re Ahat + F[q][h][1] Im Ahat, with Yhat0 the cycle's transformed r0,
// F the time spectra of g and r, and Ahat the 2D sine transform of a1 + i a2 (k_lr_contract,
// k_cols_update).
// The loads of x2 tile t: item (c, h, i) of thread tid reads rows i-1 and N1-i-1 of
// column c0+c of block row h.
template <typename P, int N1, int TX>
__device__ __forceinline__ void cols_tile_load(const cx<P> *__restrict__ W, int t, int tid,
                                               cx<P> *ra, cx<P> *rb) {
  using C = ColCfg<P, N1, TX>;
  constexpr int M = N1 - 1, NT = C::NT, H = N1 / 2, TP = H * 2 * TX;
  constexpr int LIT = (TP + NT - 1) / NT;
  const int ncx = (N1 - 2 + TX) / TX;
  const int q = t / ncx, c0 = (t % ncx) * TX;
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    const int c = idx % TX, h = (idx / TX) & 1, i = 1 + idx / (2 * TX);
    ra[it] = cx<P>{(P)0, (P)0};
    rb[it] = cx<P>{(P)0, (P)0};
    if (idx < TP && c0 + c < M) {
      const size_t o1 = (size_t)(i - 1) * M + c0 + c, o2 = (size_t)(N1 - i - 1) * M + c0 + c;
      const cx<P> *src = W + ((size_t)q * 2 + h) * M * M;
      ra[it] = src[o1];
      rb[it] = src[o2];
    }
  }
}

// The first sine transform's pre-processing of a tile's loads (cols_tile_load order): item
// (c, h, i) writes y_i and y_{N1-i} of tile column 2c+h, and slot 0 is cleared.
template <typename P, int N1, int TX>
__device__ __forceinline__ void cols_pre_lds(const cx<P> *ra, const cx<P> *rb, cx<P> *buf,
                                             const P *sn, int tid) {
  using C = ColCfg<P, N1, TX>;
  constexpr int S = C::S, PS = C::PS, NT = C::NT, H = N1 / 2, TP = H * 2 * TX;
  constexpr int LIT = (TP + NT - 1) / NT;
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (idx >= TP) continue;
    const int c = idx % TX, h = (idx / TX) & 1, i = 1 + idx / (2 * TX), col = 2 * c + h;
    const P sv = sn[i];
    const cx<P> sum = cadd(ra[it], rb[it]);
    const cx<P> dif = cscale(csub(ra[it], rb[it]), (P)0.5);
    buf[pk<PS>(i) * S + col] = cadd(cscale(sum, sv), dif);
    if (i != H) buf[pk<PS>(N1 - i) * S + col] = csub(cscale(sum, sv), dif);
    if (i == 1) buf[col] = cx<P>{(P)0, (P)0};
  }
}

template <typename P, int N1, int TX, bool TABL>
__device__ __forceinline__ void cols_mode_tile(cx<P> *__restrict__ W, const cx<P> *__restrict__ twg,
                                               const P *__restrict__ sing,
                                               const cx<P> *__restrict__ lam,
                                               const P *__restrict__ mu, int kind, P tau, P alpha,
                                               P cnorm, int t, cx<P> *buf, cx<P> *stw, P *ssin) {
  using C = ColCfg<P, N1, TX>;
  constexpr int M = N1 - 1, S = C::S, PS = C::PS;
  constexpr int CPW = TX / C::WAVES, NT = C::NT;  // columns per wave, threads
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int ncx = (N1 - 2 + TX) / TX;  // column tiles per frequency, M = N1 - 1 columns
  const int q = t / ncx;
  const int c0 = (t % ncx) * TX;
  cx<P> *slab0 = W + ((size_t)q * 2 + 0) * M * M;
  cx<P> *slab1 = W + ((size_t)q * 2 + 1) * M * M;
  // tile column 2c+h holds (block row h, x1 column c0+c).  The first sine transform's
  // pre-processing is done on the loads: item (c, h, i) reads rows i-1 and N1-i-1 and
  // writes y_i, y_{N1-i} (all loads issued first).
  constexpr int TT = 2 * TX * M;
  constexpr int H = N1 / 2, TP = H * 2 * TX;
  constexpr int LIT = (TP + NT - 1) / NT;
  cx<P> ra[LIT], rb[LIT];
  cols_tile_load<P, N1, TX>(W, t, tid, ra, rb);
  if constexpr (TABL) {
    for (int i = tid; i < N1; i += NT) {
      stw[i] = twg[i];
      ssin[i] = sing[i];
    }
  }
  __syncthreads();  // the sine table is read below
  const P *sn = TABL ? ssin : sing;
  cols_pre_lds<P, N1, TX>(ra, rb, buf, sn, tid);
  __syncthreads();
  const cx<P> *tw = TABL ? stw : twg;
  cx<P> *wb = buf + wv * 2 * CPW;
  wdst_core<P, N1, 2 * CPW, S, PS>(wb, tw, lane);
  const cx<P> l = lam[q];
  for (int idx = lane; idx < CPW * M; idx += 64) {
    const int c = idx / M, j2 = idx % M;
    const int j1 = c0 + wv * CPW + c;
    if (j1 >= M) continue;
    cx<P> a = wb[pk<PS>(j2 + 1) * S + 2 * c];
    cx<P> bb = wb[pk<PS>(j2 + 1) * S + 2 * c + 1];
    mode_op<P>(a, bb, l, mu[j1] + mu[j2], kind, tau, alpha, cnorm);
    wb[pk<PS>(j2 + 1) * S + 2 * c] = a;
    wb[pk<PS>(j2 + 1) * S + 2 * c + 1] = bb;
  }
  wave_sync();
  wdst<P, N1, 2 * CPW, S, PS>(wb, tw, sn, lane);
  __syncthreads();
  for (int idx = tid; idx < TT; idx += NT) {
    const int c = idx % TX, h = (idx / TX) & 1, x2 = idx / (2 * TX);
    if (c0 + c < M)
      (h ? slab1 : slab0)[(size_t)x2 * M + c0 + c] = buf[pk<PS>(x2 + 1) * S + 2 * c + h];
  }
}

template <typename P, int N1, int TX>
__global__ __launch_bounds__((ColCfg<P, N1, TX>::NT)) void k_cols_mode(cx<P> *__restrict__ W,
                                                        const cx<P> *__restrict__ twg,
                                                        const P *__restrict__ sing,
                                                        const cx<P> *__restrict__ lam,
                                                        const P *__restrict__ mu, int kind,
                                                        P tau, P alpha, P cnorm) {
  using C = ColCfg<P, N1, TX>;
  __shared__ cx<P> buf[C::PN * C::S];
  __shared__ cx<P> stw[C::TAB_LDS ? N1 : 1];
  __shared__ P ssin[C::TAB_LDS ? N1 : 1];
  cols_mode_tile<P, N1, TX, C::TAB_LDS>(W, twg, sing, lam, mu, kind, tau, alpha, cnorm,
                                        xcd_tile(blockIdx.x, gridDim.x), buf, stw, ssin);
}


// 2D low-rank GMRES step: the x2 pass on the generated input, contracted over time before
// the inverse x1 transform (the contraction sum_q 2 Re(rho_q Z_q) commutes with it, the
// sine transform being real), so the spectrum is never written: workgroup (chunk, column
// tile) runs the tile body for the frequencies of its chunk and writes its sums,
// part[chunk][h m + x2 M + j1].
// the compact output of a 2D low-rank step in sine coordinates: hat[0] = 0 and
// hat[1 + h m + s] = scale_h * (sum of the chunk partials of block row h at s)
__global__ __launch_bounds__(kThreads) void k_lr_hat_out(const double *__restrict__ part,
                                                         double *__restrict__ hat, int m,
                                                         double sg, double sr) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= m) return;
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int c = 0; c < kColChunks; ++c) {
    a += part[(size_t)c * 2 * m + s];
    b += part[(size_t)c * 2 * m + m + s];
  }
  if (s == 0) hat[0] = 0.0;
  hat[1 + s] = sg * a;
  hat[1 + m + s] = sr * b;
}



// x2 sine transform of both block rows of every frequency (in == out allowed: every tile is
// read whole before it is written): the cycle's r0 spectrum in full sine coordinates, from
// which a 2D low-rank step works pointwise
template <typename P, int N1, int TX>
__global__ __launch_bounds__((ColCfg<P, N1, TX>::NT)) void k_cols_dst(
    const cx<P> *in, cx<P> *out, const cx<P> *__restrict__ twg, const P *__restrict__ sing) {
  using C = ColCfg<P, N1, TX>;
  constexpr int M = N1 - 1, S = C::S, PS = C::PS, NT = C::NT, CPW = C::CPW, TT = 2 * TX * M;
  constexpr int LIT = (N1 / 2 * 2 * TX + NT - 1) / NT;
  __shared__ cx<P> buf[C::PN * C::S];
  __shared__ cx<P> stw[C::TAB_LDS ? N1 : 1];
  __shared__ P ssin[C::TAB_LDS ? N1 : 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int ncx = (N1 - 2 + TX) / TX;
  const int q = t / ncx, c0 = (t % ncx) * TX;
  cx<P> ra[LIT], rb[LIT];
  cols_tile_load<P, N1, TX>(in, t, tid, ra, rb);
  if constexpr (C::TAB_LDS) {
    for (int i = tid; i < N1; i += NT) {
      stw[i] = twg[i];
      ssin[i] = sing[i];
    }
  }
  __syncthreads();
  cols_pre_lds<P, N1, TX>(ra, rb, buf, C::TAB_LDS ? ssin : sing, tid);
  __syncthreads();
  wdst_core<P, N1, 2 * CPW, S, PS>(buf + wv * 2 * CPW, C::TAB_LDS ? stw : twg, lane);
  __syncthreads();
  cx<P> *o0 = out + (size_t)q * 2 * M * M;
  for (int idx = tid; idx < TT; idx += NT) {
    const int c = idx % TX, h = (idx / TX) & 1, j2 = idx / (2 * TX);
    if (c0 + c < M)
      o0[(size_t)h * M * M + (size_t)j2 * M + c0 + c] = buf[pk<PS>(j2 + 1) * S + 2 * c + h];
  }
}

// Ahat = (N1/2)(a1 + i a2) of the compact vector (orthonormal sine coordinates), FP64
__global__ __launch_bounds__(kThreads) void k_lr_ahat(GenIn gi, double ascale, int m,
                                                      cx<double> *__restrict__ A) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= m) return;
  const double gc = *gi.sqn0 > 0.0 ? gi.hat[0] / *gi.sqn0 : 0.0;
  A[s] = cx<double>{ascale * (gi.hat[1 + s] * gi.inv_gn - gc * gi.s0[s]),
                    ascale * (gi.hat[1 + m + s] * gi.inv_rn - gc * gi.s0[m + s])};
}

// The cycle's update in 2D low-rank GMRES, in place over the spectrum array that holds
// Yhat0: every tile forms c Yhat0 + F (Re Ahat, Im Ahat) of its modes as it loads, solves
// them, and applies the inverse x2 transform (the inverse x1 and time transforms follow as
// in the standard apply).
template <typename P, int N1, int TX>
__global__ __launch_bounds__((ColCfg<P, N1, TX>::NT)) void k_cols_update(
    cx<P> *__restrict__ W, const cx<P> *__restrict__ twg, const P *__restrict__ sing,
    const cx<P> *__restrict__ lam, const P *__restrict__ mu, int kind, P tau, P alpha, P cnorm,
    const double *__restrict__ hat, const double *__restrict__ sqn0,
    const cx<double> *__restrict__ Ah, const cx<double> *__restrict__ F) {
  using C = ColCfg<P, N1, TX>;
  constexpr int M = N1 - 1, S = C::S, PS = C::PS, NT = C::NT, CPW = C::CPW, TT = 2 * TX * M;
  constexpr int TI = TX * M, LIT = (TI + NT - 1) / NT;
  __shared__ cx<P> buf[C::PN * C::S];
  __shared__ cx<P> stw[C::TAB_LDS ? N1 : 1];
  __shared__ P ssin[C::TAB_LDS ? N1 : 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int ncx = (N1 - 2 + TX) / TX;
  const int q = t / ncx, c0 = (t % ncx) * TX;
  const size_t m = (size_t)M * M;
  cx<P> *slab0 = W + (size_t)q * 2 * m, *slab1 = slab0 + m;
  const double gc = *sqn0 > 0.0 ? hat[0] / *sqn0 : 0.0;
  // item (c, j2): both block rows of mode (c0 + c, j2); all loads issued first
  cx<P> y0[LIT], y1[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT, c = idx % TX, j2 = idx / TX;
    y0[it] = cx<P>{(P)0, (P)0};
    y1[it] = cx<P>{(P)0, (P)0};
    if (idx < TI && c0 + c < M) {
      y0[it] = load_stream(slab0 + (size_t)j2 * M + c0 + c);
      y1[it] = load_stream(slab1 + (size_t)j2 * M + c0 + c);
    }
  }
  if constexpr (C::TAB_LDS) {
    for (int i = tid; i < N1; i += NT) {
      stw[i] = twg[i];
      ssin[i] = sing[i];
    }
  }
  const cx<double> f00 = F[q * 4], f01 = F[q * 4 + 1], f10 = F[q * 4 + 2], f11 = F[q * 4 + 3];
  const cx<P> l = lam[q];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT, c = idx % TX, j2 = idx / TX, j1 = c0 + c;
    if (idx >= TI) continue;
    cx<P> u0{(P)0, (P)0}, u1{(P)0, (P)0};
    if (j1 < M) {
      const cx<double> A = Ah[j2 * M + j1];
      const double ax = A.x, ay = A.y;
      u0 = cx<P>{(P)(gc * y0[it].x + f00.x * ax + f01.x * ay),
                 (P)(gc * y0[it].y + f00.y * ax + f01.y * ay)};
      u1 = cx<P>{(P)(gc * y1[it].x + f10.x * ax + f11.x * ay),
                 (P)(gc * y1[it].y + f10.y * ax + f11.y * ay)};
      mode_op<P>(u0, u1, l, mu[j1] + mu[j2], kind, tau, alpha, cnorm);
    }
    buf[pk<PS>(j2 + 1) * S + 2 * c] = u0;
    buf[pk<PS>(j2 + 1) * S + 2 * c + 1] = u1;
  }
  __syncthreads();
  wdst<P, N1, 2 * CPW, S, PS>(buf + wv * 2 * CPW, C::TAB_LDS ? stw : twg,
                              C::TAB_LDS ? ssin : sing, lane);
  __syncthreads();
  for (int idx = tid; idx < TT; idx += NT) {
    const int c = idx % TX, h = (idx / TX) & 1, x2 = idx / (2 * TX);
    if (c0 + c < M)
      (h ? slab1 : slab0)[(size_t)x2 * M + c0 + c] = buf[pk<PS>(x2 + 1) * S + 2 * c + h];
  }
}

// 2D low-rank GMRES step, pointwise in full sine coordinates (both sine transforms are real
// matrices, so they commute with forming the input and with the real-part sum over
// frequencies).  For spatial mode s and frequency q the input is
//   u_h = c Yhat0[q][h][s] + F[q][h][0] Re Ahat[s] + F[q][h][1] Im Ahat[s]  (h = 0, 1),
// where Ahat = (N1/2) (a1 + i a2) is formed here from the compact vector and s0 (both in
// orthonormal sine coordinates), the per-mode solve maps (u_0, u_1) to (z_0, z_1), and
//   part[chunk][h][s] = sum over the chunk's q of 2 Re(rho[h nq + q] z_h).
template <typename P>
__global__ __launch_bounds__(kThreads) void k_lr_contract(
    const cx<P> *__restrict__ Yh, GenIn gi, double ascale, const cx<double> *__restrict__ F,
    const cx<P> *__restrict__ lam, const P *__restrict__ mu, int kind, P tau, P alpha, P cnorm,
    const cx<double> *__restrict__ rho, int nq, int M, double *__restrict__ part) {
  constexpr int QB = 8;  // frequencies whose loads are issued together
  const int m = M * M;
  const int s = blockIdx.x * kThreads + threadIdx.x, chunk = blockIdx.y;
  if (s >= m) return;
  const int per = (nq + kColChunks - 1) / kColChunks;
  const int q0 = chunk * per, q1 = q0 + per < nq ? q0 + per : nq;
  const double gc = *gi.sqn0 > 0.0 ? gi.hat[0] / *gi.sqn0 : 0.0;
  const int j2 = s / M, j1 = s - j2 * M;
  const P mus = mu[j1] + mu[j2];
  const cx<double> a{ascale * (gi.hat[1 + s] * gi.inv_gn - gc * gi.s0[s]),
                     ascale * (gi.hat[1 + m + s] * gi.inv_rn - gc * gi.s0[m + s])};
  double acc0 = 0.0, acc1 = 0.0;
  for (int qb = q0; qb < q1; qb += QB) {
    cx<P> y0[QB], y1[QB];
#pragma unroll
    for (int u = 0; u < QB; ++u) {
      if (qb + u < q1) {
        y0[u] = load_stream(Yh + (size_t)(qb + u) * 2 * m + s);
        y1[u] = load_stream(Yh + ((size_t)(qb + u) * 2 + 1) * m + s);
      }
    }
#pragma unroll
    for (int u = 0; u < QB; ++u) {
      const int q = qb + u;
      if (q < q1) {
        const cx<double> f00 = F[q * 4], f01 = F[q * 4 + 1], f10 = F[q * 4 + 2],
                         f11 = F[q * 4 + 3];
        cx<P> z0{(P)(gc * y0[u].x + f00.x * a.x + f01.x * a.y),
                 (P)(gc * y0[u].y + f00.y * a.x + f01.y * a.y)};
        cx<P> z1{(P)(gc * y1[u].x + f10.x * a.x + f11.x * a.y),
                 (P)(gc * y1[u].y + f10.y * a.x + f11.y * a.y)};
        mode_op<P>(z0, z1, lam[q], mus, kind, tau, alpha, cnorm);
        const cx<double> r0 = rho[q], r1 = rho[nq + q];
        acc0 += 2.0 * (r0.x * (double)z0.x - r0.y * (double)z0.y);
        acc1 += 2.0 * (r1.x * (double)z1.x - r1.y * (double)z1.y);
      }
    }
  }
  part[(size_t)chunk * 2 * m + s] = acc0;
  part[(size_t)chunk * 2 * m + m + s] = acc1;
}

// ---- low-rank GMRES: time contraction on the spectrum (replaces the inverse FFT) ----
// part[c][s] = sum over the frequencies q of chunk c of 2 Re(rho_r[q] A_q[s]), and
// part[c][m + s] likewise with rho_g and B_q[s] (A = block row 1, B = block row 2).
__global__ __launch_bounds__(kThreads) void k_contract_freq(const cx<double> *__restrict__ W,
                                                            ContractOut co, int m, int nq) {
  const int s = blockIdx.x * kThreads + threadIdx.x, c = blockIdx.y;
  if (s >= m) return;
  const int per = (nq + kContractChunks - 1) / kContractChunks;
  const int q0 = c * per, q1 = q0 + per < nq ? q0 + per : nq;
  const cx<double> *rr = reinterpret_cast<const cx<double> *>(co.rho);
  const cx<double> *rg = rr + nq;
  double a1 = 0.0, a2 = 0.0;
  for (int q = q0; q < q1; ++q) {
    const cx<double> A = W[((size_t)q * 2 + 0) * m + s], B = W[((size_t)q * 2 + 1) * m + s];
    const cx<double> u = rr[q], w = rg[q];
    a1 += u.x * A.x - u.y * A.y;
    a2 += w.x * B.x - w.y * B.y;
  }
  co.part[(size_t)c * 2 * m + s] = 2.0 * a1;
  co.part[(size_t)c * 2 * m + m + s] = 2.0 * a2;
}

__global__ __launch_bounds__(kThreads) void k_contract_final(ContractOut co, int m) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) co.hat[0] = 0.0;
  if (s >= m) return;
  double a1 = 0.0, a2 = 0.0;
#pragma unroll
  for (int c = 0; c < kContractChunks; ++c) {
    a1 += co.part[(size_t)c * 2 * m + s];
    a2 += co.part[(size_t)c * 2 * m + m + s];
  }
  co.hat[1 + s] = co.gn_omega * a1;
  co.hat[1 + m + s] = co.rn_omega * a2;
}

// ---- host dispatch -------------------------------------------------------------
template <typename P> struct Tabs;
template <> struct Tabs<double> {
  static const cx<double> *twt(const wc_plan &p) { return (const cx<double> *)p.d_twt64; }
  static const cx<double> *tws(const wc_plan &p) { return (const cx<double> *)p.d_tws64; }
  static const double *sin(const wc_plan &p) { return p.d_sin64; }
  static const cx<double> *lam(const wc_plan &p) { return (const cx<double> *)p.d_lam64; }
  static const double *mu(const wc_plan &p) { return p.d_mu64; }
  static const double *cos(const wc_plan &p) { return p.d_cos64; }
  static const cx<double> *phi(const wc_plan &p) { return (const cx<double> *)p.d_phi64; }
  static const cx<double> *lamf(const wc_plan &p) { return (const cx<double> *)p.d_lamf64; }
};
template <> struct Tabs<float> {
  static const cx<float> *twt(const wc_plan &p) { return (const cx<float> *)p.d_twt32; }
  static const cx<float> *tws(const wc_plan &p) { return (const cx<float> *)p.d_tws32; }
  static const float *sin(const wc_plan &p) { return p.d_sin32; }
  static const cx<float> *lam(const wc_plan &p) { return (const cx<float> *)p.d_lam32; }
  static const float *mu(const wc_plan &p) { return p.d_mu32; }
  static const float *cos(const wc_plan &p) { return p.d_cos32; }
  static const cx<float> *phi(const wc_plan &p) { return (const cx<float> *)p.d_phi32; }
  static const cx<float> *lamf(const wc_plan &p) { return (const cx<float> *)p.d_lamf32; }
};

int row_grid(int wave_groups, int wpb) {
  int g = (wave_groups + wpb - 1) / wpb;
  return g < 1 ? 1 : (g > 8192 ? 8192 : g);
}

// Tile widths: a plan's choice (autotuned or set) or the widest tile that keeps two
// workgroups resident per CU.
template <typename P, int N> constexpr int default_ts() {
  if constexpr (TimeCfg<P, N, 16>::FITS && blocks_per_cu(TimeCfg<P, N, 16>::TILE) >= 2) return 16;
  else if constexpr (TimeCfg<P, N, 8>::FITS && blocks_per_cu(TimeCfg<P, N, 8>::TILE) >= 2) return 8;
  else return 4;
}
template <typename P, int N1> constexpr int default_tx() {
  if constexpr (ColCfg<P, N1, 8>::FITS && blocks_per_cu(ColCfg<P, N1, 8>::TILE) >= 2) return 8;
  else return 4;
}

template <typename P, int N, int TS>
hipError_t tfft_fwd_ts(const wc_plan &p, const double *v, const GenIn *gen, cx<P> *out) {
  if constexpr (!TimeCfg<P, N, TS>::FITS) {
    return tfft_fwd_ts<P, N, 4>(p, v, gen, out);
  } else {
    dim3 grid((p.m + TS - 1) / TS);
    ProfScope ps(p, K_TFFT_FWD, (double)p.nvec * (8.0 + sizeof(P)));
    if constexpr (std::is_same<P, double>::value) {
      if (gen) {
        hipLaunchKernelGGL((k_tfft_fwd<P, N, TS, true>), grid, dim3(TimeCfg<P, N, TS>::NT), 0, p.stream, v,
                           out, (const cx<double> *)p.d_dtw, Tabs<P>::twt(p),
                           p.m, *gen);
        return hipGetLastError();
      }
    }
    if (gen) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tfft_fwd<P, N, TS, false>), grid, dim3(TimeCfg<P, N, TS>::NT), 0, p.stream, v,
                       out, (const cx<double> *)p.d_dtw, Tabs<P>::twt(p), p.m,
                       GenIn{});
    return hipGetLastError();
  }
}

template <typename P, int N, int TS>
hipError_t tfft_inv_ts(const wc_plan &p, double *w, const double *dotv, int *nparts) {
  if constexpr (!TimeCfg<P, N, TS>::FITS) {
    return tfft_inv_ts<P, N, 4>(p, w, dotv, nparts);
  } else {
    dim3 grid((p.m + TS - 1) / TS);
    *nparts = grid.x;
    ProfScope ps(p, K_TFFT_INV, (double)p.nvec * (sizeof(P) + (dotv ? 16.0 : 8.0)));
    hipLaunchKernelGGL((k_tfft_inv<P, N, TS>), grid, dim3(TimeCfg<P, N, TS, kTimeWavesInv>::NT), 0,
                       p.stream,
                       (const cx<P> *)p.d_specA, w, (const cx<double> *)p.d_dtw, Tabs<P>::twt(p),
                       p.m, dotv, p.d_partials);
    return hipGetLastError();
  }
}

// time-pass choice: ts_time > 0 the packed one-sequence kernels with that tile width, < 0
// the per-block-row kernels (n >= 64) with tile width -ts_time; 0 the default
// per-block-row tiles: 16 columns where two workgroups fit per CU, else 8; FP32 32
// columns where two still fit (measured at n = 512: 0.73 ms per pass against 0.9 ms at 16;
// in FP64 a 32-column tile leaves one workgroup per CU and is slower, 1.17 against 0.96 ms)
template <typename P, int N> constexpr bool fits_ts_h(int ts) {
  return ts == 32 ? TimeCfgH<P, N, 32, 4>::TILE <= kCuLds : true;
}
template <typename P, int N> constexpr int default_ts_h() {
  if (std::is_same<P, float>::value && blocks_per_cu(TimeCfgH<P, N, 32, 4>::TILE) >= 2) return 32;
  return blocks_per_cu(TimeCfgH<P, N, 16, 4>::TILE) >= 2 ? 16 : 8;
}
template <typename P, int N> int time_choice(const wc_plan &p) {
  if (p.ts_time) return (p.ts_time < 0 && N < 64) ? default_ts<P, N>() : p.ts_time;
  if constexpr (N >= 64) return -default_ts_h<P, N>();
  return default_ts<P, N>();
}

template <typename P, int N, int TS>
hipError_t tfft_fwd_h(const wc_plan &p, const double *v) {
  const int ntile = (p.m + TS - 1) / TS;
  ProfScope ps(p, K_TFFT_FWD, (double)p.nvec * (8.0 + sizeof(P)));
  hipLaunchKernelGGL((k_tfft_fwd_h<P, N, TS>), dim3(2 * ntile),
                     dim3(TimeCfgH<P, N, TS, time_waves_h<P, false>()>::NT), 0,
                     p.stream, v, (cx<P> *)p.d_specA, (const cx<double> *)p.d_dtw,
                     (const cx<double> *)p.d_twt64, p.m, ntile);
  return hipGetLastError();
}

template <typename P, int N, int TS>
hipError_t tfft_inv_h(const wc_plan &p, double *w, const double *dotv, int *nparts) {
  const int ntile = (p.m + TS - 1) / TS;
  *nparts = 2 * ntile;
  ProfScope ps(p, K_TFFT_INV, (double)p.nvec * (sizeof(P) + (dotv ? 16.0 : 8.0)));
  hipLaunchKernelGGL((k_tfft_inv_h<P, N, TS>), dim3(2 * ntile),
                     dim3(TimeCfgH<P, N, TS, time_waves_h<P, true>()>::NT), 0,
                     p.stream, (const cx<P> *)p.d_specA, w, (const cx<double> *)p.d_dtw,
                     (const cx<double> *)p.d_twt64, p.m, ntile, dotv, p.d_partials);
  return hipGetLastError();
}

template <typename P, int N>
hipError_t run_tfft_fwd(const wc_plan &p, const double *v, const GenIn *gen,
                        cx<P> *out = nullptr) {
  if constexpr (N >= 64) {
    const int tc = time_choice<P, N>(p);
    if (tc < 0 && !gen && !out) {
      if constexpr (fits_ts_h<P, N>(32))
        if (tc == -32) return tfft_fwd_h<P, N, 32>(p, v);
      return tc == -8 ? tfft_fwd_h<P, N, 8>(p, v) : tfft_fwd_h<P, N, 16>(p, v);
    }
  }
  if (!out) out = (cx<P> *)p.d_specA;
  switch (p.ts_time > 0 ? p.ts_time : default_ts<P, N>()) {
    case 4: return tfft_fwd_ts<P, N, 4>(p, v, gen, out);
    case 8: return tfft_fwd_ts<P, N, 8>(p, v, gen, out);
    default: return tfft_fwd_ts<P, N, 16>(p, v, gen, out);
  }
}

template <typename P, int N>
hipError_t run_tfft_inv(const wc_plan &p, double *w, const double *dotv, int *nparts) {
  if constexpr (N >= 64) {
    const int tc = time_choice<P, N>(p);
    if (tc < 0) {
      if constexpr (fits_ts_h<P, N>(32))
        if (tc == -32) return tfft_inv_h<P, N, 32>(p, w, dotv, nparts);
      return tc == -8 ? tfft_inv_h<P, N, 8>(p, w, dotv, nparts)
                      : tfft_inv_h<P, N, 16>(p, w, dotv, nparts);
    }
  }
  switch (p.ts_time > 0 ? p.ts_time : default_ts<P, N>()) {
    case 4: return tfft_inv_ts<P, N, 4>(p, w, dotv, nparts);
    case 8: return tfft_inv_ts<P, N, 8>(p, w, dotv, nparts);
    default: return tfft_inv_ts<P, N, 16>(p, w, dotv, nparts);
  }
}

template <typename P, int N1, int TX>
hipError_t cols_tx(const wc_plan &p, int kind, double c) {
  if constexpr (!ColCfg<P, N1, TX>::FITS) {
    return cols_tx<P, N1, 4>(p, kind, c);
  } else {
    constexpr int M = N1 - 1;
    const int ncx = (M + TX - 1) / TX;
    ProfScope ps(p, K_PAIR_MODE, 2.0 * p.nvec * sizeof(P));
    hipLaunchKernelGGL((k_cols_mode<P, N1, TX>), dim3(ncx * (p.n / 2)),
                       dim3(ColCfg<P, N1, TX>::NT), 0, p.stream, (cx<P> *)p.d_specA,
                       Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lam(p), Tabs<P>::mu(p), kind,
                       (P)p.tau, (P)p.alpha, (P)c);
    return hipGetLastError();
  }
}

template <typename P, int N1, typename Src, typename Dst>
hipError_t launch_rows_fn(const wc_plan &p, int nlines, Src src, Dst dst, int prof_id,
                          double bytes) {
  using R = RowCfg<P, N1>;
  dim3 gr(row_grid((nlines + R::B - 1) / R::B, R::WPB));
  ProfScope ps(p, prof_id, bytes);
  hipLaunchKernelGGL((k_dst_rows_fn<P, N1, Src, Dst>), gr, dim3(64 * R::WPB), 0, p.stream,
                     nlines, Tabs<P>::tws(p), Tabs<P>::sin(p), src, dst);
  return hipGetLastError();
}

// x1 sine transform of nlines contiguous lines in place
template <typename P, int N1>
hipError_t dst_rows_on(const wc_plan &p, cx<P> *buf, int nlines, int prof_id, double bytes) {
  using R = RowCfg<P, N1>;
  dim3 gr(row_grid((nlines + R::B - 1) / R::B, R::WPB));
  ProfScope ps(p, prof_id, bytes);
  hipLaunchKernelGGL((k_dst_rows<P, N1>), gr, dim3(64 * R::WPB), 0, p.stream, buf, nlines,
                     Tabs<P>::tws(p), Tabs<P>::sin(p));
  return hipGetLastError();
}

// rows per tile of the transposing x1 passes: 8 (128 B per transposed FP64 access) while
// two workgroups stay resident per CU, else 4
template <typename P, int N1> constexpr int default_tr() {
  return blocks_per_cu(TrCfg<P, N1, 8>::BUF) >= 2 ? 8 : 4;
}

// the 2D spatial step through the transposed copy T (N1 >= 128)
template <typename P, int N1, int R>
hipError_t space_tr(const wc_plan &p, int kind, double c) {
  constexpr int M = N1 - 1, NRB = (M + R - 1) / R;
  cx<P> *A = (cx<P> *)p.d_specA;
  cx<P> *T = (cx<P> *)p.d_specT;
  const double bytes = 2.0 * p.nvec * sizeof(P);
  hipError_t e;
  {
    ProfScope ps(p, K_DST_X1_FWD, bytes);
    hipLaunchKernelGGL((k_rows_fwd_t<P, N1, R>), dim3(p.n * NRB), dim3(64 * R), 0, p.stream, A, T,
                       Tabs<P>::tws(p), Tabs<P>::sin(p));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    const int nunits = (p.n / 2) * M, upb = kPairWaves / 2;
    ProfScope ps(p, K_PAIR_MODE, bytes);
    const dim3 grid((nunits + upb - 1) / upb), block(64 * kPairWaves);
    if (kind == 0)
      hipLaunchKernelGGL((k_pair_cols_t<P, N1, 0>), grid, block, 0, p.stream, T, nunits,
                         Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lam(p), Tabs<P>::mu(p),
                         (P)p.tau, (P)p.alpha, (P)c);
    else if (kind == 1)
      hipLaunchKernelGGL((k_pair_cols_t<P, N1, 1>), grid, block, 0, p.stream, T, nunits,
                         Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lam(p), Tabs<P>::mu(p),
                         (P)p.tau, (P)p.alpha, (P)c);
    else
      hipLaunchKernelGGL((k_pair_cols_t<P, N1, 2>), grid, block, 0, p.stream, T, nunits,
                         Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lam(p), Tabs<P>::mu(p),
                         (P)p.tau, (P)p.alpha, (P)c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  ProfScope ps(p, K_DST_X1_INV, bytes);
  hipLaunchKernelGGL((k_rows_inv_t<P, N1, R>), dim3(p.n * NRB), dim3(64 * R), 0, p.stream, T, A,
                     Tabs<P>::tws(p), Tabs<P>::sin(p));
  return hipGetLastError();
}

template <typename P, int N1>
hipError_t run_space(const wc_plan &p) {
  using R = RowCfg<P, N1>;
  constexpr int M = N1 - 1;
  const int kind = p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
  const double c = (1.0 / p.n) * (p.dims == 2 ? (2.0 / N1) * (2.0 / N1) : (2.0 / N1));
  cx<P> *W = (cx<P> *)p.d_specA;
  const double bytes = 2.0 * p.nvec * sizeof(P);
  if (p.dims == 1) {
    const int nunits = p.n / 2;
    dim3 grid(row_grid((nunits + R::UNITS - 1) / R::UNITS, R::WPBU));
    ProfScope ps(p, K_PAIR_MODE, bytes);
    hipLaunchKernelGGL((k_pair_rows<P, N1>), grid, dim3(64 * R::WPBU),
                       0, p.stream,
                       W, nunits, Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lam(p),
                       Tabs<P>::mu(p), kind, (P)p.tau, (P)p.alpha, (P)c);
    return hipGetLastError();
  }
  // x2-pass choice: tx_cols > 0 tiles of that many columns, < 0 the transposed rows with
  // -tx_cols rows per x1 tile (needs the plan's transposed copy, N1 >= 128)
  const int txc = p.tx_cols ? p.tx_cols : (p.d_specT ? -default_tr<P, N1>() : default_tx<P, N1>());
  if constexpr (N1 >= 128) {
    if (txc < 0 && p.d_specT)
      return txc == -4 ? space_tr<P, N1, 4>(p, kind, c) : space_tr<P, N1, 8>(p, kind, c);
  }
  const int nlines = p.n * M;  // n/2 frequencies x 2 block rows x M rows
  dim3 gr(row_grid((nlines + R::B - 1) / R::B, R::WPB));
  hipError_t e = dst_rows_on<P, N1>(p, W, nlines, K_DST_X1_FWD, bytes);
  if (e != hipSuccess) return e;
  switch (txc > 0 ? txc : default_tx<P, N1>()) {
    case 4: e = cols_tx<P, N1, 4>(p, kind, c); break;
    case 16: e = cols_tx<P, N1, 16>(p, kind, c); break;
    default: e = cols_tx<P, N1, 8>(p, kind, c); break;
  }
  if (e != hipSuccess) return e;
  ProfScope ps(p, K_DST_X1_INV, bytes);
  hipLaunchKernelGGL((k_dst_rows<P, N1>), gr, dim3(64 * R::WPB), 0, p.stream,
                     W, nlines, Tabs<P>::tws(p), Tabs<P>::sin(p));
  return hipGetLastError();
}

#define WC_POW2_CASES(X) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

// 2D low-rank GMRES step E v in compact coordinates, with the compact vectors, s0 and the
// cycle's Yhat0 (held in the spectrum array since the cycle began) all in sine coordinates:
// one streaming pass that forms every mode's input, solves it and contracts over
// frequencies, then the chunk sums scaled into the compact output.  With D the unnormalised
// 2D sine transform (D D = (N1/2)^2 I) and Q = (2/N1) D, the output Q (omega |g| D C) is
// omega |g| (N1/2) C.
template <typename P, int N1>
hipError_t lr_step_t(const wc_plan &p, const GenIn &gen, const ContractOut &co) {
  constexpr int M = N1 - 1;
  const int kind = p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
  const double c = (1.0 / p.n) * (2.0 / N1) * (2.0 / N1);
  const double half = 0.5 * N1;
  hipError_t e;
  {
    ProfScope ps(p, K_PAIR_CONTRACT,
                 p.nvec * (double)sizeof(P) + 32.0 * p.m + 16.0 * kColChunks * p.m);
    hipLaunchKernelGGL(k_lr_contract<P>, dim3((p.m + kThreads - 1) / kThreads, kColChunks),
                       dim3(kThreads), 0, p.stream, (const cx<P> *)p.d_specA, gen, half,
                       (const cx<double> *)p.d_lr_rank, Tabs<P>::lam(p), Tabs<P>::mu(p), kind,
                       (P)p.tau, (P)p.alpha, (P)c, (const cx<double> *)co.rho, p.n / 2, M,
                       co.part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  ProfScope ps(p, K_CONTRACT, 16.0 * kColChunks * p.m + 16.0 * p.m);
  hipLaunchKernelGGL(k_lr_hat_out, dim3((p.m + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     p.stream, co.part, co.hat, p.m, co.gn_omega * half, co.rn_omega * half);
  return hipGetLastError();
}

// s0 (two m-point fields, [x2][x1]) into orthonormal sine coordinates, in place, through
// the m complex of d_lr_a: x1 transform of s0_1 + i s0_2, then the x2 transform scaled by
// 2/N1 and split back
template <int N1> hipError_t lr_sine_s0_t(const wc_plan &p) {
  constexpr int M = N1 - 1;
  cx<double> *t = (cx<double> *)p.d_lr_a;
  hipError_t e = launch_rows_fn<double, N1>(p, M, PairSrc{p.d_lr_s0, p.m, M},
                                            StoreA<double>{t, M}, K_LR_SETUP, 32.0 * p.m);
  if (e != hipSuccess) return e;
  return launch_rows_fn<double, N1>(p, M, ColLine<double>{t, M},
                                    PairStore{p.d_lr_s0, p.m, M, 2.0 / N1}, K_LR_SETUP,
                                    32.0 * p.m);
}

// the cycle's update (2D low-rank GMRES): the x2 pass from Yhat0, then the inverse x1
// transform; the inverse time transform follows in pc_apply_t
template <typename P, int N1>
hipError_t lr_update_t(const wc_plan &p, const GenIn &gen) {
  using R = RowCfg<P, N1>;
  constexpr int M = N1 - 1, TX = default_tx<P, N1>();
  if constexpr (!ColCfg<P, N1, TX>::FITS) {
    return hipErrorInvalidValue;
  } else {
    const int kind = p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
    const double c = (1.0 / p.n) * (2.0 / N1) * (2.0 / N1);
    cx<P> *W = (cx<P> *)p.d_specA;
    cx<double> *A = (cx<double> *)p.d_lr_a;
    const int ncx = (N1 - 2 + TX) / TX;
    hipError_t e;
    {
      ProfScope ps(p, K_LR_SETUP, 48.0 * p.m);
      hipLaunchKernelGGL(k_lr_ahat, dim3((p.m + kThreads - 1) / kThreads), dim3(kThreads), 0,
                         p.stream, gen, 0.5 * N1, p.m, A);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
      ProfScope ps(p, K_PAIR_MODE, 2.0 * p.nvec * sizeof(P) + 16.0 * p.m);
      hipLaunchKernelGGL((k_cols_update<P, N1, TX>), dim3(ncx * (p.n / 2)),
                         dim3(ColCfg<P, N1, TX>::NT), 0, p.stream, W, Tabs<P>::tws(p),
                         Tabs<P>::sin(p), Tabs<P>::lam(p), Tabs<P>::mu(p), kind, (P)p.tau,
                         (P)p.alpha, (P)c, gen.hat, gen.sqn0, (const cx<double> *)A,
                         (const cx<double> *)p.d_lr_rank);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int nlines = p.n * M;
    dim3 gr(row_grid((nlines + R::B - 1) / R::B, R::WPB));
    ProfScope ps(p, K_DST_X1_INV, 2.0 * p.nvec * sizeof(P));
    hipLaunchKernelGGL((k_dst_rows<P, N1>), gr, dim3(64 * R::WPB), 0, p.stream, W, nlines,
                       Tabs<P>::tws(p), Tabs<P>::sin(p));
    return hipGetLastError();
  }
}

// step 2 in sine coordinates: the per-mode operation of every (frequency, mode)
template <typename P>
__global__ __launch_bounds__(kThreads) void k_mode_pointwise(cx<P> *__restrict__ W, int nq, int m,
                                                            int M, int dims,
                                                            const cx<P> *__restrict__ lam,
                                                            const P *__restrict__ mu, int kind,
                                                            P tau, P alpha, P cnorm) {
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (size_t)nq * m) return;
  const int q = (int)(idx / (size_t)m), s = (int)(idx - (size_t)q * m);
  const P musum = dims == 1 ? mu[s] : mu[s % M] + mu[s / M];
  cx<P> *w0 = W + (size_t)(2 * q) * m + s;
  cx<P> a = *w0, b = w0[m];
  mode_op<P>(a, b, lam[q], musum, kind, tau, alpha, cnorm);
  *w0 = a;
  w0[m] = b;
}

// ---- dense spatial steps (Neumann data: the cosine basis is not orthogonal and M is any
// size, so the steps are the dense products with C^{-1} and C) -----------------------
// Y(j, c) = sum_k A[j][k] X(k, c) for every slab of the spectral array.  ROWS: along x1,
// X(k, c) = entry k of line c (all lines of all slabs, one batch); else along x2, X(k, c)
// = row k, column c of slab blockIdx.z (M x M).  64 x 64 output tiles, k in chunks of 16
// through LDS; thread t owns the 4 x 4 outputs (j0 + tj + 16 a, c0 + tc + 16 b), with
// the output index that is contiguous in memory fastest across the lanes.
constexpr int kDenseT = 64, kDenseK = 16;
template <typename P, bool ROWS>
__global__ __launch_bounds__(256) void k_dense_apply(const cx<P> *__restrict__ X,
                                                     cx<P> *__restrict__ Y,
                                                     const P *__restrict__ A, int N, int C) {
  __shared__ P As[kDenseK][kDenseT + 1];
  __shared__ cx<P> Xs[kDenseK][kDenseT + 1];
  const int tid = threadIdx.x;
  const int tj = ROWS ? tid % 16 : tid / 16, tc = ROWS ? tid / 16 : tid % 16;
  const int j0 = blockIdx.y * kDenseT, c0 = blockIdx.x * kDenseT;
  const size_t slab = ROWS ? 0 : (size_t)blockIdx.z * N * N;
  const cx<P> *Xb = X + slab;
  cx<P> *Yb = Y + slab;
  cx<P> acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = cx<P>{(P)0, (P)0};
  for (int k0 = 0; k0 < N; k0 += kDenseK) {
    for (int e = tid; e < kDenseK * kDenseT; e += 256) {  // A rows are contiguous in k
      const int kk = e % kDenseK, jj = e / kDenseK, j = j0 + jj, k = k0 + kk;
      As[kk][jj] = (j < N && k < N) ? A[(size_t)j * N + k] : (P)0;
    }
    for (int e = tid; e < kDenseK * kDenseT; e += 256) {  // along the contiguous index
      const int kk = ROWS ? e % kDenseK : e / kDenseT, cc = ROWS ? e / kDenseK : e % kDenseT;
      const int k = k0 + kk, c = c0 + cc;
      cx<P> v{(P)0, (P)0};
      if (k < N && c < C) v = ROWS ? Xb[(size_t)c * N + k] : Xb[(size_t)k * N + c];
      Xs[kk][cc] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kDenseK; ++kk) {
      P a[4];
      cx<P> x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[kk][tj + 16 * i];
        x[i] = Xs[kk][tc + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[i][b].x += a[i] * x[b].x;
          acc[i][b].y += a[i] * x[b].y;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + tj + 16 * i, c = c0 + tc + 16 * b;
      if (j < N && c < C) {
        if (ROWS) Yb[(size_t)c * N + j] = acc[i][b];
        else Yb[(size_t)j * N + c] = acc[i][b];
      }
    }
}

// FP64 form of k_dense_apply on the matrix cores: the real and imaginary parts of X are
// two real products with the same matrix, each built from 16 x 16 x 4 FP64 MFMA steps.
// Operand layout of that instruction (checked on the device): lane l supplies
// A[l % 16][l / 16] of the 16 x 4 left operand and B[l / 16][l % 16] of the 4 x 16 right
// one, and holds D[4 i + l / 16][l % 16], i < 4, of the 16 x 16 result.  Each of the 4
// waves owns a 32 x 32 quarter of the 64 x 64 tile.  COLS: D = A X (rows j, columns c:
// consecutive lanes store consecutive columns of a slab row); ROWS: D = X^T A^T (rows c,
// columns j: consecutive lanes store consecutive entries of a line).
typedef double dx4 __attribute__((ext_vector_type(4)));
template <bool ROWS, int KC = 32>
__global__ __launch_bounds__(256) void k_dense_mfma(const cx<double> *__restrict__ X,
                                                    cx<double> *__restrict__ Y,
                                                    const double *__restrict__ A, int N, int C) {
  constexpr int PER = KC * kDenseT / 256;  // staged elements per thread and chunk
  __shared__ double As[KC][kDenseT + 1];
  __shared__ cx<double> Xs[KC][kDenseT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wj = (wv & 1) * 32, wc = (wv >> 1) * 32;  // the wave's quarter of the tile
  const int lr = lane % 16, lk = lane / 16;
  const int j0 = blockIdx.y * kDenseT, c0 = blockIdx.x * kDenseT;
  const size_t slab = ROWS ? 0 : (size_t)blockIdx.z * N * N;
  const cx<double> *Xb = X + slab;
  cx<double> *Yb = Y + slab;
  dx4 re[2][2], im[2][2];  // [j block][c block]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = dx4{0.0, 0.0, 0.0, 0.0};
  // chunk k0 of both operands into registers (A rows are contiguous in k; X along its
  // contiguous index); the next chunk's loads are issued before the current one's products
  double ra[PER];
  cx<double> rx[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      const int kk = e % KC, jj = e / KC, j = j0 + jj, k = k0 + kk;
      ra[u] = (j < N && k < N) ? A[(size_t)j * N + k] : 0.0;
      const int xk = ROWS ? e % KC : e / kDenseT, xc = ROWS ? e / KC : e % kDenseT;
      const int k2 = k0 + xk, c = c0 + xc;
      rx[u] = cx<double>{0.0, 0.0};
      if (k2 < N && c < C) rx[u] = ROWS ? Xb[(size_t)c * N + k2] : Xb[(size_t)k2 * N + c];
    }
  };
  load(0);
  for (int k0 = 0; k0 < N; k0 += KC) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      As[e % KC][e / KC] = ra[u];
      const int xk = ROWS ? e % KC : e / kDenseT, xc = ROWS ? e / KC : e % kDenseT;
      Xs[xk][xc] = rx[u];
    }
    __syncthreads();
    if (k0 + KC < N) load(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kr = ks + lk;
      double am[2];
      cx<double> xv[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        am[b] = As[kr][wj + 16 * b + lr];
        xv[b] = Xs[kr][wc + 16 * b + lr];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (ROWS) {  // left operand X^T (row c, column k), right A^T (row k, column j)
            re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[b].x, am[a], re[a][b], 0, 0, 0);
            im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[b].y, am[a], im[a][b], 0, 0, 0);
          } else {     // left operand A (row j, column k), right X (row k, column c)
            re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[a], xv[b].x, re[a][b], 0, 0, 0);
            im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[a], xv[b].y, im[a][b], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // result row 4 i + lk, column lr of the (a, b) block
        const int j = ROWS ? j0 + wj + 16 * a + lr : j0 + wj + 16 * a + 4 * i + lk;
        const int c = ROWS ? c0 + wc + 16 * b + 4 * i + lk : c0 + wc + 16 * b + lr;
        if (j < N && c < C) {
          const cx<double> v{re[a][b][i], im[a][b][i]};
          if (ROWS) Yb[(size_t)c * N + j] = v;
          else Yb[(size_t)j * N + c] = v;
        }
      }
}

// ---- general path: sizes or zeta outside the FFT path ------------------------------
// Time step as a dense product over all n frequencies, both block rows (blockIdx.z = h):
// FWD  G[h][l][s] = sum_k Phi[l][k] v[h][k][s]       (v real FP64, G complex P)
// !FWD w[h][k][s] = Re sum_l Phiinv[k][l] G[h][l][s]  (real FP64 out)
// with s = 0..m-1 contiguous: 64 x 64 output tiles of (l or k) x s, 16-deep chunks.
template <typename P, bool FWD>
__global__ __launch_bounds__(256) void k_dense_time(const void *__restrict__ Xv,
                                                    void *__restrict__ Yv,
                                                    const cx<P> *__restrict__ A, int n, int m) {
  using XT = typename std::conditional<FWD, double, cx<P>>::type;
  using YT = typename std::conditional<FWD, cx<P>, double>::type;
  using AccT = typename std::conditional<FWD, cx<P>, P>::type;
  __shared__ cx<P> As[kDenseK][kDenseT + 1];
  __shared__ XT Xs[kDenseK][kDenseT + 1];
  const int tid = threadIdx.x, tj = tid / 16, tc = tid % 16;
  const int j0 = blockIdx.y * kDenseT, c0 = blockIdx.x * kDenseT;
  const XT *X = (const XT *)Xv + (size_t)blockIdx.z * n * m;
  YT *Y = (YT *)Yv + (size_t)blockIdx.z * n * m;
  AccT acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = AccT{};
  for (int k0 = 0; k0 < n; k0 += kDenseK) {
    for (int e = tid; e < kDenseK * kDenseT; e += 256) {  // A rows contiguous in k
      const int kk = e % kDenseK, jj = e / kDenseK, j = j0 + jj, k = k0 + kk;
      As[kk][jj] = (j < n && k < n) ? A[(size_t)j * n + k] : cx<P>{(P)0, (P)0};
    }
    for (int e = tid; e < kDenseK * kDenseT; e += 256) {  // X rows contiguous in s
      const int kk = e / kDenseT, cc = e % kDenseT, k = k0 + kk, c = c0 + cc;
      Xs[kk][cc] = (k < n && c < m) ? X[(size_t)k * m + c] : XT{};
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kDenseK; ++kk) {
      cx<P> a[4];
      XT x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[kk][tj + 16 * i];
        x[i] = Xs[kk][tc + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if constexpr (FWD) {  // complex times real data
            acc[i][b].x += a[i].x * (P)x[b];
            acc[i][b].y += a[i].y * (P)x[b];
          } else {  // the real part of complex times complex
            acc[i][b] += a[i].x * x[b].x - a[i].y * x[b].y;
          }
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + tj + 16 * i, c = c0 + tc + 16 * b;
      if (j < n && c < m) {
        if constexpr (FWD) Y[(size_t)j * m + c] = acc[i][b];
        else Y[(size_t)j * m + c] = (double)acc[i][b];
      }
    }
}

// FP64 form of k_dense_time on the matrix cores (operand layout as in k_dense_mfma):
// FWD: Re G and Im G are Re Phi v and Im Phi v; !FWD: w = Re Phiinv Re G - Im Phiinv Im G.
// Rows of the 64 x 64 tile are frequencies l (FWD) or time levels k (!FWD), columns are
// spatial points s, so consecutive lanes store consecutive s.
template <bool FWD, int KC = 32>
__global__ __launch_bounds__(256) void k_dense_time_mfma(const void *__restrict__ Xv,
                                                         void *__restrict__ Yv,
                                                         const cx<double> *__restrict__ A, int n,
                                                         int m) {
  using XT = typename std::conditional<FWD, double, cx<double>>::type;
  constexpr int PER = KC * kDenseT / 256;  // staged elements per thread and chunk
  __shared__ cx<double> As[KC][kDenseT + 1];
  __shared__ XT Xs[KC][kDenseT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wj = (wv & 1) * 32, wc = (wv >> 1) * 32;
  const int lr = lane % 16, lk = lane / 16;
  const int j0 = blockIdx.y * kDenseT, c0 = blockIdx.x * kDenseT;
  const XT *X = (const XT *)Xv + (size_t)blockIdx.z * n * m;
  dx4 re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = dx4{0.0, 0.0, 0.0, 0.0};
  // chunk k0 into registers (A rows contiguous in k, X rows contiguous in s); the next
  // chunk's loads are issued before the current one's products
  cx<double> ra[PER];
  XT rx[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      const int kk = e % KC, jj = e / KC, j = j0 + jj, k = k0 + kk;
      ra[u] = (j < n && k < n) ? A[(size_t)j * n + k] : cx<double>{0.0, 0.0};
      const int xk = e / kDenseT, xc = e % kDenseT, k2 = k0 + xk, c = c0 + xc;
      rx[u] = (k2 < n && c < m) ? X[(size_t)k2 * m + c] : XT{};
    }
  };
  load(0);
  for (int k0 = 0; k0 < n; k0 += KC) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      As[e % KC][e / KC] = ra[u];
      Xs[e / kDenseT][e % kDenseT] = rx[u];
    }
    __syncthreads();
    if (k0 + KC < n) load(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kr = ks + lk;
      cx<double> am[2];
      XT xv[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        am[b] = As[kr][wj + 16 * b + lr];
        xv[b] = Xs[kr][wc + 16 * b + lr];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if constexpr (FWD) {
            re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[a].x, xv[b], re[a][b], 0, 0, 0);
            im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[a].y, xv[b], im[a][b], 0, 0, 0);
          } else {
            re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[a].x, xv[b].x, re[a][b], 0, 0, 0);
            re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-am[a].y, xv[b].y, re[a][b], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = j0 + wj + 16 * a + 4 * i + lk, c = c0 + wc + 16 * b + lr;
        if (j < n && c < m) {
          const size_t o = (size_t)blockIdx.z * n * m + (size_t)j * m + c;
          if constexpr (FWD) ((cx<double> *)Yv)[o] = cx<double>{re[a][b][i], im[a][b][i]};
          else ((double *)Yv)[o] = re[a][b][i];
        }
      }
}

// step 2 of the general path: the per-mode operation of frequency l and mode s couples
// G[0][l][s] and G[1][l][s] (lambda_l of the full table; the dense steps are normalised)
template <typename P>
__global__ __launch_bounds__(kThreads) void k_mode_full(cx<P> *__restrict__ G, int n, int m, int M,
                                                       int dims, const cx<P> *__restrict__ lam,
                                                       const P *__restrict__ mu, int kind, P tau,
                                                       P alpha) {
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const size_t nm = (size_t)n * m;
  if (idx >= nm) return;
  const int l = (int)(idx / (size_t)m), s = (int)(idx - (size_t)l * m);
  const P musum = dims == 1 ? mu[s] : mu[s % M] + mu[s / M];
  cx<P> a = G[idx], b = G[nm + idx];
  mode_op<P>(a, b, lam[l], musum, kind, tau, alpha, (P)1);
  G[idx] = a;
  G[nm + idx] = b;
}

namespace {
// the spatial step of the dense paths on nslab slabs of m complex (lines of M along x1):
// into the basis (second table matrix along x1, then x2), op(W), back (first matrix along
// x2, then x1); A -> A through B
template <typename P, typename Op>
hipError_t dense_space(const wc_plan &p, cx<P> *A, cx<P> *B, int nslab, Op op) {
  const int M = p.M;
  const P *Cf = Tabs<P>::cos(p), *Ci = Cf + (size_t)M * M;
  const int lines = p.dims == 2 ? nslab * M : nslab;
  const int gj = (M + kDenseT - 1) / kDenseT;
  const dim3 grows((lines + kDenseT - 1) / kDenseT, gj), gcols(gj, gj, nslab);
  const double bytes = 2.0 * nslab * (double)p.m * sizeof(cx<P>);
  hipError_t e;
  // FP64 on the matrix cores, FP32 on the vector ALUs
  auto rows = [&](const cx<P> *in, cx<P> *out, const P *mat, int id) {
    ProfScope ps(p, id, bytes);
    if constexpr (std::is_same<P, double>::value)
      hipLaunchKernelGGL((k_dense_mfma<true>), grows, dim3(256), 0, p.stream, in, out, mat, M,
                         lines);
    else
      hipLaunchKernelGGL((k_dense_apply<P, true>), grows, dim3(256), 0, p.stream, in, out, mat, M,
                         lines);
    return hipGetLastError();
  };
  auto cols = [&](const cx<P> *in, cx<P> *out, const P *mat, int id) {
    ProfScope ps(p, id, bytes);
    if constexpr (std::is_same<P, double>::value)
      hipLaunchKernelGGL((k_dense_mfma<false>), gcols, dim3(256), 0, p.stream, in, out, mat, M,
                         M);
    else
      hipLaunchKernelGGL((k_dense_apply<P, false>), gcols, dim3(256), 0, p.stream, in, out, mat,
                         M, M);
    return hipGetLastError();
  };
  if ((e = rows(A, B, Ci, K_DST_X1_FWD)) != hipSuccess) return e;
  cx<P> *W = B;
  if (p.dims == 2) {
    if ((e = cols(B, A, Ci, K_DST_X1_FWD)) != hipSuccess) return e;
    W = A;
  }
  if ((e = op(W)) != hipSuccess) return e;
  if (p.dims == 2 && (e = cols(A, B, Cf, K_DST_X1_INV)) != hipSuccess) return e;
  return rows(B, A, Cf, K_DST_X1_INV);
}

// ---- any zeta at power-of-two sizes: the full time spectrum --------------------------
// For omega = e^{i zeta} with zeta != pi each block row's twiddled sequence e^{i zeta k/n} v_k
// is complex, so its spectrum has no conjugate symmetry: all n frequencies are kept, an
// n-point FFT per block row and column (eqn:decompositiob_S12 as corrected).  G holds the
// spectrum as [l][half][x2][x1] (slab 2l + h, twice the half-spectrum array), so the
// transposed sine passes of the FFT path run on it unchanged over 2n slabs, with lambda_l of
// every frequency; the inverse takes the real part (the preconditioner of the real system).
template <typename P, int N, int TS> struct FullCfg {
  static constexpr int WAVES = TS < 4 ? TS : 4;
  static constexpr int NT = 64 * WAVES;
  static constexpr int CXB = 2 * (int)sizeof(P);
  static constexpr int PS = 4;
  static constexpr int PN = padded<PS>(N);
  static constexpr int S = TS + 1;
  static constexpr int TILE = PN * S * CXB;  // twiddles are read from global memory
};
// the widest tile (at most 16 columns) that keeps two workgroups resident per CU
template <typename P, int N> constexpr int full_ts() {
  if constexpr (blocks_per_cu(FullCfg<P, N, 16>::TILE) >= 2) return 16;
  else if constexpr (blocks_per_cu(FullCfg<P, N, 8>::TILE) >= 2) return 8;
  else if constexpr (blocks_per_cu(FullCfg<P, N, 4>::TILE) >= 2) return 4;
  else return 2;
}

// forward: tile (h, TS columns) of block row h of v -> G[l][h][s], l = 0..N-1
template <typename P, int N, int TS>
__global__ __launch_bounds__((FullCfg<P, N, TS>::NT)) void k_tfft_full_fwd(
    const double *__restrict__ v, cx<P> *__restrict__ G, const cx<double> *__restrict__ dtw,
    const cx<P> *__restrict__ twt, int m, int ntile) {
  using C = FullCfg<P, N, TS>;
  constexpr int S = C::S, PS = C::PS, NT = C::NT, CPW = TS / C::WAVES;
  constexpr int LIT = (N * TS + NT - 1) / NT;
  __shared__ cx<P> buf[C::PN * S];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int h = t / ntile, s0 = (t % ntile) * TS;
  const double *src = v + (size_t)h * N * m;
  double ra[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {  // every load issued before any is consumed
    const int idx = tid + it * NT, k = idx / TS, gs = s0 + idx % TS;
    ra[it] = 0.0;
    if ((N * TS % NT == 0 || idx < N * TS) && gs < m) ra[it] = src[(size_t)k * m + gs];
  }
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (N * TS % NT == 0 || idx < N * TS) {
      const int k = idx / TS, s = idx % TS;
      const cx<double> d = dtw[k];  // e^{i zeta k/n}
      buf[pk<PS>(k) * S + s] = cx<P>{(P)(ra[it] * d.x), (P)(ra[it] * d.y)};
    }
  }
  __syncthreads();
  wfft<P, N, 1, CPW, S, PS, false, true>(buf + wv * CPW, twt, lane);
  __syncthreads();
  for (int idx = tid; idx < N * TS; idx += NT) {
    const int l = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs < m) G[((size_t)l * 2 + h) * m + gs] = buf[pk<PS>(l) * S + s];
  }
}

// inverse: G[l][h][s] -> Re(e^{-i zeta k/n} sum_l e^{2 pi i k l/n} G_l), block row h of w (the
// 1/n sits in the per-mode scale)
template <typename P, int N, int TS>
__global__ __launch_bounds__((FullCfg<P, N, TS>::NT)) void k_tfft_full_inv(
    const cx<P> *__restrict__ G, double *__restrict__ w, const cx<double> *__restrict__ dtw,
    const cx<P> *__restrict__ twt, int m, int ntile) {
  using C = FullCfg<P, N, TS>;
  constexpr int S = C::S, PS = C::PS, NT = C::NT, CPW = TS / C::WAVES;
  constexpr int LIT = (N * TS + NT - 1) / NT;
  __shared__ cx<P> buf[C::PN * S];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int h = t / ntile, s0 = (t % ntile) * TS;
  cx<P> ya[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT, l = idx / TS, gs = s0 + idx % TS;
    ya[it] = cx<P>{(P)0, (P)0};
    if ((N * TS % NT == 0 || idx < N * TS) && gs < m) ya[it] = G[((size_t)l * 2 + h) * m + gs];
  }
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (N * TS % NT == 0 || idx < N * TS) buf[pk<PS>(idx / TS) * S + idx % TS] = ya[it];
  }
  __syncthreads();
  wfft<P, N, 1, CPW, S, PS, true, true>(buf + wv * CPW, twt, lane);
  __syncthreads();
  double *o = w + (size_t)h * N * m;
  for (int idx = tid; idx < N * TS; idx += NT) {
    const int k = idx / TS, s = idx % TS, gs = s0 + s;
    if (gs >= m) continue;
    const cx<P> z = buf[pk<PS>(k) * S + s];
    const cx<double> d = dtw[k];  // Re(z conj(d))
    o[(size_t)k * m + gs] = (double)z.x * d.x + (double)z.y * d.y;
  }
}

template <typename P, int N, bool INV>
hipError_t full_time(const wc_plan &p, const double *v, double *w) {
  constexpr int TS = full_ts<P, N>();
  using C = FullCfg<P, N, TS>;
  const int ntile = (p.m + TS - 1) / TS;
  const double bytes = 8.0 * p.nvec + 2.0 * p.n * (double)p.m * sizeof(cx<P>);
  cx<P> *G = (cx<P> *)p.d_specA;
  if constexpr (INV) {
    ProfScope ps(p, K_TFFT_INV, bytes);
    hipLaunchKernelGGL((k_tfft_full_inv<P, N, TS>), dim3(2 * ntile), dim3(C::NT), 0, p.stream, G,
                       w, (const cx<double> *)p.d_dtw, Tabs<P>::twt(p), p.m, ntile);
  } else {
    ProfScope ps(p, K_TFFT_FWD, bytes);
    hipLaunchKernelGGL((k_tfft_full_fwd<P, N, TS>), dim3(2 * ntile), dim3(C::NT), 0, p.stream,
                       v, G, (const cx<double> *)p.d_dtw, Tabs<P>::twt(p), p.m, ntile);
  }
  return hipGetLastError();
}

// the transposed sine passes and the per-mode solves over the 2n slabs of G (through the
// transposed copy d_specT, 2n slabs of M rows of N1)
template <typename P, int N1>
hipError_t full_space(const wc_plan &p, int kind, double c) {
  constexpr int M = N1 - 1, R = default_tr<P, N1>(), NRB = (M + R - 1) / R;
  cx<P> *A = (cx<P> *)p.d_specA;
  cx<P> *T = (cx<P> *)p.d_specT;
  const int nslab = 2 * p.n;
  const double bytes = 2.0 * nslab * (double)p.m * sizeof(cx<P>);
  hipError_t e;
  {
    ProfScope ps(p, K_DST_X1_FWD, bytes);
    hipLaunchKernelGGL((k_rows_fwd_t<P, N1, R>), dim3(nslab * NRB), dim3(64 * R), 0, p.stream, A,
                       T, Tabs<P>::tws(p), Tabs<P>::sin(p));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    const int nunits = p.n * M, upb = kPairWaves / 2;
    const dim3 grid((nunits + upb - 1) / upb), block(64 * kPairWaves);
    ProfScope ps(p, K_PAIR_MODE, bytes);
    if (kind == 0)
      hipLaunchKernelGGL((k_pair_cols_t<P, N1, 0>), grid, block, 0, p.stream, T, nunits,
                         Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lamf(p), Tabs<P>::mu(p),
                         (P)p.tau, (P)p.alpha, (P)c);
    else if (kind == 1)
      hipLaunchKernelGGL((k_pair_cols_t<P, N1, 1>), grid, block, 0, p.stream, T, nunits,
                         Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lamf(p), Tabs<P>::mu(p),
                         (P)p.tau, (P)p.alpha, (P)c);
    else
      hipLaunchKernelGGL((k_pair_cols_t<P, N1, 2>), grid, block, 0, p.stream, T, nunits,
                         Tabs<P>::tws(p), Tabs<P>::sin(p), Tabs<P>::lamf(p), Tabs<P>::mu(p),
                         (P)p.tau, (P)p.alpha, (P)c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  ProfScope ps(p, K_DST_X1_INV, bytes);
  hipLaunchKernelGGL((k_rows_inv_t<P, N1, R>), dim3(nslab * NRB), dim3(64 * R), 0, p.stream, T, A,
                     Tabs<P>::tws(p), Tabs<P>::sin(p));
  return hipGetLastError();
}

bool pow2_between(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

// the full-spectrum FFT form applies: 2D Dirichlet finite differences, n a power of two in
// [4, 1024], M + 1 a power of two in [128, 1024] (the transposed sine passes)
bool full_fft_ok(const wc_plan &p) {
  return p.dims == 2 && !p.neumann && !p.fem && !p.var_coeff && p.d_specT &&
         pow2_between(p.n, 4, 1024) && pow2_between(p.M + 1, 128, 1024);
}

template <typename P>
hipError_t pc_apply_full(const wc_plan &p, const double *v, double *w, const double *dotv,
                         int *nparts) {
  hipError_t e = hipErrorInvalidValue;
  switch (p.n) {
#define CASE_N(NN) case NN: e = full_time<P, NN, false>(p, v, nullptr); break;
    WC_POW2_CASES(CASE_N)
#undef CASE_N
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int kind = p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
  const double c = (1.0 / p.n) * (2.0 / (p.M + 1)) * (2.0 / (p.M + 1));
  switch (p.M + 1) {
    case 128: e = full_space<P, 128>(p, kind, c); break;
    case 256: e = full_space<P, 256>(p, kind, c); break;
    case 512: e = full_space<P, 512>(p, kind, c); break;
    case 1024: e = full_space<P, 1024>(p, kind, c); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (p.n) {
#define CASE_N(NN) case NN: e = full_time<P, NN, true>(p, nullptr, w); break;
    WC_POW2_CASES(CASE_N)
#undef CASE_N
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  *nparts = 0;
  if (dotv) return launch_dot_partials(p, w, dotv, nparts);
  return hipSuccess;
}

// P^{-1} v on the general path: dense time transform of both block rows over all n
// frequencies (any n, any zeta), dense spatial steps, per-mode solves, the inverse
// steps, the real part (the preconditioner of a real system)
template <typename P>
hipError_t pc_apply_general(const wc_plan &p, const double *v, double *w, const double *dotv,
                            int *nparts) {
  if (full_fft_ok(p)) return pc_apply_full<P>(p, v, w, dotv, nparts);
  cx<P> *G = (cx<P> *)p.d_specA, *B = (cx<P> *)p.d_specB;
  const int n = p.n, m = p.m;
  const dim3 gt((m + kDenseT - 1) / kDenseT, (n + kDenseT - 1) / kDenseT, 2);
  const double vbytes = 8.0 * p.nvec, gbytes = 2.0 * n * (double)m * sizeof(cx<P>);
  hipError_t e;
  {
    ProfScope ps(p, K_TFFT_FWD, vbytes + gbytes);
    if constexpr (std::is_same<P, double>::value)
      hipLaunchKernelGGL((k_dense_time_mfma<true>), gt, dim3(256), 0, p.stream, (const void *)v,
                         (void *)G, Tabs<P>::phi(p), n, m);
    else
      hipLaunchKernelGGL((k_dense_time<P, true>), gt, dim3(256), 0, p.stream, (const void *)v,
                         (void *)G, Tabs<P>::phi(p), n, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int kind = p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
  e = dense_space<P>(p, G, B, 2 * n, [&](cx<P> *W) {
    const size_t cnt = (size_t)n * m;
    ProfScope ps(p, K_PAIR_MODE, 2.0 * gbytes);
    hipLaunchKernelGGL((k_mode_full<P>), dim3((unsigned)((cnt + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, p.stream, W, n, m, p.M, p.dims, Tabs<P>::lamf(p),
                       Tabs<P>::mu(p), kind, (P)p.tau, (P)p.alpha);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  {
    ProfScope ps(p, K_TFFT_INV, vbytes + gbytes);
    if constexpr (std::is_same<P, double>::value)
      hipLaunchKernelGGL((k_dense_time_mfma<false>), gt, dim3(256), 0, p.stream,
                         (const void *)G, (void *)w, Tabs<P>::phi(p) + (size_t)n * n, n, m);
    else
      hipLaunchKernelGGL((k_dense_time<P, false>), gt, dim3(256), 0, p.stream, (const void *)G,
                         (void *)w, Tabs<P>::phi(p) + (size_t)n * n, n, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  *nparts = 0;
  if (dotv) return launch_dot_partials(p, w, dotv, nparts);
  return hipSuccess;
}

// Neumann data on the FFT time path, step 2 between the time transforms: into the cosine
// basis, the per-mode solves of the n/2 kept frequencies, back (d_specA via d_specB)
template <typename P> hipError_t neumann_space(const wc_plan &p) {
  return dense_space<P>(p, (cx<P> *)p.d_specA, (cx<P> *)p.d_specB, p.n, [&](cx<P> *W) {
    const size_t cnt = (size_t)(p.n / 2) * p.m;
    ProfScope ps(p, K_PAIR_MODE, 2.0 * p.nvec * sizeof(P));
    hipLaunchKernelGGL((k_mode_pointwise<P>), dim3((unsigned)((cnt + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, p.stream, W, p.n / 2, p.m, p.M, p.dims, Tabs<P>::lam(p),
                       Tabs<P>::mu(p), 0, (P)p.tau, (P)p.alpha, (P)(1.0 / p.n));
    return hipGetLastError();
  });
}
}  // namespace

template <typename P>
hipError_t pc_apply_t(const wc_plan &p, const double *v, double *w, const double *dotv,
                      int *nparts, const GenIn *gen, const ContractOut *co) {
  hipError_t e = hipErrorInvalidValue;
  if (p.general) {
    if (gen || co) return hipErrorInvalidValue;  // the low-rank form runs on the FFT path
    return pc_apply_general<P>(p, v, w, dotv, nparts);
  }
  // 2D low-rank GMRES (Arnoldi steps and the cycle's update): the spectrum comes from the
  // cycle's transformed r0, in the first sine pass
  const bool hoist = gen && p.lr_2d;
  if (hoist && co) {
    *nparts = 0;
    switch (p.N1) {
#define CASE_S(NN) case NN: return lr_step_t<P, NN>(p, *gen, *co);
      WC_POW2_CASES(CASE_S)
#undef CASE_S
      default: return hipErrorInvalidValue;
    }
  }
  if (hoist) {  // the cycle's update: the spectrum of its input is generated from Yhat0
    switch (p.N1) {
#define CASE_S(NN) case NN: e = lr_update_t<P, NN>(p, *gen); break;
      WC_POW2_CASES(CASE_S)
#undef CASE_S
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (p.n) {
#define CASE_N(NN) case NN: e = run_tfft_fwd<P, NN>(p, v, gen); break;
      WC_POW2_CASES(CASE_N)
#undef CASE_N
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (p.neumann) {
      e = neumann_space<P>(p);
    } else if (p.fem) {  // sine coordinates: step 2 is pointwise
      const int kind = p.opts.method == WC_GMRES_PS ? 0 : (p.opts.method == WC_MINRES_ABS_PS ? 1 : 2);
      const size_t cnt = (size_t)(p.n / 2) * p.m;
      ProfScope ps(p, K_PAIR_MODE, 2.0 * p.nvec * sizeof(P));
      hipLaunchKernelGGL((k_mode_pointwise<P>), dim3((unsigned)((cnt + kThreads - 1) / kThreads)),
                         dim3(kThreads), 0, p.stream, (cx<P> *)p.d_specA, p.n / 2, p.m, p.M,
                         p.dims, Tabs<P>::lam(p), Tabs<P>::mu(p), kind, (P)p.tau, (P)p.alpha,
                         (P)(1.0 / p.n));
      e = hipGetLastError();
    } else if (p.var_coeff) {
      e = mg_space_apply(p);
    } else {
      switch (p.N1) {
#define CASE_S(NN) case NN: e = run_space<P, NN>(p); break;
        WC_POW2_CASES(CASE_S)
#undef CASE_S
        default: return hipErrorInvalidValue;
      }
    }
  }
  if (e != hipSuccess) return e;
  if (co) {  // 1D low-rank GMRES: contract over time on the spectrum (2D: lr_step_t)
    if (p.dims != 1) return hipErrorInvalidValue;
    if constexpr (!std::is_same<P, double>::value) {
      return hipErrorInvalidValue;  // the 1D low-rank form is FP64 only
    } else {
      const int nq = p.n / 2;
      {
        ProfScope ps(p, K_CONTRACT, (double)p.n * p.m * sizeof(cx<double>) +
                                        16.0 * kContractChunks * p.m);
        hipLaunchKernelGGL(k_contract_freq, dim3((p.m + kThreads - 1) / kThreads, kContractChunks),
                           dim3(kThreads), 0, p.stream, (const cx<double> *)p.d_specA, *co, p.m,
                           nq);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      *nparts = 0;
      ProfScope ps(p, K_CONTRACT, 16.0 * kContractChunks * p.m + 16.0 * p.m);
      hipLaunchKernelGGL(k_contract_final, dim3((p.m + kThreads - 1) / kThreads), dim3(kThreads),
                         0, p.stream, *co, p.m);
      return hipGetLastError();
    }
  }
  switch (p.n) {
#define CASE_N(NN) case NN: e = run_tfft_inv<P, NN>(p, w, dotv, nparts); break;
    WC_POW2_CASES(CASE_N)
#undef CASE_N
    default: return hipErrorInvalidValue;
  }
  return e;
}


// ---- many instances of uneven (n, M) in one persistent launch per pass ------------
// A pass lists the work units of the instances back to back (time tiles, x1 row groups,
// x2 column tiles) and launches one workgroup per unit; each finds its instance from the
// prefix counts and runs the tile body of the single-instance kernels at that instance's
// sizes.  Instances of every grid M share a time-pass launch when their n is the same,
// and instances of every n share a sine-pass launch when their M is the same: a launch
// whose LDS is sized for the largest tile runs the small tiles at the large tile's
// occupancy, so a pass launches once per tile shape present (at most four).  (A
// grid-stride loop over the units keeps loop-invariant addressing live across units:
// about 60 more VGPRs, one workgroup per CU.)  The dynamic LDS holds the largest tile of the batch and, behind it, the
// unit's own twiddle and sine tables, staged like the single kernels do; units are
// spread over the XCDs like the single kernels' tiles.
struct BatchArgs {
  int count;
  int inst[kBatchMax];
  const double *v[kBatchMax];
  double *w[kBatchMax];
  int t0[kBatchMax + 1];  // first work unit of each instance in this pass
  int aux;                // byte offset of the per-unit tables in the dynamic LDS
};

#define WC_BATCH_CASES(X) X(64) X(128) X(256) X(512)

__device__ __forceinline__ int batch_find(const BatchArgs &a, int t) {
  int i = 0;
  while (i + 1 < a.count && t >= a.t0[i + 1]) ++i;
  return i;
}

template <typename P, bool TBL>
__global__ __launch_bounds__(64 * kTimeWavesFwd) void k_batch_tfft_fwd(const BatchInst *__restrict__ tab,
                                                             BatchArgs a) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  cx<P> *buf = reinterpret_cast<cx<P> *>(dyn_lds);
  cx<P> *stw = reinterpret_cast<cx<P> *>(dyn_lds + a.aux);
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= a.t0[a.count]) return;
  const int i = batch_find(a, t);
  const BatchInst &I = tab[a.inst[i]];
  cx<P> *W = static_cast<cx<P> *>(I.W);
  const auto *dtw = static_cast<const cx<double> *>(I.dtw);
  const auto *tw = static_cast<const cx<P> *>(I.twt);
  switch (I.n) {
#define CASE_B(NN)                                                                             \
  case NN:                                                                                     \
    tfft_fwd_tile<P, NN, default_ts<P, NN>(), false, TBL>(a.v[i], W, dtw, tw, I.m, GenIn{},   \
                                                         t - a.t0[i], buf, stw);               \
    break;
    WC_BATCH_CASES(CASE_B)
#undef CASE_B
    default: break;
  }
}

template <typename P, bool TBL>
__global__ __launch_bounds__(64 * kTimeWavesInv) void k_batch_tfft_inv(const BatchInst *__restrict__ tab,
                                                             BatchArgs a) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  cx<P> *buf = reinterpret_cast<cx<P> *>(dyn_lds);
  cx<P> *stw = reinterpret_cast<cx<P> *>(dyn_lds + a.aux);
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= a.t0[a.count]) return;
  const int i = batch_find(a, t);
  const BatchInst &I = tab[a.inst[i]];
  const cx<P> *W = static_cast<const cx<P> *>(I.W);
  const auto *dtw = static_cast<const cx<double> *>(I.dtw);
  const auto *tw = static_cast<const cx<P> *>(I.twt);
  switch (I.n) {
#define CASE_B(NN)                                                                             \
  case NN:                                                                                     \
    static_assert(TimeCfg<P, NN, default_ts<P, NN>(), kTimeWavesInv>::NT ==                    \
                  64 * kTimeWavesInv, "the launch has 64 * kTimeWavesInv threads");            \
    tfft_inv_tile<P, NN, default_ts<P, NN>(), TBL>(W, a.w[i], dtw, tw, I.m, nullptr,         \
                                                   nullptr, t - a.t0[i], buf, stw,         \
                                                   nullptr);                                   \
    break;
    WC_BATCH_CASES(CASE_B)
#undef CASE_B
    default: break;
  }
}

template <typename P>
__global__ __launch_bounds__(kThreads) void k_batch_rows(const BatchInst *__restrict__ tab,
                                                         BatchArgs a, int slice) {
  // a unit is kThreads/64 consecutive line groups of one instance, one per wave
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int WPB = kThreads / 64;
  const int t = blockIdx.x;
  if (t >= a.t0[a.count]) return;
  const int i = batch_find(a, t);
  const BatchInst &I = tab[a.inst[i]];
  cx<P> *W = static_cast<cx<P> *>(I.W);
  cx<P> *buf = reinterpret_cast<cx<P> *>(dyn_lds + (size_t)wv * slice);
  cx<P> *stw = reinterpret_cast<cx<P> *>(dyn_lds + a.aux);
  P *ssin = reinterpret_cast<P *>(stw + I.N1);
  const auto *tw = static_cast<const cx<P> *>(I.tws);
  const auto *sn = static_cast<const P *>(I.sin);
  for (int k = threadIdx.x; k < I.N1; k += kThreads) {
    stw[k] = tw[k];
    ssin[k] = sn[k];
  }
  __syncthreads();
  const int grp = (t - a.t0[i]) * WPB + wv;
  switch (I.N1) {
#define CASE_B(NN)                                                                             \
  case NN:                                                                                     \
    if (grp < (I.n * (NN - 1) + RowCfg<P, NN>::B - 1) / RowCfg<P, NN>::B)                      \
      dst_rows_group<P, NN>(W, I.n * (NN - 1), grp, stw, ssin, buf, lane);                     \
    break;
    WC_BATCH_CASES(CASE_B)
#undef CASE_B
    default: break;
  }
}

template <typename P, bool TBL>
__global__ __launch_bounds__(64 * kColWaves) void k_batch_cols(const BatchInst *__restrict__ tab,
                                                         BatchArgs a) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  cx<P> *buf = reinterpret_cast<cx<P> *>(dyn_lds);
  cx<P> *stw = reinterpret_cast<cx<P> *>(dyn_lds + a.aux);
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= a.t0[a.count]) return;
  const int i = batch_find(a, t);
  const BatchInst &I = tab[a.inst[i]];
  cx<P> *W = static_cast<cx<P> *>(I.W);
  const auto *tw = static_cast<const cx<P> *>(I.tws);
  const auto *sn = static_cast<const P *>(I.sin);
  P *ssin = reinterpret_cast<P *>(stw + I.N1);
  const auto *lam = static_cast<const cx<P> *>(I.lam);
  const auto *mu = static_cast<const P *>(I.mu);
  switch (I.N1) {
#define CASE_B(NN)                                                                             \
  case NN:                                                                                     \
    cols_mode_tile<P, NN, default_tx<P, NN>(), TBL>(W, tw, sn, lam, mu, I.kind, (P)I.tau,    \
                                                    (P)I.alpha, (P)I.cnorm, t - a.t0[i],       \
                                                    buf, stw, ssin);                    \
    break;
    WC_BATCH_CASES(CASE_B)
#undef CASE_B
    default: break;
  }
}

// work units and LDS bytes of one instance in each pass
template <typename P> struct BatchShape {
  int time_units, time_lds, time_tab, row_units, row_slice, col_units, col_lds, space_tab,
      col_threads;
};
template <typename P> BatchShape<P> batch_shape(int n, int N1, int m) {
  BatchShape<P> b{};
  switch (n) {
#define CASE_B(NN)                                                                             \
  case NN: {                                                                                   \
    constexpr int TS = default_ts<P, NN>();                                                    \
    b.time_units = (m + TS - 1) / TS;                                                          \
    b.time_lds = TimeCfg<P, NN, TS>::TILE;                                                     \
    b.time_tab = NN * TimeCfg<P, NN, TS>::CXB;                                                 \
    break;                                                                                     \
  }
    WC_BATCH_CASES(CASE_B)
#undef CASE_B
    default: break;
  }
  switch (N1) {
#define CASE_B(NN)                                                                             \
  case NN: {                                                                                   \
    using R = RowCfg<P, NN>;                                                                   \
    constexpr int TX = default_tx<P, NN>();                                                    \
    b.row_units = ((n * (NN - 1) + R::B - 1) / R::B + kThreads / 64 - 1) / (kThreads / 64);    \
    b.row_slice = R::PN * R::S * R::CXB;                                                       \
    b.col_units = ((NN - 1 + TX - 1) / TX) * (n / 2);                                          \
    b.col_lds = ColCfg<P, NN, TX>::TILE;                                                       \
    b.space_tab = ColCfg<P, NN, TX>::TAB;                                                      \
    b.col_threads = ColCfg<P, NN, TX>::NT;                                                     \
    break;                                                                                     \
  }
    WC_BATCH_CASES(CASE_B)
#undef CASE_B
    default: break;
  }
  return b;
}

// Dynamic LDS above 64 KiB must be allowed per kernel; done once per kernel, for the
// whole CU budget.
hipError_t allow_lds(const void *kernel, int lds) {
  static std::mutex mu;
  static std::vector<const void *> done;
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(done.begin(), done.end(), kernel) != done.end()) return hipSuccess;
  if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kCuLds) ==
      hipSuccess) {
    done.push_back(kernel);
    return hipSuccess;
  }
  (void)hipGetLastError();  // the whole budget refused: allow this launch's size only
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

template <typename K>
hipError_t batch_launch(K kernel, int units, int lds, hipStream_t st, const BatchInst *tab,
                        const BatchArgs &a, int threads = kThreads) {
  if (lds > 65536 && allow_lds((const void *)kernel, lds) != hipSuccess)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(kernel, dim3(std::max(1, units)), dim3(threads), (size_t)lds, st, tab, a);
  return hipGetLastError();
}

// tables behind the largest tile when that keeps the same number of resident workgroups
int with_tables(int tile, int tab, BatchArgs &a) {
  a.aux = (tile + 15) & ~15;
  return blocks_per_cu(a.aux + tab) == blocks_per_cu(tile) ? a.aux + tab : 0;
}

// One pass over the instances whose tile shape matches `key` (n for the time passes, M+1
// for the sine passes): their work units back to back in one launch.
template <typename P>
BatchArgs batch_args(const BatchInst *h_tab, int cnt, const int *idx, const double *const *v,
                     double *const *w, bool time, int key, int *lds, int *tab, int *slice) {
  BatchArgs a{};
  *lds = *tab = *slice = 0;
  for (int i = 0; i < cnt; ++i) {
    const BatchInst &I = h_tab[idx[i]];
    if ((time ? I.n : I.N1) != key) continue;
    const BatchShape<P> b = batch_shape<P>(I.n, I.N1, I.m);
    const int k = a.count++;
    a.inst[k] = idx[i];
    a.v[k] = v ? v[i] : nullptr;
    a.w[k] = w ? w[i] : nullptr;
    a.t0[k + 1] = a.t0[k] + (time ? b.time_units : b.row_units);
    *lds = time ? b.time_lds : b.col_lds;
    *tab = time ? b.time_tab : b.space_tab;
    *slice = b.row_slice;
  }
  return a;
}

// the distinct values of n (time) or M+1 (sine passes) among the instances
std::vector<int> batch_keys(const BatchInst *h_tab, int cnt, const int *idx, bool time) {
  std::vector<int> k;
  for (int i = 0; i < cnt; ++i) {
    const int x = time ? h_tab[idx[i]].n : h_tab[idx[i]].N1;
    if (std::find(k.begin(), k.end(), x) == k.end()) k.push_back(x);
  }
  return k;
}

template <typename P>
hipError_t time_pass(hipStream_t st, const BatchInst *d_tab, const BatchInst *h_tab, int cnt,
                     const int *idx, const double *const *v, double *const *w, bool inverse) {
  for (int key : batch_keys(h_tab, cnt, idx, true)) {
    int tl, tt, unused;
    BatchArgs a = batch_args<P>(h_tab, cnt, idx, v, w, true, key, &tl, &tt, &unused);
    const int tlt = with_tables(tl, tt, a);
    hipError_t e;
    constexpr int NF = 64 * kTimeWavesFwd, NI = 64 * kTimeWavesInv;
    if (inverse)
      e = tlt ? batch_launch(k_batch_tfft_inv<P, true>, a.t0[a.count], tlt, st, d_tab, a, NI)
              : batch_launch(k_batch_tfft_inv<P, false>, a.t0[a.count], tl, st, d_tab, a, NI);
    else
      e = tlt ? batch_launch(k_batch_tfft_fwd<P, true>, a.t0[a.count], tlt, st, d_tab, a, NF)
              : batch_launch(k_batch_tfft_fwd<P, false>, a.t0[a.count], tl, st, d_tab, a, NF);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename P>
hipError_t space_pass(hipStream_t st, const BatchInst *d_tab, const BatchInst *h_tab, int cnt,
                      const int *idx, bool cols) {
  for (int key : batch_keys(h_tab, cnt, idx, false)) {
    int cl, ct, rs;
    BatchArgs a = batch_args<P>(h_tab, cnt, idx, nullptr, nullptr, false, key, &cl, &ct, &rs);
    hipError_t e;
    if (cols) {
      // column tiles: recount the units (the list above holds the row units)
      int NC = kThreads;  // the tile body's width for this M
      for (int k = 0; k < a.count; ++k) {
        const BatchInst &I = h_tab[a.inst[k]];
        const BatchShape<P> b = batch_shape<P>(I.n, I.N1, I.m);
        a.t0[k + 1] = a.t0[k] + b.col_units;
        NC = b.col_threads;
      }
      const int clt = with_tables(cl, ct, a);
      e = clt ? batch_launch(k_batch_cols<P, true>, a.t0[a.count], clt, st, d_tab, a, NC)
              : batch_launch(k_batch_cols<P, false>, a.t0[a.count], cl, st, d_tab, a, NC);
    } else {
      a.aux = rs * (kThreads / 64);  // the row passes always stage their tables
      const int rl = a.aux + ct;
      if (rl > 65536) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_batch_rows<P>, dim3(std::max(1, a.t0[a.count])), dim3(kThreads),
                         (size_t)rl, st, d_tab, a, rs);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename P>
hipError_t pc_batch_t(hipStream_t st, const BatchInst *d_tab, const BatchInst *h_tab, int cnt,
                      const int *idx, const double *const *v, double *const *w) {
  hipError_t e;
  if ((e = time_pass<P>(st, d_tab, h_tab, cnt, idx, v, w, false)) != hipSuccess) return e;
  if ((e = space_pass<P>(st, d_tab, h_tab, cnt, idx, false)) != hipSuccess) return e;
  if ((e = space_pass<P>(st, d_tab, h_tab, cnt, idx, true)) != hipSuccess) return e;
  if ((e = space_pass<P>(st, d_tab, h_tab, cnt, idx, false)) != hipSuccess) return e;
  return time_pass<P>(st, d_tab, h_tab, cnt, idx, v, w, true);
}

}  // namespace

bool pc_supported(int n, int N1) {
  auto pow2 = [](int x) { return x >= 4 && x <= 1024 && (x & (x - 1)) == 0; };
  return pow2(n) && pow2(N1);
}

bool batch_sizes_ok(int n, int N1) {
  auto ok = [](int x) { return x == 64 || x == 128 || x == 256 || x == 512; };
  return ok(n) && ok(N1);
}

hipError_t launch_pc_batch(hipStream_t st, const BatchInst *d_tab, const BatchInst *h_tab,
                           int cnt, const int *idx, const double *const *v, double *const *w,
                           bool fp32) {
  if (cnt < 1 || cnt > kBatchMax) return hipErrorInvalidValue;
  for (int i = 0; i < cnt; ++i)
    if (!batch_sizes_ok(h_tab[idx[i]].n, h_tab[idx[i]].N1)) return hipErrorInvalidValue;
  return fp32 ? pc_batch_t<float>(st, d_tab, h_tab, cnt, idx, v, w)
              : pc_batch_t<double>(st, d_tab, h_tab, cnt, idx, v, w);
}

hipError_t launch_pc_apply(const wc_plan &p, const double *v, double *w, bool dot,
                           int *nparts) {
  int np = 0;
  const double *dotv = dot ? v : nullptr;
  hipError_t e = p.opts.precision == WC_MIXED
                    ? pc_apply_t<float>(p, v, w, dotv, &np, nullptr, nullptr)
                    : pc_apply_t<double>(p, v, w, dotv, &np, nullptr, nullptr);
  if (nparts) *nparts = np;
  return e;
}

hipError_t launch_pc_lowrank(const wc_plan &p, const double *r0, const double *hat_in,
                             double *hat_out, double *w) {
  if (p.opts.precision != WC_FP64 && !p.lr_2d) return hipErrorInvalidValue;
  GenIn gen{hat_in, p.d_lr_s0, p.d_lr_gr, p.d_scal + S_LR_SQN0, 1.0 / p.lr_gn, 1.0 / p.lr_rn};
  ContractOut co{hat_out, -p.lr_gn, -p.lr_rn, p.d_lr_rho, p.d_lr_part};  // omega = e^{i pi} = -1
  int np = 0;
  return p.opts.precision == WC_MIXED
             ? pc_apply_t<float>(p, r0, w, nullptr, &np, &gen, hat_out ? &co : nullptr)
             : pc_apply_t<double>(p, r0, w, nullptr, &np, &gen, hat_out ? &co : nullptr);
}

namespace {
// x2 sine transform of the whole spectrum (the cycle's Yhat0 for the pointwise step)
template <typename P, int N1>
hipError_t cols_dst_t(const wc_plan &p, const cx<P> *in, cx<P> *out, int npairs = 0) {
  constexpr int TX = default_tx<P, N1>();
  if constexpr (!ColCfg<P, N1, TX>::FITS) {
    return hipErrorInvalidValue;
  } else {
    // slab pairs (2q, 2q + 1) transformed: all n/2 of the spectrum by default
    const int nq = npairs > 0 ? npairs : p.n / 2;
    const int ncx = (N1 - 2 + TX) / TX;
    ProfScope ps(p, K_DST_X2_FWD, 2.0 * (2.0 * nq * p.m * sizeof(cx<P>)));
    hipLaunchKernelGGL((k_cols_dst<P, N1, TX>), dim3(ncx * nq),
                       dim3(ColCfg<P, N1, TX>::NT), 0, p.stream, in, out, Tabs<P>::tws(p),
                       Tabs<P>::sin(p));
    return hipGetLastError();
  }
}

template <typename P> hipError_t lr_spectrum_t(const wc_plan &p, const double *r0) {
  hipError_t e = hipErrorInvalidValue;
  cx<P> *Y = (cx<P> *)p.d_specA;  // transformed in place, kept for the cycle
  switch (p.n) {
#define CASE_N(NN) case NN: e = run_tfft_fwd<P, NN>(p, r0, nullptr, Y); break;
    WC_POW2_CASES(CASE_N)
#undef CASE_N
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int nlines = p.n * p.M;
  switch (p.N1) {
#define CASE_S(NN)                                                                 \
  case NN:                                                                         \
    e = dst_rows_on<P, NN>(p, Y, nlines, K_DST_X1_FWD, 2.0 * p.nvec * sizeof(P));  \
    if (e == hipSuccess) e = cols_dst_t<P, NN>(p, Y, Y);                            \
    return e;
    WC_POW2_CASES(CASE_S)
#undef CASE_S
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_lr_sine_s0(const wc_plan &p) {
  if (!p.lr_2d) return hipErrorInvalidValue;
  switch (p.N1) {
#define CASE_S(NN) case NN: return lr_sine_s0_t<NN>(p);
    WC_POW2_CASES(CASE_S)
#undef CASE_S
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lr_spectrum(const wc_plan &p, const double *r0) {
  if (!p.lr_2d) return hipErrorInvalidValue;
  return p.opts.precision == WC_MIXED ? lr_spectrum_t<float>(p, r0)
                                      : lr_spectrum_t<double>(p, r0);
}

// ---- finite elements (a == 1) in sine coordinates --------------------------------------
// The mass and stiffness matrices of the linear / bilinear elements are diagonal in the
// orthonormal sine basis: mass m_j1 (m_j2), M^{-1/2} K M^{-1/2} mu_j1 (+ mu_j2), so the
// system is solved in sine coordinates, where step 2 of the preconditioner is one
// pointwise pass and the data and the solution are transformed once per solve.
__device__ __forceinline__ double fem_mass(const double *__restrict__ m1, int s, int M,
                                           int dims) {
  return dims == 1 ? m1[s] : m1[s % M] * m1[s / M];
}

// W[k m + s] = (A + i B)[k m + s] * mass_s^power, k < nslab (B may be null: zero)
__global__ __launch_bounds__(kThreads) void k_fem_pack(const double *__restrict__ A,
                                                       const double *__restrict__ B,
                                                       cx<double> *__restrict__ W, size_t cnt,
                                                       int m, int M, int dims,
                                                       const double *__restrict__ m1,
                                                       double power) {
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= cnt) return;
  const int s = (int)(idx % (size_t)m);
  const double w = power == 0.0 ? 1.0 : pow(fem_mass(m1, s, M, dims), power);
  W[idx] = cx<double>{A[idx] * w, B ? B[idx] * w : 0.0};
}

// A = scale mass^power Re W, B likewise with Im W, U = ucoef B when U is not null
__global__ __launch_bounds__(kThreads) void k_fem_unpack(const cx<double> *__restrict__ W,
                                                         double *__restrict__ A,
                                                         double *__restrict__ B,
                                                         double *__restrict__ U, size_t cnt, int m,
                                                         int M, int dims,
                                                         const double *__restrict__ m1,
                                                         double power, double scale, double ucoef) {
  const size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= cnt) return;
  const int s = (int)(idx % (size_t)m);
  const double w = scale * (power == 0.0 ? 1.0 : pow(fem_mass(m1, s, M, dims), power));
  const cx<double> z = W[idx];
  A[idx] = w * z.x;
  B[idx] = w * z.y;
  if (U) U[idx] = ucoef * w * z.y;
}

// the y0 terms of the first block rows in sine coordinates, y0' = scale Re W[0 .. m):
// f_1 += M^{-1/2} (M - (1 - theta) tau K) y0 = sqrt(mass) (1 - (1 - theta) tau mu) y0'
// (times sqrt(gamma) in the system's right-hand side), g_1 -= tau (1 - theta) sqrt(mass) y0'
__global__ __launch_bounds__(kThreads) void k_fem_y0(const cx<double> *__restrict__ W,
                                                     double *__restrict__ bf,
                                                     double *__restrict__ bg, int m, int M,
                                                     int dims, const double *__restrict__ m1,
                                                     const double *__restrict__ mu, double scale,
                                                     double sqrt_gamma, double tau, double theta) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= m) return;
  const double y = scale * W[s].x, sm = sqrt(fem_mass(m1, s, M, dims));
  const double musum = dims == 1 ? mu[s] : mu[s % M] + mu[s / M];
  bf[s] += sqrt_gamma * sm * (1.0 - (1.0 - theta) * tau * musum) * y;
  bg[s] -= tau * (1.0 - theta) * sm * y;
}

namespace {
// unnormalised sine transform of the first nslab slabs of d_femW (2D: both directions)
template <int N1> hipError_t fem_dst_t(const wc_plan &p, int nslab) {
  constexpr int M = N1 - 1;
  cx<double> *W = (cx<double> *)p.d_femW;
  hipError_t e = dst_rows_on<double, N1>(p, W, p.dims == 2 ? nslab * M : nslab, K_DST_X1_FWD,
                                         2.0 * nslab * p.m * sizeof(cx<double>));
  if (e != hipSuccess || p.dims == 1) return e;
  return cols_dst_t<double, N1>(p, W, W, (nslab + 1) / 2);
}
hipError_t fem_dst(const wc_plan &p, int nslab) {
  switch (p.N1) {
#define CASE_S(NN) case NN: return fem_dst_t<NN>(p, nslab);
    WC_POW2_CASES(CASE_S)
#undef CASE_S
    default: return hipErrorInvalidValue;
  }
}
unsigned blocks_of(size_t cnt) { return (unsigned)((cnt + kThreads - 1) / kThreads); }
// orthonormal sine basis = (2/N1)^{dims/2} times the unnormalised transform
double fem_scale(const wc_plan &p) { return std::pow(2.0 / p.N1, 0.5 * p.dims); }
}  // namespace

hipError_t launch_fem_rhs_finish(const wc_plan &p, const double *y0, double *b) {
  if (!p.fem || !p.d_femW || p.n % 2) return hipErrorInvalidValue;
  const size_t nm = (size_t)p.n * p.m;
  cx<double> *W = (cx<double> *)p.d_femW;
  hipError_t e;
  {  // both block rows into sine coordinates, times M^{-1/2} M = M^{1/2}
    ProfScope ps(p, K_RHS, 16.0 * nm + 16.0 * nm);
    hipLaunchKernelGGL(k_fem_pack, dim3(blocks_of(nm)), dim3(kThreads), 0, p.stream, b, b + nm, W,
                       nm, p.m, p.M, p.dims, p.d_mass64, 0.0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = fem_dst(p, p.n)) != hipSuccess) return e;
  {
    ProfScope ps(p, K_RHS, 16.0 * nm + 16.0 * nm);
    hipLaunchKernelGGL(k_fem_unpack, dim3(blocks_of(nm)), dim3(kThreads), 0, p.stream, W, b, b + nm,
                       nullptr, nm, p.m, p.M, p.dims, p.d_mass64, 0.5, fem_scale(p), 0.0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {  // y0 into sine coordinates (slab 0), then its terms in the first block rows
    ProfScope ps(p, K_RHS, 24.0 * p.m);
    hipLaunchKernelGGL(k_fem_pack, dim3(blocks_of(p.m)), dim3(kThreads), 0, p.stream, y0, nullptr,
                       W, (size_t)p.m, p.m, p.M, p.dims, p.d_mass64, 0.0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = fem_dst(p, 1)) != hipSuccess) return e;
  // GMRES: b = [sqrt(gamma) f; g]; MINRES: b = [g; sqrt(gamma) f]
  const bool sym = p.opts.method != WC_GMRES_PS;
  double *bf = sym ? b + nm : b, *bg = sym ? b : b + nm;
  ProfScope ps(p, K_RHS, 40.0 * p.m);
  hipLaunchKernelGGL(k_fem_y0, dim3(blocks_of(p.m)), dim3(kThreads), 0, p.stream, W, bf, bg, p.m,
                     p.M, p.dims, p.d_mass64, p.d_mu64, fem_scale(p), std::sqrt(p.gamma), p.tau,
                     p.theta);
  return hipGetLastError();
}

hipError_t launch_fem_recover_finish(const wc_plan &p, double *y, double *pp, double *u) {
  if (!p.fem || !p.d_femW || p.n % 2) return hipErrorInvalidValue;
  const size_t nm = (size_t)p.n * p.m;
  cx<double> *W = (cx<double> *)p.d_femW;
  hipError_t e;
  {  // M^{-1/2} in sine coordinates, then back to nodal values
    ProfScope ps(p, K_RECOVER, 16.0 * nm + 16.0 * nm);
    hipLaunchKernelGGL(k_fem_pack, dim3(blocks_of(nm)), dim3(kThreads), 0, p.stream, y, pp, W, nm,
                       p.m, p.M, p.dims, p.d_mass64, -0.5);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = fem_dst(p, p.n)) != hipSuccess) return e;
  ProfScope ps(p, K_RECOVER, 16.0 * nm + (u ? 24.0 : 16.0) * nm);
  hipLaunchKernelGGL(k_fem_unpack, dim3(blocks_of(nm)), dim3(kThreads), 0, p.stream, W, y, pp, u,
                     nm, p.m, p.M, p.dims, p.d_mass64, 0.0, fem_scale(p), 1.0 / p.gamma);
  return hipGetLastError();
}

int pc_partials_needed(int n, int m, int precision) {
  // bound on the inverse time FFT's grid: tiles of at least 4 spatial columns (packed
  // form) or of at least 8 columns of each block row
  (void)n;
  (void)precision;
  return (m + 3) / 4 + 2;
}

}  // namespace wc
