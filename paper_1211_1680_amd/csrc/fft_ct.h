// Transforms whose length and radix plan are compile-time constants (the 4095-point odd DFT
// and the 4096-point FFT of band-limit 2048), for the specialised kernels of that size.  Same
// Stockham autosort passes as fft_lds.h, with three differences that matter for speed:
//  - element i of a transform lives in LDS slot i + i/8 (one pad slot per 8), so the strided
//    writes of the early passes (stride = radix) spread over the LDS banks;
//  - twiddles W_N^p = lo[p mod 64] hi[p / 64] come from 64-entry tables staged in LDS;
//  - every index computation divides by compile-time constants.
#pragma once
#include "fft_lds.h"

#include <type_traits>

namespace s2let {

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 3); }
constexpr int lds_padded(int n) { return n + (n >> 3) + 1; }
// LDS slot of element i of a transform: padded for the power-of-two FFTs, whose strided writes
// would otherwise share banks; plain for the odd-length DFT, whose strides (its radices) are odd
// and whose sub-transform counts are not multiples of 8, so that pad slots would split groups of 8
// consecutive lanes across two LDS cycles
template <bool PAD>
__device__ __forceinline__ int lds_at(int i) { return PAD ? lds_pad(i) : i; }

// Input of the theta stage for an even order mE and the odd order mE + 1 of one column pair:
// ring r < K of both orders, r = lt + i T.  Every gather is issued before the first one is
// consumed, and each ring is read once for both of its nodes on the 2 pi extension (t = r and
// t = 2K-2-r).
// Ring t of one phi problem into LDS slots q < N: REAL packs map ma (real part) and map ma + 1
// (imaginary part, zero without it); otherwise map ma is complex.  Every load is issued before
// the first store.
template <int N, int T, int REAL, bool PAD = true, typename C2 = double2>
__device__ __forceinline__ void load_ring(const double* __restrict__ f, long long map_stride, int ma, bool hasb,
                                          int t, bool valid, C2* buf, int lt) {
  constexpr int PER = (N + T - 1) / T;
  double2 z[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int q = lt + i * T;
    const size_t off = (size_t)t * N + (q < N ? q : 0);
    if (REAL) {
      z[i].x = f[(size_t)ma * map_stride + off];
      z[i].y = hasb ? f[(size_t)(ma + 1) * map_stride + off] : 0.0;
    } else {
      z[i] = reinterpret_cast<const double2*>(f)[(size_t)ma * map_stride + off];
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int q = lt + i * T;
    if (q < N) buf[lds_at<PAD>(q)] = valid ? cplx<C2>(z[i]) : czero<C2>();
  }
}

// Input of the inverse phi DFT of ring t (rows FT[(t*K + m)*C + c]): slot m < K takes order m,
// slot N - m (0 < m < K) order -m.  REAL: the unit packs maps ma and ma + 1 as a + i b, with the
// negative orders their conjugates; otherwise columns 4 ma .. 4 ma + 3 hold orders +m and -m of
// map ma.  Each row is read once for both slots, and every load is issued before the first store.
// (TF: the element type of FT, double or float; C2: the complex type of the LDS buffer)
// QUAD: FT in the column-quad layout, element (t, m, c) at ((t (C/4) + c/4) K + m) 4 + c mod 4 (the
// unit's four columns are one quad).
template <int K, int T, int REAL, bool PAD = true, typename TF = double, typename C2 = double2, bool QUAD = false>
__device__ __forceinline__ void load_orders(const TF* __restrict__ FT, int C, int ma, bool hasb, int t,
                                            bool valid, C2* buf, int lt) {
  typedef decltype(C2::x) S;
  constexpr int N = 2 * K - 1;
  constexpr int PER = K / T;
  static_assert(K % T == 0, "orders per thread");
  typedef typename std::conditional<sizeof(TF) == 8, double2, float2>::type V2;
  V2 ra[PER], rb[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if constexpr (QUAD) {
      const TF* q = FT + (((size_t)t * (C >> 2) + (REAL ? ma >> 1 : ma)) * K + lt + i * T) * 4;
      ra[i] = *reinterpret_cast<const V2*>(q);
      rb[i] = (!REAL || hasb) ? *reinterpret_cast<const V2*>(q + 2) : V2{};
      continue;
    }
    const TF* row = FT + ((size_t)t * K + lt + i * T) * C;
    if (REAL) {
      ra[i] = *reinterpret_cast<const V2*>(row + 2 * ma);
      rb[i] = hasb ? *reinterpret_cast<const V2*>(row + 2 * ma + 2) : V2{};
    } else {
      ra[i] = *reinterpret_cast<const V2*>(row + 4 * ma);
      rb[i] = *reinterpret_cast<const V2*>(row + 4 * ma + 2);
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int m = lt + i * T;
    const S ax = valid ? (S)ra[i].x : S(0), ay = valid ? (S)ra[i].y : S(0);
    const S bx = valid ? (S)rb[i].x : S(0), by = valid ? (S)rb[i].y : S(0);
    if (REAL) {
      buf[lds_at<PAD>(m)] = CplxTraits<C2>::make(ax - by, ay + bx);
      if (m > 0) buf[lds_at<PAD>(N - m)] = CplxTraits<C2>::make(ax + by, bx - ay);
    } else {
      buf[lds_at<PAD>(m)] = CplxTraits<C2>::make(ax, ay);
      if (m > 0) buf[lds_at<PAD>(N - m)] = CplxTraits<C2>::make(bx, by);
    }
  }
}

template <int K, int T, typename TG = double>
struct RingGather {
  typedef typename std::conditional<sizeof(TG) == 8, double2, float2>::type V2;
  static constexpr int PER = K / T;
  static_assert(K % T == 0, "rings per thread");
  V2 ge[PER], go[PER];
  __device__ __forceinline__ void load(const TG* __restrict__ GT, int C, int mE, int s, int lt) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const TG* row = GT + ((size_t)(lt + i * T) * K + mE) * C + 2 * s;
      ge[i] = *reinterpret_cast<const V2*>(row);
      go[i] = *reinterpret_cast<const V2*>(row + C);
    }
  }
};

// Twiddle tables: W^p = lo[p mod 64] hi[p / 64].  The low table of a power-of-two transform
// leaves one spare slot after every eight entries (twlo_at): in the passes whose twiddle index steps
// by 8 (NS = 64 at 4096 points, and the passes of the shorter transforms that use those tables),
// the eight lanes an LDS cycle serves read entries 0, 8, ..., 56, which the plain layout puts in
// the same four banks.  The 4095-point tables keep the plain layout, which is better for their
// index patterns.
constexpr int TWLO_SLOTS = 72;
__host__ __device__ constexpr int twlo_at(int i) { return i + (i >> 3); }

template <int R, bool INV, typename C2>
__device__ __forceinline__ void dft_small(C2* v) {
  if constexpr (R == 2 || R == 4 || R == 8 || R == 16)
    SmallDft<R, INV, C2>::run(v);
  else
    OddDft<R, INV, C2>::run(v);
}

// One pass: N points, radix R, NS = product of the radices of the earlier passes, T threads.
// The twiddle tables hold W_{N TS}^p (TS > 1: a shorter transform with the tables of a longer one).
// LM / SM: bit r clear = input r of every butterfly is known to be zero (not loaded) / output r is
// not needed (not stored).  PAD: the slot layout (lds_at).
// inputs j + r N/R of butterfly j of a pass, with the pass's twiddles applied
template <int N, int R, int NS, bool INV, int TS, unsigned LM, bool PAD = true, typename C2>
__device__ __forceinline__ void ct_gather(const C2* buf, int j, C2* v, const C2* wlo, const C2* whi) {
  constexpr int NB = N / R;
  constexpr int STRIDE = N / (NS * R);
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = ((LM >> r) & 1u) ? buf[lds_at<PAD>(j + r * NB)] : czero<C2>();
  if constexpr (NS > 1) {
    const int p = (j % NS) * STRIDE * TS;
    constexpr bool P2 = (N & (N - 1)) == 0;
    C2 w1 = cmul(wlo[P2 ? twlo_at(p & 63) : (p & 63)], whi[p >> 6]);
    if (INV) w1 = conjd(w1);
    C2 w = w1;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = cmul(v[r], w);
      if (r + 1 < R) w = cmul(w, w1);
    }
  }
}

template <int N, int R, int NS, bool INV, int T, int TS = 1, unsigned LM = 0xFFFFu, unsigned SM = 0xFFFFu,
          bool PAD = true, typename C2>
__device__ __forceinline__ void ct_pass(C2* buf, int lt, const C2* wlo, const C2* whi) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + T - 1) / T;
  static_assert(N % (NS * R) == 0, "radix plan does not divide the length");
  C2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) ct_gather<N, R, NS, INV, TS, LM, PAD>(buf, j, v[i], wlo, whi);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
      dft_small<R, INV>(v[i]);
      const int kk = j % NS;
      const int base = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((SM >> r) & 1u) buf[lds_at<PAD>(base + r * NS)] = v[i][r];
    }
  }
  __syncthreads();
}

// 4096 = 8^4 with every thread active: fewer registers than the radix-16 plan below, for kernels
// that keep other values live across their transforms
template <bool INV, int T, typename C2>
__device__ __forceinline__ void fft4096_r8(C2* buf, int lt, const C2* wlo, const C2* whi) {
  ct_pass<4096, 8, 1, INV, T>(buf, lt, wlo, whi);
  ct_pass<4096, 8, 8, INV, T>(buf, lt, wlo, whi);
  ct_pass<4096, 8, 64, INV, T>(buf, lt, wlo, whi);
  ct_pass<4096, 8, 512, INV, T>(buf, lt, wlo, whi);
}

// Circular convolution of one frequency-parity class of the theta stage (NL = 2k slots, tables of
// W_{NL TS}) with a kernel whose spectrum kr is real (unnormalised transforms: kr carries the
// 1/NL).  The input lies on [0, NL/4) and [3NL/4, NL) and the output is read there only, so the
// first pass loads and the last pass stores no other slots.  The forward plan is the inverse plan
// reversed, so both meet in a radix-8 pass: the last forward pass and the first inverse pass touch
// the same slots j + r NL/8 (j < NL/8), and one pass does both with the spectrum scaling in
// between, in registers (one LDS round trip and two barriers fewer than transform, scale,
// transform).
template <int NL, int T, int TS, typename C2>
__device__ __forceinline__ void corr_conv_mid(C2* buf, int lt, const C2* wlo, const C2* whi,
                                              const double* __restrict__ kr) {
  typedef typename CplxTraits<C2>::S S;
  constexpr int NB = NL / 8;
  constexpr int PER = (NB + T - 1) / T;
  C2 v[PER][8];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) ct_gather<NL, 8, NB, false, TS, 0xFFFFu>(buf, j, v[i], wlo, whi);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
      S k[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) k[r] = (S)kr[j + r * NB];
      dft_small<8, false>(v[i]);   // bin j + NB r in v[i][r]
#pragma unroll
      for (int r = 0; r < 8; ++r) v[i][r] = CplxTraits<C2>::make(v[i][r].x * k[r], v[i][r].y * k[r]);
      dft_small<8, true>(v[i]);    // first inverse pass (no twiddles), outputs 8 j + r
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[lds_pad(8 * j + r)] = v[i][r];
    }
  }
  __syncthreads();
}

template <int NL, int T, int TS, typename C2>
__device__ __forceinline__ void corr_conv(C2* buf, int lt, const C2* wlo, const C2* whi,
                                          const double* __restrict__ kr) {
  // a radix-8 first (last) pass keeps inputs (outputs) 0, 1, 6, 7; a radix-4 one keeps 0 and 3
  constexpr unsigned M8 = 0xC3u, M4 = 0x9u;
  if constexpr (NL == 4096) {   // 8 8 8 | 8 | 8 8 8
    ct_pass<4096, 8, 1, false, T, TS, M8>(buf, lt, wlo, whi);
    ct_pass<4096, 8, 8, false, T, TS>(buf, lt, wlo, whi);
    ct_pass<4096, 8, 64, false, T, TS>(buf, lt, wlo, whi);
    corr_conv_mid<4096, T, TS>(buf, lt, wlo, whi, kr);
    ct_pass<4096, 8, 8, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<4096, 8, 64, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<4096, 8, 512, true, T, TS, 0xFFFFu, M8>(buf, lt, wlo, whi);
  } else if constexpr (NL == 2048) {   // 4 8 8 | 8 | 8 8 4
    ct_pass<2048, 4, 1, false, T, TS, M4>(buf, lt, wlo, whi);
    ct_pass<2048, 8, 4, false, T, TS>(buf, lt, wlo, whi);
    ct_pass<2048, 8, 32, false, T, TS>(buf, lt, wlo, whi);
    corr_conv_mid<2048, T, TS>(buf, lt, wlo, whi, kr);
    ct_pass<2048, 8, 8, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<2048, 8, 64, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<2048, 4, 512, true, T, TS, 0xFFFFu, M4>(buf, lt, wlo, whi);
  } else if constexpr (NL == 1024) {   // 4 4 8 | 8 | 8 4 4
    ct_pass<1024, 4, 1, false, T, TS, M4>(buf, lt, wlo, whi);
    ct_pass<1024, 4, 4, false, T, TS>(buf, lt, wlo, whi);
    ct_pass<1024, 8, 16, false, T, TS>(buf, lt, wlo, whi);
    corr_conv_mid<1024, T, TS>(buf, lt, wlo, whi, kr);
    ct_pass<1024, 8, 8, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<1024, 4, 64, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<1024, 4, 256, true, T, TS, 0xFFFFu, M4>(buf, lt, wlo, whi);
  } else if constexpr (NL == 512) {   // 8 8 | 8 | 8 8
    ct_pass<512, 8, 1, false, T, TS, M8>(buf, lt, wlo, whi);
    ct_pass<512, 8, 8, false, T, TS>(buf, lt, wlo, whi);
    corr_conv_mid<512, T, TS>(buf, lt, wlo, whi, kr);
    ct_pass<512, 8, 8, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<512, 8, 64, true, T, TS, 0xFFFFu, M8>(buf, lt, wlo, whi);
  } else if constexpr (NL == 256) {   // 4 8 | 8 | 8 4
    ct_pass<256, 4, 1, false, T, TS, M4>(buf, lt, wlo, whi);
    ct_pass<256, 8, 4, false, T, TS>(buf, lt, wlo, whi);
    corr_conv_mid<256, T, TS>(buf, lt, wlo, whi, kr);
    ct_pass<256, 8, 8, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<256, 4, 64, true, T, TS, 0xFFFFu, M4>(buf, lt, wlo, whi);
  } else {   // 4 4 | 8 | 4 4
    static_assert(NL == 128, "correlation lengths: 128 to 4096");
    ct_pass<128, 4, 1, false, T, TS, M4>(buf, lt, wlo, whi);
    ct_pass<128, 4, 4, false, T, TS>(buf, lt, wlo, whi);
    corr_conv_mid<128, T, TS>(buf, lt, wlo, whi, kr);
    ct_pass<128, 4, 8, true, T, TS>(buf, lt, wlo, whi);
    ct_pass<128, 4, 32, true, T, TS, 0xFFFFu, M4>(buf, lt, wlo, whi);
  }
}

// 4096 = 16^3 (unnormalised, sign -1 or +1 with INV): three passes, half of 512 threads active
// in each; 10 % faster than four radix-8 passes with every thread active (fewer LDS round trips
// and barriers)
template <bool INV, int T, unsigned LM0 = 0xFFFFu, unsigned SML = 0xFFFFu, typename C2>
__device__ __forceinline__ void fft4096(C2* buf, int lt, const C2* wlo, const C2* whi) {
  ct_pass<4096, 16, 1, INV, T, 1, LM0>(buf, lt, wlo, whi);
  ct_pass<4096, 16, 16, INV, T>(buf, lt, wlo, whi);
  ct_pass<4096, 16, 256, INV, T, 1, 0xFFFFu, SML>(buf, lt, wlo, whi);
}

// 2048 = 8^3 * 4, with the twiddle tables of length 4096 (unnormalised, sign -1 or +1 with INV)
// (LM0 / SML: the first pass's load mask and the last pass's store mask, see ct_pass)
template <bool INV, int T, int TS = 2, unsigned LM0 = 0xFFFFu, unsigned SML = 0xFFFFu>
__device__ __forceinline__ void fft2048(double2* buf, int lt, const double2* wlo, const double2* whi) {
  ct_pass<2048, 8, 1, INV, T, TS, LM0>(buf, lt, wlo, whi);
  ct_pass<2048, 8, 8, INV, T, TS>(buf, lt, wlo, whi);
  ct_pass<2048, 8, 64, INV, T, TS>(buf, lt, wlo, whi);
  ct_pass<2048, 4, 512, INV, T, TS, 0xFFFFu, SML>(buf, lt, wlo, whi);
}

// 1024 points (8 * 8 * 4 * 4) from the tables of W_{1024 TS}
template <bool INV, int T, int TS, unsigned LM0 = 0xFFFFu, unsigned SML = 0xFFFFu>
__device__ __forceinline__ void fft1024(double2* buf, int lt, const double2* wlo, const double2* whi) {
  ct_pass<1024, 8, 1, INV, T, TS, LM0>(buf, lt, wlo, whi);
  ct_pass<1024, 8, 8, INV, T, TS>(buf, lt, wlo, whi);
  ct_pass<1024, 4, 64, INV, T, TS>(buf, lt, wlo, whi);
  ct_pass<1024, 4, 256, INV, T, TS, 0xFFFFu, SML>(buf, lt, wlo, whi);
}

// 512 points (8 * 8 * 8) from the tables of W_{512 TS}
template <bool INV, int T, int TS, unsigned LM0 = 0xFFFFu, unsigned SML = 0xFFFFu>
__device__ __forceinline__ void fft512(double2* buf, int lt, const double2* wlo, const double2* whi) {
  ct_pass<512, 8, 1, INV, T, TS, LM0>(buf, lt, wlo, whi);
  ct_pass<512, 8, 8, INV, T, TS>(buf, lt, wlo, whi);
  ct_pass<512, 8, 64, INV, T, TS, 0xFFFFu, SML>(buf, lt, wlo, whi);
}

// 128 points (8 * 4 * 4) from the tables of W_{128 TS}
template <bool INV, int T, int TS, unsigned LM0 = 0xFFFFu, unsigned SML = 0xFFFFu>
__device__ __forceinline__ void fft128(double2* buf, int lt, const double2* wlo, const double2* whi) {
  ct_pass<128, 8, 1, INV, T, TS, LM0>(buf, lt, wlo, whi);
  ct_pass<128, 4, 8, INV, T, TS>(buf, lt, wlo, whi);
  ct_pass<128, 4, 32, INV, T, TS, 0xFFFFu, SML>(buf, lt, wlo, whi);
}

// 256 points (8 * 8 * 4) from the tables of W_{256 TS}
template <bool INV, int T, int TS, unsigned LM0 = 0xFFFFu, unsigned SML = 0xFFFFu>
__device__ __forceinline__ void fft256(double2* buf, int lt, const double2* wlo, const double2* whi) {
  ct_pass<256, 8, 1, INV, T, TS, LM0>(buf, lt, wlo, whi);
  ct_pass<256, 8, 8, INV, T, TS>(buf, lt, wlo, whi);
  ct_pass<256, 4, 64, INV, T, TS, 0xFFFFu, SML>(buf, lt, wlo, whi);
}

// The compiled power-of-two FFT of length NL from the tables of W_{NL TS}.  LOW_IN: the input
// vanishes on [NL/2, NL) (the first pass loads the lower half of each butterfly's inputs only);
// LOW_OUT: only [0, NL/2) of the output is used (the last pass stores the lower half only).
template <int NL, bool INV, int T, int TS, bool LOW_IN = false, bool LOW_OUT = false>
__device__ __forceinline__ void fft_ct(double2* buf, int lt, const double2* wlo, const double2* whi) {
  // first radix 16 (4096) or 8; last radix 16 (4096), 8 (512) or 4
  constexpr unsigned LM0 = !LOW_IN ? 0xFFFFu : (NL == 4096 ? 0xFFu : 0xFu);
  constexpr unsigned SML = !LOW_OUT ? 0xFFFFu : (NL == 4096 ? 0xFFu : NL == 512 ? 0xFu : 0x3u);
  if constexpr (NL == 4096) {
    static_assert(TS == 1, "the 4096-point plan reads W_4096 directly");
    fft4096<INV, T, LM0, SML>(buf, lt, wlo, whi);
  } else if constexpr (NL == 2048) {
    fft2048<INV, T, TS, LM0, SML>(buf, lt, wlo, whi);
  } else if constexpr (NL == 1024) {
    fft1024<INV, T, TS, LM0, SML>(buf, lt, wlo, whi);
  } else if constexpr (NL == 512) {
    fft512<INV, T, TS, LM0, SML>(buf, lt, wlo, whi);
  } else if constexpr (NL == 256) {
    fft256<INV, T, TS, LM0, SML>(buf, lt, wlo, whi);
  } else {
    static_assert(NL == 128, "compiled lengths: 128 to 4096");
    fft128<INV, T, TS, LM0, SML>(buf, lt, wlo, whi);
  }
}

// The middle of Bluestein's convolution: forward NL-point FFT of an input that vanishes on
// [NL/2, NL), product with bhat (conjugated and reflected for INV), inverse FFT of which only
// [0, NL/2) is stored.  The forward plan is the inverse plan reversed, and the pass where they meet
// does the last forward butterfly, the product and the first inverse butterfly in registers.
template <int NL, int RM, bool INV, int T>
__device__ __forceinline__ void bluestein_mid(double2* buf, int lt, const double2* wlo, const double2* whi,
                                              const double2* __restrict__ bhat) {
  constexpr int NB = NL / RM;
  constexpr int PER = (NB + T - 1) / T;
  double2 v[PER][RM];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) ct_gather<NL, RM, NB, false, 1, 0xFFFFu>(buf, j, v[i], wlo, whi);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
      dft_small<RM, false>(v[i]);   // bin j + NB r in v[i][r]
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        const int q = j + r * NB;
        v[i][r] = cmul(v[i][r], INV ? conjd(bhat[(NL - q) & (NL - 1)]) : bhat[q]);
      }
      dft_small<RM, true>(v[i]);    // first inverse pass (no twiddles), outputs RM j + r
#pragma unroll
      for (int r = 0; r < RM; ++r) buf[lds_pad(RM * j + r)] = v[i][r];
    }
  }
  __syncthreads();
}

// First forward pass of Bluestein's convolution with the input chirp applied on load: input q < n
// times c_q (conjugated for INV), zero on [n, NL); the upper half [NL/2, NL) is not loaded.
template <int NL, int R, bool INV, int T>
__device__ __forceinline__ void bluestein_first(double2* buf, int lt, int n, const double2* __restrict__ chirp) {
  constexpr int NB = NL / R;
  constexpr int PER = (NB + T - 1) / T;
  double2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = j + r * NB;
        v[i][r] = (r < R / 2 && q < n) ? cmul(buf[lds_pad(q)], INV ? conjd(chirp[q]) : chirp[q])
                                       : make_double2(0.0, 0.0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
      dft_small<R, false>(v[i]);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lds_pad(j * R + r)] = v[i][r];
    }
  }
  __syncthreads();
}

// Last inverse pass of Bluestein's convolution with the output chirp applied on store: outputs
// j + r NL/R of the lower half only, output q < n times c_q (conjugated for INV).
template <int NL, int R, bool INV, int T>
__device__ __forceinline__ void bluestein_last(double2* buf, int lt, const double2* wlo, const double2* whi, int n,
                                               const double2* __restrict__ chirp) {
  constexpr int NB = NL / R;
  constexpr int PER = (NB + T - 1) / T;
  double2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) ct_gather<NL, R, NB, true, 1, 0xFFFFu>(buf, j, v[i], wlo, whi);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
      dft_small<R, true>(v[i]);
#pragma unroll
      for (int r = 0; r < R / 2; ++r) {
        const int q = j + r * NB;
        buf[lds_pad(q)] = q < n ? cmul(v[i][r], INV ? conjd(chirp[q]) : chirp[q]) : v[i][r];
      }
    }
  }
  __syncthreads();
}

template <int NL, bool INV, int T>
__device__ __forceinline__ void bluestein_conv(double2* buf, int n, int lt, const double2* wlo, const double2* whi,
                                               const double2* __restrict__ chirp, const double2* __restrict__ bhat) {
  if constexpr (NL == 4096) {   // 16 16 | 16 | 16 16
    bluestein_first<4096, 16, INV, T>(buf, lt, n, chirp);
    ct_pass<4096, 16, 16, false, T>(buf, lt, wlo, whi);
    bluestein_mid<4096, 16, INV, T>(buf, lt, wlo, whi, bhat);
    ct_pass<4096, 16, 16, true, T>(buf, lt, wlo, whi);
    bluestein_last<4096, 16, INV, T>(buf, lt, wlo, whi, n, chirp);
  } else if constexpr (NL == 2048) {   // 4 8 8 | 8 | 8 8 4
    bluestein_first<2048, 4, INV, T>(buf, lt, n, chirp);
    ct_pass<2048, 8, 4, false, T>(buf, lt, wlo, whi);
    ct_pass<2048, 8, 32, false, T>(buf, lt, wlo, whi);
    bluestein_mid<2048, 8, INV, T>(buf, lt, wlo, whi, bhat);
    ct_pass<2048, 8, 8, true, T>(buf, lt, wlo, whi);
    ct_pass<2048, 8, 64, true, T>(buf, lt, wlo, whi);
    bluestein_last<2048, 4, INV, T>(buf, lt, wlo, whi, n, chirp);
  } else if constexpr (NL == 1024) {   // 4 4 8 | 8 | 8 4 4
    bluestein_first<1024, 4, INV, T>(buf, lt, n, chirp);
    ct_pass<1024, 4, 4, false, T>(buf, lt, wlo, whi);
    ct_pass<1024, 8, 16, false, T>(buf, lt, wlo, whi);
    bluestein_mid<1024, 8, INV, T>(buf, lt, wlo, whi, bhat);
    ct_pass<1024, 8, 8, true, T>(buf, lt, wlo, whi);
    ct_pass<1024, 4, 64, true, T>(buf, lt, wlo, whi);
    bluestein_last<1024, 4, INV, T>(buf, lt, wlo, whi, n, chirp);
  } else if constexpr (NL == 512) {   // 8 8 | 8 | 8 8
    bluestein_first<512, 8, INV, T>(buf, lt, n, chirp);
    ct_pass<512, 8, 8, false, T>(buf, lt, wlo, whi);
    bluestein_mid<512, 8, INV, T>(buf, lt, wlo, whi, bhat);
    ct_pass<512, 8, 8, true, T>(buf, lt, wlo, whi);
    bluestein_last<512, 8, INV, T>(buf, lt, wlo, whi, n, chirp);
  } else if constexpr (NL == 256) {   // 4 8 | 8 | 8 4
    bluestein_first<256, 4, INV, T>(buf, lt, n, chirp);
    ct_pass<256, 8, 4, false, T>(buf, lt, wlo, whi);
    bluestein_mid<256, 8, INV, T>(buf, lt, wlo, whi, bhat);
    ct_pass<256, 8, 8, true, T>(buf, lt, wlo, whi);
    bluestein_last<256, 4, INV, T>(buf, lt, wlo, whi, n, chirp);
  } else {   // 4 4 | 8 | 4 4
    static_assert(NL == 128, "Bluestein lengths: 128 to 4096");
    bluestein_first<128, 4, INV, T>(buf, lt, n, chirp);
    ct_pass<128, 4, 4, false, T>(buf, lt, wlo, whi);
    bluestein_mid<128, 8, INV, T>(buf, lt, wlo, whi, bhat);
    ct_pass<128, 4, 8, true, T>(buf, lt, wlo, whi);
    bluestein_last<128, 4, INV, T>(buf, lt, wlo, whi, n, chirp);
  }
}

// Bluestein DFT of length n < NL / 2 in buf[0..n), natural order in and out, over the NL-point
// FFT (tables of W_NL): X_j = c_j sum_q (x_q c_q) conj(c_{j-q}), c_q = exp(-+ i pi q^2 / n); bhat is
// the FFT of conj(c) wrapped to NL, divided by NL.  Ends with a barrier.
// (n < NL / 2: the upper half of the first transform's input is zero and is neither written nor
// read, and only the lower half of the second transform's output is stored)
template <int NL, bool INV, int T>
__device__ __forceinline__ void dft_bluestein(double2* buf, int n, int lt, const double2* wlo,
                                              const double2* whi, const double2* __restrict__ chirp,
                                              const double2* __restrict__ bhat) {
  bluestein_conv<NL, INV, T>(buf, n, lt, wlo, whi, chirp, bhat);
}

// 4095 = 13 * 9 * 7 * 5, in the plain slot layout (element i in slot i, see lds_at)
template <bool INV, int T, typename C2>
__device__ __forceinline__ void dft4095(C2* buf, int lt, const C2* wlo, const C2* whi) {
  constexpr unsigned A = 0xFFFFu;
  ct_pass<4095, 13, 1, INV, T, 1, A, A, false>(buf, lt, wlo, whi);
  ct_pass<4095, 9, 13, INV, T, 1, A, A, false>(buf, lt, wlo, whi);
  ct_pass<4095, 7, 117, INV, T, 1, A, A, false>(buf, lt, wlo, whi);
  ct_pass<4095, 5, 819, INV, T, 1, A, A, false>(buf, lt, wlo, whi);
}

}  // namespace s2let
