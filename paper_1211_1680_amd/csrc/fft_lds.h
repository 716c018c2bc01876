// Power-of-two complex FFT held in LDS, executed cooperatively by the Tp threads of one
// problem (a slice of a workgroup).  Stockham autosort: every pass reads all of its inputs
// into registers, synchronises, and writes its outputs in natural order, so a single LDS
// buffer of M values suffices.  Radix-16 passes, preceded by one radix-2/4/8 pass when
// log2(M) is not a multiple of 4.  Every thread of the workgroup must call these functions
// (they contain __syncthreads()).
#pragma once
#include <hip/hip_runtime.h>

namespace s2let {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// multiply by exp(-i pi/2) = -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 mul_quarter(double2 a) {
  return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// cos / sin of 2 pi q / 16, q = 0..7
__device__ __forceinline__ double cos16(int q) {
  constexpr double c[8] = {1.0,
                           0.92387953251128675613,
                           0.70710678118654752440,
                           0.38268343236508977173,
                           0.0,
                           -0.38268343236508977173,
                           -0.70710678118654752440,
                           -0.92387953251128675613};
  return c[q];
}
__device__ __forceinline__ double sin16(int q) {
  constexpr double s[8] = {0.0,
                           0.38268343236508977173,
                           0.70710678118654752440,
                           0.92387953251128675613,
                           1.0,
                           0.92387953251128675613,
                           0.70710678118654752440,
                           0.38268343236508977173};
  return s[q];
}
// exp(-+ 2 pi i q / 16)
template <bool INV>
__device__ __forceinline__ double2 w16(int q) {
  return make_double2(cos16(q), INV ? sin16(q) : -sin16(q));
}

// In-register DFT of size R (R = 1, 2, 4, 8, 16) on v[0..R-1], sign -1 (forward) or +1.
template <int R, bool INV>
struct SmallDft;

template <bool INV>
struct SmallDft<1, INV> {
  __device__ __forceinline__ static void run(double2*) {}
};
template <bool INV>
struct SmallDft<2, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <bool INV>
struct SmallDft<4, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    double2 t2 = cadd(v[1], v[3]), t3 = mul_quarter<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};
template <bool INV>
struct SmallDft<8, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    SmallDft<4, INV>::run(e);
    SmallDft<4, INV>::run(o);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double2 t = cmul(o[q], w16<INV>(2 * q));
      v[q] = cadd(e[q], t);
      v[q + 4] = csub(e[q], t);
    }
  }
};
template <bool INV>
struct SmallDft<16, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    double2 e[8], o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      e[q] = v[2 * q];
      o[q] = v[2 * q + 1];
    }
    SmallDft<8, INV>::run(e);
    SmallDft<8, INV>::run(o);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double2 t = cmul(o[q], w16<INV>(q));
      v[q] = cadd(e[q], t);
      v[q + 8] = csub(e[q], t);
    }
  }
};

// W_M^p (sign chosen by INV) from the two-level table.
template <bool INV>
__device__ __forceinline__ double2 twiddle(int p, const double2* __restrict__ tlo,
                                           const double2* __restrict__ thi, int loglo) {
  double2 w = cmul(tlo[p & ((1 << loglo) - 1)], thi[p >> loglo]);
  return INV ? conjd(w) : w;
}

// One Stockham pass of radix R over the M values of buf, sub-transform length Ns.
// Butterflies j = lt, lt+Tp, ... < M/R; at most 16/R per thread.
template <int R, bool INV>
__device__ __forceinline__ void stockham_pass(double2* buf, int M, int Ns, int lt, int Tp,
                                              const double2* __restrict__ tlo,
                                              const double2* __restrict__ thi, int loglo) {
  constexpr int PER = 16 / R;
  const int nb = M / R;
  const int stride = M / (Ns * R);
  double2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * Tp;
    if (j < nb) {
      const int kk = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[j + r * nb];
      if (Ns > 1 && kk != 0) {
        const double2 w1 = twiddle<INV>(kk * stride, tlo, thi, loglo);
        double2 w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[i][r] = cmul(v[i][r], w);
          if (r + 1 < R) w = cmul(w, w1);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * Tp;
    if (j < nb) {
      SmallDft<R, INV>::run(v[i]);
      const int kk = j & (Ns - 1);
      const int base = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

// Full FFT of length M = 2^logM (unnormalised), sign -1 (INV = false) or +1.
template <bool INV>
__device__ void fft_pow2(double2* buf, int M, int logM, int lt, int Tp,
                         const double2* __restrict__ tlo, const double2* __restrict__ thi, int loglo) {
  int Ns = 1;
  const int rem = logM & 3;
  if (rem == 1) {
    stockham_pass<2, INV>(buf, M, 1, lt, Tp, tlo, thi, loglo);
    Ns = 2;
  } else if (rem == 2) {
    stockham_pass<4, INV>(buf, M, 1, lt, Tp, tlo, thi, loglo);
    Ns = 4;
  } else if (rem == 3) {
    stockham_pass<8, INV>(buf, M, 1, lt, Tp, tlo, thi, loglo);
    Ns = 8;
  }
  for (; Ns < M; Ns *= 16) stockham_pass<16, INV>(buf, M, Ns, lt, Tp, tlo, thi, loglo);
}

// Problems per workgroup and threads per problem for an FFT of length M: every pass gives a
// thread at most 16 values; a workgroup holds at most 4096 values (64 KiB), except M = 8192.
struct FftShape {
  int P;    // problems per workgroup
  int Tp;   // threads per problem
  __host__ __device__ static FftShape of(int M) {
    FftShape s;
    s.Tp = M >= 16 ? M / 16 : 1;
    if (M >= 4096) {
      s.P = 1;
    } else {
      s.P = 4096 / M;
      if (s.P * s.Tp > 256) s.P = 256 / s.Tp;
    }
    return s;
  }
};

// Workgroups are handed to the 8 XCDs round-robin; give consecutive logical indices to the
// same XCD so that problems writing neighbouring columns of a row share an L2.
__device__ __forceinline__ int xcd_swizzle(int b, int nblk) {
  constexpr int X = 8;
  const int per = nblk / X, rem = nblk % X;
  const int x = b % X, idx = b / X;
  return x * per + (x < rem ? x : rem) + idx;
}

}  // namespace s2let
