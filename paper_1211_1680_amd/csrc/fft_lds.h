// Complex FFTs held in LDS, executed cooperatively by the Tp threads of one problem (a slice
// of a workgroup).  Stockham autosort: every pass reads all of its inputs into registers,
// synchronises, and writes its outputs in natural order, so a single LDS buffer suffices.
// Power-of-two lengths use radix-8 (or 16) passes after one smaller pass; odd lengths use
// radices 3..13.  A thread holds at most VPT values per pass.  Every thread of the workgroup
// must call these functions (they contain __syncthreads()).
#pragma once
#include <hip/hip_runtime.h>

#include "fft_consts.h"

namespace s2let {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// The same for single-precision complex values (the transforms' FP32 instantiations)
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 conjd(float2 a) { return make_float2(a.x, -a.y); }

// Scalar type of a complex type, a complex value from two scalars, and a double2 constant or
// table entry taken to the working precision
template <typename C2> struct CplxTraits;
template <> struct CplxTraits<double2> {
  typedef double S;
  __device__ __forceinline__ static double2 make(double x, double y) { return make_double2(x, y); }
};
template <> struct CplxTraits<float2> {
  typedef float S;
  __device__ __forceinline__ static float2 make(float x, float y) { return make_float2(x, y); }
};
template <typename C2>
__device__ __forceinline__ C2 cplx(double2 a) {
  return CplxTraits<C2>::make((typename CplxTraits<C2>::S)a.x, (typename CplxTraits<C2>::S)a.y);
}
template <typename C2>
__device__ __forceinline__ C2 czero() {
  return CplxTraits<C2>::make(0, 0);
}

// multiply by exp(-i pi/2) = -i (forward) or +i (inverse)
template <bool INV, typename C2>
__device__ __forceinline__ C2 mul_quarter(C2 a) {
  return INV ? CplxTraits<C2>::make(-a.y, a.x) : CplxTraits<C2>::make(a.y, -a.x);
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

// In-register DFT of size R (R = 1, 2, 4, 8, 16) on v[0..R-1], sign -1 (forward) or +1, in the
// precision of the complex type C2.
template <int R, bool INV, typename C2 = double2>
struct SmallDft;

template <bool INV, typename C2>
struct SmallDft<1, INV, C2> {
  __device__ __forceinline__ static void run(C2*) {}
};
template <bool INV, typename C2>
struct SmallDft<2, INV, C2> {
  __device__ __forceinline__ static void run(C2* v) {
    C2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <bool INV, typename C2>
struct SmallDft<4, INV, C2> {
  __device__ __forceinline__ static void run(C2* v) {
    C2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C2 t2 = cadd(v[1], v[3]), t3 = mul_quarter<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};
template <bool INV, typename C2>
struct SmallDft<8, INV, C2> {
  __device__ __forceinline__ static void run(C2* v) {
    C2 e[4] = {v[0], v[2], v[4], v[6]};
    C2 o[4] = {v[1], v[3], v[5], v[7]};
    SmallDft<4, INV, C2>::run(e);
    SmallDft<4, INV, C2>::run(o);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      C2 t = cmul(o[q], cplx<C2>(w16<INV>(2 * q)));
      v[q] = cadd(e[q], t);
      v[q + 4] = csub(e[q], t);
    }
  }
};
template <bool INV, typename C2>
struct SmallDft<16, INV, C2> {
  __device__ __forceinline__ static void run(C2* v) {
    C2 e[8], o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      e[q] = v[2 * q];
      o[q] = v[2 * q + 1];
    }
    SmallDft<8, INV, C2>::run(e);
    SmallDft<8, INV, C2>::run(o);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      C2 t = cmul(o[q], cplx<C2>(w16<INV>(q)));
      v[q] = cadd(e[q], t);
      v[q + 8] = csub(e[q], t);
    }
  }
};

// Sum of v over the T threads of one problem (T a power of two; problems occupy consecutive
// threads of the workgroup), in a fixed order so that equal inputs give equal sums.  Every
// thread of the workgroup must call it (it synchronises when T > 64); scratch holds one value per
// wave of the workgroup (at most 8).
__device__ __forceinline__ double2 problem_sum(double2 v, int T, double2* scratch) {
  const int w = T < 64 ? T : 64;
  for (int off = w >> 1; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  if (T <= 64) return v;
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[wave] = v;
  __syncthreads();
  const int nw = T >> 6, first = (wave / nw) * nw;
  double2 s = make_double2(0.0, 0.0);
  for (int i = 0; i < nw; ++i) {
    s.x += scratch[first + i].x;
    s.y += scratch[first + i].y;
  }
  return s;
}

// W^p (sign chosen by INV) from a two-level table: W^p = lo[p mod 2^loglo] * hi[p >> loglo].
template <bool INV>
__device__ __forceinline__ double2 twiddle(int p, const double2* __restrict__ tlo,
                                           const double2* __restrict__ thi, int loglo) {
  double2 w = cmul(tlo[p & ((1 << loglo) - 1)], thi[p >> loglo]);
  return INV ? conjd(w) : w;
}

// One Stockham pass of radix R over the M values of buf, sub-transform length Ns.
// Butterflies j = lt, lt+Tp, ... < M/R; a thread holds at most VPT values (Tp >= M/VPT).
template <int R, bool INV, int VPT>
__device__ __forceinline__ void stockham_pass(double2* buf, int M, int Ns, int lt, int Tp,
                                              const double2* __restrict__ tlo,
                                              const double2* __restrict__ thi, int loglo, int tsh) {
  constexpr int PER = VPT / R > 0 ? VPT / R : 1;
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
        const double2 w1 = twiddle<INV>((kk * stride) << tsh, tlo, thi, loglo);
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

// Full FFT of length M = 2^logM (unnormalised), sign -1 (INV = false) or +1.  The twiddle
// table holds W_P for P = M << tsh.
template <bool INV, int VPT>
__device__ void fft_pow2(double2* buf, int M, int logM, int lt, int Tp,
                         const double2* __restrict__ tlo, const double2* __restrict__ thi, int loglo,
                         int tsh) {
  // leading pass of radix 2^rem so that the remaining passes have the full radix (16 or 8)
  int Ns = 1;
  const int rem = VPT >= 16 ? (logM & 3) : (logM % 3);
  if (rem == 1) {
    stockham_pass<2, INV, VPT>(buf, M, 1, lt, Tp, tlo, thi, loglo, tsh);
    Ns = 2;
  } else if (rem == 2) {
    stockham_pass<4, INV, VPT>(buf, M, 1, lt, Tp, tlo, thi, loglo, tsh);
    Ns = 4;
  } else if (rem == 3) {
    stockham_pass<8, INV, VPT>(buf, M, 1, lt, Tp, tlo, thi, loglo, tsh);
    Ns = 8;
  }
  if (VPT >= 16) {
    for (; Ns < M; Ns *= 16) stockham_pass<16, INV, VPT>(buf, M, Ns, lt, Tp, tlo, thi, loglo, tsh);
  } else {
    for (; Ns < M; Ns *= 8) stockham_pass<8, INV, VPT>(buf, M, Ns, lt, Tp, tlo, thi, loglo, tsh);
  }
}

// ---- odd radices ----
template <int R>
__device__ __forceinline__ double cosR(int q);
template <int R>
__device__ __forceinline__ double sinR(int q);
#define S2LET_TRIG(R)                                                              \
  template <>                                                                      \
  __device__ __forceinline__ double cosR<R>(int q) { return kCos##R[q]; }          \
  template <>                                                                      \
  __device__ __forceinline__ double sinR<R>(int q) { return kSin##R[q]; }
S2LET_TRIG(3)
S2LET_TRIG(5)
S2LET_TRIG(7)
S2LET_TRIG(9)
S2LET_TRIG(11)
S2LET_TRIG(13)
#undef S2LET_TRIG

// DFT of odd size R on v[0..R-1] using the symmetric pairs (j, R-j):
// X_q = A_q -+ i B_q, X_{R-q} = A_q +- i B_q with A_q = v_0 + sum_j (v_j + v_{R-j}) cos(2 pi j q/R),
// B_q = sum_j (v_j - v_{R-j}) sin(2 pi j q/R).
template <int R, bool INV, typename C2 = double2>
struct OddDft {
  __device__ __forceinline__ static void run(C2* v) {
    typedef typename CplxTraits<C2>::S S;
    constexpr int h = (R - 1) / 2;
    C2 a[h], b[h];
#pragma unroll
    for (int j = 1; j <= h; ++j) {
      a[j - 1] = cadd(v[j], v[R - j]);
      b[j - 1] = csub(v[j], v[R - j]);
    }
    const C2 x0 = v[0];
    C2 sum = x0;
#pragma unroll
    for (int j = 0; j < h; ++j) sum = cadd(sum, a[j]);
    v[0] = sum;
#pragma unroll
    for (int q = 1; q <= h; ++q) {
      S ax = x0.x, ay = x0.y, bx = 0, by = 0;
#pragma unroll
      for (int j = 1; j <= h; ++j) {
        const S c = (S)cosR<R>((j * q) % R), sn = (S)sinR<R>((j * q) % R);
        ax = fma(a[j - 1].x, c, ax);
        ay = fma(a[j - 1].y, c, ay);
        bx = fma(b[j - 1].x, sn, bx);
        by = fma(b[j - 1].y, sn, by);
      }
      if (INV) {   // A + i B, A - i B
        v[q] = CplxTraits<C2>::make(ax - by, ay + bx);
        v[R - q] = CplxTraits<C2>::make(ax + by, ay - bx);
      } else {     // A - i B, A + i B
        v[q] = CplxTraits<C2>::make(ax + by, ay - bx);
        v[R - q] = CplxTraits<C2>::make(ax - by, ay + bx);
      }
    }
  }
};

// One Stockham pass of odd radix R over n values (n divisible by R), sub-transform length Ns.
// Needs Tp >= n/VPT so that a thread has at most MAXB = ceil(VPT/R) butterflies.  Twiddles
// W_n^p come from a two-level table with 64-entry low part.
template <int R, bool INV, int VPT>
__device__ __forceinline__ void stockham_odd_pass(double2* buf, int n, int Ns, int lt, int Tp,
                                                  const double2* __restrict__ tlo,
                                                  const double2* __restrict__ thi) {
  constexpr int MAXB = (VPT + R - 1) / R;
  const int nb = n / R;
  const int stride = n / (Ns * R);
  double2 v[MAXB][R];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int j = lt + i * Tp;
    if (j < nb) {
      const int kk = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[j + r * nb];
      if (kk != 0) {
        const double2 w1 = twiddle<INV>(kk * stride, tlo, thi, 6);
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
  for (int i = 0; i < MAXB; ++i) {
    const int j = lt + i * Tp;
    if (j < nb) {
      OddDft<R, INV>::run(v[i]);
      const int kk = j % Ns;
      const int base = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

}  // namespace s2let
