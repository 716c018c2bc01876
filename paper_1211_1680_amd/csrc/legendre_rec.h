// Device helpers of the Legendre kernels: the scaled three-term recursion in Reinsch's
// difference form with per-lane binary exponents (see kernels_legendre.hip for the method).
#pragma once
#include "common.h"

namespace s2let {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// s^m = mant * 2^e with mant in [0.5, 1) (or 0), by binary powering.
__device__ __forceinline__ double pow_scaled(double s, int m, int* e_out) {
  int be;
  double b = frexp(s, &be);
  double r = 1.0;
  int re = 0;
  while (m) {
    if (m & 1) {
      int ex;
      r = frexp(r * b, &ex);
      re += ex + be;
    }
    m >>= 1;
    if (m) {
      int ex;
      b = frexp(b * b, &ex);
      be = 2 * be + ex;
    }
  }
  *e_out = re;
  return r;
}

__device__ __forceinline__ int exponent_of(double v) {
  int ex;
  frexp(v, &ex);
  return ex;
}

// Moves magnitude between (z1, z2) and e while e < 0 (keeps z1 in a safe range).
__device__ __forceinline__ void renorm(double& z1, double& z2, int& e) {
  if (e < 0) {
    const int ex = exponent_of(z1);
    if (ex > 60 || ex >= -e) {
      const int sh = ex < -e ? ex : -e;
      z1 = ldexp(z1, -sh);
      z2 = ldexp(z2, -sh);
      e += sh;
    }
  }
}

__device__ __forceinline__ bool negligible(double z1, double z2, int e) {
  const double a = fmax(fabs(z1), fabs(z2));
  return a == 0.0 || e + exponent_of(a) < -1100;
}

// value of v in lane l (l uniform), through two scalar registers
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __hiloint2double(hi, lo);
}

// Recursion coefficients of one chunk of LC degrees starting at row i0 of column m (len rows
// below the band-limit): lane j < LC holds alpha, lane LC + j holds beta, zero past the end
// (alpha = beta = 0 keeps the state finite).  One vector load per lane replaces 2 LC scalar
// loads whose latency would otherwise sit in every step of the recursion.
template <int LC>
__device__ __forceinline__ double chunk_coef(const double* __restrict__ am, const double* __restrict__ bm,
                                             int i0, int len, int lane) {
  const bool isb = lane >= LC;
  const int i = i0 + (isb ? lane - LC : lane);
  const double* p = isb ? bm : am;
  return (lane < 2 * LC && i < len) ? p[i] : 0.0;
}

// Where a step's recursion coefficients (alpha_l, beta_l) come from.  RegCoef: one register per
// lane (lane j < LC holds alpha, lane LC + j beta, as chunk_coef loads them), broadcast with
// v_readlane (four per step, plus two moves to put beta in a vector register).  LdsCoef: a
// wave-private LDS copy of the chunk as (alpha, beta) pairs, one broadcast 16-byte LDS load per
// step (every lane the same address) and no further vector instructions.
template <int LC>
struct RegCoef {
  double cf;
  __device__ __forceinline__ double2 operator()(int j) const {
    return make_double2(readlane_d(cf, j), readlane_d(cf, LC + j));
  }
};
struct LdsCoef {
  const double2* cfl;
  __device__ __forceinline__ double2 operator()(int j) const { return cfl[j]; }
};

// Writes one chunk's coefficients, as chunk_coef loaded them, to a wave-private LDS buffer of
// LC (alpha, beta) pairs; the caller orders it before the reads with wave_lds_sync().
template <int LC>
__device__ __forceinline__ void stage_coef(double2* cfl, double cf, int lane) {
  if (lane < 2 * LC) reinterpret_cast<double*>(cfl)[2 * (lane % LC) + (lane >= LC ? 1 : 0)] = cf;
}

// One chunk of the difference recursion: degrees l0 .. l0 + LC - 1; the z value of step j
// (scaled by 2^e) goes to sink(j, value).  The state enters as (z_{l0-1}, E_{l0-1}).  SIGN = +1 / -1: every lane of the
// wave is in the northern / southern hemisphere (s uniform, folded into the operations);
// SIGN = 0: mixed.  SCALED = false: every lane has e = 0 (no scaling, no renormalisation).
template <int LC, int SIGN, bool SCALED, typename Coef, typename Sink>
__device__ __forceinline__ void recur_steps(const Coef& coef, double u, double sg, double& z1, double& z2, int& e,
                                            Sink& sink) {
#pragma unroll
  for (int j = 0; j < LC; ++j) {
    const double2 ab = coef(j);
    const double g = fma(ab.x, u, ab.y);
    if (SIGN > 0) {
      z2 = fma(g, z1, z2);
      z1 = z1 + z2;
    } else if (SIGN < 0) {
      z2 = fma(-g, z1, -z2);
      z1 = z2 - z1;
    } else {
      z2 = sg * fma(g, z1, z2);
      z1 = fma(sg, z1, z2);
    }
    sink(j, SCALED ? ldexp(z1, e) : z1);
    if (SCALED && (j & 7) == 7) renorm(z1, z2, e);
  }
}

template <int LC, typename Coef, typename Sink>
__device__ __forceinline__ void recur_chunk_with(const Coef& coef, double u, double sg, double& z1, double& z2,
                                                 int& e, Sink&& sink) {
  const bool scaled = !__all(e == 0);
  if (__all(sg > 0.0)) {
    if (scaled)
      recur_steps<LC, 1, true>(coef, u, sg, z1, z2, e, sink);
    else
      recur_steps<LC, 1, false>(coef, u, sg, z1, z2, e, sink);
  } else if (__all(sg < 0.0)) {
    if (scaled)
      recur_steps<LC, -1, true>(coef, u, sg, z1, z2, e, sink);
    else
      recur_steps<LC, -1, false>(coef, u, sg, z1, z2, e, sink);
  } else {
    recur_steps<LC, 0, true>(coef, u, sg, z1, z2, e, sink);
  }
}

template <int LC, typename Sink>
__device__ __forceinline__ void recur_chunk(double cf, double u, double sg, double& z1, double& z2, int& e,
                                            Sink&& sink) {
  recur_chunk_with<LC>(RegCoef<LC>{cf}, u, sg, z1, z2, e, sink);
}

// The same with the chunk's coefficients staged in LDS (see LdsCoef).
template <int LC, typename Sink>
__device__ __forceinline__ void recur_chunk_lds(const double2* cfl, double u, double sg, double& z1, double& z2,
                                                int& e, Sink&& sink) {
  recur_chunk_with<LC>(LdsCoef{cfl}, u, sg, z1, z2, e, sink);
}

// Start of the recursion one degree early: z_{m-1} = 0 and E = s z_m, so that the first step
// (alpha_m = 0, beta_m = -2 in the tables) yields z_m and E_m = z_m.
__device__ __forceinline__ void recur_start(double cmm, double s, double sg, int m, double& z1, double& z2,
                                            int& e) {
  double zm = cmm * pow_scaled(s, m, &e);
  if (e > 0) {
    zm = ldexp(zm, e);
    e = 0;
  }
  z1 = 0.0;
  z2 = sg * zm;
}

// orders this wave's LDS writes before its later reads (and the reverse) without a block barrier
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace s2let
