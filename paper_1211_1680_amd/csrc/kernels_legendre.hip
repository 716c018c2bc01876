// Legendre contraction of the MW transform, the O(k^3) part (Sect. 3.2):
//   synthesis (Eq. (1)):  F_m(theta_t) = sum_{l=m}^{k-1} f_lm lambda_lm(theta_t)
//   analysis  (Eq. (2)):  f_lm = sum_{t<k} lambda_lm(theta_t) H'_m(theta_t)
// batched over C data columns (maps x {re, im} x {+m, -m}).
//
// lambda_lm is never stored: it is regenerated per (m, theta) by the three-term recursion,
// in FP64, in the scaled form  z_l = alpha_l x z_{l-1} - z_{l-2}  (x = cos theta), with
// lambda_lm = d_lm z_lm; the d_lm are folded into the coefficients by the pack / unpack /
// tiling kernels.  Start: z_m = lambda_mm = c_m sin^m(theta), z_{m-1} = 0.
// Near the poles (x -> +-1) the plain recursion loses about l^2 ulps (1e-10 at l = 2047), so it
// runs in Reinsch's difference form: with s = sign(x), u = |x| - 1 = -2 sin^2(theta'/2) and
// beta_l = alpha_l - 2 both tabulated exactly,
//   g = alpha_l u + beta_l  (= alpha_l |x| - 2),  E_l = s (E_{l-1} + g z_{l-1}),  z_l = E_l + s z_{l-1},
// E_m = z_m; the small quantity g is formed without cancellation.  Near the poles lambda_mm underflows far below the double
// range (2^-17000 at m = 2047), so each lane carries an integer exponent e (value = z 2^e),
// renormalised every 8 steps; while every lane of a wave is below 2^-1100 the contraction
// is skipped, and once every lane has e = 0 the plain recursion runs.
#include "common.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

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

// ------------------------------------------------------------------------------------------
// Synthesis: one lane per theta_t, 4 waves per block; a block handles the m pair
// (pair, k-1-pair) so every block does k+1 rows of work.  The coefficient rows S[l][0..C)
// are uniform across the wave and come through the scalar cache.
// ------------------------------------------------------------------------------------------
template <int C>
__global__ __launch_bounds__(256) void k_legendre_inv(const double* __restrict__ S, double* __restrict__ FT,
                                                      const double* __restrict__ alpha,
                                                      const double* __restrict__ beta,
                                                      const double* __restrict__ cm,
                                                      const double* __restrict__ ut,
                                                      const double* __restrict__ sx,
                                                      const double* __restrict__ st, int k, int Lt,
                                                      int ntb, unsigned long long* __restrict__ counter) {
  const int pair = blockIdx.x / ntb;
  const int tb = blockIdx.x % ntb;
  const int t = tb * 256 + threadIdx.x;
  const bool valid = t < k;
  const double u = valid ? ut[t] : -1.0;
  const double sg = valid ? sx[t] : 1.0;
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ Sm = S + tri_off(k, m) * C;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;

    int e;
    double z1 = cm[m] * pow_scaled(s, m, &e);
    if (e > 0) {
      z1 = ldexp(z1, e);
      e = 0;
    }
    double z2 = z1;   // E_m = z_m
    {
      const double w = ldexp(z1, e);
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = fma(Sm[c], w, acc[c]);
    }
    int l = m + 1;
    // (a) every lane negligible: advance the recursion only
    while (l + 8 <= k && __all(!valid || negligible(z1, z2, e))) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double g = fma(am[l + i - m], u, bm[l + i - m]);
        z2 = sg * fma(g, z1, z2);
        z1 = fma(sg, z1, z2);
      }
      renorm(z1, z2, e);
      l += 8;
    }
    if (counter != nullptr) {
      // rows contracted by this wave times its valid lanes (one vector atomic per wave)
      const unsigned long long nv = __popcll(__ballot(valid));
      if ((threadIdx.x & 63) == __ffsll((unsigned long long)__ballot(valid)) - 1 && nv > 0)
        atomicAdd(counter, (unsigned long long)(k - l + 1) * nv);
    }
    // (b) scaled lanes present
    while (l + 8 <= k && !__all(!valid || e == 0)) {
#pragma unroll 1
      for (int i = 0; i < 8; ++i) {
        const double g = fma(am[l + i - m], u, bm[l + i - m]);
        z2 = sg * fma(g, z1, z2);
        z1 = fma(sg, z1, z2);
        const double w = ldexp(z1, e);
        const double* __restrict__ row = Sm + (size_t)(l + i - m) * C;
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = fma(row[c], w, acc[c]);
      }
      renorm(z1, z2, e);
      l += 8;
    }
    // (c) plain recursion
#pragma unroll 1
    for (; l < k; ++l) {
      {
        const int i = 0;
        const double g = fma(am[l + i - m], u, bm[l + i - m]);
        z2 = sg * fma(g, z1, z2);
        z1 = fma(sg, z1, z2);
        const double* __restrict__ row = Sm + (size_t)(l + i - m) * C;
        const double w = ldexp(z1, e);   // e == 0 except in the last partial chunk
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = fma(row[c], w, acc[c]);
      }
    }
    if (valid) {
      double* out = FT + ((size_t)t * k + m) * C;
#pragma unroll
      for (int c = 0; c < C; ++c) out[c] = acc[c];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Analysis: D[c][l] = sum_t H'[t][c] z_l(theta_t) on the FP64 matrix cores
// (v_mfma_f64_16x16x4: A = 16 columns x 4 thetas, B = 4 thetas x 16 degrees).
// Block = 8 waves, one m pair.  Wave w owns theta tiles w, w+8, ... of 64 thetas and keeps
// their recursion state in registers; per chunk of 32 degrees it writes its tile of z values
// to LDS, multiplies, and the eight partial sums are reduced through LDS.
// ------------------------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int FWD_NW = 8;       // waves per block
constexpr int FWD_NTMAX = 4;    // theta tiles per wave: k <= 4 * 8 * 64 = 2048
constexpr int FWD_LC = 32;      // degrees per chunk
constexpr int FWD_ZS = 65;      // padded LDS row (doubles)

template <int C>
__global__ __launch_bounds__(512) void k_legendre_fwd(const double* __restrict__ HM, double* __restrict__ R,
                                                      const double* __restrict__ alpha,
                                                      const double* __restrict__ beta,
                                                      const double* __restrict__ cm,
                                                      const double* __restrict__ ut,
                                                      const double* __restrict__ sx,
                                                      const double* __restrict__ st, int k, int Lt,
                                                      unsigned long long* __restrict__ counter) {
  constexpr int CT = C >= 16 ? C / 16 : 1;
  unsigned long long retained = 0;   // (l, theta) pairs multiplied by this wave
  __shared__ double Z[FWD_NW][FWD_LC][FWD_ZS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int pair = blockIdx.x;
  const int ntiles = (k + 63) / 64;
  const int NT = (ntiles + FWD_NW - 1) / FWD_NW;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  const int li = lane & 15, lq = lane >> 4;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Hm = HM + (size_t)m * k * C;
    double z1[FWD_NTMAX], z2[FWD_NTMAX], us[FWD_NTMAX], sgs[FWD_NTMAX];
    int ee[FWD_NTMAX];
#pragma unroll
    for (int i = 0; i < FWD_NTMAX; ++i) {
      z1[i] = 0.0;
      z2[i] = 0.0;
      us[i] = -1.0;
      sgs[i] = 1.0;
      ee[i] = 0;
      if (i < NT) {
        const int t = (w + FWD_NW * i) * 64 + lane;
        if (t < k) {
          int e;
          z1[i] = cm[m] * pow_scaled(st[t], m, &e);
          if (e > 0) {
            z1[i] = ldexp(z1[i], e);
            e = 0;
          }
          z2[i] = z1[i];   // E_m = z_m
          ee[i] = e;
          us[i] = ut[t];
          sgs[i] = sx[t];
        }
      }
    }

    for (int l0 = m; l0 < k; l0 += FWD_LC) {
      v4d acc[2][CT];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

#pragma unroll
      for (int i = 0; i < FWD_NTMAX; ++i) {
        if (i < NT) {
          const int tile = w + FWD_NW * i;
          // z values for degrees l0 .. l0+31 at this lane's theta
          const bool skip = __all(negligible(z1[i], z2[i], ee[i]) || tile * 64 + lane >= k);
#pragma unroll
          for (int j = 0; j < FWD_LC; ++j) {
            const int l = l0 + j;
            double v = 0.0;
            if (l < k) {
              if (l > m) {
                const double g = fma(am[l - m], us[i], bm[l - m]);
                z2[i] = sgs[i] * fma(g, z1[i], z2[i]);
                z1[i] = fma(sgs[i], z1[i], z2[i]);
              }
              v = ldexp(z1[i], ee[i]);
            }
            Z[w][j][lane] = v;
            if ((j & 7) == 7) renorm(z1[i], z2[i], ee[i]);
          }
          __syncthreads();
          if (!skip) {
            const int nl = (k - l0) < FWD_LC ? (k - l0) : FWD_LC;
            const int nt = (k - tile * 64) < 64 ? (k - tile * 64) : 64;
            retained += (unsigned long long)nl * (unsigned long long)nt;
#pragma unroll 4
            for (int kk = 0; kk < 16; ++kk) {
              const int tl = 4 * kk + lq;
              const int tg = tile * 64 + tl;
              double a[CT];
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
                const int c = ct * 16 + li;
                a[ct] = (tg < k && c < C) ? Hm[(size_t)tg * C + c] : 0.0;
              }
#pragma unroll
              for (int lt2 = 0; lt2 < 2; ++lt2) {
                const double bv = Z[w][lt2 * 16 + li][tl];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
                  acc[lt2][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ct], bv, acc[lt2][ct], 0, 0, 0);
              }
            }
          }
          __syncthreads();
        }
      }
      // reduce the waves' partial sums: red[w][l][c]
      double* red = &Z[0][0][0];
#pragma unroll
      for (int lt2 = 0; lt2 < 2; ++lt2)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // result register v of lane l holds row (l / 16) + 4 v, column l % 16
            const int c = ct * 16 + lq + 4 * v;
            const int lloc = lt2 * 16 + li;
            if (c < C) red[((size_t)w * FWD_LC + lloc) * C + c] = acc[lt2][ct][v];
          }
      __syncthreads();
      for (int idx = threadIdx.x; idx < FWD_LC * C; idx += FWD_NW * 64) {
        const int lloc = idx / C, c = idx % C;
        const int l = l0 + lloc;
        if (l < k) {
          double sum = 0.0;
#pragma unroll
          for (int ww = 0; ww < FWD_NW; ++ww) sum += red[(ww * FWD_LC + lloc) * C + c];
          R[(tri_off(k, m) + (l - m)) * C + c] = sum;
        }
      }
      __syncthreads();
    }
  }
  if (counter != nullptr && lane == 0 && retained > 0) atomicAdd(counter, retained);
}

// ------------------------------------------------------------------------------------------
template <int C>
static hipError_t inv_c(const ShtTables& T, const LegTables& G, const double* S, double* FT,
                        unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  const int ntb = (k + 255) / 256;
  const int npairs = (k + 1) / 2;
  k_legendre_inv<C><<<npairs * ntb, 256, 0, s>>>(S, FT, G.alpha, G.beta, G.cm, T.ut, T.sx, T.st, k, G.Lt,
                                                 ntb, counter);
  return hipGetLastError();
}

template <int C>
static hipError_t fwd_c(const ShtTables& T, const LegTables& G, const double* HM, double* R,
                        unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  const int npairs = (k + 1) / 2;
  k_legendre_fwd<C><<<npairs, FWD_NW * 64, 0, s>>>(HM, R, G.alpha, G.beta, G.cm, T.ut, T.sx, T.st, k, G.Lt,
                                                   counter);
  return hipGetLastError();
}

hipError_t launch_legendre_inverse(const ShtTables& T, const LegTables& G, const Batch& b,
                                   const double* S, double* FT, int precision,
                                   unsigned long long* counter, hipStream_t s) {
  (void)precision;
  switch (b.C) {
    case 2: return inv_c<2>(T, G, S, FT, counter, s);
    case 4: return inv_c<4>(T, G, S, FT, counter, s);
    case 8: return inv_c<8>(T, G, S, FT, counter, s);
    case 16: return inv_c<16>(T, G, S, FT, counter, s);
    case 32: return inv_c<32>(T, G, S, FT, counter, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_legendre_forward(const ShtTables& T, const LegTables& G, const Batch& b,
                                   const double* HM, double* R, int precision,
                                   unsigned long long* counter, hipStream_t s) {
  (void)precision;
  if (T.k > FWD_NTMAX * FWD_NW * 64) return hipErrorInvalidValue;
  switch (b.C) {
    case 2: return fwd_c<2>(T, G, HM, R, counter, s);
    case 4: return fwd_c<4>(T, G, HM, R, counter, s);
    case 8: return fwd_c<8>(T, G, HM, R, counter, s);
    case 16: return fwd_c<16>(T, G, HM, R, counter, s);
    case 32: return fwd_c<32>(T, G, HM, R, counter, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace s2let
