// The O(k^2 log k) stages of the MW transform (Sect. 2.1; the fast algorithm of the MW
// sampling theorem that Sect. 3.2 calls through SSHT):
//   phi stage:   G_m(theta_t) = (2 pi/n) sum_p f(theta_t, phi_p) e^{-i m phi_p}, n = 2k-1,
//   theta stage: the exact sin(theta) quadrature of the band-limited product, producing the
//                weighted values H'_m(theta_t) that the Legendre contraction sums against,
//   inverse phi: f(theta_t, phi_p) = sum_m F_m(theta_t) e^{i m phi_p}.
// All DFTs of odd length n are Bluestein transforms on a power-of-two LDS FFT of length
// M >= 2n-1.  Real maps are packed two per complex transform (phi stages); in the theta stage
// an even and an odd m are packed into one transform (their extensions have opposite
// symmetry about theta = pi and the even quadrature weight preserves it).
#include "common.h"
#include "fft_lds.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

struct FftArgs {
  int k, n, M, logM, loglo;
  const double2* chirp;
  const double2* bhat;
  const double2* what;
  const double2* tw_lo;
  const double2* tw_hi;
  const double2* hphase;
};

static FftArgs fft_args(const ShtTables& T) {
  FftArgs a;
  a.k = T.k;
  a.n = T.n;
  a.M = T.M;
  a.logM = T.logM;
  a.loglo = T.loglo;
  a.chirp = T.chirp;
  a.bhat = T.bhat;
  a.what = T.what;
  a.tw_lo = T.tw_lo;
  a.tw_hi = T.tw_hi;
  a.hphase = T.hphase;
  return a;
}

// buf <- Bluestein convolution stage: FFT, pointwise product with tab, inverse FFT.
__device__ __forceinline__ void convolve(double2* buf, const FftArgs& A, const double2* __restrict__ tab,
                                         int lt, int Tp) {
  fft_pow2<false>(buf, A.M, A.logM, lt, Tp, A.tw_lo, A.tw_hi, A.loglo);
  for (int q = lt; q < A.M; q += Tp) buf[q] = cmul(buf[q], tab[q]);
  __syncthreads();
  fft_pow2<true>(buf, A.M, A.logM, lt, Tp, A.tw_lo, A.tw_hi, A.loglo);
}

// ------------------------------------------------------------------------------------------
// phi stage, forward.  Problem = (ring t, map pair) for real maps, (ring t, map) for complex.
// Output GT[(t*k + m)*C + c] for m < k.
// ------------------------------------------------------------------------------------------
template <int REAL>
__global__ __launch_bounds__(512) void k_phi_forward(FftArgs A, const double* __restrict__ f, long long map_stride,
                              double* __restrict__ GT, int C, int nb, int used, int nprob) {
  extern __shared__ double2 smem[];
  const FftShape sh = FftShape::of(A.M);
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pl = threadIdx.x / sh.Tp, lt = threadIdx.x % sh.Tp;
  const int p = blk * sh.P + pl;
  const bool valid = p < nprob;
  double2* buf = smem + (size_t)pl * A.M;
  const int k = A.k, n = A.n;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);

  for (int q = lt; q < A.M; q += sh.Tp) {
    double2 z = make_double2(0.0, 0.0);
    if (valid && q < n) {
      if (REAL) {
        z.x = f[(size_t)ma * map_stride + (size_t)t * n + q];
        z.y = hasb ? f[(size_t)(ma + 1) * map_stride + (size_t)t * n + q] : 0.0;
      } else {
        const double2* fc = reinterpret_cast<const double2*>(f);
        z = fc[(size_t)ma * map_stride + (size_t)t * n + q];
      }
      z = cmul(z, A.chirp[q]);
    }
    buf[q] = z;
  }
  __syncthreads();
  convolve(buf, A, A.bhat, lt, sh.Tp);

  const double wphi = 2.0 * M_PI / (double)n;
  if (valid) {
    for (int m = lt; m < k; m += sh.Tp) {
      const double2 zp = cmul(A.chirp[m], buf[m]);                 // Z_m
      const int mm = (m == 0) ? 0 : n - m;
      const double2 zn = cmul(A.chirp[mm], buf[mm]);               // Z_{-m}
      double* row = GT + ((size_t)t * k + m) * C;
      if (REAL) {
        // A_m = (Z_m + conj Z_{-m}) / 2,  B_m = (Z_m - conj Z_{-m}) / (2i)
        const double ax = 0.5 * (zp.x + zn.x), ay = 0.5 * (zp.y - zn.y);
        const double dx = zp.x - zn.x, dy = zp.y + zn.y;
        row[2 * ma] = wphi * ax;
        row[2 * ma + 1] = wphi * ay;
        if (hasb) {
          row[2 * ma + 2] = wphi * 0.5 * dy;
          row[2 * ma + 3] = -wphi * 0.5 * dx;
        }
      } else {
        row[4 * ma] = wphi * zp.x;
        row[4 * ma + 1] = wphi * zp.y;
        row[4 * ma + 2] = (m == 0) ? 0.0 : wphi * zn.x;
        row[4 * ma + 3] = (m == 0) ? 0.0 : wphi * zn.y;
      }
      if (u == 0)
        for (int c = used; c < C; ++c) row[c] = 0.0;
    }
  }
}

// ------------------------------------------------------------------------------------------
// theta stage.  Problem = (m pair (2mu, 2mu+1), series s = column pair (2s, 2s+1)).
// Input GT[(t*k + m)*C + c], output HM[(m*k + t)*C + c].
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_theta(FftArgs A, const double* __restrict__ GT, double* __restrict__ HM, int C,
                        int nprob) {
  extern __shared__ double2 smem[];
  const FftShape sh = FftShape::of(A.M);
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pl = threadIdx.x / sh.Tp, lt = threadIdx.x % sh.Tp;
  const int p = blk * sh.P + pl;
  const bool valid = p < nprob;
  double2* buf = smem + (size_t)pl * A.M;
  const int k = A.k, n = A.n, M = A.M;
  const int ns = C / 2;
  const int mu = valid ? p / ns : 0;
  const int s = valid ? p % ns : 0;
  const int mE = 2 * mu, mO = 2 * mu + 1;
  const bool hasO = mO < k;

  // 1. packed extension g_t = G_E(t) + G_O(t) (t < k);  G_E(n-1-t) - G_O(n-1-t) (t >= k)
  for (int t = lt; t < M; t += sh.Tp) {
    double2 g = make_double2(0.0, 0.0);
    if (valid && t < n) {
      const int tt = (t < k) ? t : n - 1 - t;
      const double sg = (t < k) ? 1.0 : -1.0;
      const double* rE = GT + ((size_t)tt * k + mE) * C + 2 * s;
      g.x = rE[0];
      g.y = rE[1];
      if (hasO) {
        const double* rO = GT + ((size_t)tt * k + mO) * C + 2 * s;
        g.x += sg * rO[0];
        g.y += sg * rO[1];
      }
      g = cmul(g, A.chirp[t]);
    }
    buf[t] = g;
  }
  __syncthreads();
  // 2. D_j = sum_t g_t e^{-2 pi i j t/n} (Bluestein)
  convolve(buf, A, A.bhat, lt, sh.Tp);

  // 3. u_j = e^{-i pi j/n} D_j for |j| <= k-1, placed at j mod M (the 1/n^2 is in what)
  constexpr int MAXV = 8;    // (2k-1)/Tp <= 8 for every FFT shape (M >= 4k-3, Tp = M/16)
  double2 keep[MAXV];
  const int nj = 2 * k - 1;
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * sh.Tp;
    if (idx < nj) {
      const int j = idx - (k - 1);
      const int jj = j < 0 ? j + n : j;
      keep[i] = cmul(A.hphase[idx], cmul(A.chirp[jj], buf[jj]));
    }
  }
  __syncthreads();
  for (int q = lt; q < M; q += sh.Tp) buf[q] = make_double2(0.0, 0.0);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * sh.Tp;
    if (idx < nj) {
      const int j = idx - (k - 1);
      buf[j < 0 ? j + M : j] = keep[i];
    }
  }
  __syncthreads();
  // 4. correlation with the even weight w_e(p) = 2/(1-p^2), p even
  convolve(buf, A, A.what, lt, sh.Tp);

  // 5. v_j' = e^{-i pi j'/n} I_j' with I_j' at index -j' mod M; place at j' mod n (times chirp)
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * sh.Tp;
    if (idx < nj) {
      const int jp = idx - (k - 1);
      const int src = jp > 0 ? M - jp : -jp;
      keep[i] = cmul(A.hphase[idx], buf[src]);
    }
  }
  __syncthreads();
  for (int q = lt; q < M; q += sh.Tp) buf[q] = make_double2(0.0, 0.0);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * sh.Tp;
    if (idx < nj) {
      const int jp = idx - (k - 1);
      const int tp = jp < 0 ? jp + n : jp;
      buf[tp] = cmul(keep[i], A.chirp[tp]);
    }
  }
  __syncthreads();
  // 6. H_t = sum_j' v_j' e^{-2 pi i j' t / n} (Bluestein)
  convolve(buf, A, A.bhat, lt, sh.Tp);

  // 7. fold onto t < k and separate the even and odd m
  if (valid) {
    for (int t = lt; t < k; t += sh.Tp) {
      const double2 h1 = cmul(A.chirp[t], buf[t]);
      double2 he = h1, ho = make_double2(0.0, 0.0);
      if (t < k - 1) {
        const double2 h2 = cmul(A.chirp[n - 1 - t], buf[n - 1 - t]);
        he = cadd(h1, h2);
        ho = csub(h1, h2);
      }
      double* wE = HM + ((size_t)mE * k + t) * C + 2 * s;
      wE[0] = he.x;
      wE[1] = he.y;
      if (hasO) {
        double* wO = HM + ((size_t)mO * k + t) * C + 2 * s;
        wO[0] = ho.x;
        wO[1] = ho.y;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// phi stage, inverse.  Problem = (ring t, map pair) / (ring t, map).  Input FT[(t*k + m)*C + c].
// ------------------------------------------------------------------------------------------
template <int REAL>
__global__ __launch_bounds__(512) void k_phi_inverse(FftArgs A, const double* __restrict__ FT, double* __restrict__ f,
                              long long map_stride, int C, int nb, int nprob) {
  extern __shared__ double2 smem[];
  const FftShape sh = FftShape::of(A.M);
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pl = threadIdx.x / sh.Tp, lt = threadIdx.x % sh.Tp;
  const int p = blk * sh.P + pl;
  const bool valid = p < nprob;
  double2* buf = smem + (size_t)pl * A.M;
  const int k = A.k, n = A.n;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);

  // spectrum Z_m at index m mod n, times conj(chirp) for the +1 sign Bluestein
  for (int q = lt; q < A.M; q += sh.Tp) {
    double2 z = make_double2(0.0, 0.0);
    if (valid && q < n) {
      const bool neg = q >= k;              // q = n - m  <->  m = -(n - q)
      const int m = neg ? n - q : q;
      const double* row = FT + ((size_t)t * k + m) * C;
      if (REAL) {
        double2 a = make_double2(row[2 * ma], row[2 * ma + 1]);
        double2 b = hasb ? make_double2(row[2 * ma + 2], row[2 * ma + 3]) : make_double2(0.0, 0.0);
        if (neg) {
          a = conjd(a);
          b = conjd(b);
        }
        z = make_double2(a.x - b.y, a.y + b.x);   // a + i b
      } else {
        z = neg ? make_double2(row[4 * ma + 2], row[4 * ma + 3]) : make_double2(row[4 * ma], row[4 * ma + 1]);
      }
      z = cmul(z, conjd(A.chirp[q]));
    }
    buf[q] = z;
  }
  __syncthreads();
  // +1-sign Bluestein: conj of the -1 kernel, i.e. FFT with conj(bhat) applied to conj data is
  // avoided by using the identity sum_q z_q e^{+2 pi i pq/n} = conj(sum_q conj(z_q) e^{-...}).
  // Here: buf holds z_q * conj(c_q); convolve with conj(b) via conj(bhat[-j]).
  fft_pow2<false>(buf, A.M, A.logM, lt, sh.Tp, A.tw_lo, A.tw_hi, A.loglo);
  for (int q = lt; q < A.M; q += sh.Tp) {
    const int qn = q == 0 ? 0 : A.M - q;
    buf[q] = cmul(buf[q], conjd(A.bhat[qn]));
  }
  __syncthreads();
  fft_pow2<true>(buf, A.M, A.logM, lt, sh.Tp, A.tw_lo, A.tw_hi, A.loglo);

  if (valid) {
    for (int q = lt; q < n; q += sh.Tp) {
      const double2 v = cmul(conjd(A.chirp[q]), buf[q]);
      if (REAL) {
        f[(size_t)ma * map_stride + (size_t)t * n + q] = v.x;
        if (hasb) f[(size_t)(ma + 1) * map_stride + (size_t)t * n + q] = v.y;
      } else {
        double2* fc = reinterpret_cast<double2*>(f);
        fc[(size_t)ma * map_stride + (size_t)t * n + q] = v;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
template <typename K>
static hipError_t prep(K kernel, size_t lds) {
  static_assert(sizeof(K) > 0, "");
  if (lds > 65536) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  return hipSuccess;
}

hipError_t launch_phi_forward(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                              double* GT, hipStream_t s) {
  const FftArgs A = fft_args(T);
  const FftShape sh = FftShape::of(T.M);
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = T.k * nunits;
  const int nblk = (nprob + sh.P - 1) / sh.P;
  const size_t lds = (size_t)sh.P * T.M * sizeof(double2);
  hipError_t e;
  if (b.reality == S2LET_REAL) {
    if ((e = prep(k_phi_forward<1>, lds)) != hipSuccess) return e;
    k_phi_forward<1><<<nblk, sh.P * sh.Tp, lds, s>>>(A, (const double*)f, map_stride, GT, b.C, b.nb,
                                                    b.used, nprob);
  } else {
    if ((e = prep(k_phi_forward<0>, lds)) != hipSuccess) return e;
    k_phi_forward<0><<<nblk, sh.P * sh.Tp, lds, s>>>(A, (const double*)f, map_stride, GT, b.C, b.nb,
                                                    b.used, nprob);
  }
  return hipGetLastError();
}

hipError_t launch_theta(const ShtTables& T, const Batch& b, const double* GT, double* HM, hipStream_t s) {
  const FftArgs A = fft_args(T);
  const FftShape sh = FftShape::of(T.M);
  const int nprob = ((T.k + 1) / 2) * (b.C / 2);
  const int nblk = (nprob + sh.P - 1) / sh.P;
  const size_t lds = (size_t)sh.P * T.M * sizeof(double2);
  hipError_t e;
  if ((e = prep(k_theta, lds)) != hipSuccess) return e;
  k_theta<<<nblk, sh.P * sh.Tp, lds, s>>>(A, GT, HM, b.C, nprob);
  return hipGetLastError();
}

hipError_t launch_phi_inverse(const ShtTables& T, const Batch& b, const double* FT, void* f,
                              int64_t map_stride, hipStream_t s) {
  const FftArgs A = fft_args(T);
  const FftShape sh = FftShape::of(T.M);
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = T.k * nunits;
  const int nblk = (nprob + sh.P - 1) / sh.P;
  const size_t lds = (size_t)sh.P * T.M * sizeof(double2);
  hipError_t e;
  if (b.reality == S2LET_REAL) {
    if ((e = prep(k_phi_inverse<1>, lds)) != hipSuccess) return e;
    k_phi_inverse<1><<<nblk, sh.P * sh.Tp, lds, s>>>(A, FT, (double*)f, map_stride, b.C, b.nb, nprob);
  } else {
    if ((e = prep(k_phi_inverse<0>, lds)) != hipSuccess) return e;
    k_phi_inverse<0><<<nblk, sh.P * sh.Tp, lds, s>>>(A, FT, (double*)f, map_stride, b.C, b.nb, nprob);
  }
  return hipGetLastError();
}

}  // namespace s2let
