// The O(k^2 log k) stages of the MW transform (Sect. 2.1; the fast algorithm of the MW
// sampling theorem that Sect. 3.2 calls through SSHT):
//   phi stage:   G_m(theta_t) = (2 pi/n) sum_p f(theta_t, phi_p) e^{-i m phi_p}, n = 2k-1,
//   theta stage: the exact sin(theta) quadrature of the band-limited product, producing the
//                weighted values H'_m(theta_t) that the Legendre contraction sums against,
//   inverse phi: f(theta_t, phi_p) = sum_m F_m(theta_t) e^{i m phi_p}.
// DFTs of odd length n run in LDS: a Stockham mixed-radix transform (radices 3..13) when n
// factors into them (n = 4095 at k = 2048), otherwise Bluestein's chirp transform on a
// power-of-two FFT of length M >= 2n-1.  Real maps are packed two per complex transform (phi
// stages); in the theta stage an even and an odd m share one transform (their extensions have
// opposite symmetry about theta = pi, which the even part of the quadrature weight preserves).
// The weight correlation splits by the parity of the frequency, since the even weight w_e(p)
// vanishes for odd p: two circular correlations of length Nc >= 2k-1 instead of one of 4k-3.
#include "common.h"
#include "fft_lds.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

struct FftArgs {
  int k, n;
  int mixed;                 // 1: Stockham mixed radix over the radices in rad_code
  int nrad;
  unsigned int rad_code;     // radix s in bits [4s, 4s+4)
  const double2* twn_lo;     // W_n^p = lo[p & 63] * hi[p >> 6]
  const double2* twn_hi;
  int M, logM;               // Bluestein length (when not mixed)
  const double2* chirp;      // exp(-i pi q^2/n)
  const double2* bhat;       // FFT_M(conj chirp, wrapped) / M
  int Nc, logNc;             // correlation length
  const double2* khat0;      // FFT_Nc of the even-frequency weight kernel / (Nc n^2)
  const double2* khat1;      // same, odd frequencies
  const double2* tw_lo;      // W_P two-level table, P = 2^logP the largest power of two used
  const double2* tw_hi;
  int loglo, logP;
  const double2* hphase;     // exp(-i pi j/n), j in [-(k-1), k-1]
  const double* pole;        // pole column of the odd-parity theta operator
  int T, P, buf;             // threads per problem, problems per block, LDS values per problem
};

// The two-level twiddle tables (at most TWMAX entries each at the supported band-limits) copied
// into LDS once per block: each FFT pass reads them after its LDS loads, and from global memory
// that read put a memory latency into every pass.  The caller synchronises before the first pass.
constexpr int TWMAX = 128;
__device__ __forceinline__ FftArgs stage_twiddles(const FftArgs& A, double2 (*tw)[TWMAX]) {
  FftArgs L = A;
  const int nlo = 1 << A.loglo, nhi = (1 << A.logP) >> A.loglo, nnhi = (A.n + 63) / 64;
  if (nlo <= TWMAX && nhi <= TWMAX && nnhi <= TWMAX) {
    for (int i = threadIdx.x; i < TWMAX; i += blockDim.x) {
      if (i < nlo) tw[0][i] = A.tw_lo[i];
      if (i < nhi) tw[1][i] = A.tw_hi[i];
      if (i < 64) tw[2][i] = A.twn_lo[i];
      if (i < nnhi) tw[3][i] = A.twn_hi[i];
    }
    L.tw_lo = tw[0];
    L.tw_hi = tw[1];
    L.twn_lo = tw[2];
    L.twn_hi = tw[3];
  }
  return L;
}

// In-place DFT of length n of buf[0..n) (natural order in and out), sign -1 or +1 (INV).
template <bool INV, int VPT>
__device__ void dft_odd(double2* buf, const FftArgs& A, int lt) {
  if (A.mixed) {
    int Ns = 1;
    for (int s = 0; s < A.nrad; ++s) {
      const int R = (A.rad_code >> (4 * s)) & 15;
      switch (R) {
        case 3: stockham_odd_pass<3, INV, VPT>(buf, A.n, Ns, lt, A.T, A.twn_lo, A.twn_hi); break;
        case 5: stockham_odd_pass<5, INV, VPT>(buf, A.n, Ns, lt, A.T, A.twn_lo, A.twn_hi); break;
        case 7: stockham_odd_pass<7, INV, VPT>(buf, A.n, Ns, lt, A.T, A.twn_lo, A.twn_hi); break;
        case 9: stockham_odd_pass<9, INV, VPT>(buf, A.n, Ns, lt, A.T, A.twn_lo, A.twn_hi); break;
        case 11: stockham_odd_pass<11, INV, VPT>(buf, A.n, Ns, lt, A.T, A.twn_lo, A.twn_hi); break;
        default: stockham_odd_pass<13, INV, VPT>(buf, A.n, Ns, lt, A.T, A.twn_lo, A.twn_hi); break;
      }
      Ns *= R;
    }
    return;
  }
  // Bluestein: X_j = c_j sum_q (x_q c_q) conj(c_{j-q}) with c_q = exp(-+ i pi q^2 / n)
  // (the table loops are unrolled over VPT, T VPT >= M, so that their loads issue together)
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int q = lt + i * A.T;
    if (q < A.M) {
      double2 v = make_double2(0.0, 0.0);
      if (q < A.n) v = cmul(buf[q], INV ? conjd(A.chirp[q]) : A.chirp[q]);
      buf[q] = v;
    }
  }
  __syncthreads();
  fft_pow2<false, VPT>(buf, A.M, A.logM, lt, A.T, A.tw_lo, A.tw_hi, A.loglo, A.logP - A.logM);
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int q = lt + i * A.T;
    if (q < A.M) buf[q] = cmul(buf[q], INV ? conjd(A.bhat[(A.M - q) & (A.M - 1)]) : A.bhat[q]);
  }
  __syncthreads();
  fft_pow2<true, VPT>(buf, A.M, A.logM, lt, A.T, A.tw_lo, A.tw_hi, A.loglo, A.logP - A.logM);
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int q = lt + i * A.T;
    if (q < A.n) buf[q] = cmul(buf[q], INV ? conjd(A.chirp[q]) : A.chirp[q]);
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------------------
// phi stage, forward.  Problem = (ring t, map pair) for real maps, (ring t, map) for complex.
// Output GT[(t*k + m)*C + c] for m < k.
// ------------------------------------------------------------------------------------------
template <int REAL, int VPT>
__global__ __launch_bounds__(512) void k_phi_forward(FftArgs Ain, const double* __restrict__ f,
                                                     long long map_stride, double* __restrict__ GT,
                                                     int C, int nb, int used, int nprob) {
  extern __shared__ double2 smem[];
  __shared__ double2 s_tw[4][TWMAX];
  const FftArgs A = stage_twiddles(Ain, s_tw);
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pl = threadIdx.x / A.T, lt = threadIdx.x % A.T;
  const int p = blk * A.P + pl;
  const bool valid = p < nprob;
  double2* buf = smem + (size_t)pl * A.buf;
  const int k = A.k, n = A.n;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);

  {
    // every load of the ring is issued before the first store (VPT >= n / T)
    double2 z[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int q = lt + i * A.T;
      const size_t off = (size_t)t * n + (q < n ? q : 0);
      if (REAL) {
        z[i].x = f[(size_t)ma * map_stride + off];
        z[i].y = hasb ? f[(size_t)(ma + 1) * map_stride + off] : 0.0;
      } else {
        z[i] = reinterpret_cast<const double2*>(f)[(size_t)ma * map_stride + off];
      }
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int q = lt + i * A.T;
      if (q < n) buf[q] = valid ? z[i] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  dft_odd<false, VPT>(buf, A, lt);

  const double wphi = 2.0 * M_PI / (double)n;
  if (valid) {
    for (int m = lt; m < k; m += A.T) {
      const double2 zp = buf[m];                     // Z_m
      const double2 zn = buf[m == 0 ? 0 : n - m];    // Z_{-m}
      double* row = GT + ((size_t)t * k + m) * C;
      if (REAL) {
        // A_m = (Z_m + conj Z_{-m}) / 2,  B_m = (Z_m - conj Z_{-m}) / (2i)
        row[2 * ma] = wphi * 0.5 * (zp.x + zn.x);
        row[2 * ma + 1] = wphi * 0.5 * (zp.y - zn.y);
        if (hasb) {
          row[2 * ma + 2] = wphi * 0.5 * (zp.y + zn.y);
          row[2 * ma + 3] = -wphi * 0.5 * (zp.x - zn.x);
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
//   D_j  = sum_t g_t e^{-2 pi i j t/n}        (g: packed extension, period n)
//   u_j  = e^{-i pi j/n} D_j,                  |j| <= k-1
//   I_j' = sum_j u_j w_e(j + j')               (w_e(p) = 2/(1-p^2) for even p, 0 for odd p)
//   H_t  = sum_j' e^{-i pi j'/n} I_j' e^{-2 pi i j' t/n} / n^2
// and the fold H'_E(t) = H_t + H_{n-1-t}, H'_O(t) = H_t - H_{n-1-t} (t < k-1).
// The weight's odd p = +-1 terms, left out of the correlation, act on odd m only through the
// south-pole sample: the odd pole value G_O(k-1) stays out of the packed transform and the
// operator's pole row and column are applied directly (H'_O(t) += c_t G_O(k-1) for t < k-1,
// H'_O(k-1) = sum_{t<k-1} c_t G_O(t) + c_{k-1} G_O(k-1), c = A.pole).  For band-limited maps
// G_O(k-1) = 0 and lambda_lm(pi) = 0 for m != 0, so the correction matters for other inputs and
// for the adjoint transform, which applies the same operator.
// ------------------------------------------------------------------------------------------
template <int VPT>
__global__ __launch_bounds__(512) void k_theta(FftArgs Ain, const double* __restrict__ GT,
                                               double* __restrict__ HM, int C, int nprob) {
  extern __shared__ double2 smem[];
  __shared__ double2 s_tw[4][TWMAX];
  const FftArgs A = stage_twiddles(Ain, s_tw);
  __shared__ double2 red_scratch[8];
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pl = threadIdx.x / A.T, lt = threadIdx.x % A.T;
  const int p = blk * A.P + pl;
  const bool valid = p < nprob;
  double2* buf = smem + (size_t)pl * A.buf;
  const int k = A.k, n = A.n, Nc = A.Nc;
  const int ns = C / 2;
  const int mu = valid ? p / ns : 0;
  const int s = valid ? p % ns : 0;
  const int mE = 2 * mu, mO = 2 * mu + 1;
  const bool hasO = mO < k;

  // packed extension g_t = G_E(t) + G_O(t) (t < k);  G_E(n-1-t) - G_O(n-1-t) (t >= k), without
  // the odd pole value; racc accumulates the pole row sum_{t<k-1} c_t G_O(t)
  double2 racc = make_double2(0.0, 0.0);
  {
    // each ring r < k is read once for nodes r and n-1-r, every load issued before the first
    // store (VPT >= n / T > k / T)
    double2 ge[VPT], go[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int r = lt + i * A.T;
      const double* rE = GT + ((size_t)(r < k ? r : 0) * k + mE) * C + 2 * s;
      ge[i] = *reinterpret_cast<const double2*>(rE);
      go[i] = hasO ? *reinterpret_cast<const double2*>(rE + C) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int r = lt + i * A.T;
      if (r < k) {
        const double2 e = valid ? ge[i] : make_double2(0.0, 0.0);
        if (valid && hasO && r < k - 1) {
          const double2 o = go[i];
          buf[r] = cadd(e, o);
          buf[n - 1 - r] = csub(e, o);
          racc.x = fma(A.pole[r], o.x, racc.x);
          racc.y = fma(A.pole[r], o.y, racc.y);
        } else {
          buf[r] = e;
          if (r < k - 1) buf[n - 1 - r] = e;
        }
      }
    }
  }
  const double2 prow = problem_sum(racc, A.T, red_scratch);
  __syncthreads();
  dft_odd<false, VPT>(buf, A, lt);

  // u_j = e^{-i pi j/n} D_j, kept in registers (index idx = j + k - 1, idx = lt + i*T)
  constexpr int MAXV = VPT;  // (2k-1)/T <= VPT since T >= n/VPT
  double2 keep[MAXV];
  const int nj = 2 * k - 1;
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * A.T;
    if (idx < nj) {
      const int j = idx - (k - 1);
      keep[i] = cmul(A.hphase[idx], buf[j < 0 ? j + n : j]);
    }
  }
  // correlation, one parity class at a time: U_a = u_{2a+P}, I_{2b+P} = (U * Kt_P)(-b)
#pragma unroll
  for (int P = 0; P < 2; ++P) {
    __syncthreads();
    for (int q = lt; q < Nc; q += A.T) buf[q] = make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = lt + i * A.T;
      if (idx < nj) {
        const int j = idx - (k - 1);
        if (((j - P) & 1) == 0) buf[((j - P) / 2) & (Nc - 1)] = keep[i];
      }
    }
    __syncthreads();
    fft_pow2<false, VPT>(buf, Nc, A.logNc, lt, A.T, A.tw_lo, A.tw_hi, A.loglo, A.logP - A.logNc);
    const double2* kh = P == 0 ? A.khat0 : A.khat1;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int q = lt + i * A.T;
      if (q < Nc) buf[q] = cmul(buf[q], kh[q]);
    }
    __syncthreads();
    fft_pow2<true, VPT>(buf, Nc, A.logNc, lt, A.T, A.tw_lo, A.tw_hi, A.loglo, A.logP - A.logNc);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = lt + i * A.T;
      if (idx < nj) {
        const int jp = idx - (k - 1);
        if (((jp - P) & 1) == 0) keep[i] = cmul(A.hphase[idx], buf[(-(jp - P) / 2) & (Nc - 1)]);
      }
    }
  }
  __syncthreads();
  // v_j' at index j' mod n, then H = DFT_n(v)
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * A.T;
    if (idx < nj) {
      const int jp = idx - (k - 1);
      buf[jp < 0 ? jp + n : jp] = keep[i];
    }
  }
  __syncthreads();
  dft_odd<false, VPT>(buf, A, lt);

  // fold onto t < k and separate the even and odd m; pole row and column of the odd operator
  if (valid) {
    double2 pO = make_double2(0.0, 0.0);
    if (hasO) {
      const double* rO = GT + ((size_t)(k - 1) * k + mO) * C + 2 * s;
      pO = make_double2(rO[0], rO[1]);
    }
    for (int t = lt; t < k; t += A.T) {
      const double2 h1 = buf[t];
      double2 he = h1, ho;
      if (t < k - 1) {
        const double2 h2 = buf[n - 1 - t];
        he = cadd(h1, h2);
        ho = csub(h1, h2);
        ho.x = fma(A.pole[t], pO.x, ho.x);
        ho.y = fma(A.pole[t], pO.y, ho.y);
      } else {
        ho = make_double2(fma(A.pole[t], pO.x, prow.x), fma(A.pole[t], pO.y, prow.y));
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
template <int REAL, int VPT>
__global__ __launch_bounds__(512) void k_phi_inverse(FftArgs Ain, const double* __restrict__ FT,
                                                     double* __restrict__ f, long long map_stride,
                                                     int C, int nb, int nprob) {
  extern __shared__ double2 smem[];
  __shared__ double2 s_tw[4][TWMAX];
  const FftArgs A = stage_twiddles(Ain, s_tw);
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pl = threadIdx.x / A.T, lt = threadIdx.x % A.T;
  const int p = blk * A.P + pl;
  const bool valid = p < nprob;
  double2* buf = smem + (size_t)pl * A.buf;
  const int k = A.k, n = A.n;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);

  // spectrum Z_m at index m mod n
  // (slot n - m holds order -m; each row is read once for both signs, every load issued before
  // the first store)
  {
    double2 ra[VPT], rb[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int m = lt + i * A.T;
      const double* row = FT + ((size_t)t * k + (m < k ? m : 0)) * C;
      if (REAL) {
        ra[i] = *reinterpret_cast<const double2*>(row + 2 * ma);
        rb[i] = hasb ? *reinterpret_cast<const double2*>(row + 2 * ma + 2) : make_double2(0.0, 0.0);
      } else {
        ra[i] = *reinterpret_cast<const double2*>(row + 4 * ma);
        rb[i] = *reinterpret_cast<const double2*>(row + 4 * ma + 2);
      }
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int m = lt + i * A.T;
      if (m < k) {
        const double2 a = valid ? ra[i] : make_double2(0.0, 0.0);
        const double2 b = valid ? rb[i] : make_double2(0.0, 0.0);
        if (REAL) {
          buf[m] = make_double2(a.x - b.y, a.y + b.x);   // a + i b
          if (m > 0) buf[n - m] = make_double2(a.x + b.y, b.x - a.y);   // conj(a) + i conj(b)
        } else {
          buf[m] = a;
          if (m > 0) buf[n - m] = b;
        }
      }
    }
  }
  __syncthreads();
  dft_odd<true, VPT>(buf, A, lt);

  if (valid) {
    for (int q = lt; q < n; q += A.T) {
      const double2 v = buf[q];
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
// Launch shapes: a problem gets T threads (T >= every transform length / VPT with VPT = 8, or
// 16 for the 8192-point Bluestein transforms of non-smooth n > 2048), a block holds P problems
// within 512 threads and 64 KiB of LDS.
static FftArgs fft_args(const ShtTables& T, bool theta) {
  FftArgs a;
  a.k = T.k;
  a.n = T.n;
  a.mixed = T.nrad > 0 ? 1 : 0;
  a.nrad = T.nrad;
  a.rad_code = 0;
  for (int s = 0; s < T.nrad; ++s) a.rad_code |= (unsigned)T.rad[s] << (4 * s);
  a.twn_lo = T.twn_lo;
  a.twn_hi = T.twn_hi;
  a.M = T.M;
  a.logM = T.logM;
  a.chirp = T.chirp;
  a.bhat = T.bhat;
  a.Nc = T.Nc;
  a.logNc = T.logNc;
  a.khat0 = T.khat0;
  a.khat1 = T.khat1;
  a.tw_lo = T.tw_lo;
  a.tw_hi = T.tw_hi;
  a.loglo = T.loglo;
  a.logP = T.logP;
  a.hphase = T.hphase;
  a.pole = T.pole;
  int need = a.mixed ? a.n : a.M;          // LDS values of the odd-length DFT
  if (theta && a.Nc > need) need = a.Nc;
  const int vpt = need > 4096 ? 16 : 8;
  int tn = (need + vpt - 1) / vpt;
  int Tt = 1;
  while (Tt < tn) Tt <<= 1;
  a.T = Tt;
  a.buf = need;
  int P = 1;
  if (Tt < 512) {
    P = 512 / Tt;
    const int bylds = 4096 / (need > 0 ? need : 1);
    if (bylds < P) P = bylds > 0 ? bylds : 1;
  }
  a.P = P;
  return a;
}

template <typename K>
static hipError_t prep(K kernel, size_t lds) {
  if (lds > 65536) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  return hipSuccess;
}

// Problems per block for a launch of nprob problems.  fft_args packs as many problems into a block
// as its LDS and 512 threads allow, which at the small band-limits puts every problem of a launch
// in one or two blocks (one compute unit busy, tens of microseconds for microseconds of work).
// Spread them over up to 256 blocks instead, keeping at least one full wavefront per block.
static FftArgs spread_problems(FftArgs A, int nprob) {
  const int pmin = A.T >= 64 ? 1 : 64 / A.T;
  const int pspread = (nprob + 255) / 256;
  const int p = pspread > pmin ? pspread : pmin;
  if (p < A.P) A.P = p;
  return A;
}

template <int REAL, int VPT>
static hipError_t phi_fwd_v(const FftArgs& Ain, const void* f, int64_t map_stride, double* GT, const Batch& b,
                            int nprob, hipStream_t s) {
  const FftArgs A = spread_problems(Ain, nprob);
  const int nblk = (nprob + A.P - 1) / A.P;
  const size_t lds = (size_t)A.P * A.buf * sizeof(double2);
  hipError_t e;
  if ((e = prep(k_phi_forward<REAL, VPT>, lds)) != hipSuccess) return e;
  k_phi_forward<REAL, VPT><<<nblk, A.P * A.T, lds, s>>>(A, (const double*)f, map_stride, GT, b.C, b.nb,
                                                         b.used, nprob);
  return hipGetLastError();
}

hipError_t launch_phi_forward(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                              double* GT, hipStream_t s) {
  if (fft_k2048_applies(T)) return launch_phi_forward_2048(T, b, f, map_stride, GT, s);
  if (fft_bs_applies(T)) return launch_phi_forward_bs(T, b, f, map_stride, GT, s);
  const FftArgs A = fft_args(T, false);
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = T.k * nunits;
  const bool big = A.buf > 4096;
  if (b.reality == S2LET_REAL)
    return big ? phi_fwd_v<1, 16>(A, f, map_stride, GT, b, nprob, s) : phi_fwd_v<1, 8>(A, f, map_stride, GT, b, nprob, s);
  return big ? phi_fwd_v<0, 16>(A, f, map_stride, GT, b, nprob, s) : phi_fwd_v<0, 8>(A, f, map_stride, GT, b, nprob, s);
}

template <int VPT>
static hipError_t theta_v(const FftArgs& Ain, const double* GT, double* HM, const Batch& b, int nprob,
                          hipStream_t s) {
  const FftArgs A = spread_problems(Ain, nprob);
  const int nblk = (nprob + A.P - 1) / A.P;
  const size_t lds = (size_t)A.P * A.buf * sizeof(double2);
  hipError_t e;
  if ((e = prep(k_theta<VPT>, lds)) != hipSuccess) return e;
  k_theta<VPT><<<nblk, A.P * A.T, lds, s>>>(A, GT, HM, b.C, nprob);
  return hipGetLastError();
}

hipError_t launch_theta(const ShtTables& T, const Batch& b, const double* GT, double* HM, hipStream_t s) {
  if (fft_k2048_applies(T)) return launch_theta_2048(T, b, GT, HM, s);
  const FftArgs A = fft_args(T, true);
  const int nprob = ((T.k + 1) / 2) * (b.C / 2);
  return A.buf > 4096 ? theta_v<16>(A, GT, HM, b, nprob, s) : theta_v<8>(A, GT, HM, b, nprob, s);
}

template <int REAL, int VPT>
static hipError_t phi_inv_v(const FftArgs& Ain, const double* FT, void* f, int64_t map_stride, const Batch& b,
                            int nprob, hipStream_t s) {
  const FftArgs A = spread_problems(Ain, nprob);
  const int nblk = (nprob + A.P - 1) / A.P;
  const size_t lds = (size_t)A.P * A.buf * sizeof(double2);
  hipError_t e;
  if ((e = prep(k_phi_inverse<REAL, VPT>, lds)) != hipSuccess) return e;
  k_phi_inverse<REAL, VPT><<<nblk, A.P * A.T, lds, s>>>(A, FT, (double*)f, map_stride, b.C, b.nb, nprob);
  return hipGetLastError();
}

hipError_t launch_phi_inverse(const ShtTables& T, const Batch& b, const double* FT, void* f,
                              int64_t map_stride, hipStream_t s, bool quad) {
  if (fft_k2048_applies(T)) return launch_phi_inverse_2048(T, b, FT, f, map_stride, s, quad);
  if (fft_bs_applies(T)) return launch_phi_inverse_bs(T, b, FT, f, map_stride, s);
  const FftArgs A = fft_args(T, false);
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = T.k * nunits;
  const bool big = A.buf > 4096;
  if (b.reality == S2LET_REAL)
    return big ? phi_inv_v<1, 16>(A, FT, f, map_stride, b, nprob, s) : phi_inv_v<1, 8>(A, FT, f, map_stride, b, nprob, s);
  return big ? phi_inv_v<0, 16>(A, FT, f, map_stride, b, nprob, s) : phi_inv_v<0, 8>(A, FT, f, map_stride, b, nprob, s);
}

}  // namespace s2let
