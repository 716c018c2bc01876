// The O(k^2 log k) stages of the MW transform at the band-limits k = 64 to 1024, compiled for those
// sizes.  n = 2k - 1 (127 prime, 255 = 3 * 5 * 17, 511 = 7 * 73, 1023 = 3 * 11 * 31, 2047 = 23 * 89)
// has a prime factor beyond the compiled radices, so the odd-length DFT is Bluestein's chirp
// transform over the 4k-point FFT; the correlation of the theta stage and the symmetric grid
// psi_s = pi (2s+1) / (2k) use the 2k-point FFT.  Same arithmetic as the general kernels
// (kernels_fft.hip) and as the band-limit 2048 kernels (kernels_fft_k2048.hip): phi DFT (Sect. 2.1,
// MW sampling), theta stage evaluated on the symmetric grid (its last transform), resampling from
// the symmetric grid to the MW nodes, inverse phi DFT.  One problem per block of BsCfg<k>::TT threads
// (two for the resampling); 74 KiB of LDS per problem at k = 1024, proportionally less below.
#include "common.h"
#include "fft_ct.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

namespace {
// per band-limit: threads per problem and log2 of the twiddle table length 4k
template <int K_> struct BsCfg;
template <> struct BsCfg<1024> { static constexpr int TT = 512, LOGP = 12; };
template <> struct BsCfg<512> { static constexpr int TT = 256, LOGP = 11; };
template <> struct BsCfg<256> { static constexpr int TT = 128, LOGP = 10; };
template <> struct BsCfg<128> { static constexpr int TT = 64, LOGP = 9; };
template <> struct BsCfg<64> { static constexpr int TT = 32, LOGP = 8; };

#define S2LET_BS_CONSTANTS                                                          \
  constexpr int N = 2 * K - 1;          /* odd ring length */                        \
  constexpr int NB = 4 * K;             /* Bluestein length and twiddle tables */    \
  constexpr int NC = 2 * K;             /* correlation length and psi circle */      \
  constexpr int TT = BsCfg<K>::TT;                                                  \
  constexpr int NBUF = lds_padded(NB);

struct BsArgs {
  const double2* tw_lo;    // W_4k^p, p < 64
  const double2* tw_hi;    // W_4k^(64 q), q < 4k / 64
  const double2* chirp;    // exp(-i pi q^2 / n), q < n
  const double2* bhat;     // FFT_4k of conj(chirp), wrapped, / 4k
  const double* khr;          // real correlation spectrum (both parity classes)
  const double2* hphase;
  const double2* psph;
  const double* pole_s;
  const double2* rsph;
};

template <int NB>
__device__ __forceinline__ void stage_tw(const BsArgs& A, double2* wlo, double2* whi) {
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    wlo[twlo_at(i)] = A.tw_lo[i];
    if (i < NB / 64) whi[i] = A.tw_hi[i];
  }
}
}  // namespace

// phi stage, forward (see k_phi_forward): GT[(t*k + m)*C + c] for m < k.
template <int K, int REAL>
__global__ __launch_bounds__(BsCfg<K>::TT, 4) void k_phi_forward_bs(BsArgs A, const double* __restrict__ f,
                                                                    long long map_stride, double* __restrict__ GT,
                                                                    int C, int nb, int used, int nprob) {
  S2LET_BS_CONSTANTS
  __shared__ double2 buf[NBUF];
  __shared__ double2 wlo[TWLO_SLOTS], whi[64];
  stage_tw<NB>(A, wlo, whi);
  const int p = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x;
  const bool valid = p < nprob;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);
  load_ring<N, TT, REAL>(f, map_stride, ma, hasb, t, valid, buf, lt);
  __syncthreads();
  dft_bluestein<NB, false, TT>(buf, N, lt, wlo, whi, A.chirp, A.bhat);
  const double wphi = 2.0 * M_PI / (double)N;
  if (valid) {
    for (int m = lt; m < K; m += TT) {
      const double2 zp = buf[lds_pad(m)];
      const double2 zn = buf[lds_pad(m == 0 ? 0 : N - m)];
      double* row = GT + ((size_t)t * K + m) * C;
      if (REAL) {
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

// theta stage on the symmetric grid (see k_theta_2048<true>): GT[(t*k + m)*C + c] -> HM, column-pair
// major, entry s < k/2 the north/south sums, entry k/2 + s the differences.
template <int K>
__global__ __launch_bounds__(BsCfg<K>::TT, 4) void k_theta_sym_bs(BsArgs A, const double* __restrict__ GT,
                                                                  double* __restrict__ HM, int C, int nprob) {
  S2LET_BS_CONSTANTS
  __shared__ double2 buf[NBUF];
  __shared__ double2 wlo[TWLO_SLOTS], whi[64];
  stage_tw<NB>(A, wlo, whi);
  const int p = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x;
  const bool valid = p < nprob;
  const int ns = C / 2;
  const int mu = valid ? p / ns : 0;
  const int s = valid ? p % ns : 0;
  const int mE = 2 * mu, mO = 2 * mu + 1;
  // packed extension without the odd pole value
  {
    RingGather<K, TT> x;
    x.load(GT, C, mE, s, lt);
    // node r: even + odd order; node 2K-2-r (r < K-1): even - odd, the reflection's parity
#pragma unroll
    for (int i = 0; i < x.PER; ++i) {
      const int r = lt + i * TT;
      const double2 ge = valid ? x.ge[i] : make_double2(0.0, 0.0);
      const double2 go = valid ? x.go[i] : make_double2(0.0, 0.0);
      if (r < K - 1) {
        buf[lds_pad(r)] = cadd(ge, go);
        buf[lds_pad(N - 1 - r)] = csub(ge, go);
      } else {
        buf[lds_pad(r)] = ge;
      }
    }
  }
  __syncthreads();
  dft_bluestein<NB, false, TT>(buf, N, lt, wlo, whi, A.chirp, A.bhat);
  constexpr int MAXV = NB / TT;   // >= ceil((2K-1) / TT)
  constexpr int NJ = 2 * K - 1;
  double2 keep[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * TT;
    if (idx < NJ) {
      const int j = idx - (K - 1);
      keep[i] = cmul(A.hphase[idx], buf[lds_pad(j < 0 ? j + N : j)]);
    }
  }
#pragma unroll
  for (int P = 0; P < 2; ++P) {
    __syncthreads();
    // the class fills slots [0, k/2) and [3k/2, 2k) except slot 3k/2 for P = 0; the middle is never
    // read (the first FFT pass skips it), so only that slot needs a zero
    if (P == 0 && lt == 0) buf[lds_pad(3 * K / 2)] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = lt + i * TT;
      if (idx < NJ) {
        const int j = idx - (K - 1);
        if (((j - P) & 1) == 0) buf[lds_pad(((j - P) / 2) & (NC - 1))] = keep[i];
      }
    }
    __syncthreads();
    // the class-1 kernel is the class-0 kernel shifted by one slot: convolve with the class-0
    // kernel and read class 1 one slot lower (either class then reads slots [0, k/2) and
    // [3k/2, 2k) only).  The opaque copy of the table address keeps the compiler from holding
    // the spectrum in registers across both classes.
    const double* kr = A.khr;
    asm volatile("" : "+s"(kr));
    corr_conv<NC, TT, 2>(buf, lt, wlo, whi, kr);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = lt + i * TT;
      if (idx < NJ) {
        const int jp = idx - (K - 1);
        if (((jp - P) & 1) == 0) keep[i] = cmul(A.psph[idx], buf[lds_pad((-(jp - P) / 2 - P) & (NC - 1))]);
      }
    }
  }
  __syncthreads();
  // I(j') at j' mod 2k (slot k stays empty), FFT onto the psi grid
  if (lt == 0) buf[lds_pad(K)] = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * TT;
    if (idx < NJ) buf[lds_pad((idx - (K - 1)) & (NC - 1))] = keep[i];
  }
  __syncthreads();
  fft_ct<NC, false, TT, 2>(buf, lt, wlo, whi);
  if (valid) {
    const double* rP = GT + ((size_t)(K - 1) * K + mO) * C + 2 * s;
    const double2 pO = make_double2(rP[0], rP[1]);
    for (int q = lt; q < K / 2; q += TT) {
      const int qs = K - 1 - q;
      const double2 a1 = buf[lds_pad(q)], a2 = buf[lds_pad(NC - 1 - q)];
      const double2 b1 = buf[lds_pad(qs)], b2 = buf[lds_pad(NC - 1 - qs)];
      const double2 hea = cadd(a1, a2), heb = cadd(b1, b2);
      double2 hoa = csub(a1, a2), hob = csub(b1, b2);
      hoa.x = fma(A.pole_s[q], pO.x, hoa.x);
      hoa.y = fma(A.pole_s[q], pO.y, hoa.y);
      hob.x = fma(A.pole_s[qs], pO.x, hob.x);
      hob.y = fma(A.pole_s[qs], pO.y, hob.y);
      double2* colE = reinterpret_cast<double2*>(HM) + ((size_t)mE * ns + s) * K;
      double2* colO = reinterpret_cast<double2*>(HM) + ((size_t)mO * ns + s) * K;
      colE[q] = cadd(hea, heb);
      colE[K / 2 + q] = csub(hea, heb);
      colO[q] = cadd(hoa, hob);
      colO[K / 2 + q] = csub(hoa, hob);
    }
  }
}

// Resampling from the symmetric grid to the MW nodes (see k_resample_2048; two problems per
// block, for 32-byte output pieces).
template <int K>
__global__ __launch_bounds__(2 * BsCfg<K>::TT) void k_resample_bs(BsArgs A, const double* __restrict__ FS,
                                                                  double* __restrict__ FT, int C, int nprob) {
  S2LET_BS_CONSTANTS
  __shared__ double2 bufs[2][NBUF];
  __shared__ double2 wlo[TWLO_SLOTS], whi[64];
  stage_tw<NB>(A, wlo, whi);
  double2* buf = bufs[threadIdx.x / TT];
  const int p2 = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x % TT;
  const int p = 2 * p2 + (int)(threadIdx.x / TT);
  const bool valid = p < nprob;
  const int ns = C / 2;
  const int mu = valid ? p / ns : 0;
  const int s = valid ? p % ns : 0;
  const int mE = 2 * mu, mO = 2 * mu + 1;
  constexpr int NL = K / TT;
  double2 fe[NL], fo[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int q = lt + i * TT;
    fe[i] = make_double2(0.0, 0.0);
    fo[i] = make_double2(0.0, 0.0);
    if (valid) {
      fe[i] = reinterpret_cast<const double2*>(FS)[((size_t)mE * ns + s) * K + q];
      fo[i] = reinterpret_cast<const double2*>(FS)[((size_t)mO * ns + s) * K + q];
    }
  }
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int q = lt + i * TT;
    buf[lds_pad(q)] = cadd(fe[i], fo[i]);
    buf[lds_pad(NC - 1 - q)] = csub(fe[i], fo[i]);
  }
  __syncthreads();
  fft_ct<NC, false, TT, 2>(buf, lt, wlo, whi);
  constexpr int MAXV = NC / TT;   // >= ceil((2K-1) / TT)
  constexpr int NJ = 2 * K - 1;
  double2 keep[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * TT;
    if (idx < NJ) keep[i] = cmul(A.rsph[idx], buf[lds_pad((idx - (K - 1)) & (NC - 1))]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * TT;
    if (idx < NJ) {
      const int j = idx - (K - 1);
      buf[lds_pad(j < 0 ? j + N : j)] = keep[i];
    }
  }
  __syncthreads();
  dft_bluestein<NB, true, TT>(buf, N, lt, wlo, whi, A.chirp, A.bhat);
  __syncthreads();
  // thread T writes problem 2 p2 + (T & 1) at rings T / 2 + TT i
  const int h = threadIdx.x & 1, rr = threadIdx.x >> 1;
  const int ph = 2 * p2 + h;
  if (ph < nprob) {
    const int muh = ph / ns, sh = ph % ns;
    const double2* bh = bufs[h];
#pragma unroll
    for (int i = 0; i < K / TT; ++i) {
      const int t = rr + i * TT;
      const double2 h1 = bh[lds_pad(t)];
      double2 he, ho;
      if (t < K - 1) {
        const double2 h2 = bh[lds_pad(N - 1 - t)];
        he = cadd(h1, h2);
        ho = csub(h1, h2);
      } else {
        he = cadd(h1, h1);
        ho = make_double2(0.0, 0.0);
      }
      *reinterpret_cast<double2*>(FT + ((size_t)t * K + 2 * muh) * C + 2 * sh) = he;
      *reinterpret_cast<double2*>(FT + ((size_t)t * K + 2 * muh + 1) * C + 2 * sh) = ho;
    }
  }
}

// phi stage, inverse (see k_phi_inverse): FT[(t*k + m)*C + c] -> maps.
template <int K, int REAL>
__global__ __launch_bounds__(BsCfg<K>::TT, 4) void k_phi_inverse_bs(BsArgs A, const double* __restrict__ FT,
                                                                    double* __restrict__ f, long long map_stride,
                                                                    int C, int nb, int nprob) {
  S2LET_BS_CONSTANTS
  __shared__ double2 buf[NBUF];
  __shared__ double2 wlo[TWLO_SLOTS], whi[64];
  stage_tw<NB>(A, wlo, whi);
  const int p = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x;
  const bool valid = p < nprob;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);
  load_orders<K, TT, REAL>(FT, C, ma, hasb, t, valid, buf, lt);
  __syncthreads();
  dft_bluestein<NB, true, TT>(buf, N, lt, wlo, whi, A.chirp, A.bhat);
  if (valid) {
    for (int q = lt; q < N; q += TT) {
      const double2 v = buf[lds_pad(q)];
      if (REAL) {
        f[(size_t)ma * map_stride + (size_t)t * N + q] = v.x;
        if (hasb) f[(size_t)(ma + 1) * map_stride + (size_t)t * N + q] = v.y;
      } else {
        reinterpret_cast<double2*>(f)[(size_t)ma * map_stride + (size_t)t * N + q] = v;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
template <int K>
static bool bs_tables_match(const ShtTables& T) {
  return T.k == K && T.n == 2 * K - 1 && T.nrad == 0 && T.M == 4 * K && T.Nc == 2 * K &&
         T.logP == BsCfg<K>::LOGP && T.loglo == 6;
}

bool fft_bs_applies(const ShtTables& T) {
  return bs_tables_match<1024>(T) || bs_tables_match<512>(T) || bs_tables_match<256>(T) ||
         bs_tables_match<128>(T) || bs_tables_match<64>(T);
}

static BsArgs bs_args(const ShtTables& T) {
  BsArgs a;
  a.tw_lo = T.tw_lo;
  a.tw_hi = T.tw_hi;
  a.chirp = T.chirp;
  a.bhat = T.bhat;
  a.khr = T.khr;
  a.hphase = T.hphase;
  a.psph = T.psph;
  a.pole_s = T.pole_s;
  a.rsph = T.rsph;
  return a;
}

template <int K>
static hipError_t phi_forward_k(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride, double* GT,
                                hipStream_t s) {
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = K * nunits;
  const BsArgs a = bs_args(T);
  if (b.reality == S2LET_REAL)
    k_phi_forward_bs<K, 1><<<nprob, BsCfg<K>::TT, 0, s>>>(a, (const double*)f, map_stride, GT, b.C, b.nb, b.used,
                                                          nprob);
  else
    k_phi_forward_bs<K, 0><<<nprob, BsCfg<K>::TT, 0, s>>>(a, (const double*)f, map_stride, GT, b.C, b.nb, b.used,
                                                          nprob);
  return hipGetLastError();
}

template <int K>
static hipError_t phi_inverse_k(const ShtTables& T, const Batch& b, const double* FT, void* f, int64_t map_stride,
                                hipStream_t s) {
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = K * nunits;
  const BsArgs a = bs_args(T);
  if (b.reality == S2LET_REAL)
    k_phi_inverse_bs<K, 1><<<nprob, BsCfg<K>::TT, 0, s>>>(a, FT, (double*)f, map_stride, b.C, b.nb, nprob);
  else
    k_phi_inverse_bs<K, 0><<<nprob, BsCfg<K>::TT, 0, s>>>(a, FT, (double*)f, map_stride, b.C, b.nb, nprob);
  return hipGetLastError();
}

hipError_t launch_phi_forward_bs(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride, double* GT,
                                 hipStream_t s) {
  if (bs_tables_match<1024>(T)) return phi_forward_k<1024>(T, b, f, map_stride, GT, s);
  if (bs_tables_match<512>(T)) return phi_forward_k<512>(T, b, f, map_stride, GT, s);
  if (bs_tables_match<256>(T)) return phi_forward_k<256>(T, b, f, map_stride, GT, s);
  if (bs_tables_match<128>(T)) return phi_forward_k<128>(T, b, f, map_stride, GT, s);
  if (bs_tables_match<64>(T)) return phi_forward_k<64>(T, b, f, map_stride, GT, s);
  return hipErrorInvalidValue;
}

hipError_t launch_phi_inverse_bs(const ShtTables& T, const Batch& b, const double* FT, void* f, int64_t map_stride,
                                 hipStream_t s) {
  if (bs_tables_match<1024>(T)) return phi_inverse_k<1024>(T, b, FT, f, map_stride, s);
  if (bs_tables_match<512>(T)) return phi_inverse_k<512>(T, b, FT, f, map_stride, s);
  if (bs_tables_match<256>(T)) return phi_inverse_k<256>(T, b, FT, f, map_stride, s);
  if (bs_tables_match<128>(T)) return phi_inverse_k<128>(T, b, FT, f, map_stride, s);
  if (bs_tables_match<64>(T)) return phi_inverse_k<64>(T, b, FT, f, map_stride, s);
  return hipErrorInvalidValue;
}

hipError_t launch_theta_sym_bs(const ShtTables& T, const Batch& b, const double* GT, double* HM, hipStream_t s) {
  if (!T.sym) return hipErrorInvalidValue;
  const int nprob = (T.k / 2) * (b.C / 2);
  if (bs_tables_match<1024>(T))
    k_theta_sym_bs<1024><<<nprob, BsCfg<1024>::TT, 0, s>>>(bs_args(T), GT, HM, b.C, nprob);
  else if (bs_tables_match<512>(T))
    k_theta_sym_bs<512><<<nprob, BsCfg<512>::TT, 0, s>>>(bs_args(T), GT, HM, b.C, nprob);
  else if (bs_tables_match<256>(T))
    k_theta_sym_bs<256><<<nprob, BsCfg<256>::TT, 0, s>>>(bs_args(T), GT, HM, b.C, nprob);
  else if (bs_tables_match<128>(T))
    k_theta_sym_bs<128><<<nprob, BsCfg<128>::TT, 0, s>>>(bs_args(T), GT, HM, b.C, nprob);
  else if (bs_tables_match<64>(T))
    k_theta_sym_bs<64><<<nprob, BsCfg<64>::TT, 0, s>>>(bs_args(T), GT, HM, b.C, nprob);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_resample_bs(const ShtTables& T, const Batch& b, const double* FS, double* FT, hipStream_t s) {
  if (!T.sym) return hipErrorInvalidValue;
  const int nprob = (T.k / 2) * (b.C / 2);   // even: k / 2 is
  if (bs_tables_match<1024>(T))
    k_resample_bs<1024><<<nprob / 2, 2 * BsCfg<1024>::TT, 0, s>>>(bs_args(T), FS, FT, b.C, nprob);
  else if (bs_tables_match<512>(T))
    k_resample_bs<512><<<nprob / 2, 2 * BsCfg<512>::TT, 0, s>>>(bs_args(T), FS, FT, b.C, nprob);
  else if (bs_tables_match<256>(T))
    k_resample_bs<256><<<nprob / 2, 2 * BsCfg<256>::TT, 0, s>>>(bs_args(T), FS, FT, b.C, nprob);
  else if (bs_tables_match<128>(T))
    k_resample_bs<128><<<nprob / 2, 2 * BsCfg<128>::TT, 0, s>>>(bs_args(T), FS, FT, b.C, nprob);
  else if (bs_tables_match<64>(T))
    k_resample_bs<64><<<nprob / 2, 2 * BsCfg<64>::TT, 0, s>>>(bs_args(T), FS, FT, b.C, nprob);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace s2let
