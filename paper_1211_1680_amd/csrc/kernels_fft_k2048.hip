// The O(k^2 log k) stages of the MW transform at band-limit k = 2048 (n = 2k - 1 = 4095 =
// 13 * 9 * 7 * 5, correlation length 4096), with the transforms compiled for that size
// (fft_ct.h).  Same arithmetic as the general kernels in kernels_fft.hip: phi DFT (Sect. 2.1,
// MW sampling), the theta stage (extension, DFT, parity-split correlation with the even part of
// the sin(theta) weight, DFT back, fold), and the inverse phi DFT.  One problem per 512-thread
// block; 74-76 KiB of LDS and at most 128 VGPRs (4 waves per SIMD), so two blocks share a CU.
// The kernels are templates over their working precision Rt; FP32 instantiations serve the BF16x3
// contraction mode, with FP32 buffers between them and the Legendre kernels.  They take 38 KiB of
// LDS (a resampling block 76 KiB) and at most 64 VGPRs (the theta stage 80), so four (three)
// problems share a CU.  The driver uses them where the rounding is relative to what is judged: the
// inverse stages (relative to the output maps), and the forward stages of the wavelet synthesis's
// per-scale transforms (relative to each scale's map).  The forward transform of an input map keeps
// FP64: there the rounding is relative to the whole map, and a steep spectrum carries it to the high
// degrees amplified (1.5e-4 of the finest wavelet scale, measured).
#include "common.h"
#include "fft_ct.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

namespace {
constexpr int K = 2048;
constexpr int N = 2 * K - 1;    // 4095
constexpr int NC = 4096;
constexpr int TT = 512;         // threads per problem
constexpr int NBUF = lds_padded(NC);
// complex type of a working precision, and the waves per SIMD its kernels are built for
template <typename Rt>
using Cx = typename std::conditional<sizeof(Rt) == 8, double2, float2>::type;

// The column-quad layout of a stage buffer: element (t, m, c) at ((t (C/4) + c/4) K + m) 4 + c mod 4.
// A phi problem (ring t and one unit: a map, or a pair of real maps) owns one column quad, so it
// writes (reads) whole lines, 64 KiB contiguous; in the row layout ((t K + m) C + c) the same bytes
// lie in 32-byte pieces 8 C bytes apart, each line shared with the problems of three other units,
// and that, not HBM bandwidth, bounds the phi stages (their time hardly changes without the DFT,
// nor when lane pairs make each store cover 32 contiguous bytes per row).
// The theta and resampling problems (orders 2 mu and 2 mu + 1 of one column pair, every ring) pay
// for it: in the column-quad layout the theta stage fetches about four times its bytes from HBM.
// FT (resampling -> inverse phi) is column-quad on the symmetric path, a net gain; GT (forward phi
// -> theta) keeps the row layout, where the theta stage's loss would outweigh the phi stage's gain.
__device__ __forceinline__ size_t quad_at(int t, int m, int c, int C) {
  return (((size_t)t * (C >> 2) + (c >> 2)) * K + m) * 4 + (c & 3);
}

// Problem p of a theta / resampling launch (order pair mu, column pair s; ns = C/2 column pairs).
// Row layout: p = mu ns + s, so the problems that share a GT / FT line (one order, eight column
// pairs) are consecutive.  Column-quad layout: a line holds orders 4j .. 4j+3 of one quad, shared
// by the problems (mu, s) with mu in {2j, 2j+1} and s in {2c, 2c+1}; those four are consecutive
// (p = 4 (j ns/2 + c) + 2 (mu mod 2) + s mod 2), and a resampling block (two consecutive problems)
// writes a whole quad of its two orders, 64 contiguous bytes per ring.
template <bool QUAD>
__device__ __forceinline__ void theta_problem(int p, int ns, int& mu, int& s) {
  if (QUAD) {
    const int q = p >> 2, r = p & 3, nc = ns >> 1;
    mu = 2 * (q / nc) + (r >> 1);
    s = 2 * (q % nc) + (r & 1);
  } else {
    mu = p / ns;
    s = p % ns;
  }
}

struct K2048Args {
  const double2* tw4096_lo;   // W_4096^p, p < 64
  const double2* tw4096_hi;   // W_4096^(64 q), q < 64
  const double2* tw4095_lo;
  const double2* tw4095_hi;
  const double* khr;          // real correlation spectrum (both parity classes)
  const double2* hphase;
  const double* pole;         // pole column of the odd-parity theta operator
  const double2* psph;        // symmetric grid: theta-stage output phase
  const double* pole_s;       // symmetric grid: pole column
  const double2* rsph;        // symmetric grid: resampling phase
};

// First radix-13 pass of the inverse 4095-point DFT, straight from the 4096-point FFT's output:
// DFT input i is bin j = i (i < K) or j = i - 4095 (i >= K), held in FFT slot j mod 4096, i.e. slot
// i or i + 1 (padded layout), and is taken times the phase ph[j + K - 1]; the outputs go to the
// DFT's plain layout.  Replaces a gather into registers, a barrier, a scatter to the DFT's order
// and another barrier.
template <int T, typename C2>
__device__ __forceinline__ void dft4095_inv_first_from_fft(C2* buf, int lt, const double2* __restrict__ ph) {
  constexpr int R = 13, NB = N / R;
  constexpr int PER = (NB + T - 1) / T;
  C2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = j + r * NB;
        const bool lo = x < K;
        v[i][r] = cmul(cplx<C2>(ph[lo ? x + K - 1 : x - K]), buf[lds_pad(lo ? x : x + 1)]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = lt + i * T;
    if (j < NB) {
      dft_small<R, true>(v[i]);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[j * R + r] = v[i][r];
    }
  }
  __syncthreads();
}

template <typename C2>
__device__ __forceinline__ void stage_tables(const K2048Args& A, C2* w6lo, C2* w6hi, C2* w5lo, C2* w5hi) {
  const int lt = threadIdx.x;
  if (lt < 64) {
    w6lo[twlo_at(lt)] = cplx<C2>(A.tw4096_lo[lt]);
    w6hi[lt] = cplx<C2>(A.tw4096_hi[lt]);
    w5lo[lt] = cplx<C2>(A.tw4095_lo[lt]);
    w5hi[lt] = cplx<C2>(A.tw4095_hi[lt]);
  }
}
}  // namespace

// phi stage, forward (see k_phi_forward): GT[(t*k + m)*C + c] for m < k.
template <int REAL, typename Rt>
__global__ __launch_bounds__(TT, sizeof(Rt) == 8 ? 4 : 8) void k_phi_forward_2048(K2048Args A, const double* __restrict__ f,
                                                            long long map_stride, Rt* __restrict__ GT,
                                                            int C, int nb, int used, int nprob) {
  typedef Cx<Rt> C2;
  __shared__ C2 buf[NBUF];
  __shared__ C2 w5lo[64], w5hi[64], w6lo[TWLO_SLOTS], w6hi[64];
  stage_tables(A, w6lo, w6hi, w5lo, w5hi);
  const int p = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x;
  const bool valid = p < nprob;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);

  load_ring<N, TT, REAL, false>(f, map_stride, ma, hasb, t, valid, buf, lt);
  __syncthreads();
  dft4095<false, TT>(buf, lt, w5lo, w5hi);

  const Rt wphi = (Rt)(2.0 * M_PI / (double)N), half = (Rt)0.5;
  if (valid) {
    for (int m = lt; m < K; m += TT) {
      const C2 zp = buf[m];
      const C2 zn = buf[m == 0 ? 0 : N - m];
      Rt* row = GT + ((size_t)t * K + m) * C;
      if (REAL) {
        if constexpr (sizeof(Rt) == 4) {
          if (hasb && (C & 3) == 0) {
            // one 16-byte store (the unit's four columns start at a multiple of 4 floats): as two
            // 8-byte pieces per row the writes reach HBM as partial writes, about 1.5 times the bytes
            float4 q;
            q.x = wphi * half * (zp.x + zn.x);
            q.y = wphi * half * (zp.y - zn.y);
            q.z = wphi * half * (zp.y + zn.y);
            q.w = -wphi * half * (zp.x - zn.x);
            *reinterpret_cast<float4*>(row + 2 * ma) = q;
            if (u == 0)
              for (int c = used; c < C; ++c) row[c] = Rt(0);
            continue;
          }
        }
        row[2 * ma] = wphi * half * (zp.x + zn.x);
        row[2 * ma + 1] = wphi * half * (zp.y - zn.y);
        if (hasb) {
          row[2 * ma + 2] = wphi * half * (zp.y + zn.y);
          row[2 * ma + 3] = -wphi * half * (zp.x - zn.x);
        }
      } else {
        row[4 * ma] = wphi * zp.x;
        row[4 * ma + 1] = wphi * zp.y;
        row[4 * ma + 2] = (m == 0) ? Rt(0) : wphi * zn.x;
        row[4 * ma + 3] = (m == 0) ? Rt(0) : wphi * zn.y;
      }
      if (u == 0)
        for (int c = used; c < C; ++c) row[c] = Rt(0);
    }
  }
}

// theta stage (see k_theta): GT[(t*k + m)*C + c] -> HM[(m*k + t)*C + c].
// SYM: the output transform evaluates on the symmetric grid psi_s = pi (2s+1) / (2k) instead of
// the MW nodes (a 4096-point FFT in place of the 4095-point DFT; the weight's p = +-1 terms still
// act only through the odd-m pole sample, now through the psi-grid pole column), folds s and
// 2k-1-s, and writes the north/south sums and differences for the Legendre analysis on s < k/2,
// column-pair major: row (m*(C/2) + cp)*k of double2, entry s = H(s) + H(k-1-s) and entry
// k/2 + s = H(s) - H(k-1-s).
// (FP32: 6 waves per SIMD, three problems per CU; at 8 the kernel spills and is slower)
template <bool SYM, typename Rt>
__global__ __launch_bounds__(TT, sizeof(Rt) == 8 ? 4 : 6) void k_theta_2048(K2048Args A, const Rt* __restrict__ GT,
                                                      Rt* __restrict__ HM, int C, int nprob) {
  typedef Cx<Rt> C2;
  static_assert(SYM || sizeof(Rt) == 8, "the MW-node output is FP64 only");
  __shared__ C2 buf[NBUF];
  __shared__ C2 w5lo[64], w5hi[64], w6lo[TWLO_SLOTS], w6hi[64];
  __shared__ double2 red_scratch[8];
  __shared__ double2 prow_s;   // pole row sum, kept in LDS through the transforms
  stage_tables(A, w6lo, w6hi, w5lo, w5hi);
  const int p = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x;
  const bool valid = p < nprob;
  const int ns = C / 2;
  int mu = 0, s = 0;
  if (valid) theta_problem<false>(p, ns, mu, s);
  const int mE = 2 * mu, mO = 2 * mu + 1;   // mO < K always (K even)

  // packed extension without the odd pole value (applied by the pole correction, see k_theta)
  double2 racc = make_double2(0.0, 0.0);
  {
    RingGather<K, TT, Rt> x;
    x.load(GT, C, mE, s, lt);
    // node r: even + odd order; node 2K-2-r (r < K-1): even - odd, the reflection's parity
#pragma unroll
    for (int i = 0; i < x.PER; ++i) {
      const int r = lt + i * TT;
      const C2 ge = valid ? x.ge[i] : czero<C2>();
      const C2 go = valid ? x.go[i] : czero<C2>();
      if (r < K - 1) {
        buf[r] = cadd(ge, go);
        buf[N - 1 - r] = csub(ge, go);
        if constexpr (!SYM) {
          racc.x = fma(A.pole[r], go.x, racc.x);
          racc.y = fma(A.pole[r], go.y, racc.y);
        }
      } else {
        buf[r] = ge;
      }
    }
  }
  if constexpr (!SYM) {
    const double2 prow = problem_sum(racc, TT, red_scratch);
    if (lt == 0) prow_s = prow;
  }
  __syncthreads();
  dft4095<false, TT>(buf, lt, w5lo, w5hi);

  constexpr int MAXV = NC / TT;   // 8 >= ceil((2K-1) / TT)
  constexpr int NJ = 2 * K - 1;
  C2 keep[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int idx = lt + i * TT;
    if (idx < NJ) {
      const int j = idx - (K - 1);
      keep[i] = cmul(cplx<C2>(A.hphase[idx]), buf[j < 0 ? j + N : j]);
    }
  }
#pragma unroll
  for (int P = 0; P < 2; ++P) {
    __syncthreads();
    // the class fills slots [0, 1024) and [3072, 4096) except slot 3072 for P = 0; the middle half
    // is never read (the first FFT pass skips it), so only that slot needs a zero
    if (P == 0 && lt == 0) buf[lds_pad(3 * K / 2)] = czero<C2>();
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
    // kernel and read class 1 one slot lower (either class then reads slots [0, 1024) and
    // [3072, 4096) only).  The opaque copy of the table address keeps the compiler from holding
    // the spectrum in registers across both classes, which spills.
    const double* kr = A.khr;
    asm volatile("" : "+s"(kr));
    corr_conv<NC, TT, 1>(buf, lt, w6lo, w6hi, kr);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = lt + i * TT;
      if (idx < NJ) {
        const int jp = idx - (K - 1);
        if (((jp - P) & 1) == 0)
          keep[i] = cmul(cplx<C2>(SYM ? A.psph[idx] : A.hphase[idx]), buf[lds_pad((-(jp - P) / 2 - P) & (NC - 1))]);
      }
    }
  }
  __syncthreads();
  if constexpr (SYM) {
    // I(j') at j' mod 4096 (slot 2048 stays empty), FFT onto the psi grid
    if (lt == 0) buf[lds_pad(K)] = czero<C2>();
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = lt + i * TT;
      if (idx < NJ) buf[lds_pad((idx - (K - 1)) & (NC - 1))] = keep[i];
    }
    __syncthreads();
    fft4096_r8<false, TT>(buf, lt, w6lo, w6hi);
    if (valid) {
      const Rt* rP = GT + ((size_t)(K - 1) * K + mO) * C + 2 * s;
      const C2 pO = CplxTraits<C2>::make(rP[0], rP[1]);
      for (int q = lt; q < K / 2; q += TT) {
        const int qs = K - 1 - q;   // the southern mirror of node q
        const C2 a1 = buf[lds_pad(q)], a2 = buf[lds_pad(NC - 1 - q)];
        const C2 b1 = buf[lds_pad(qs)], b2 = buf[lds_pad(NC - 1 - qs)];
        const C2 hea = cadd(a1, a2), heb = cadd(b1, b2);
        C2 hoa = csub(a1, a2), hob = csub(b1, b2);
        const Rt ps = (Rt)A.pole_s[q], pss = (Rt)A.pole_s[qs];
        hoa.x = fma(ps, pO.x, hoa.x);
        hoa.y = fma(ps, pO.y, hoa.y);
        hob.x = fma(pss, pO.x, hob.x);
        hob.y = fma(pss, pO.y, hob.y);
        C2* colE = reinterpret_cast<C2*>(HM) + ((size_t)mE * ns + s) * K;
        C2* colO = reinterpret_cast<C2*>(HM) + ((size_t)mO * ns + s) * K;
        colE[q] = cadd(hea, heb);
        colE[K / 2 + q] = csub(hea, heb);
        colO[q] = cadd(hoa, hob);
        colO[K / 2 + q] = csub(hoa, hob);
      }
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = lt + i * TT;
      if (idx < NJ) {
        const int jp = idx - (K - 1);
        buf[jp < 0 ? jp + N : jp] = keep[i];
      }
    }
    __syncthreads();
    dft4095<false, TT>(buf, lt, w5lo, w5hi);

    if (valid) {
      const double* rP = GT + ((size_t)(K - 1) * K + mO) * C + 2 * s;
      const double2 pO = make_double2(rP[0], rP[1]);
      for (int t = lt; t < K; t += TT) {
        const double2 h1 = buf[t];
        double2 he = h1, ho;
        if (t < K - 1) {
          const double2 h2 = buf[N - 1 - t];
          he = cadd(h1, h2);
          ho = csub(h1, h2);
          ho.x = fma(A.pole[t], pO.x, ho.x);
          ho.y = fma(A.pole[t], pO.y, ho.y);
        } else {
          ho = make_double2(fma(A.pole[t], pO.x, prow_s.x), fma(A.pole[t], pO.y, prow_s.y));
        }
        double* wE = HM + ((size_t)mE * K + t) * C + 2 * s;
        double* wO = HM + ((size_t)mO * K + t) * C + 2 * s;
        wE[0] = he.x;
        wE[1] = he.y;
        wO[0] = ho.x;
        wO[1] = ho.y;
      }
    }
  }
}


// Resampling from the symmetric grid to the MW nodes (inverse transforms on the symmetric grid):
// FS holds F_m(psi_s), s < k, column-pair major (row (m*(C/2) + cp)*k of double2; band-limited
// in theta); an even and an odd m
// share one complex sequence on the 2k-point circle (F(2 pi - psi) = (-1)^m F(psi)), a 4096-point
// FFT gives the Fourier coefficients |j| <= k-1, and the 4095-point inverse DFT evaluates them at
// theta_t = pi (2t+1) / n; the parities separate by the reflection t -> n-1-t.
// Output FT[(t*k + m)*C + c], t < k.  Two problems (adjacent column pairs) per 1024-thread
// block, so that neighbouring lanes write whole pieces of the output rows: 16-byte pieces from
// separate blocks reach HBM as partial writes (about 2.8 times the bytes in the row layout; 1.4
// times with the column-quad layout's 32-byte pieces, 1.1 times with its 64-byte pieces).
// QUAD: FT in the column-quad layout (else the row layout, for the general theta stage of the adjoint)
template <typename Rt, bool QUAD>
__global__ __launch_bounds__(2 * TT, sizeof(Rt) == 8 ? 4 : 8) void k_resample_2048(K2048Args A, const Rt* __restrict__ FS,
                                                          Rt* __restrict__ FT, int C, int nprob) {
  typedef Cx<Rt> C2;
  __shared__ C2 bufs[2][NBUF];
  __shared__ C2 w5lo[64], w5hi[64], w6lo[TWLO_SLOTS], w6hi[64];
  stage_tables(A, w6lo, w6hi, w5lo, w5hi);
  C2* buf = bufs[threadIdx.x / TT];
  const int p2 = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x % TT;
  const int p = 2 * p2 + (int)(threadIdx.x / TT);
  const bool valid = p < nprob;
  const int ns = C / 2;
  int mu = 0, s = 0;
  if (valid) theta_problem<QUAD>(p, ns, mu, s);
  const int mE = 2 * mu, mO = 2 * mu + 1;
  constexpr int NL = K / TT;   // 4
  C2 fe[NL], fo[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int q = lt + i * TT;
    fe[i] = czero<C2>();
    fo[i] = czero<C2>();
    if (valid) {
      fe[i] = reinterpret_cast<const C2*>(FS)[((size_t)mE * ns + s) * K + q];
      fo[i] = reinterpret_cast<const C2*>(FS)[((size_t)mO * ns + s) * K + q];
    }
  }
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int q = lt + i * TT;
    buf[lds_pad(q)] = cadd(fe[i], fo[i]);
    buf[lds_pad(NC - 1 - q)] = csub(fe[i], fo[i]);
  }
  __syncthreads();
  fft4096<false, TT>(buf, lt, w6lo, w6hi);
  // bins |j| <= K-1 times the phase, inverse 4095-point DFT onto the MW nodes
  dft4095_inv_first_from_fft<TT>(buf, lt, A.rsph);
  constexpr unsigned A8 = 0xFFFFu;
  ct_pass<4095, 9, 13, true, TT, 1, A8, A8, false>(buf, lt, w5lo, w5hi);
  ct_pass<4095, 7, 117, true, TT, 1, A8, A8, false>(buf, lt, w5lo, w5hi);
  ct_pass<4095, 5, 819, true, TT, 1, A8, A8, false>(buf, lt, w5lo, w5hi);
  if constexpr (QUAD && sizeof(Rt) == 4) {
    // FP32: thread T writes order 2 mu + (T & 1) of both problems at rings T / 2 + 512 i, the quad's
    // four columns as one 16-byte store (problem 2 p2 takes the quad's first column pair)
    const int od = threadIdx.x & 1, rr = threadIdx.x >> 1;
    if (2 * p2 + 1 < nprob) {
      int mu0, s0;
      theta_problem<QUAD>(2 * p2, ns, mu0, s0);
#pragma unroll
      for (int i = 0; i < K / TT; ++i) {
        const int t = rr + i * TT;
        C2 v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const C2 h1 = bufs[h][t];
          if (t < K - 1) {
            const C2 h2 = bufs[h][N - 1 - t];
            v[h] = od ? csub(h1, h2) : cadd(h1, h2);
          } else {
            v[h] = od ? czero<C2>() : cadd(h1, h1);
          }
        }
        float4 q;
        q.x = v[0].x;
        q.y = v[0].y;
        q.z = v[1].x;
        q.w = v[1].y;
        *reinterpret_cast<float4*>(FT + quad_at(t, 2 * mu0 + od, 2 * s0, C)) = q;
      }
    }
  } else if constexpr (QUAD) {
    // thread T writes order 2 mu + ((T >> 1) & 1) of problem 2 p2 + (T & 1) at rings T / 4 + 256 i:
    // the block's two problems are the two column pairs of one quad, so the four lanes of a ring
    // write its two orders' 64 contiguous bytes (32 in FP32) in one store instruction
    const int h = threadIdx.x & 1, od = (threadIdx.x >> 1) & 1, rq = threadIdx.x >> 2;
    const int ph = 2 * p2 + h;
    if (ph < nprob) {
      int muh, sh;
      theta_problem<QUAD>(ph, ns, muh, sh);
      const C2* bh = bufs[h];
      constexpr int RPI = 2 * TT / 4;   // rings per iteration
#pragma unroll
      for (int i = 0; i < K / RPI; ++i) {
        const int t = rq + i * RPI;
        const C2 h1 = bh[t];
        C2 v;
        if (t < K - 1) {
          const C2 h2 = bh[N - 1 - t];
          v = od ? csub(h1, h2) : cadd(h1, h2);
        } else {
          v = od ? czero<C2>() : cadd(h1, h1);
        }
        *reinterpret_cast<C2*>(FT + quad_at(t, 2 * muh + od, 2 * sh, C)) = v;
      }
    }
  } else {
    // row layout: thread T writes problem 2 p2 + (T & 1) at rings T / 2 + 512 i, the two problems'
    // adjacent column pairs as 32-byte pieces
    const int h = threadIdx.x & 1, rr = threadIdx.x >> 1;
    const int ph = 2 * p2 + h;
    if (ph < nprob) {
      int muh, sh;
      theta_problem<QUAD>(ph, ns, muh, sh);
      const C2* bh = bufs[h];
#pragma unroll
      for (int i = 0; i < K / TT; ++i) {
        const int t = rr + i * TT;
        const C2 h1 = bh[t];
        C2 he, ho;
        if (t < K - 1) {
          const C2 h2 = bh[N - 1 - t];
          he = cadd(h1, h2);
          ho = csub(h1, h2);
        } else {
          he = cadd(h1, h1);
          ho = czero<C2>();
        }
        *reinterpret_cast<C2*>(FT + ((size_t)t * K + 2 * muh) * C + 2 * sh) = he;
        *reinterpret_cast<C2*>(FT + ((size_t)t * K + 2 * muh + 1) * C + 2 * sh) = ho;
      }
    }
  }
}

// phi stage, inverse (see k_phi_inverse): FT[(t*k + m)*C + c] -> maps.
// QUAD: FT in the column-quad layout
template <int REAL, typename Rt, bool QUAD>
__global__ __launch_bounds__(TT, sizeof(Rt) == 8 ? 4 : 8) void k_phi_inverse_2048(K2048Args A, const Rt* __restrict__ FT,
                                                            double* __restrict__ f, long long map_stride, int C,
                                                            int nb, int nprob) {
  typedef Cx<Rt> C2;
  __shared__ C2 buf[NBUF];
  __shared__ C2 w5lo[64], w5hi[64], w6lo[TWLO_SLOTS], w6hi[64];
  stage_tables(A, w6lo, w6hi, w5lo, w5hi);
  const int p = xcd_swizzle(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x;
  const bool valid = p < nprob;
  const int nunits = REAL ? (nb + 1) / 2 : nb;
  const int t = valid ? p / nunits : 0;
  const int u = valid ? p % nunits : 0;
  const int ma = REAL ? 2 * u : u;
  const bool hasb = REAL && (ma + 1 < nb);

  load_orders<K, TT, REAL, false, Rt, C2, QUAD>(FT, C, ma, hasb, t, valid, buf, lt);
  __syncthreads();
  dft4095<true, TT>(buf, lt, w5lo, w5hi);

  if (valid) {
    for (int q = lt; q < N; q += TT) {
      const C2 v = buf[q];
      if (REAL) {
        f[(size_t)ma * map_stride + (size_t)t * N + q] = v.x;
        if (hasb) f[(size_t)(ma + 1) * map_stride + (size_t)t * N + q] = v.y;
      } else {
        reinterpret_cast<double2*>(f)[(size_t)ma * map_stride + (size_t)t * N + q] = make_double2(v.x, v.y);
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
static bool k2048_ok(const ShtTables& T) {
  return T.k == K && T.n == N && T.nrad == 4 && T.rad[0] == 13 && T.rad[1] == 9 && T.rad[2] == 7 &&
         T.rad[3] == 5 && T.Nc == NC && T.logP == 12 && T.loglo == 6;
}

static K2048Args k2048_args(const ShtTables& T) {
  K2048Args a;
  a.tw4096_lo = T.tw_lo;
  a.tw4096_hi = T.tw_hi;
  a.tw4095_lo = T.twn_lo;
  a.tw4095_hi = T.twn_hi;
  a.khr = T.khr;
  a.hphase = T.hphase;
  a.pole = T.pole;
  a.psph = T.psph;
  a.pole_s = T.pole_s;
  a.rsph = T.rsph;
  return a;
}

bool fft_k2048_applies(const ShtTables& T) { return k2048_ok(T); }

template <typename Rt>
static hipError_t phi_forward_2048(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride, Rt* GT,
                                   hipStream_t s) {
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = K * nunits;
  const K2048Args a = k2048_args(T);
  const double* fd = (const double*)f;
  if (b.reality == S2LET_REAL)
    k_phi_forward_2048<1, Rt><<<nprob, TT, 0, s>>>(a, fd, map_stride, GT, b.C, b.nb, b.used, nprob);
  else
    k_phi_forward_2048<0, Rt><<<nprob, TT, 0, s>>>(a, fd, map_stride, GT, b.C, b.nb, b.used, nprob);
  return hipGetLastError();
}

hipError_t launch_phi_forward_2048(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                                   double* GT, hipStream_t s) {
  return phi_forward_2048(T, b, f, map_stride, GT, s);
}

hipError_t launch_phi_forward_2048_f32(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                                       float* GT, hipStream_t s) {
  return phi_forward_2048(T, b, f, map_stride, GT, s);
}

hipError_t launch_theta_2048(const ShtTables& T, const Batch& b, const double* GT, double* HM, hipStream_t s,
                             bool sym) {
  const int nprob = (K / 2) * (b.C / 2);
  if (sym) {
    if (!T.sym) return hipErrorInvalidValue;
    k_theta_2048<true, double><<<nprob, TT, 0, s>>>(k2048_args(T), GT, HM, b.C, nprob);
  } else {
    k_theta_2048<false, double><<<nprob, TT, 0, s>>>(k2048_args(T), GT, HM, b.C, nprob);
  }
  return hipGetLastError();
}

hipError_t launch_theta_2048_f32(const ShtTables& T, const Batch& b, const float* GT, float* HM, hipStream_t s) {
  if (!T.sym) return hipErrorInvalidValue;
  const int nprob = (K / 2) * (b.C / 2);
  k_theta_2048<true, float><<<nprob, TT, 0, s>>>(k2048_args(T), GT, HM, b.C, nprob);
  return hipGetLastError();
}

template <typename Rt>
static hipError_t resample_2048(const ShtTables& T, const Batch& b, const Rt* FS, Rt* FT, hipStream_t s, bool quad) {
  if (!T.sym || !k2048_ok(T) || (quad && (b.C & 3))) return hipErrorInvalidValue;
  const int nprob = (K / 2) * (b.C / 2);   // even: K / 2 is
  if (quad)
    k_resample_2048<Rt, true><<<nprob / 2, 2 * TT, 0, s>>>(k2048_args(T), FS, FT, b.C, nprob);
  else
    k_resample_2048<Rt, false><<<nprob / 2, 2 * TT, 0, s>>>(k2048_args(T), FS, FT, b.C, nprob);
  return hipGetLastError();
}

hipError_t launch_resample_2048(const ShtTables& T, const Batch& b, const double* FS, double* FT, hipStream_t s,
                                bool quad) {
  return resample_2048(T, b, FS, FT, s, quad);
}

hipError_t launch_resample_2048_f32(const ShtTables& T, const Batch& b, const float* FS, float* FT,
                                    hipStream_t s) {
  return resample_2048(T, b, FS, FT, s, true);
}

template <typename Rt>
static hipError_t phi_inverse_2048(const ShtTables& T, const Batch& b, const Rt* FT, void* f, int64_t map_stride,
                                   hipStream_t s, bool quad) {
  if (quad && (b.C & 3)) return hipErrorInvalidValue;
  const int nunits = b.reality == S2LET_REAL ? (b.nb + 1) / 2 : b.nb;
  const int nprob = K * nunits;
  const K2048Args a = k2048_args(T);
  double* fd = (double*)f;
  if (b.reality == S2LET_REAL) {
    if (quad)
      k_phi_inverse_2048<1, Rt, true><<<nprob, TT, 0, s>>>(a, FT, fd, map_stride, b.C, b.nb, nprob);
    else
      k_phi_inverse_2048<1, Rt, false><<<nprob, TT, 0, s>>>(a, FT, fd, map_stride, b.C, b.nb, nprob);
  } else {
    if (quad)
      k_phi_inverse_2048<0, Rt, true><<<nprob, TT, 0, s>>>(a, FT, fd, map_stride, b.C, b.nb, nprob);
    else
      k_phi_inverse_2048<0, Rt, false><<<nprob, TT, 0, s>>>(a, FT, fd, map_stride, b.C, b.nb, nprob);
  }
  return hipGetLastError();
}

hipError_t launch_phi_inverse_2048(const ShtTables& T, const Batch& b, const double* FT, void* f,
                                   int64_t map_stride, hipStream_t s, bool quad) {
  return phi_inverse_2048(T, b, FT, f, map_stride, s, quad);
}

hipError_t launch_phi_inverse_2048_f32(const ShtTables& T, const Batch& b, const float* FT, void* f,
                                       int64_t map_stride, hipStream_t s) {
  return phi_inverse_2048(T, b, FT, f, map_stride, s, true);
}

}  // namespace s2let
