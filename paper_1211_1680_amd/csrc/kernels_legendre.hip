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
#include "legendre_rec.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

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
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);   // blocks of one pair share an L2
  const int pair = blk / ntb;
  const int tb = blk % ntb;
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
// Block = 8 waves = 512 thetas of one m pair; wave w owns 64 thetas: their recursion state and
// their H' operands (64 thetas x C columns) stay in registers for the whole m.  Per chunk of
// 32 degrees a wave writes its z values to a private LDS tile, multiplies, and the eight
// partial sums are reduced through LDS.  Blocks covering different theta ranges (g) write
// separate partial sums R[g]; the consumer of R adds them.
// ------------------------------------------------------------------------------------------

// The 16x16x4 matrix instruction per operand type: FP64, or FP32 with FP32 accumulation (the
// mixed-precision contraction; the recursion stays FP64).  A lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16]; result register v holds column l % 16 and the row given by row().
template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t zero() { return v4d{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lq, int v) { return lq + 4 * v; }
};
template <> struct Mma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t zero() { return v4f{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lq, int v) { return 4 * lq + v; }
};

constexpr int FWD_NW = 8;       // waves per block
constexpr int FWD_LC = 32;      // degrees per chunk
constexpr int FWD_ZS = 66;      // LDS row stride (doubles): 2 x odd, conflict-free B reads
constexpr int FWD_TB = FWD_NW * 64;   // thetas per block

template <int C, typename T>
__global__ __launch_bounds__(512) void k_legendre_fwd(const double* __restrict__ HM, double* __restrict__ R,
                                                      long long part_stride,
                                                      const double* __restrict__ alpha,
                                                      const double* __restrict__ beta,
                                                      const double* __restrict__ cm,
                                                      const double* __restrict__ ut,
                                                      const double* __restrict__ sx,
                                                      const double* __restrict__ st, int k, int Lt, int ng,
                                                      unsigned long long* __restrict__ counter) {
  constexpr int CT = C >= 16 ? C / 16 : 1;
  // wave-private z tiles; after each chunk the same memory holds the FP64 partial sums
  // red[w][l][c], row stride 2 x odd doubles so that the 16 degrees x 2 columns written by a
  // half wave fall in different LDS banks
  constexpr int RS = 2 * ((C / 2) | 1);
  constexpr int ZBYTES = FWD_NW * FWD_LC * FWD_ZS * (int)sizeof(T);
  constexpr int RBYTES = FWD_NW * FWD_LC * RS * (int)sizeof(double);
  __shared__ __align__(16) char smem[ZBYTES > RBYTES ? ZBYTES : RBYTES];
  T (*Z)[FWD_LC][FWD_ZS] = reinterpret_cast<T (*)[FWD_LC][FWD_ZS]>(smem);
  double* red = reinterpret_cast<double*>(smem);
  unsigned long long retained = 0;   // (l, theta) pairs multiplied by this wave
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int pair = blockIdx.x / ng;
  const int grp = blockIdx.x % ng;
  const int tile = grp * FWD_NW + w;
  const int t = tile * 64 + lane;
  const bool valid = t < k;
  const bool tile_live = tile * 64 < k;
  const double u = valid ? ut[t] : -1.0;
  const double sg = valid ? sx[t] : -1.0;   // lanes past the pole join the southern hemisphere
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  double* __restrict__ Rg = R + (size_t)grp * part_stride;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Hm = HM + (size_t)m * k * C;
    // this wave's operands: a[kk][ct] = H'[tile*64 + 4 kk + lq][ct*16 + li]
    T a[16][CT];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int tg = tile * 64 + 4 * kk + lq;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = ct * 16 + li;
        a[kk][ct] = (T)((tg < k && c < C) ? Hm[(size_t)tg * C + c] : 0.0);
      }
    }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf_next = chunk_coef<FWD_LC>(am, bm, 0, k - m, lane);

    for (int l0 = m; l0 < k; l0 += FWD_LC) {
      typename Mma<T>::acc_t acc[2][CT];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[x][ct] = Mma<T>::zero();
      const bool skip = !tile_live || __all(!valid || negligible(z1, z2, e));
      // z values for degrees l0 .. l0+31 at this lane's theta (lanes past k hold finite values
      // that meet zero operands)
      const double cf = cf_next;
      cf_next = chunk_coef<FWD_LC>(am, bm, l0 + FWD_LC - m, k - m, lane);
      // (a skipped chunk's z values are read by no product: the recursion stores none)
      if (skip)
        recur_chunk<FWD_LC>(cf, u, sg, z1, z2, e, [](int, double) {});
      else
        recur_chunk<FWD_LC>(cf, u, sg, z1, z2, e, [&](int j, double v) { Z[w][j][lane] = (T)v; });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < FWD_LC ? (k - l0) : FWD_LC;
        const int nt = (k - tile * 64) < 64 ? (k - tile * 64) : 64;
        retained += (unsigned long long)nl * (unsigned long long)nt;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const int tl = 4 * kk + lq;
#pragma unroll
          for (int lt2 = 0; lt2 < 2; ++lt2) {
            const T bv = Z[w][lt2 * 16 + li][tl];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[lt2][ct] = Mma<T>::mma(a[kk][ct], bv, acc[lt2][ct]);
          }
        }
      }
      // reduce the waves' partial sums
      __syncthreads();
#pragma unroll
      for (int lt2 = 0; lt2 < 2; ++lt2)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = ct * 16 + Mma<T>::row(lq, v);
            const int lloc = lt2 * 16 + li;
            if (c < C) red[((size_t)w * FWD_LC + lloc) * RS + c] = (double)acc[lt2][ct][v];
          }
      __syncthreads();
      for (int idx = threadIdx.x; idx < FWD_LC * C; idx += FWD_NW * 64) {
        const int lloc = idx / C, c = idx % C;
        const int l = l0 + lloc;
        if (l < k) {
          double sum = 0.0;
#pragma unroll
          for (int ww = 0; ww < FWD_NW; ++ww) sum += red[(ww * FWD_LC + lloc) * RS + c];
          Rg[(tri_off(k, m) + (l - m)) * C + c] = sum;
        }
      }
      __syncthreads();
    }
  }
  if (counter != nullptr && lane == 0 && retained > 0) atomicAdd(counter, retained);
}

// ------------------------------------------------------------------------------------------
// Synthesis on the matrix cores (C >= 16): D[t][c] = sum_l z_l(theta_t) S[l][c] with
// v_mfma_f64_16x16x4 (A = 16 thetas x 4 degrees, B = 4 degrees x 16 columns).  Each wave owns
// 64 thetas and streams every degree of its m pair; z values pass through a wave-private LDS
// tile (16 degrees), the coefficient rows are vector loads issued before the recursion.
// ------------------------------------------------------------------------------------------
constexpr int INVM_LC = 16;     // degrees per chunk
constexpr int INVM_ZS = 80;     // LDS row stride (elements): = 16 mod 32, conflict-free A reads
constexpr int INVM_FLUSH = 4;   // FP32 path: chunks (64 degrees) accumulated in FP32 between flushes

template <int C, typename T>
__global__ __launch_bounds__(256) void k_legendre_inv_mfma(const double* __restrict__ S, double* __restrict__ FT,
                                                           const double* __restrict__ alpha,
                                                           const double* __restrict__ beta,
                                                           const double* __restrict__ cm,
                                                           const double* __restrict__ ut,
                                                           const double* __restrict__ sx,
                                                           const double* __restrict__ st, int k, int Lt,
                                                           int ntb, unsigned long long* __restrict__ counter) {
  constexpr int CT = C / 16;
  constexpr bool F64 = sizeof(T) == sizeof(double);
  __shared__ T Z[4][INVM_LC][INVM_ZS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  // the ntb blocks of one m pair read the same coefficient columns: keep them on one XCD
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pair = blk / ntb;
  const int tile = (blk % ntb) * 4 + w;
  const int t = tile * 64 + lane;
  const bool valid = t < k;
  const double u = valid ? ut[t] : -1.0;
  const double sg = valid ? sx[t] : -1.0;   // lanes past the pole join the southern hemisphere
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  unsigned long long retained = 0;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Sm = S + tri_off(k, m) * C;
    typename Mma<T>::acc_t acc[4][CT];
    // FP32 path: the FP32 accumulators are added into FP64 sums every INVM_FLUSH chunks
    double accd[F64 ? 1 : 4][F64 ? 1 : CT][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[g][ct] = Mma<T>::zero();
    if constexpr (!F64) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) accd[g][ct][v] = 0.0;
    }
    int since_flush = 0;

    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf_next = chunk_coef<INVM_LC>(am, bm, 0, k - m, lane);
    // coefficient rows l0 + 4 sl + lq, columns ct*16 + li; the rows of the next chunk are
    // requested while the current chunk is multiplied
    // (kept in FP64 until used, so that the loads stay in flight across the recursion)
    double bn[INVM_LC / 4][CT];
#pragma unroll
    for (int sl = 0; sl < INVM_LC / 4; ++sl) {
      const int l = m + 4 * sl + lq;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) bn[sl][ct] = l < k ? Sm[(size_t)(l - m) * C + ct * 16 + li] : 0.0;
    }
    for (int l0 = m; l0 < k; l0 += INVM_LC) {
      const bool skip = __all(!valid || negligible(z1, z2, e));
      T b[INVM_LC / 4][CT];
#pragma unroll
      for (int sl = 0; sl < INVM_LC / 4; ++sl)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) b[sl][ct] = (T)bn[sl][ct];
      if (l0 + INVM_LC < k) {
#pragma unroll
        for (int sl = 0; sl < INVM_LC / 4; ++sl) {
          const int l = l0 + INVM_LC + 4 * sl + lq;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) bn[sl][ct] = l < k ? Sm[(size_t)(l - m) * C + ct * 16 + li] : 0.0;
        }
      }
      const double cf = cf_next;
      cf_next = chunk_coef<INVM_LC>(am, bm, l0 + INVM_LC - m, k - m, lane);
      // degrees past k meet zero coefficient rows; thetas past k are not stored
      if (skip)
        recur_chunk<INVM_LC>(cf, u, sg, z1, z2, e, [](int, double) {});
      else
        recur_chunk<INVM_LC>(cf, u, sg, z1, z2, e, [&](int j, double v) { Z[w][j][lane] = (T)v; });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < INVM_LC ? (k - l0) : INVM_LC;
        retained += (unsigned long long)nl * (unsigned long long)(valid ? 1 : 0);
#pragma unroll
        for (int sl = 0; sl < INVM_LC / 4; ++sl) {
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const T av = Z[w][4 * sl + lq][16 * g + li];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[g][ct] = Mma<T>::mma(av, b[sl][ct], acc[g][ct]);
          }
        }
        wave_lds_sync();
        if constexpr (!F64) {
          if (++since_flush == INVM_FLUSH) {
            since_flush = 0;
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
                for (int v = 0; v < 4; ++v) accd[g][ct][v] += (double)acc[g][ct][v];
                acc[g][ct] = Mma<T>::zero();
              }
          }
        }
      }
    }
    // result register v of lane l holds theta row Mma<T>::row(l / 16, v), column l % 16
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int tt = tile * 64 + 16 * g + Mma<T>::row(lq, v);
        if (tt < k) {
          double* out = FT + ((size_t)tt * k + m) * C;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            if constexpr (F64)
              out[ct * 16 + li] = acc[g][ct][v];
            else
              out[ct * 16 + li] = accd[g][ct][v] + (double)acc[g][ct][v];
          }
        }
      }
  }
  if (counter != nullptr) {
    // retained counts this lane's (l, theta) pairs
    for (int off = 32; off > 0; off >>= 1) retained += __shfl_down(retained, off);
    if (lane == 0 && retained > 0) atomicAdd(counter, retained);
  }
}

// ------------------------------------------------------------------------------------------
// The two contractions on the northern half of the symmetric grid psi_s = pi (2s+1) / (2k),
// s < k/2 (FP64, C >= 16).  With lambda_lm(pi - psi) = (-1)^(l+m) lambda_lm(psi), a degree of
// even l+m meets the sum H(s) + H(k-1-s) of the theta stage's output and one of odd l+m the
// difference, so every (l, m) runs the recursion and the contraction over k/2 nodes instead of
// k.  A chunk starts at l0 = m + 32 i (16 i), so l+m has the parity of the step j within it.
//
// Analysis.  Block: one m pair, one group of 512 northern nodes, 8 waves.  Each wave runs the
// recursion for 64 nodes and writes a 32-degree chunk into a block-wide LDS tile Z[32][512] (even
// steps in rows 0..15, odd steps in rows 16..31).  The contraction is divided by output tile
// rather than by node: wave w owns the 16-column x 16-degree tile (column block ct, parity p) over
// one slice of the 512 nodes (2 slices for C = 32, 4 for C = 16), with that slice's operands
// (sums or differences of H) in registers.  So the cross-wave reduction adds 2 (4) partial tiles
// per output instead of 8, and it runs while the next chunk's recursion fills Z.  Two barriers
// per chunk: Z complete before the products; products done (Z free, partial tiles written)
// before the next recursion.  Wave-uniform skips: a recursion wave whose 64 nodes are all below
// 2^-1100 (or past k/2) flags the chunk, and the contraction skips its 16 k-steps.
// ------------------------------------------------------------------------------------------
constexpr int FS_NW = 8;                 // waves per block
constexpr int FS_LC = 32;                // degrees per chunk (16 even + 16 odd)
constexpr int FS_TB = FS_NW * 64;        // northern nodes per block
constexpr int FS_PS = 18;                // partial-tile row stride (elements)
// row stride of Z: (stride x row + k) mod (banks / element) distinct for the 16 rows x 4 nodes a
// half-wave (FP64) or wave (FP32) reads per k-step
template <typename T> struct FsZStride;
template <> struct FsZStride<double> { static constexpr int v = FS_TB + 3; };
template <> struct FsZStride<float> { static constexpr int v = FS_TB + 4; };

template <int C, typename T>
__global__ __launch_bounds__(512) void k_legendre_fwd_sym(const double* __restrict__ HM, double* __restrict__ R,
                                                          long long part_stride,
                                                          const double* __restrict__ alpha,
                                                          const double* __restrict__ beta,
                                                          const double* __restrict__ cm,
                                                          const double* __restrict__ ut,
                                                          const double* __restrict__ sx,
                                                          const double* __restrict__ st, int k, int Lt, int ng,
                                                          int lmin, unsigned long long* __restrict__ counter) {
  constexpr int CT = C / 16;
  constexpr int NKS = FS_NW / (2 * CT);   // node slices per output tile
  constexpr int KS = FS_TB / NKS;         // nodes per slice
  constexpr int NK = KS / 4;              // k-steps per slice
  constexpr int SRC = KS / 64;            // recursion waves per slice
  constexpr int ZS = FsZStride<T>::v;
  __shared__ __align__(16) T Z[FS_LC][ZS];
  __shared__ __align__(16) T P[FS_NW][16][FS_PS];
  __shared__ double2 coef[FS_NW][FS_LC];   // each wave's copy of a chunk's recursion coefficients
  __shared__ int negl[FS_NW];              // recursion wave w contributes nothing to this chunk
  unsigned long long retained = 0;
  const int kh = k / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int pair = blockIdx.x / ng;
  const int grp = blockIdx.x % ng;
  // recursion role: nodes grp*512 + w*64 + lane
  const int tile = grp * FS_NW + w;
  const int t = tile * 64 + lane;
  const bool valid = t < kh;
  const bool tile_live = tile * 64 < kh;
  const int nt = tile_live ? ((kh - tile * 64) < 64 ? (kh - tile * 64) : 64) : 0;
  const double u = valid ? ut[t] : -1.0;
  const double sg = 1.0;   // every node (and every idle lane) is northern
  const double s = valid ? st[t] : 1.0;
  // contraction role: column block ct, parity p, node slice h
  const int ct = w % CT, p = (w / CT) & 1, h = w / (2 * CT);
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  double* __restrict__ Rg = R + (size_t)grp * part_stride;
  double2* cfl = coef[w];

  // the output rows of one chunk: the slices' partial tiles added in order, one column pair per
  // thread, 16-byte global stores
  auto reduce = [&](int m, int l0) {
    for (int idx = threadIdx.x; idx < FS_LC * C / 2; idx += FS_NW * 64) {
      const int cp = idx % (C / 2), rest = idx / (C / 2);
      const int r = rest & 15, pr = rest >> 4;
      const int c = 2 * cp, ctt = c >> 4, cl = c & 15;
      const int l = l0 + 2 * r + pr;
      if (l < k) {
        double2 sum = make_double2(0.0, 0.0);
#pragma unroll
        for (int hh = 0; hh < NKS; ++hh) {
          const T* pt = &P[(hh * 2 + pr) * CT + ctt][r][cl];
          sum.x += (double)pt[0];
          sum.y += (double)pt[1];
        }
        *reinterpret_cast<double2*>(&Rg[(tri_off(k, m) + (l - m)) * C + c]) = sum;
      }
    }
  };

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Hm = HM + (size_t)m * k * C;
    // operands of this wave's tile: H(s) + H(k-1-s) (p = 0) or H(s) - H(k-1-s) (p = 1) at the slice's
    // nodes; the theta stage stores them at nodes [0, k/2) and [k/2, k), column-pair major
    T a[NK];
    {
      // k/2 is a multiple of 32 and the slice starts on a multiple of 128, so whether node
      // base + 4 kk + lq exists does not depend on lq: nkv k-steps of the slice are in range
      const int base = grp * FS_TB + h * KS;
      const int nkv = kh <= base ? 0 : ((kh - base) / 4 < NK ? (kh - base) / 4 : NK);
      const int c = ct * 16 + li;
      const double* col = Hm + (size_t)(c >> 1) * k * 2 + (c & 1) + (p ? (size_t)kh * 2 : 0) +
                          (size_t)(base + lq) * 2;
      if (nkv == NK) {
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) a[kk] = (T)col[(size_t)kk * 8];
      } else {
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) a[kk] = (T)(kk < nkv ? col[(size_t)kk * 8] : 0.0);
      }
    }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf = chunk_coef<FS_LC>(am, bm, 0, k - m, lane);
    int lprev = -1;   // the chunk whose partial tiles wait to be reduced

    for (int l0 = m; l0 < k; l0 += FS_LC) {
      // below the degree floor: no products, and no rows of R (the caller reads none of them)
      const bool below = l0 + FS_LC <= lmin;   // block-uniform
      stage_coef<FS_LC>(cfl, cf, lane);
      cf = chunk_coef<FS_LC>(am, bm, l0 + FS_LC - m, k - m, lane);   // the next chunk's, in flight
      wave_lds_sync();
      const bool ngw = !tile_live || __all(!valid || negligible(z1, z2, e));
      auto nosink = [](int, double) {};
      if (below) {
        recur_chunk_lds<FS_LC>(cfl, u, sg, z1, z2, e, nosink);
        continue;
      }
      // phase A: this chunk's recursion into Z (none when the products skip this wave's nodes), the
      // previous chunk's reduction
      if (ngw)
        recur_chunk_lds<FS_LC>(cfl, u, sg, z1, z2, e, nosink);
      else
        recur_chunk_lds<FS_LC>(cfl, u, sg, z1, z2, e,
                               [&](int j, double v) { Z[(j & 1) * 16 + (j >> 1)][w * 64 + lane] = (T)v; });
      if (lane == 0) negl[w] = ngw;
      if (!ngw) retained += (unsigned long long)((k - l0) < FS_LC ? (k - l0) : FS_LC) * nt;
      if (lprev >= 0) reduce(m, lprev);
      __syncthreads();   // Z holds the chunk; the previous partial tiles are read
      // phase B: the products of this wave's tile
      typename Mma<T>::acc_t acc0 = Mma<T>::zero(), acc1 = Mma<T>::zero();
#pragma unroll
      for (int sw = 0; sw < SRC; ++sw) {
        if (negl[h * SRC + sw]) continue;   // wave-uniform
#pragma unroll
        for (int q = 0; q < 16; q += 2) {
          const int kk = sw * 16 + q;
          const T b0 = Z[p * 16 + li][h * KS + 4 * kk + lq];
          const T b1 = Z[p * 16 + li][h * KS + 4 * kk + 4 + lq];
          acc0 = Mma<T>::mma(a[kk], b0, acc0);
          acc1 = Mma<T>::mma(a[kk + 1], b1, acc1);
        }
      }
      // partial tile: register v holds column row(lq, v) of the tile, degree row li
#pragma unroll
      for (int v = 0; v < 4; ++v) P[w][li][Mma<T>::row(lq, v)] = acc0[v] + acc1[v];
      __syncthreads();   // partial tiles written; every wave is done reading Z
      lprev = l0;
    }
    if (lprev >= 0) reduce(m, lprev);
  }
  if (counter != nullptr && lane == 0 && retained > 0) atomicAdd(counter, retained);
}

// The same analysis with the FP32 contraction, organised by node instead: each wave multiplies
// its own 64 nodes' z tile (wave-private, no barrier between recursion and products) into partial
// sums of all 32 x C outputs, which the waves write to a double-buffered area and add up after one
// barrier per chunk.  (The block-wide tile of the FP64 kernel, with one chain of FP32 products over
// 256 nodes per tile, measured slower here and rounds more: FP32 sums of 64 products per partial
// keep the error of this mode at a quarter of its bound.)
constexpr int FWW_ZS = 66;      // z-tile row stride (elements): conflict-free B reads
template <int C>
__global__ __launch_bounds__(512) void k_legendre_fwd_sym_f32(const double* __restrict__ HM, double* __restrict__ R,
                                                              long long part_stride,
                                                              const double* __restrict__ alpha,
                                                              const double* __restrict__ beta,
                                                              const double* __restrict__ cm,
                                                              const double* __restrict__ ut,
                                                              const double* __restrict__ st, int k, int Lt, int ng,
                                                              int lmin, unsigned long long* __restrict__ counter) {
  typedef float T;
  constexpr int CT = C / 16;
  constexpr int RS = 2 * ((C / 2) | 1);
  __shared__ __align__(16) T Z[FS_NW][FS_LC][FWW_ZS];
  __shared__ __align__(16) T P[2][FS_NW][FS_LC][RS];
  __shared__ double2 coef[FS_NW][FS_LC];
  unsigned long long retained = 0;
  const int kh = k / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  double2* cfl = coef[w];
  const int pair = blockIdx.x / ng;
  const int grp = blockIdx.x % ng;
  const int tile = grp * FS_NW + w;
  const int t = tile * 64 + lane;
  const bool valid = t < kh;
  const bool tile_live = tile * 64 < kh;
  const double u = valid ? ut[t] : -1.0;
  const double sg = 1.0;
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  double* __restrict__ Rg = R + (size_t)grp * part_stride;
  int nred = 0;   // chunks reduced so far (selects the partial-sum buffer)

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Hm = HM + (size_t)m * k * C;
    // operands: ap = H(s) + H(k-1-s) (even l+m), an = H(s) - H(k-1-s) (odd l+m)
    T ap[16][CT], an[16][CT];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int tg = tile * 64 + 4 * kk + lq;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = ct * 16 + li;
        const double* col = Hm + (size_t)(c >> 1) * k * 2 + (c & 1);
        ap[kk][ct] = (T)(tg < kh ? col[(size_t)tg * 2] : 0.0);
        an[kk][ct] = (T)(tg < kh ? col[(size_t)(kh + tg) * 2] : 0.0);
      }
    }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf = chunk_coef<FS_LC>(am, bm, 0, k - m, lane);

    for (int l0 = m; l0 < k; l0 += FS_LC) {
      typename Mma<T>::acc_t acc[2][CT];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[x][ct] = Mma<T>::zero();
      const bool below = l0 + FS_LC <= lmin;
      const bool skip = !tile_live || below || __all(!valid || negligible(z1, z2, e));
      stage_coef<FS_LC>(cfl, cf, lane);
      cf = chunk_coef<FS_LC>(am, bm, l0 + FS_LC - m, k - m, lane);   // the next chunk's, in flight
      wave_lds_sync();
      if (skip)
        recur_chunk_lds<FS_LC>(cfl, u, sg, z1, z2, e, [](int, double) {});
      else
        recur_chunk_lds<FS_LC>(cfl, u, sg, z1, z2, e,
                               [&](int j, double v) { Z[w][(j & 1) * (FS_LC / 2) + (j >> 1)][lane] = (T)v; });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < FS_LC ? (k - l0) : FS_LC;
        const int nt = (kh - tile * 64) < 64 ? (kh - tile * 64) : 64;
        retained += (unsigned long long)nl * (unsigned long long)nt;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const int tl = 4 * kk + lq;
          const T b0 = Z[w][li][tl], b1 = Z[w][16 + li][tl];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            acc[0][ct] = Mma<T>::mma(ap[kk][ct], b0, acc[0][ct]);
            acc[1][ct] = Mma<T>::mma(an[kk][ct], b1, acc[1][ct]);
          }
        }
      }
      if (below) continue;   // block-uniform
      const int pb = nred & 1;
#pragma unroll
      for (int lt2 = 0; lt2 < 2; ++lt2)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) P[pb][w][lt2 * 16 + li][ct * 16 + Mma<T>::row(lq, v)] = acc[lt2][ct][v];
      __syncthreads();
      for (int idx = threadIdx.x; idx < FS_LC * C / 2; idx += FS_NW * 64) {
        const int lloc = idx / (C / 2), c = 2 * (idx % (C / 2));
        const int l = l0 + 2 * (lloc & 15) + (lloc >> 4);
        if (l < k) {
          double2 sum = make_double2(0.0, 0.0);
#pragma unroll
          for (int ww = 0; ww < FS_NW; ++ww) {
            const float2 v = *reinterpret_cast<const float2*>(&P[pb][ww][lloc][c]);
            sum.x += (double)v.x;
            sum.y += (double)v.y;
          }
          *reinterpret_cast<double2*>(&Rg[(tri_off(k, m) + (l - m)) * C + c]) = sum;
        }
      }
      ++nred;
    }
  }
  if (counter != nullptr && lane == 0 && retained > 0) atomicAdd(counter, retained);
}

// Synthesis: E(s) = sum over even l+m, O(s) = sum over odd l+m of z_l(psi_s) S[l][c] on the
// northern nodes; F(psi_s) = E + O and F(psi_{k-1-s}) = E - O, written column-pair major,
// FS[((m*(C/2) + c/2)*k + s)*2 + c%2], s < k (read by the resampling to the MW nodes).
template <int C, int NW, typename T>
__device__ __forceinline__ void inv_sym_body(const double* __restrict__ S, double* __restrict__ FS,
                                             const double* __restrict__ alpha, const double* __restrict__ beta,
                                             const double* __restrict__ cm, const double* __restrict__ ut,
                                             const double* __restrict__ st, int k, int Lt, int pair, int tb,
                                             int lmin, unsigned long long& retained) {
  constexpr int CT = C / 16;
  constexpr bool F64 = sizeof(T) == sizeof(double);
  // the coefficient rows of a chunk, loaded once per block (the four waves share them) into a
  // double-buffered tile; row stride 40 doubles puts the rows a half wave reads (2 apart) 16
  // banks apart
  constexpr int SBS = 40;
  constexpr int PER = INVM_LC * C / (NW * 64);   // doubles per thread per chunk (2 for C = 32, NW = 4)
  __shared__ T Z[NW][INVM_LC][INVM_ZS];
  __shared__ double Sb[2][INVM_LC][SBS];
  const int kh = k / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int tile = tb * NW + w;
  const int t = tile * 64 + lane;
  const bool valid = t < kh;
  const double u = valid ? ut[t] : -1.0;
  const double sg = 1.0;
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Sm = S + tri_off(k, m) * C;
    typename Mma<T>::acc_t accE[4][CT], accO[4][CT];
    // FP32 path: north (E + O) and south (E - O) sums in FP64, fed every INVM_FLUSH chunks
    double accN[F64 ? 1 : 4][F64 ? 1 : CT][4], accS[F64 ? 1 : 4][F64 ? 1 : CT][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        accE[g][ct] = Mma<T>::zero();
        accO[g][ct] = Mma<T>::zero();
      }
    if constexpr (!F64) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) accN[g][ct][v] = accS[g][ct][v] = 0.0;
    }
    int since_flush = 0;
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf_next = chunk_coef<INVM_LC>(am, bm, 0, k - m, lane);
    // tile element (row r, column c) of this thread: r = (tid * PER) / C, c = (tid * PER) % C + i
    const int tr = (threadIdx.x * PER) / C, tc = (threadIdx.x * PER) % C;
    double pre[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) pre[i] = (m + tr < k) ? Sm[(size_t)tr * C + tc + i] : 0.0;
    __syncthreads();   // the previous m's last tile has been read
#pragma unroll
    for (int i = 0; i < PER; ++i) Sb[0][tr][tc + i] = pre[i];
    __syncthreads();
    int cur = 0;
    for (int l0 = m; l0 < k; l0 += INVM_LC) {
      // below the degree floor the rows are zero: no products; while the next chunk is below it too,
      // no rows are staged and the block does not synchronise (block-uniform)
      const bool below = l0 + INVM_LC <= lmin;
      const bool stage = l0 + INVM_LC < k && l0 + 2 * INVM_LC > lmin;
      const bool skip = below || __all(!valid || negligible(z1, z2, e));
      // the next chunk's rows, in flight during this chunk's recursion and products
      if (stage) {
#pragma unroll
        for (int i = 0; i < PER; ++i)
          pre[i] = (l0 + INVM_LC + tr < k) ? Sm[(size_t)(l0 + INVM_LC - m + tr) * C + tc + i] : 0.0;
      }
      // (coefficients by lane broadcasts: staging them in LDS, as the analysis does, measured slower
      // here, where the z tile and the coefficient rows already load the LDS every chunk)
      const double cf = cf_next;
      cf_next = chunk_coef<INVM_LC>(am, bm, l0 + INVM_LC - m, k - m, lane);
      if (skip)
        recur_chunk<INVM_LC>(cf, u, sg, z1, z2, e, [](int, double) {});
      else
        recur_chunk<INVM_LC>(cf, u, sg, z1, z2, e,
                             [&](int j, double v) { Z[w][(j & 1) * (INVM_LC / 2) + (j >> 1)][lane] = (T)v; });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < INVM_LC ? (k - l0) : INVM_LC;
        retained += (unsigned long long)nl * (unsigned long long)(valid ? 1 : 0);
#pragma unroll
        for (int sl = 0; sl < INVM_LC / 4; ++sl) {
          // k-step sl covers the steps jd = (sl >> 1) + 8 (sl & 1) + 2 lq: sl = 0, 1 even, sl = 2, 3 odd
          const int jd = (sl >> 1) + 8 * (sl & 1) + 2 * lq;
          T bv[CT];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) bv[ct] = (T)Sb[cur][jd][ct * 16 + li];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const T av = Z[w][4 * sl + lq][16 * g + li];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              if (sl < 2)
                accE[g][ct] = Mma<T>::mma(av, bv[ct], accE[g][ct]);
              else
                accO[g][ct] = Mma<T>::mma(av, bv[ct], accO[g][ct]);
            }
          }
        }
        wave_lds_sync();
        if constexpr (!F64) {
          if (++since_flush == INVM_FLUSH) {
            since_flush = 0;
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                  const double E = (double)accE[g][ct][v], O = (double)accO[g][ct][v];
                  accN[g][ct][v] += E + O;
                  accS[g][ct][v] += E - O;
                }
                accE[g][ct] = Mma<T>::zero();
                accO[g][ct] = Mma<T>::zero();
              }
          }
        }
      }
      if (stage) {
#pragma unroll
        for (int i = 0; i < PER; ++i) Sb[cur ^ 1][tr][tc + i] = pre[i];
        __syncthreads();   // the next tile is written and this one has been read by every wave
        cur ^= 1;
      }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int tt = tile * 64 + 16 * g + Mma<T>::row(lq, v);
        if (tt < kh) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const int c = ct * 16 + li;
            double* col = FS + ((size_t)m * C + (c & ~1)) * k + (c & 1);
            const double E = (double)accE[g][ct][v], O = (double)accO[g][ct][v];
            if constexpr (F64) {
              col[(size_t)tt * 2] = E + O;
              col[(size_t)(k - 1 - tt) * 2] = E - O;
            } else {
              col[(size_t)tt * 2] = accN[g][ct][v] + (E + O);
              col[(size_t)(k - 1 - tt) * 2] = accS[g][ct][v] + (E - O);
            }
          }
        }
      }
  }
}


template <int C, typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 1) void k_legendre_inv_sym(const double* __restrict__ S, double* __restrict__ FS,
                                                          const double* __restrict__ alpha,
                                                          const double* __restrict__ beta,
                                                          const double* __restrict__ cm,
                                                          const double* __restrict__ ut,
                                                          const double* __restrict__ sx,
                                                          const double* __restrict__ st, int k, int Lt, int ntb,
                                                          int lmin, unsigned long long* __restrict__ counter) {
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  unsigned long long retained = 0;
  inv_sym_body<C, 4, T>(S, FS, alpha, beta, cm, ut, st, k, Lt, spread_pairs(blk / ntb, (k + 1) / 2), blk % ntb, lmin,
                        retained);
  if (counter != nullptr) {
    for (int off = 32; off > 0; off >>= 1) retained += __shfl_down(retained, off);
    if ((threadIdx.x & 63) == 0 && retained > 0) atomicAdd(counter, retained);
  }
}

int legendre_forward_groups_sym(int k) { return (k / 2 + FWD_TB - 1) / FWD_TB; }

hipError_t launch_legendre_forward_sym(const ShtTables& T, const LegTables& G, const Batch& b, const double* HM,
                                       double* R, long long part_stride, int precision, int lmin,
                                       unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  if (!T.sym || (k & 1)) return hipErrorInvalidValue;
  if (precision == S2LET_MIXED_BF16X3)
    return launch_legendre_forward_bf16_sym(T, G, b, HM, R, part_stride, lmin, counter, s);
  const int ng = legendre_forward_groups_sym(k);
  const dim3 grid(((k + 1) / 2) * ng), block(FWD_NW * 64);
  const bool f32 = precision == S2LET_MIXED_FP32;
  if (b.C == 32 && f32)
    k_legendre_fwd_sym_f32<32><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s, T.st_s, k,
                                                      G.Lt, ng, lmin, counter);
  else if (b.C == 32)
    k_legendre_fwd_sym<32, double><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s, T.sx_s,
                                                          T.st_s, k, G.Lt, ng, lmin, counter);
  else if (b.C == 16 && f32)
    k_legendre_fwd_sym_f32<16><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s, T.st_s, k,
                                                      G.Lt, ng, lmin, counter);
  else if (b.C == 16)
    k_legendre_fwd_sym<16, double><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s, T.sx_s,
                                                          T.st_s, k, G.Lt, ng, lmin, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_legendre_inverse_sym(const ShtTables& T, const LegTables& G, const Batch& b, const double* S,
                                       double* FS, int precision, int lmin, unsigned long long* counter,
                                       hipStream_t s) {
  const int k = T.k;
  if (!T.sym || (k & 1)) return hipErrorInvalidValue;
  if (precision == S2LET_MIXED_BF16X3) return launch_legendre_inverse_bf16_sym(T, G, b, S, FS, lmin, counter, s);
  const int ntb = (k / 2 + 255) / 256;
  const dim3 grid(((k + 1) / 2) * ntb), block(256);
  const bool f32 = precision == S2LET_MIXED_FP32;
  // 32 columns in FP32 would need 310 registers (FP64 north/south running sums beside the FP32
  // partial sums): one wave per SIMD, slower than the FP64 kernel at two.  The FP64 kernel serves.
  if (b.C == 32)
    k_legendre_inv_sym<32, double><<<grid, block, 0, s>>>(S, FS, G.alpha, G.beta, G.cm, T.ut_s, T.sx_s, T.st_s, k,
                                                          G.Lt, ntb, lmin, counter);
  else if (b.C == 16 && f32)
    k_legendre_inv_sym<16, float><<<grid, block, 0, s>>>(S, FS, G.alpha, G.beta, G.cm, T.ut_s, T.sx_s, T.st_s, k,
                                                         G.Lt, ntb, lmin, counter);
  else if (b.C == 16)
    k_legendre_inv_sym<16, double><<<grid, block, 0, s>>>(S, FS, G.alpha, G.beta, G.cm, T.ut_s, T.sx_s, T.st_s, k,
                                                          G.Lt, ntb, lmin, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Persistent launches for uneven batches: the items of many transforms (band-limits 64 to 2048)
// in one launch.  The analysis body is the node-organised form (each wave multiplies its own 64
// nodes' z tile into partial sums of all 32 x C outputs; the partial sums of the block's nw
// waves overwrite their z tiles and are added in order), which works for any number of waves per
// block; the synthesis body is inv_sym_body.  Blocks take items from a device counter.
// ------------------------------------------------------------------------------------------
template <int C, int NW>
__device__ __forceinline__ void fwd_sym_wave_body(const double* __restrict__ HM, double* __restrict__ R,
                                                  long long part_stride, const double* __restrict__ alpha,
                                                  const double* __restrict__ beta, const double* __restrict__ cm,
                                                  const double* __restrict__ ut, const double* __restrict__ st,
                                                  int k, int Lt, int pair, int grp, int lmin,
                                                  unsigned long long& retained) {
  typedef double T;
  constexpr int CT = C / 16;
  constexpr int RS = 2 * ((C / 2) | 1);
  static_assert(RS <= FWW_ZS, "a wave's partial sums must fit in its z tile");
  __shared__ __align__(16) T Z[NW][FS_LC][FWW_ZS];
  __shared__ double2 coef[NW][FS_LC];
  const int kh = k / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  double2* cfl = coef[w];
  const int tile = grp * NW + w;
  const int t = tile * 64 + lane;
  const bool valid = t < kh;
  const bool tile_live = tile * 64 < kh;
  const double u = valid ? ut[t] : -1.0;
  const double sg = 1.0;
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  double* __restrict__ Rg = R + (size_t)grp * part_stride;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Hm = HM + (size_t)m * k * C;
    T ap[16][CT], an[16][CT];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int tg = tile * 64 + 4 * kk + lq;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = ct * 16 + li;
        const double* col = Hm + (size_t)(c >> 1) * k * 2 + (c & 1);
        ap[kk][ct] = tg < kh ? col[(size_t)tg * 2] : 0.0;
        an[kk][ct] = tg < kh ? col[(size_t)(kh + tg) * 2] : 0.0;
      }
    }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf = chunk_coef<FS_LC>(am, bm, 0, k - m, lane);

    for (int l0 = m; l0 < k; l0 += FS_LC) {
      typename Mma<T>::acc_t acc[2][CT];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[x][ct] = Mma<T>::zero();
      const bool below = l0 + FS_LC <= lmin;
      const bool skip = !tile_live || below || __all(!valid || negligible(z1, z2, e));
      stage_coef<FS_LC>(cfl, cf, lane);
      cf = chunk_coef<FS_LC>(am, bm, l0 + FS_LC - m, k - m, lane);
      wave_lds_sync();
      if (skip)
        recur_chunk_lds<FS_LC>(cfl, u, sg, z1, z2, e, [](int, double) {});
      else
        recur_chunk_lds<FS_LC>(cfl, u, sg, z1, z2, e,
                               [&](int j, double v) { Z[w][(j & 1) * (FS_LC / 2) + (j >> 1)][lane] = v; });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < FS_LC ? (k - l0) : FS_LC;
        const int nt = (kh - tile * 64) < 64 ? (kh - tile * 64) : 64;
        retained += (unsigned long long)nl * (unsigned long long)nt;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const int tl = 4 * kk + lq;
          const T b0 = Z[w][li][tl], b1 = Z[w][16 + li][tl];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            acc[0][ct] = Mma<T>::mma(ap[kk][ct], b0, acc[0][ct]);
            acc[1][ct] = Mma<T>::mma(an[kk][ct], b1, acc[1][ct]);
          }
        }
      }
      if (below) continue;   // block-uniform
      wave_lds_sync();       // this wave's reads of its z tile are done
      T* Pw = &Z[w][0][0];
#pragma unroll
      for (int lt2 = 0; lt2 < 2; ++lt2)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) Pw[(lt2 * 16 + li) * RS + ct * 16 + Mma<T>::row(lq, v)] = acc[lt2][ct][v];
      __syncthreads();
      for (int idx = threadIdx.x; idx < FS_LC * C / 2; idx += NW * 64) {
        const int lloc = idx / (C / 2), c = 2 * (idx % (C / 2));
        const int l = l0 + 2 * (lloc & 15) + (lloc >> 4);
        if (l < k) {
          double2 sum = make_double2(0.0, 0.0);
#pragma unroll
          for (int ww = 0; ww < NW; ++ww) {
            const double2 v = *reinterpret_cast<const double2*>(&Z[ww][0][0] + lloc * RS + c);
            sum.x += v.x;
            sum.y += v.y;
          }
          *reinterpret_cast<double2*>(&Rg[(tri_off(k, m) + (l - m)) * C + c]) = sum;
        }
      }
      __syncthreads();   // the next chunk's recursion overwrites the partial sums
    }
  }
}

__global__ void k_reset_u32(unsigned* __restrict__ p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Takes the next item index for the whole block (thread 0 draws it, the barriers publish it and
// keep it until every thread has read it).
__device__ __forceinline__ int next_item(unsigned* __restrict__ next) {
  __shared__ int s_item;
  __syncthreads();
  if (threadIdx.x == 0) s_item = (int)atomicAdd(next, 1u);
  __syncthreads();
  return s_item;
}

// (two waves per SIMD: at most 256 registers, whatever the block size)
template <int C, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_legendre_fwd_persist(const LegTask* __restrict__ tasks,
                                                                  const LegItem* __restrict__ items, int nitems,
                                                                  unsigned* __restrict__ next,
                                                                  const double* __restrict__ alpha,
                                                                  const double* __restrict__ beta,
                                                                  const double* __restrict__ cm, int Lt) {
  unsigned long long retained = 0;
  for (int it = next_item(next); it < nitems; it = next_item(next)) {
    const LegItem I = items[it];
    const LegTask T = tasks[I.task];
    fwd_sym_wave_body<C, NW>(T.in, T.out, T.part_stride, alpha, beta, cm, T.ut, T.st, T.k, Lt, I.pair, I.sub, T.lmin,
                             retained);
  }
}

template <int C, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_legendre_inv_persist(const LegTask* __restrict__ tasks,
                                                                  const LegItem* __restrict__ items, int nitems,
                                                                  unsigned* __restrict__ next,
                                                                  const double* __restrict__ alpha,
                                                                  const double* __restrict__ beta,
                                                                  const double* __restrict__ cm, int Lt) {
  unsigned long long retained = 0;
  for (int it = next_item(next); it < nitems; it = next_item(next)) {
    const LegItem I = items[it];
    const LegTask T = tasks[I.task];
    inv_sym_body<C, NW, double>(T.in, T.out, alpha, beta, cm, T.ut, T.st, T.k, Lt, I.pair, I.sub, T.lmin, retained);
  }
}

int legendre_persist_groups(int k, int nw) { return (k / 2 + nw * 64 - 1) / (nw * 64); }

bool legendre_persist_shape_ok(bool, int nw) { return nw == 1 || nw == 2 || nw == 4; }

int legendre_persist_blocks_per_cu(bool analysis, int nw) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define S2LET_OCC(NWV)                                                                                       \
  if (nw == NWV)                                                                                             \
    e = analysis ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_legendre_fwd_persist<32, NWV>, NWV * 64, 0) \
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_legendre_inv_persist<32, NWV>, NWV * 64, 0);
  S2LET_OCC(1)
  S2LET_OCC(2)
  S2LET_OCC(4)
#undef S2LET_OCC
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_legendre_persist(bool analysis, int nw, const LegTask* tasks, const LegItem* items, int nitems,
                                   unsigned* next, const LegTables& G, int nblocks, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (!legendre_persist_shape_ok(analysis, nw) || nblocks < 1) return hipErrorInvalidValue;
  k_reset_u32<<<1, 64, 0, s>>>(next, 1);
  const dim3 grid(nblocks), block(nw * 64);
  if (analysis) {
    switch (nw) {
      case 1: k_legendre_fwd_persist<32, 1><<<grid, block, 0, s>>>(tasks, items, nitems, next, G.alpha, G.beta, G.cm, G.Lt); break;
      case 2: k_legendre_fwd_persist<32, 2><<<grid, block, 0, s>>>(tasks, items, nitems, next, G.alpha, G.beta, G.cm, G.Lt); break;
      default: k_legendre_fwd_persist<32, 4><<<grid, block, 0, s>>>(tasks, items, nitems, next, G.alpha, G.beta, G.cm, G.Lt); break;
    }
  } else {
    switch (nw) {
      case 1: k_legendre_inv_persist<32, 1><<<grid, block, 0, s>>>(tasks, items, nitems, next, G.alpha, G.beta, G.cm, G.Lt); break;
      case 2: k_legendre_inv_persist<32, 2><<<grid, block, 0, s>>>(tasks, items, nitems, next, G.alpha, G.beta, G.cm, G.Lt); break;
      default: k_legendre_inv_persist<32, 4><<<grid, block, 0, s>>>(tasks, items, nitems, next, G.alpha, G.beta, G.cm, G.Lt); break;
    }
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Batches below 16 columns run the FP64 VALU kernel in every precision mode.
template <int C>
static hipError_t inv_c(const ShtTables& T, const LegTables& G, const double* S, double* FT, int precision,
                        unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  const int ntb = (k + 255) / 256;
  const int npairs = (k + 1) / 2;
  if (C >= 16) {
    constexpr int CC = C >= 16 ? C : 16;
    if (precision == S2LET_MIXED_FP32)
      k_legendre_inv_mfma<CC, float><<<npairs * ntb, 256, 0, s>>>(S, FT, G.alpha, G.beta, G.cm, T.ut, T.sx,
                                                                  T.st, k, G.Lt, ntb, counter);
    else
      k_legendre_inv_mfma<CC, double><<<npairs * ntb, 256, 0, s>>>(S, FT, G.alpha, G.beta, G.cm, T.ut, T.sx,
                                                                   T.st, k, G.Lt, ntb, counter);
    return hipGetLastError();
  }
  k_legendre_inv<C><<<npairs * ntb, 256, 0, s>>>(S, FT, G.alpha, G.beta, G.cm, T.ut, T.sx, T.st, k, G.Lt,
                                                 ntb, counter);
  return hipGetLastError();
}

int legendre_forward_groups(int k) { return (k + FWD_TB - 1) / FWD_TB; }

template <int C>
static hipError_t fwd_c(const ShtTables& T, const LegTables& G, const double* HM, double* R,
                        long long part_stride, int precision, unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  const int npairs = (k + 1) / 2;
  const int ng = legendre_forward_groups(k);
  if (precision == S2LET_MIXED_FP32)
    k_legendre_fwd<C, float><<<npairs * ng, FWD_NW * 64, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm,
                                                                 T.ut, T.sx, T.st, k, G.Lt, ng, counter);
  else
    k_legendre_fwd<C, double><<<npairs * ng, FWD_NW * 64, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm,
                                                                  T.ut, T.sx, T.st, k, G.Lt, ng, counter);
  return hipGetLastError();
}

hipError_t launch_legendre_inverse(const ShtTables& T, const LegTables& G, const Batch& b,
                                   const double* S, double* FT, int precision,
                                   unsigned long long* counter, hipStream_t s) {
  if (precision == S2LET_MIXED_BF16X3 && b.C >= 16) return launch_legendre_inverse_bf16(T, G, b, S, FT, counter, s);
  switch (b.C) {
    case 2: return inv_c<2>(T, G, S, FT, precision, counter, s);
    case 4: return inv_c<4>(T, G, S, FT, precision, counter, s);
    case 8: return inv_c<8>(T, G, S, FT, precision, counter, s);
    case 16: return inv_c<16>(T, G, S, FT, precision, counter, s);
    case 32: return inv_c<32>(T, G, S, FT, precision, counter, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_legendre_forward(const ShtTables& T, const LegTables& G, const Batch& b,
                                   const double* HM, double* R, long long part_stride, int precision,
                                   unsigned long long* counter, hipStream_t s) {
  if (precision == S2LET_MIXED_BF16X3) return launch_legendre_forward_bf16(T, G, b, HM, R, part_stride, counter, s);
  switch (b.C) {
    case 2: return fwd_c<2>(T, G, HM, R, part_stride, precision, counter, s);
    case 4: return fwd_c<4>(T, G, HM, R, part_stride, precision, counter, s);
    case 8: return fwd_c<8>(T, G, HM, R, part_stride, precision, counter, s);
    case 16: return fwd_c<16>(T, G, HM, R, part_stride, precision, counter, s);
    case 32: return fwd_c<32>(T, G, HM, R, part_stride, precision, counter, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace s2let
