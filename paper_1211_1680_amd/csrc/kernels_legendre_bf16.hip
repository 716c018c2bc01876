// Legendre contraction in mixed precision "BF16x3" (S2LET_MIXED_BF16X3): the same products as
// the FP64 kernels (Eqs. (1) and (2) on the MW grid, Sect. 3.2), with both operands split into
// two bfloat16 parts, x = x_hi + x_lo (x_hi = bf16(x), x_lo = bf16(x - x_hi), both rounded to
// nearest), and the three leading products x_hi y_hi + x_hi y_lo + x_lo y_hi accumulated in FP32
// on v_mfma_f32_16x16x32_bf16.  The dropped x_lo y_lo term and the split residuals are about
// 2^-16 of each product.  The recursion that generates lambda_lm stays in FP64 (legendre_rec.h);
// FP32 partial sums are carried into FP64 every 64 terms.
//
// v_mfma_f32_16x16x32_bf16 lane layout (lane l, lq = l / 16, li = l % 16): A holds
// A[li][8 lq + e] and B holds B[8 lq + e][li] for e = 0..7 (eight bf16 per operand); result
// register v holds D[4 lq + v][li].
#include "common.h"
#include "legendre_rec.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const float f = (float)x;
  hi = (__bf16)f;
  lo = (__bf16)(f - (float)hi);
}

__device__ __forceinline__ v4f mma_bf16(bf16x8 a, bf16x8 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// three-product update acc += a_hi b_hi + a_hi b_lo + a_lo b_hi
__device__ __forceinline__ v4f mma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, v4f c) {
  c = mma_bf16(ah, bh, c);
  c = mma_bf16(ah, bl, c);
  return mma_bf16(al, bh, c);
}

// ------------------------------------------------------------------------------------------
// Analysis, D[c][l] = sum_t H'[t][c] z_l(theta_t): A = 16 columns x 32 thetas, B = 32 thetas x
// 16 degrees.  Same decomposition as the FP64 kernel: block = 8 waves x 64 thetas of one m pair,
// H' operands in registers for the whole m (split once), z tiles per 32 degrees in a
// wave-private LDS tile [degree][theta] of bf16 hi and lo parts, FP64 reduction across waves.
// ------------------------------------------------------------------------------------------
constexpr int FB_NW = 8;         // waves per block
constexpr int FB_LC = 32;        // degrees per chunk
constexpr int FB_ZR = 72;        // LDS row (bf16 elements): 64 thetas + 8, rows 16-byte aligned

template <int C>
__global__ __launch_bounds__(512) void k_legendre_fwd_bf16(const double* __restrict__ HM, double* __restrict__ R,
                                                           long long part_stride,
                                                           const double* __restrict__ alpha,
                                                           const double* __restrict__ beta,
                                                           const double* __restrict__ cm,
                                                           const double* __restrict__ ut,
                                                           const double* __restrict__ sx,
                                                           const double* __restrict__ st, int k, int Lt, int ng,
                                                           unsigned long long* __restrict__ counter) {
  constexpr int CT = C >= 16 ? C / 16 : 1;
  constexpr int RS = 2 * ((C / 2) | 1);
  constexpr int ZBYTES = FB_NW * 2 * FB_LC * FB_ZR * 2;
  constexpr int RBYTES = FB_NW * FB_LC * RS * (int)sizeof(double);
  __shared__ __align__(16) char smem[ZBYTES > RBYTES ? ZBYTES : RBYTES];
  // Zt[w][0] = hi parts, Zt[w][1] = lo parts, each [degree][theta]
  __bf16 (*Zt)[2][FB_LC][FB_ZR] = reinterpret_cast<__bf16 (*)[2][FB_LC][FB_ZR]>(smem);
  double* red = reinterpret_cast<double*>(smem);
  unsigned long long retained = 0;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int pair = blockIdx.x / ng;
  const int grp = blockIdx.x % ng;
  const int tile = grp * FB_NW + w;
  const int t = tile * 64 + lane;
  const bool valid = t < k;
  const bool tile_live = tile * 64 < k;
  const double u = valid ? ut[t] : -1.0;
  const double sg = valid ? sx[t] : -1.0;
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  double* __restrict__ Rg = R + (size_t)grp * part_stride;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Hm = HM + (size_t)m * k * C;
    // operands: element e of a?[kb][ct] = H'[tile*64 + 32 kb + 8 lq + e][ct*16 + li]
    bf16x8 ah[2][CT], al[2][CT];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int tg = tile * 64 + 32 * kb + 8 * lq + e;
          const int c = ct * 16 + li;
          const double h = (tg < k && c < C) ? Hm[(size_t)tg * C + c] : 0.0;
          __bf16 hi, lo;
          split_bf16(h, hi, lo);
          ah[kb][ct][e] = hi;
          al[kb][ct][e] = lo;
        }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf_next = chunk_coef<FB_LC>(am, bm, 0, k - m, lane);

    for (int l0 = m; l0 < k; l0 += FB_LC) {
      v4f acc[2][CT];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[x][ct] = v4f{0.f, 0.f, 0.f, 0.f};
      const bool skip = !tile_live || __all(!valid || negligible(z1, z2, e));
      const double cf = cf_next;
      cf_next = chunk_coef<FB_LC>(am, bm, l0 + FB_LC - m, k - m, lane);
      recur_chunk<FB_LC>(cf, u, sg, z1, z2, e, [&](int j, double v) {
        __bf16 hi, lo;
        split_bf16(v, hi, lo);
        Zt[w][0][j][lane] = hi;
        Zt[w][1][j][lane] = lo;
      });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < FB_LC ? (k - l0) : FB_LC;
        const int nt = (k - tile * 64) < 64 ? (k - tile * 64) : 64;
        retained += (unsigned long long)nl * (unsigned long long)nt;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int lt = 0; lt < 2; ++lt) {
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Zt[w][0][lt * 16 + li][32 * kb + 8 * lq]);
            const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Zt[w][1][lt * 16 + li][32 * kb + 8 * lq]);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[lt][ct] = mma3(ah[kb][ct], al[kb][ct], bh, bl, acc[lt][ct]);
          }
      }
      __syncthreads();
#pragma unroll
      for (int lt = 0; lt < 2; ++lt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = ct * 16 + 4 * lq + v;
            const int lloc = lt * 16 + li;
            if (c < C) red[((size_t)w * FB_LC + lloc) * RS + c] = (double)acc[lt][ct][v];
          }
      __syncthreads();
      for (int idx = threadIdx.x; idx < FB_LC * C; idx += FB_NW * 64) {
        const int lloc = idx / C, c = idx % C;
        const int l = l0 + lloc;
        if (l < k) {
          double sum = 0.0;
#pragma unroll
          for (int ww = 0; ww < FB_NW; ++ww) sum += red[(ww * FB_LC + lloc) * RS + c];
          Rg[(tri_off(k, m) + (l - m)) * C + c] = sum;
        }
      }
      __syncthreads();
    }
  }
  if (counter != nullptr && lane == 0 && retained > 0) atomicAdd(counter, retained);
}

// ------------------------------------------------------------------------------------------
// Synthesis (C >= 16), D[t][c] = sum_l z_l(theta_t) S[l][c]: A = 16 thetas x 32 degrees,
// B = 32 degrees x 16 columns.  4 waves per block, 64 thetas per wave, 32 degrees per chunk; the
// z tile is [theta][hi: 32 degrees | lo: 32 degrees] in wave-private LDS, written 4 degrees at a
// time; coefficient rows are loaded a chunk ahead and split in registers.
// ------------------------------------------------------------------------------------------
constexpr int IB_LC = 32;
constexpr int IB_ZR = 72;        // LDS row (bf16): 32 hi + 32 lo + 8, rows 16-byte aligned
constexpr int IB_FLUSH = 2;      // chunks (64 degrees) accumulated in FP32 between FP64 flushes

template <int C>
__global__ __launch_bounds__(256) void k_legendre_inv_bf16(const double* __restrict__ S, double* __restrict__ FT,
                                                           const double* __restrict__ alpha,
                                                           const double* __restrict__ beta,
                                                           const double* __restrict__ cm,
                                                           const double* __restrict__ ut,
                                                           const double* __restrict__ sx,
                                                           const double* __restrict__ st, int k, int Lt,
                                                           int ntb, unsigned long long* __restrict__ counter) {
  constexpr int CT = C / 16;
  __shared__ __align__(16) __bf16 Z[4][64][IB_ZR];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pair = blk / ntb;
  const int tile = (blk % ntb) * 4 + w;
  const int t = tile * 64 + lane;
  const bool valid = t < k;
  const double u = valid ? ut[t] : -1.0;
  const double sg = valid ? sx[t] : -1.0;
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  unsigned long long retained = 0;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Sm = S + tri_off(k, m) * C;
    v4f acc[4][CT];
    double accd[4][CT][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        acc[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[g][ct][v] = 0.0;
      }
    int since_flush = 0;
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf_next = chunk_coef<IB_LC>(am, bm, 0, k - m, lane);
    // coefficient rows l0 + 8 lq + e, column ct*16 + li, one chunk ahead
    double bn[CT][8];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int l = m + 8 * lq + q;
        bn[ct][q] = l < k ? Sm[(size_t)(l - m) * C + ct * 16 + li] : 0.0;
      }
    for (int l0 = m; l0 < k; l0 += IB_LC) {
      const bool skip = __all(!valid || negligible(z1, z2, e));
      bf16x8 bh[CT], bl[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          __bf16 hi, lo;
          split_bf16(bn[ct][q], hi, lo);
          bh[ct][q] = hi;
          bl[ct][q] = lo;
        }
      if (l0 + IB_LC < k) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int l = l0 + IB_LC + 8 * lq + q;
            bn[ct][q] = l < k ? Sm[(size_t)(l - m) * C + ct * 16 + li] : 0.0;
          }
      }
      const double cf = cf_next;
      cf_next = chunk_coef<IB_LC>(am, bm, l0 + IB_LC - m, k - m, lane);
      // z values: 4 consecutive degrees per 8-byte store (hi and lo parts)
      bf16x4 ph, pl;
      recur_chunk<IB_LC>(cf, u, sg, z1, z2, e, [&](int j, double v) {
        __bf16 hi, lo;
        split_bf16(v, hi, lo);
        ph[j & 3] = hi;
        pl[j & 3] = lo;
        if ((j & 3) == 3) {
          *reinterpret_cast<bf16x4*>(&Z[w][lane][j - 3]) = ph;
          *reinterpret_cast<bf16x4*>(&Z[w][lane][32 + j - 3]) = pl;
        }
      });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < IB_LC ? (k - l0) : IB_LC;
        retained += (unsigned long long)nl * (unsigned long long)(valid ? 1 : 0);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const bf16x8 zh = *reinterpret_cast<const bf16x8*>(&Z[w][16 * g + li][8 * lq]);
          const bf16x8 zl = *reinterpret_cast<const bf16x8*>(&Z[w][16 * g + li][32 + 8 * lq]);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc[g][ct] = mma3(zh, zl, bh[ct], bl[ct], acc[g][ct]);
        }
        if (++since_flush == IB_FLUSH) {
          since_flush = 0;
#pragma unroll
          for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
              for (int v = 0; v < 4; ++v) accd[g][ct][v] += (double)acc[g][ct][v];
              acc[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
            }
        }
      }
      wave_lds_sync();
    }
    // result register v of lane l holds theta row 4 (l / 16) + v, column l % 16
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int tt = tile * 64 + 16 * g + 4 * lq + v;
        if (tt < k) {
          double* out = FT + ((size_t)tt * k + m) * C;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) out[ct * 16 + li] = accd[g][ct][v] + (double)acc[g][ct][v];
        }
      }
  }
  if (counter != nullptr) {
    for (int off = 32; off > 0; off >>= 1) retained += __shfl_down(retained, off);
    if (lane == 0 && retained > 0) atomicAdd(counter, retained);
  }
}

// ------------------------------------------------------------------------------------------
// The same two contractions on the northern half of the symmetric grid (see the FP64 kernels
// k_legendre_fwd_sym / k_legendre_inv_sym): even l+m meets the north/south sums of the theta
// stage, odd l+m the differences.
// Analysis: as k_legendre_fwd_bf16 with two operand sets; z tile rows 0..15 hold the even steps
// of the 32-degree chunk, rows 16..31 the odd steps.
// ------------------------------------------------------------------------------------------
template <int C>
__global__ __launch_bounds__(512) void k_legendre_fwd_bf16_sym(const double* __restrict__ HM,
                                                               double* __restrict__ R, long long part_stride,
                                                               const double* __restrict__ alpha,
                                                               const double* __restrict__ beta,
                                                               const double* __restrict__ cm,
                                                               const double* __restrict__ ut,
                                                               const double* __restrict__ st, int k, int Lt, int ng,
                                                               int lmin,
                                                               unsigned long long* __restrict__ counter) {
  constexpr int CT = C / 16;
  constexpr int RS = 2 * ((C / 2) | 1);
  constexpr int ZBYTES = FB_NW * 2 * FB_LC * FB_ZR * 2;
  constexpr int RBYTES = FB_NW * FB_LC * RS * (int)sizeof(double);
  __shared__ __align__(16) char smem[ZBYTES > RBYTES ? ZBYTES : RBYTES];
  __bf16 (*Zt)[2][FB_LC][FB_ZR] = reinterpret_cast<__bf16 (*)[2][FB_LC][FB_ZR]>(smem);
  double* red = reinterpret_cast<double*>(smem);
  unsigned long long retained = 0;
  const int kh = k / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int pair = blockIdx.x / ng;
  const int grp = blockIdx.x % ng;
  const int tile = grp * FB_NW + w;
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
    // element e of a*[kb][ct]: node tile*64 + 32 kb + 8 lq + e, column ct*16 + li (column-pair major)
    bf16x8 aph[2][CT], apl[2][CT], anh[2][CT], anl[2][CT];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int tg = tile * 64 + 32 * kb + 8 * lq + e;
          const int c = ct * 16 + li;
          const double* col = Hm + (size_t)(c >> 1) * k * 2 + (c & 1);
          const double hp = tg < kh ? col[(size_t)tg * 2] : 0.0;
          const double hn = tg < kh ? col[(size_t)(kh + tg) * 2] : 0.0;
          __bf16 hi, lo;
          split_bf16(hp, hi, lo);
          aph[kb][ct][e] = hi;
          apl[kb][ct][e] = lo;
          split_bf16(hn, hi, lo);
          anh[kb][ct][e] = hi;
          anl[kb][ct][e] = lo;
        }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cf_next = chunk_coef<FB_LC>(am, bm, 0, k - m, lane);

    for (int l0 = m; l0 < k; l0 += FB_LC) {
      v4f acc[2][CT];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[x][ct] = v4f{0.f, 0.f, 0.f, 0.f};
      // below the degree floor: no products, and no rows of R (the caller reads none of them)
      const bool below = l0 + FB_LC <= lmin;
      const bool skip = !tile_live || below || __all(!valid || negligible(z1, z2, e));
      const double cf = cf_next;
      cf_next = chunk_coef<FB_LC>(am, bm, l0 + FB_LC - m, k - m, lane);
      recur_chunk<FB_LC>(cf, u, sg, z1, z2, e, [&](int j, double v) {
        __bf16 hi, lo;
        split_bf16(v, hi, lo);
        const int row = (j & 1) * (FB_LC / 2) + (j >> 1);
        Zt[w][0][row][lane] = hi;
        Zt[w][1][row][lane] = lo;
      });
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < FB_LC ? (k - l0) : FB_LC;
        const int nt = (kh - tile * 64) < 64 ? (kh - tile * 64) : 64;
        retained += (unsigned long long)nl * (unsigned long long)nt;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          const bf16x8 b0h = *reinterpret_cast<const bf16x8*>(&Zt[w][0][li][32 * kb + 8 * lq]);
          const bf16x8 b0l = *reinterpret_cast<const bf16x8*>(&Zt[w][1][li][32 * kb + 8 * lq]);
          const bf16x8 b1h = *reinterpret_cast<const bf16x8*>(&Zt[w][0][16 + li][32 * kb + 8 * lq]);
          const bf16x8 b1l = *reinterpret_cast<const bf16x8*>(&Zt[w][1][16 + li][32 * kb + 8 * lq]);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            acc[0][ct] = mma3(aph[kb][ct], apl[kb][ct], b0h, b0l, acc[0][ct]);
            acc[1][ct] = mma3(anh[kb][ct], anl[kb][ct], b1h, b1l, acc[1][ct]);
          }
        }
      }
      if (below) continue;   // block-uniform
      __syncthreads();
#pragma unroll
      for (int lt = 0; lt < 2; ++lt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = ct * 16 + 4 * lq + v;
            red[((size_t)w * FB_LC + lt * 16 + li) * RS + c] = (double)acc[lt][ct][v];
          }
      __syncthreads();
      // one column pair per thread and step: 16-byte LDS reads and global stores
      for (int idx = threadIdx.x; idx < FB_LC * C / 2; idx += FB_NW * 64) {
        const int lloc = idx / (C / 2), c = 2 * (idx % (C / 2));
        const int l = l0 + 2 * (lloc & 15) + (lloc >> 4);
        if (l < k) {
          double2 sum = make_double2(0.0, 0.0);
#pragma unroll
          for (int ww = 0; ww < FB_NW; ++ww) {
            const double2 v = *reinterpret_cast<const double2*>(&red[(ww * FB_LC + lloc) * RS + c]);
            sum.x += v.x;
            sum.y += v.y;
          }
          *reinterpret_cast<double2*>(&Rg[(tri_off(k, m) + (l - m)) * C + c]) = sum;
        }
      }
      __syncthreads();
    }
  }
  if (counter != nullptr && lane == 0 && retained > 0) atomicAdd(counter, retained);
}

// Synthesis: 64-degree chunks, so that one v_mfma_f32_16x16x32_bf16 contracts the 32 even or the
// 32 odd degrees; z tile row per node [even hi 32 | odd hi 32 | even lo 32 | odd lo 32 | 8 pad];
// FP32 partial sums (32 terms per chunk and parity) carried into the FP64 north and south sums
// every IBS_FLUSH chunks.
constexpr int IBS_LC = 64;
constexpr int IBS_ZR = 136;
constexpr int IBS_FLUSH = 2;

template <int C>
__global__ __launch_bounds__(256, 1) void k_legendre_inv_bf16_sym(const double* __restrict__ S,
                                                                  double* __restrict__ FS,
                                                                  const double* __restrict__ alpha,
                                                                  const double* __restrict__ beta,
                                                                  const double* __restrict__ cm,
                                                                  const double* __restrict__ ut,
                                                                  const double* __restrict__ st, int k, int Lt,
                                                                  int ntb, int lmin,
                                                                  unsigned long long* __restrict__ counter) {
  constexpr int CT = C / 16;
  __shared__ __align__(16) __bf16 Z[4][64][IBS_ZR];
  const int kh = k / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int pair = spread_pairs(blk / ntb, (k + 1) / 2);
  const int tile = (blk % ntb) * 4 + w;
  const int t = tile * 64 + lane;
  const bool valid = t < kh;
  const double u = valid ? ut[t] : -1.0;
  const double sg = 1.0;
  const double s = valid ? st[t] : 1.0;
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  unsigned long long retained = 0;

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const double* __restrict__ Sm = S + tri_off(k, m) * C;
    v4f accE[4][CT], accO[4][CT];
    double accN[4][CT][4], accS[4][CT][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        accE[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
        accO[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) accN[g][ct][v] = accS[g][ct][v] = 0.0;
      }
    int since_flush = 0;
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cfa_next = chunk_coef<32>(am, bm, 0, k - m, lane);
    double cfb_next = chunk_coef<32>(am, bm, 32, k - m, lane);
    // coefficient rows of the chunk: even degree l0 + 2 (8 lq + q), odd l0 + 2 (8 lq + q) + 1
    double bn[2][CT][8];
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int l = m + 2 * (8 * lq + q) + par;
          bn[par][ct][q] = l < k ? Sm[(size_t)(l - m) * C + ct * 16 + li] : 0.0;
        }
    for (int l0 = m; l0 < k; l0 += IBS_LC) {
      const bool skip = l0 + IBS_LC <= lmin || __all(!valid || negligible(z1, z2, e));
      bf16x8 bh[2][CT], bl[2][CT];
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            __bf16 hi, lo;
            split_bf16(bn[par][ct][q], hi, lo);
            bh[par][ct][q] = hi;
            bl[par][ct][q] = lo;
          }
      if (l0 + IBS_LC < k) {
#pragma unroll
        for (int par = 0; par < 2; ++par)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int l = l0 + IBS_LC + 2 * (8 * lq + q) + par;
              bn[par][ct][q] = l < k ? Sm[(size_t)(l - m) * C + ct * 16 + li] : 0.0;
            }
      }
      const double cfa = cfa_next, cfb = cfb_next;
      cfa_next = chunk_coef<32>(am, bm, l0 + IBS_LC - m, k - m, lane);
      cfb_next = chunk_coef<32>(am, bm, l0 + IBS_LC + 32 - m, k - m, lane);
      // z values: 4 consecutive even (odd) steps per 8-byte store of hi and lo parts
      bf16x4 peh, pel, poh, pol;
      auto sink = [&](int base) {
        return [&, base](int j, double v) {
          const int jj = base + j;
          __bf16 hi, lo;
          split_bf16(v, hi, lo);
          const int i = jj >> 1;   // position within the parity half
          if (jj & 1) {
            poh[i & 3] = hi;
            pol[i & 3] = lo;
          } else {
            peh[i & 3] = hi;
            pel[i & 3] = lo;
          }
          if ((jj & 7) == 7) {
            *reinterpret_cast<bf16x4*>(&Z[w][lane][i - 3]) = peh;
            *reinterpret_cast<bf16x4*>(&Z[w][lane][32 + i - 3]) = poh;
            *reinterpret_cast<bf16x4*>(&Z[w][lane][64 + i - 3]) = pel;
            *reinterpret_cast<bf16x4*>(&Z[w][lane][96 + i - 3]) = pol;
          }
        };
      };
      recur_chunk<32>(cfa, u, sg, z1, z2, e, sink(0));
      recur_chunk<32>(cfb, u, sg, z1, z2, e, sink(32));
      if (!skip) {
        wave_lds_sync();
        const int nl = (k - l0) < IBS_LC ? (k - l0) : IBS_LC;
        retained += (unsigned long long)nl * (unsigned long long)(valid ? 1 : 0);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const __bf16* row = &Z[w][16 * g + li][0];
          const bf16x8 zeh = *reinterpret_cast<const bf16x8*>(row + 8 * lq);
          const bf16x8 zoh = *reinterpret_cast<const bf16x8*>(row + 32 + 8 * lq);
          const bf16x8 zel = *reinterpret_cast<const bf16x8*>(row + 64 + 8 * lq);
          const bf16x8 zol = *reinterpret_cast<const bf16x8*>(row + 96 + 8 * lq);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            accE[g][ct] = mma3(zeh, zel, bh[0][ct], bl[0][ct], accE[g][ct]);
            accO[g][ct] = mma3(zoh, zol, bh[1][ct], bl[1][ct], accO[g][ct]);
          }
        }
        if (++since_flush == IBS_FLUSH) {
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
              accE[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
              accO[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
            }
        }
      }
      wave_lds_sync();
    }
    // result register v of lane l holds node row 4 (l / 16) + v, column l % 16
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int tt = tile * 64 + 16 * g + 4 * lq + v;
        if (tt < kh) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const int c = ct * 16 + li;
            double* col = FS + ((size_t)m * C + (c & ~1)) * k + (c & 1);
            const double E = (double)accE[g][ct][v], O = (double)accO[g][ct][v];
            col[(size_t)tt * 2] = accN[g][ct][v] + (E + O);
            col[(size_t)(k - 1 - tt) * 2] = accS[g][ct][v] + (E - O);
          }
        }
      }
  }
  if (counter != nullptr) {
    for (int off = 32; off > 0; off >>= 1) retained += __shfl_down(retained, off);
    if (lane == 0 && retained > 0) atomicAdd(counter, retained);
  }
}

hipError_t launch_legendre_forward_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b,
                                            const double* HM, double* R, long long part_stride, int lmin,
                                            unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  if (!T.sym || (k & 1)) return hipErrorInvalidValue;
  const int ng = legendre_forward_groups_sym(k);
  const dim3 grid(((k + 1) / 2) * ng), block(FB_NW * 64);
  if (b.C == 32)
    k_legendre_fwd_bf16_sym<32><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s, T.st_s,
                                                       k, G.Lt, ng, lmin, counter);
  else if (b.C == 16)
    k_legendre_fwd_bf16_sym<16><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s, T.st_s,
                                                       k, G.Lt, ng, lmin, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_legendre_inverse_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b,
                                            const double* S, double* FS, int lmin, unsigned long long* counter,
                                            hipStream_t s) {
  const int k = T.k;
  if (!T.sym || (k & 1)) return hipErrorInvalidValue;
  const int ntb = (k / 2 + 255) / 256;
  const dim3 grid(((k + 1) / 2) * ntb), block(256);
  if (b.C == 32)
    k_legendre_inv_bf16_sym<32><<<grid, block, 0, s>>>(S, FS, G.alpha, G.beta, G.cm, T.ut_s, T.st_s, k, G.Lt, ntb,
                                                       lmin, counter);
  else if (b.C == 16)
    k_legendre_inv_bf16_sym<16><<<grid, block, 0, s>>>(S, FS, G.alpha, G.beta, G.cm, T.ut_s, T.st_s, k, G.Lt, ntb,
                                                       lmin, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
template <int C>
static hipError_t fwd_bf16_c(const ShtTables& T, const LegTables& G, const double* HM, double* R,
                             long long part_stride, unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  const int npairs = (k + 1) / 2;
  const int ng = legendre_forward_groups(k);   // the partial-sum layout the consumers expect
  k_legendre_fwd_bf16<C><<<npairs * ng, FB_NW * 64, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut,
                                                             T.sx, T.st, k, G.Lt, ng, counter);
  return hipGetLastError();
}

template <int C>
static hipError_t inv_bf16_c(const ShtTables& T, const LegTables& G, const double* S, double* FT,
                             unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  const int ntb = (k + 255) / 256;
  const int npairs = (k + 1) / 2;
  k_legendre_inv_bf16<C><<<npairs * ntb, 256, 0, s>>>(S, FT, G.alpha, G.beta, G.cm, T.ut, T.sx, T.st, k, G.Lt,
                                                       ntb, counter);
  return hipGetLastError();
}

// Same partial-sum layout as the FP64 analysis kernel (512 thetas per block group).
hipError_t launch_legendre_forward_bf16(const ShtTables& T, const LegTables& G, const Batch& b,
                                        const double* HM, double* R, long long part_stride,
                                        unsigned long long* counter, hipStream_t s) {
  switch (b.C) {
    case 2: return fwd_bf16_c<2>(T, G, HM, R, part_stride, counter, s);
    case 4: return fwd_bf16_c<4>(T, G, HM, R, part_stride, counter, s);
    case 8: return fwd_bf16_c<8>(T, G, HM, R, part_stride, counter, s);
    case 16: return fwd_bf16_c<16>(T, G, HM, R, part_stride, counter, s);
    case 32: return fwd_bf16_c<32>(T, G, HM, R, part_stride, counter, s);
  }
  return hipErrorInvalidValue;
}

// C >= 16 only; smaller batches use the FP64 vector kernel.
hipError_t launch_legendre_inverse_bf16(const ShtTables& T, const LegTables& G, const Batch& b,
                                        const double* S, double* FT, unsigned long long* counter,
                                        hipStream_t s) {
  switch (b.C) {
    case 16: return inv_bf16_c<16>(T, G, S, FT, counter, s);
    case 32: return inv_bf16_c<32>(T, G, S, FT, counter, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace s2let
