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

// x -> FP32 (round to nearest) -> bf16 hi and lo parts.  The empty asm statement keeps the FP32
// value opaque, so the compiler rounds hi from it with one v_cvt_pk_bf16_f32 rather than fusing the
// two conversions into a correctly rounded double -> bf16 sequence (nine more instructions).
__device__ __forceinline__ float opaque_f32(float f) {
  __asm__("" : "+v"(f));
  return f;
}

__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const float f = opaque_f32((float)x);
  hi = (__bf16)f;
  lo = (__bf16)(f - (float)hi);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two values at once: hi = bf16(a, b) with one packed conversion, widened back by a shift and a
// mask, lo = bf16 of the two exact FP32 residuals with a second packed conversion.
__device__ __forceinline__ void split_bf16_pair(float a, float b, bf16x2& hi, bf16x2& lo) {
  hi = __builtin_convertvector(f32x2{a, b}, bf16x2);
  const unsigned hb = __builtin_bit_cast(unsigned, hi);
  const float ha = __uint_as_float(hb << 16), hbf = __uint_as_float(hb & 0xffff0000u);
  lo = __builtin_convertvector(f32x2{a - ha, b - hbf}, bf16x2);
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
      // (a skipped chunk's z values are read by no product: neither split nor stored)
      if (skip)
        recur_chunk<FB_LC>(cf, u, sg, z1, z2, e, [](int, double) {});
      else
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
      if (skip)
        recur_chunk<IB_LC>(cf, u, sg, z1, z2, e, [](int, double) {});
      else
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
// Analysis: the block-wide, double-buffered z tile of k_legendre_fwd_sym_f32, in bf16 hi and lo
// parts.  Each wave runs the recursion for 64 nodes (steps 2i and 2i+1 split together) into
// Z[buf][hi/lo][row][node]; wave w owns the output tile (column block ct, parity p) over one node
// slice, its operands split once per m; one barrier per chunk, FP32 partial tiles added in FP64.
// ------------------------------------------------------------------------------------------
constexpr int FBS_ZR = 520;   // Z row (bf16): 512 nodes + 8; the 16 rows a quarter-wave reads sit
                              // 4 banks apart

// HT: the element type of HM (double, or float when the theta stage runs in FP32)
template <int C, typename HT>
__global__ __launch_bounds__(512) void k_legendre_fwd_bf16_sym(const HT* __restrict__ HM,
                                                               double* __restrict__ R, long long part_stride,
                                                               const double* __restrict__ alpha,
                                                               const double* __restrict__ beta,
                                                               const double* __restrict__ cm,
                                                               const double* __restrict__ ut,
                                                               const double* __restrict__ st, int k, int Lt, int ng,
                                                               int lmin,
                                                               unsigned long long* __restrict__ counter) {
  constexpr int NW = 8, LC = 32, TB = NW * 64, PS = 18;
  constexpr int CT = C / 16;
  constexpr int NKS = NW / (2 * CT);   // node slices per output tile
  constexpr int KS = TB / NKS;         // nodes per slice
  constexpr int NB = KS / 32;          // 32-node k-blocks per slice
  constexpr int SRC = KS / 64;         // recursion waves per slice (2 k-blocks each)
  __shared__ __align__(16) __bf16 Z[2][2][LC][FBS_ZR];
  __shared__ __align__(16) float P[2][NW][16][PS];
  __shared__ double2 coef[NW][LC];
  __shared__ int negl[2][NW];
  unsigned long long retained = 0;
  const int kh = k / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int pair = blockIdx.x / ng;
  const int grp = blockIdx.x % ng;
  const int tile = grp * NW + w;
  const int t = tile * 64 + lane;
  const bool valid = t < kh;
  const bool tile_live = tile * 64 < kh;
  const int nt = tile_live ? ((kh - tile * 64) < 64 ? (kh - tile * 64) : 64) : 0;
  const double u = valid ? ut[t] : -1.0;
  const double sg = 1.0;
  const double s = valid ? st[t] : 1.0;
  const int ct = w % CT, p = (w / CT) & 1, h = w / (2 * CT);
  const int nm = (k - 1 - pair > pair) ? 2 : 1;
  double* __restrict__ Rg = R + (size_t)grp * part_stride;
  double2* cfl = coef[w];

  auto reduce = [&](int pb, int m, int l0) {
    for (int idx = threadIdx.x; idx < LC * C / 2; idx += NW * 64) {
      const int cp = idx % (C / 2), rest = idx / (C / 2);
      const int r = rest & 15, pr = rest >> 4;
      const int c = 2 * cp, ctt = c >> 4, cl = c & 15;
      const int l = l0 + 2 * r + pr;
      if (l < k) {
        double2 sum = make_double2(0.0, 0.0);
#pragma unroll
        for (int hh = 0; hh < NKS; ++hh) {
          const float2 v = *reinterpret_cast<const float2*>(&P[pb][(hh * 2 + pr) * CT + ctt][r][cl]);
          sum.x += (double)v.x;
          sum.y += (double)v.y;
        }
        *reinterpret_cast<double2*>(&Rg[(tri_off(k, m) + (l - m)) * C + c]) = sum;
      }
    }
  };

  for (int im = 0; im < nm; ++im) {
    const int m = im == 0 ? pair : k - 1 - pair;
    const double* __restrict__ am = alpha + tri_off(Lt, m);
    const double* __restrict__ bm = beta + tri_off(Lt, m);
    const HT* __restrict__ Hm = HM + (size_t)m * k * C;
    // operands: element e of ah/al[kb] = node base + 32 kb + 8 lq + e, column ct*16 + li, the sums
    // (p = 0) or differences (p = 1) the theta stage stores at nodes [0, k/2) / [k/2, k)
    bf16x8 ah[NB], al[NB];
    {
      const int base = grp * TB + h * KS;
      const int c = ct * 16 + li;
      const HT* col = Hm + (size_t)(c >> 1) * k * 2 + (c & 1) + (p ? (size_t)kh * 2 : 0);
#pragma unroll
      for (int kb = 0; kb < NB; ++kb) {
        // k/2 is a multiple of 32: a k-block is in range or not as a whole
        const bool in = base + 32 * kb < kh;
#pragma unroll
        for (int e2 = 0; e2 < 8; e2 += 2) {
          const size_t tg = (size_t)(base + 32 * kb + 8 * lq + e2);
          const float f0 = opaque_f32((float)(in ? col[tg * 2] : HT(0)));
          const float f1 = opaque_f32((float)(in ? col[(tg + 1) * 2] : HT(0)));
          bf16x2 hi, lo;
          split_bf16_pair(f0, f1, hi, lo);
          ah[kb][e2] = hi.x;
          ah[kb][e2 + 1] = hi.y;
          al[kb][e2] = lo.x;
          al[kb][e2 + 1] = lo.y;
        }
      }
    }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    // chunk c of this m starts at degree m + 32 c; its z values go to Z[c & 1]
    auto recur_into = [&](int c, int l0c) {
      const bool fill = l0c + LC > lmin;
      const bool ngw = !tile_live || __all(!valid || negligible(z1, z2, e));
      const int zb = c & 1;
      if (fill && !ngw) {
        float fe = 0.f;
        recur_chunk_lds<LC>(cfl, u, sg, z1, z2, e, [&](int j, double v) {
          const float f = opaque_f32((float)v);
          if ((j & 1) == 0) {
            fe = f;
            return;
          }
          bf16x2 hi, lo;
          split_bf16_pair(fe, f, hi, lo);
          const int i = j >> 1;
          Z[zb][0][i][w * 64 + lane] = hi.x;
          Z[zb][0][16 + i][w * 64 + lane] = hi.y;
          Z[zb][1][i][w * 64 + lane] = lo.x;
          Z[zb][1][16 + i][w * 64 + lane] = lo.y;
        });
        retained += (unsigned long long)((k - l0c) < LC ? (k - l0c) : LC) * nt;
      } else {
        // below the floor, or products that skip this wave's nodes: no z values stored
        recur_chunk_lds<LC>(cfl, u, sg, z1, z2, e, [](int, double) {});
      }
      if (fill && lane == 0) negl[zb][w] = ngw;
    };
    double cf = chunk_coef<LC>(am, bm, 0, k - m, lane);
    stage_coef<LC>(cfl, cf, lane);
    cf = chunk_coef<LC>(am, bm, LC, k - m, lane);
    wave_lds_sync();
    recur_into(0, m);
    wave_lds_sync();
    stage_coef<LC>(cfl, cf, lane);   // chunk 1
    cf = chunk_coef<LC>(am, bm, 2 * LC, k - m, lane);
    if (m + LC > lmin) __syncthreads();

    int ci = 0;
    for (int l0 = m; l0 < k; l0 += LC, ++ci) {
      const bool below = l0 + LC <= lmin;   // block-uniform
      const int l1 = l0 + LC;
      const bool has_next = l1 < k;
      const bool fill_next = has_next && l1 + LC > lmin;
      if (has_next) {
        wave_lds_sync();
        recur_into(ci + 1, l1);
      }
      if (!below) {
        v4f acc0 = v4f{0.f, 0.f, 0.f, 0.f}, acc1 = v4f{0.f, 0.f, 0.f, 0.f};
        const int zb = ci & 1;
#pragma unroll
        for (int sw = 0; sw < SRC; ++sw) {
          if (negl[zb][h * SRC + sw]) continue;   // wave-uniform
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int kb = 2 * sw + q;
            const int col = h * KS + 32 * kb + 8 * lq;
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Z[zb][0][p * 16 + li][col]);
            const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Z[zb][1][p * 16 + li][col]);
            if (q == 0)
              acc0 = mma3(ah[kb], al[kb], bh, bl, acc0);
            else
              acc1 = mma3(ah[kb], al[kb], bh, bl, acc1);
          }
        }
        if (l0 - LC >= m && l0 > lmin) reduce((ci - 1) & 1, m, l0 - LC);
        // register v holds column 4 lq + v of the tile, degree row li
#pragma unroll
        for (int v = 0; v < 4; ++v) P[zb][w][li][4 * lq + v] = acc0[v] + acc1[v];
      }
      if (has_next) {
        wave_lds_sync();
        stage_coef<LC>(cfl, cf, lane);   // chunk ci + 2
        cf = chunk_coef<LC>(am, bm, l1 + 2 * LC - m, k - m, lane);
      }
      if (!below || fill_next) __syncthreads();
    }
    {
      const int nch = (k - m + LC - 1) / LC;
      const int llast = m + (nch - 1) * LC;
      if (llast + LC > lmin) reduce((nch - 1) & 1, m, llast);
    }
    __syncthreads();   // the next m overwrites Z, P and the flags
  }
  if (counter != nullptr && lane == 0 && retained > 0) atomicAdd(counter, retained);
}

// Synthesis: 64-degree chunks, so that one v_mfma_f32_16x16x32_bf16 contracts the 32 even or the
// 32 odd degrees; z tile row per node [even hi 32 | odd hi 32 | even lo 32 | odd lo 32 | 8 pad].
// The even and odd sums accumulate in FP32 over the whole column m: the split products carry a
// relative error near 2^-16 each, which FP32 accumulation (2^-24 per addition) does not change,
// and without FP64 running sums the kernel fits two blocks per CU.
constexpr int IBS_LC = 64;
constexpr int IBS_ZR = 136;

// FT_: the element type of FS (double, or float when the resampling runs in FP32)
template <int C, typename FT_>
__global__ __launch_bounds__(256, 2) void k_legendre_inv_bf16_sym(const double* __restrict__ S,
                                                                  FT_* __restrict__ FS,
                                                                  const double* __restrict__ alpha,
                                                                  const double* __restrict__ beta,
                                                                  const double* __restrict__ cm,
                                                                  const double* __restrict__ ut,
                                                                  const double* __restrict__ st, int k, int Lt,
                                                                  int ntb, int lmin,
                                                                  unsigned long long* __restrict__ counter) {
  constexpr int CT = C / 16;
  __shared__ __align__(16) __bf16 Z[4][64][IBS_ZR];
  __shared__ double2 coef[4][IBS_LC];   // each wave's copy of the chunk's recursion coefficients
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
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        accE[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
        accO[g][ct] = v4f{0.f, 0.f, 0.f, 0.f};
      }
    int e;
    double z1, z2;
    recur_start(cm[m], s, sg, m, z1, z2, e);
    double cfa = chunk_coef<32>(am, bm, 0, k - m, lane);
    double cfb = chunk_coef<32>(am, bm, 32, k - m, lane);
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
      stage_coef<32>(coef[w], cfa, lane);
      stage_coef<32>(coef[w] + 32, cfb, lane);
      cfa = chunk_coef<32>(am, bm, l0 + IBS_LC - m, k - m, lane);   // the next chunk's, in flight
      cfb = chunk_coef<32>(am, bm, l0 + IBS_LC + 32 - m, k - m, lane);
      wave_lds_sync();
      // z values: steps 2i and 2i+1 split together; 4 consecutive even (odd) steps per 8-byte store
      // of hi and lo parts
      bf16x4 peh, pel, poh, pol;
      float fe = 0.f;
      auto sink = [&](int base) {
        return [&, base](int j, double v) {
          const int jj = base + j;
          const float f = opaque_f32((float)v);
          if ((jj & 1) == 0) {
            fe = f;
            return;
          }
          bf16x2 hi, lo;
          split_bf16_pair(fe, f, hi, lo);
          const int i = jj >> 1;   // position within the parity half
          peh[i & 3] = hi.x;
          poh[i & 3] = hi.y;
          pel[i & 3] = lo.x;
          pol[i & 3] = lo.y;
          if ((jj & 7) == 7) {
            *reinterpret_cast<bf16x4*>(&Z[w][lane][i - 3]) = peh;
            *reinterpret_cast<bf16x4*>(&Z[w][lane][32 + i - 3]) = poh;
            *reinterpret_cast<bf16x4*>(&Z[w][lane][64 + i - 3]) = pel;
            *reinterpret_cast<bf16x4*>(&Z[w][lane][96 + i - 3]) = pol;
          }
        };
      };
      if (skip) {
        // a skipped chunk's z values are read by no product: neither split nor stored
        auto nosink = [](int, double) {};
        recur_chunk_lds<32>(coef[w], u, sg, z1, z2, e, nosink);
        recur_chunk_lds<32>(coef[w] + 32, u, sg, z1, z2, e, nosink);
      } else {
        recur_chunk_lds<32>(coef[w], u, sg, z1, z2, e, sink(0));
        recur_chunk_lds<32>(coef[w] + 32, u, sg, z1, z2, e, sink(32));
      }
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
            FT_* col = FS + ((size_t)m * C + (c & ~1)) * k + (c & 1);
            const double E = (double)accE[g][ct][v], O = (double)accO[g][ct][v];
            col[(size_t)tt * 2] = (FT_)(E + O);
            col[(size_t)(k - 1 - tt) * 2] = (FT_)(E - O);
          }
        }
      }
  }
  if (counter != nullptr) {
    for (int off = 32; off > 0; off >>= 1) retained += __shfl_down(retained, off);
    if (lane == 0 && retained > 0) atomicAdd(counter, retained);
  }
}

template <typename HT>
static hipError_t fwd_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b, const HT* HM, double* R,
                               long long part_stride, int lmin, unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  if (!T.sym || (k & 1)) return hipErrorInvalidValue;
  const int ng = legendre_forward_groups_sym(k);
  const dim3 grid(((k + 1) / 2) * ng), block(FB_NW * 64);
  if (b.C == 32)
    k_legendre_fwd_bf16_sym<32, HT><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s,
                                                           T.st_s, k, G.Lt, ng, lmin, counter);
  else if (b.C == 16)
    k_legendre_fwd_bf16_sym<16, HT><<<grid, block, 0, s>>>(HM, R, part_stride, G.alpha, G.beta, G.cm, T.ut_s,
                                                           T.st_s, k, G.Lt, ng, lmin, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_legendre_forward_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b,
                                            const double* HM, double* R, long long part_stride, int lmin,
                                            unsigned long long* counter, hipStream_t s) {
  return fwd_bf16_sym(T, G, b, HM, R, part_stride, lmin, counter, s);
}

hipError_t launch_legendre_forward_bf16_sym_f32(const ShtTables& T, const LegTables& G, const Batch& b,
                                                const float* HM, double* R, long long part_stride, int lmin,
                                                unsigned long long* counter, hipStream_t s) {
  return fwd_bf16_sym(T, G, b, HM, R, part_stride, lmin, counter, s);
}

template <typename FT_>
static hipError_t inv_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b, const double* S, FT_* FS,
                               int lmin, unsigned long long* counter, hipStream_t s) {
  const int k = T.k;
  if (!T.sym || (k & 1)) return hipErrorInvalidValue;
  const int ntb = (k / 2 + 255) / 256;
  const dim3 grid(((k + 1) / 2) * ntb), block(256);
  if (b.C == 32)
    k_legendre_inv_bf16_sym<32, FT_><<<grid, block, 0, s>>>(S, FS, G.alpha, G.beta, G.cm, T.ut_s, T.st_s, k, G.Lt,
                                                            ntb, lmin, counter);
  else if (b.C == 16)
    k_legendre_inv_bf16_sym<16, FT_><<<grid, block, 0, s>>>(S, FS, G.alpha, G.beta, G.cm, T.ut_s, T.st_s, k, G.Lt,
                                                            ntb, lmin, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_legendre_inverse_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b,
                                            const double* S, double* FS, int lmin, unsigned long long* counter,
                                            hipStream_t s) {
  return inv_bf16_sym(T, G, b, S, FS, lmin, counter, s);
}

hipError_t launch_legendre_inverse_bf16_sym_f32(const ShtTables& T, const LegTables& G, const Batch& b,
                                                const double* S, float* FS, int lmin, unsigned long long* counter,
                                                hipStream_t s) {
  return inv_bf16_sym(T, G, b, S, FS, lmin, counter, s);
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
