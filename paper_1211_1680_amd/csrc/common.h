// Internal declarations shared by the host driver and the HIP kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace s2let {

// Packed (m, l) row index of a triangle of band-limit k: column m holds l = m..k-1 and starts
// at m*k - m*(m-1)/2.  rows(k) = k(k+1)/2.
__host__ __device__ inline int64_t tri_off(int k, int m) {
  return (int64_t)m * k - (int64_t)m * (m - 1) / 2;
}
__host__ __device__ inline int64_t tri_rows(int k) { return (int64_t)k * (k + 1) / 2; }

// Workgroups are handed to the 8 XCDs round-robin; this maps the hardware index to a logical
// one so that consecutive logical indices run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_swizzle(int b, int nblk) {
  constexpr int X = 8;
  const int per = nblk / X, rem = nblk % X;
  const int x = b % X, idx = b / X;
  return x * per + (x < rem ? x : rem) + idx;
}

// A logical m-pair slot q (XCD-contiguous after xcd_swizzle) -> pair index: slot i of XCD x takes
// pair 8 i + x, so that pairs of unequal cost (a degree floor makes the low pairs cheaper) are
// shared evenly by the XCDs.  Identity unless npairs is a multiple of 8.
__device__ __forceinline__ int spread_pairs(int q, int npairs) {
  if (npairs & 7) return q;
  const int per = npairs >> 3;
  return (q % per) * 8 + q / per;
}

inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
inline int ilog2(int v) {
  int e = 0;
  while ((1 << e) < v) ++e;
  return e;
}

// Per-band-limit tables (device memory), built once per device by the plan cache.
struct ShtTables {
  int k = 0;        // band-limit
  int n = 0;        // 2k-1 samples per ring / extended theta period
  int nrad = 0;     // > 0: n = rad[0] * ... * rad[nrad-1] (odd radices <= 13), mixed-radix DFT
  int rad[8] = {0};
  double2* twn_lo = nullptr;   // exp(-2 pi i p / n), p < 64
  double2* twn_hi = nullptr;   // exp(-2 pi i 64 p / n), p < ceil(n / 64)
  int M = 0;        // Bluestein power-of-two length >= 2n-1 (when nrad == 0)
  int logM = 0;
  double2* chirp = nullptr;    // c_q = exp(-i pi q^2 / n), q < n
  double2* bhat = nullptr;     // FFT_M of conj(c_q) for |q| <= n-1 (wrapped), divided by M
  int Nc = 0;       // power-of-two correlation length >= 2k-1
  int logNc = 0;
  double2* khat0 = nullptr;    // FFT_Nc of Kt_0(c) = w_e(-2c), wrapped, / (Nc n^2)
  double2* khat1 = nullptr;    // FFT_Nc of Kt_1(c) = w_e(2 - 2c), wrapped, / (Nc n^2)
  double* khr = nullptr;       // real part of khat0 (Kt_0 is real and even, so khat0 is real; Kt_1 is
                               // Kt_0 shifted by one, so class 1 may use it with the output read one slot lower)
  int logP = 0;     // P = 2^logP = max(M, Nc): one twiddle table for every power-of-two length
  int loglo = 0;    // two-level twiddle split: W_P^p = lo[p & (2^loglo - 1)] * hi[p >> loglo]
  double2* tw_lo = nullptr;    // exp(-2 pi i p / P), p < 2^loglo
  double2* tw_hi = nullptr;    // exp(-2 pi i p 2^loglo / P), p < P / 2^loglo
  double* xt = nullptr;        // cos(theta_t), t < k
  double* st = nullptr;        // sin(theta_t), t < k
  double* ut = nullptr;        // |cos(theta_t)| - 1 = -2 sin^2(theta'/2), theta' = min(theta, pi - theta)
  double* sx = nullptr;        // sign of cos(theta_t) (+1 at the equator)
  double* pole = nullptr;      // column t = k-1 of the odd-parity theta operator (see plan.cpp)
  double2* hphase = nullptr;   // exp(-i pi j / n) for j in [-(k-1), k-1], index j+k-1
  // Symmetric auxiliary grid psi_s = pi (2s+1) / (2k), s < 2k on the circle (built for the band-limits
  // that have the compiled transforms): the theta stage evaluates its output there, and the
  // Legendre steps run on the northern half s < k/2, where lambda_lm(pi - psi) = (-1)^(l+m) lambda_lm(psi).
  int sym = 0;
  double* ut_s = nullptr;      // |cos psi_s| - 1 = -2 sin^2(psi_s / 2), s < k/2
  double* st_s = nullptr;      // sin psi_s, s < k/2
  double* sx_s = nullptr;      // +1 (northern nodes)
  double2* psph = nullptr;     // (n / 2k) exp(-i pi j / 2k), j in [-(k-1), k-1]: theta-stage output phase
  double* pole_s = nullptr;    // psi-grid column of the odd-parity theta operator for the pole input, s < k
  double2* rsph = nullptr;     // exp(-i pi j / 2k) exp(i pi j / n) / (4k), j in [-(k-1), k-1]: resampling
};

// Tables indexed by (l, m) up to a maximum band-limit Lt (shared by every k <= Lt).
struct LegTables {
  int Lt = 0;
  double* alpha = nullptr;  // tri_off(Lt,m) + (l-m): alpha_lm of z_l = alpha_l x z_{l-1} - z_{l-2}
  double* beta = nullptr;   // alpha_lm - 2, rounded from the exact value
  double* dfac = nullptr;   // d_lm with lambda_lm = d_lm z_lm
  double* cm = nullptr;     // lambda_mm(theta) = cm[m] sin^m(theta)
};

// Kernel stages, for the optional per-stage timing.
enum Stage {
  ST_PHI_FWD = 0, ST_THETA = 1, ST_LEG_FWD = 2, ST_LEG_INV = 3, ST_PHI_INV = 4, ST_TILE = 5, ST_RESAMPLE = 6, ST_N = 7
};

// Column layout of a batch: C columns of doubles per (row) entry.  Real maps: 2 columns per
// map (re, im of m >= 0).  Complex maps: 4 per map (re, im of +m, then re, im of -m).
struct Batch {
  int nb = 0;        // maps in this batch
  int reality = 0;   // S2LET_REAL / S2LET_COMPLEX
  int C = 0;         // columns (template size, >= used columns)
  int used = 0;      // 2*nb or 4*nb
};

// ---- kernel launchers (kernels_*.hip) ----
// phi stage, forward: maps -> GT[t][m][c]  (m < k, C columns), weight 2 pi / n included.
hipError_t launch_phi_forward(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                              double* GT, hipStream_t s);
// theta stage: GT[t][m][c] -> HM[m][t][c]  (the quadrature-weighted values H'_m(theta_t)).
hipError_t launch_theta(const ShtTables& T, const Batch& b, const double* GT, double* HM, hipStream_t s);
// phi stage, inverse: FT[t][m][c] -> maps (ring stride n, map stride map_stride samples).
// quad: at band-limit 2048, FT in the column-quad layout (as launch_resample_2048 writes it).
hipError_t launch_phi_inverse(const ShtTables& T, const Batch& b, const double* FT, void* f,
                              int64_t map_stride, hipStream_t s, bool quad = false);
// The same three stages compiled for band-limit 2048 (n = 4095); used when applicable.
bool fft_k2048_applies(const ShtTables& T);
hipError_t launch_phi_forward_2048(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                                   double* GT, hipStream_t s);
hipError_t launch_theta_2048(const ShtTables& T, const Batch& b, const double* GT, double* HM, hipStream_t s,
                             bool sym = false);
// Symmetric-grid variants (T.sym; FP64, C in {16, 32}): theta stage onto the psi grid (HM holds
// the north/south sums in rows s < k/2 and differences in rows k/2 + s), the Legendre steps on
// the northern nodes (the synthesis writes FS[m][s][c], s < k), and the resampling FS -> FT[t][m][c].
// At band-limit 2048 the resampling with quad writes FT in the column-quad layout: element
// (t, m, c) at ((t (C/4) + c/4) k + m) 4 + c mod 4, so that the inverse phi stage reads 64 KiB
// contiguous per problem; without quad it writes the row layout, for the general theta stage of
// the adjoint transform.  (FP64 GT keeps the row layout: there the theta stage's loss in the
// column-quad layout outweighs the phi stage's gain.)
hipError_t launch_resample_2048(const ShtTables& T, const Batch& b, const double* FS, double* FT, hipStream_t s,
                                bool quad);
// The same stages compiled for band-limit 1024 (n = 2047 by Bluestein over 4096 points).
// band-limits 512 and 1024 (kernels_fft_bluestein.hip): compiled phi, symmetric-grid theta and
// resampling kernels; fft_bs_applies says whether T is one of them
bool fft_bs_applies(const ShtTables& T);
hipError_t launch_phi_forward_bs(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                                 double* GT, hipStream_t s);
hipError_t launch_phi_inverse_bs(const ShtTables& T, const Batch& b, const double* FT, void* f,
                                 int64_t map_stride, hipStream_t s);
hipError_t launch_theta_sym_bs(const ShtTables& T, const Batch& b, const double* GT, double* HM, hipStream_t s);
hipError_t launch_resample_bs(const ShtTables& T, const Batch& b, const double* FS, double* FT, hipStream_t s);
int legendre_forward_groups_sym(int k);
// lmin: the degrees below it take no products.  Forward: their rows of R are left unwritten (the
// caller reads none of them: the tiling skips rows whose kernel value is zero).  Inverse: their rows
// of S must be zero.  0 = every degree.
hipError_t launch_legendre_forward_sym(const ShtTables& T, const LegTables& G, const Batch& b, const double* HM,
                                       double* R, long long part_stride, int precision, int lmin,
                                       unsigned long long* counter, hipStream_t s);
hipError_t launch_legendre_inverse_sym(const ShtTables& T, const LegTables& G, const Batch& b, const double* S,
                                       double* FS, int precision, int lmin, unsigned long long* counter,
                                       hipStream_t s);
hipError_t launch_legendre_forward_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b,
                                            const double* HM, double* R, long long part_stride, int lmin,
                                            unsigned long long* counter, hipStream_t s);
hipError_t launch_legendre_inverse_bf16_sym(const ShtTables& T, const LegTables& G, const Batch& b,
                                            const double* S, double* FS, int lmin, unsigned long long* counter,
                                            hipStream_t s);
hipError_t launch_phi_inverse_2048(const ShtTables& T, const Batch& b, const double* FT, void* f,
                                   int64_t map_stride, hipStream_t s, bool quad);
// FP32 variants of the band-limit 2048 stages and of the BF16x3 symmetric-grid Legendre kernels'
// ends that meet them: GT, HM, FS and FT hold floats in the same layouts (FT column-quad); the
// maps, R and S stay FP64.
hipError_t launch_phi_forward_2048_f32(const ShtTables& T, const Batch& b, const void* f, int64_t map_stride,
                                       float* GT, hipStream_t s);
hipError_t launch_theta_2048_f32(const ShtTables& T, const Batch& b, const float* GT, float* HM, hipStream_t s);
hipError_t launch_legendre_forward_bf16_sym_f32(const ShtTables& T, const LegTables& G, const Batch& b,
                                                const float* HM, double* R, long long part_stride, int lmin,
                                                unsigned long long* counter, hipStream_t s);
hipError_t launch_resample_2048_f32(const ShtTables& T, const Batch& b, const float* FS, float* FT,
                                    hipStream_t s);
hipError_t launch_phi_inverse_2048_f32(const ShtTables& T, const Batch& b, const float* FT, void* f,
                                       int64_t map_stride, hipStream_t s);
hipError_t launch_legendre_inverse_bf16_sym_f32(const ShtTables& T, const LegTables& G, const Batch& b,
                                                const double* S, float* FS, int lmin, unsigned long long* counter,
                                                hipStream_t s);
// Legendre contraction, forward: HM[m][t][c] -> R[tri_off(k,m)+l-m][c] = sum_t z_lm(theta_t) H',
// written as legendre_forward_groups(k) partial sums over theta ranges, part g at R + g*part_stride.
int legendre_forward_groups(int k);
hipError_t launch_legendre_forward(const ShtTables& T, const LegTables& G, const Batch& b,
                                   const double* HM, double* R, long long part_stride, int precision,
                                   unsigned long long* counter, hipStream_t s);
// Legendre synthesis: S[tri_off(k,m)+l-m][c] (pre-scaled by d_lm) -> FT[t][m][c]
hipError_t launch_legendre_inverse(const ShtTables& T, const LegTables& G, const Batch& b,
                                   const double* S, double* FT, int precision,
                                   unsigned long long* counter, hipStream_t s);
// The same two contractions with BF16x3 operands on the matrix cores (the synthesis for C >= 16).
hipError_t launch_legendre_forward_bf16(const ShtTables& T, const LegTables& G, const Batch& b,
                                        const double* HM, double* R, long long part_stride,
                                        unsigned long long* counter, hipStream_t s);
hipError_t launch_legendre_inverse_bf16(const ShtTables& T, const LegTables& G, const Batch& b,
                                        const double* S, double* FT, unsigned long long* counter,
                                        hipStream_t s);
// ---- persistent Legendre launches over the work items of many transforms (uneven batches) ----
// One task is one symmetric-grid Legendre step of one batch of 32 columns at band-limit k; one item is
// one (m pair, node group) of a task.  A launch's blocks take items in the order given (the caller
// sorts them by decreasing cost) from a device counter until none is left.
struct LegTask {
  const double* in;       // HM (analysis) or S (synthesis), layouts as launch_legendre_*_sym
  double* out;            // R (analysis: node group g's partial sums at out + g * part_stride) or FS
  const double* ut;       // the symmetric-grid tables of band-limit k
  const double* st;
  long long part_stride;
  int k, lmin;
};
struct LegItem {
  int task, pair, sub;    // sub: node group of nw x 64 northern nodes
};
// Tile shapes: nw waves (64 northern nodes each) per block, 1, 2 or 4; a task at band-limit k has
// legendre_persist_groups(k, nw) node groups per m pair.
int legendre_persist_groups(int k, int nw);
bool legendre_persist_shape_ok(bool analysis, int nw);
// Resident blocks per CU of the persistent kernel (for the grid size), 0 if unknown.
int legendre_persist_blocks_per_cu(bool analysis, int nw);
// FP64, 32 columns.  next: one device counter, reset by the launch (a kernel, no memset).
hipError_t launch_legendre_persist(bool analysis, int nw, const LegTask* tasks, const LegItem* items, int nitems,
                                   unsigned* next, const LegTables& G, int nblocks, hipStream_t s);

// Records e as the HIP error behind the status and returns S2LET_EHIP (defined with the C ABI).
int hip_fail(hipError_t e);
int to_status(hipError_t e);
hipError_t launch_hard_threshold(double* w, long long off, long long n, long long stride, int nmaps, bool cplx,
                                 double thr, hipStream_t s);
// dst[b][a][c] = scale * src[a][b][c] over a k x k grid of C-column rows.
hipError_t launch_transpose_rows(const Batch& b, int k, const double* src, double* dst, double scale,
                                 hipStream_t s);
// flm (user layout) -> S (k-packed rows, scaled by d_lm, -m columns by (-1)^m).
hipError_t launch_unpack_flm(const LegTables& G, const Batch& b, int k, const double2* flm,
                             double* S, hipStream_t s, bool herm = false);
// R (k-packed raw forward sums, nparts partials) -> flm (user layout): f_lm = d_lm sum_g R_g
// (and the symmetry for real maps).
hipError_t launch_pack_flm(const LegTables& G, const Batch& b, int k, const double* R, int nparts,
                           long long part_stride, double2* flm, hipStream_t s);
// Tiling: dst[tri_off(kd,m)+l-m][c] (+= for l < kacc, = above) kern[l] * d_lm^2 *
// sum_g src_g[tri_off(ks,m)+l-m][c] for l < min(ks, kd); with zero_fill, rows l >= ks of dst (up to
// kd) are set to zero, otherwise they are left as they are.
hipError_t launch_tile(const LegTables& G, const Batch& b, const double* src, int ks, int nparts,
                       long long part_stride, double* dst, int kd, const double* kern, int kacc, bool zero_fill,
                       hipStream_t s);

}  // namespace s2let
