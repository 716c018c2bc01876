// C ABI of the library: argument validation, the per-device plan cache, workspace layout and
// the per-scale driver of the wavelet transforms (Sects. 2.2, 3.1, 3.2).
#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/s2let_mi355x.h"
#include "common.h"
#include "plan.h"

#define S2LET_API extern "C" __attribute__((visibility("default")))

namespace s2let {

// The HIP error behind the last S2LET_EHIP returned on this thread.
thread_local hipError_t g_last_hip = hipSuccess;

int hip_fail(hipError_t e) {
  g_last_hip = e;
  return S2LET_EHIP;
}

int to_status(hipError_t e) { return e == hipSuccess ? S2LET_OK : hip_fail(e); }

namespace {

struct WavTables {
  int J = 0;
  double* kappa = nullptr;  // [(J-J_min+1) * L]
  double* eta = nullptr;    // [L]
  std::vector<int> lmin;    // per scale: the lowest degree where kappa is not zero
};

struct DevCache {
  std::map<int, ShtTables> sht;
  LegTables leg;
  std::map<std::tuple<int, int, int, int>, WavTables> wav;   // (L, B, J_min, kernel)
};

std::mutex g_mu;
std::map<int, DevCache> g_cache;

// ---- optional per-stage timing (HIP events on the launch stream) ----
struct ProfRec {
  int stage;
  int k;                // band-limit of the launch
  hipEvent_t a, b;
  double flops_full;    // algorithmic flops of the launch (Legendre stages)
  double bytes;         // algorithmic HBM bytes of the launch
  double triples;       // (l, m, theta) triples of the launch
  double rec_flops;     // recursion flops per triple (shared by all columns)
  double col_flops;     // contraction flops per retained triple
  int slot;             // retained-triple counter slot, -1 if none
};
struct Prof {
  bool on = false;
  int dev = -1;
  std::deque<ProfRec> recs;   // stable addresses while records are appended
  unsigned long long* counters = nullptr;   // device, kProfSlots entries
  int next_slot = 0;
};
constexpr int kProfSlots = 8192;
Prof g_prof;

// set while an allocation-free call runs on this thread: no events are created for it
thread_local bool g_prof_suspended = false;

ProfRec* prof_begin(int stage, hipStream_t s, int k) {
  if (!g_prof.on || g_prof_suspended) return nullptr;
  ProfRec r{};
  r.stage = stage;
  r.k = k;
  r.slot = -1;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return nullptr;
  hipEventRecord(r.a, s);
  g_prof.recs.push_back(r);
  return &g_prof.recs.back();
}

unsigned long long* prof_counter(ProfRec* r) {
  if (!r || !g_prof.counters || g_prof.next_slot >= kProfSlots) return nullptr;
  r->slot = g_prof.next_slot++;
  return g_prof.counters + r->slot;
}

void prof_end(ProfRec* r, hipStream_t s) {
  if (r) hipEventRecord(r->b, s);
}

constexpr int kMaxRealPerBatch = 16;     // 2 columns per real map -> 32 columns
constexpr int kMaxComplexPerBatch = 8;   // 4 columns per complex map -> 32 columns

int col_template(int used) {
  int c = 2;
  while (c < used) c <<= 1;
  return c;
}

Batch make_batch(int reality, int nb) {
  Batch b;
  b.nb = nb;
  b.reality = reality;
  b.used = (reality == S2LET_REAL ? 2 : 4) * nb;
  b.C = col_template(b.used);
  return b;
}

int batch_cap(int reality) { return reality == S2LET_REAL ? kMaxRealPerBatch : kMaxComplexPerBatch; }

int jmax_int(int L, int B) {
  int J = 0;
  long long p = 1;
  while (p < L - 1) {
    p *= B;
    ++J;
  }
  return J;
}

long long ipow_cap(int B, int e, long long cap) {
  long long p = 1;
  for (int i = 0; i < e; ++i) {
    p *= B;
    if (p >= cap) return cap;
  }
  return p;
}

// ceil(L / B^e), e >= 0
int ceil_div_pow(int L, int B, int e) {
  long long p = 1;
  for (int i = 0; i < e; ++i) {
    p *= B;
    if (p >= L) return 1;
  }
  return (int)((L + p - 1) / p);
}

int bl_wav(int j, int L, int B, int multires, int kernel = S2LET_KERNEL_SD) {
  if (!multires) return L;
  if (kernel == S2LET_KERNEL_BSPLINE) {
    const int e = jmax_int(L, B) - j - 2;
    return e <= 0 ? L : std::min(L, ceil_div_pow(L, B, e));
  }
  return (int)ipow_cap(B, j + 1, L);
}
int bl_scal(int J_min, int L, int B, int multires, int kernel = S2LET_KERNEL_SD) {
  if (!multires) return L;
  if (kernel == S2LET_KERNEL_BSPLINE) {
    const int e = jmax_int(L, B) - J_min - 1;
    return e <= 0 ? L : std::min(L, ceil_div_pow(L, B, e));
  }
  return (int)ipow_cap(B, J_min, L);
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Workspace {
  double* GT;
  double* HM;
  double* R;
  double* S;
};

// Workspace for transforms up to band-limit L with C columns: GT and HM (k x k x C), R (the
// partial sums of the forward Legendre step, legendre_forward_groups(L) triangles) and S.
size_t ws_bytes_for(int L, int C, bool wavelet) {
  const size_t sq = align_up(sizeof(double) * (size_t)L * L * C);
  const size_t tri = align_up(sizeof(double) * (size_t)tri_rows(L) * C);
  const size_t rp = align_up(sizeof(double) * (size_t)tri_rows(L) * C * legendre_forward_groups(L));
  return 2 * sq + rp + (wavelet ? tri : 0);
}

Workspace carve(void* ws, int L, int C, bool wavelet) {
  Workspace w;
  char* p = (char*)ws;
  const size_t sq = align_up(sizeof(double) * (size_t)L * L * C);
  const size_t rp = align_up(sizeof(double) * (size_t)tri_rows(L) * C * legendre_forward_groups(L));
  w.GT = (double*)p;
  w.HM = (double*)(p + sq);
  w.R = (double*)(p + 2 * sq);
  w.S = wavelet ? (double*)(p + 2 * sq + rp) : w.R;
  return w;
}

// partial-sum layout of the forward Legendre step at band-limit k
// The forward and inverse transforms at the band-limits with compiled transforms (64 to 2048) run
// their Legendre steps on the symmetric grid (see launch_theta_2048 / launch_resample_2048).
// The adjoint of the inverse transform (a Legendre analysis of unweighted phi sums at the MW
// nodes, with no quadrature whose output could be evaluated on another grid) keeps the MW nodes.
bool sym_path(int k, const Batch& b, int precision, bool adjoint) {
  return (k == 2048 || k == 1024 || k == 512 || k == 256 || k == 128 || k == 64) && !adjoint && b.C >= 16;
}
// The Legendre synthesis F_m(theta) = sum_l f_lm lambda_lm(theta) is a band-limited function of
// theta whatever it feeds, so the inverse transform and the adjoint of the forward transform
// (synthesis, then the quadrature's transpose) both evaluate it on the symmetric grid and
// resample it to the MW nodes.
bool sym_inverse_path(int k, const Batch& b) { return sym_path(k, b, S2LET_FP64, false); }
// In the BF16x3 mode at band-limit 2048 the phi, theta and resampling stages may run in FP32 with FP32
// buffers between them and the Legendre kernels (rounding near 1e-7, and half the LDS per problem,
// so that four problems share a CU) where that rounding is relative to what is judged: the inverse
// stages (relative to the output maps) and the forward stages of the wavelet synthesis's per-scale
// transforms (relative to each scale's map, whose sum is the output).  The forward transform of an
// input map keeps FP64 stages: there the rounding is relative to the whole map, and a steep spectrum
// carries it to the high degrees amplified (1.5e-4 of the finest wavelet scale, above the mode's
// bound, measured).  The adjoint transforms (whose theta stage is the general one) stay FP64.
bool f32_stages(const ShtTables& T, bool sym_not_adjoint, int precision) {
  return sym_not_adjoint && precision == S2LET_MIXED_BF16X3 && fft_k2048_applies(T);
}
int nparts_of(int k, const Batch& b, int precision, bool adjoint) {
  return sym_path(k, b, precision, adjoint) ? legendre_forward_groups_sym(k) : legendre_forward_groups(k);
}
long long pstride_of(int k, const Batch& b) { return (long long)tri_rows(k) * b.C; }

// ---- plan cache (lock held by caller) ----
int get_device(int* dev) { return to_status(hipGetDevice(dev)); }

// build = false: look up only; a missing table gives S2LET_ENOTREADY (nothing is allocated).
int ensure_leg(DevCache& dc, bool build = true) {
  if (dc.leg.Lt == 0) {
    if (!build) return S2LET_ENOTREADY;
    hipError_t e = build_leg_tables(S2LET_MAX_L, &dc.leg);
    if (e != hipSuccess) {
      free_leg_tables(&dc.leg);
      return e == hipErrorOutOfMemory ? S2LET_ENOMEM : hip_fail(e);
    }
  }
  return S2LET_OK;
}

int ensure_sht(DevCache& dc, int k, ShtTables** out, bool build = true) {
  auto it = dc.sht.find(k);
  if (it == dc.sht.end()) {
    if (!build) return S2LET_ENOTREADY;
    ShtTables T;
    hipError_t e = build_sht_tables(k, &T);
    if (e != hipSuccess) {
      free_sht_tables(&T);
      return e == hipErrorOutOfMemory ? S2LET_ENOMEM : hip_fail(e);
    }
    it = dc.sht.emplace(k, T).first;
  }
  *out = &it->second;
  return S2LET_OK;
}

int ensure_wav(DevCache& dc, int L, int B, int J_min, int kernel, WavTables** out, bool build = true) {
  auto key = std::make_tuple(L, B, J_min, kernel);
  auto it = dc.wav.find(key);
  if (it == dc.wav.end()) {
    if (!build) return S2LET_ENOTREADY;
    WavTables W;
    W.J = jmax_int(L, B);
    const int ns = W.J - J_min + 1;
    std::vector<double> kappa((size_t)ns * L), eta(L);
    tiling_host_kernel(L, B, J_min, W.J, kernel, kappa.data(), eta.data());
    // the wavelet kernels vanish below their support: coefficients there need no Legendre products
    W.lmin.assign(ns, L);
    for (int i = 0; i < ns; ++i)
      for (int l = 0; l < L; ++l)
        if (kappa[(size_t)i * L + l] != 0.0) {
          W.lmin[i] = l;
          break;
        }
    if (hipMalloc((void**)&W.kappa, sizeof(double) * kappa.size()) != hipSuccess) return S2LET_ENOMEM;
    if (hipMalloc((void**)&W.eta, sizeof(double) * eta.size()) != hipSuccess) {
      hipFree(W.kappa);
      return S2LET_ENOMEM;
    }
    hipError_t e = hipMemcpy(W.kappa, kappa.data(), sizeof(double) * kappa.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(W.eta, eta.data(), sizeof(double) * eta.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      hipFree(W.kappa);
      hipFree(W.eta);
      return hip_fail(e);
    }
    it = dc.wav.emplace(key, W).first;
  }
  *out = &it->second;
  return S2LET_OK;
}

// ---- the harmonic transforms on one batch ----
double triples_of(int k) { return (double)k * (double)k * (double)(k + 1) / 2.0; }

// Maps -> partial Legendre sums R.  adjoint = false: the forward transform (phi DFT, theta
// quadrature, Legendre analysis).  adjoint = true: the adjoint of the inverse transform,
// g_lm = sum_{t,p} conj(Y_lm(theta_t, phi_p)) f(theta_t, phi_p): the phi DFT without its 2 pi/n
// weight, no theta quadrature, the same Legendre analysis.
// lmin > 0: the caller needs no degree below lmin; whole chunks of rows below it stay unwritten (the
// tiling does not read rows where its kernel vanishes).
// scale_maps: the maps are the wavelet or scaling maps of a synthesis, so that the stages' rounding
// is judged against each map (see f32_stages).
int forward_batch(const ShtTables& T, const LegTables& G, const Batch& b, const void* f,
                  int64_t map_stride, const Workspace& w, int precision, hipStream_t s, bool adjoint = false,
                  int lmin = 0, bool scale_maps = false) {
  hipError_t e;
  const double k = T.k, n = T.n;
  const bool sym = sym_path(T.k, b, precision, adjoint);
  const bool f32 = scale_maps && f32_stages(T, sym && !adjoint, precision);
  const double mapb = (b.reality == S2LET_REAL ? 8.0 : 16.0) * b.nb * k * n;
  const double colb = (f32 ? 4.0 : 8.0) * b.used * k * k;
  ProfRec* r = prof_begin(ST_PHI_FWD, s, T.k);
  if (r) r->bytes = mapb + colb;
  e = f32 ? launch_phi_forward_2048_f32(T, b, f, map_stride, (float*)w.GT, s)
          : launch_phi_forward(T, b, f, map_stride, w.GT, s);
  if (e != hipSuccess) return to_status(e);
  prof_end(r, s);
  r = prof_begin(ST_THETA, s, T.k);
  if (r) r->bytes = 2.0 * colb;
  if (adjoint)
    e = launch_transpose_rows(b, T.k, w.GT, w.HM, n / (2.0 * M_PI), s);
  else if (f32)
    e = launch_theta_2048_f32(T, b, (const float*)w.GT, (float*)w.HM, s);
  else if (sym)
    e = T.k == 2048 ? launch_theta_2048(T, b, w.GT, w.HM, s, true) : launch_theta_sym_bs(T, b, w.GT, w.HM, s);
  else
    e = launch_theta(T, b, w.GT, w.HM, s);
  if (e != hipSuccess) return to_status(e);
  prof_end(r, s);
  r = prof_begin(ST_LEG_FWD, s, T.k);
  if (r) {
    r->triples = sym ? triples_of(T.k) / 2.0 : triples_of(T.k);
    r->rec_flops = 3.0;
    r->col_flops = 2.0 * b.used;
    r->flops_full = r->triples * (r->rec_flops + r->col_flops);
    r->bytes = colb + 8.0 * b.used * (double)tri_rows(T.k);
  }
  if (f32)
    e = launch_legendre_forward_bf16_sym_f32(T, G, b, (const float*)w.HM, w.R, pstride_of(T.k, b), lmin,
                                             prof_counter(r), s);
  else if (sym)
    e = launch_legendre_forward_sym(T, G, b, w.HM, w.R, pstride_of(T.k, b), precision, lmin, prof_counter(r), s);
  else
    e = launch_legendre_forward(T, G, b, w.HM, w.R, pstride_of(T.k, b), precision, prof_counter(r), s);
  if (e != hipSuccess) return to_status(e);
  prof_end(r, s);
  return S2LET_OK;
}

// Scaled coefficients S -> maps.  adjoint = false: the inverse transform (Legendre synthesis,
// inverse phi DFT).  adjoint = true: the adjoint of the forward transform: Legendre synthesis,
// the theta quadrature (a real symmetric operator per m, its own transpose), and the inverse phi
// DFT times the phi weight 2 pi/n.
// lmin > 0: the rows of S below degree lmin are zero.
int inverse_batch(const ShtTables& T, const LegTables& G, const Batch& b, const double* S, void* f,
                  int64_t map_stride, const Workspace& w, int precision, hipStream_t s, bool adjoint = false,
                  int lmin = 0) {
  hipError_t e;
  const double k = T.k, n = T.n;
  const bool sym = sym_inverse_path(T.k, b);
  const bool f32 = f32_stages(T, sym && !adjoint, precision);
  const double mapb = (b.reality == S2LET_REAL ? 8.0 : 16.0) * b.nb * k * n;
  const double colb = (f32 ? 4.0 : 8.0) * b.used * k * k;
  ProfRec* r = prof_begin(ST_LEG_INV, s, T.k);
  if (r) {
    r->triples = sym ? triples_of(T.k) / 2.0 : triples_of(T.k);
    r->rec_flops = 3.0;
    r->col_flops = 2.0 * b.used;
    r->flops_full = r->triples * (r->rec_flops + r->col_flops);
    r->bytes = colb + 8.0 * b.used * (double)tri_rows(T.k);
  }
  if (f32)
    e = launch_legendre_inverse_bf16_sym_f32(T, G, b, S, (float*)w.HM, lmin, prof_counter(r), s);
  else if (sym)
    e = launch_legendre_inverse_sym(T, G, b, S, w.HM, precision, lmin, prof_counter(r), s);
  else
    e = launch_legendre_inverse(T, G, b, S, w.GT, precision, prof_counter(r), s);
  if (e != hipSuccess) return to_status(e);
  prof_end(r, s);
  if (sym) {
    // symmetric grid -> MW nodes
    r = prof_begin(ST_RESAMPLE, s, T.k);
    if (r) r->bytes = 2.0 * colb;
    if (f32)
      e = launch_resample_2048_f32(T, b, (const float*)w.HM, (float*)w.GT, s);
    else
      e = T.k == 2048 ? launch_resample_2048(T, b, w.HM, w.GT, s, !adjoint) : launch_resample_bs(T, b, w.HM, w.GT, s);
    if (e != hipSuccess) return to_status(e);
    prof_end(r, s);
  }
  if (adjoint) {
    r = prof_begin(ST_THETA, s, T.k);
    if (r) r->bytes = 4.0 * colb;
    if ((e = launch_theta(T, b, w.GT, w.HM, s)) != hipSuccess) return to_status(e);
    if ((e = launch_transpose_rows(b, T.k, w.HM, w.GT, 2.0 * M_PI / n, s)) != hipSuccess) return to_status(e);
    prof_end(r, s);
  }
  r = prof_begin(ST_PHI_INV, s, T.k);
  if (r) r->bytes = mapb + colb;
  e = f32 ? launch_phi_inverse_2048_f32(T, b, (const float*)w.GT, f, map_stride, s)
          : launch_phi_inverse(T, b, w.GT, f, map_stride, s, sym && !adjoint);
  if (e != hipSuccess) return to_status(e);
  prof_end(r, s);
  return S2LET_OK;
}

// (kacc: rows below it accumulate into dst, rows above are written; zero_fill: rows >= ks of dst
// up to kd are zeroed)
hipError_t tile_prof(const LegTables& G, const Batch& b, const double* src, int ks, int nparts, double* dst, int kd,
                     const double* kern, int kacc, bool zero_fill, hipStream_t s) {
  ProfRec* r = prof_begin(ST_TILE, s, kd);
  if (r) {
    // coefficients read once, destination written (and read where accumulating)
    const double kk = std::min(ks, kd), ka = std::min(kacc, (int)kk);
    const double tk = kk * (kk + 1) / 2.0, ta = ka * (ka + 1) / 2.0;
    r->bytes = 8.0 * b.used * (2.0 * tk + ta + (zero_fill ? (double)tri_rows(kd) - tk : 0.0));
  }
  hipError_t e = launch_tile(G, b, src, ks, nparts, pstride_of(ks, b), dst, kd, kern, kacc, zero_fill, s);
  prof_end(r, s);
  return e;
}

int check_common(int reality, int precision, int nmaps) {
  if (reality != S2LET_REAL && reality != S2LET_COMPLEX) return S2LET_EINVAL;
  if (precision != S2LET_FP64 && precision != S2LET_MIXED_FP32 && precision != S2LET_MIXED_BF16X3)
    return S2LET_EINVAL;
  if (nmaps < 1) return S2LET_EINVAL;
  return S2LET_OK;
}

int check_wavelet(int L, int B, int J_min, int multires) {
  if (L < 3 || B < 2) return S2LET_EINVAL;
  if (multires != 0 && multires != 1) return S2LET_EINVAL;
  const int J = jmax_int(L, B);
  if (J_min < 0 || J_min >= J) return S2LET_EINVAL;
  return S2LET_OK;
}

int64_t wav_size_int(int L, int B, int J_min, int multires, int kernel = S2LET_KERNEL_SD) {
  const int J = jmax_int(L, B);
  int64_t tot = 0;
  for (int j = J_min; j <= J; ++j) {
    const int64_t k = bl_wav(j, L, B, multires, kernel);
    tot += k * (2 * k - 1);
  }
  return tot;
}

}  // namespace

// Plan tables of the current device for the uneven-batch executor (built on first use; the cache
// keeps them at stable addresses until s2let_finalize).
int cached_leg(const LegTables** G) {
  int dev, st;
  if ((st = get_device(&dev)) != S2LET_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  DevCache& dc = g_cache[dev];
  if ((st = ensure_leg(dc)) != S2LET_OK) return st;
  *G = &dc.leg;
  return S2LET_OK;
}

int cached_sht(int k, const ShtTables** T) {
  int dev, st;
  if ((st = get_device(&dev)) != S2LET_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  DevCache& dc = g_cache[dev];
  ShtTables* t;
  if ((st = ensure_sht(dc, k, &t)) != S2LET_OK) return st;
  *T = t;
  return S2LET_OK;
}

int cached_wav(int L, int B, int J_min, const double** kappa, const double** eta, std::vector<int>* lmin) {
  int dev, st;
  if ((st = get_device(&dev)) != S2LET_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  DevCache& dc = g_cache[dev];
  WavTables* W;
  if ((st = ensure_wav(dc, L, B, J_min, S2LET_KERNEL_SD, &W)) != S2LET_OK) return st;
  *kappa = W->kappa;
  *eta = W->eta;
  *lmin = W->lmin;
  return S2LET_OK;
}

}  // namespace s2let

using namespace s2let;

S2LET_API int s2let_j_max(int L, int B) {
  if (L < 3 || B < 2) return S2LET_EINVAL;
  return jmax_int(L, B);
}

S2LET_API int s2let_bandlimit_wav(int j, int L, int B, int multires) {
  if (j < 0 || L < 1 || B < 2) return S2LET_EINVAL;
  return bl_wav(j, L, B, multires);
}

S2LET_API int s2let_bandlimit_scal(int J_min, int L, int B, int multires) {
  if (J_min < 0 || L < 1 || B < 2) return S2LET_EINVAL;
  return bl_scal(J_min, L, B, multires);
}

S2LET_API int64_t s2let_mw_size(int k) { return k < 1 ? -1 : (int64_t)k * (2 * k - 1); }

S2LET_API int64_t s2let_wav_size(int L, int B, int J_min, int multires) {
  if (check_wavelet(L, B, J_min, multires) != S2LET_OK) return -1;
  return wav_size_int(L, B, J_min, multires);
}

S2LET_API int s2let_tiling_axisym(double* kappa, double* eta, int L, int B, int J_min) {
  if (!kappa || !eta) return S2LET_EINVAL;
  if (check_wavelet(L, B, J_min, 0) != S2LET_OK) return S2LET_EINVAL;
  tiling_host(L, B, J_min, jmax_int(L, B), kappa, eta);
  return S2LET_OK;
}

S2LET_API size_t s2let_workspace_size(int L, int B, int J_min, int multires, int reality,
                                      int precision, int nmaps, int wavelet) {
  if (check_common(reality, precision, nmaps) != S2LET_OK) return 0;
  if (L < 1 || L > S2LET_MAX_L) return 0;
  if (wavelet && check_wavelet(L, B, J_min, multires) != S2LET_OK) return 0;
  const int nb = std::min(nmaps, batch_cap(reality));
  const Batch b = make_batch(reality, nb);
  return ws_bytes_for(L, b.C, wavelet != 0);
}

static int prologue(int L, int reality, int precision, int nmaps, void* ws, size_t ws_bytes,
                    bool wavelet, int* dev, int cap = 0) {
  int st = check_common(reality, precision, nmaps);
  if (st != S2LET_OK) return st;
  if (L < 1) return S2LET_EINVAL;
  if (L > S2LET_MAX_L) return S2LET_EUNSUPPORTED;
  if (!ws || !aligned16(ws)) return S2LET_EINVAL;
  const Batch b = make_batch(reality, std::min(nmaps, cap > 0 ? cap : batch_cap(reality)));
  if (ws_bytes < ws_bytes_for(L, b.C, wavelet)) return S2LET_ENOMEM;
  return get_device(dev);
}

// Maps -> coefficients: the forward transform (adjoint = false) or the adjoint of the inverse
// transform (adjoint = true).
static int sht_maps_to_coefs(void* flm, const void* f, int L, int reality, int precision, int nmaps, void* ws,
                             size_t ws_bytes, void* stream, bool adjoint) {
  if (!flm || !f || !aligned16(flm) || !aligned16(f)) return S2LET_EINVAL;
  int dev;
  int st = prologue(L, reality, precision, nmaps, ws, ws_bytes, false, &dev);
  if (st != S2LET_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DevCache& dc = g_cache[dev];
  if ((st = ensure_leg(dc)) != S2LET_OK) return st;
  ShtTables* T;
  if ((st = ensure_sht(dc, L, &T)) != S2LET_OK) return st;
  const int cap = batch_cap(reality);
  const int64_t msz = s2let_mw_size(L);
  const int cmul = reality == S2LET_REAL ? 1 : 2;
  for (int start = 0; start < nmaps; start += cap) {
    const Batch b = make_batch(reality, std::min(cap, nmaps - start));
    const Workspace w = carve(ws, L, b.C, false);
    const double* fin = (const double*)f + (size_t)start * msz * cmul;
    if ((st = forward_batch(*T, dc.leg, b, fin, msz, w, precision, s, adjoint)) != S2LET_OK) return st;
    double2* out = (double2*)flm + (size_t)start * L * L;
    hipError_t e = launch_pack_flm(dc.leg, b, L, w.R, nparts_of(L, b, precision, adjoint), pstride_of(L, b), out, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  return S2LET_OK;
}

// Coefficients -> maps: the inverse transform (adjoint = false) or the adjoint of the forward
// transform (adjoint = true; for real maps the coefficients are first replaced by their Hermitian
// part, which makes the result the adjoint with respect to the real inner products).
static int sht_coefs_to_maps(void* f, const void* flm, int L, int reality, int precision, int nmaps, void* ws,
                             size_t ws_bytes, void* stream, bool adjoint) {
  if (!flm || !f || !aligned16(flm) || !aligned16(f)) return S2LET_EINVAL;
  int dev;
  int st = prologue(L, reality, precision, nmaps, ws, ws_bytes, false, &dev);
  if (st != S2LET_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DevCache& dc = g_cache[dev];
  if ((st = ensure_leg(dc)) != S2LET_OK) return st;
  ShtTables* T;
  if ((st = ensure_sht(dc, L, &T)) != S2LET_OK) return st;
  const int cap = batch_cap(reality);
  const int64_t msz = s2let_mw_size(L);
  const int cmul = reality == S2LET_REAL ? 1 : 2;
  for (int start = 0; start < nmaps; start += cap) {
    const Batch b = make_batch(reality, std::min(cap, nmaps - start));
    const Workspace w = carve(ws, L, b.C, false);
    const double2* in = (const double2*)flm + (size_t)start * L * L;
    hipError_t e = launch_unpack_flm(dc.leg, b, L, in, w.S, s, adjoint);
    if (e != hipSuccess) return hip_fail(e);
    double* fout = (double*)f + (size_t)start * msz * cmul;
    if ((st = inverse_batch(*T, dc.leg, b, w.S, fout, msz, w, precision, s, adjoint)) != S2LET_OK) return st;
  }
  return S2LET_OK;
}

S2LET_API int mw_forward(void* flm, const void* f, int L, int reality, int precision, int nmaps,
                         void* ws, size_t ws_bytes, void* stream) {
  return sht_maps_to_coefs(flm, f, L, reality, precision, nmaps, ws, ws_bytes, stream, false);
}

S2LET_API int mw_inverse(void* f, const void* flm, int L, int reality, int precision, int nmaps,
                         void* ws, size_t ws_bytes, void* stream) {
  return sht_coefs_to_maps(f, flm, L, reality, precision, nmaps, ws, ws_bytes, stream, false);
}

S2LET_API int mw_inverse_adjoint(void* flm, const void* f, int L, int reality, int precision, int nmaps,
                                 void* ws, size_t ws_bytes, void* stream) {
  return sht_maps_to_coefs(flm, f, L, reality, precision, nmaps, ws, ws_bytes, stream, true);
}

S2LET_API int mw_forward_adjoint(void* f, const void* flm, int L, int reality, int precision, int nmaps,
                                 void* ws, size_t ws_bytes, void* stream) {
  return sht_coefs_to_maps(f, flm, L, reality, precision, nmaps, ws, ws_bytes, stream, true);
}

// Map at L -> wavelet and scaling maps.  adjoint = false: the analysis, Eqs. (4) and (6).
// adjoint = true: the adjoint of the synthesis of Eq. (8) (inverse-transform adjoint at L, the
// real diagonal kernels and truncation, forward-transform adjoints at each scale).
// build_plans = false: the plan tables must already be cached for this device (S2LET_ENOTREADY
// otherwise), so that the call allocates nothing.
int s2let_wav_map_to_scales(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min, int multires,
                             int reality, int precision, int nmaps, void* ws, size_t ws_bytes, void* stream,
                             bool adjoint, int cap, int kernel, bool build_plans) {
  if (!f_wav || !f_scal || !f || !aligned16(f_wav) || !aligned16(f_scal) || !aligned16(f))
    return S2LET_EINVAL;
  int st = check_wavelet(L, B, J_min, multires);
  if (st != S2LET_OK) return st;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE)
    return kernel == S2LET_KERNEL_NEEDLET ? S2LET_EUNSUPPORTED : S2LET_EINVAL;
  int dev;
  if ((st = prologue(L, reality, precision, nmaps, ws, ws_bytes, true, &dev, cap)) != S2LET_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!build_plans && g_cache.find(dev) == g_cache.end()) return S2LET_ENOTREADY;
  DevCache& dc = g_cache[dev];
  if ((st = ensure_leg(dc, build_plans)) != S2LET_OK) return st;
  WavTables* W;
  if ((st = ensure_wav(dc, L, B, J_min, kernel, &W, build_plans)) != S2LET_OK) return st;
  const int J = W->J;
  const int kP = bl_scal(J_min, L, B, multires, kernel);
  ShtTables *TL, *TP;
  if ((st = ensure_sht(dc, L, &TL, build_plans)) != S2LET_OK) return st;
  if ((st = ensure_sht(dc, kP, &TP, build_plans)) != S2LET_OK) return st;
  std::vector<ShtTables*> TJ;
  for (int j = J_min; j <= J; ++j) {
    ShtTables* t;
    if ((st = ensure_sht(dc, bl_wav(j, L, B, multires, kernel), &t, build_plans)) != S2LET_OK) return st;
    TJ.push_back(t);
  }
  const int bcap = cap > 0 ? std::min(cap, batch_cap(reality)) : batch_cap(reality);
  const int cmul = reality == S2LET_REAL ? 1 : 2;
  const int64_t msz = s2let_mw_size(L), wsz = wav_size_int(L, B, J_min, multires, kernel),
                psz = s2let_mw_size(kP);
  for (int start = 0; start < nmaps; start += bcap) {
    const Batch b = make_batch(reality, std::min(bcap, nmaps - start));
    const Workspace w = carve(ws, L, b.C, true);
    const double* fin = (const double*)f + (size_t)start * msz * cmul;
    if ((st = forward_batch(*TL, dc.leg, b, fin, msz, w, precision, s, adjoint)) != S2LET_OK) return st;
    // scaling part, Eq. (6)
    hipError_t e = tile_prof(dc.leg, b, w.R, L, nparts_of(L, b, precision, adjoint), w.S, kP, W->eta, 0, true, s);
    if (e != hipSuccess) return hip_fail(e);
    double* pout = (double*)f_scal + (size_t)start * psz * cmul;
    if ((st = inverse_batch(*TP, dc.leg, b, w.S, pout, psz, w, precision, s, adjoint)) != S2LET_OK) return st;
    // wavelet scales, Eq. (4)
    int64_t off = 0;
    for (int j = J_min; j <= J; ++j) {
      const int kj = bl_wav(j, L, B, multires, kernel);
      e = tile_prof(dc.leg, b, w.R, L, nparts_of(L, b, precision, adjoint), w.S, kj,
                    W->kappa + (size_t)(j - J_min) * L, 0, true, s);
      if (e != hipSuccess) return hip_fail(e);
      double* wout = (double*)f_wav + ((size_t)start * wsz + off) * cmul;
      if ((st = inverse_batch(*TJ[j - J_min], dc.leg, b, w.S, wout, wsz, w, precision, s, adjoint,
                              W->lmin[j - J_min])) != S2LET_OK)
        return st;
      off += (int64_t)kj * (2 * kj - 1);
    }
  }
  return S2LET_OK;
}

// Wavelet and scaling maps -> map at L.  adjoint = false: the synthesis, Eq. (8).  adjoint =
// true: the adjoint of the analysis (inverse-transform adjoints at each scale, the kernels,
// forward-transform adjoint at L).
int s2let_wav_scales_to_map(void* f, const void* f_wav, const void* f_scal, int L, int B, int J_min,
                             int multires, int reality, int precision, int nmaps, void* ws, size_t ws_bytes,
                             void* stream, bool adjoint, int cap, int kernel) {
  if (!f_wav || !f_scal || !f || !aligned16(f_wav) || !aligned16(f_scal) || !aligned16(f))
    return S2LET_EINVAL;
  int st = check_wavelet(L, B, J_min, multires);
  if (st != S2LET_OK) return st;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE)
    return kernel == S2LET_KERNEL_NEEDLET ? S2LET_EUNSUPPORTED : S2LET_EINVAL;
  int dev;
  if ((st = prologue(L, reality, precision, nmaps, ws, ws_bytes, true, &dev, cap)) != S2LET_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DevCache& dc = g_cache[dev];
  if ((st = ensure_leg(dc)) != S2LET_OK) return st;
  WavTables* W;
  if ((st = ensure_wav(dc, L, B, J_min, kernel, &W)) != S2LET_OK) return st;
  const int J = W->J;
  const int kP = bl_scal(J_min, L, B, multires, kernel);
  ShtTables *TL, *TP;
  if ((st = ensure_sht(dc, L, &TL)) != S2LET_OK) return st;
  if ((st = ensure_sht(dc, kP, &TP)) != S2LET_OK) return st;
  std::vector<ShtTables*> TJ;
  for (int j = J_min; j <= J; ++j) {
    ShtTables* t;
    if ((st = ensure_sht(dc, bl_wav(j, L, B, multires, kernel), &t)) != S2LET_OK) return st;
    TJ.push_back(t);
  }
  const int bcap = cap > 0 ? std::min(cap, batch_cap(reality)) : batch_cap(reality);
  const int cmul = reality == S2LET_REAL ? 1 : 2;
  const int64_t msz = s2let_mw_size(L), wsz = wav_size_int(L, B, J_min, multires, kernel),
                psz = s2let_mw_size(kP);
  for (int start = 0; start < nmaps; start += bcap) {
    const Batch b = make_batch(reality, std::min(bcap, nmaps - start));
    const Workspace w = carve(ws, L, b.C, true);
    // scaling part
    const double* pin = (const double*)f_scal + (size_t)start * psz * cmul;
    if ((st = forward_batch(*TP, dc.leg, b, pin, psz, w, precision, s, adjoint, 0, true)) != S2LET_OK) return st;
    // S is built over the degrees the contributions cover so far (kcov): each tiling accumulates
    // below kcov and writes the new rows above it, so no row is zero-filled first -- unless the scales
    // stop short of L, which the band-limits of Eqs. (4), (8) rule out
    int kmax = kP;
    for (int j = J_min; j <= J; ++j) kmax = std::max(kmax, bl_wav(j, L, B, multires, kernel));
    hipError_t e = tile_prof(dc.leg, b, w.R, kP, nparts_of(kP, b, precision, adjoint), w.S, L, W->eta, 0,
                             kmax < L, s);
    if (e != hipSuccess) return hip_fail(e);
    int kcov = kmax < L ? L : kP;
    // wavelet scales, accumulated per Eq. (8)
    int64_t off = 0;
    for (int j = J_min; j <= J; ++j) {
      const int kj = bl_wav(j, L, B, multires, kernel);
      const double* win = (const double*)f_wav + ((size_t)start * wsz + off) * cmul;
      if ((st = forward_batch(*TJ[j - J_min], dc.leg, b, win, wsz, w, precision, s, adjoint,
                              W->lmin[j - J_min], true)) != S2LET_OK)
        return st;
      e = tile_prof(dc.leg, b, w.R, kj, nparts_of(kj, b, precision, adjoint), w.S, L,
                    W->kappa + (size_t)(j - J_min) * L, kcov, false, s);
      if (e != hipSuccess) return hip_fail(e);
      kcov = std::max(kcov, kj);
      off += (int64_t)kj * (2 * kj - 1);
    }
    double* fout = (double*)f + (size_t)start * msz * cmul;
    if ((st = inverse_batch(*TL, dc.leg, b, w.S, fout, msz, w, precision, s, adjoint)) != S2LET_OK) return st;
  }
  return S2LET_OK;
}

S2LET_API int s2let_axisym_analysis(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min,
                                    int multires, int reality, int precision, int nmaps, void* ws,
                                    size_t ws_bytes, void* stream) {
  return s2let_wav_map_to_scales(f_wav, f_scal, f, L, B, J_min, multires, reality, precision, nmaps, ws, ws_bytes,
                           stream, false, 0, S2LET_KERNEL_SD, true);
}

// ---- the allocation-free analysis ----
// Its workspace is this file-scope device array: each device that loads the library holds its own
// copy until the process ends.  Host code never uses the array's name as an address (on the host it
// names a stand-in, not device memory); it uses the per-device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
static __device__ __align__(256) char scratch[S2LET_NOALLOC_SCRATCH_BYTES];

namespace {
std::map<int, void*> g_scratch_addr;   // device -> that device's copy of scratch (under g_mu)

// Clears the per-thread switch that keeps profiling events out of an allocation-free call.
struct ProfSuspend {
  ProfSuspend() { g_prof_suspended = true; }
  ~ProfSuspend() { g_prof_suspended = false; }
};
}  // namespace

S2LET_API int s2let_axisym_analysis_noalloc(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min,
                                            int multires, int reality, int precision, int nmaps, void* stream) {
  int st = check_common(reality, precision, nmaps);
  if (st != S2LET_OK) return st;
  if ((st = check_wavelet(L, B, J_min, multires)) != S2LET_OK) return st;
  if (L > S2LET_MAX_L) return S2LET_EUNSUPPORTED;
  const Batch b = make_batch(reality, std::min(nmaps, batch_cap(reality)));
  const size_t need = ws_bytes_for(L, b.C, true);
  if (need > (size_t)S2LET_NOALLOC_SCRATCH_BYTES) return S2LET_ESCRATCH;
  int dev;
  if ((st = get_device(&dev)) != S2LET_OK) return st;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || p == nullptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
      it = g_scratch_addr.emplace(dev, p).first;
    }
    ws = it->second;
  }
  ProfSuspend quiet;
  return s2let_wav_map_to_scales(f_wav, f_scal, f, L, B, J_min, multires, reality, precision, nmaps, ws,
                                 (size_t)S2LET_NOALLOC_SCRATCH_BYTES, stream, false, 0, S2LET_KERNEL_SD, false);
}

S2LET_API int s2let_axisym_synthesis(void* f, const void* f_wav, const void* f_scal, int L, int B,
                                     int J_min, int multires, int reality, int precision, int nmaps,
                                     void* ws, size_t ws_bytes, void* stream) {
  return s2let_wav_scales_to_map(f, f_wav, f_scal, L, B, J_min, multires, reality, precision, nmaps, ws, ws_bytes,
                           stream, false, 0, S2LET_KERNEL_SD);
}

S2LET_API int s2let_axisym_analysis_adjoint(void* f, const void* f_wav, const void* f_scal, int L, int B,
                                            int J_min, int multires, int reality, int precision, int nmaps,
                                            void* ws, size_t ws_bytes, void* stream) {
  return s2let_wav_scales_to_map(f, f_wav, f_scal, L, B, J_min, multires, reality, precision, nmaps, ws, ws_bytes,
                           stream, true, 0, S2LET_KERNEL_SD);
}

S2LET_API int s2let_axisym_synthesis_adjoint(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min,
                                             int multires, int reality, int precision, int nmaps, void* ws,
                                             size_t ws_bytes, void* stream) {
  return s2let_wav_map_to_scales(f_wav, f_scal, f, L, B, J_min, multires, reality, precision, nmaps, ws, ws_bytes,
                           stream, true, 0, S2LET_KERNEL_SD, true);
}

S2LET_API int s2let_bandlimit_wav_kernel(int j, int L, int B, int multires, int kernel) {
  if (j < 0 || L < 1 || B < 2) return S2LET_EINVAL;
  if (kernel == S2LET_KERNEL_BSPLINE && L < 3) return S2LET_EINVAL;
  if (kernel == S2LET_KERNEL_NEEDLET) return S2LET_EUNSUPPORTED;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE) return S2LET_EINVAL;
  return bl_wav(j, L, B, multires, kernel);
}

S2LET_API int s2let_bandlimit_scal_kernel(int J_min, int L, int B, int multires, int kernel) {
  if (J_min < 0 || L < 1 || B < 2) return S2LET_EINVAL;
  if (kernel == S2LET_KERNEL_BSPLINE && L < 3) return S2LET_EINVAL;
  if (kernel == S2LET_KERNEL_NEEDLET) return S2LET_EUNSUPPORTED;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE) return S2LET_EINVAL;
  return bl_scal(J_min, L, B, multires, kernel);
}

S2LET_API int64_t s2let_wav_size_kernel(int L, int B, int J_min, int multires, int kernel) {
  if (check_wavelet(L, B, J_min, multires) != S2LET_OK) return -1;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE) return -1;
  return wav_size_int(L, B, J_min, multires, kernel);
}

S2LET_API int s2let_tiling_axisym_kernel(double* kappa, double* eta, int L, int B, int J_min, int kernel) {
  if (!kappa || !eta) return S2LET_EINVAL;
  if (check_wavelet(L, B, J_min, 0) != S2LET_OK) return S2LET_EINVAL;
  if (kernel == S2LET_KERNEL_NEEDLET) return S2LET_EUNSUPPORTED;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE) return S2LET_EINVAL;
  tiling_host_kernel(L, B, J_min, jmax_int(L, B), kernel, kappa, eta);
  return S2LET_OK;
}

S2LET_API int s2let_axisym_analysis_kernel(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min,
                                           int multires, int kernel, int reality, int precision, int nmaps,
                                           void* ws, size_t ws_bytes, void* stream) {
  return s2let_wav_map_to_scales(f_wav, f_scal, f, L, B, J_min, multires, reality, precision, nmaps, ws, ws_bytes,
                                 stream, false, 0, kernel, true);
}

S2LET_API int s2let_axisym_synthesis_kernel(void* f, const void* f_wav, const void* f_scal, int L, int B,
                                            int J_min, int multires, int kernel, int reality, int precision,
                                            int nmaps, void* ws, size_t ws_bytes, void* stream) {
  return s2let_wav_scales_to_map(f, f_wav, f_scal, L, B, J_min, multires, reality, precision, nmaps, ws, ws_bytes,
                                 stream, false, 0, kernel);
}

S2LET_API int s2let_noise_std_axisym(double* sigma_wav, int L, int B, int J_min, int kernel, double sigma) {
  if (!sigma_wav || !(sigma >= 0.0)) return S2LET_EINVAL;
  if (check_wavelet(L, B, J_min, 0) != S2LET_OK) return S2LET_EINVAL;
  if (kernel == S2LET_KERNEL_NEEDLET) return S2LET_EUNSUPPORTED;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE) return S2LET_EINVAL;
  const int J = jmax_int(L, B), ns = J - J_min + 1;
  std::vector<double> kappa((size_t)ns * L), eta(L);
  tiling_host_kernel(L, B, J_min, J, kernel, kappa.data(), eta.data());
  for (int j = 0; j < ns; ++j) {
    long double acc = 0.0L;
    for (int l = 0; l < L; ++l) {
      const long double kv = kappa[(size_t)j * L + l];
      acc += (2.0L * l + 1.0L) / (4.0L * 3.141592653589793238462643383279502884L) * kv * kv;
    }
    sigma_wav[j] = (double)(sigma * sqrtl(acc));
  }
  return S2LET_OK;
}

S2LET_API int s2let_hard_threshold(void* f_wav, const double* thresholds, int L, int B, int J_min, int multires,
                                   int kernel, int reality, int nmaps, void* stream) {
  if (!f_wav || !thresholds || !aligned16(f_wav) || nmaps < 1) return S2LET_EINVAL;
  if (reality != S2LET_REAL && reality != S2LET_COMPLEX) return S2LET_EINVAL;
  if (check_wavelet(L, B, J_min, multires) != S2LET_OK) return S2LET_EINVAL;
  if (kernel == S2LET_KERNEL_NEEDLET) return S2LET_EUNSUPPORTED;
  if (kernel != S2LET_KERNEL_SD && kernel != S2LET_KERNEL_BSPLINE) return S2LET_EINVAL;
  const int J = jmax_int(L, B);
  const int64_t wsz = wav_size_int(L, B, J_min, multires, kernel);
  int64_t off = 0;
  for (int j = J_min; j <= J; ++j) {
    const int64_t k = bl_wav(j, L, B, multires, kernel);
    const int64_t n = k * (2 * k - 1);
    hipError_t e = launch_hard_threshold((double*)f_wav, off, n, wsz, nmaps, reality == S2LET_COMPLEX,
                                         thresholds[j - J_min], (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    off += n;
  }
  return S2LET_OK;
}

S2LET_API int s2let_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_prof.recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  g_prof.recs.clear();
  g_prof.next_slot = 0;
  g_prof.on = false;
  if (!on) return S2LET_OK;
  int dev;
  if (hipGetDevice(&dev) != hipSuccess) return S2LET_EHIP;
  if (g_prof.counters && g_prof.dev != dev) {
    hipFree(g_prof.counters);
    g_prof.counters = nullptr;
  }
  if (!g_prof.counters) {
    if (hipMalloc((void**)&g_prof.counters, sizeof(unsigned long long) * kProfSlots) != hipSuccess)
      return S2LET_ENOMEM;
    g_prof.dev = dev;
  }
  if (hipMemset(g_prof.counters, 0, sizeof(unsigned long long) * kProfSlots) != hipSuccess) return S2LET_EHIP;
  g_prof.on = true;
  return S2LET_OK;
}

S2LET_API int s2let_profile_query_k(int stage, int k, double* ms, int64_t* launches, double* flops_full,
                                    double* flops_retained, double* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (stage < 0 || stage >= ST_N || !ms || !launches || !flops_full || !flops_retained || !bytes)
    return S2LET_EINVAL;
  std::vector<unsigned long long> cnt(kProfSlots, 0);
  if (g_prof.counters && g_prof.next_slot > 0) {
    if (hipDeviceSynchronize() != hipSuccess) return S2LET_EHIP;
    if (hipMemcpy(cnt.data(), g_prof.counters, sizeof(unsigned long long) * g_prof.next_slot,
                  hipMemcpyDeviceToHost) != hipSuccess)
      return S2LET_EHIP;
  }
  *ms = 0.0;
  *launches = 0;
  *flops_full = 0.0;
  *flops_retained = 0.0;
  *bytes = 0.0;
  for (auto& r : g_prof.recs) {
    if (r.stage != stage || (k > 0 && r.k != k)) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return S2LET_EHIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return S2LET_EHIP;
    *ms += t;
    *launches += 1;
    *flops_full += r.flops_full;
    *bytes += r.bytes;
    if (r.slot >= 0) *flops_retained += r.triples * r.rec_flops + (double)cnt[r.slot] * r.col_flops;
  }
  return S2LET_OK;
}

S2LET_API int s2let_profile_query(int stage, double* ms, int64_t* launches, double* flops_full,
                                  double* flops_retained, double* bytes) {
  return s2let_profile_query_k(stage, 0, ms, launches, flops_full, flops_retained, bytes);
}

S2LET_API int s2let_sync(void* stream) {
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e);
  e = hipGetLastError();
  return e == hipSuccess ? S2LET_OK : S2LET_EHIP;
}

S2LET_API void s2let_finalize(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  hipGetDevice(&cur);
  for (auto& kv : g_cache) {
    hipSetDevice(kv.first);
    for (auto& t : kv.second.sht) free_sht_tables(&t.second);
    free_leg_tables(&kv.second.leg);
    for (auto& w : kv.second.wav) {
      hipFree(w.second.kappa);
      hipFree(w.second.eta);
    }
  }
  g_cache.clear();
  hipSetDevice(cur);
}

S2LET_API const char* s2let_strerror(int status) {
  switch (status) {
    case S2LET_OK: return "ok";
    case S2LET_EINVAL: return "invalid argument";
    case S2LET_ENOMEM: return "workspace too small or out of device memory";
    case S2LET_EHIP: return "HIP runtime error";
    case S2LET_EUNSUPPORTED: return "unsupported by this library (size or precision)";
    case S2LET_ENOTREADY:
      return "plan tables for these sizes are not built on this device yet (run the allocating call once first)";
    case S2LET_ESCRATCH:
      return "the call needs more workspace than the allocation-free entry point's static scratch holds";
  }
  return "unknown status";
}

S2LET_API int s2let_last_hip_error(void) { return (int)g_last_hip; }

S2LET_API const char* s2let_last_hip_error_name(void) { return hipGetErrorName(g_last_hip); }

S2LET_API const char* s2let_version(void) { return "s2let_mi355x 0.1 (gfx950)"; }
