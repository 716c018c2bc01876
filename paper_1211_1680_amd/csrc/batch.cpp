// Batched wavelet analysis + synthesis of many maps with uneven band-limits and wavelet
// parameters (the paper's transforms, Sects. 2.2 and 3.1-3.2, applied map by map).
//
// Maps with equal (L, B) form a group, gathered into contiguous staging copies (a segmented copy
// kernel gathers the inputs and scatters the outputs back to the caller's order).  Two ways to run
// the job, both on worker streams (default priority) that fork from and join back to the caller's
// stream through events, so that the whole job can be captured into one HIP graph:
//  - streams: each group runs the library's batched wavelet drivers on its own worker stream
//    (longest work first);
//  - persistent (FP64): the job runs level by level across every map and scale.  The O(k^3)
//    Legendre steps of one level -- the signal's analysis at L, the inverse transforms of every
//    scale, the forward transforms of every scale, the synthesis at L -- become work items
//    (batch of maps, scale, m pair, node group) sorted by decreasing cost and taken from a device
//    counter by one persistent launch per tile shape; the phi, theta, tiling and resampling stages
//    between them run per transform on the worker streams.  The tile shape (waves, i.e. 64-node
//    groups, per block) is chosen per band-limit bucket.
// s2let_batch_autotune times the stream counts and batch widths, then the persistent mode with
// its tile shapes (one bucket at a time), on the caller's buffers, and keeps the fastest.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/s2let_mi355x.h"
#include "common.h"

#define S2LET_API extern "C" __attribute__((visibility("default")))

// capped wavelet drivers of abi.cpp
int s2let_wav_map_to_scales(void* f_wav, void* f_scal, const void* f, int L, int B, int J_min, int multires,
                            int reality, int precision, int nmaps, void* ws, size_t ws_bytes, void* stream,
                            bool adjoint, int cap, int kernel, bool build_plans);
int s2let_wav_scales_to_map(void* f, const void* f_wav, const void* f_scal, int L, int B, int J_min,
                            int multires, int reality, int precision, int nmaps, void* ws, size_t ws_bytes,
                            void* stream, bool adjoint, int cap, int kernel);

namespace s2let {
int cached_leg(const LegTables** G);
int cached_sht(int k, const ShtTables** T);
int cached_wav(int L, int B, int J_min, const double** kappa, const double** eta, std::vector<int>* lmin);
}  // namespace s2let

namespace {

// dst[seg.dst + i] = src[seg.src + i], i < seg.len (doubles); blockIdx.y = segment
struct Seg {
  long long src, dst, len;
};

// One segment per blockIdx.y.  Where source and destination are alike modulo 16 bytes, the body
// moves 16-byte pairs (after a one-element head that aligns them); otherwise single elements.
__global__ void k_seg_copy(const double* __restrict__ src, double* __restrict__ dst, const Seg* __restrict__ segs) {
  const Seg sg = segs[blockIdx.y];
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const double* ps = src + sg.src;
  double* pd = dst + sg.dst;
  // (doubles are 8-byte aligned: an address is 16-byte aligned or 8 past it)
  const uintptr_t as = reinterpret_cast<uintptr_t>(ps), ad = reinterpret_cast<uintptr_t>(pd);
  if (((as ^ ad) & 15) == 0) {
    const long long head = (ad & 15) ? 1 : 0;   // one element before both are 16-byte aligned
    if (tid == 0 && head && sg.len > 0) pd[0] = ps[0];
    const long long body = sg.len > head ? (sg.len - head) / 2 : 0;
    const double2* s2 = reinterpret_cast<const double2*>(ps + head);
    double2* d2 = reinterpret_cast<double2*>(pd + head);
    for (long long i = tid; i < body; i += stride) d2[i] = s2[i];
    const long long tail = head + 2 * body;   // one element left when len - head is odd
    if (tid == 0 && tail < sg.len) pd[tail] = ps[tail];
  } else {
    for (long long i = tid; i < sg.len; i += stride) pd[i] = ps[i];
  }
}

constexpr int kMaxStreams = 8;

struct Group {
  int L = 0, B = 0;
  std::vector<int> maps;          // map indices, in caller order
  double work = 0;                // (l, m, theta) triples of analysis + synthesis, all maps
  long long st_in = 0, st_wav = 0, st_scal = 0, st_rec = 0;   // staging offsets (doubles)
  long long msz = 0, wsz = 0, psz = 0;                         // per-map sizes (doubles)
  int seg_first[4] = {0, 0, 0, 0};   // descriptor ranges: gather f, scatter wav, scatter scal, scatter rec
  int stream = 0;
};

int64_t wav_size_of(int L, int B, int J_min, int multires) { return s2let_wav_size(L, B, J_min, multires); }

// ---- persistent (level) execution ----
constexpr int kLvC = 32;          // columns of every level batch (fewer maps leave columns unused)
constexpr int kBuckets = 6;       // tile-shape buckets: band-limits 64, 128, ..., 2048
constexpr int kLevels = 4;        // Legendre levels: analysis at L, inverse per scale, forward per scale, synthesis at L
constexpr int kShapes = 3;        // waves per block: 1, 2, 4

int bucket_of(int k) {
  for (int i = 0; i < kBuckets; ++i)
    if (k == (64 << i)) return i;
  return -1;
}
int shape_index(int nw) { return nw == 1 ? 0 : nw == 2 ? 1 : 2; }

// One transform band-limit of one batch of maps: the signal's (L), the scaling map's or a scale's.
struct Slot {
  int k = 0, lmin = 0, ng = 0;          // band-limit, lowest degree with products, partial groups of R
  bool sym = false;                     // Legendre steps on the symmetric grid (persistent items)
  const s2let::ShtTables* T = nullptr;
  const double* kern = nullptr;         // eta or kappa_j (device), for the scales
  long long out_off = 0;                // scales: sample offset of this map within one map's output
  bool scal = false;                    // the scaling map (output to f_scal)
  double *GT = nullptr, *HM = nullptr, *R = nullptr, *S = nullptr;
};
struct LvBatch {
  int group = 0, first = 0, nb = 0;
  s2let::Batch b;
  Slot sig;
  std::vector<Slot> sc;   // the scaling map first, then j = J_min .. J
};

double triples(int k) { return (double)k * k * (k + 1) / 2.0; }

}  // namespace

struct s2let_batch {
  int dev = 0;
  int nmaps = 0, J_min = 0, multires = 1, reality = S2LET_REAL, precision = S2LET_FP64;
  int cmul = 1;
  std::vector<int> L, B;
  std::vector<long long> map_off, wav_off, scal_off;   // caller layout (doubles)
  long long map_total = 0, wav_total = 0, scal_total = 0;
  std::vector<Group> groups;
  int nstreams = 4, cap = 0;                           // 0: the library's default batch width
  hipStream_t streams[kMaxStreams] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kMaxStreams] = {};
  std::vector<Seg> segs;
  Seg* segs_dev = nullptr;
  size_t ws_stream = 0;          // transform workspace per worker stream (largest batch width)
  long long staging = 0;         // staging doubles
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // persistent mode
  int mode = S2LET_BATCH_STREAMS;
  int nw_fwd[kBuckets] = {1, 1, 2, 4, 4, 4}, nw_inv[kBuckets] = {1, 1, 2, 4, 4, 4};
  size_t lv_bytes = 0;                 // level workspace (before the staging areas)
  std::vector<LvBatch> lv;             // built on the first persistent run (needs the device tables)
  const s2let::LegTables* G = nullptr;
  bool lv_items_ok = false;            // items match the current tile shapes
  s2let::LegTask* d_tasks = nullptr;
  s2let::LegItem* d_items = nullptr;
  unsigned* d_next = nullptr;          // one counter per (level, shape)
  int item_off[kLevels][kShapes] = {}, item_cnt[kLevels][kShapes] = {};
  size_t items_cap = 0, tasks_cap = 0;
  int occ[2][kShapes] = {};            // resident blocks per CU of the persistent kernels (0: not asked yet)
  int st_streams = 4, st_cap = 0;      // the streams mode's configuration (restored when switching back)
  int ncu = 0;
  void* lv_ws = nullptr;               // workspace the slots were carved from
};

namespace {

int assign_streams(s2let_batch* b) {
  std::vector<int> order(b->groups.size());
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return b->groups[x].work > b->groups[y].work; });
  std::vector<double> load(b->nstreams, 0.0);
  for (int g : order) {
    const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->groups[g].stream = s;
    load[s] += b->groups[g].work;
  }
  return S2LET_OK;
}

int copy_segments(const s2let_batch* b, const double* src, double* dst, int first, int count, hipStream_t s) {
  if (count <= 0) return S2LET_OK;
  long long maxlen = 0;
  for (int i = first; i < first + count; ++i) maxlen = std::max(maxlen, b->segs[i].len);
  const unsigned gx = (unsigned)std::min<long long>((maxlen + 255) / 256, 1024);
  k_seg_copy<<<dim3(gx > 0 ? gx : 1, count), 256, 0, s>>>(src, dst, b->segs_dev + first);
  return s2let::to_status(hipGetLastError());
}

// analysis (f -> f_wav, f_scal), then optionally synthesis of the analysis output (-> rec), of
// every group, forked over the worker streams and joined back to `caller`.
int run_levels(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f, void* ws, hipStream_t caller,
               bool do_synthesis);

int run(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f, void* ws, size_t ws_bytes,
        hipStream_t caller, bool do_synthesis) {
  if (ws_bytes < s2let_batch_workspace_size(b)) return S2LET_ENOMEM;
  if (b->mode == S2LET_BATCH_PERSISTENT) return run_levels(b, f_wav, f_scal, rec, f, ws, caller, do_synthesis);
  char* base = (char*)ws;
  double* stage = (double*)(base + std::max(kMaxStreams * b->ws_stream, b->lv_bytes));
  if (hipEventRecord(b->ev_fork, caller) != hipSuccess) return S2LET_EHIP;
  for (int s = 0; s < b->nstreams; ++s)
    if (hipStreamWaitEvent(b->streams[s], b->ev_fork, 0) != hipSuccess) return S2LET_EHIP;
  int st = S2LET_OK;
  for (const Group& g : b->groups) {
    hipStream_t s = b->streams[g.stream];
    void* wsg = base + g.stream * b->ws_stream;
    const int n = (int)g.maps.size();
    double* in = stage + g.st_in;
    double* wv = stage + g.st_wav;
    double* sc = stage + g.st_scal;
    double* rc = stage + g.st_rec;
    if ((st = copy_segments(b, (const double*)f, in, g.seg_first[0], n, s)) != S2LET_OK) return st;
    if ((st = s2let_wav_map_to_scales(wv, sc, in, g.L, g.B, b->J_min, b->multires, b->reality, b->precision, n,
                                      wsg, b->ws_stream, s, false, b->cap, S2LET_KERNEL_SD, true)) != S2LET_OK)
      return st;
    if ((st = copy_segments(b, wv, (double*)f_wav, g.seg_first[1], n, s)) != S2LET_OK) return st;
    if ((st = copy_segments(b, sc, (double*)f_scal, g.seg_first[2], n, s)) != S2LET_OK) return st;
    if (do_synthesis) {
      if ((st = s2let_wav_scales_to_map(rc, wv, sc, g.L, g.B, b->J_min, b->multires, b->reality, b->precision, n,
                                        wsg, b->ws_stream, s, false, b->cap, S2LET_KERNEL_SD)) != S2LET_OK)
        return st;
      if ((st = copy_segments(b, rc, (double*)rec, g.seg_first[3], n, s)) != S2LET_OK) return st;
    }
  }
  for (int s = 0; s < b->nstreams; ++s) {
    if (hipEventRecord(b->ev_join[s], b->streams[s]) != hipSuccess) return S2LET_EHIP;
    if (hipStreamWaitEvent(caller, b->ev_join[s], 0) != hipSuccess) return S2LET_EHIP;
  }
  return S2LET_OK;
}

// ---- persistent (level) execution ----

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

int lv_cap(int reality) { return reality == S2LET_REAL ? kLvC / 2 : kLvC / 4; }

// Tile shapes worth trying at band-limit k: waves per block that the k/2 northern nodes fill, and
// at most 4 node groups (partial sums) per m pair.
bool lv_shape_ok(int k, int nw) {
  const int g = s2let::legendre_persist_groups(k, nw);
  return nw * 64 <= ((k / 2 + 63) / 64) * 64 && g <= 4;
}
int lv_groups_max(int k) {
  if (bucket_of(k) < 0) return s2let::legendre_forward_groups(k);
  int g = 1;
  for (int nw : {1, 2, 4})
    if (lv_shape_ok(k, nw)) g = std::max(g, s2let::legendre_persist_groups(k, nw));
  return g;
}
size_t lv_slot_bytes(int k) {
  const size_t sq = sizeof(double) * (size_t)k * k * kLvC;
  const size_t tri = sizeof(double) * (size_t)s2let::tri_rows(k) * kLvC;
  return 2 * al256(sq) + al256(tri * lv_groups_max(k)) + al256(tri);
}

// band-limits of one map's transforms: the signal, the scaling map, the scales J_min..J
std::vector<int> lv_bandlimits(int L, int B, int J_min, int multires) {
  std::vector<int> ks{L, s2let_bandlimit_scal(J_min, L, B, multires)};
  for (int j = J_min; j <= s2let_j_max(L, B); ++j) ks.push_back(s2let_bandlimit_wav(j, L, B, multires));
  return ks;
}

size_t lv_workspace(const s2let_batch* b) {
  size_t tot = 0;
  for (const Group& g : b->groups) {
    const int nbat = ((int)g.maps.size() + lv_cap(b->reality) - 1) / lv_cap(b->reality);
    size_t per = 0;
    for (int k : lv_bandlimits(g.L, g.B, b->J_min, b->multires)) per += lv_slot_bytes(k);
    tot += per * nbat;
  }
  return tot;
}

int lv_tile_of(const s2let_batch* b, int k, bool analysis) {
  const int i = bucket_of(k);
  return i < 0 ? 0 : (analysis ? b->nw_fwd[i] : b->nw_inv[i]);
}

// Slots of every batch, carved from the workspace (device tables built here, outside any capture).
int lv_build_slots(s2let_batch* b, void* ws) {
  using namespace s2let;
  int st;
  if ((st = cached_leg(&b->G)) != S2LET_OK) return st;
  b->lv.clear();
  char* p = (char*)ws;
  const int cap = lv_cap(b->reality);
  for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
    const Group& g = b->groups[gi];
    const double *kappa, *eta;
    std::vector<int> lmin;
    if ((st = cached_wav(g.L, g.B, b->J_min, &kappa, &eta, &lmin)) != S2LET_OK) return st;
    const std::vector<int> ks = lv_bandlimits(g.L, g.B, b->J_min, b->multires);
    for (int first = 0; first < (int)g.maps.size(); first += cap) {
      LvBatch t;
      t.group = gi;
      t.first = first;
      t.nb = std::min(cap, (int)g.maps.size() - first);
      t.b.nb = t.nb;
      t.b.reality = b->reality;
      t.b.used = (b->reality == S2LET_REAL ? 2 : 4) * t.nb;
      t.b.C = kLvC;
      long long off = 0;
      for (size_t i = 0; i < ks.size(); ++i) {
        Slot X;
        X.k = ks[i];
        X.sym = bucket_of(X.k) >= 0;
        if ((st = cached_sht(X.k, &X.T)) != S2LET_OK) return st;
        const size_t sq = al256(sizeof(double) * (size_t)X.k * X.k * kLvC);
        const size_t tri = sizeof(double) * (size_t)tri_rows(X.k) * kLvC;
        X.GT = (double*)p;
        X.HM = (double*)(p + sq);
        X.R = (double*)(p + 2 * sq);
        X.S = (double*)(p + 2 * sq + al256(tri * lv_groups_max(X.k)));
        p += lv_slot_bytes(X.k);
        if (i == 0) {
          t.sig = X;
        } else if (i == 1) {
          X.scal = true;
          X.kern = eta;
          t.sc.push_back(X);
        } else {
          X.kern = kappa + (size_t)(i - 2) * g.L;
          X.lmin = lmin[i - 2];
          X.out_off = off;
          off += (long long)X.k * (2 * X.k - 1);
          t.sc.push_back(X);
        }
      }
      b->lv.push_back(t);
    }
  }
  b->lv_ws = ws;
  b->lv_items_ok = false;
  return S2LET_OK;
}

// Work items of the four Legendre levels, per tile shape, sorted by decreasing cost, uploaded once
// per configuration (not in the timed or captured run).
int lv_build_items(s2let_batch* b) {
  using namespace s2let;
  struct Item {
    LegItem it;
    double cost;
  };
  std::vector<LegTask> tasks;
  std::vector<Item> lists[kLevels][kShapes];
  auto add = [&](int level, Slot& X, bool analysis, const double* in, double* out) {
    const int nw = lv_tile_of(b, X.k, analysis);
    const int ng = legendre_persist_groups(X.k, nw);
    if (analysis) X.ng = ng;
    LegTask tk;
    tk.in = in;
    tk.out = out;
    tk.ut = X.T->ut_s;
    tk.st = X.T->st_s;
    tk.part_stride = (long long)tri_rows(X.k) * kLvC;
    tk.k = X.k;
    tk.lmin = X.lmin;
    const int ti = (int)tasks.size();
    tasks.push_back(tk);
    const int kh = X.k / 2;
    for (int pair = 0; pair < (X.k + 1) / 2; ++pair) {
      // rows of the pair's columns m1 = pair, m2 = k-1-pair (one column when they coincide), and the
      // rows that take products (degrees l >= lmin)
      const int m1 = pair, m2 = X.k - 1 - pair;
      int rows = X.k - m1, prod = std::max(0, X.k - std::max(m1, X.lmin));
      if (m2 > m1) {
        rows += X.k - m2;
        prod += std::max(0, X.k - std::max(m2, X.lmin));
      }
      for (int g = 0; g < ng; ++g) {
        const int nodes = std::min(nw * 64, kh - g * nw * 64);
        Item I;
        I.it.task = ti;
        I.it.pair = pair;
        I.it.sub = g;
        I.cost = (double)nodes * (3.0 * rows + 64.0 * prod);
        lists[level][shape_index(nw)].push_back(I);
      }
    }
  };
  for (LvBatch& t : b->lv) {
    if (t.sig.sym) add(0, t.sig, true, t.sig.HM, t.sig.R);
    else t.sig.ng = legendre_forward_groups(t.sig.k);
    for (Slot& X : t.sc) {
      if (X.sym) {
        add(1, X, false, X.S, X.HM);
        add(2, X, true, X.HM, X.R);
      } else {
        X.ng = legendre_forward_groups(X.k);
      }
    }
    if (t.sig.sym) add(3, t.sig, false, t.sig.S, t.sig.HM);
  }
  std::vector<LegItem> all;
  for (int l = 0; l < kLevels; ++l)
    for (int sh = 0; sh < kShapes; ++sh) {
      auto& v = lists[l][sh];
      std::stable_sort(v.begin(), v.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
      b->item_off[l][sh] = (int)all.size();
      b->item_cnt[l][sh] = (int)v.size();
      for (const Item& I : v) all.push_back(I.it);
    }
  if (tasks.size() > b->tasks_cap) {
    if (b->d_tasks) hipFree(b->d_tasks);
    b->d_tasks = nullptr;
    if (hipMalloc((void**)&b->d_tasks, sizeof(LegTask) * tasks.size()) != hipSuccess) return S2LET_ENOMEM;
    b->tasks_cap = tasks.size();
  }
  if (all.size() > b->items_cap) {
    if (b->d_items) hipFree(b->d_items);
    b->d_items = nullptr;
    if (hipMalloc((void**)&b->d_items, sizeof(LegItem) * all.size()) != hipSuccess) return S2LET_ENOMEM;
    b->items_cap = all.size();
  }
  if (!b->d_next && hipMalloc((void**)&b->d_next, sizeof(unsigned) * kLevels * kShapes) != hipSuccess)
    return S2LET_ENOMEM;
  if (!tasks.empty() &&
      hipMemcpy(b->d_tasks, tasks.data(), sizeof(LegTask) * tasks.size(), hipMemcpyHostToDevice) != hipSuccess)
    return S2LET_EHIP;
  if (!all.empty() && hipMemcpy(b->d_items, all.data(), sizeof(LegItem) * all.size(), hipMemcpyHostToDevice) != hipSuccess)
    return S2LET_EHIP;
  b->lv_items_ok = true;
  return S2LET_OK;
}

// phi and theta stages of the forward transform of slot X (maps at f, map stride in samples)
hipError_t lv_fwd_pre(const Slot& X, const s2let::Batch& bt, const double* f, int64_t stride, hipStream_t s) {
  using namespace s2let;
  hipError_t e = launch_phi_forward(*X.T, bt, f, stride, X.GT, s);
  if (e != hipSuccess) return e;
  if (X.sym) return X.k == 2048 ? launch_theta_2048(*X.T, bt, X.GT, X.HM, s, true) : launch_theta_sym_bs(*X.T, bt, X.GT, X.HM, s);
  return launch_theta(*X.T, bt, X.GT, X.HM, s);
}
// resampling (symmetric grid) and inverse phi stage of slot X, after its Legendre synthesis
hipError_t lv_inv_post(const Slot& X, const s2let::Batch& bt, double* f, int64_t stride, hipStream_t s) {
  using namespace s2let;
  if (X.sym) {
    hipError_t e = X.k == 2048 ? launch_resample_2048(*X.T, bt, X.HM, X.GT, s, true)
                               : launch_resample_bs(*X.T, bt, X.HM, X.GT, s);
    if (e != hipSuccess) return e;
  }
  return launch_phi_inverse(*X.T, bt, X.GT, f, stride, s, X.sym);
}

int lv_persistent_level(s2let_batch* b, int level, bool analysis, int& rr) {
  using namespace s2let;
  for (int sh = 0; sh < kShapes; ++sh) {
    const int n = b->item_cnt[level][sh];
    if (n == 0) continue;
    const int nw = sh == 0 ? 1 : sh == 1 ? 2 : 4;
    int& per_cu = b->occ[analysis ? 0 : 1][sh];
    if (per_cu < 1) per_cu = std::max(1, legendre_persist_blocks_per_cu(analysis, nw));
    if (b->ncu < 1 && (hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->dev) != hipSuccess ||
                       b->ncu < 1))
      b->ncu = 256;
    const int nblocks = std::min(n, per_cu * b->ncu);
    hipError_t e = launch_legendre_persist(analysis, nw, b->d_tasks, b->d_items + b->item_off[level][sh], n,
                                           b->d_next + level * kShapes + sh, *b->G, nblocks,
                                           b->streams[rr++ % b->nstreams]);
    if (e != hipSuccess) return hip_fail(e);
  }
  return S2LET_OK;
}

int fork_streams(s2let_batch* b, hipStream_t caller) {
  if (hipEventRecord(b->ev_fork, caller) != hipSuccess) return S2LET_EHIP;
  for (int s = 0; s < b->nstreams; ++s)
    if (hipStreamWaitEvent(b->streams[s], b->ev_fork, 0) != hipSuccess) return S2LET_EHIP;
  return S2LET_OK;
}
int join_streams(s2let_batch* b, hipStream_t caller) {
  for (int s = 0; s < b->nstreams; ++s) {
    if (hipEventRecord(b->ev_join[s], b->streams[s]) != hipSuccess) return S2LET_EHIP;
    if (hipStreamWaitEvent(caller, b->ev_join[s], 0) != hipSuccess) return S2LET_EHIP;
  }
  return S2LET_OK;
}

// The whole job level by level (FP64).  Level k waits for level k-1 through a join into the
// caller's stream and a fork out of it.
int run_levels(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f, void* ws, hipStream_t caller,
               bool do_synthesis) {
  using namespace s2let;
  int st;
  if (b->lv_ws != ws || b->lv.empty())
    if ((st = lv_build_slots(b, ws)) != S2LET_OK) return st;
  if (!b->lv_items_ok)
    if ((st = lv_build_items(b)) != S2LET_OK) return st;
  double* stage = (double*)((char*)ws + std::max(kMaxStreams * b->ws_stream, b->lv_bytes));
  const int cm = b->cmul;
  hipError_t e;
  int rr = 0;
  auto next_stream = [&]() { return b->streams[rr++ % b->nstreams]; };
#define S2LET_TRY(x)                                   \
  do {                                                 \
    if ((e = (x)) != hipSuccess) return hip_fail(e);   \
  } while (0)
#define S2LET_TRYS(x)                                  \
  do {                                                 \
    if ((st = (x)) != S2LET_OK) return st;             \
  } while (0)
  // staged pointers of one batch
  auto in_of = [&](const LvBatch& t) { const Group& g = b->groups[t.group]; return stage + g.st_in + (long long)t.first * g.msz; };
  auto wav_of = [&](const LvBatch& t, const Slot& X) {
    const Group& g = b->groups[t.group];
    return X.scal ? stage + g.st_scal + (long long)t.first * g.psz : stage + g.st_wav + (long long)t.first * g.wsz + X.out_off * cm;
  };
  auto wstride = [&](const LvBatch& t, const Slot& X) -> int64_t {
    const Group& g = b->groups[t.group];
    return X.scal ? g.psz / cm : g.wsz / cm;
  };
  // gather the inputs; the signal's phi and theta stages
  S2LET_TRYS(fork_streams(b, caller));
  for (const Group& g : b->groups)
    S2LET_TRYS(copy_segments(b, (const double*)f, stage + g.st_in, g.seg_first[0], (int)g.maps.size(), b->streams[g.stream % b->nstreams]));
  S2LET_TRYS(join_streams(b, caller));
  S2LET_TRYS(fork_streams(b, caller));
  for (LvBatch& t : b->lv) S2LET_TRY(lv_fwd_pre(t.sig, t.b, in_of(t), b->groups[t.group].msz / cm, next_stream()));
  S2LET_TRYS(join_streams(b, caller));
  // level 0: the signal's Legendre analysis
  S2LET_TRYS(fork_streams(b, caller));
  S2LET_TRYS(lv_persistent_level(b, 0, true, rr));
  for (LvBatch& t : b->lv)
    if (!t.sig.sym)
      S2LET_TRY(launch_legendre_forward(*t.sig.T, *b->G, t.b, t.sig.HM, t.sig.R, (long long)tri_rows(t.sig.k) * kLvC,
                                        S2LET_FP64, nullptr, next_stream()));
  S2LET_TRYS(join_streams(b, caller));
  // tiling into every scale (Eqs. (4), (6)); the non-symmetric scales' synthesis
  S2LET_TRYS(fork_streams(b, caller));
  for (LvBatch& t : b->lv) {
    hipStream_t s = next_stream();
    for (Slot& X : t.sc) {
      S2LET_TRY(launch_tile(*b->G, t.b, t.sig.R, t.sig.k, t.sig.ng, (long long)tri_rows(t.sig.k) * kLvC, X.S, X.k,
                            X.kern, 0, true, s));
      if (!X.sym) S2LET_TRY(launch_legendre_inverse(*X.T, *b->G, t.b, X.S, X.GT, S2LET_FP64, nullptr, s));
    }
  }
  S2LET_TRYS(join_streams(b, caller));
  // level 1: the scales' Legendre synthesis
  S2LET_TRYS(fork_streams(b, caller));
  S2LET_TRYS(lv_persistent_level(b, 1, false, rr));
  S2LET_TRYS(join_streams(b, caller));
  // the scales' maps; for the synthesis, their forward transforms up to the Legendre step
  S2LET_TRYS(fork_streams(b, caller));
  for (LvBatch& t : b->lv)
    for (Slot& X : t.sc) {
      hipStream_t s = next_stream();
      double* out = wav_of(t, X);
      S2LET_TRY(lv_inv_post(X, t.b, out, wstride(t, X), s));
      if (do_synthesis) {
        S2LET_TRY(lv_fwd_pre(X, t.b, out, wstride(t, X), s));
        if (!X.sym)
          S2LET_TRY(launch_legendre_forward(*X.T, *b->G, t.b, X.HM, X.R, (long long)tri_rows(X.k) * kLvC, S2LET_FP64,
                                            nullptr, s));
      }
    }
  S2LET_TRYS(join_streams(b, caller));
  if (do_synthesis) {
    // level 2: the scales' Legendre analysis
    S2LET_TRYS(fork_streams(b, caller));
    S2LET_TRYS(lv_persistent_level(b, 2, true, rr));
    S2LET_TRYS(join_streams(b, caller));
    // Eq. (8): the tiling sum at L (as the single-batch driver builds it), non-symmetric synthesis at L
    S2LET_TRYS(fork_streams(b, caller));
    for (LvBatch& t : b->lv) {
      hipStream_t s = next_stream();
      const int L = t.sig.k;
      int kmax = 0;
      for (const Slot& X : t.sc) kmax = std::max(kmax, X.k);
      const Slot& P = t.sc[0];
      S2LET_TRY(launch_tile(*b->G, t.b, P.R, P.k, P.ng, (long long)tri_rows(P.k) * kLvC, t.sig.S, L, P.kern, 0,
                            kmax < L, s));
      int kcov = kmax < L ? L : P.k;
      for (size_t i = 1; i < t.sc.size(); ++i) {
        const Slot& X = t.sc[i];
        S2LET_TRY(launch_tile(*b->G, t.b, X.R, X.k, X.ng, (long long)tri_rows(X.k) * kLvC, t.sig.S, L, X.kern, kcov,
                              false, s));
        kcov = std::max(kcov, X.k);
      }
      if (!t.sig.sym) S2LET_TRY(launch_legendre_inverse(*t.sig.T, *b->G, t.b, t.sig.S, t.sig.GT, S2LET_FP64, nullptr, s));
    }
    S2LET_TRYS(join_streams(b, caller));
    // level 3: the synthesis at L
    S2LET_TRYS(fork_streams(b, caller));
    S2LET_TRYS(lv_persistent_level(b, 3, false, rr));
    S2LET_TRYS(join_streams(b, caller));
    S2LET_TRYS(fork_streams(b, caller));
    for (LvBatch& t : b->lv) {
      const Group& g = b->groups[t.group];
      S2LET_TRY(lv_inv_post(t.sig, t.b, stage + g.st_rec + (long long)t.first * g.msz, g.msz / cm, next_stream()));
    }
    S2LET_TRYS(join_streams(b, caller));
  }
  // scatter the outputs to the caller's order
  S2LET_TRYS(fork_streams(b, caller));
  for (const Group& g : b->groups) {
    hipStream_t s = b->streams[g.stream % b->nstreams];
    const int n = (int)g.maps.size();
    S2LET_TRYS(copy_segments(b, stage + g.st_wav, (double*)f_wav, g.seg_first[1], n, s));
    S2LET_TRYS(copy_segments(b, stage + g.st_scal, (double*)f_scal, g.seg_first[2], n, s));
    if (do_synthesis) S2LET_TRYS(copy_segments(b, stage + g.st_rec, (double*)rec, g.seg_first[3], n, s));
  }
  S2LET_TRYS(join_streams(b, caller));
#undef S2LET_TRY
#undef S2LET_TRYS
  return S2LET_OK;
}

void drop_graph(s2let_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

int set_config(s2let_batch* b, int nstreams, int cap) {
  drop_graph(b);
  b->nstreams = nstreams;
  b->cap = cap;
  return assign_streams(b);
}

}  // namespace

S2LET_API int s2let_batch_create(s2let_batch** out, int nmaps, const int* L, const int* B, int J_min,
                                 int multires, int reality, int precision) {
  if (!out || nmaps < 1 || !L || !B) return S2LET_EINVAL;
  if (reality != S2LET_REAL && reality != S2LET_COMPLEX) return S2LET_EINVAL;
  if (precision != S2LET_FP64 && precision != S2LET_MIXED_FP32 && precision != S2LET_MIXED_BF16X3)
    return S2LET_EINVAL;
  *out = nullptr;
  for (int i = 0; i < nmaps; ++i) {
    if (L[i] < 3 || B[i] < 2 || J_min < 0 || J_min >= s2let_j_max(L[i], B[i])) return S2LET_EINVAL;
    if (L[i] > S2LET_MAX_L) return S2LET_EUNSUPPORTED;
  }
  s2let_batch* b = new (std::nothrow) s2let_batch();
  if (!b) return S2LET_ENOMEM;
  if (hipGetDevice(&b->dev) != hipSuccess) {
    delete b;
    return S2LET_EHIP;
  }
  b->nmaps = nmaps;
  b->J_min = J_min;
  b->multires = multires ? 1 : 0;
  b->reality = reality;
  b->precision = precision;
  b->cmul = reality == S2LET_REAL ? 1 : 2;
  b->L.assign(L, L + nmaps);
  b->B.assign(B, B + nmaps);
  // caller layout: maps concatenated in order
  b->map_off.resize(nmaps);
  b->wav_off.resize(nmaps);
  b->scal_off.resize(nmaps);
  for (int i = 0; i < nmaps; ++i) {
    b->map_off[i] = b->map_total;
    b->wav_off[i] = b->wav_total;
    b->scal_off[i] = b->scal_total;
    b->map_total += s2let_mw_size(L[i]) * b->cmul;
    b->wav_total += wav_size_of(L[i], B[i], J_min, multires) * b->cmul;
    b->scal_total += s2let_mw_size(s2let_bandlimit_scal(J_min, L[i], B[i], multires)) * b->cmul;
  }
  // groups by (L, B), in order of first appearance
  for (int i = 0; i < nmaps; ++i) {
    auto it = std::find_if(b->groups.begin(), b->groups.end(),
                           [&](const Group& g) { return g.L == L[i] && g.B == B[i]; });
    if (it == b->groups.end()) {
      Group g;
      g.L = L[i];
      g.B = B[i];
      b->groups.push_back(g);
      it = b->groups.end() - 1;
    }
    it->maps.push_back(i);
  }
  // staging layout and copy descriptors
  for (Group& g : b->groups) {
    const int n = (int)g.maps.size();
    g.msz = s2let_mw_size(g.L) * b->cmul;
    g.wsz = wav_size_of(g.L, g.B, J_min, multires) * b->cmul;
    g.psz = s2let_mw_size(s2let_bandlimit_scal(J_min, g.L, g.B, multires)) * b->cmul;
    double w = triples(g.L);
    const int J = s2let_j_max(g.L, g.B);
    for (int j = J_min; j <= J; ++j) w += triples(s2let_bandlimit_wav(j, g.L, g.B, multires));
    w += triples(s2let_bandlimit_scal(J_min, g.L, g.B, multires));
    g.work = 2.0 * w * n;
    // every staging area starts on a 256-byte boundary (32 doubles)
    auto take = [&](long long count) {
      const long long at = b->staging;
      b->staging = (b->staging + count + 31) & ~31LL;
      return at;
    };
    g.st_in = take((long long)n * g.msz);
    g.st_wav = take((long long)n * g.wsz);
    g.st_scal = take((long long)n * g.psz);
    g.st_rec = take((long long)n * g.msz);
    g.seg_first[0] = (int)b->segs.size();
    for (int q = 0; q < n; ++q) b->segs.push_back({b->map_off[g.maps[q]], (long long)q * g.msz, g.msz});
    g.seg_first[1] = (int)b->segs.size();
    for (int q = 0; q < n; ++q) b->segs.push_back({(long long)q * g.wsz, b->wav_off[g.maps[q]], g.wsz});
    g.seg_first[2] = (int)b->segs.size();
    for (int q = 0; q < n; ++q) b->segs.push_back({(long long)q * g.psz, b->scal_off[g.maps[q]], g.psz});
    g.seg_first[3] = (int)b->segs.size();
    for (int q = 0; q < n; ++q) b->segs.push_back({(long long)q * g.msz, b->map_off[g.maps[q]], g.msz});
  }
  int st = S2LET_OK;
  if (hipMalloc((void**)&b->segs_dev, sizeof(Seg) * b->segs.size()) != hipSuccess ||
      hipMemcpy(b->segs_dev, b->segs.data(), sizeof(Seg) * b->segs.size(), hipMemcpyHostToDevice) != hipSuccess)
    st = S2LET_ENOMEM;
  for (int s = 0; st == S2LET_OK && s < kMaxStreams; ++s)
    if (hipStreamCreateWithFlags(&b->streams[s], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join[s], hipEventDisableTiming) != hipSuccess)
      st = S2LET_EHIP;
  if (st == S2LET_OK && hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) st = S2LET_EHIP;
  if (st == S2LET_OK) {
    size_t wmax = 0;
    for (const Group& g : b->groups)
      wmax = std::max(wmax, s2let_workspace_size(g.L, g.B, J_min, b->multires, reality, precision,
                                                 std::min<int>(reality == S2LET_REAL ? 16 : 8, (int)g.maps.size()), 1));
    b->ws_stream = (wmax + 255) & ~(size_t)255;
    b->lv_bytes = precision == S2LET_FP64 ? lv_workspace(b) : 0;
    st = set_config(b, 4, 0);
  }
  if (st != S2LET_OK) {
    s2let_batch_destroy(b);
    return st;
  }
  *out = b;
  return S2LET_OK;
}

S2LET_API int s2let_batch_destroy(s2let_batch* b) {
  if (!b) return S2LET_OK;
  drop_graph(b);
  for (int s = 0; s < kMaxStreams; ++s) {
    if (b->streams[s]) hipStreamDestroy(b->streams[s]);
    if (b->ev_join[s]) hipEventDestroy(b->ev_join[s]);
  }
  if (b->ev_fork) hipEventDestroy(b->ev_fork);
  if (b->segs_dev) hipFree(b->segs_dev);
  if (b->d_tasks) hipFree(b->d_tasks);
  if (b->d_items) hipFree(b->d_items);
  if (b->d_next) hipFree(b->d_next);
  delete b;
  return S2LET_OK;
}

S2LET_API int s2let_batch_layout(const s2let_batch* b, int64_t* totals, int64_t* map_off, int64_t* wav_off,
                                 int64_t* scal_off) {
  if (!b) return S2LET_EINVAL;
  if (totals) {
    totals[0] = b->map_total;
    totals[1] = b->wav_total;
    totals[2] = b->scal_total;
  }
  for (int i = 0; i < b->nmaps; ++i) {
    if (map_off) map_off[i] = b->map_off[i];
    if (wav_off) wav_off[i] = b->wav_off[i];
    if (scal_off) scal_off[i] = b->scal_off[i];
  }
  return S2LET_OK;
}

S2LET_API size_t s2let_batch_workspace_size(const s2let_batch* b) {
  if (!b) return 0;
  // a transform workspace per possible worker stream, sized for the largest batch width (so
  // that autotuning never needs more), then the staging areas
  // (the persistent mode's level buffers share the space of the per-stream workspaces)
  return std::max(kMaxStreams * b->ws_stream, b->lv_bytes) + sizeof(double) * (size_t)b->staging;
}

S2LET_API int s2let_batch_run(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f, void* ws,
                              size_t ws_bytes, void* stream) {
  if (!b || !f_wav || !f_scal || !rec || !f || !ws) return S2LET_EINVAL;
  return run(b, f_wav, f_scal, rec, f, ws, ws_bytes, (hipStream_t)stream, true);
}

S2LET_API int s2let_batch_analysis(s2let_batch* b, void* f_wav, void* f_scal, const void* f, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!b || !f_wav || !f_scal || !f || !ws) return S2LET_EINVAL;
  return run(b, f_wav, f_scal, nullptr, f, ws, ws_bytes, (hipStream_t)stream, false);
}

namespace {
// times one run of the current configuration (after one warm-up run)
int time_run(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f, void* ws, size_t ws_bytes,
             hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms) {
  int st;
  if ((st = run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, true)) != S2LET_OK) return st;   // warm
  if (hipEventRecord(e0, s) != hipSuccess) return S2LET_EHIP;
  if ((st = run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, true)) != S2LET_OK) return st;
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return S2LET_EHIP;
  return hipEventElapsedTime(ms, e0, e1) == hipSuccess ? S2LET_OK : S2LET_EHIP;
}

int set_persistent(s2let_batch* b, const int* nwf, const int* nwi) {
  drop_graph(b);
  b->mode = S2LET_BATCH_PERSISTENT;
  b->nstreams = kMaxStreams;
  for (int i = 0; i < kBuckets; ++i) {
    if (nwf) b->nw_fwd[i] = nwf[i];
    if (nwi) b->nw_inv[i] = nwi[i];
  }
  b->lv_items_ok = false;
  return assign_streams(b);
}
}  // namespace

S2LET_API int s2let_batch_autotune(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f, void* ws,
                                   size_t ws_bytes, void* stream, int* best_streams, int* best_cap, float* best_ms) {
  if (!b || !f_wav || !f_scal || !rec || !f || !ws) return S2LET_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return S2LET_EHIP;
  const int caps_real[] = {4, 8, 16}, caps_cplx[] = {2, 4, 8};
  const int* caps = b->reality == S2LET_REAL ? caps_real : caps_cplx;
  const int nstr[] = {1, 2, 4, 8};
  float best = -1.0f;
  int bs = 4, bc = 0, st = S2LET_OK;
  // streams: worker-stream count x maps per batch
  b->mode = S2LET_BATCH_STREAMS;
  for (int a = 0; a < 4 && st == S2LET_OK; ++a)
    for (int c = 0; c < 3 && st == S2LET_OK; ++c) {
      float ms = 0;
      if ((st = set_config(b, nstr[a], caps[c])) != S2LET_OK) break;
      if ((st = time_run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, e0, e1, &ms)) != S2LET_OK) break;
      if (best < 0 || ms < best) {
        best = ms;
        bs = nstr[a];
        bc = caps[c];
      }
    }
  b->st_streams = bs;
  b->st_cap = bc;
  // persistent (FP64): the tile shape of each band-limit bucket the job uses, one bucket and one
  // direction at a time, starting from the shapes that fill a block with the bucket's nodes
  bool persistent = false;
  int nwf[kBuckets], nwi[kBuckets];
  if (st == S2LET_OK && b->precision == S2LET_FP64) {
    bool used[kBuckets] = {};
    for (const Group& g : b->groups)
      for (int k : lv_bandlimits(g.L, g.B, b->J_min, b->multires))
        if (bucket_of(k) >= 0) used[bucket_of(k)] = true;
    for (int i = 0; i < kBuckets; ++i) {
      const int k = 64 << i;
      nwf[i] = nwi[i] = std::min(4, std::max(1, k / 128));
      while (!lv_shape_ok(k, nwf[i]) && nwf[i] > 1) nwf[i] /= 2, nwi[i] = nwf[i];
    }
    float pbest = -1.0f;
    if ((st = set_persistent(b, nwf, nwi)) == S2LET_OK)
      st = time_run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, e0, e1, &pbest);
    for (int dir = 0; dir < 2 && st == S2LET_OK; ++dir)
      for (int i = 0; i < kBuckets && st == S2LET_OK; ++i) {
        if (!used[i]) continue;
        int* cur = dir == 0 ? nwf : nwi;
        const int start = cur[i];
        int bestnw = start;
        for (int nw : {1, 2, 4}) {
          if (nw == start || !lv_shape_ok(64 << i, nw)) continue;
          cur[i] = nw;
          float ms = 0;
          if ((st = set_persistent(b, nwf, nwi)) != S2LET_OK) break;
          if ((st = time_run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, e0, e1, &ms)) != S2LET_OK) break;
          if (ms < pbest) {
            pbest = ms;
            bestnw = nw;
          }
        }
        cur[i] = bestnw;
      }
    if (st == S2LET_OK && pbest > 0 && pbest < best) {
      best = pbest;
      persistent = true;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != S2LET_OK) return st;
  if (persistent) {
    if ((st = set_persistent(b, nwf, nwi)) != S2LET_OK) return st;
  } else {
    b->mode = S2LET_BATCH_STREAMS;
    if ((st = set_config(b, bs, bc)) != S2LET_OK) return st;
  }
  if (best_streams) *best_streams = bs;
  if (best_cap) *best_cap = bc;
  if (best_ms) *best_ms = best;
  return S2LET_OK;
}

S2LET_API int s2let_batch_set_execution(s2let_batch* b, int mode, const int* nw_analysis, const int* nw_synthesis) {
  if (!b) return S2LET_EINVAL;
  if (mode == S2LET_BATCH_STREAMS) {
    b->mode = mode;
    return set_config(b, b->st_streams, b->st_cap);
  }
  if (mode != S2LET_BATCH_PERSISTENT) return S2LET_EINVAL;
  if (b->precision != S2LET_FP64) return S2LET_EUNSUPPORTED;
  for (int i = 0; i < kBuckets; ++i) {
    const int k = 64 << i;
    if (nw_analysis && !lv_shape_ok(k, nw_analysis[i])) return S2LET_EINVAL;
    if (nw_synthesis && !lv_shape_ok(k, nw_synthesis[i])) return S2LET_EINVAL;
  }
  return set_persistent(b, nw_analysis, nw_synthesis);
}

S2LET_API int s2let_batch_get_execution(const s2let_batch* b, int* mode, int* nstreams, int* maps_per_batch,
                                        int* nw_analysis, int* nw_synthesis) {
  if (!b) return S2LET_EINVAL;
  if (mode) *mode = b->mode;
  if (nstreams) *nstreams = b->nstreams;
  if (maps_per_batch) *maps_per_batch = b->mode == S2LET_BATCH_PERSISTENT ? lv_cap(b->reality) : b->cap;
  for (int i = 0; i < kBuckets; ++i) {
    if (nw_analysis) nw_analysis[i] = b->nw_fwd[i];
    if (nw_synthesis) nw_synthesis[i] = b->nw_inv[i];
  }
  return S2LET_OK;
}

S2LET_API int s2let_batch_graph_capture(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f,
                                        void* ws, size_t ws_bytes, void* stream) {
  if (!b || !f_wav || !f_scal || !rec || !f || !ws) return S2LET_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!s) return S2LET_EINVAL;   // the legacy default stream cannot be captured
  drop_graph(b);
  // one eager run first: every plan table exists before capture (no allocation while capturing)
  int st = run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, true);
  if (st != S2LET_OK) return st;
  if (hipStreamSynchronize(s) != hipSuccess) return S2LET_EHIP;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return S2LET_EHIP;
  st = run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, true);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &g);
  if (st != S2LET_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess || !g) return S2LET_EHIP;
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(b);
    return S2LET_EHIP;
  }
  return S2LET_OK;
}

S2LET_API int s2let_batch_graph_launch(s2let_batch* b, void* stream) {
  if (!b || !b->exec) return S2LET_EINVAL;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? S2LET_OK : S2LET_EHIP;
}
