// Batched wavelet analysis + synthesis of many maps with uneven band-limits and wavelet
// parameters (the paper's transforms, Sects. 2.2 and 3.1-3.2, applied map by map).
//
// Execution plan: maps with equal (L, B) form a group; each group runs the library's batched
// wavelet drivers on contiguous staging copies of its maps (a segmented copy kernel gathers
// the inputs and scatters the outputs back to the caller's order).  Groups are spread over
// worker streams (default priority, longest work first) that fork from and join back to the
// caller's stream through events, so the whole job can be captured into one HIP graph and
// replayed without per-kernel launch overhead.  The number of worker streams and the maps per
// batch are chosen by timing the candidates on the caller's buffers (s2let_batch_autotune).
#include <algorithm>
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

namespace {

// dst[seg.dst + i] = src[seg.src + i], i < seg.len (doubles); blockIdx.y = segment
struct Seg {
  long long src, dst, len;
};

__global__ void k_seg_copy(const double* __restrict__ src, double* __restrict__ dst, const Seg* __restrict__ segs) {
  const Seg sg = segs[blockIdx.y];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x)
    dst[sg.dst + i] = src[sg.src + i];
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
int run(s2let_batch* b, void* f_wav, void* f_scal, void* rec, const void* f, void* ws, size_t ws_bytes,
        hipStream_t caller, bool do_synthesis) {
  if (ws_bytes < s2let_batch_workspace_size(b)) return S2LET_ENOMEM;
  char* base = (char*)ws;
  double* stage = (double*)(base + kMaxStreams * b->ws_stream);
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
  return kMaxStreams * b->ws_stream + sizeof(double) * (size_t)b->staging;
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
  for (int a = 0; a < 4 && st == S2LET_OK; ++a)
    for (int c = 0; c < 3 && st == S2LET_OK; ++c) {
      if ((st = set_config(b, nstr[a], caps[c])) != S2LET_OK) break;
      if ((st = run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, true)) != S2LET_OK) break;   // warm
      hipEventRecord(e0, s);
      if ((st = run(b, f_wav, f_scal, rec, f, ws, ws_bytes, s, true)) != S2LET_OK) break;
      hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = S2LET_EHIP;
        break;
      }
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      if (best < 0 || ms < best) {
        best = ms;
        bs = nstr[a];
        bc = caps[c];
      }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != S2LET_OK) return st;
  if ((st = set_config(b, bs, bc)) != S2LET_OK) return st;
  if (best_streams) *best_streams = bs;
  if (best_cap) *best_cap = bc;
  if (best_ms) *best_ms = best;
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
