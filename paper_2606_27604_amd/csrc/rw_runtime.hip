// Host runtime of the C ABI declared in include/rw.h.
//
// Responsibilities: argument validation (before anything is enqueued), the
// context's device workspace (adjoint sums, the persistent queue counter and
// the longest-first schedule), launch shapes (plain static grid, or a persistent grid sized from
// the device's compute-unit count and the kernel's occupancy), the autotuner
// that picks the chunk size and workgroup shape by timing candidates with HIP
// events, and hipGraph replay of the batched launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rw.h"
#include "rw_internal.hpp"

using namespace rw;

namespace {

// Launch shape of a walk.  chunk / 64 is the number of paths each lane of a
// wave walks from one work item (lanes regenerate: a lane takes the item's
// next path as soon as its path ends, so the paths per thread follow from the
// chunk); wgs_per_cu sets the wave occupancy of the persistent grid.
struct TuneCfg {
  int chunk = 2048;        // paths per work item (multiple of 64)
  int waves_per_wg = 4;    // workgroup = waves_per_wg wavefronts
  int wgs_per_cu = 0;      // persistent grid: workgroups per CU (0: occupancy limit)
  // the default shape of a batched call: items shrink for calls with few of
  // them (a shape from the tuner or its cache is kept as it is)
  bool adapt = false;
};

// One instantiation of a captured launch sequence and the event recorded after
// its last replay.
struct GraphExec {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool launched = false;
};

// A launch sequence as a graph, with a small ring of instantiations: a call
// updates the kernel arguments of one whose last replay has finished, so
// back-to-back calls queue without the host waiting for the GPU.
constexpr size_t kMaxGraphExecs = 4;
struct GraphEntry {
  hipGraph_t graph = nullptr;
  std::vector<hipGraphNode_t> nodes;
  std::vector<const void*> funcs;
  std::vector<GraphExec> execs;
  size_t oldest = 0;  // the instantiation replayed longest ago
};

}  // namespace

// ---- scratch of the allocation-free forward (rw_forward_noalloc) ----------
// The forward slot sums of a call whose units span several work items, in a
// file-scope device array: every device the library runs on holds its own
// copy until the process ends, and every rw_forward_noalloc call on a device
// shares it (calls that overlap on one device race).  Host code never passes
// the array's name to a kernel (on the host it only names the symbol): it
// uses the device address that rw_create looks up once per device.
constexpr int64_t kNoAllocScratchBytes = int64_t(64) << 20;
// largest work item the allocation-free plan grows to before it gives up
constexpr int kNoAllocMaxChunk = 1 << 16;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device
}  // namespace

struct rw_context {
  int device = -1;          // -1: validation-only context (no device)
  void* scratch = nullptr;  // this device's copy of `scratch` (device address)
  int n_cu = 0;
  int max_lds = 0;          // bytes of LDS a workgroup may allocate
  char last_error[512] = {0};  // a fixed buffer: reporting an error allocates nothing
  void* workspace = nullptr;      // adjoint sums (128-bit) and vertex counts
  size_t workspace_bytes = 0;
  uint32_t* queue = nullptr;
  // longest-first schedule: [hist (kOrderBuckets u32) | bucket (n i32) | order (n i32)]
  char* sched = nullptr;
  size_t sched_bytes = 0;
  std::map<std::string, TuneCfg> tune;
  std::map<std::string, GraphEntry> graphs;
  bool tune_cache_loaded = false;
};

namespace {

rw_status fail(rw_context* ctx, rw_status st, const char* fmt, ...) {
  if (ctx) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->last_error, sizeof(ctx->last_error), fmt, ap);
    va_end(ap);
  }
  return st;
}

bool fault_injected(const char* what) {
  const char* e = std::getenv("RW_FAULT_INJECT");
  return e && std::strcmp(e, what) == 0;
}

#define RW_HIP(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, RW_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));           \
  } while (0)

rw_status check_geom(rw_context* ctx, const rw_geometry* g) {
  if (!g) return fail(ctx, RW_E_INVALID, "geometry is NULL");
  if (g->n_media < 1) return fail(ctx, RW_E_INVALID, "n_media must be >= 1 (got %d)", g->n_media);
  if (g->n_media > kMaxMedia)
    return fail(ctx, RW_E_UNSUPPORTED, "n_media %d > %d is not supported", g->n_media, kMaxMedia);
  if (g->n_bins < 1 || g->n_bins > 4096)
    return fail(ctx, RW_E_INVALID, "n_bins must be in [1, 4096] (got %d)", g->n_bins);
  if (!(g->n_rel > 0.0f) || !std::isfinite(g->n_rel))
    return fail(ctx, RW_E_INVALID, "n_rel must be finite and > 0");
  if (!(g->r_min_mm > 0.0f) || !std::isfinite(g->r_max_mm) || !(g->r_max_mm > g->r_min_mm))
    return fail(ctx, RW_E_INVALID, "need 0 < r_min_mm < r_max_mm < inf");
  if (!std::isfinite(g->slab_mm)) return fail(ctx, RW_E_INVALID, "slab_mm must be finite");
  if (!std::isfinite(g->rr_weight)) return fail(ctx, RW_E_INVALID, "rr_weight must be finite");
  if (g->rr_weight > 0.0f && !(g->rr_survive > 0.0f && g->rr_survive <= 1.0f))
    return fail(ctx, RW_E_INVALID, "rr_survive must be in (0, 1]");
  if (g->max_vertices < 1 || g->max_vertices > (int64_t(1) << 31))
    return fail(ctx, RW_E_INVALID, "max_vertices must be in [1, 2^31]");
  if (g->incidence != RW_INCIDENCE_NORMAL && g->incidence != RW_INCIDENCE_COSINE)
    return fail(ctx, RW_E_INVALID, "incidence must be RW_INCIDENCE_NORMAL or RW_INCIDENCE_COSINE");
  return RW_OK;
}

// Indices of the two-layer walk: bottom layer n_bot over the outside, the
// interface n_rel / n_bot seen from the top and n_bot / n_rel from the bottom.
void set_bottom_index(WalkGeom& w, float n_bot) {
  w.n_bot = n_bot;
  w.n_bot2 = n_bot * n_bot;
  w.bot_matched = n_bot == 1.0f;
  w.interface_matched = n_bot == w.n_rel;
  w.rel_down = float(double(w.n_rel) / double(n_bot));
  w.rel_down2 = w.rel_down * w.rel_down;
  w.rel_up = float(double(n_bot) / double(w.n_rel));
  w.rel_up2 = w.rel_up * w.rel_up;
}

WalkGeom make_geom(const rw_geometry* g) {
  WalkGeom w{};
  w.n_bins = g->n_bins;
  w.index_matched = g->n_rel == 1.0f;
  w.slab = g->slab_mm > 0.0f;
  w.n_rel = g->n_rel;
  w.n_rel2 = g->n_rel * g->n_rel;
  const double n = g->n_rel;
  const double F0 = ((n - 1.0) / (n + 1.0)) * ((n - 1.0) / (n + 1.0));
  w.entry_weight = float(1.0 - F0);
  w.slab_mm = g->slab_mm > 0.0f ? g->slab_mm : 0.0f;
  w.z_bottom = w.slab ? w.slab_mm : std::numeric_limits<float>::infinity();
  w.r_min = g->r_min_mm;
  w.r_max = g->r_max_mm;
  w.log2_rmin = float(std::log2(double(g->r_min_mm)));
  w.bin_scale = float(double(g->n_bins) / std::log2(double(g->r_max_mm) / double(g->r_min_mm)));
  w.rr_weight = g->rr_weight > 0.0f ? g->rr_weight : 0.0f;
  w.rr_survive = g->rr_weight > 0.0f ? g->rr_survive : 1.0f;
  w.rr_boost = float(1.0 / double(w.rr_survive));
  w.max_vertices = uint32_t(std::min<int64_t>(g->max_vertices, int64_t(0xFFFFFFFFu)));
  w.incidence = g->incidence;
  set_bottom_index(w, g->n_rel);  // one medium: no interface, same index below
  return w;
}

rw_status check_media(rw_context* ctx, const rw_media* m, int64_t* n_units) {
  if (!m) return fail(ctx, RW_E_INVALID, "media is NULL");
  if (!m->sigma_t || !m->albedo || !m->g || !m->weight)
    return fail(ctx, RW_E_INVALID, "a media parameter pointer is NULL");
  if (m->n_sets < 0 || m->n_wl < 0) return fail(ctx, RW_E_INVALID, "n_sets and n_wl must be >= 0");
  if (m->n_wl > 0 && m->n_sets > (int64_t(1) << 40) / m->n_wl)
    return fail(ctx, RW_E_INVALID, "too many units");
  *n_units = m->n_sets * m->n_wl;
  if (*n_units > (int64_t(1) << 32))
    return fail(ctx, RW_E_UNSUPPORTED, "more than 2^32 units per call");
  if (m->k_stride != 0 && m->k_stride < *n_units)
    return fail(ctx, RW_E_INVALID, "k_stride (%lld) < n_units (%lld)", (long long)m->k_stride,
                (long long)*n_units);
  return RW_OK;
}

// What a walk call reads of its media: the K-media mixture (rw_media) or the
// two-layer tissue (rw_layers), with the model id of the launch switches.
struct MediaView {
  const float* sigma_t = nullptr;
  const float* albedo = nullptr;
  const float* g = nullptr;
  const float* weight = nullptr;
  const float* layer_d = nullptr;
  int32_t logits = 0;
  int64_t k_stride = 0;
  int64_t unit_base = 0;
  int model = 0;          // K of the mixture, or kLayeredModel
  float n_bottom = 1.0f;  // two layers: the bottom layer's index
};

MediaView view_of(const rw_media* m, const rw_geometry* geom, int64_t n_units) {
  MediaView v;
  v.sigma_t = m->sigma_t;
  v.albedo = m->albedo;
  v.g = m->g;
  v.weight = m->weight;
  v.logits = m->weights_are_logits ? 1 : 0;
  v.k_stride = m->k_stride ? m->k_stride : n_units;
  v.unit_base = m->unit_base;
  v.model = geom->n_media;
  return v;
}

rw_status check_layers(rw_context* ctx, const rw_layers* l, const rw_geometry* geom,
                       MediaView* v) {
  if (!l) return fail(ctx, RW_E_INVALID, "layers is NULL");
  if (!l->sigma_t || !l->albedo || !l->g || !l->thickness_mm)
    return fail(ctx, RW_E_INVALID, "a layer parameter pointer is NULL");
  if (geom->n_media != 2)
    return fail(ctx, RW_E_INVALID, "the two-layer walk needs n_media = 2 (got %d)", geom->n_media);
  if (!(l->n_rel_bottom > 0.0f) || !(l->n_rel_bottom < 1e30f))
    return fail(ctx, RW_E_INVALID, "n_rel_bottom must be a positive finite index");
  if (l->n_units < 0) return fail(ctx, RW_E_INVALID, "n_units must be >= 0");
  if (l->n_units > (int64_t(1) << 32))
    return fail(ctx, RW_E_UNSUPPORTED, "more than 2^32 units per call");
  if (l->k_stride != 0 && l->k_stride < l->n_units)
    return fail(ctx, RW_E_INVALID, "k_stride (%lld) < n_units (%lld)", (long long)l->k_stride,
                (long long)l->n_units);
  *v = MediaView{};
  v->sigma_t = l->sigma_t;
  v->albedo = l->albedo;
  v->g = l->g;
  v->layer_d = l->thickness_mm;
  v->k_stride = l->k_stride ? l->k_stride : l->n_units;
  v->unit_base = l->unit_base;
  v->model = kLayeredModel;
  v->n_bottom = l->n_rel_bottom;
  return RW_OK;
}

rw_status need_device(rw_context* ctx) {
  if (ctx->device < 0)
    return fail(ctx, RW_E_UNSUPPORTED, "validation-only context (created with hip_device = -1)");
  RW_HIP(ctx, hipSetDevice(ctx->device));
  return RW_OK;
}

rw_status ensure_workspace(rw_context* ctx, size_t bytes) {
  if (bytes <= ctx->workspace_bytes) return RW_OK;
  if (fault_injected("alloc")) return fail(ctx, RW_E_NOMEM, "injected allocation failure");
  if (ctx->workspace) {
    // the old buffer may still be read by queued work
    RW_HIP(ctx, hipDeviceSynchronize());
    RW_HIP(ctx, hipFree(ctx->workspace));
    ctx->workspace = nullptr;
    ctx->workspace_bytes = 0;
  }
  size_t want = std::max(bytes, size_t(1) << 20);
  if (hipMalloc(&ctx->workspace, want) != hipSuccess) {
    ctx->workspace = nullptr;
    (void)hipGetLastError();
    return fail(ctx, RW_E_NOMEM, "workspace allocation of %zu bytes failed", want);
  }
  ctx->workspace_bytes = want;
  return RW_OK;
}

rw_status ensure_sched(rw_context* ctx, int64_t n_units) {
  const size_t bytes = 256 + size_t(n_units) * 8;
  if (bytes <= ctx->sched_bytes) return RW_OK;
  if (fault_injected("alloc")) return fail(ctx, RW_E_NOMEM, "injected allocation failure");
  if (ctx->sched) {
    RW_HIP(ctx, hipDeviceSynchronize());
    RW_HIP(ctx, hipFree(ctx->sched));
    ctx->sched = nullptr;
    ctx->sched_bytes = 0;
  }
  const size_t want = std::max(bytes, size_t(1) << 16);
  if (hipMalloc(&ctx->sched, want) != hipSuccess) {
    ctx->sched = nullptr;
    (void)hipGetLastError();
    return fail(ctx, RW_E_NOMEM, "schedule workspace allocation of %zu bytes failed", want);
  }
  ctx->sched_bytes = want;
  return RW_OK;
}

struct SchedPtrs {
  uint32_t* hist;
  int32_t* bucket;
  int32_t* order;
};

SchedPtrs sched_ptrs(rw_context* ctx, int64_t n_units) {
  SchedPtrs p;
  p.hist = reinterpret_cast<uint32_t*>(ctx->sched);
  p.bucket = reinterpret_cast<int32_t*>(ctx->sched + 256);
  p.order = p.bucket + n_units;
  return p;
}

// Work description shared by the four walk entry points.
struct Plan {
  WalkArgs a{};
  int K = 0;  // media count of the mixture walk, or kLayeredModel
  bool adjoint = false;
  TuneCfg cfg;
  int64_t n_window = 0;
};

int round_up(int64_t v, int64_t m) { return int((v + m - 1) / m * m); }

// Forward calls with several items per unit keep one slot of sums per item;
// max_slot_bytes bounds that workspace, and items grow (doubling, up to
// max_chunk paths) until it fits.
rw_status build_plan(rw_context* ctx, Plan& P, const MediaView& media, const rw_geometry* geom,
                     int64_t n_units, const int32_t* paths, int64_t paths_uniform, uint64_t seed,
                     int64_t ub, int64_t ue, bool adjoint, const TuneCfg& cfg,
                     int64_t max_slot_bytes = kMaxSlotBytes, int max_chunk = 1 << 30) {
  WalkArgs& a = P.a;
  a = WalkArgs{};
  a.sigma_t = media.sigma_t;
  a.albedo = media.albedo;
  a.g = media.g;
  a.weight = media.weight;
  a.layer_d = media.layer_d;
  a.weights_are_logits = media.logits;
  a.n_units_total = n_units;
  a.k_stride = media.k_stride;
  a.unit_base = uint32_t(uint64_t(media.unit_base));
  a.geo = make_geom(geom);
  if (media.model == kLayeredModel) set_bottom_index(a.geo, media.n_bottom);
  a.key0 = uint32_t(seed);
  a.key1 = uint32_t(seed >> 32);
  a.tag = kForwardTag;
  P.K = media.model;
  P.adjoint = adjoint;
  P.cfg = cfg;
  P.n_window = ue - ub;
  // chunk: at most the configured size, and no larger than the (rounded) path
  // count.  Forward calls with several items per unit keep one slot of sums
  // per item in the workspace; when that would exceed max_slot_bytes, items
  // grow (up to one item per unit, which needs no workspace at all, or to
  // max_chunk paths).
  int chunk = cfg.chunk;
  if (paths_uniform > 0 && paths_uniform < chunk) chunk = std::max(64, round_up(paths_uniform, 64));
  if (cfg.adapt) {
    // fewer items than about twice the device's resident waves (7 per SIMD):
    // halve them, down to 512 paths, so that waves done early take more work
    // instead of the last ones carrying the launch (16 units x 2^20 paths:
    // 2.57 -> 1.75 ms)
    const int64_t want = 2 * int64_t(ctx->n_cu) * 28;
    while (chunk >= 1024 && (chunk / 2) % 64 == 0 &&
           double(ue - ub) * double((paths_uniform + chunk - 1) / chunk) < double(want))
      chunk /= 2;
  }
  if (!adjoint && paths_uniform > chunk) {
    const double slot_bytes = double(forward_slot_words(geom->n_bins)) * 8.0;
    while (paths_uniform > chunk &&
           double(ue - ub) * double((paths_uniform + chunk - 1) / chunk) * slot_bytes >
               double(max_slot_bytes) &&
           chunk < max_chunk)
      chunk *= 2;
    if (paths_uniform <= chunk) chunk = std::max(64, round_up(paths_uniform, 64));
  }
  WorkMap& m = a.map;
  m.n_units = ue - ub;
  m.unit_begin = ub;
  m.paths_uniform = paths_uniform;
  m.paths = paths;
  m.chunk = chunk;
  m.chunks_per_unit = paths_uniform > 0 ? int((paths_uniform + chunk - 1) / chunk) : 0;
  m.n_items = m.n_units * int64_t(m.chunks_per_unit);
  m.unit_order = nullptr;
  m.queue = nullptr;
  if (m.n_items >= (int64_t(1) << 32))
    return fail(ctx, RW_E_UNSUPPORTED, "more than 2^32 work items (%lld) in one call",
                (long long)m.n_items);
  // fixed point of the forward sums: every per-path value (weight, squared
  // weight, absorbed weight) is below x_max, so with s = 31 - ceil(log2 x_max)
  // fraction bits it fits 32 bits, and N <= 2^31 paths keep a unit's 64-bit
  // sum below 2^63
  const double x_max = 2.0 * std::max(1.0, double(a.geo.rr_weight) * double(a.geo.rr_boost));
  const int frac_bits = 31 - int(std::ceil(std::log2(x_max)));
  a.fix_scale32 = float(std::ldexp(1.0, frac_bits));
  a.fix_cap = float(x_max * (1.0 - 0x1p-20));
  a.acc_words = adjoint ? adjoint_acc_words(adjoint_media(P.K)) : forward_acc_words(geom->n_bins);
  a.lds_words_per_wave = walk_lds_words_per_wave(a.acc_words, adjoint);
  // fewer waves per workgroup when the per-wave LDS (mostly the radial
  // histogram) would not fit a workgroup's allocation
  if (ctx->device >= 0) {
    while (P.cfg.waves_per_wg > 1 && walk_lds_bytes(a, P.cfg.waves_per_wg) > ctx->max_lds)
      P.cfg.waves_per_wg /= 2;
    if (walk_lds_bytes(a, 1) > ctx->max_lds)
      return fail(ctx, RW_E_UNSUPPORTED, "%d bins need %d bytes of LDS per wave (device: %d)",
                  geom->n_bins, walk_lds_bytes(a, 1), ctx->max_lds);
  }
  return RW_OK;
}

int occupancy_wgs(const Plan& P, int waves_per_wg) {
  int blocks = 0;
  const int lds = walk_lds_bytes(P.a, waves_per_wg);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel_ptr(P.K, P.adjoint,
                                                                   P.a.live_mask != nullptr),
                                                   waves_per_wg * kWave, lds) != hipSuccess ||
      blocks < 1) {
    (void)hipGetLastError();
    blocks = 1;
  }
  return blocks;
}

// Tally buffers of a plan.  Forward: slot sums in the workspace, [n_items]
// x ((n_bins+2)*2 + 4 + 1) int64 (bins, T/A at 2/3, vertices), reduced into the
// caller's tally; or, when every unit is one item, the caller's tally itself
// (slot = unit).  Adjoint: [n_items] x (8K) FP64 + [n_items] int64 in the
// workspace.  `clear` receives the regions to zero before the walk.
struct Region {
  uint64_t* p;
  int64_t n;
};
// the regions a launch sequence clears (at most three; no heap)
struct Regions {
  Region r[3];
  int n = 0;
  void add(uint64_t* p, int64_t count) { r[n++] = Region{p, count}; }
};

// Bytes of forward slot workspace a plan needs (0 when every unit is one item).
int64_t forward_slot_bytes(const Plan& P) {
  if (P.adjoint || P.a.map.chunks_per_unit <= 1) return 0;
  return P.a.map.n_items * int64_t(forward_slot_words(P.a.geo.n_bins)) * int64_t(sizeof(int64_t));
}

// fixed_ws: when non-NULL, the forward slots go there (the caller checked its
// size with forward_slot_bytes) instead of the context's workspace.
rw_status setup_tallies(rw_context* ctx, Plan& P, rw_tally* out, Regions& clear,
                        void* fixed_ws = nullptr) {
  WalkArgs& a = P.a;
  const int64_t ub = a.map.unit_begin;
  const int64_t nb2 = 2 * (a.geo.n_bins + 2);
  const int64_t ni = a.map.n_items;
  clear.n = 0;
  if (!P.adjoint) {
    a.out_R = out->R;
    a.out_bins = out->bins;
    a.out_vertices = out->vertices;
    a.direct = a.map.chunks_per_unit == 1 ? 1 : 0;
    if (a.direct) {
      a.tb = reinterpret_cast<int64_t*>(out->bins);
      a.tc = reinterpret_cast<int64_t*>(out->R);
      a.tv = out->vertices;
      clear.add(reinterpret_cast<uint64_t*>(a.tb + ub * nb2), P.n_window * nb2);
      clear.add(reinterpret_cast<uint64_t*>(a.tc + ub * 4), P.n_window * 4);
      clear.add(reinterpret_cast<uint64_t*>(a.tv + ub), P.n_window);
    } else {
      void* ws = fixed_ws;
      if (!ws) {
        rw_status st = ensure_workspace(ctx, size_t(forward_slot_bytes(P)));
        if (st != RW_OK) return st;
        ws = ctx->workspace;
      }
      a.tb = reinterpret_cast<int64_t*>(ws);
      a.tc = a.tb + ni * nb2;
      a.tv = a.tc + ni * 4;
      clear.add(reinterpret_cast<uint64_t*>(a.tb), ni * (nb2 + 5));
    }
  } else {
    const int km = adjoint_media(P.K);
    rw_status st = ensure_workspace(ctx, size_t(ni) * size_t(8 * km + 1) * sizeof(double));
    if (st != RW_OK) return st;
    a.adj = reinterpret_cast<double*>(ctx->workspace);
    a.adj_vertices = reinterpret_cast<int64_t*>(a.adj + ni * (8 * km));
    clear.add(reinterpret_cast<uint64_t*>(a.adj), ni * (8 * km + 1));
  }
  return RW_OK;
}

int64_t persistent_grid(rw_context* ctx, const Plan& P) {
  const int wpw = P.cfg.waves_per_wg;
  const int per_cu = P.cfg.wgs_per_cu > 0 ? P.cfg.wgs_per_cu : occupancy_wgs(P, wpw);
  return std::min<int64_t>(int64_t(ctx->n_cu) * per_cu, (P.a.map.n_items + wpw - 1) / wpw);
}

// Enqueue the launch sequence of a plan (no graph).
rw_status enqueue(rw_context* ctx, Plan& P, bool persistent, rw_tally* out, double* grad,
                  double* grad_sumsq, int64_t* adj_vertices, int32_t* flags, hipStream_t s,
                  void* fixed_ws = nullptr) {
  WalkArgs& a = P.a;
  if (fault_injected("launch")) return fail(ctx, RW_E_HIP, "injected launch failure");
  RW_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(flags), 1, 0u, s));
  a.flags = flags;
  if (P.n_window <= 0) return RW_OK;
  Regions clear;
  rw_status st0 = setup_tallies(ctx, P, out, clear, fixed_ws);
  if (st0 != RW_OK) return st0;
  for (int i = 0; i < clear.n; ++i) RW_HIP(ctx, launch_fill_u64(clear.r[i].p, clear.r[i].n, s));
  if (!P.adjoint && a.live_mask)
    RW_HIP(ctx, launch_fill_u32(a.live_mask + a.map.unit_begin * a.mask_words,
                                P.n_window * a.mask_words, 0u, s));
  if (a.map.n_items > 0) {
    const int wpw = P.cfg.waves_per_wg;
    int64_t grid;
    if (persistent) {
      a.map.queue = ctx->queue;
      RW_HIP(ctx, launch_fill_u32(ctx->queue, 1, 0u, s));
      rw_status st = ensure_sched(ctx, a.map.n_units);
      if (st != RW_OK) return st;
      const SchedPtrs sp = sched_ptrs(ctx, a.map.n_units);
      RW_HIP(ctx, launch_fill_u32(sp.hist, kOrderBuckets, 0u, s));
      RW_HIP(ctx, launch_unit_order(a, P.K, sp.bucket, sp.hist, sp.order, s));
      a.map.unit_order = sp.order;
      grid = persistent_grid(ctx, P);
    } else {
      a.map.queue = nullptr;
      grid = (a.map.n_items + wpw - 1) / wpw;
    }
    if (grid > 0x7FFFFFFF) return fail(ctx, RW_E_UNSUPPORTED, "grid too large");
    RW_HIP(ctx, launch_walk(a, P.K, P.adjoint, wpw, int(grid), s));
  }
  if (P.adjoint) {
    RW_HIP(ctx, launch_convert_adjoint(a, P.K, grad, grad_sumsq, adj_vertices, s));
  } else {
    RW_HIP(ctx, launch_convert_forward(a, s));
  }
  return RW_OK;
}

// ---- autotuner ------------------------------------------------------------
std::string tune_key(const Plan& P, bool persistent, int64_t paths_uniform, bool masked) {
  char buf[160];
  std::snprintf(buf, sizeof(buf), "gfx950 K%d %s %s nb%d p%lld m%d", P.K,
                P.adjoint ? "adj" : "fwd", persistent ? "persistent" : "static", P.a.geo.n_bins,
                (long long)std::min<int64_t>(paths_uniform, 1 << 16), masked ? 1 : 0);
  return buf;
}

void load_tune_cache(rw_context* ctx) {
  if (ctx->tune_cache_loaded) return;
  ctx->tune_cache_loaded = true;
  const char* path = std::getenv("RW_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    char* bar = std::strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    TuneCfg c;
    if (std::sscanf(bar + 1, "%d %d %d", &c.chunk, &c.waves_per_wg, &c.wgs_per_cu) == 3 &&
        c.chunk >= 64 && c.chunk % 64 == 0 && c.chunk <= (1 << 20) &&
        (c.waves_per_wg == 1 || c.waves_per_wg == 2 || c.waves_per_wg == 4) &&
        c.wgs_per_cu >= 0 && c.wgs_per_cu <= 64)
      ctx->tune[line] = c;
  }
  std::fclose(f);
}

void save_tune_cache(rw_context* ctx) {
  const char* path = std::getenv("RW_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (auto& kv : ctx->tune)
    std::fprintf(f, "%s|%d %d %d\n", kv.first.c_str(), kv.second.chunk, kv.second.waves_per_wg,
                 kv.second.wgs_per_cu);
  std::fclose(f);
}

// Time candidate shapes on a sample window of units (the real call overwrites
// every output of its window afterwards).
rw_status autotune(rw_context* ctx, Plan base, bool persistent, rw_tally* out, double* grad,
                   double* grad_sumsq, int64_t* adj_vertices, int32_t* flags, hipStream_t s,
                   TuneCfg* best) {
  const int64_t paths = base.a.map.paths_uniform;
  // sample: enough units for ~2^22 paths, at most the window
  int64_t n_sample = std::max<int64_t>(1, (int64_t(1) << 22) / std::max<int64_t>(paths, 1));
  n_sample = std::max<int64_t>(n_sample, 2 * ctx->n_cu);
  n_sample = std::min<int64_t>(n_sample, base.n_window);
  // paths per item (each lane walks chunk / 64 of them), waves per workgroup,
  // and the wave occupancy of the persistent grid as quarters of the kernel's
  // occupancy limit
  const int chunks[] = {1024, 2048, 4096, 8192};
  const int wpws[] = {1, 2, 4};
  const int occ_quarters[] = {4, 3, 2};
  hipEvent_t e0, e1;
  RW_HIP(ctx, hipEventCreate(&e0));
  RW_HIP(ctx, hipEventCreate(&e1));
  float best_ms = 1e30f;
  *best = base.cfg;
  best->adapt = false;
  for (int chunk : chunks) {
    for (int wpw : wpws) {
     for (int oq : occ_quarters) {
      Plan P = base;
      if (walk_lds_bytes(P.a, wpw) > ctx->max_lds) continue;
      P.cfg.chunk = chunk;
      P.cfg.waves_per_wg = wpw;
      P.cfg.wgs_per_cu = oq == 4 ? 0 : std::max(1, occupancy_wgs(P, wpw) * oq / 4);
      P.n_window = n_sample;
      WorkMap& m = P.a.map;
      m.n_units = n_sample;
      int c = chunk;
      if (paths > 0 && paths < c) c = std::max(64, round_up(paths, 64));
      m.chunk = c;
      m.chunks_per_unit = int((paths + c - 1) / c);
      m.n_items = m.n_units * int64_t(m.chunks_per_unit);
      float ms_sum = 0.0f;
      bool ok = true;
      for (int rep = 0; rep < 3 && ok; ++rep) {
        if (hipEventRecord(e0, s) != hipSuccess) { ok = false; break; }
        if (enqueue(ctx, P, persistent, out, grad, grad_sumsq, adj_vertices, flags, s) != RW_OK) {
          ok = false;
          break;
        }
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          ok = false;
          break;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_sum += ms;  // first repetition warms up
      }
      if (ok && ms_sum < best_ms) {
        best_ms = ms_sum;
        *best = P.cfg;
        best->adapt = false;  // a measured shape is kept as it is
      }
     }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  (void)hipGetLastError();
  return RW_OK;
}

// ---- graphs ---------------------------------------------------------------
// The batched sequence is built as an explicit graph of kernel nodes (no memset
// nodes): fill flags -> fill queue -> [fill outputs] -> walk -> [reduce].
// Topology is keyed by the kernels and launch shapes; each call updates the
// kernel arguments of the instantiated graph and launches it.
struct NodeSpec {
  const void* func;
  dim3 grid, block;
  unsigned lds;
  std::vector<std::vector<char>> args;  // argument bytes in order
};

template <class T>
std::vector<char> arg_bytes(const T& v) {
  std::vector<char> b(sizeof(T));
  std::memcpy(b.data(), &v, sizeof(T));
  return b;
}

hipKernelNodeParams node_params(const NodeSpec& spec, std::vector<void*>& ptrs) {
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(spec.func);
  kp.gridDim = spec.grid;
  kp.blockDim = spec.block;
  kp.sharedMemBytes = spec.lds;
  kp.kernelParams = ptrs.data();
  kp.extra = nullptr;
  return kp;
}

rw_status graph_launch(rw_context* ctx, const std::string& key, std::vector<NodeSpec>& specs,
                       hipStream_t s) {
  auto it = ctx->graphs.find(key);
  std::vector<std::vector<void*>> ptrs(specs.size());
  for (size_t i = 0; i < specs.size(); ++i)
    for (auto& a : specs[i].args) ptrs[i].push_back(a.data());
  if (it == ctx->graphs.end()) {
    GraphEntry ge;
    RW_HIP(ctx, hipGraphCreate(&ge.graph, 0));
    hipGraphNode_t prev = nullptr;
    for (size_t i = 0; i < specs.size(); ++i) {
      const hipKernelNodeParams kp = node_params(specs[i], ptrs[i]);
      hipGraphNode_t node;
      RW_HIP(ctx, hipGraphAddKernelNode(&node, ge.graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
      ge.nodes.push_back(node);
      ge.funcs.push_back(specs[i].func);
      prev = node;
    }
    it = ctx->graphs.emplace(key, ge).first;
  }
  GraphEntry& ge = it->second;
  // an instantiation whose last replay has finished (its arguments are no
  // longer read), else a new one while the ring has room, else the oldest,
  // after its replay
  size_t pick = ge.execs.size();
  for (size_t j = 0; j < ge.execs.size(); ++j) {
    const size_t c = (ge.oldest + j) % ge.execs.size();
    if (!ge.execs[c].launched) { pick = c; break; }
    const hipError_t q = hipEventQuery(ge.execs[c].done);
    if (q == hipSuccess) { pick = c; break; }
    if (q != hipErrorNotReady) return fail(ctx, RW_E_HIP, "hipEventQuery failed: %s",
                                           hipGetErrorString(q));
  }
  if (pick == ge.execs.size()) {
    if (ge.execs.size() < kMaxGraphExecs) {
      GraphExec gx;
      RW_HIP(ctx, hipGraphInstantiate(&gx.exec, ge.graph, nullptr, nullptr, 0));
      RW_HIP(ctx, hipEventCreateWithFlags(&gx.done, hipEventDisableTiming));
      ge.execs.push_back(gx);
    } else {
      pick = ge.oldest;
      RW_HIP(ctx, hipEventSynchronize(ge.execs[pick].done));
    }
  }
  GraphExec& gx = ge.execs[pick];
  // this call's arguments (an instantiation holds those of its last replay,
  // or of the call that built the graph)
  for (size_t i = 0; i < specs.size(); ++i) {
    const hipKernelNodeParams kp = node_params(specs[i], ptrs[i]);
    RW_HIP(ctx, hipGraphExecKernelNodeSetParams(gx.exec, ge.nodes[i], &kp));
  }
  RW_HIP(ctx, hipGraphLaunch(gx.exec, s));
  RW_HIP(ctx, hipEventRecord(gx.done, s));
  gx.launched = true;
  ge.oldest = (pick + 1) % ge.execs.size();
  return RW_OK;
}

rw_status enqueue_graph(rw_context* ctx, Plan& P, rw_tally* out, double* grad, double* grad_sumsq,
                        int64_t* adj_vertices, int32_t* flags, hipStream_t s) {
  WalkArgs& a = P.a;
  a.flags = flags;
  if (P.n_window <= 0 || a.map.n_items == 0)
    return enqueue(ctx, P, true, out, grad, grad_sumsq, adj_vertices, flags, s);
  Regions clear;
  rw_status st0 = setup_tallies(ctx, P, out, clear);
  if (st0 != RW_OK) return st0;
  const int wpw = P.cfg.waves_per_wg;
  a.map.queue = ctx->queue;
  rw_status st = ensure_sched(ctx, a.map.n_units);
  if (st != RW_OK) return st;
  const SchedPtrs sp = sched_ptrs(ctx, a.map.n_units);
  a.map.unit_order = sp.order;
  const int64_t grid = persistent_grid(ctx, P);
  std::vector<NodeSpec> specs;
  uint32_t* flags_u = reinterpret_cast<uint32_t*>(flags);
  const int64_t one = 1;
  const int64_t nbuck = kOrderBuckets;
  const uint32_t zero = 0;
  const unsigned ugrid = unsigned((a.map.n_units + 255) / 256);
  auto fill64 = [&](void* p, int64_t n) {
    uint64_t* q = reinterpret_cast<uint64_t*>(p);
    int64_t g = (n + 255) / 256;
    g = std::max<int64_t>(1, std::min<int64_t>(g, 65536));
    specs.push_back({fill_u64_kernel_ptr(), dim3(unsigned(g)), dim3(256), 0,
                     {arg_bytes(q), arg_bytes(n)}});
  };
  specs.push_back({fill_u32_kernel_ptr(), dim3(1), dim3(256), 0,
                   {arg_bytes(flags_u), arg_bytes(one), arg_bytes(zero)}});
  for (int i = 0; i < clear.n; ++i) fill64(clear.r[i].p, clear.r[i].n);
  if (!P.adjoint && a.live_mask) {
    uint32_t* m0 = a.live_mask + a.map.unit_begin * a.mask_words;
    const int64_t nw = P.n_window * a.mask_words;
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>((nw + 255) / 256, 65536));
    specs.push_back({fill_u32_kernel_ptr(), dim3(unsigned(g)), dim3(256), 0,
                     {arg_bytes(m0), arg_bytes(nw), arg_bytes(zero)}});
  }
  specs.push_back({fill_u32_kernel_ptr(), dim3(1), dim3(256), 0,
                   {arg_bytes(ctx->queue), arg_bytes(one), arg_bytes(zero)}});
  specs.push_back({fill_u32_kernel_ptr(), dim3(1), dim3(256), 0,
                   {arg_bytes(sp.hist), arg_bytes(nbuck), arg_bytes(zero)}});
  specs.push_back({unit_cost_kernel_ptr(P.K), dim3(ugrid), dim3(256), 0,
                   {arg_bytes(a), arg_bytes(sp.bucket), arg_bytes(sp.hist)}});
  specs.push_back({order_scan_kernel_ptr(), dim3(1), dim3(64), 0, {arg_bytes(sp.hist)}});
  specs.push_back({order_scatter_kernel_ptr(), dim3(ugrid), dim3(256), 0,
                   {arg_bytes(a.map.n_units), arg_bytes(sp.bucket), arg_bytes(sp.hist),
                    arg_bytes(sp.order)}});
  specs.push_back({walk_kernel_ptr(P.K, P.adjoint, !P.adjoint && a.live_mask != nullptr),
                   dim3(unsigned(grid)), dim3(wpw * kWave),
                   unsigned(walk_lds_bytes(a, wpw)), {arg_bytes(a)}});
  if (P.adjoint) {
    specs.push_back({convert_adjoint_kernel_ptr(P.K), dim3(convert_blocks(a.map.n_units)),
                     dim3(kConvWords * kConvGroups), 0,
                     {arg_bytes(a), arg_bytes(grad), arg_bytes(grad_sumsq),
                      arg_bytes(adj_vertices)}});
  } else {
    specs.push_back({convert_forward_kernel_ptr(), convert_forward_grid(a.map.n_units, a.geo.n_bins),
                     dim3(kConvWords * kConvGroups), 0, {arg_bytes(a)}});
  }
  char key[200];
  std::snprintf(key, sizeof(key),
                "K%d adj%d mark%d grid%lld wpw%d lds%d units%lld direct%d nodes%zu", P.K,
                int(P.adjoint), int(!P.adjoint && a.live_mask != nullptr), (long long)grid, wpw,
                walk_lds_bytes(a, wpw), (long long)a.map.n_units, int(a.direct), specs.size());
  return graph_launch(ctx, key, specs, s);
}

// ---- shared body of the four walk entry points -----------------------------
rw_status run_walk(rw_context* ctx, const MediaView& media, int64_t n_units,
                   const rw_geometry* geom, const int32_t* paths, int64_t paths_uniform,
                   uint64_t seed, rw_tally* out, const float* cot_R, const float* cot_bins,
                   double* grad, double* grad_sumsq, int64_t* adj_vertices, int32_t* flags,
                   const rw_batch_opts* opts, bool batched, bool adjoint, void* stream) {
  rw_status st;
  if (paths_uniform < 0 || paths_uniform > (int64_t(1) << 31))
    return fail(ctx, RW_E_INVALID, "path count must be in [0, 2^31] (got %lld)",
                (long long)paths_uniform);
  if (paths && paths_uniform <= 0 && n_units > 0)
    return fail(ctx, RW_E_INVALID,
                "with a per-unit path array, paths_uniform must give the largest count (> 0)");
  if (!adjoint) {
    if (!out || !out->R || !out->bins || !out->vertices || !out->flags)
      return fail(ctx, RW_E_INVALID, "tally pointers must be non-NULL");
    flags = out->flags;
  } else {
    if (!grad) return fail(ctx, RW_E_INVALID, "grad is NULL");
    if (!flags) return fail(ctx, RW_E_INVALID, "flags is NULL");
  }
  int64_t ub = 0, ue = n_units;
  bool use_graph = false, tune = false;
  uint32_t* mask = nullptr;
  if (opts) {
    use_graph = opts->use_graph != 0;
    tune = opts->autotune != 0;
    mask = opts->path_mask;
    if (opts->unit_end > 0 || opts->unit_begin != 0) {
      ub = opts->unit_begin;
      ue = opts->unit_end > 0 ? opts->unit_end : n_units;
      if (ub < 0 || ue > n_units || ub > ue)
        return fail(ctx, RW_E_INVALID, "unit window [%lld, %lld) outside [0, %lld)", (long long)ub,
                    (long long)ue, (long long)n_units);
    }
  }
  st = need_device(ctx);
  if (st != RW_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  Plan P;
  TuneCfg cfg;
  cfg.adapt = batched;
  std::string key;
  if (batched) {
    load_tune_cache(ctx);
    // a tune-key probe plan (shape only)
    st = build_plan(ctx, P, media, geom, n_units, paths, paths_uniform, seed, ub, ue, adjoint, cfg);
    if (st != RW_OK) return st;
    key = tune_key(P, true, paths_uniform, mask != nullptr);
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) cfg = it->second;
  }
  st = build_plan(ctx, P, media, geom, n_units, paths, paths_uniform, seed, ub, ue, adjoint, cfg);
  if (st != RW_OK) return st;
  if (adjoint) {
    P.a.cot_R = cot_R;
    P.a.cot_bins = cot_bins;
  }
  P.a.live_mask = mask;
  P.a.mask_words = (paths_uniform + 31) / 32;
  if (batched && tune && ctx->tune.find(key) == ctx->tune.end() && P.a.map.n_items > 0 &&
      P.n_window > 0) {
    TuneCfg best;
    st = autotune(ctx, P, true, out, grad, grad_sumsq, adj_vertices, flags, s, &best);
    if (st != RW_OK) return st;
    ctx->tune[key] = best;
    save_tune_cache(ctx);
    st = build_plan(ctx, P, media, geom, n_units, paths, paths_uniform, seed, ub, ue, adjoint, best);
    if (st != RW_OK) return st;
    if (adjoint) {
      P.a.cot_R = cot_R;
      P.a.cot_bins = cot_bins;
    }
    P.a.live_mask = mask;
    P.a.mask_words = (paths_uniform + 31) / 32;
  }
  if (batched && use_graph)
    return enqueue_graph(ctx, P, out, grad, grad_sumsq, adj_vertices, flags, s);
  return enqueue(ctx, P, batched, out, grad, grad_sumsq, adj_vertices, flags, s);
}

rw_status lut_args(rw_context* ctx, const rw_lut* lut, const rw_lut_targets* t, int64_t n_units,
                   int32_t n_media, const float* params, LutArgs* a) {
  if (!lut || !t) return fail(ctx, RW_E_INVALID, "lut and targets must be non-NULL");
  if (!lut->R || !lut->Pd) return fail(ctx, RW_E_INVALID, "the tables must be non-NULL");
  if (lut->n_alpha < 2 || lut->n_g < 2 || lut->n_bins < 2)
    return fail(ctx, RW_E_INVALID, "tables need at least 2 points per axis");
  if (!(lut->alpha_max > 0.0f) || !(lut->g_max > 0.0f) || !(lut->r_min_mm > 0.0f) ||
      !(lut->r_max_mm > lut->r_min_mm))
    return fail(ctx, RW_E_INVALID, "need alpha_max > 0, g_max > 0 and 0 < r_min < r_max");
  if (!t->R || !t->Pd || !t->mass || !t->r_mm)
    return fail(ctx, RW_E_INVALID, "target pointers must be non-NULL");
  if (t->n_r < 1 || t->n_r > 512) return fail(ctx, RW_E_INVALID, "n_r must be in [1, 512]");
  if (n_media < 1 || n_media > kMaxMedia)
    return fail(ctx, RW_E_INVALID, "n_media must be in [1, %d]", kMaxMedia);
  if (n_units < 0 || n_units > (int64_t(1) << 31))
    return fail(ctx, RW_E_INVALID, "n_units must be in [0, 2^31]");
  if (!params) return fail(ctx, RW_E_INVALID, "params is NULL");
  *a = LutArgs{};
  a->R = lut->R;
  a->Pd = lut->Pd;
  a->n_alpha = lut->n_alpha;
  a->n_g = lut->n_g;
  a->n_bins = lut->n_bins;
  a->alpha_max = lut->alpha_max;
  a->g_max = lut->g_max;
  a->log_rmin = float(std::log(double(lut->r_min_mm)));
  a->inv_step = float(double(lut->n_bins) / std::log(double(lut->r_max_mm) / double(lut->r_min_mm)));
  a->t_R = t->R;
  a->t_Pd = t->Pd;
  a->t_mass = t->mass;
  a->r_mm = t->r_mm;
  a->n_r = t->n_r;
  a->lambda_R = t->lambda_R;
  a->min_mass = t->min_mass;
  a->shape_floor = t->shape_floor;
  if (t->shape_form != RW_LUT_SHAPE_PAPER && t->shape_form != RW_LUT_SHAPE_MIXTURE)
    return fail(ctx, RW_E_INVALID, "shape_form must be RW_LUT_SHAPE_PAPER or RW_LUT_SHAPE_MIXTURE");
  a->shape_form = t->shape_form;
  a->n_units = n_units;
  a->params = params;
  return RW_OK;
}

// argument checks of the mixture entry points, then the shared body
rw_status run_media(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                    const int32_t* paths, int64_t paths_uniform, uint64_t seed, rw_tally* out,
                    const float* cot_R, const float* cot_bins, double* grad, double* grad_sumsq,
                    int64_t* adj_vertices, int32_t* flags, const rw_batch_opts* opts, bool batched,
                    bool adjoint, void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  int64_t n_units = 0;
  st = check_media(ctx, media, &n_units);
  if (st != RW_OK) return st;
  return run_walk(ctx, view_of(media, geom, n_units), n_units, geom, paths, paths_uniform, seed,
                  out, cot_R, cot_bins, grad, grad_sumsq, adj_vertices, flags, opts, batched,
                  adjoint, stream);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* rw_version(void) { return "rwmc-gfx950 1.0"; }

const char* rw_status_string(rw_status s) {
  switch (s) {
    case RW_OK: return "RW_OK";
    case RW_E_INVALID: return "RW_E_INVALID";
    case RW_E_HIP: return "RW_E_HIP";
    case RW_E_NOMEM: return "RW_E_NOMEM";
    case RW_E_UNSUPPORTED: return "RW_E_UNSUPPORTED";
    case RW_E_DEVICE_FLAG: return "RW_E_DEVICE_FLAG";
  }
  return "RW_E_UNKNOWN";
}

rw_status rw_create(rw_context** out, int hip_device) {
  if (!out) return RW_E_INVALID;
  *out = nullptr;
  rw_context* ctx = new (std::nothrow) rw_context();
  if (!ctx) return RW_E_NOMEM;
  if (hip_device < 0) {  // validation-only context
    *out = ctx;
    return RW_OK;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device >= count) {
    (void)hipGetLastError();
    delete ctx;
    return RW_E_HIP;
  }
  ctx->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete ctx;
    return RW_E_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    delete ctx;
    return RW_E_HIP;
  }
  ctx->n_cu = prop.multiProcessorCount;
  if (hipDeviceGetAttribute(&ctx->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            hip_device) != hipSuccess ||
      ctx->max_lds <= 0) {
    delete ctx;
    return RW_E_HIP;
  }
  if (hipMalloc(&ctx->queue, 256) != hipSuccess) {
    delete ctx;
    return RW_E_NOMEM;
  }
  // the allocation-free forward's scratch: its device address on this device,
  // looked up once per device with the device current
  if (hip_device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[hip_device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        hipFree(ctx->queue);
        delete ctx;
        return RW_E_HIP;
      }
      g_scratch_ptr[hip_device] = p;
    }
    ctx->scratch = g_scratch_ptr[hip_device];
  }
  *out = ctx;
  return RW_OK;
}

rw_status rw_destroy(rw_context* ctx) {
  if (!ctx) return RW_OK;
  if (ctx->device >= 0) {
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (auto& kv : ctx->graphs) {
      for (GraphExec& gx : kv.second.execs) {
        if (gx.exec) hipGraphExecDestroy(gx.exec);
        if (gx.done) hipEventDestroy(gx.done);
      }
      if (kv.second.graph) hipGraphDestroy(kv.second.graph);
    }
    if (ctx->workspace) hipFree(ctx->workspace);
    if (ctx->sched) hipFree(ctx->sched);
    if (ctx->queue) hipFree(ctx->queue);
  }
  delete ctx;
  return RW_OK;
}

const char* rw_last_error(const rw_context* ctx) { return ctx ? ctx->last_error : ""; }

rw_status rw_forward(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                     int64_t paths_per_unit, uint64_t seed, rw_tally* out, void* stream) {
  return run_media(ctx, media, geom, nullptr, paths_per_unit, seed, out, nullptr, nullptr, nullptr,
                  nullptr, nullptr, nullptr, nullptr, false, false, stream);
}

rw_status rw_forward_noalloc(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                             int64_t paths_per_unit, uint64_t seed, rw_tally* out, void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  int64_t n_units = 0;
  st = check_media(ctx, media, &n_units);
  if (st != RW_OK) return st;
  if (paths_per_unit < 0 || paths_per_unit > (int64_t(1) << 31))
    return fail(ctx, RW_E_INVALID, "path count must be in [0, 2^31] (got %lld)",
                (long long)paths_per_unit);
  if (!out || !out->R || !out->bins || !out->vertices || !out->flags)
    return fail(ctx, RW_E_INVALID, "tally pointers must be non-NULL");
  // the plan of rw_forward, with the slot workspace bounded by the scratch
  Plan P;
  st = build_plan(ctx, P, view_of(media, geom, n_units), geom, n_units, nullptr, paths_per_unit,
                  seed, 0, n_units, false, TuneCfg{}, kNoAllocScratchBytes, kNoAllocMaxChunk);
  if (st != RW_OK) return st;
  const int64_t need = forward_slot_bytes(P);
  if (need > kNoAllocScratchBytes)
    return fail(ctx, RW_E_UNSUPPORTED,
                "rw_forward_noalloc: %lld units x %lld paths at %d bins need %lld bytes of "
                "scratch; the limit is %lld (at most %d paths per work item)",
                (long long)n_units, (long long)paths_per_unit, geom->n_bins, (long long)need,
                (long long)kNoAllocScratchBytes, kNoAllocMaxChunk);
  st = need_device(ctx);
  if (st != RW_OK) return st;
  if (!ctx->scratch)
    return fail(ctx, RW_E_UNSUPPORTED, "no scratch on device %d (device index >= %d)", ctx->device,
                kMaxDevices);
  return enqueue(ctx, P, false, out, nullptr, nullptr, nullptr, out->flags,
                 reinterpret_cast<hipStream_t>(stream), ctx->scratch);
}

rw_status rw_batch_forward(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                           const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                           rw_tally* out, const rw_batch_opts* opts, void* stream) {
  rw_batch_opts def{1, 0, 0, 0, nullptr};
  return run_media(ctx, media, geom, paths_per_unit, paths_uniform, seed, out, nullptr, nullptr,
                  nullptr, nullptr, nullptr, nullptr, opts ? opts : &def, true, false, stream);
}

rw_status rw_adjoint(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                     int64_t paths_per_unit, uint64_t seed, const float* cot_R,
                     const float* cot_bins, double* grad, double* grad_sumsq, int64_t* vertices,
                     int32_t* flags, void* stream) {
  return run_media(ctx, media, geom, nullptr, paths_per_unit, seed, nullptr, cot_R, cot_bins, grad,
                  grad_sumsq, vertices, flags, nullptr, false, true, stream);
}

rw_status rw_batch_adjoint(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                           const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                           const float* cot_R, const float* cot_bins, double* grad,
                           double* grad_sumsq, int64_t* vertices, int32_t* flags,
                           const rw_batch_opts* opts, void* stream) {
  rw_batch_opts def{1, 0, 0, 0, nullptr};
  return run_media(ctx, media, geom, paths_per_unit, paths_uniform, seed, nullptr, cot_R, cot_bins,
                  grad, grad_sumsq, vertices, flags, opts ? opts : &def, true, true, stream);
}

rw_status rw_layered_forward(rw_context* ctx, const rw_layers* layers, const rw_geometry* geom,
                             const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                             rw_tally* out, const rw_batch_opts* opts, void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  MediaView v;
  st = check_layers(ctx, layers, geom, &v);
  if (st != RW_OK) return st;
  rw_batch_opts def{1, 0, 0, 0, nullptr};
  return run_walk(ctx, v, layers->n_units, geom, paths_per_unit, paths_uniform, seed, out, nullptr,
                  nullptr, nullptr, nullptr, nullptr, nullptr, opts ? opts : &def, true, false,
                  stream);
}

rw_status rw_layered_adjoint(rw_context* ctx, const rw_layers* layers, const rw_geometry* geom,
                             const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                             const float* cot_R, const float* cot_bins, double* grad,
                             double* grad_sumsq, int64_t* vertices, int32_t* flags,
                             const rw_batch_opts* opts, void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  MediaView v;
  st = check_layers(ctx, layers, geom, &v);
  if (st != RW_OK) return st;
  rw_batch_opts def{1, 0, 0, 0, nullptr};
  return run_walk(ctx, v, layers->n_units, geom, paths_per_unit, paths_uniform, seed, nullptr,
                  cot_R, cot_bins, grad, grad_sumsq, vertices, flags, opts ? opts : &def, true,
                  true, stream);
}

rw_status rw_layered_hero_forward(rw_context* ctx, const rw_layers* layers,
                                  const rw_geometry* geom, int32_t n_hero,
                                  int64_t paths_per_group, uint64_t seed, rw_tally* out,
                                  void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  MediaView v;
  st = check_layers(ctx, layers, geom, &v);
  if (st != RW_OK) return st;
  if (!hero_group_supported(n_hero))
    return fail(ctx, RW_E_UNSUPPORTED, "hero groups of %d wavelengths are not supported "
                "(1, 2, 3, 4, 8 or 9)", n_hero);
  const int64_t n_units = layers->n_units;
  if (n_units % n_hero != 0)
    return fail(ctx, RW_E_INVALID, "n_units (%lld) is not a multiple of the group size %d",
                (long long)n_units, n_hero);
  if (paths_per_group < 0 || paths_per_group > (int64_t(1) << 31) || paths_per_group % n_hero)
    return fail(ctx, RW_E_INVALID, "paths per group must be a multiple of %d in [0, 2^31]",
                n_hero);
  if (!out || !out->R || !out->bins || !out->vertices || !out->flags)
    return fail(ctx, RW_E_INVALID, "tally pointers must be non-NULL");
  st = need_device(ctx);
  if (st != RW_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HeroArgs a{};
  a.sigma_t = v.sigma_t;
  a.albedo = v.albedo;
  a.g = v.g;
  a.layer_d = v.layer_d;
  a.k_stride = v.k_stride;
  a.unit_base = uint64_t(v.unit_base);
  a.geo = make_geom(geom);
  set_bottom_index(a.geo, v.n_bottom);
  a.key0 = uint32_t(seed);
  a.key1 = uint32_t(seed >> 32);
  a.tag = kForwardTag;
  a.n_groups = n_units / n_hero;
  a.group_begin = 0;
  a.paths_per_group = paths_per_group;
  // items of 2048 paths, grown so that the slots stay within kMaxSlotBytes
  const int64_t words = int64_t(n_hero) * (2 * (geom->n_bins + 2) + 2);
  int64_t chunk = 2048;
  while (paths_per_group > chunk &&
         a.n_groups * ((paths_per_group + chunk - 1) / chunk) * words * 8 > kMaxSlotBytes)
    chunk *= 2;
  a.chunk = chunk;
  a.chunks_per_group = (paths_per_group + chunk - 1) / chunk;
  a.n_items = a.n_groups * a.chunks_per_group;
  // each contribution is at most C times a weight below x_max: 32-bit fixed
  // point with s = 31 - ceil(log2(C x_max)) fraction bits
  const double x_max = 2.0 * double(n_hero) *
                       std::max(1.0, double(a.geo.rr_weight) * double(a.geo.rr_boost));
  a.fix_scale32 = float(std::ldexp(1.0, 31 - int(std::ceil(std::log2(x_max)))));
  a.fix_cap = float(x_max * (1.0 - 0x1p-20));
  a.out_R = out->R;
  a.out_bins = out->bins;
  a.out_vertices = out->vertices;
  a.flags = out->flags;
  RW_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(out->flags), 1, 0u, s));
  if (a.n_items > 0) {
    st = ensure_workspace(ctx, size_t(a.n_items * words * 8));
    if (st != RW_OK) return st;
    a.slots = ctx->workspace;
    RW_HIP(ctx, launch_fill_u64(reinterpret_cast<uint64_t*>(a.slots), a.n_items * words, s));
  }
  RW_HIP(ctx, launch_hero(a, n_hero, s));
  return RW_OK;
}

rw_status rw_dwivedi_forward(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                             int64_t paths_per_unit, uint64_t seed, float q, rw_tally* out,
                             void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  int64_t n_units = 0;
  st = check_media(ctx, media, &n_units);
  if (st != RW_OK) return st;
  if (!(q > 0.0f) || !(q <= 1.0f))
    return fail(ctx, RW_E_INVALID, "the Dwivedi technique probability q must be in (0, 1]");
  if (geom->incidence != RW_INCIDENCE_NORMAL)
    return fail(ctx, RW_E_UNSUPPORTED, "the Dwivedi walk supports normal incidence only");
  if (paths_per_unit < 0 || paths_per_unit > (int64_t(1) << 31))
    return fail(ctx, RW_E_INVALID, "path count must be in [0, 2^31] (got %lld)",
                (long long)paths_per_unit);
  if (!out || !out->R || !out->bins || !out->vertices || !out->flags)
    return fail(ctx, RW_E_INVALID, "tally pointers must be non-NULL");
  st = need_device(ctx);
  if (st != RW_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const MediaView v = view_of(media, geom, n_units);
  DwivediArgs a{};
  a.w.sigma_t = v.sigma_t;
  a.w.albedo = v.albedo;
  a.w.g = v.g;
  a.w.weight = v.weight;
  a.w.weights_are_logits = v.logits;
  a.w.k_stride = v.k_stride;
  a.w.unit_base = uint32_t(v.unit_base);
  a.w.n_units_total = n_units;
  a.w.geo = make_geom(geom);
  a.w.map.paths_uniform = paths_per_unit;
  a.w.key0 = uint32_t(seed);
  a.w.key1 = uint32_t(seed >> 32);
  a.w.tag = kForwardTag;
  a.w.out_R = out->R;
  a.w.out_bins = out->bins;
  a.w.out_vertices = out->vertices;
  a.w.flags = out->flags;
  a.q = q;
  a.n_units = n_units;
  // items of 2048 paths; halved (down to 512) while there are fewer items than
  // about twice the device's resident waves, so that waves ending early make
  // room for others instead of leaving the last round to the slowest items
  // (16 units x 2^20 paths: 1.93 -> 1.66 ms); grown so that the slots stay
  // within kMaxSlotBytes
  const int64_t words = dwivedi_slot_words(geom->n_bins);
  int64_t chunk = 2048;
  const int64_t want_items = 2 * int64_t(ctx->n_cu) * 32;
  while (chunk > 512 && n_units * ((paths_per_unit + chunk - 1) / chunk) < want_items) chunk /= 2;
  while (paths_per_unit > chunk &&
         n_units * ((paths_per_unit + chunk - 1) / chunk) * words * 8 > kMaxSlotBytes)
    chunk *= 2;
  a.chunk = chunk;
  a.chunks_per_unit = paths_per_unit > 0 ? (paths_per_unit + chunk - 1) / chunk : 0;
  a.n_items = n_units * a.chunks_per_unit;
  RW_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(out->flags), 1, 0u, s));
  if (a.n_items > 0) {
    const size_t slot_bytes = (size_t(a.n_items * words * 8) + 15) & ~size_t(15);
    st = ensure_workspace(ctx, slot_bytes + size_t(n_units) * geom->n_media * 16);
    if (st != RW_OK) return st;
    a.slots = reinterpret_cast<double*>(ctx->workspace);
    a.nu = reinterpret_cast<float*>(reinterpret_cast<char*>(ctx->workspace) + slot_bytes);
  } else if (n_units > 0) {
    // no paths: zero tallies
    RW_HIP(ctx, launch_fill_u64(reinterpret_cast<uint64_t*>(out->R), n_units * 4, s));
    RW_HIP(ctx, launch_fill_u64(reinterpret_cast<uint64_t*>(out->bins),
                                n_units * 2 * (geom->n_bins + 2), s));
    RW_HIP(ctx, launch_fill_u64(reinterpret_cast<uint64_t*>(out->vertices), n_units, s));
    return RW_OK;
  }
  RW_HIP(ctx, launch_dwivedi(a, geom->n_media, 4, s));
  return RW_OK;
}

rw_status rw_finalize(rw_context* ctx, const rw_geometry* geom, int64_t n_units,
                      const int32_t* paths_per_unit, int64_t paths_uniform, const rw_tally* tally,
                      double* R_mean, double* R_se, double* Rr, double* Rr_se, double* Pd,
                      void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  if (n_units < 0) return fail(ctx, RW_E_INVALID, "n_units must be >= 0");
  if (!tally || !tally->R || !tally->bins)
    return fail(ctx, RW_E_INVALID, "tally R and bins must be non-NULL");
  if (paths_uniform < 0 || paths_uniform > (int64_t(1) << 31))
    return fail(ctx, RW_E_INVALID, "paths_uniform must be in [0, 2^31]");
  if (paths_per_unit && paths_uniform <= 0 && n_units > 0)
    return fail(ctx, RW_E_INVALID,
                "with a per-unit path array, paths_uniform must give the largest count (> 0)");
  st = need_device(ctx);
  if (st != RW_OK) return st;
  RW_HIP(ctx, launch_finalize(make_geom(geom), n_units, paths_per_unit, paths_uniform, tally->R,
                              tally->bins, R_mean, R_se, Rr, Rr_se, Pd,
                              reinterpret_cast<hipStream_t>(stream)));
  return RW_OK;
}

rw_status rw_check(rw_context* ctx, const int32_t* flags, int32_t* out_flags, void* stream) {
  if (!ctx) return RW_E_INVALID;
  if (!flags) return fail(ctx, RW_E_INVALID, "flags is NULL");
  rw_status st = need_device(ctx);
  if (st != RW_OK) return st;
  int32_t h = 0;
  RW_HIP(ctx, hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  RW_HIP(ctx, hipMemcpy(&h, flags, sizeof(h), hipMemcpyDeviceToHost));
  if (out_flags) *out_flags = h;
  if (h) return fail(ctx, RW_E_DEVICE_FLAG, "device flags 0x%x", unsigned(h));
  return RW_OK;
}

rw_status rw_debug_trace(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                         const uint32_t* words, int64_t n_paths, int64_t n_blocks, uint64_t seed,
                         uint32_t unit_index, float* events, float* path_out, float* path_adj,
                         void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  int64_t n_units = 0;
  st = check_media(ctx, media, &n_units);
  if (st != RW_OK) return st;
  if (n_units != 1) return fail(ctx, RW_E_INVALID, "rw_debug_trace takes exactly one unit");
  if (n_paths < 0 || n_paths > (int64_t(1) << 24) || n_blocks < 1 || n_blocks > (int64_t(1) << 24))
    return fail(ctx, RW_E_INVALID, "n_paths in [0, 2^24] and n_blocks in [1, 2^24] required");
  if (!path_out) return fail(ctx, RW_E_INVALID, "path_out is NULL");
  st = need_device(ctx);
  if (st != RW_OK) return st;
  if (n_paths == 0) return RW_OK;
  WalkArgs a{};
  a.sigma_t = media->sigma_t;
  a.albedo = media->albedo;
  a.g = media->g;
  a.weight = media->weight;
  a.weights_are_logits = media->weights_are_logits ? 1 : 0;
  a.n_units_total = 1;
  a.k_stride = media->k_stride ? media->k_stride : 1;
  a.geo = make_geom(geom);
  a.key0 = uint32_t(seed);
  a.key1 = uint32_t(seed >> 32);
  a.tag = kForwardTag;
  RW_HIP(ctx, launch_trace(a, geom->n_media, words, n_paths, n_blocks, unit_index, events,
                           path_out, path_adj, reinterpret_cast<hipStream_t>(stream)));
  return RW_OK;
}

rw_status rw_debug_trace_layered(rw_context* ctx, const rw_layers* layers,
                                 const rw_geometry* geom, const uint32_t* words, int64_t n_paths,
                                 int64_t n_blocks, uint64_t seed, uint32_t unit_index,
                                 float* events, float* path_out, void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  rw_status st = check_geom(ctx, geom);
  if (st != RW_OK) return st;
  MediaView v;
  st = check_layers(ctx, layers, geom, &v);
  if (st != RW_OK) return st;
  if (layers->n_units != 1)
    return fail(ctx, RW_E_INVALID, "rw_debug_trace_layered takes exactly one unit");
  if (n_paths < 0 || n_paths > (int64_t(1) << 24) || n_blocks < 1 || n_blocks > (int64_t(1) << 24))
    return fail(ctx, RW_E_INVALID, "n_paths in [0, 2^24] and n_blocks in [1, 2^24] required");
  if (!path_out) return fail(ctx, RW_E_INVALID, "path_out is NULL");
  st = need_device(ctx);
  if (st != RW_OK) return st;
  if (n_paths == 0) return RW_OK;
  WalkArgs a{};
  a.sigma_t = v.sigma_t;
  a.albedo = v.albedo;
  a.g = v.g;
  a.layer_d = v.layer_d;
  a.n_units_total = 1;
  a.k_stride = v.k_stride;
  a.geo = make_geom(geom);
  set_bottom_index(a.geo, v.n_bottom);
  a.key0 = uint32_t(seed);
  a.key1 = uint32_t(seed >> 32);
  a.tag = kForwardTag;
  RW_HIP(ctx, launch_trace(a, kLayeredModel, words, n_paths, n_blocks, unit_index, events,
                           path_out, nullptr, reinterpret_cast<hipStream_t>(stream)));
  return RW_OK;
}

rw_status rw_lut_loss_grad(rw_context* ctx, const rw_lut* lut, const rw_lut_targets* targets,
                           int64_t n_units, int32_t n_media, const float* params, float* grad,
                           float* loss, void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  LutArgs a;
  rw_status st = lut_args(ctx, lut, targets, n_units, n_media, params, &a);
  if (st != RW_OK) return st;
  st = need_device(ctx);
  if (st != RW_OK) return st;
  a.grad = grad;
  a.loss = loss;
  RW_HIP(ctx, launch_lut(a, n_media, reinterpret_cast<hipStream_t>(stream)));
  return RW_OK;
}

rw_status rw_lut_fit_step(rw_context* ctx, const rw_lut* lut, const rw_lut_targets* targets,
                          int64_t n_units, int32_t n_media, float* params, float* adam_m,
                          float* adam_v, int32_t step, float lr, float* loss, void* stream) {
  if (!ctx) return RW_E_INVALID;
  ctx->last_error[0] = 0;
  LutArgs a;
  rw_status st = lut_args(ctx, lut, targets, n_units, n_media, params, &a);
  if (st != RW_OK) return st;
  if (!adam_m || !adam_v) return fail(ctx, RW_E_INVALID, "Adam moments must be non-NULL");
  if (step < 1) return fail(ctx, RW_E_INVALID, "step must be >= 1");
  if (!(lr >= 0.0f) || !(lr < 1e30f)) return fail(ctx, RW_E_INVALID, "lr must be finite and >= 0");
  st = need_device(ctx);
  if (st != RW_OK) return st;
  a.params_out = params;
  a.adam_m = adam_m;
  a.adam_v = adam_v;
  a.adam = 1;
  a.step = step;
  a.lr = lr;
  a.loss = loss;
  RW_HIP(ctx, launch_lut(a, n_media, reinterpret_cast<hipStream_t>(stream)));
  return RW_OK;
}

rw_status rw_debug_philox(rw_context* ctx, const uint32_t* ctr, uint64_t key, int64_t n,
                          uint32_t* out, void* stream) {
  if (!ctx) return RW_E_INVALID;
  if (!ctr || !out || n < 0) return fail(ctx, RW_E_INVALID, "bad arguments");
  rw_status st = need_device(ctx);
  if (st != RW_OK) return st;
  RW_HIP(ctx, launch_philox(ctr, uint32_t(key), uint32_t(key >> 32), n, out,
                            reinterpret_cast<hipStream_t>(stream)));
  return RW_OK;
}

}  // extern "C"
