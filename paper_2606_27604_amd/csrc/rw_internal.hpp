// Internal interface between the host runtime (rw_runtime.hip) and the
// kernels (rw_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rw {

constexpr int kMaxMedia = 4;
// model id of the two-layer walk in the launch switches (which otherwise take
// the media count K of the mixture walk)
constexpr int kLayeredModel = 16;
constexpr int kWave = 64;
constexpr uint32_t kForwardTag = 0;  // Philox stream tag shared by forward and adjoint replay
// LDS table of the walk kernel's current unit: per medium 8 floats, then the
// cumulative medium weights
constexpr int kMediumFloats = 8;
constexpr int kMediaTableFloats = kMediumFloats * kMaxMedia + kMaxMedia;

// Geometry and estimator constants, in the form the kernels use.
struct WalkGeom {
  int32_t n_bins;
  int32_t index_matched;  // n_rel == 1: the surface never reflects
  int32_t slab;           // 1: finite slab of thickness slab_mm
  float n_rel, n_rel2;
  float entry_weight;     // 1 - F(0)
  float slab_mm;
  float z_bottom;         // slab_mm for a slab, else +inf
  float r_min, r_max;
  float log2_rmin;        // log2(r_min)
  float bin_scale;        // n_bins / log2(r_max / r_min)
  float rr_weight, rr_survive, rr_boost;  // rr_boost = 1 / rr_survive
  uint32_t max_vertices;
  int32_t incidence;      // 1: cosine-weighted lobe at entry (else normal pencil beam)
  // two-layer walk: the bottom layer's index over the outside (its slab face),
  // the relative indices of the interface seen from the top (down) and from
  // the bottom (up), and which faces are index-matched
  float n_bot, n_bot2;
  float rel_down, rel_down2, rel_up, rel_up2;
  int32_t bot_matched, interface_matched;
};

// How work items map to (unit, path range).  Item i covers local unit
// i / chunks_per_unit and its chunk i % chunks_per_unit; a unit with fewer
// paths than the bound leaves its trailing items empty.
struct WorkMap {
  int64_t n_units;             // units covered: [unit_begin, unit_begin + n_units)
  int64_t unit_begin;
  int64_t n_items;             // n_units * chunks_per_unit
  int64_t paths_uniform;       // paths per unit, or the upper bound when paths != nullptr
  const int32_t* paths;        // device [n_units_total] or nullptr
  int32_t chunk;               // paths per item
  int32_t chunks_per_unit;     // ceil(paths_uniform / chunk)
  const int32_t* unit_order;   // optional device [n_units]: processing order of the local
                               // units (longest estimated paths first)
  uint32_t* queue;             // persistent schedule: device counter (nullptr = static grid)
};

struct WalkArgs {
  // media, SoA [K][k_stride]
  const float* sigma_t;
  const float* albedo;
  const float* g;
  const float* weight;
  const float* layer_d;        // two-layer walk: top-layer thickness [k_stride], mm
  int32_t weights_are_logits;
  int64_t k_stride;            // elements between consecutive media in the SoA arrays
  uint32_t unit_base;          // counter index of unit 0 of the call
  int64_t n_units_total;
  WalkGeom geo;
  WorkMap map;
  uint32_t key0, key1, tag;
  // forward: exact fixed-point sums (64-bit counters of 32-bit per-path
  // values), one set per slot.  A slot is the work item that opened a wave's
  // visit of a unit (the visit takes further items of the same unit until the
  // wave moves to another unit), so no two waves share one; the reduce kernel
  // sums a unit's slots and converts them to FP64.  When every unit is a single
  // item (direct), the slot is the unit and the slots are the caller's tally
  // buffers, converted in place.
  float fix_scale32;           // 2^s: one unit of weight = 2^s counts
  float fix_cap;               // per-path values are clamped below x_max (never reached)
  int32_t direct;
  int64_t* tb;                 // [slot][n_bins+2][2]
  int64_t* tc;                 // [slot][4]: T at 2, A at 3
  int64_t* tv;                 // [slot] vertices
  double* out_R;               // [n_units_total][4]
  double* out_bins;            // [n_units_total][n_bins+2][2]
  int64_t* out_vertices;       // [n_units_total]
  int32_t* flags;
  // adjoint: FP64 sums [slot][K][8] and vertex counts [slot], slot = work item
  double* adj;
  int64_t* adj_vertices;
  const float* cot_R;          // [n_units_total] or nullptr
  const float* cot_bins;       // [n_units_total][n_bins+2] or nullptr
  // live-path mask [n_units_total][mask_words], bit p of unit u = path p left
  // the top surface: the forward sets it, the adjoint replays only those
  // paths (the others add nothing to any gradient sum); nullptr: not used
  uint32_t* live_mask;
  int64_t mask_words;          // words per unit: ceil(paths_uniform / 32)
  // per-wave LDS accumulators (8-byte words)
  int32_t acc_words;
  int32_t lds_words_per_wave;
};

// per-wave LDS of the walk kernel (8-byte words): accumulators (forward:
// (x, x^2) per slot + T, A, vertices; adjoint: K media x 8 FP64 sums +
// vertices), the media table, the cold constants, the exit ring (kExitRing
// records of 16 bytes forward, 32 bytes adjoint; a power of two, >= 64).  The
// end of the walk reuses the ring for kWave vertex draws of kTailDrawFloats
// floats each, stored as arrays of one field.
constexpr int kExitRing = 64;
constexpr int kTailDrawFloats(bool adjoint) { return adjoint ? 6 : 5; }
constexpr int walk_ring_words(bool adjoint) {
  return kExitRing * (adjoint ? 4 : 2) > kWave * kTailDrawFloats(adjoint) / 2
             ? kExitRing * (adjoint ? 4 : 2)
             : kWave * kTailDrawFloats(adjoint) / 2;
}
constexpr int kMediaTableWords = (kMediaTableFloats + 1) / 2;
constexpr int kColdConstWords = 4;  // 32 bytes after the media table
// bound on the forward slot workspace of one call (bytes)
constexpr int64_t kMaxSlotBytes = int64_t(1) << 30;
inline int forward_acc_words(int n_bins) { return 2 * (n_bins + 2) + 4; }
// int64 words of one forward slot in global memory: bins, (x, x^2, T, A), vertices
inline int forward_slot_words(int n_bins) { return 2 * (n_bins + 2) + 5; }
inline int adjoint_acc_words(int K) { return 8 * K + 2; }
// media of the adjoint sums: K for the mixture, the two layers for the
// two-layer walk
inline int adjoint_media(int model) { return model == kLayeredModel ? 2 : model; }
// the masked adjoint's pick table (kWave lane indices) and window of kWave
// mask words, behind the exit ring
constexpr int kAdjExtraWords = kWave;
inline int walk_lds_words_per_wave(int acc_words, bool adjoint) {
  return acc_words + kMediaTableWords + kColdConstWords + walk_ring_words(adjoint) +
         (adjoint ? kAdjExtraWords : 0);
}

// Lookup-table fit (rw_lut.hip): tables, targets, raw parameters [4K-1][n_units]
struct LutArgs {
  const float* R;              // [n_alpha][n_g]
  const float* Pd;             // [n_alpha][n_g][n_bins]
  int32_t n_alpha, n_g, n_bins;
  float alpha_max, g_max;
  float log_rmin, inv_step;    // ln r_min, n_bins / ln(r_max / r_min)
  const float* t_R;            // [n_units]
  const float* t_Pd;           // [n_units][n_r]
  const float* t_mass;         // [n_units][n_r]
  const float* r_mm;           // [n_r]
  int32_t n_r;
  float lambda_R, min_mass, shape_floor;
  int32_t shape_form;          // RW_LUT_SHAPE_PAPER or RW_LUT_SHAPE_MIXTURE
  int64_t n_units;
  const float* params;         // read
  float* params_out;           // Adam writes here (the same array: in place)
  float* grad;                 // or nullptr
  float* loss;                 // or nullptr
  float* adam_m;
  float* adam_v;
  int32_t adam;                // 1: take an Adam step
  int32_t step;
  float lr;
};
hipError_t launch_lut(const LutArgs& a, int K, hipStream_t stream);

// Hero-wavelength two-layer walk (rw_hero.hip): units in groups of C
// consecutive units, group q drawing Philox counter (v, p, tag, unit_base + q)
// with hero member p mod C; per-item slots [n_items][C][2 (n_bins + 2) + 2]
// int64 (bins, T, vertices of the paths the member was hero of).
struct HeroArgs {
  const float* sigma_t;        // SoA [2][k_stride] (top, bottom)
  const float* albedo;
  const float* g;
  const float* layer_d;        // [k_stride] top-layer thickness
  int64_t k_stride;
  uint64_t unit_base;          // counter index of group 0
  WalkGeom geo;
  uint32_t key0, key1, tag;
  int64_t n_groups, group_begin;
  int64_t paths_per_group;
  int64_t chunk, chunks_per_group, n_items;
  float fix_scale32, fix_cap;
  void* slots;
  double* out_R;               // [n_units][4]
  double* out_bins;            // [n_units][n_bins + 2][2]
  int64_t* out_vertices;       // [n_units]
  int32_t* flags;
};
constexpr bool hero_group_supported(int C) {
  return C == 1 || C == 2 || C == 3 || C == 4 || C == 8 || C == 9;
}
hipError_t launch_hero(const HeroArgs& a, int C, hipStream_t stream);

// Dwivedi walk (rw_dwivedi.hip): the mixture walk's arguments plus the
// technique probability, the work items (unit, chunk of paths), their FP64
// slots [n_items][2 (n_bins + 2) + 4 sums + vertex count] and the per unit
// and medium constants of nu0 [n_units][K] x 4 floats
struct DwivediArgs {
  WalkArgs w;                  // media, geometry, keys, tag, unit_base, outputs, flags;
                               // w.map.paths_uniform = paths per unit
  float q;                     // probability of the Dwivedi technique, (0, 1]
  int64_t n_units, chunk, chunks_per_unit, n_items;
  double* slots;
  float* nu;
};
hipError_t launch_dwivedi(const DwivediArgs& a, int K, int waves_per_wg, hipStream_t stream);
int dwivedi_lds_bytes(int n_bins, int waves_per_wg);
int64_t dwivedi_slot_words(int n_bins);

// launchers (rw_kernels.hip); all asynchronous on `stream`
hipError_t launch_walk(const WalkArgs& a, int K, bool adjoint, int waves_per_wg, int grid_wgs,
                       hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_fill_u64(uint64_t* p, int64_t n, hipStream_t stream);
// forward: sum each unit's int64 fixed-point slots -> FP64 outputs.  The
// convert kernels use blocks of kConvWords words x kConvGroups slot groups and
// loop over units with a grid stride.
constexpr int kConvWords = 64;
constexpr int kConvGroups = 4;
inline unsigned convert_blocks(int64_t n_units) {
  return unsigned(n_units < (int64_t(1) << 20) ? n_units : (int64_t(1) << 20));
}
inline dim3 convert_forward_grid(int64_t n_units, int n_bins) {
  const int words = 2 * (n_bins + 2) + 5;
  const int64_t rows = (words + kConvWords - 1) / kConvWords;
  const int64_t cap = (int64_t(1) << 22) / rows;
  return dim3(unsigned(n_units < cap ? n_units : cap), unsigned(rows));
}
hipError_t launch_convert_forward(const WalkArgs& a, hipStream_t stream);
// adjoint: FP64 sums -> gradients (and sums of squares), logits from the weights
hipError_t launch_convert_adjoint(const WalkArgs& a, int K, double* grad, double* grad_sumsq,
                                  int64_t* vertices_out, hipStream_t stream);
hipError_t launch_finalize(const WalkGeom& geo, int64_t n_units, const int32_t* paths,
                           int64_t paths_uniform, const double* R, const double* bins,
                           double* R_mean, double* R_se, double* Rr, double* Rr_se, double* Pd,
                           hipStream_t stream);
hipError_t launch_trace(const WalkArgs& a, int K, const uint32_t* words, int64_t n_paths,
                        int64_t n_blocks, uint32_t unit_index, float* events, float* path_out,
                        float* path_adj, hipStream_t stream);
hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                         hipStream_t stream);

// longest-first unit order for the persistent schedule: bucket[n_units] and
// unit_order[n_units] int32, hist[kOrderBuckets] uint32 (cleared by the caller)
constexpr int kOrderBuckets = 64;
hipError_t launch_unit_order(const WalkArgs& a, int K, int32_t* bucket, uint32_t* hist,
                             int32_t* unit_order, hipStream_t stream);

// kernel entry points, for graph nodes
// the walk instantiation of a launch: adjoint, or forward with (mark) or
// without the live-path mask
const void* walk_kernel_ptr(int K, bool adjoint, bool mark);
const void* fill_u32_kernel_ptr();
const void* fill_u64_kernel_ptr();
const void* unit_cost_kernel_ptr(int K);
const void* order_scan_kernel_ptr();
const void* order_scatter_kernel_ptr();
const void* convert_forward_kernel_ptr();
const void* convert_adjoint_kernel_ptr(int K);
int walk_lds_bytes(const WalkArgs& a, int waves_per_wg);

}  // namespace rw
