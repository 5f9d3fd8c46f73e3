// Internal interface between the host runtime (rw_runtime.hip) and the
// kernels (rw_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rw {

constexpr int kMaxMedia = 4;
constexpr int kWave = 64;
constexpr uint32_t kForwardTag = 0;  // Philox stream tag shared by forward and adjoint replay

// Geometry and estimator constants, in the form the kernels use.
struct WalkGeom {
  int32_t n_bins;
  int32_t index_matched;  // n_rel == 1: the surface never reflects
  int32_t slab;           // 1: finite slab of thickness slab_mm
  float n_rel, n_rel2;
  float entry_weight;     // 1 - F(0)
  float slab_mm;
  float r_min, r_max;
  float log2_rmin;        // log2(r_min)
  float bin_scale;        // n_bins / log2(r_max / r_min)
  float rr_weight, rr_survive, rr_boost;  // rr_boost = 1 / rr_survive
  uint32_t max_vertices;
};

// How work items map to (unit, path range).  Item i covers unit
// unit_begin + i / chunks_per_unit and its chunk i % chunks_per_unit; a unit
// with fewer paths than the bound leaves its trailing items empty.
struct WorkMap {
  int64_t n_units;             // units covered: [unit_begin, unit_begin + n_units)
  int64_t unit_begin;
  int64_t n_items;             // n_units * chunks_per_unit
  int64_t paths_uniform;       // paths per unit, or the upper bound when paths != nullptr
  const int32_t* paths;        // device [n_units_total] or nullptr
  int32_t chunk;               // paths per item
  int32_t chunks_per_unit;     // ceil(paths_uniform / chunk)
  const int32_t* order;        // optional device [n_items] processing order
  uint32_t* queue;             // persistent schedule: device counter (nullptr = static grid)
};

struct WalkArgs {
  // media, SoA [K][n_units_total]
  const float* sigma_t;
  const float* albedo;
  const float* g;
  const float* weight;
  int32_t weights_are_logits;
  int64_t k_stride;            // elements between consecutive media in the SoA arrays
  int64_t n_units_total;
  WalkGeom geo;
  WorkMap map;
  uint32_t key0, key1, tag;
  // forward outputs: per-item partials (deterministic) or direct/atomic outputs
  double* partial;             // [n_items][part_len] (reduce mode) or nullptr
  int32_t part_len;
  int32_t direct;              // 1: one item per unit, write outputs directly
  int32_t atomic;              // 1: accumulate into zero-filled outputs with device atomics
  double* R;                   // [n_units_total][4]
  double* bins;                // [n_units_total][n_bins+2][2]
  int64_t* vertices;           // [n_units_total]
  int32_t* flags;
  // adjoint inputs
  const float* cot_R;          // [n_units_total] or nullptr
  const float* cot_bins;       // [n_units_total][n_bins+2] or nullptr
  int32_t lds_doubles_per_wave;
};

// forward partial layout: [0..3] R sums, [4] vertices, [5..] bins (n_bins+2)*2
inline int forward_part_len(int n_bins) { return 5 + (n_bins + 2) * 2; }
// adjoint partial layout: [K][8] = (C, Q, Ss, Ss2, Sa, Sa2, Sg, Sg2), then vertices
inline int adjoint_part_len(int K) { return K * 8 + 1; }

// launchers (rw_kernels.hip); all asynchronous on `stream`
hipError_t launch_walk(const WalkArgs& a, int K, bool adjoint, int waves_per_wg, int grid_wgs,
                       hipStream_t stream);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t stream);
hipError_t launch_fill_i64(int64_t* p, int64_t n, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_reduce_forward(const WalkArgs& a, hipStream_t stream);
hipError_t launch_reduce_adjoint(const WalkArgs& a, int K, double* grad, double* grad_sumsq,
                                 hipStream_t stream);
const void* walk_kernel_ptr(int K, bool adjoint);
const void* fill_u32_kernel_ptr();
const void* reduce_forward_kernel_ptr();
const void* reduce_adjoint_kernel_ptr(int K);
int walk_lds_bytes(const WalkArgs& a, int waves_per_wg);
hipError_t launch_finalize(const WalkGeom& geo, int64_t n_units, const int32_t* paths,
                           int64_t paths_uniform, const double* R, const double* bins,
                           double* R_mean, double* R_se, double* Rr, double* Rr_se, double* Pd,
                           hipStream_t stream);
hipError_t launch_trace(const WalkArgs& a, int K, const uint32_t* words, int64_t n_paths,
                        int64_t n_blocks, uint32_t unit_index, float* events, float* path_out,
                        float* path_adj, hipStream_t stream);
hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                         hipStream_t stream);

}  // namespace rw
