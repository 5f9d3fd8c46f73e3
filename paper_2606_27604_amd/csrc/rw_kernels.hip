// HIP kernels of the random walk for gfx950 and their launchers.
//
// Work decomposition: a work item is (unit, chunk of consecutive path indices)
// and is processed by ONE wavefront.  Lanes regenerate: a lane whose path
// ended takes the next path index of the chunk (ballot + mbcnt, no atomics),
// so a wave stays full until its chunk runs dry.  Each loop iteration draws one
// Philox block per lane and processes one vertex.  Tallies: per-lane FP64
// registers for the totals, a per-wave FP64 histogram in LDS (ds_add_f64) for
// the radial slots; at the end of an item the wave writes its partial sums to
// the item's slot of a workspace (or straight to the outputs when a unit is a
// single item), and a reduction kernel sums the slots of each unit in item
// order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include "../../include/rw.h"
#include "rw_device.hpp"
#include "rw_internal.hpp"

namespace rw {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// item -> (local unit, first path, end path); pb >= pe for an empty item
__device__ __forceinline__ void map_item(const WorkMap& m, int64_t item, int64_t& u, int64_t& pb,
                                         int64_t& pe) {
  u = item / m.chunks_per_unit;
  const int64_t c = item - u * m.chunks_per_unit;
  int64_t n = m.paths_uniform;
  if (m.paths != nullptr) {
    const int64_t q = m.paths[m.unit_begin + u];
    n = q < 0 ? 0 : (q < n ? q : n);
  }
  pb = c * m.chunk;
  pe = pb + m.chunk;
  if (pe > n) pe = n;
}

// number of non-empty items of a unit
__device__ __forceinline__ int64_t unit_items(const WorkMap& m, int64_t ul) {
  int64_t n = m.paths_uniform;
  if (m.paths != nullptr) {
    const int64_t q = m.paths[m.unit_begin + ul];
    n = q < 0 ? 0 : (q < n ? q : n);
  }
  return (n + m.chunk - 1) / m.chunk;
}

// One work item: paths [pb, pe) of unit u, processed by the calling wave.
template <int K, bool ADJ>
__device__ void walk_item(const WalkArgs& a, const PhiloxKey& ks, int64_t u, int64_t pb, int64_t pe,
                          int64_t item, double* wl, int lane) {
  if (pb >= pe && !a.direct) return;  // empty trailing item: the reduction skips it
  const UnitParams<K> up = load_unit<K>(a, u);
  const WalkGeom& geo = a.geo;
  if (!up.ok) {
    if (lane == 0) atomicOr(a.flags, RW_FLAG_BAD_PARAMS);
    pe = pb;
  }
  float cotR = 0.0f;
  const float* cotB = nullptr;
  if (ADJ) {
    if (a.cot_R) cotR = a.cot_R[u];
    if (a.cot_bins) cotB = a.cot_bins + u * int64_t(geo.n_bins + 2);
  }
  double sx = 0.0, sx2 = 0.0, sT = 0.0, sA = 0.0;
  uint32_t nv = 0;
  bool capped = false;
  Path p;
  bool alive = false;
  uint32_t path = 0, v = 0;
  int64_t cursor = pb;
  for (;;) {
    const uint64_t need = __ballot(!alive);
    if (need) {
      if (!alive) {
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi(uint32_t(need >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(need), 0u));
        const int64_t cand = cursor + rank;
        if (cand < pe) {
          path = uint32_t(cand);
          v = 0;
          alive = true;
        }
      }
      cursor += __popcll(need);
    }
    if (!__any(alive)) break;
    if (alive) {
      const uint4 w = philox(v, path, uint32_t(u), a.tag, ks);
      if (v == 0) {
        start_path<K>(p, w, up, geo);
      } else {
        ++nv;
        const int ev = vertex_step<ADJ>(p, w, geo);
        if (ev >= EV_EXIT_TOP) {
          alive = false;
          sA += double(p.A);
          if (ev == EV_EXIT_TOP) {
            const int slot = radial_slot(p.x, p.y, geo);
            const double x = double(p.W);
            if (!ADJ) {
              sx += x;
              sx2 += x * x;
              atomicAdd(&wl[2 * slot], x);
              atomicAdd(&wl[2 * slot + 1], x * x);
            } else {
              const double c = x * double(cotR + (cotB ? cotB[slot] : 0.0f));
              if (c != 0.0) {
                const float nc = float(p.ncoll);
                const double ss = double(p.D);
                const double sa = p.ncoll ? double(nc / p.m.alb) : 0.0;
                const double sg = double(fmaf(nc, p.m.gc, p.Sg));
                double* acc = wl + 8 * p.k;
                atomicAdd(&acc[0], c);
                atomicAdd(&acc[1], c * c);
                atomicAdd(&acc[2], c * ss);
                atomicAdd(&acc[3], (c * ss) * (c * ss));
                atomicAdd(&acc[4], c * sa);
                atomicAdd(&acc[5], (c * sa) * (c * sa));
                atomicAdd(&acc[6], c * sg);
                atomicAdd(&acc[7], (c * sg) * (c * sg));
              }
            }
          } else if (ev == EV_EXIT_BOTTOM) {
            sT += double(p.W);
          }
        }
      }
      ++v;
      if (alive && v > geo.max_vertices) {
        alive = false;
        capped = true;
        sA += double(p.A);
      }
    }
  }
  if (__any(capped) && lane == 0) atomicOr(a.flags, RW_FLAG_VERTEX_CAP);

  // flush: per-wave sums -> item slot (or the unit's outputs)
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const uint64_t nvt = wave_sum_u64(uint64_t(nv));
  const int nd = a.lds_doubles_per_wave;
  if (!ADJ) {
    sx = wave_sum(sx);
    sx2 = wave_sum(sx2);
    sT = wave_sum(sT);
    sA = wave_sum(sA);
    if (a.direct || a.atomic) {
      double* R = a.R + u * 4;
      double* B = a.bins + u * int64_t(nd);
      if (a.direct) {
        if (lane == 0) {
          R[0] = sx; R[1] = sx2; R[2] = sT; R[3] = sA;
          a.vertices[u] = int64_t(nvt);
        }
        for (int i = lane; i < nd; i += kWave) {
          B[i] = wl[i];
          wl[i] = 0.0;
        }
      } else {
        if (lane == 0) {
          unsafeAtomicAdd(&R[0], sx); unsafeAtomicAdd(&R[1], sx2);
          unsafeAtomicAdd(&R[2], sT); unsafeAtomicAdd(&R[3], sA);
          atomicAdd(reinterpret_cast<unsigned long long*>(&a.vertices[u]),
                    static_cast<unsigned long long>(nvt));
        }
        for (int i = lane; i < nd; i += kWave) {
          const double t = wl[i];
          if (t != 0.0) unsafeAtomicAdd(&B[i], t);
          wl[i] = 0.0;
        }
      }
    } else {
      double* P = a.partial + item * int64_t(a.part_len);
      if (lane == 0) {
        P[0] = sx; P[1] = sx2; P[2] = sT; P[3] = sA; P[4] = double(nvt);
      }
      for (int i = lane; i < nd; i += kWave) {
        P[5 + i] = wl[i];
        wl[i] = 0.0;
      }
    }
  } else {
    double* P = a.partial + item * int64_t(a.part_len);
    for (int i = lane; i < nd; i += kWave) {
      P[i] = wl[i];
      wl[i] = 0.0;
    }
    if (lane == 0) P[nd] = double(nvt);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int K, bool ADJ>
__global__ void __launch_bounds__(256) walk_kernel(const WalkArgs a) {
  extern __shared__ double lds[];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  const int waves_per_wg = blockDim.x / kWave;
  double* wl = lds + int64_t(wid) * a.lds_doubles_per_wave;
  for (int i = lane; i < a.lds_doubles_per_wave; i += kWave) wl[i] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const PhiloxKey ks = philox_schedule(a.key0, a.key1);
  int64_t next = int64_t(blockIdx.x) * waves_per_wg + wid;
  const int64_t stride = int64_t(gridDim.x) * waves_per_wg;
  for (;;) {
    int64_t item;
    if (a.map.queue) {
      uint32_t it = 0;
      if (lane == 0) it = atomicAdd(a.map.queue, 1u);
      item = int64_t(__builtin_amdgcn_readfirstlane(it));
    } else {
      item = next;
      next += stride;
    }
    if (item >= a.map.n_items) break;
    if (a.map.order) item = a.map.order[item];
    int64_t ul, pb, pe;
    map_item(a.map, item, ul, pb, pe);
    walk_item<K, ADJ>(a, ks, a.map.unit_begin + ul, pb, pe, item, wl, lane);
  }
}

// Sum the item slots of each unit in item order.  One block per unit; the
// threads split the slot entries.
__global__ void __launch_bounds__(256) reduce_forward_kernel(const WalkArgs a) {
  const int64_t ul = blockIdx.x;
  const WorkMap& m = a.map;
  const int64_t i0 = ul * m.chunks_per_unit;
  const int64_t i1 = i0 + unit_items(m, ul);
  const int64_t u = m.unit_begin + ul;
  const int len = a.part_len;
  const int nb2 = (a.geo.n_bins + 2) * 2;
  for (int e = threadIdx.x; e < len; e += blockDim.x) {
    double s = 0.0;
    for (int64_t it = i0; it < i1; ++it) s += a.partial[it * len + e];
    if (e < 4) {
      a.R[u * 4 + e] = s;
    } else if (e == 4) {
      a.vertices[u] = int64_t(s);
    } else if (e - 5 < nb2) {
      a.bins[u * nb2 + (e - 5)] = s;
    }
  }
}

// Adjoint: per unit, sum the [K][8] slots of its items, then map the per-medium
// sums to gradients:  sigma_t_k, alpha_k, g_k directly;  logit_j = C_j - w_j C
// with sumsq (1 - w_j)^2 Q_j + w_j^2 (Q - Q_j).  One thread per unit.
template <int K>
__global__ void __launch_bounds__(256) reduce_adjoint_kernel(const WalkArgs a, double* grad,
                                                             double* grad_sumsq) {
  const int64_t ul = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const WorkMap& m = a.map;
  if (ul >= m.n_units) return;
  const int64_t i0 = ul * m.chunks_per_unit;
  const int64_t i1 = i0 + unit_items(m, ul);
  const int64_t u = m.unit_begin + ul;
  double acc[K * 8 + 1];
#pragma unroll
  for (int e = 0; e < K * 8 + 1; ++e) acc[e] = 0.0;
  for (int64_t it = i0; it < i1; ++it) {
    const double* P = a.partial + it * a.part_len;
#pragma unroll
    for (int e = 0; e < K * 8 + 1; ++e) acc[e] += P[e];
  }
  const UnitParams<K> up = load_unit<K>(a, u);
  double C = 0.0, Q = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    C += acc[8 * k + 0];
    Q += acc[8 * k + 1];
  }
  double* G = grad + u * (4 * K);
  double* S = grad_sumsq ? grad_sumsq + u * (4 * K) : nullptr;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double w = double(up.w[k]);
    G[k] = acc[8 * k + 2];
    G[K + k] = acc[8 * k + 4];
    G[2 * K + k] = acc[8 * k + 6];
    G[3 * K + k] = acc[8 * k + 0] - w * C;
    if (S) {
      S[k] = acc[8 * k + 3];
      S[K + k] = acc[8 * k + 5];
      S[2 * K + k] = acc[8 * k + 7];
      S[3 * K + k] = (1.0 - w) * (1.0 - w) * acc[8 * k + 1] + w * w * (Q - acc[8 * k + 1]);
    }
  }
  if (a.vertices) a.vertices[u] = int64_t(acc[K * 8]);
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void fill_i64_kernel(int64_t* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// eq. radsss: mean, SE, per-area radial density and normalised profile
__global__ void finalize_kernel(const WalkGeom geo, int64_t n_units, const int32_t* paths,
                                int64_t paths_uniform, const double* R, const double* bins,
                                double* R_mean, double* R_se, double* Rr, double* Rr_se,
                                double* Pd) {
  const int nb = geo.n_bins;
  const int64_t total = n_units * int64_t(nb + 1);
  const double lr = log2(double(geo.r_max) / double(geo.r_min)) / nb;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t u = t / (nb + 1);
    const int j = int(t - u * (nb + 1));  // j == nb: the unit's totals, else bin j
    const double N = double(paths ? paths[u] : paths_uniform);
    const double sx = R[u * 4 + 0], sx2 = R[u * 4 + 1];
    const double mean = N > 0 ? sx / N : 0.0;
    if (j == nb) {
      if (R_mean) R_mean[u] = mean;
      if (R_se) {
        double var = N > 1 ? (sx2 - sx * sx / N) / (N - 1.0) : 0.0;
        R_se[u] = N > 1 ? sqrt(fmax(var, 0.0) / N) : 0.0;
      }
      continue;
    }
    const double* B = bins + u * int64_t(nb + 2) * 2 + 2 * (j + 1);
    const double r0 = double(geo.r_min) * exp2(lr * j);
    const double r1 = double(geo.r_min) * exp2(lr * (j + 1));
    const double area = 3.14159265358979323846 * (r1 * r1 - r0 * r0);
    const double dens = N > 0 ? B[0] / (N * area) : 0.0;
    if (Rr) Rr[u * nb + j] = dens;
    if (Rr_se) {
      double var = N > 1 ? (B[1] - B[0] * B[0] / N) / (N - 1.0) : 0.0;
      Rr_se[u * nb + j] = N > 1 ? sqrt(fmax(var, 0.0) / N) / area : 0.0;
    }
    if (Pd) Pd[u * nb + j] = mean > 0.0 ? dens / mean : 0.0;
  }
}

// Per-path replay (tests): one thread per path, same steps as the walk kernel.
template <int K>
__global__ void trace_kernel(const WalkArgs a, const uint32_t* words, int64_t n_paths,
                             int64_t n_blocks, uint32_t unit_index, float* events, float* path_out,
                             float* path_adj) {
  const int64_t pth = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (pth >= n_paths) return;
  const PhiloxKey ks = philox_schedule(a.key0, a.key1);
  const UnitParams<K> up = load_unit<K>(a, 0);
  const WalkGeom& geo = a.geo;
  float* ev = events ? events + pth * n_blocks * 8 : nullptr;
  Path p;
  int end = 7, slot = -1;
  uint32_t nvert = 0;
  for (int64_t v = 0; v < n_blocks; ++v) {
    if (v > 0 && v > int64_t(geo.max_vertices)) {
      end = 4;
      if (ev) {
        float* e = ev + v * 8;
        e[0] = EV_CAP; e[1] = p.x; e[2] = p.y; e[3] = p.z;
        e[4] = p.ux; e[5] = p.uy; e[6] = p.uz; e[7] = p.W;
      }
      break;
    }
    uint4 w;
    if (words) {
      const uint32_t* q = words + (pth * n_blocks + v) * 4;
      w = make_uint4(q[0], q[1], q[2], q[3]);
    } else {
      w = philox(uint32_t(v), uint32_t(pth), unit_index, a.tag, ks);
    }
    int code;
    if (v == 0) {
      start_path<K>(p, w, up, geo);
      code = EV_START;
    } else {
      nvert = uint32_t(v);
      code = vertex_step<true>(p, w, geo);
    }
    if (ev) {
      float* e = ev + v * 8;
      e[0] = float(code); e[1] = p.x; e[2] = p.y; e[3] = p.z;
      e[4] = p.ux; e[5] = p.uy; e[6] = p.uz; e[7] = code == EV_RR_KILL ? 0.0f : p.W;
    }
    if (code == EV_EXIT_TOP) { end = 1; slot = radial_slot(p.x, p.y, geo); break; }
    if (code == EV_EXIT_BOTTOM) { end = 2; break; }
    if (code == EV_RR_KILL) { end = 3; break; }
  }
  float* o = path_out + pth * 8;
  o[0] = float(end);
  o[1] = float(p.k);
  o[2] = float(slot);
  o[3] = (end == 1 || end == 2) ? p.W : 0.0f;
  o[4] = end == 1 ? __builtin_amdgcn_sqrtf(fmaf(p.x, p.x, p.y * p.y)) : 0.0f;
  o[5] = float(nvert);
  o[6] = float(p.ncoll);
  o[7] = p.A;
  if (path_adj) {
    path_adj[pth * 2 + 0] = p.D;
    path_adj[pth * 2 + 1] = fmaf(float(p.ncoll), p.m.gc, p.Sg);
  }
}

__global__ void philox_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n,
                              uint32_t* out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PhiloxKey ks = philox_schedule(k0, k1);
  const uint4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], ks);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int K>
static hipError_t launch_walk_k(const WalkArgs& a, bool adjoint, int waves_per_wg, int grid,
                                hipStream_t s) {
  const size_t lds = size_t(waves_per_wg) * a.lds_doubles_per_wave * sizeof(double);
  if (adjoint)
    hipLaunchKernelGGL((walk_kernel<K, true>), dim3(grid), dim3(waves_per_wg * kWave), lds, s, a);
  else
    hipLaunchKernelGGL((walk_kernel<K, false>), dim3(grid), dim3(waves_per_wg * kWave), lds, s, a);
  return hipGetLastError();
}

int walk_lds_bytes(const WalkArgs& a, int waves_per_wg) {
  return waves_per_wg * a.lds_doubles_per_wave * int(sizeof(double));
}

const void* walk_kernel_ptr(int K, bool adjoint) {
  switch (K) {
    case 1: return adjoint ? (const void*)walk_kernel<1, true> : (const void*)walk_kernel<1, false>;
    case 2: return adjoint ? (const void*)walk_kernel<2, true> : (const void*)walk_kernel<2, false>;
    case 3: return adjoint ? (const void*)walk_kernel<3, true> : (const void*)walk_kernel<3, false>;
    case 4: return adjoint ? (const void*)walk_kernel<4, true> : (const void*)walk_kernel<4, false>;
    default: return nullptr;
  }
}

const void* fill_u32_kernel_ptr() { return (const void*)fill_u32_kernel; }
const void* reduce_forward_kernel_ptr() { return (const void*)reduce_forward_kernel; }
const void* reduce_adjoint_kernel_ptr(int K) {
  switch (K) {
    case 1: return (const void*)reduce_adjoint_kernel<1>;
    case 2: return (const void*)reduce_adjoint_kernel<2>;
    case 3: return (const void*)reduce_adjoint_kernel<3>;
    case 4: return (const void*)reduce_adjoint_kernel<4>;
    default: return nullptr;
  }
}

hipError_t launch_walk(const WalkArgs& a, int K, bool adjoint, int waves_per_wg, int grid_wgs,
                       hipStream_t stream) {
  switch (K) {
    case 1: return launch_walk_k<1>(a, adjoint, waves_per_wg, grid_wgs, stream);
    case 2: return launch_walk_k<2>(a, adjoint, waves_per_wg, grid_wgs, stream);
    case 3: return launch_walk_k<3>(a, adjoint, waves_per_wg, grid_wgs, stream);
    case 4: return launch_walk_k<4>(a, adjoint, waves_per_wg, grid_wgs, stream);
    default: return hipErrorInvalidValue;
  }
}

static int fill_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return int(g < 1 ? 1 : g);
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i64_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_reduce_forward(const WalkArgs& a, hipStream_t s) {
  if (a.map.n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_forward_kernel, dim3(unsigned(a.map.n_units)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce_adjoint(const WalkArgs& a, int K, double* grad, double* grad_sumsq,
                                 hipStream_t s) {
  if (a.map.n_units <= 0) return hipSuccess;
  const unsigned grid = unsigned((a.map.n_units + 255) / 256);
  switch (K) {
    case 1: hipLaunchKernelGGL(reduce_adjoint_kernel<1>, dim3(grid), dim3(256), 0, s, a, grad, grad_sumsq); break;
    case 2: hipLaunchKernelGGL(reduce_adjoint_kernel<2>, dim3(grid), dim3(256), 0, s, a, grad, grad_sumsq); break;
    case 3: hipLaunchKernelGGL(reduce_adjoint_kernel<3>, dim3(grid), dim3(256), 0, s, a, grad, grad_sumsq); break;
    case 4: hipLaunchKernelGGL(reduce_adjoint_kernel<4>, dim3(grid), dim3(256), 0, s, a, grad, grad_sumsq); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const WalkGeom& geo, int64_t n_units, const int32_t* paths,
                           int64_t paths_uniform, const double* R, const double* bins,
                           double* R_mean, double* R_se, double* Rr, double* Rr_se, double* Pd,
                           hipStream_t s) {
  const int64_t total = n_units * int64_t(geo.n_bins + 1);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(fill_grid(total)), dim3(256), 0, s, geo, n_units, paths,
                     paths_uniform, R, bins, R_mean, R_se, Rr, Rr_se, Pd);
  return hipGetLastError();
}

hipError_t launch_trace(const WalkArgs& a, int K, const uint32_t* words, int64_t n_paths,
                        int64_t n_blocks, uint32_t unit_index, float* events, float* path_out,
                        float* path_adj, hipStream_t s) {
  const unsigned grid = unsigned((n_paths + 63) / 64);
  switch (K) {
    case 1: hipLaunchKernelGGL(trace_kernel<1>, dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    case 2: hipLaunchKernelGGL(trace_kernel<2>, dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    case 3: hipLaunchKernelGGL(trace_kernel<3>, dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    case 4: hipLaunchKernelGGL(trace_kernel<4>, dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, ctr, k0, k1,
                     n, out);
  return hipGetLastError();
}

}  // namespace rw
