// HIP kernels of the random walk for gfx950 and their launchers.
//
// Work decomposition.  A work item is (unit, chunk of consecutive path
// indices).  A wavefront takes items one after another (a static grid takes
// one item per wave; the persistent grid pulls items from a device queue in
// longest-first unit order) and its lanes regenerate: a lane whose path ended
// takes the next path index, from the current item or, once that is used up,
// from the next item, so lanes never wait for the slowest path of an item.
// Each pass of the loop takes kStepsPerIteration vertex steps per lane, one
// Philox block per vertex.
//
// Tallies.  The forward sums are exact integers (32-bit fixed point per
// path, 64-bit counters), so they are bit-identical whatever the schedule,
// the launch shape or the order of atomics; the adjoint sums are FP64.  The
// wave's current unit accumulates in LDS, stored into a slot of global memory
// that only this wave writes when the wave moves to another unit; paths of an
// earlier unit still in flight add straight to that unit's slot.
#include <hip/hip_runtime.h>

#include "../../include/rw.h"
#include "rw_device.hpp"
#include "rw_internal.hpp"

namespace rw {

using u64 = unsigned long long;

// vertex count above which a path counts as long (priority boost)
constexpr uint32_t kLongPath = 256;
// vertex steps per pass of the walk loop's schedule (regeneration, ballots,
// exit ring): more steps spread that bookkeeping over more vertices, at the
// cost of lanes that end early in a pass idling for its remaining steps
constexpr int kStepsPerIteration = 4;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// The stream tag is Philox's third counter word and the same for every vertex
// of a launch, so the compiler hoists its first-round product out of the walk
// loop; that 64-bit value is then spilled and reloaded with v_readlane at
// every block.  An empty asm makes the tag opaque at each call: the product
// is recomputed with two scalar multiplies instead.
__device__ __forceinline__ uint32_t opaque_tag(uint32_t tag) {
  asm volatile("" : "+s"(tag));
  return tag;
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// Forward: a path of unit u that left the top surface sets its bit of the
// live mask.  The words of a work item belong to that item alone (items span
// whole words: their first path is a multiple of the chunk, itself a
// multiple of 64, and every unit starts on a word), and one wave runs all of
// an item's paths, so the OR needs no ordering beyond the workgroup.  The
// counters show such atomics writing through to memory, one 32-byte write
// each; the main loop therefore gathers the bits of its current item in LDS
// (live_window below) and this direct form serves only the paths that end
// after their wave moved on, and the tail.
__device__ __forceinline__ void mark_live(const WalkArgs& a, uint32_t u, uint32_t path) {
  __hip_atomic_fetch_or(a.live_mask + int64_t(u) * a.mask_words + (path >> 5), 1u << (path & 31u),
                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The live bits of the first kLiveWindow mask words of the wave's current
// work item, gathered in LDS (the part of the exit ring's area that only the
// tail's draws use) and ORed into the mask when the wave takes another item:
// one atomic per nonzero word instead of one per path that leaves the top.
// Only the wave's own paths set bits here, so the OR leaves the bits of other
// waves' items as they are.
constexpr uint32_t kLiveWindow = kWave;
constexpr uint32_t kNoUnit = 0xFFFFFFFFu;
static_assert(2 * walk_ring_words(false) >= 4 * kExitRing + int(kLiveWindow),
              "the live window must fit behind the forward exit ring");

// wave-wide: lane l ORs word wb + l of unit wu into the mask and clears it
__device__ __forceinline__ void flush_live(const WalkArgs& a, uint32_t* win, uint32_t wu,
                                           uint32_t wb, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const uint32_t bits = win[lane];
  const uint32_t w = wb + uint32_t(lane);
  if (bits != 0u && wu != kNoUnit && w < uint32_t(a.mask_words))
    __hip_atomic_fetch_or(a.live_mask + int64_t(wu) * a.mask_words + w, bits, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
  win[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
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

// next work item of the calling wave (wave-uniform), or -1 when none is left
__device__ __forceinline__ int64_t next_item(const WalkArgs& a, int64_t& static_item, int lane) {
  if (a.map.queue == nullptr) {
    const int64_t it = static_item;
    static_item = -1;
    return (it >= 0 && it < a.map.n_items) ? it : -1;
  }
  uint32_t t = 0;
  if (lane == 0) t = atomicAdd(a.map.queue, 1u);
  const int64_t k = int64_t(__builtin_amdgcn_readfirstlane(t));
  if (k >= a.map.n_items) return -1;
  if (a.map.unit_order == nullptr) return k;
  const int64_t pos = k / a.map.chunks_per_unit;
  return int64_t(a.map.unit_order[pos]) * a.map.chunks_per_unit + (k - pos * a.map.chunks_per_unit);
}

// ---- accumulation ------------------------------------------------------------
// Forward sums are exact integers: a per-path value x in [0, x_max) becomes
// round(x * 2^s) (32 bits, s = 31 - ceil(log2 x_max)) and is added to 64-bit
// counters, so a unit's sums do not depend on the order in which paths end,
// on the schedule or on the launch shape.
__device__ __forceinline__ u64 fix32(float x, float scale, float cap) {
  return u64(uint32_t(fmaf(__builtin_amdgcn_fmed3f(x, 0.0f, cap), scale, 0.5f)));
}

// In a 64-lane wave some lane ends its path in almost every iteration, so
// whatever an ending path costs inline is paid per iteration.  A path of the
// wave's current unit therefore only appends an exit record to a ring in LDS;
// once a batch of 64 records is waiting, the whole wave tallies them, one per
// lane.  Records (forward, 16 bytes): {W, A, where, vertices} with where = the
// exit radius for a top exit, -1 for a bottom exit, -2 otherwise.  Adjoint (32
// bytes): {W at a top exit else 0, radius, score_sigma, score_alpha} and
// {score_g, medium, vertices, 0}.
constexpr float kWhereBottom = -1.0f;
constexpr float kWhereNone = -2.0f;

// LDS region of one wave (8-byte words).  Forward: bins [n_bins+2][2] (sum of
// x and x^2 per slot), then the counters T, A, vertices.  Adjoint: FP64
// [K][8], then the vertex counter.  Both: then the unit's media table, the
// cold constants and the exit ring of kExitRing records.  Before a batch of
// ending paths is appended, the ring is tallied if the batch might not fit, so
// it never holds more than kExitRing records.
struct WaveLds {
  u64* acc;         // accumulators (cleared at start and at each flush)
  u64* ctr;         // wave counters inside acc
  float* media;
  ColdConst* cold;
  float4* ring;
  uint32_t* live;   // forward: the live window, behind the exit ring
  uint32_t* pick;   // adjoint: lanes of the live candidates in rank order
  uint32_t* mwin;   // adjoint: kWave consecutive words of the live mask
};

// Read from LDS where used: reads that a store in the loop may alias stay in
// place instead of being hoisted into registers for the whole loop.
__device__ __forceinline__ ColdConst read_cold(const WaveLds& L) {
  const float4* q = reinterpret_cast<const float4*>(L.cold);
  const float4 c0 = q[0], c1 = q[1];
  ColdConst c;
  c.r_min = c0.x; c.r_max = c0.y; c.log2_rmin = c0.z; c.bin_scale = c0.w;
  c.n_bins = __float_as_int(c1.x); c.entry_weight = c1.y; c.fix_scale = c1.z; c.fix_cap = c1.w;
  return c;
}

__device__ __forceinline__ float exit_where(int ev, const Path& p) {
  return ev == EV_EXIT_TOP ? exit_radius(p.x, p.y)
                           : (ev == EV_EXIT_BOTTOM ? kWhereBottom : kWhereNone);
}

// Exit records of an ending path (layout above).
__device__ __forceinline__ float4 forward_record(int ev, const Path& p, uint32_t nv) {
  return make_float4(p.W, p.A, exit_where(ev, p), __uint_as_float(nv));
}

// Adjoint scores of an ending path: c = x * (cot_R + cot_bins[slot]) with the
// per-path sigma_t, albedo and g scores of its medium.
__device__ __forceinline__ float score_alpha(const Path& p) {
  return p.ncoll ? float(p.ncoll) * __builtin_amdgcn_rcpf(p.m.alb) : 0.0f;
}
__device__ __forceinline__ float score_g(const Path& p) { return fmaf(float(p.ncoll), p.m.gc, p.Sg); }


__device__ __forceinline__ void adjoint_record(int ev, const Path& p, uint32_t nv, float4& r0,
                                               float4& r1) {
  const bool top = ev == EV_EXIT_TOP;
  r0 = make_float4(top ? p.W : 0.0f, exit_where(ev, p), p.D, score_alpha(p));
  r1 = make_float4(score_g(p), __uint_as_float(uint32_t(p.k)), __uint_as_float(nv), 0.0f);
}

// Add one record to the wave's LDS sums of the current unit.
__device__ __forceinline__ void tally_forward_record(const WaveLds& L, const ColdConst& cc,
                                                     float4 r) {
  const float sc = cc.fix_scale, cap = cc.fix_cap;
  if (r.z >= 0.0f) {
    const int slot = radial_slot_r(r.z, cc);
    atomicAdd(&L.acc[2 * slot], fix32(r.x, sc, cap));
    atomicAdd(&L.acc[2 * slot + 1], fix32(r.x * r.x, sc, cap));
  } else if (r.z == kWhereBottom) {
    atomicAdd(&L.ctr[0], fix32(r.x, sc, cap));
  }
  atomicAdd(&L.ctr[1], fix32(r.y, sc, cap));
  atomicAdd(&L.ctr[2], u64(__float_as_uint(r.w)));
}

__device__ __forceinline__ void tally_adjoint_record(const WalkArgs& a, const WaveLds& L,
                                                     uint32_t unit, float4 r0, float4 r1) {
  atomicAdd(&L.ctr[0], u64(__float_as_uint(r1.z)));
  if (r0.x > 0.0f) {
    const ColdConst cc = read_cold(L);
    const int slot = radial_slot_r(r0.y, cc);
    float cot = a.cot_R ? a.cot_R[unit] : 0.0f;
    if (a.cot_bins) cot += a.cot_bins[int64_t(unit) * (cc.n_bins + 2) + slot];
    const double c = double(r0.x) * double(cot);
    if (c != 0.0) {
      const double css = c * double(r0.z), csa = c * double(r0.w), csg = c * double(r1.x);
      double* t = reinterpret_cast<double*>(L.acc) + 8 * __float_as_uint(r1.y);
      atomicAdd(&t[0], c);
      atomicAdd(&t[1], c * c);
      atomicAdd(&t[2], css);
      atomicAdd(&t[3], css * css);
      atomicAdd(&t[4], csa);
      atomicAdd(&t[5], csa * csa);
      atomicAdd(&t[6], csg);
      atomicAdd(&t[7], csg * csg);
    }
  }
}

// Tally records [head, head + n) of the ring (n <= 64), one per lane.
__device__ __forceinline__ void tally_forward(const WaveLds& L, uint32_t head, uint32_t n,
                                              int lane) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (uint32_t(lane) < n) {
    const ColdConst cc = read_cold(L);
    tally_forward_record(L, cc, L.ring[(head + lane) & (kExitRing - 1)]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int K>
__device__ __forceinline__ void tally_adjoint(const WalkArgs& a, const WaveLds& L, uint32_t unit,
                                              uint32_t head, uint32_t n, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (uint32_t(lane) < n) {
    const uint32_t i = (head + lane) & (kExitRing - 1);
    tally_adjoint_record(a, L, unit, L.ring[2 * i], L.ring[2 * i + 1]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Path of an earlier visit (still in flight after the wave moved to another
// unit): tally straight into that visit's slot, which only this wave writes
// and which it has already flushed.
__device__ __forceinline__ void exit_global_forward(const WalkArgs& a, const WaveLds& L,
                                                    uint32_t slot, int ev, const Path& p,
                                                    uint32_t nv) {
  const ColdConst cc = read_cold(L);
  const float sc = cc.fix_scale, cap = cc.fix_cap;
  const int nb2 = 2 * (cc.n_bins + 2);
  if (ev == EV_EXIT_TOP) {
    const int b = radial_slot(p.x, p.y, cc);
    u64* B = reinterpret_cast<u64*>(a.tb + int64_t(slot) * nb2);
    const u64 q1 = fix32(p.W, sc, cap), q2 = fix32(p.W * p.W, sc, cap);
    atomicAdd(&B[2 * b], q1);
    atomicAdd(&B[2 * b + 1], q2);
    atomicAdd(reinterpret_cast<u64*>(&a.tc[int64_t(slot) * 4 + 0]), q1);
    atomicAdd(reinterpret_cast<u64*>(&a.tc[int64_t(slot) * 4 + 1]), q2);
  } else if (ev == EV_EXIT_BOTTOM) {
    atomicAdd(reinterpret_cast<u64*>(&a.tc[int64_t(slot) * 4 + 2]), fix32(p.W, sc, cap));
  }
  atomicAdd(reinterpret_cast<u64*>(&a.tc[int64_t(slot) * 4 + 3]), fix32(p.A, sc, cap));
  atomicAdd(reinterpret_cast<u64*>(&a.tv[slot]), u64(nv));
}

template <int K>
__device__ __forceinline__ void exit_global_adjoint(const WalkArgs& a, const WaveLds& L,
                                                    uint32_t slot, uint32_t unit, int ev,
                                                    const Path& p, uint32_t nv) {
  if (ev == EV_EXIT_TOP) {
    const ColdConst cc = read_cold(L);
    const int b = radial_slot(p.x, p.y, cc);
    float cot = a.cot_R ? a.cot_R[unit] : 0.0f;
    if (a.cot_bins) cot += a.cot_bins[int64_t(unit) * (cc.n_bins + 2) + b];
    const double c = double(p.W) * double(cot);
    if (c != 0.0) {
      const double css = c * double(p.D), csa = c * double(score_alpha(p)),
                   csg = c * double(score_g(p));
      double* t = a.adj + (int64_t(slot) * K + p.k) * 8;
      unsafeAtomicAdd(&t[0], c);
      unsafeAtomicAdd(&t[1], c * c);
      unsafeAtomicAdd(&t[2], css);
      unsafeAtomicAdd(&t[3], css * css);
      unsafeAtomicAdd(&t[4], csa);
      unsafeAtomicAdd(&t[5], csa * csa);
      unsafeAtomicAdd(&t[6], csg);
      unsafeAtomicAdd(&t[7], csg * csg);
    }
  }
  atomicAdd(reinterpret_cast<u64*>(&a.adj_vertices[slot]), u64(nv));
}

// Two-layer adjoint: a path scores both layers (the flights, collisions and
// scatterings it had in each), so it adds to the sums of both.  It tallies
// directly, into the wave's LDS sums when its unit is the wave's current one,
// else into its slot (no exit ring: the record would not fit 32 bytes).
__device__ __forceinline__ void layer_scores(const Path& p, int j, float& D, float& sa,
                                             float& sg) {
  const bool cur = j == p.k;
  const uint32_t n = cur ? p.ncoll : p.ncoll2;
  const float alb = cur ? p.m.alb : p.m2.alb;
  const float gc = cur ? p.m.gc : p.m2.gc;
  D = cur ? p.D : p.D2;
  sa = n ? float(n) * __builtin_amdgcn_rcpf(alb) : 0.0f;
  sg = fmaf(float(n), gc, cur ? p.Sg : p.Sg2);
}

__device__ __forceinline__ void exit_adjoint_layered(const WalkArgs& a, const WaveLds& L,
                                                     bool local, uint32_t slot, uint32_t unit,
                                                     int ev, const Path& p, uint32_t nv) {
  if (local) atomicAdd(&L.ctr[0], u64(nv));
  else atomicAdd(reinterpret_cast<u64*>(&a.adj_vertices[slot]), u64(nv));
  if (ev != EV_EXIT_TOP) return;
  const ColdConst cc = read_cold(L);
  const int b = radial_slot(p.x, p.y, cc);
  float cot = a.cot_R ? a.cot_R[unit] : 0.0f;
  if (a.cot_bins) cot += a.cot_bins[int64_t(unit) * (cc.n_bins + 2) + b];
  const double c = double(p.W) * double(cot);
  if (c == 0.0) return;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float D, sa, sg;
    layer_scores(p, j, D, sa, sg);
    const double css = c * double(D), csa = c * double(sa), csg = c * double(sg);
    if (local) {
      double* t = reinterpret_cast<double*>(L.acc) + 8 * j;
      atomicAdd(&t[0], c);
      atomicAdd(&t[1], c * c);
      atomicAdd(&t[2], css);
      atomicAdd(&t[3], css * css);
      atomicAdd(&t[4], csa);
      atomicAdd(&t[5], csa * csa);
      atomicAdd(&t[6], csg);
      atomicAdd(&t[7], csg * csg);
    } else {
      double* t = a.adj + (int64_t(slot) * 2 + j) * 8;
      unsafeAtomicAdd(&t[0], c);
      unsafeAtomicAdd(&t[1], c * c);
      unsafeAtomicAdd(&t[2], css);
      unsafeAtomicAdd(&t[3], css * css);
      unsafeAtomicAdd(&t[4], csa);
      unsafeAtomicAdd(&t[5], csa * csa);
      unsafeAtomicAdd(&t[6], csg);
      unsafeAtomicAdd(&t[7], csg * csg);
    }
  }
}

// Tally what is left in the ring, then store the wave's sums of the visit
// (unit u) into its slot and clear them.  The slot belongs to this wave alone,
// so plain stores do; paths of the visit still in flight add to it afterwards.
template <int K, bool ADJ>
__device__ __forceinline__ void flush_unit(const WalkArgs& a, const WaveLds& L, uint32_t& head,
                                           uint32_t tail, int64_t slot, int64_t u, int lane) {
  while (head != tail) {
    const uint32_t n = (tail - head) < uint32_t(kWave) ? (tail - head) : uint32_t(kWave);
    if (!ADJ) tally_forward(L, head, n, lane);
    else tally_adjoint<K>(a, L, uint32_t(u), head, n, lane);
    head += n;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (!ADJ) {
    const int nb2 = 2 * (a.geo.n_bins + 2);
    u64* B = reinterpret_cast<u64*>(a.tb + slot * nb2);
    u64 s1 = 0, s2 = 0;  // top totals: every top exit lands in one slot
    for (int i = lane; i < nb2; i += kWave) {
      const u64 x = L.acc[i];
      B[i] = x;
      if (i & 1) s2 += x; else s1 += x;
      L.acc[i] = 0ull;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1 += __shfl_xor(s1, off, kWave);
      s2 += __shfl_xor(s2, off, kWave);
    }
    if (lane == 0) {
      a.tc[slot * 4 + 0] = int64_t(s1);
      a.tc[slot * 4 + 1] = int64_t(s2);
      a.tc[slot * 4 + 2] = int64_t(L.ctr[0]);
      a.tc[slot * 4 + 3] = int64_t(L.ctr[1]);
      a.tv[slot] = int64_t(L.ctr[2]);
      L.ctr[0] = 0ull;
      L.ctr[1] = 0ull;
      L.ctr[2] = 0ull;
    }
  } else {
    double* accd = reinterpret_cast<double*>(L.acc);
    double* G = a.adj + slot * (8 * K);
    for (int m = lane; m < 8 * K; m += kWave) {
      G[m] = accd[m];
      accd[m] = 0.0;
    }
    if (lane == 0) {
      a.adj_vertices[slot] = int64_t(L.ctr[0]);
      L.ctr[0] = 0ull;
    }
  }
  // the stores land before any later add to the same slot
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// The two walk variants behind one kernel: the mixture of K media (LAYERED
// false) and the two-layer tissue (forward only).
template <int K, bool LAYERED>
__device__ __forceinline__ void start_any(Path& p, uint4 w, const float* tab, float entry_weight,
                                          const WalkGeom& geo) {
  if constexpr (LAYERED) start_path_layers(p, w, tab, entry_weight, geo);
  else start_path_lds<K>(p, w, tab, entry_weight, geo);
}

template <bool ADJ, bool LAYERED>
__device__ __forceinline__ int step_any(Path& p, uint4 w, const WalkGeom& geo) {
  if constexpr (LAYERED) return vertex_step_layered<ADJ>(p, w, geo);
  else return vertex_step<ADJ>(p, w, geo);
}

// Load, validate and stage the parameters of unit u; an invalid unit raises
// the flag and returns false.  (The flag store sits in the else branch of the
// staging: testing the returned value again at the call site cost the mixture
// kernel 11-15 VGPRs and a wave of occupancy.)
template <int K, bool LAYERED>
__device__ __forceinline__ bool stage_any(const WalkArgs& a, int64_t u, float* tab, int lane) {
  if constexpr (LAYERED) {
    const LayerParams lp = load_layers(a, u);
    if (lp.ok) stage_layers(lp, tab, lane);
    else if (lane == 0) atomicOr(a.flags, RW_FLAG_BAD_PARAMS);
    return lp.ok;
  } else {
    const UnitParams<K> up = load_unit<K>(a, u);
    if (up.ok) stage_unit<K>(up, tab, lane);
    else if (lane == 0) atomicOr(a.flags, RW_FLAG_BAD_PARAMS);
    return up.ok;
  }
}

// An empty asm statement that takes a draw's fields as register inputs: the
// draw's reads must have completed there.
template <bool ADJ>
__device__ __forceinline__ void hold_draw(const VertexDraw& d) {
  if constexpr (ADJ)
    asm volatile("" ::"v"(d.s), "v"(d.mu), "v"(d.p), "v"(d.q), "v"(d.w3), "v"(d.den));
  else
    asm volatile("" ::"v"(d.s), "v"(d.mu), "v"(d.p), "v"(d.q), "v"(d.w3));
}

// Draw i of the tail's LDS arrays (field f at dr[f * kWave + i]).
template <bool ADJ>
__device__ __forceinline__ VertexDraw load_draw(const float* dr, uint32_t i) {
  VertexDraw d;
  d.s = dr[i];
  d.mu = dr[kWave + i];
  d.p = dr[2 * kWave + i];
  d.q = dr[3 * kWave + i];
  d.w3 = __float_as_uint(dr[4 * kWave + i]);
  d.den = ADJ ? dr[5 * kWave + i] : 0.0f;
  return d;
}

// The two-layer adjoint carries both layers' scores and would take 81 VGPRs,
// i.e. 5 waves per SIMD; asking for 6 fits it in 79 without spills (7 would
// spill in the vertex loop).  The other instantiations are left to the
// compiler (7 waves at 63-74 VGPRs).  MARK: a forward that sets the live-path
// mask; its own instantiation, so that a forward without the mask carries
// none of the marking code.
template <int K, bool ADJ, bool LAYERED, bool MARK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ADJ && LAYERED ? 6 : 1)))
walk_kernel(const WalkArgs a) {
  static_assert(!(ADJ && MARK), "only the forward marks paths");
  extern __shared__ u64 lds[];
  const int lane = lane_id();
  // the wave index is uniform; say so, or every schedule value derived from it
  // is treated as divergent
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wpw = blockDim.x / kWave;
  WaveLds L;
  L.acc = lds + int64_t(wid) * a.lds_words_per_wave;
  L.ctr = L.acc + (ADJ ? 8 * K : 2 * (a.geo.n_bins + 2));
  L.media = reinterpret_cast<float*>(L.acc + a.acc_words);
  L.cold = reinterpret_cast<ColdConst*>(L.acc + a.acc_words + kMediaTableWords);
  L.ring = reinterpret_cast<float4*>(L.acc + a.acc_words + kMediaTableWords + kColdConstWords);
  L.live = MARK ? reinterpret_cast<uint32_t*>(L.ring + kExitRing) : nullptr;
  L.pick = ADJ ? reinterpret_cast<uint32_t*>(L.acc + a.acc_words + kMediaTableWords +
                                             kColdConstWords + walk_ring_words(true))
               : nullptr;
  L.mwin = ADJ ? L.pick + kWave : nullptr;
  for (int i = lane; i < a.acc_words; i += kWave) L.acc[i] = 0ull;
  if (MARK) L.live[lane] = 0u;
  if (lane == 0) {
    float4* q = reinterpret_cast<float4*>(L.cold);
    q[0] = make_float4(a.geo.r_min, a.geo.r_max, a.geo.log2_rmin, a.geo.bin_scale);
    q[1] = make_float4(__int_as_float(a.geo.n_bins), a.geo.entry_weight, a.fix_scale32, a.fix_cap);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const PhiloxKey ks = philox_schedule(a.key0, a.key1);
  WalkGeom geo = step_geom_in_vgprs(a.geo);
  if constexpr (LAYERED) {
    geo.rel_down = in_vgpr(a.geo.rel_down);
    geo.rel_down2 = in_vgpr(a.geo.rel_down2);
    geo.rel_up = in_vgpr(a.geo.rel_up);
    geo.rel_up2 = in_vgpr(a.geo.rel_up2);
    geo.n_bot = in_vgpr(a.geo.n_bot);
    geo.n_bot2 = in_vgpr(a.geo.n_bot2);
  }

  // wave-uniform schedule state: the current item's next path index and end,
  // the unit whose parameters are staged and whose sums sit in LDS, the slot
  // of this visit, the ring
  int64_t u_cur = -1, cur_slot = -1;
  uint32_t cursor = 0, pend = 0, head = 0, tail = 0, iter = 0;
  // the live window: unit and first word
  uint32_t wu = kNoUnit, wb = 0;
  // the masked adjoint's window of mask words: unit and first word
  uint32_t mu = kNoUnit, mw = 0;
  int64_t static_item = int64_t(blockIdx.x) * wpw + wid;
  bool done = false, unit_ok = false, boosted = false;
  // lane state
  Path p;
  bool alive = false, capped = false;
  uint32_t path = 0, v = 0, lunit = 0, lslot = 0, lctr = 0;

  // A look-ahead round for the lanes with `sel` set (running paths, at most
  // kWave / 2 of them, vertex >= 1), used where one path's dependent chain
  // sets the pace.  The idle lanes take off that chain what does not depend
  // on the path's state: lane l draws vertex v + (l mod d) of the (l / d)-th
  // selected path (d = 64 / selected paths, rounded to a power of two) into
  // LDS, and every selected path then takes d steps, reading one draw per
  // step.  In the mixture walk, whose medium is fixed from the start, a draw
  // is the whole VertexDraw (flight length, scattering cosine and azimuth);
  // the two-layer walk, whose medium changes at the interface, stores the
  // Philox block.  Ending paths tally directly (few lanes).  The exit ring
  // must be empty: its LDS holds the draws.
  auto lookahead_round = [&](bool sel) {
    uint4* blk = reinterpret_cast<uint4*>(L.ring);
    // draws as arrays of one field: field f of draw i at dr[f * kWave + i]
    float* dr = reinterpret_cast<float*>(L.ring);
    const uint64_t am = __ballot(sel);
    const uint32_t na = uint32_t(__popcll(am));
    const uint32_t lg = na <= 1 ? 6u : na <= 2 ? 5u : na <= 4 ? 4u : na <= 8 ? 3u
                      : na <= 16 ? 2u : na <= 32 ? 1u : 0u;
    const uint32_t rank = lane_rank(am);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (sel) {
      blk[rank] = make_uint4(path, v, lctr, __float_as_uint(p.m.flight));
      if constexpr (!LAYERED)
        blk[kWave / 2 + rank] = make_uint4(__float_as_uint(p.m.g), __float_as_uint(p.m.hq), 0u, 0u);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint32_t j = uint32_t(lane) >> lg;
    const uint32_t t = uint32_t(lane) & ((1u << lg) - 1u);
    uint4 q = make_uint4(0u, 0u, 0u, 0u), mq = q;
    if (j < na) {
      q = blk[j];
      if constexpr (!LAYERED) mq = blk[kWave / 2 + j];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (j < na) {
      const uint4 w = philox(q.y + t, q.x, opaque_tag(a.tag), q.z, ks);
      if constexpr (LAYERED) {
        blk[lane] = w;
      } else {
        const VertexDraw d = draw_vertex(__uint_as_float(q.w), __uint_as_float(mq.x),
                                         __uint_as_float(mq.y), w);
        dr[lane] = d.s;
        dr[kWave + lane] = d.mu;
        dr[2 * kWave + lane] = d.p;
        dr[3 * kWave + lane] = d.q;
        dr[4 * kWave + lane] = __uint_as_float(d.w3);
        if (ADJ) dr[5 * kWave + lane] = d.den;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint32_t depth = 1u << lg;
    // this lane's draws (a lane outside the selection reads the first ones)
    const uint32_t base = sel ? (rank << lg) : 0u;
    uint32_t s = 0;
    while (s < depth && __ballot(sel) != 0) {
      if constexpr (!LAYERED) {
        // A long path spends nearly all its vertices colliding away from the
        // surface above the roulette threshold.  While that holds for every
        // selected path, one ballot per step says so and the step runs as
        // straight-line code; the first step where it does not goes through
        // the general step below.  The straight-line step runs on every lane:
        // a lane outside the selection holds no running path (the tail calls
        // this with the running lanes), so its state is free to overwrite.
        // The vertex cap is checked once for the round.  (The next step's
        // draw is read before this step's arithmetic, so that the LDS latency
        // overlaps it.)
        const bool room = __ballot(sel && v + (depth - s) > geo.max_vertices) == 0;
        VertexDraw d = load_draw<ADJ>(dr, base + s);
        // two steps per pass, the draws alternating between d and d1, so that
        // no draw is copied from one variable to the other; each next draw is
        // held in registers by the end of the step it overlaps (else the
        // compiler defers the reads past the next test and exposes them)
        while (room && s < depth) {
          float zn;
          if (__ballot(sel & !plain_collision(p, d, geo, zn)) != 0) break;
          const VertexDraw d1 = load_draw<ADJ>(dr, base + (s + 1 < depth ? s + 1 : s));
          absorb_at<ADJ>(p, d, zn);
          scatter<ADJ>(p, d);
          ++v;
          hold_draw<ADJ>(d1);
          if (++s == depth) break;
          if (__ballot(sel & !plain_collision(p, d1, geo, zn)) != 0) break;
          d = load_draw<ADJ>(dr, base + (s + 1 < depth ? s + 1 : s));
          absorb_at<ADJ>(p, d1, zn);
          scatter<ADJ>(p, d1);
          ++v;
          ++s;
          hold_draw<ADJ>(d);
        }
        if (s == depth) break;
      }
      if (sel) {
        const uint32_t i = base + s;
        int ev;
        if constexpr (LAYERED) {
          ev = step_any<ADJ, LAYERED>(p, blk[i], geo);
        } else {
          ev = vertex_step_drawn<ADJ>(p, load_draw<ADJ>(dr, i), geo);
        }
        if (ev < EV_EXIT_TOP && v >= geo.max_vertices) {
          ev = EV_CAP;
          capped = true;
        }
        if (ev >= EV_EXIT_TOP) {
          sel = false;
          alive = false;
          if (MARK && ev == EV_EXIT_TOP) mark_live(a, lunit, path);
          if constexpr (ADJ && LAYERED) {
            exit_adjoint_layered(a, L, lslot == uint32_t(cur_slot), lslot, lunit, ev, p, v);
          } else if (lslot == uint32_t(cur_slot)) {
            if (!ADJ) {
              tally_forward_record(L, read_cold(L), forward_record(ev, p, v));
            } else {
              float4 r0, r1;
              adjoint_record(ev, p, v, r0, r1);
              tally_adjoint_record(a, L, lunit, r0, r1);
            }
          } else {
            if (!ADJ) exit_global_forward(a, L, lslot, ev, p, v);
            else exit_global_adjoint<K>(a, L, lslot, lunit, ev, p, v);
          }
        } else {
          ++v;
        }
      }
      ++s;
    }
  };

  for (;;) {
    // Idle lanes take the next path indices of the current item.  When the
    // item is used up, the wave moves to the next item of a valid unit (paths
    // of the previous unit still in flight finish with that unit's medium and
    // tally to global memory); lanes left idle by the end of an item wait for
    // the next iteration.
    const uint64_t idle = __ballot(!alive);
    if (idle != 0) {
      if (cursor >= pend && !done) {
        for (;;) {
          const int64_t item = next_item(a, static_item, lane);
          if (item < 0) {
            done = true;
            break;
          }
          int64_t ul, pb, pe;
          map_item(a.map, item, ul, pb, pe);
          if (pb >= pe) continue;
          const int64_t u = a.map.unit_begin + ul;
          if (u != u_cur) {
            if (u_cur >= 0) flush_unit<K, ADJ>(a, L, head, tail, cur_slot, u_cur, lane);
            u_cur = u;
            cur_slot = (!ADJ && a.direct) ? u : item;
            unit_ok = stage_any<K, LAYERED>(a, u, L.media, lane);
          }
          if (!unit_ok) continue;  // an invalid unit keeps zero tallies
          cursor = uint32_t(pb);
          pend = uint32_t(pe);
          break;
        }
        cursor = __builtin_amdgcn_readfirstlane(cursor);
        pend = __builtin_amdgcn_readfirstlane(pend);
        if constexpr (MARK) {
          flush_live(a, L.live, wu, wb, lane);
          wu = done ? kNoUnit : uint32_t(u_cur);
          wb = cursor >> 5;
        }
      }
      if (ADJ && a.live_mask) {
        // replay only the paths the forward saw leave the top: of the next 64
        // path indices, the r-th idle lane takes the r-th live one, and the
        // cursor moves past the last one taken (or past all 64)
        // the candidates' mask words from an LDS window of kWave words, read
        // from memory once per kWave words (an item of 2 048 paths: once)
        // (a wave that never took an item has u_cur = -1 and no candidates)
        const uint32_t cw = cursor >> 5;
        if (u_cur >= 0 && (uint32_t(u_cur) != mu || cw < mw || cw + 2u >= mw + uint32_t(kWave))) {
          mu = uint32_t(u_cur);
          mw = cw;
          const uint32_t w = mw + uint32_t(lane);
          L.mwin[lane] = int64_t(w) < a.mask_words ? a.live_mask[u_cur * a.mask_words + w] : 0u;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        const uint32_t c = cursor + uint32_t(lane);
        bool live = false;
        if (c < pend) live = (L.mwin[(c >> 5) - mw] >> (c & 31u)) & 1u;
        const uint64_t lb = __ballot(live);
        const uint32_t n_live = uint32_t(__popcll(lb));
        const uint32_t n_idle = uint32_t(__popcll(idle));
        // the live candidates' lanes in rank order, so that the r-th idle lane
        // reads the r-th live one instead of searching the ballot's bits
        if (live) L.pick[lane_rank(lb)] = uint32_t(lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (!alive) {
          const uint32_t r = lane_rank(idle);
          if (r < n_live) {
            path = cursor + L.pick[r];
            v = 0;
            alive = true;
            lunit = uint32_t(u_cur);
            lslot = uint32_t(cur_slot);
            lctr = a.unit_base + lunit;
          }
        }
        const uint32_t next =
            n_live > n_idle ? cursor + __builtin_amdgcn_readfirstlane(L.pick[n_idle]) : cursor + 64u;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        cursor = next < pend ? next : pend;
      } else {
        if (!alive) {
          const uint32_t cand = cursor + lane_rank(idle);
          if (cand < pend) {
            path = cand;
            v = 0;
            alive = true;
            lunit = uint32_t(u_cur);
            lslot = uint32_t(cur_slot);
            lctr = a.unit_base + lunit;
          }
        }
        const uint32_t next = cursor + uint32_t(__popcll(idle));
        cursor = next < pend ? next : pend;
      }
    }
    // no lane alive: the last item has been handed out and every path ended
    const uint64_t busy = __ballot(alive);
    if (busy == 0) break;
    // no further path will come and at most half the lanes are busy: finish
    // in the tail loop below
    if (done && cursor >= pend && __popcll(busy) <= kWave / 2) break;

    // A wave carrying a long path is on the critical path of the launch:
    // raise its issue priority while it does (checked every 16 iterations).
    if ((++iter & 15u) == 0) {
      const bool want = __ballot(alive && v > kLongPath) != 0;
      if (want != boosted) {
        if (want) __builtin_amdgcn_s_setprio(2); else __builtin_amdgcn_s_setprio(0);
        boosted = want;
      }
    }

    // kStepsPerIteration vertices per pass of the schedule above; a lane whose
    // path ends in an earlier step sits out the later ones (its end code and
    // state stay as they were) and is tallied below with the others
    int ev = EV_COLLIDE;
#pragma unroll
    for (int rep = 0; rep < kStepsPerIteration; ++rep) {
      if (alive) {
        const uint4 w = philox(v, path, opaque_tag(a.tag), lctr, ks);
        if (v == 0) {
          start_any<K, LAYERED>(p, w, L.media, L.cold->entry_weight, geo);
          v = 1;
        } else {
          ev = step_any<ADJ, LAYERED>(p, w, geo);
          if (ev < EV_EXIT_TOP && v >= geo.max_vertices) {
            ev = EV_CAP;
            capped = true;
          }
          if (ev >= EV_EXIT_TOP) alive = false;
          else ++v;
        }
      }
    }
    const bool ending = ev >= EV_EXIT_TOP;
    if constexpr (ADJ && LAYERED) {
      if (ending) exit_adjoint_layered(a, L, lslot == uint32_t(cur_slot), lslot, lunit, ev, p, v);
    } else if (__ballot(ending) != 0) {
      const bool local = lslot == uint32_t(cur_slot);
      const uint64_t lm = __ballot(ending && local);
      const uint32_t n_new = uint32_t(__popcll(lm));
      if (tail - head + n_new > uint32_t(kExitRing)) {
        // make room: tally what is waiting (at most one wave's worth)
        const uint32_t n = (tail - head) < uint32_t(kWave) ? (tail - head) : uint32_t(kWave);
        if (!ADJ) tally_forward(L, head, n, lane);
        else tally_adjoint<K>(a, L, uint32_t(u_cur), head, n, lane);
        head += n;
      }
      if (ending) {
        if (MARK && ev == EV_EXIT_TOP) {
          const uint32_t wd = (path >> 5) - wb;
          if (lunit == wu && wd < kLiveWindow)
            __hip_atomic_fetch_or(L.live + wd, 1u << (path & 31u), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WAVEFRONT);
          else
            mark_live(a, lunit, path);
        }
        if (local) {
          const uint32_t i = (tail + lane_rank(lm)) & (kExitRing - 1);
          if (!ADJ) {
            L.ring[i] = forward_record(ev, p, v);
          } else {
            adjoint_record(ev, p, v, L.ring[2 * i], L.ring[2 * i + 1]);
          }
        } else {
          if (!ADJ) exit_global_forward(a, L, lslot, ev, p, v);
          else exit_global_adjoint<K>(a, L, lslot, lunit, ev, p, v);
        }
      }
      tail += n_new;
    }
  }

  // the tail reuses the ring's area: the window goes to the mask first
  if constexpr (MARK) {
    flush_live(a, L.live, wu, wb, lane);
    wu = kNoUnit;
  }

  // ---- tail: the paths still running after the last one was handed out ----
  // A wave here holds at most kWave / 2 running paths (the loop above hands
  // over at half occupancy) and little else, so its iterations are bound by
  // the latency of a vertex's dependent chain: it finishes them in look-ahead
  // rounds.
  if (__ballot(alive) != 0) {
    while (head != tail) {  // the ring's LDS is reused for the draws
      const uint32_t n = (tail - head) < uint32_t(kWave) ? (tail - head) : uint32_t(kWave);
      if (!ADJ) tally_forward(L, head, n, lane);
      else tally_adjoint<K>(a, L, uint32_t(u_cur), head, n, lane);
      head += n;
    }
    __builtin_amdgcn_s_setprio(3);
    boosted = true;
    // a path handed out just before the loop above ended starts here, so that
    // every running path has its medium
    if (alive && v == 0) {
      start_any<K, LAYERED>(p, philox(0u, path, a.tag, lctr, ks), L.media, L.cold->entry_weight,
                            geo);
      v = 1;
    }
    while (__ballot(alive) != 0) lookahead_round(alive);
  }
  if (boosted) __builtin_amdgcn_s_setprio(0);
  if (u_cur >= 0) flush_unit<K, ADJ>(a, L, head, tail, cur_slot, u_cur, lane);
  if (__any(capped) && lane == 0) atomicOr(a.flags, RW_FLAG_VERTEX_CAP);
}

// Forward: per unit, the sums of its slots -> outputs.  A slot holds the words
// bins[(n_bins+2)*2] | R[4] = (sum x, sum x^2, T, A) | vertices, all exact
// int64; the unit's slots are added exactly and converted to FP64 (vertices
// stay int64).  Block = kConvWords words x kConvGroups groups of slots;
// blockIdx.y picks the words, blockIdx.x strides over the units.  Direct: the
// unit's single slot is its output, converted in place (every word is read
// before the barrier and written after it by the same thread).
__global__ void __launch_bounds__(kConvWords * kConvGroups) convert_forward_kernel(const WalkArgs a) {
  __shared__ long long part[kConvGroups][kConvWords];
  const int nb2 = 2 * (a.geo.n_bins + 2);
  const int wi = threadIdx.x % kConvWords, grp = threadIdx.x / kConvWords;
  const int w = blockIdx.y * kConvWords + wi;
  const double inv = 1.0 / double(a.fix_scale32);
  const int64_t ns = a.direct ? 1 : a.map.chunks_per_unit;
  for (int64_t ul = blockIdx.x; ul < a.map.n_units; ul += gridDim.x) {
    const int64_t u = a.map.unit_begin + ul;
    const int64_t s0 = a.direct ? u : ul * a.map.chunks_per_unit;
    long long v = 0;
    if (w < nb2 + 5) {
      for (int64_t c = grp; c < ns; c += kConvGroups) {
        const int64_t sl = s0 + c;
        v += w < nb2 ? a.tb[sl * nb2 + w] : (w < nb2 + 4 ? a.tc[sl * 4 + (w - nb2)] : a.tv[sl]);
      }
    }
    part[grp][wi] = v;
    __syncthreads();
    if (grp == 0 && w < nb2 + 5) {
#pragma unroll
      for (int g = 1; g < kConvGroups; ++g) v += part[g][wi];
      if (w < nb2) a.out_bins[u * nb2 + w] = double(v) * inv;
      else if (w < nb2 + 4) a.out_R[u * 4 + (w - nb2)] = double(v) * inv;
      else a.out_vertices[u] = v;
    }
    __syncthreads();
  }
}

// Adjoint: per unit, the sums of its slots (fixed order: by group, groups
// combined in group order), then the [K][8] sums (C, Q, Ss, Ss2, Sa, Sa2, Sg,
// Sg2) to gradients: sigma_t_k, alpha_k, g_k directly; logit_j = C_j - w_j C
// with sum of squares (1 - w_j)^2 Q_j + w_j^2 (Q - Q_j).  The two-layer walk
// (LAYERED, K = 2 layers) has no mixture weights: its logit columns are 0.
// One block per unit (grid-stride), kConvWords x kConvGroups threads.
template <int K, bool LAYERED = false>
__global__ void __launch_bounds__(kConvWords * kConvGroups) convert_adjoint_kernel(
    const WalkArgs a, double* grad, double* grad_sumsq, int64_t* vertices_out) {
  static_assert(8 * K + 1 <= kConvWords, "adjoint slot wider than a block row");
  __shared__ double part[kConvGroups][kConvWords];
  __shared__ long long vpart[kConvGroups];
  const int wi = threadIdx.x % kConvWords, grp = threadIdx.x / kConvWords;
  const int64_t ns = a.map.chunks_per_unit;
  for (int64_t ul = blockIdx.x; ul < a.map.n_units; ul += gridDim.x) {
    const int64_t u = a.map.unit_begin + ul;
    const int64_t s0 = ul * ns;
    if (wi < 8 * K) {
      double v = 0.0;
      for (int64_t c = grp; c < ns; c += kConvGroups) v += a.adj[(s0 + c) * (8 * K) + wi];
      part[grp][wi] = v;
    } else if (wi == 8 * K) {
      long long nv = 0;
      for (int64_t c = grp; c < ns; c += kConvGroups) nv += a.adj_vertices[s0 + c];
      vpart[grp] = nv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s[8 * K];
      for (int m = 0; m < 8 * K; ++m) {
        double v = part[0][m];
        for (int g = 1; g < kConvGroups; ++g) v += part[g][m];
        s[m] = v;
      }
      if (vertices_out) {
        long long nv = 0;
        for (int g = 0; g < kConvGroups; ++g) nv += vpart[g];
        vertices_out[u] = nv;
      }
      double wts[K];
      if constexpr (LAYERED) {
#pragma unroll
        for (int k = 0; k < K; ++k) wts[k] = 0.0;
      } else {
        const UnitParams<K> up = load_unit<K>(a, u);
#pragma unroll
        for (int k = 0; k < K; ++k) wts[k] = double(up.w[k]);
      }
      double C = 0.0, Q = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        C += s[8 * k + 0];
        Q += s[8 * k + 1];
      }
      double* G = grad + u * (4 * K);
      double* S = grad_sumsq ? grad_sumsq + u * (4 * K) : nullptr;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double wk = wts[k];
        G[k] = s[8 * k + 2];
        G[K + k] = s[8 * k + 4];
        G[2 * K + k] = s[8 * k + 6];
        G[3 * K + k] = LAYERED ? 0.0 : s[8 * k + 0] - wk * C;
        if (S) {
          S[k] = s[8 * k + 3];
          S[K + k] = s[8 * k + 5];
          S[2 * K + k] = s[8 * k + 7];
          S[3 * K + k] = LAYERED ? 0.0
                                 : (1.0 - wk) * (1.0 - wk) * s[8 * k + 1] +
                                       wk * wk * (Q - s[8 * k + 1]);
        }
      }
    }
    __syncthreads();
  }
}

// Longest-first order of the units (persistent schedule).  The estimate of
// the mean vertices per path of a medium only orders work and never changes a
// result: paths end at the surface or by roulette, which starts after
// n_rr = ln(rr_weight / W0) / ln(alpha) collisions; before that the walk
// leaves like a diffusing particle, about c sqrt(n / (1 - g)) collisions for a
// horizon of n (c ~ 5 fitted on walks of this kind).
__device__ __forceinline__ float est_path_vertices(float alb, float g, const WalkGeom& geo) {
  const float cap = float(geo.max_vertices);
  float n_rr;
  if (!(geo.rr_weight > 0.0f) || alb >= 1.0f) {
    n_rr = cap;
  } else if (alb <= 0.0f) {
    n_rr = 1.0f;
  } else {
    n_rr = fminf(__logf(geo.rr_weight / geo.entry_weight) / __logf(alb), cap);
  }
  return 2.0f + fminf(n_rr, 5.0f * sqrtf(n_rr / fmaxf(1.0f - g, 1e-3f)));
}

// Bucket of a unit's estimated cost (descending cost order), counted in the
// block's LDS histogram; the block then adds its non-zero counts to the global
// histogram, one atomic per bucket (adjacent units tend to share buckets, and
// per-unit global atomics on 64 counters serialise: ~1 ms per 10^5 units).
__device__ __forceinline__ int cost_bucket(float c) {
  int b = int(4.0f * __log2f(c + 1.0f));
  b = b < 0 ? 0 : (b > kOrderBuckets - 1 ? kOrderBuckets - 1 : b);
  return kOrderBuckets - 1 - b;
}

__device__ __forceinline__ void block_histogram_add(uint32_t* local, uint32_t* hist) {
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x)
    if (local[i]) atomicAdd(&hist[i], local[i]);
}

template <int K>
__global__ void __launch_bounds__(256) unit_cost_kernel(const WalkArgs a, int32_t* bucket,
                                                        uint32_t* hist) {
  __shared__ uint32_t local[kOrderBuckets];
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) local[i] = 0u;
  __syncthreads();
  const int64_t ul = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (ul < a.map.n_units) {
    const UnitParams<K> up = load_unit<K>(a, a.map.unit_begin + ul);
    float c = 1.0f;
    if (up.ok) {
      c = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) c += up.w[k] * est_path_vertices(up.alb[k], up.g[k], a.geo);
    }
    const int b = cost_bucket(c);
    bucket[ul] = b;
    atomicAdd(&local[b], 1u);
  }
  block_histogram_add(local, hist);
}

// two-layer units: a path spends most of its vertices in the bottom layer
__global__ void __launch_bounds__(256) unit_cost_layered_kernel(const WalkArgs a, int32_t* bucket,
                                                                uint32_t* hist) {
  __shared__ uint32_t local[kOrderBuckets];
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) local[i] = 0u;
  __syncthreads();
  const int64_t ul = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (ul < a.map.n_units) {
    const LayerParams lp = load_layers(a, a.map.unit_begin + ul);
    const int b = cost_bucket(lp.ok ? est_path_vertices(lp.alb[1], lp.g[1], a.geo) : 1.0f);
    bucket[ul] = b;
    atomicAdd(&local[b], 1u);
  }
  block_histogram_add(local, hist);
}

// exclusive prefix of the bucket counts, in place (one wave)
__global__ void order_scan_kernel(uint32_t* hist) {
  if (threadIdx.x != 0) return;
  uint32_t acc = 0;
  for (int b = 0; b < kOrderBuckets; ++b) {
    const uint32_t c = hist[b];
    hist[b] = acc;
    acc += c;
  }
}

// scatter local unit indices to their bucket ranges (order within a bucket is
// arbitrary; it only affects timing): each block counts its units per bucket
// in LDS, reserves one range per non-empty bucket with one global atomic, and
// places its units inside the ranges by their LDS ranks
__global__ void __launch_bounds__(256) order_scatter_kernel(int64_t n_units, const int32_t* bucket,
                                                            uint32_t* cursor, int32_t* unit_order) {
  __shared__ uint32_t cnt[kOrderBuckets], base[kOrderBuckets];
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) cnt[i] = 0u;
  __syncthreads();
  const int64_t ul = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int b = -1;
  uint32_t rank = 0;
  if (ul < n_units) {
    b = bucket[ul];
    rank = atomicAdd(&cnt[b], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x)
    base[i] = cnt[i] ? atomicAdd(&cursor[i], cnt[i]) : 0u;
  __syncthreads();
  if (b >= 0) unit_order[base[b] + rank] = int32_t(ul);
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void fill_u64_kernel(uint64_t* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0ull;
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
    // the path count the walk ran: a per-unit entry clamped to [0, paths_uniform]
    // exactly as the walk's work map clamps it
    int64_t n_run = paths_uniform;
    if (paths) {
      const int64_t q = paths[u];
      n_run = q < 0 ? 0 : (q < paths_uniform ? q : paths_uniform);
    }
    const double N = double(n_run);
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
// Event codes are written in the oracle's numbering.
template <int K, bool LAYERED>
__global__ void trace_kernel(const WalkArgs a, const uint32_t* words, int64_t n_paths,
                             int64_t n_blocks, uint32_t unit_index, float* events, float* path_out,
                             float* path_adj) {
  const int64_t pth = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (pth >= n_paths) return;
  const PhiloxKey ks = philox_schedule(a.key0, a.key1);
  const WalkGeom& geo = a.geo;
  float* ev = events ? events + pth * n_blocks * 8 : nullptr;
  Path p;
  int end = 7, slot = -1;
  uint32_t nvert = 0, ncoll = 0;  // the two-layer step keeps no collision count
  for (int64_t v = 0; v < n_blocks; ++v) {
    if (v > 0 && v > int64_t(geo.max_vertices)) {
      end = 4;
      if (ev) {
        float* e = ev + v * 8;
        e[0] = float(trace_code(EV_CAP)); e[1] = p.x; e[2] = p.y; e[3] = p.z;
        e[4] = p.ux; e[5] = p.uy; e[6] = p.uz; e[7] = p.W;
      }
      break;
    }
    uint4 w;
    if (words) {
      const uint32_t* q = words + (pth * n_blocks + v) * 4;
      w = make_uint4(q[0], q[1], q[2], q[3]);
    } else {
      w = philox(uint32_t(v), uint32_t(pth), a.tag, unit_index, ks);
    }
    int code;
    if (v == 0) {
      if constexpr (LAYERED) start_path_layers(p, w, load_layers(a, 0), geo);
      else start_path<K>(p, w, load_unit<K>(a, 0), geo);
      code = EV_START;
    } else {
      nvert = uint32_t(v);
      if constexpr (LAYERED) code = vertex_step_layered<false>(p, w, geo);
      else code = vertex_step<true>(p, w, geo);
      if (code == EV_COLLIDE || code == EV_RR_KILL) ++ncoll;
    }
    if (ev) {
      float* e = ev + v * 8;
      e[0] = float(trace_code(code)); e[1] = p.x; e[2] = p.y; e[3] = p.z;
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
  o[6] = float(ncoll);
  o[7] = p.A;
  if (!LAYERED && path_adj) {
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
int walk_lds_bytes(const WalkArgs& a, int waves_per_wg) {
  return waves_per_wg * a.lds_words_per_wave * int(sizeof(u64));
}

template <int K>
static hipError_t launch_walk_k(const WalkArgs& a, bool adjoint, int waves_per_wg, int grid,
                                hipStream_t s) {
  const size_t lds = size_t(walk_lds_bytes(a, waves_per_wg));
  if (adjoint)
    hipLaunchKernelGGL((walk_kernel<K, true, false, false>), dim3(grid),
                       dim3(waves_per_wg * kWave), lds, s, a);
  else if (a.live_mask)
    hipLaunchKernelGGL((walk_kernel<K, false, false, true>), dim3(grid),
                       dim3(waves_per_wg * kWave), lds, s, a);
  else
    hipLaunchKernelGGL((walk_kernel<K, false, false, false>), dim3(grid),
                       dim3(waves_per_wg * kWave), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_walk(const WalkArgs& a, int K, bool adjoint, int waves_per_wg, int grid_wgs,
                       hipStream_t stream) {
  switch (K) {
    case 1: return launch_walk_k<1>(a, adjoint, waves_per_wg, grid_wgs, stream);
    case 2: return launch_walk_k<2>(a, adjoint, waves_per_wg, grid_wgs, stream);
    case 3: return launch_walk_k<3>(a, adjoint, waves_per_wg, grid_wgs, stream);
    case 4: return launch_walk_k<4>(a, adjoint, waves_per_wg, grid_wgs, stream);
    case kLayeredModel:
      if (adjoint)
        hipLaunchKernelGGL((walk_kernel<2, true, true, false>), dim3(grid_wgs),
                           dim3(waves_per_wg * kWave), size_t(walk_lds_bytes(a, waves_per_wg)),
                           stream, a);
      else if (a.live_mask)
        hipLaunchKernelGGL((walk_kernel<2, false, true, true>), dim3(grid_wgs),
                           dim3(waves_per_wg * kWave), size_t(walk_lds_bytes(a, waves_per_wg)),
                           stream, a);
      else
        hipLaunchKernelGGL((walk_kernel<2, false, true, false>), dim3(grid_wgs),
                           dim3(waves_per_wg * kWave), size_t(walk_lds_bytes(a, waves_per_wg)),
                           stream, a);
      return hipGetLastError();
    default: return hipErrorInvalidValue;
  }
}

// The walk instantiation a launch uses: adjoint, or forward with (mark) or
// without the live-path mask.
template <int K, bool LAYERED>
static const void* walk_ptr(bool adjoint, bool mark) {
  if (adjoint) return reinterpret_cast<const void*>(walk_kernel<K, true, LAYERED, false>);
  return mark ? reinterpret_cast<const void*>(walk_kernel<K, false, LAYERED, true>)
              : reinterpret_cast<const void*>(walk_kernel<K, false, LAYERED, false>);
}

const void* walk_kernel_ptr(int K, bool adjoint, bool mark) {
  switch (K) {
    case 1: return walk_ptr<1, false>(adjoint, mark);
    case 2: return walk_ptr<2, false>(adjoint, mark);
    case 3: return walk_ptr<3, false>(adjoint, mark);
    case 4: return walk_ptr<4, false>(adjoint, mark);
    case kLayeredModel: return walk_ptr<2, true>(adjoint, mark);
    default: return nullptr;
  }
}

const void* fill_u32_kernel_ptr() { return (const void*)fill_u32_kernel; }
const void* fill_u64_kernel_ptr() { return (const void*)fill_u64_kernel; }
const void* unit_cost_kernel_ptr(int K) {
  switch (K) {
    case kLayeredModel: return (const void*)unit_cost_layered_kernel;
    case 1: return (const void*)unit_cost_kernel<1>;
    case 2: return (const void*)unit_cost_kernel<2>;
    case 3: return (const void*)unit_cost_kernel<3>;
    case 4: return (const void*)unit_cost_kernel<4>;
    default: return nullptr;
  }
}
const void* order_scan_kernel_ptr() { return (const void*)order_scan_kernel; }
const void* order_scatter_kernel_ptr() { return (const void*)order_scatter_kernel; }
const void* convert_forward_kernel_ptr() { return (const void*)convert_forward_kernel; }
const void* convert_adjoint_kernel_ptr(int K) {
  switch (K) {
    case 1: return (const void*)convert_adjoint_kernel<1>;
    case 2: return (const void*)convert_adjoint_kernel<2>;
    case 3: return (const void*)convert_adjoint_kernel<3>;
    case 4: return (const void*)convert_adjoint_kernel<4>;
    case kLayeredModel: return (const void*)convert_adjoint_kernel<2, true>;
    default: return nullptr;
  }
}

hipError_t launch_unit_order(const WalkArgs& a, int K, int32_t* bucket, uint32_t* hist,
                             int32_t* unit_order, hipStream_t s) {
  const int64_t n = a.map.n_units;
  if (n <= 0) return hipSuccess;
  const unsigned grid = unsigned((n + 255) / 256);
  switch (K) {
    case 1: hipLaunchKernelGGL(unit_cost_kernel<1>, dim3(grid), dim3(256), 0, s, a, bucket, hist); break;
    case 2: hipLaunchKernelGGL(unit_cost_kernel<2>, dim3(grid), dim3(256), 0, s, a, bucket, hist); break;
    case 3: hipLaunchKernelGGL(unit_cost_kernel<3>, dim3(grid), dim3(256), 0, s, a, bucket, hist); break;
    case 4: hipLaunchKernelGGL(unit_cost_kernel<4>, dim3(grid), dim3(256), 0, s, a, bucket, hist); break;
    case kLayeredModel: hipLaunchKernelGGL(unit_cost_layered_kernel, dim3(grid), dim3(256), 0, s, a, bucket, hist); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(64), 0, s, hist);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(grid), dim3(256), 0, s, n, bucket, hist, unit_order);
  return hipGetLastError();
}

static int fill_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return int(g < 1 ? 1 : g);
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_convert_forward(const WalkArgs& a, hipStream_t s) {
  if (a.map.n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_forward_kernel, convert_forward_grid(a.map.n_units, a.geo.n_bins),
                     dim3(kConvWords * kConvGroups), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_convert_adjoint(const WalkArgs& a, int K, double* grad, double* grad_sumsq,
                                  int64_t* vertices_out, hipStream_t s) {
  if (a.map.n_units <= 0) return hipSuccess;
  const unsigned grid = convert_blocks(a.map.n_units);
  switch (K) {
    case 1: hipLaunchKernelGGL(convert_adjoint_kernel<1>, dim3(grid), dim3(kConvWords * kConvGroups), 0, s, a, grad, grad_sumsq, vertices_out); break;
    case 2: hipLaunchKernelGGL(convert_adjoint_kernel<2>, dim3(grid), dim3(kConvWords * kConvGroups), 0, s, a, grad, grad_sumsq, vertices_out); break;
    case 3: hipLaunchKernelGGL(convert_adjoint_kernel<3>, dim3(grid), dim3(kConvWords * kConvGroups), 0, s, a, grad, grad_sumsq, vertices_out); break;
    case 4: hipLaunchKernelGGL(convert_adjoint_kernel<4>, dim3(grid), dim3(kConvWords * kConvGroups), 0, s, a, grad, grad_sumsq, vertices_out); break;
    case kLayeredModel: hipLaunchKernelGGL((convert_adjoint_kernel<2, true>), dim3(grid), dim3(kConvWords * kConvGroups), 0, s, a, grad, grad_sumsq, vertices_out); break;
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
    case 1: hipLaunchKernelGGL((trace_kernel<1, false>), dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    case 2: hipLaunchKernelGGL((trace_kernel<2, false>), dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    case 3: hipLaunchKernelGGL((trace_kernel<3, false>), dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    case 4: hipLaunchKernelGGL((trace_kernel<4, false>), dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, path_adj); break;
    case kLayeredModel: hipLaunchKernelGGL((trace_kernel<2, true>), dim3(grid), dim3(64), 0, s, a, words, n_paths, n_blocks, unit_index, events, path_out, nullptr); break;
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
