// Hero-wavelength two-layer walk for gfx950: one path serves a group of C
// wavelengths of one tissue (Wilkie et al. 2014's hero wavelength, named in
// Sec. 2; Sec. 3's simulator propagates all its wavelengths together).
//
// Path p of group q is sampled with the optics of member h = p mod C: its
// free flights from sigma_t of h, its scatterings from g of h (the surface
// and interface decisions depend on the indices alone, which the group
// shares).  Every member i carries its own weight x_i, multiplied by its
// albedo at each collision; roulette decides on the largest weight and boosts
// all of them, so every x_i <= 1.  Each member's path density differs from
// the hero's only through sigma_t (per layer: sigma^n_coll exp(-sigma L)) and
// the phase densities of the scatterings, so the path keeps per layer its
// collision count and length, and per member the sum of log2 p_HG(mu; g_i).
// A path that leaves contributes, to member i, the one-sample
// balance-heuristic estimate F_i = C x_i p_i / sum_j p_j <= C.
//
// Work: one wavefront per work item (group, chunk of paths); its lanes take
// the item's paths in turn.  Tallies: exact fixed-point sums per member in the
// item's own slot (only this wave writes it, so workgroup-scope atomics do),
// added up per unit by the convert kernel.  A path walks about 430 vertices
// in the tissue workloads, so its handful of tally atomics is negligible.
#include <hip/hip_runtime.h>

#include "../../include/rw.h"
#include "rw_device.hpp"
#include "rw_internal.hpp"

namespace rw {

using u64h = unsigned long long;

// LDS table per member i and layer l (12 floats): {flight, g, hq, albedo},
// {log2 sigma_t, sigma_t log2(e), 2 g, (1 - g)^2}, {log2((1 - g^2) / 2), 0, 0, 0}
constexpr int kHeroFloats = 12;

__device__ __forceinline__ const float* hero_entry(const float* tab, int i, int layer) {
  return tab + (i * 2 + layer) * kHeroFloats;
}

__device__ __forceinline__ void hero_add(u64h* p, u64h v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ u64h hero_fix(float x, float scale, float cap) {
  return u64h(uint32_t(fmaf(__builtin_amdgcn_fmed3f(x, 0.0f, cap), scale, 0.5f)));
}

template <int C>
struct HeroPath {
  float x, y, z, ux, uy, uz;
  int layer;
  float w[C];    // member weights
  float hg[C];   // member sums of log2 p_HG over the scatterings
  uint32_t nc0, nc1;  // collisions in the top and bottom layer
  float L0, L1;       // path length in the top and bottom layer
};

// Load and check a group's members; stage them in the wave's LDS table.
// Returns false (and raises the flag) for invalid layers or members whose
// top-layer thicknesses differ.
template <int C>
__device__ __forceinline__ bool stage_hero(const HeroArgs& a, int64_t q, float* tab, float& d,
                                           int lane) {
  bool ok = true;
  const float d0 = a.layer_d[q * C];
  for (int i = 0; i < C; ++i) {
    const int64_t u = q * C + i;
    const float di = a.layer_d[u];
    ok = ok && di == d0 && di > 0.0f && di < 3.0e38f && (!a.geo.slab || di < a.geo.slab_mm);
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const float s = a.sigma_t[l * a.k_stride + u], al = a.albedo[l * a.k_stride + u],
                  g = a.g[l * a.k_stride + u];
      ok = ok && s > 0.0f && s < 3.0e38f && al >= 0.0f && al <= 1.0f && fabsf(g) < 1.0f;
      if (lane == i * 2 + l) {
        const Medium m = make_medium(s, al, g);
        float* e = tab + (i * 2 + l) * kHeroFloats;
        e[0] = m.flight; e[1] = g; e[2] = m.hq; e[3] = al;
        e[4] = __builtin_amdgcn_logf(s);
        e[5] = s * 1.4426950408889634f;
        e[6] = 2.0f * g;
        e[7] = (1.0f - g) * (1.0f - g);
        e[8] = __builtin_amdgcn_logf(0.5f * (1.0f - g * g));
        e[9] = 0.0f; e[10] = 0.0f; e[11] = 0.0f;
      }
    }
  }
  d = d0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (!ok && lane == 0) atomicOr(a.flags, RW_FLAG_BAD_PARAMS);
  return ok;
}

// One vertex of a hero path (v >= 1).  Returns the vertex event.
template <int C>
__device__ __forceinline__ int hero_step(HeroPath<C>& p, uint4 w, const float* tab, int hero,
                                         float d, const WalkGeom& geo) {
  const float* eh = hero_entry(tab, hero, p.layer);
  const VertexDraw dr = draw_vertex(eh[0], eh[1], eh[2], w);
  const float s = dr.s;
  const float zn = fmaf(s, p.uz, p.z);
  const bool top_layer = p.layer == 0;
  int face = 0;
  if (top_layer) {
    if (p.uz < 0.0f && zn <= 0.0f) face = 1;
    else if (p.uz > 0.0f && zn >= d) face = 2;
  } else {
    if (p.uz < 0.0f && zn <= d) face = 2;
    else if (geo.slab && p.uz > 0.0f && zn >= geo.slab_mm) face = 3;
  }
  // the move is the same arithmetic for a flight that reaches a face after
  // l = db and one that collides after l = s, so all lanes make it together
  const float zf = face == 1 ? 0.0f : (face == 2 ? d : geo.slab_mm);
  const float l = face != 0 ? (zf - p.z) * __builtin_amdgcn_rcpf(p.uz) : s;
  p.x = fmaf(l, p.ux, p.x);
  p.y = fmaf(l, p.uy, p.y);
  p.z = face != 0 ? zf : zn;
  if (top_layer) p.L0 += l; else p.L1 += l;
  if (face != 0) {
    if (face == 2) {
      if (!geo.interface_matched) {
        const float rel = top_layer ? geo.rel_down : geo.rel_up;
        const float rel2 = top_layer ? geo.rel_down2 : geo.rel_up2;
        if (u01(dr.w3) < fresnel(fabsf(p.uz), rel, rel2)) {
          p.uz = -p.uz;
          return EV_REFLECT;
        }
        const float ct =
            __builtin_amdgcn_sqrtf(fmaxf(0.0f, fmaf(-rel2, fmaf(-p.uz, p.uz, 1.0f), 1.0f)));
        p.ux *= rel;
        p.uy *= rel;
        p.uz = p.uz > 0.0f ? ct : -ct;
      }
      p.layer ^= 1;
      return EV_CROSS;
    }
    const bool top = face == 1;
    if (!(top ? geo.index_matched : geo.bot_matched)) {
      const float F = top ? fresnel(fabsf(p.uz), geo.n_rel, geo.n_rel2)
                          : fresnel(fabsf(p.uz), geo.n_bot, geo.n_bot2);
      if (u01(dr.w3) < F) {
        p.uz = -p.uz;
        return EV_REFLECT;
      }
    }
    return top ? EV_EXIT_TOP : EV_EXIT_BOTTOM;
  }
  // collision: every member's weight times its albedo, roulette on the
  // largest, the hero's scattering and every member's phase density of it
  if (top_layer) ++p.nc0; else ++p.nc1;
  float wmax = 0.0f;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    p.w[i] *= hero_entry(tab, i, p.layer)[3];
    wmax = fmaxf(wmax, p.w[i]);
  }
  if (wmax < geo.rr_weight) {
    if (u01(dr.w3) < geo.rr_survive) {
#pragma unroll
      for (int i = 0; i < C; ++i) p.w[i] *= geo.rr_boost;
    } else {
      return EV_RR_KILL;
    }
  }
  const float omm = 1.0f - dr.mu;  // 1 - mu of the scattering
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const float* e = hero_entry(tab, i, p.layer);
    // 1 + g^2 - 2 g mu = (1 - g)^2 + 2 g (1 - mu), without cancellation near mu = 1
    const float t = fmaf(e[6], omm, e[7]);
    p.hg[i] += fmaf(-1.5f, __builtin_amdgcn_logf(t), e[8]);
  }
  rotate(p.ux, p.uy, p.uz, dr.mu, dr.p, dr.q);
  return EV_COLLIDE;
}

// The members' balance-heuristic contributions of a path that leaves.
template <int C>
__device__ __forceinline__ void hero_contrib(const HeroPath<C>& p, const float* tab, float* F) {
  float lp[C];
  float m = -3.0e38f;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const float* e0 = hero_entry(tab, i, 0);
    const float* e1 = hero_entry(tab, i, 1);
    float v = p.hg[i];
    v = fmaf(float(p.nc0), e0[4], v);
    v = fmaf(-p.L0, e0[5], v);
    v = fmaf(float(p.nc1), e1[4], v);
    v = fmaf(-p.L1, e1[5], v);
    lp[i] = v;
    m = fmaxf(m, v);
  }
  float S = 0.0f;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    lp[i] = __builtin_amdgcn_exp2f(lp[i] - m);
    S += lp[i];
  }
  const float k = float(C) * __builtin_amdgcn_rcpf(S);
#pragma unroll
  for (int i = 0; i < C; ++i) F[i] = p.w[i] * lp[i] * k;
}

template <int C>
__device__ __forceinline__ void hero_tally(const HeroArgs& a, int64_t item, int ev,
                                           const HeroPath<C>& p, const float* tab, int hero,
                                           uint32_t nv) {
  const int nw = 2 * (a.geo.n_bins + 2) + 2;  // per member: bins, T, vertices
  u64h* slot = reinterpret_cast<u64h*>(a.slots) + item * int64_t(C * nw);
  hero_add(&slot[hero * nw + nw - 1], u64h(nv));
  if (ev != EV_EXIT_TOP && ev != EV_EXIT_BOTTOM) return;
  float F[C];
  hero_contrib<C>(p, tab, F);
  const float sc = a.fix_scale32, cap = a.fix_cap;
  if (ev == EV_EXIT_TOP) {
    const int b = radial_slot(p.x, p.y, a.geo);
#pragma unroll
    for (int i = 0; i < C; ++i) {
      hero_add(&slot[i * nw + 2 * b], hero_fix(F[i], sc, cap));
      hero_add(&slot[i * nw + 2 * b + 1], hero_fix(F[i] * F[i], sc, cap));
    }
  } else {
#pragma unroll
    for (int i = 0; i < C; ++i) hero_add(&slot[i * nw + nw - 2], hero_fix(F[i], sc, cap));
  }
}

template <int C>
__global__ void __launch_bounds__(256) hero_walk_kernel(const HeroArgs a) {
  extern __shared__ float hero_lds[];
  const int lane = __lane_id();
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t item = int64_t(blockIdx.x) * (blockDim.x / kWave) + wid;
  if (item >= a.n_items) return;  // whole waves
  float* tab = hero_lds + wid * (C * 2 * kHeroFloats);
  const int64_t q = a.group_begin + item / a.chunks_per_group;
  const int64_t c = item - (item / a.chunks_per_group) * a.chunks_per_group;
  const uint32_t pb = uint32_t(c * a.chunk);
  const uint32_t pe = uint32_t(min(int64_t(pb) + a.chunk, a.paths_per_group));
  float d;
  if (!stage_hero<C>(a, q, tab, d, lane)) return;  // the group keeps zero tallies
  const PhiloxKey ks = philox_schedule(a.key0, a.key1);
  const uint32_t ctr3 = uint32_t(a.unit_base + uint64_t(q));
  const WalkGeom geo = a.geo;

  HeroPath<C> p;
  bool alive = false, capped = false;
  uint32_t path = 0, v = 0, cursor = pb;
  int hero = 0;
  for (;;) {
    const uint64_t idle = __ballot(!alive);
    if (idle != 0 && cursor < pe) {
      if (!alive) {
        const uint32_t cand = cursor + __builtin_amdgcn_mbcnt_hi(
                                           uint32_t(idle >> 32),
                                           __builtin_amdgcn_mbcnt_lo(uint32_t(idle), 0u));
        if (cand < pe) {
          path = cand;
          v = 0;
          alive = true;
          hero = int(cand % uint32_t(C));
        }
      }
      const uint32_t next = cursor + uint32_t(__popcll(idle));
      cursor = next < pe ? next : pe;
    }
    if (__ballot(alive) == 0) break;
    // four vertex steps per pass of the regeneration (two: about 2 % slower;
    // six and eight: within noise); a lane whose path ends in an earlier step
    // sits out the later ones
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      if (alive) {
        const uint4 w = philox(v, path, a.tag, ctr3, ks);
        if (v == 0) {
          // entry through the surface, shared by all members
          Path e;
          e.W = geo.entry_weight;
          e.ux = 0.0f; e.uy = 0.0f; e.uz = 1.0f;
          if (geo.incidence) cosine_entry(e, w, geo);
          p.x = 0.0f; p.y = 0.0f; p.z = 0.0f;
          p.ux = e.ux; p.uy = e.uy; p.uz = e.uz;
          p.layer = 0;
          p.nc0 = 0; p.nc1 = 0;
          p.L0 = 0.0f; p.L1 = 0.0f;
#pragma unroll
          for (int i = 0; i < C; ++i) {
            p.w[i] = e.W;
            p.hg[i] = 0.0f;
          }
          v = 1;
        } else {
          int ev = hero_step<C>(p, w, tab, hero, d, geo);
          if (ev < EV_EXIT_TOP && v >= geo.max_vertices) {
            ev = EV_CAP;
            capped = true;
          }
          if (ev >= EV_EXIT_TOP) {
            alive = false;
            hero_tally<C>(a, item, ev, p, tab, hero, v);
          } else {
            ++v;
          }
        }
      }
    }
  }
  if (__any(capped) && lane == 0) atomicOr(a.flags, RW_FLAG_VERTEX_CAP);
}

// Per unit u = q C + i: the sums of member i over the group's items, exact,
// converted to FP64: bins, then R = (sum x, sum x^2 over the slots, T, 0) and
// the vertices of the paths u was hero of.  One block per unit (grid stride).
template <int C>
__global__ void __launch_bounds__(256) hero_convert_kernel(const HeroArgs a) {
  __shared__ long long red[2][256 / kWave];
  const int nb2 = 2 * (a.geo.n_bins + 2);
  const int nw = nb2 + 2;
  const double inv = 1.0 / double(a.fix_scale32);
  const long long* S = reinterpret_cast<const long long*>(a.slots);
  const int64_t n_units = a.n_groups * C;
  for (int64_t ul = blockIdx.x; ul < n_units; ul += gridDim.x) {
    const int64_t ql = ul / C;
    const int i = int(ul - ql * C);
    const int64_t u = a.group_begin * C + ul;
    long long s1 = 0, s2 = 0;
    for (int wd = threadIdx.x; wd < nw; wd += blockDim.x) {
      long long v = 0;
      for (int64_t c = 0; c < a.chunks_per_group; ++c)
        v += S[((ql * a.chunks_per_group + c) * C + i) * nw + wd];
      if (wd < nb2) {
        a.out_bins[u * nb2 + wd] = double(v) * inv;
        if (wd & 1) s2 += v; else s1 += v;
      } else if (wd == nb2) {
        a.out_R[u * 4 + 2] = double(v) * inv;
        a.out_R[u * 4 + 3] = 0.0;
      } else {
        a.out_vertices[u] = v;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1 += __shfl_xor(s1, off, kWave);
      s2 += __shfl_xor(s2, off, kWave);
    }
    if (__lane_id() == 0) {
      red[0][threadIdx.x / kWave] = s1;
      red[1][threadIdx.x / kWave] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      long long t1 = 0, t2 = 0;
      for (int k = 0; k < int(blockDim.x / kWave); ++k) {
        t1 += red[0][k];
        t2 += red[1][k];
      }
      a.out_R[u * 4 + 0] = double(t1) * inv;
      a.out_R[u * 4 + 1] = double(t2) * inv;
    }
    __syncthreads();
  }
}

template <int C>
static hipError_t launch_hero_c(const HeroArgs& a, hipStream_t s) {
  constexpr int wpw = 4;
  static_assert(wpw * kWave <= 256, "hero_walk_kernel is built for at most 256 threads");
  const int64_t blocks = (a.n_items + wpw - 1) / wpw;
  const size_t lds = size_t(wpw) * C * 2 * kHeroFloats * sizeof(float);
  if (blocks > 0)
    hipLaunchKernelGGL(hero_walk_kernel<C>, dim3(unsigned(blocks)), dim3(wpw * kWave), lds, s, a);
  const int64_t n_units = a.n_groups * C;
  if (n_units > 0) {
    const unsigned g = unsigned(n_units < (int64_t(1) << 20) ? n_units : (int64_t(1) << 20));
    hipLaunchKernelGGL(hero_convert_kernel<C>, dim3(g), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_hero(const HeroArgs& a, int C, hipStream_t s) {
  switch (C) {
    case 1: return launch_hero_c<1>(a, s);
    case 2: return launch_hero_c<2>(a, s);
    case 3: return launch_hero_c<3>(a, s);
    case 4: return launch_hero_c<4>(a, s);
    case 8: return launch_hero_c<8>(a, s);
    case 9: return launch_hero_c<9>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rw
