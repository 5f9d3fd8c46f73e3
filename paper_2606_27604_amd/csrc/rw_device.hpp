// Device-side pieces of the random walk (gfx950, FP32 path arithmetic).
//
// The walk realises the paper's mixture-of-media BSSRDF (Sec. 4.1, second form
// of eq. sss): one medium is chosen per path with probability w_k, then the
// path samples the homogeneous path-integral contribution (transmittance
// exp(-sigma_t s), albedo-weighted Henyey-Greenstein scattering) under a smooth
// Fresnel surface (Sec. 8) for a normally incident beam (eq. radsss).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rw_internal.hpp"

namespace rw {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round is two
// 32x32->64 products (one v_mad_u64_u32 each) and two three-way XORs (one
// v_bitop3_b32 each).  The
// key schedule k + r * (0x9E3779B9, 0xBB67AE85) is wave-uniform; it is
// recomputed with scalar adds inside every call (the empty asm makes the base
// key opaque, so the compiler cannot hoist the ten round keys out of the walk
// loop, where they would occupy twenty scalar registers and spill).
// ---------------------------------------------------------------------------
struct PhiloxKey {
  uint32_t k0, k1;
};

__device__ __forceinline__ PhiloxKey philox_schedule(uint32_t k0, uint32_t k1) {
  return PhiloxKey{k0, k1};
}

// a ^ b ^ k in one instruction: gfx950's three-input bitwise operation with
// the truth table of a three-way XOR (0x96).  Left to itself the compiler
// emits two v_xor_b32 per three-way XOR, twenty per Philox block.  k must be
// wave-uniform (it is a round key): the operand is a scalar register.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        const PhiloxKey& key) {
  uint32_t k0 = key.k0, k1 = key.k1;
  asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c0;
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t n0 = xor3(uint32_t(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3(uint32_t(p0 >> 32), c3, k1);
    c1 = uint32_t(p1);
    c3 = uint32_t(p0);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// word -> uniform ((w >> 9) + 0.5) * 2^-23 in (0, 1): the mantissa trick gives
// 1 + m 2^-23 exactly, and the subtraction is exact (Sterbenz).
__device__ __forceinline__ float u01(uint32_t w) {
  return __uint_as_float(0x3f800000u | (w >> 9)) - (1.0f - 0x1p-24f);
}

// ---------------------------------------------------------------------------
// Per-medium constants of the chosen medium (selected per lane at path start).
// ---------------------------------------------------------------------------
struct Medium {
  float flight;  // ln(2) / sigma_t: s = -log2(u) * flight
  float inv_sig; // 1 / sigma_t (adjoint)
  float alb;     // albedo
  float g;
  float hq;             // 2 (1 - g)^2, Henyey-Greenstein inversion
  float gq;             // 3 / (1 - g^2)^2, for the g score (adjoint)
  float gc;             // -2 g / (1 - g^2): per-scattering constant of the g score
};

__device__ __forceinline__ Medium make_medium(float sigma_t, float alb, float g) {
  Medium m;
  m.inv_sig = 1.0f / sigma_t;
  m.flight = 0.69314718055994531f * m.inv_sig;
  m.alb = alb;
  m.g = g;
  m.hq = 2.0f * (1.0f - g) * (1.0f - g);
  const float omg2 = 1.0f - g * g;
  m.gq = 3.0f / (omg2 * omg2);
  m.gc = -2.0f * g / omg2;
  return m;
}

// Henyey-Greenstein 1 - cos(theta) from u, by inverting its CDF.  The textbook
// inversion mu = (1 + g^2 - tau^2) / (2g), tau = (1 - g^2) / (1 + g t),
// t = 2u - 1, cancels badly in FP32 for g near 1; factoring tau^2 - (1-g)^2
// gives the equivalent
//   1 - mu = 2 (1 - g)^2 (1 - u) (1 + g u) / (1 + g t)^2,
// a product of positive terms (accurate to a few ulp for every g and u, exact
// isotropic limit).  Also returns (1 + g t)^2, which equals
// (1 - g^2)^2 / (1 + g^2 - 2 g mu) and feeds the g score without a division.
__device__ __forceinline__ float hg_omm(float g, float hq, float u, float& den) {
  const float b = fmaf(g, fmaf(2.0f, u, -1.0f), 1.0f);
  den = b * b;
  return fminf(hq * (1.0f - u) * fmaf(g, u, 1.0f) * __builtin_amdgcn_rcpf(den), 2.0f);
}

// New direction mu u + p t1 + q t2 about u = (ux, uy, uz): polar cosine mu,
// (p, q) = sin(theta) (cos phi, sin phi) with the azimuth phi measured from the
// first tangent of the Duff et al. (JCGT 2017) frame:
// t1 = (1 + s ux^2 a, s ux uy a, -s ux), t2 = (ux uy a, s + uy^2 a, -uy) with
// s = sign(uz), a = -1/(s + uz).  Renormalised in FP32.
__device__ __forceinline__ void rotate(float& ux, float& uy, float& uz, float mu, float p,
                                       float q) {
  const float s = copysignf(1.0f, uz);
  const float a = -__builtin_amdgcn_rcpf(s + uz);
  const float b = ux * uy * a;
  const float t1x = fmaf(s * ux * ux, a, 1.0f), t1y = s * b, t1z = -s * ux;
  const float t2x = b, t2y = fmaf(uy * uy, a, s), t2z = -uy;
  float nx = fmaf(p, t1x, fmaf(q, t2x, mu * ux));
  float ny = fmaf(p, t1y, fmaf(q, t2y, mu * uy));
  float nz = fmaf(p, t1z, fmaf(q, t2z, mu * uz));
  // |n|^2 = mu^2 + sin^2(theta) = 1 up to rounding for a unit u, so one
  // Newton step of 1/sqrt from 1 renormalises to second order
  const float inv = fmaf(-0.5f, fmaf(nx, nx, fmaf(ny, ny, nz * nz)), 1.5f);
  ux = nx * inv;
  uy = ny * inv;
  uz = nz * inv;
}

// Unpolarised Fresnel reflectance for light inside the medium (index n
// relative to the outside) at cos(theta_i) = ci; 1 under total internal
// reflection.  Mean of the s and p amplitude-squared coefficients.
__device__ __forceinline__ float fresnel(float ci, float n, float n2) {
  const float st2 = n2 * fmaf(-ci, ci, 1.0f);
  if (st2 >= 1.0f) return 1.0f;
  const float ct = __builtin_amdgcn_sqrtf(1.0f - st2);
  const float nci = n * ci, nct = n * ct;
  // one reciprocal for both ratios (both denominators lie in (0, 2n + 2])
  const float ds = nci + ct, dp = ci + nct;
  const float inv = __builtin_amdgcn_rcpf(ds * dp);
  const float rs = (nci - ct) * dp * inv;
  const float rp = (ci - nct) * ds * inv;
  return 0.5f * fmaf(rs, rs, rp * rp);
}

// The same reflectance from both cosines: ci inside, co outside (Snell pair).
__device__ __forceinline__ float fresnel_pair(float ci, float co, float n) {
  const float nci = n * ci, nco = n * co;
  const float rs = (nci - co) * __builtin_amdgcn_rcpf(nci + co);
  const float rp = (ci - nco) * __builtin_amdgcn_rcpf(ci + nco);
  return 0.5f * fmaf(rs, rs, rp * rp);
}

// Radial slot of an exit radius: 0 below r_min, 1..n_bins, n_bins+1 at/above r_max.
template <class G>
__device__ __forceinline__ int radial_slot_r(float r, const G& geo) {
  if (!(r >= geo.r_min)) return 0;
  if (r >= geo.r_max) return geo.n_bins + 1;
  const float t = (__builtin_amdgcn_logf(r) - geo.log2_rmin) * geo.bin_scale;
  int b = int(t);
  b = b < 0 ? 0 : (b > geo.n_bins - 1 ? geo.n_bins - 1 : b);
  return b + 1;
}

__device__ __forceinline__ float exit_radius(float x, float y) {
  return __builtin_amdgcn_sqrtf(fmaf(x, x, y * y));
}

template <class G>
__device__ __forceinline__ int radial_slot(float x, float y, const G& geo) {
  return radial_slot_r(exit_radius(x, y), geo);
}

// The same value, held in a vector register.  The walk loop needs more
// wave-uniform constants than fit in scalar registers next to its control
// state; constants it reads as VALU operands cost nothing in vector registers,
// whereas spilled scalars are re-read with one v_readlane per use.
template <typename T>
__device__ __forceinline__ T in_vgpr(T x) {
  asm("" : "+v"(x));
  return x;
}

// The constants the vertex step reads, in vector registers; the rest of the
// geometry is read from LDS where it is needed (cold constants, below).
__device__ __forceinline__ WalkGeom step_geom_in_vgprs(const WalkGeom& g) {
  WalkGeom r = g;
  r.n_rel = in_vgpr(g.n_rel);
  r.n_rel2 = in_vgpr(g.n_rel2);
  r.slab_mm = in_vgpr(g.slab_mm);
  r.z_bottom = in_vgpr(g.z_bottom);
  r.rr_weight = in_vgpr(g.rr_weight);
  r.rr_survive = in_vgpr(g.rr_survive);
  r.rr_boost = in_vgpr(g.rr_boost);
  r.max_vertices = in_vgpr(g.max_vertices);
  return r;
}

// Constants needed only when a path starts or a batch of ends is tallied;
// the walk kernel keeps them in LDS (two 16-byte words).
struct ColdConst {
  float r_min, r_max, log2_rmin, bin_scale;
  int32_t n_bins;
  float entry_weight, fix_scale, fix_cap;
};

// ---------------------------------------------------------------------------
// Unit parameters (wave-uniform) and their device-side validation.
// ---------------------------------------------------------------------------
template <int K>
struct UnitParams {
  float sigma_t[K], alb[K], g[K], w[K], cum[K];
  bool ok;
};

template <int K>
__device__ __forceinline__ UnitParams<K> load_unit(const WalkArgs& a, int64_t u) {
  UnitParams<K> p;
  const int64_t n = a.k_stride;
  float wsum = 0.0f, wmax = -3.0e38f;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    p.sigma_t[k] = a.sigma_t[k * n + u];
    p.alb[k] = a.albedo[k * n + u];
    p.g[k] = a.g[k * n + u];
    p.w[k] = a.weight[k * n + u];
    ok = ok && (p.sigma_t[k] > 0.0f) && (p.sigma_t[k] < 3.0e38f) && (p.alb[k] >= 0.0f) &&
         (p.alb[k] <= 1.0f) && (fabsf(p.g[k]) < 1.0f);
    wmax = fmaxf(wmax, p.w[k]);
  }
  if (a.weights_are_logits) {
    ok = ok && (wmax < 3.0e38f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ok = ok && (p.w[k] == p.w[k]) && (p.w[k] < 3.0e38f) && (p.w[k] > -3.0e38f);
      p.w[k] = __expf(p.w[k] - wmax);
      wsum += p.w[k];
    }
    const float inv = 1.0f / wsum;
#pragma unroll
    for (int k = 0; k < K; ++k) p.w[k] *= inv;
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ok = ok && (p.w[k] >= 0.0f);
      wsum += p.w[k];
    }
    ok = ok && (fabsf(wsum - 1.0f) <= 1e-5f);
  }
  float c = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    c += p.w[k];
    p.cum[k] = c;
  }
  p.cum[K - 1] = 1.0f;
  p.ok = ok;
  return p;
}

// ---------------------------------------------------------------------------
// Path state and the two steps of the walk.
// ---------------------------------------------------------------------------
struct Path {
  float x, y, z, ux, uy, uz, W, A;
  Medium m;
  int k;
  // two-layer walk only: the other layer's medium (swapped with m at each
  // crossing, so a path never needs its unit's table again) and the depth of
  // the interface
  Medium m2;
  float d;
  // adjoint bookkeeping: collisions, D = sum over flights of (1/sigma_t - s)
  // for collisions and (-s) for boundary-terminated flights, which equals
  // n_coll / sigma_t - L without the cancellation of accumulating L; and the
  // part of the g score that depends on the sampled cosines
  uint32_t ncoll;
  float D, Sg;
  // two-layer adjoint: the same sums for the other layer (swapped with the
  // above at each crossing, like m and m2)
  uint32_t ncoll2;
  float D2, Sg2;
};

// Events of a vertex; the codes from EV_EXIT_TOP on end the path.  Traces
// report them in the oracle's numbering (trace_code).
enum VertexEvent : int {
  EV_START = 0,
  EV_COLLIDE = 1,
  EV_REFLECT = 2,
  EV_CROSS = 3,       // two-layer walk: transmitted through the interface
  EV_EXIT_TOP = 4,
  EV_EXIT_BOTTOM = 5,
  EV_RR_KILL = 6,
  EV_CAP = 7
};

__device__ __forceinline__ int trace_code(int ev) {
  // start, collide, reflect, cross, exit top, exit bottom, roulette, cap
  constexpr int kOracle[8] = {0, 1, 2, 8, 3, 4, 5, 6};
  return kOracle[ev];
}

// vertex 0 after the medium k has been chosen: pencil beam entering at the
// origin along +z with the transmitted weight 1 - F(0)
__device__ __forceinline__ void init_path(Path& p, int k, const Medium& m, float entry_weight) {
  p.k = k;
  p.m = m;
  p.x = 0.0f; p.y = 0.0f; p.z = 0.0f;
  p.ux = 0.0f; p.uy = 0.0f; p.uz = 1.0f;
  p.W = entry_weight;
  p.A = 0.0f;
  p.ncoll = 0;
  p.D = 0.0f;
  p.Sg = 0.0f;
  p.ncoll2 = 0;
  p.D2 = 0.0f;
  p.Sg2 = 0.0f;
}

// Entry through a cosine-weighted lobe (Sec. 8): cos(theta_i) = sqrt(u1) and
// azimuth 2 pi u2 outside, refracted by Snell's law (sin^2 theta_t =
// sin^2 theta_i / n^2), transmitted weight 1 - F: the Fresnel reflectance of
// the entry equals that of the reverse crossing from inside at theta_t.  F is
// taken from the drawn outside cosine sqrt(u1) itself rather than recomputed
// from theta_t, which near grazing incidence would cost FP32 digits.
template <class G>
__device__ __forceinline__ void cosine_entry(Path& p, uint4 w, const G& geo) {
  const float u1 = u01(w.y), u2 = u01(w.z);
  const float s2 = (1.0f - u1) * __builtin_amdgcn_rcpf(geo.n_rel2);
  if (s2 >= 1.0f) {  // no transmitted ray (outside denser than the medium)
    p.W = 0.0f;
    return;
  }
  const float ct = __builtin_amdgcn_sqrtf(1.0f - s2), st = __builtin_amdgcn_sqrtf(s2);
  p.W = 1.0f - fresnel_pair(ct, __builtin_amdgcn_sqrtf(u1), geo.n_rel);
  p.ux = st * __builtin_amdgcn_cosf(u2);  // cos(2 pi u2)
  p.uy = st * __builtin_amdgcn_sinf(u2);
  p.uz = ct;
}

// vertex 0: choose the medium from u0 (first k with u0 < cumulative weight)
template <int K>
__device__ __forceinline__ void start_path(Path& p, uint4 w, const UnitParams<K>& up,
                                           const WalkGeom& geo) {
  const float u0 = u01(w.x);
  int k = 0;
#pragma unroll
  for (int j = 0; j < K - 1; ++j) k += (u0 >= up.cum[j]) ? 1 : 0;
  float s = up.sigma_t[0], a = up.alb[0], g = up.g[0];
#pragma unroll
  for (int j = 1; j < K; ++j) {
    s = (k == j) ? up.sigma_t[j] : s;
    a = (k == j) ? up.alb[j] : a;
    g = (k == j) ? up.g[j] : g;
  }
  init_path(p, k, make_medium(s, a, g), geo.entry_weight);
  if (geo.incidence) cosine_entry(p, w, geo);
}

// The walk kernel keeps the current unit's media in LDS rather than in scalar
// registers (which the vertex loop needs for its own constants): per medium
// the eight floats {flight, alb, g, hq, inv_sig, gq, gc, 0}, then the
// cumulative weights.
template <int K>
__device__ __forceinline__ void stage_unit(const UnitParams<K>& up, float* tab, int lane) {
  if (lane < K) {
    float s = up.sigma_t[0], a = up.alb[0], g = up.g[0], c = up.cum[0];
#pragma unroll
    for (int j = 1; j < K; ++j) {
      s = (lane == j) ? up.sigma_t[j] : s;
      a = (lane == j) ? up.alb[j] : a;
      g = (lane == j) ? up.g[j] : g;
      c = (lane == j) ? up.cum[j] : c;
    }
    const Medium m = make_medium(s, a, g);
    float4* e = reinterpret_cast<float4*>(tab + lane * kMediumFloats);
    e[0] = make_float4(m.flight, m.alb, m.g, m.hq);
    e[1] = make_float4(m.inv_sig, m.gq, m.gc, 0.0f);
    tab[kMediumFloats * kMaxMedia + lane] = c;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int K>
__device__ __forceinline__ void start_path_lds(Path& p, uint4 w, const float* tab,
                                               float entry_weight, const WalkGeom& geo) {
  const float u0 = u01(w.x);
  int k = 0;
#pragma unroll
  for (int j = 0; j < K - 1; ++j) k += (u0 >= tab[kMediumFloats * kMaxMedia + j]) ? 1 : 0;
  const float4* e = reinterpret_cast<const float4*>(tab + k * kMediumFloats);
  const float4 e0 = e[0], e1 = e[1];
  Medium m;
  m.flight = e0.x; m.alb = e0.y; m.g = e0.z; m.hq = e0.w;
  m.inv_sig = e1.x; m.gq = e1.y; m.gc = e1.z;
  init_path(p, k, m, entry_weight);
  if (geo.incidence) cosine_entry(p, w, geo);
}

// The parts of a vertex fixed by its random words and the path's medium
// alone, not by the path's position or direction: the flight length s, the
// Henyey-Greenstein cosine mu with the g-score factor den, the components
// (p, q) = sin(theta) (cos phi, sin phi) of the new direction in the plane
// normal to the old one, and the word of the Fresnel / roulette decision.
struct VertexDraw {
  float s, mu, p, q, den;
  uint32_t w3;
};

__device__ __forceinline__ VertexDraw draw_vertex(float flight, float g, float hq, uint4 w) {
  VertexDraw d;
  d.s = -__builtin_amdgcn_logf(u01(w.x)) * flight;
  const float omm = hg_omm(g, hq, u01(w.y), d.den);
  // sin(theta) from (1 - mu)(1 + mu): no cancellation near mu = 1
  const float st = __builtin_amdgcn_sqrtf(omm * (2.0f - omm));
  d.mu = 1.0f - omm;
  const float u2 = u01(w.z);
  d.p = st * __builtin_amdgcn_cosf(u2);  // cos(2 pi u2)
  d.q = st * __builtin_amdgcn_sinf(u2);  // sin(2 pi u2)
  d.w3 = w.w;
  return d;
}

template <bool ADJ>
__device__ __forceinline__ int collide(Path& p, const VertexDraw& d, const WalkGeom& geo, float zn);

// vertex v >= 1: flight, then boundary interaction or collision.  Returns the
// vertex event.  ADJ adds the score bookkeeping (collisions, flight length,
// g score).
// Does a flight from depth z along uz to the new depth zn reach the top (or,
// for a slab, the bottom) surface?
__device__ __forceinline__ bool reaches_top(const Path& p, float zn) {
  return (p.uz < 0.0f) && (zn <= 0.0f);
}
__device__ __forceinline__ bool reaches_bottom(const Path& p, float zn, const WalkGeom& geo) {
  return geo.slab && (p.uz > 0.0f) && (zn >= geo.slab_mm);
}

template <bool ADJ>
__device__ __forceinline__ int vertex_step_drawn(Path& p, const VertexDraw& d, const WalkGeom& geo) {
  const float s = d.s;
  const float zn = fmaf(s, p.uz, p.z);
  const bool top = reaches_top(p, zn);
  const bool bottom = reaches_bottom(p, zn, geo);
  if (top || bottom) {
    const float db = (top ? -p.z : (geo.slab_mm - p.z)) * __builtin_amdgcn_rcpf(p.uz);
    p.x = fmaf(db, p.ux, p.x);
    p.y = fmaf(db, p.uy, p.y);
    p.z = top ? 0.0f : geo.slab_mm;
    if (ADJ) p.D -= db;
    if (!geo.index_matched) {
      const float F = fresnel(fabsf(p.uz), geo.n_rel, geo.n_rel2);
      if (u01(d.w3) < F) {
        p.uz = -p.uz;
        return EV_REFLECT;
      }
    }
    return top ? EV_EXIT_TOP : EV_EXIT_BOTTOM;
  }
  return collide<ADJ>(p, d, geo, zn);
}

template <bool ADJ>
__device__ __forceinline__ int vertex_step(Path& p, uint4 w, const WalkGeom& geo) {
  return vertex_step_drawn<ADJ>(p, draw_vertex(p.m.flight, p.m.g, p.m.hq, w), geo);
}

// Collision at the end of a flight of length s (new depth zn): implicit
// capture (A += W (1 - alpha), W *= alpha), roulette, Henyey-Greenstein
// scattering.
// The two halves of a collision around the roulette test: the move to the
// collision point with implicit capture, then the scattering.
// implicit capture at a collision after a flight of length s (the move made)
template <bool ADJ>
__device__ __forceinline__ void capture(Path& p, float s) {
  if (ADJ) {
    p.D += p.m.inv_sig - s;
    p.ncoll += 1;
  }
  p.A = fmaf(p.W, 1.0f - p.m.alb, p.A);
  p.W *= p.m.alb;
}

template <bool ADJ>
__device__ __forceinline__ void absorb_at(Path& p, const VertexDraw& d, float zn) {
  const float s = d.s;
  p.x = fmaf(s, p.ux, p.x);
  p.y = fmaf(s, p.uy, p.y);
  p.z = zn;
  capture<ADJ>(p, s);
}

template <bool ADJ>
__device__ __forceinline__ void scatter(Path& p, const VertexDraw& d) {
  if (ADJ) p.Sg = fmaf((d.mu - p.m.g) * d.den, p.m.gq, p.Sg);
  rotate(p.ux, p.uy, p.uz, d.mu, d.p, d.q);
}

template <bool ADJ>
__device__ __forceinline__ int collide(Path& p, const VertexDraw& d, const WalkGeom& geo, float zn) {
  absorb_at<ADJ>(p, d, zn);
  if (p.W < geo.rr_weight) {
    if (u01(d.w3) < geo.rr_survive) {
      p.W *= geo.rr_boost;
    } else {
      return EV_RR_KILL;
    }
  }
  scatter<ADJ>(p, d);
  return EV_COLLIDE;
}

// A vertex of the mixture walk that is a plain collision: the flight ends
// strictly between the top surface (z = 0) and z_bottom (the slab bottom, else
// +inf), and the new weight is at or above the roulette threshold.  For such
// a vertex vertex_step_drawn reduces to absorb_at then scatter, the same
// operations in the same order.  The test errs only towards the general
// step: a flight ending exactly on a surface is not taken as plain.
__device__ __forceinline__ bool plain_collision(const Path& p, const VertexDraw& d,
                                                const WalkGeom& geo, float& zn) {
  zn = fmaf(d.s, p.uz, p.z);
  // evaluated in full (no short circuit): it is tested by a ballot
  const int in = int(zn > 0.0f) & int(zn < geo.z_bottom) &
                 int(!(p.W * p.m.alb < geo.rr_weight));
  return in != 0;
}

// ---------------------------------------------------------------------------
// Two-layer tissue (Sec. 3): a top layer of thickness d over a bottom layer
// that is semi-infinite (or a slab, for tests).  A flight that reaches the
// interface stops there; the interface reflects with the unpolarised Fresnel
// reflectance of the relative index n_from / n_to, else the path crosses,
// refracted by Snell's law, and the next flight is drawn afresh in the other
// layer (free flights are memoryless).  The adjoint keeps the score sums of
// each layer: those of the current layer in (ncoll, D, Sg), the other's in
// (ncoll2, D2, Sg2), swapped at each crossing.
// ---------------------------------------------------------------------------
struct LayerParams {
  float sigma_t[2], alb[2], g[2];  // top, bottom
  float d;
  bool ok;
};

__device__ __forceinline__ LayerParams load_layers(const WalkArgs& a, int64_t u) {
  LayerParams p;
  const int64_t n = a.k_stride;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    p.sigma_t[k] = a.sigma_t[k * n + u];
    p.alb[k] = a.albedo[k * n + u];
    p.g[k] = a.g[k * n + u];
    ok = ok && (p.sigma_t[k] > 0.0f) && (p.sigma_t[k] < 3.0e38f) && (p.alb[k] >= 0.0f) &&
         (p.alb[k] <= 1.0f) && (fabsf(p.g[k]) < 1.0f);
  }
  p.d = a.layer_d[u];
  ok = ok && (p.d > 0.0f) && (p.d < 3.0e38f) && (!a.geo.slab || p.d < a.geo.slab_mm);
  p.ok = ok;
  return p;
}

// LDS table of a two-layer unit: the two media as in stage_unit, the
// interface depth in the spare fourth float of each entry's second word.
__device__ __forceinline__ void stage_layers(const LayerParams& lp, float* tab, int lane) {
  if (lane < 2) {
    const float s = lane ? lp.sigma_t[1] : lp.sigma_t[0];
    const float a = lane ? lp.alb[1] : lp.alb[0];
    const float g = lane ? lp.g[1] : lp.g[0];
    const Medium m = make_medium(s, a, g);
    float4* e = reinterpret_cast<float4*>(tab + lane * kMediumFloats);
    e[0] = make_float4(m.flight, m.alb, m.g, m.hq);
    e[1] = make_float4(m.inv_sig, m.gq, m.gc, lp.d);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ Medium medium_from_table(const float* tab, int k, float& d) {
  const float4* e = reinterpret_cast<const float4*>(tab + k * kMediumFloats);
  const float4 e0 = e[0], e1 = e[1];
  Medium m;
  m.flight = e0.x; m.alb = e0.y; m.g = e0.z; m.hq = e0.w;
  m.inv_sig = e1.x; m.gq = e1.y; m.gc = e1.z;
  d = e1.w;
  return m;
}

// vertex 0 of a two-layer path: the top layer, entered through the surface
__device__ __forceinline__ void start_path_layers(Path& p, uint4 w, const float* tab,
                                                  float entry_weight, const WalkGeom& geo) {
  float d;
  const Medium top = medium_from_table(tab, 0, d);
  p.m2 = medium_from_table(tab, 1, d);
  p.d = d;
  init_path(p, 0, top, entry_weight);
  if (geo.incidence) cosine_entry(p, w, geo);
}

// the same from parameters in registers (trace kernel)
__device__ __forceinline__ void start_path_layers(Path& p, uint4 w, const LayerParams& lp,
                                                  const WalkGeom& geo) {
  p.m2 = make_medium(lp.sigma_t[1], lp.alb[1], lp.g[1]);
  p.d = lp.d;
  init_path(p, 0, make_medium(lp.sigma_t[0], lp.alb[0], lp.g[0]), geo.entry_weight);
  if (geo.incidence) cosine_entry(p, w, geo);
}

// vertex v >= 1 of a two-layer path
template <bool ADJ>
__device__ __forceinline__ int vertex_step_layered(Path& p, uint4 w, const WalkGeom& geo) {
  const VertexDraw d = draw_vertex(p.m.flight, p.m.g, p.m.hq, w);
  const float s = d.s;
  const float zn = fmaf(s, p.uz, p.z);
  const bool top_layer = p.k == 0;
  // the face of the current layer this flight reaches: 1 surface, 2 interface,
  // 3 the bottom of a slab
  int face = 0;
  if (top_layer) {
    if (p.uz < 0.0f && zn <= 0.0f) face = 1;
    else if (p.uz > 0.0f && zn >= p.d) face = 2;
  } else {
    if (p.uz < 0.0f && zn <= p.d) face = 2;
    else if (geo.slab && p.uz > 0.0f && zn >= geo.slab_mm) face = 3;
  }
  // the move is the same arithmetic for a flight that reaches a face after
  // l = db and one that collides after l = s, so all lanes make it together
  const float zf = face == 1 ? 0.0f : (face == 2 ? p.d : geo.slab_mm);
  const float l = face != 0 ? (zf - p.z) * __builtin_amdgcn_rcpf(p.uz) : s;
  p.x = fmaf(l, p.ux, p.x);
  p.y = fmaf(l, p.uy, p.y);
  p.z = face != 0 ? zf : zn;
  if (face == 0) {
    capture<ADJ>(p, s);
    if (p.W < geo.rr_weight) {
      if (u01(d.w3) < geo.rr_survive) {
        p.W *= geo.rr_boost;
      } else {
        return EV_RR_KILL;
      }
    }
    scatter<ADJ>(p, d);
    return EV_COLLIDE;
  }
  if (ADJ) p.D -= l;
  if (face == 2) {
    if (!geo.interface_matched) {
      const float rel = top_layer ? geo.rel_down : geo.rel_up;
      const float rel2 = top_layer ? geo.rel_down2 : geo.rel_up2;
      if (u01(w.w) < fresnel(fabsf(p.uz), rel, rel2)) {
        p.uz = -p.uz;
        return EV_REFLECT;
      }
      // Snell: tangential components scale by rel, the normal one keeps its sign
      const float ct = __builtin_amdgcn_sqrtf(fmaxf(0.0f, fmaf(-rel2, fmaf(-p.uz, p.uz, 1.0f), 1.0f)));
      p.ux *= rel;
      p.uy *= rel;
      p.uz = p.uz > 0.0f ? ct : -ct;
    }
    const Medium other = p.m2;
    p.m2 = p.m;
    p.m = other;
    p.k ^= 1;
    if (ADJ) {
      const uint32_t n = p.ncoll2;
      p.ncoll2 = p.ncoll;
      p.ncoll = n;
      const float D = p.D2;
      p.D2 = p.D;
      p.D = D;
      const float Sg = p.Sg2;
      p.Sg2 = p.Sg;
      p.Sg = Sg;
    }
    return EV_CROSS;
  }
  const bool top = face == 1;
  if (!(top ? geo.index_matched : geo.bot_matched)) {
    const float F = top ? fresnel(fabsf(p.uz), geo.n_rel, geo.n_rel2)
                        : fresnel(fabsf(p.uz), geo.n_bot, geo.n_bot2);
    if (u01(w.w) < F) {
      p.uz = -p.uz;
      return EV_REFLECT;
    }
  }
  return top ? EV_EXIT_TOP : EV_EXIT_BOTTOM;
}

}  // namespace rw
