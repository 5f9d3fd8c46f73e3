// Dwivedi sampling in the mixture walk for gfx950: the zero-variance-based
// scheme of Krivanek and d'Eon ("A zero-variance-based sampling scheme for
// Monte Carlo subsurface scattering", SIGGRAPH 2014 Talks, after Dwivedi 1982),
// one of the two variance reductions the paper names beside its random walk
// (Sec. 2).
//
// At every scattering the walk picks, with probability q, the Dwivedi
// technique: a direction with density 1 / (2 pi lam (nu0 - mu_s)) in the
// cosine mu_s with the outward normal of the top surface, and a flight against
// sigma' = sigma_t (1 - mu_s / nu0), which favour flights back to the
// surface; otherwise the plain technique (Henyey-Greenstein direction, flight
// against sigma_t).  nu0 > 1 is the root of alpha nu atanh(1/nu) = 1, the
// decay constant of the diffusion mode of a half-space, lam =
// ln((nu0 + 1) / (nu0 - 1)).  One-sample MIS with the balance heuristic: the
// flight's end multiplies the weight by the true density of (direction,
// flight) over the two techniques' mixture, at most 1 / (1 - q).  With q = 1 in
// an isotropic medium the factors telescope and every exit weight is a
// function of the first collision's depth and the exit cosine alone.
//
// Work: one wavefront per work item (unit, chunk of paths), lanes taking the
// item's paths in turn; the weights vary from path to path (they can exceed
// 1), so the sums are FP64, gathered per wave in LDS and stored to the item's
// slot, then added up per unit in a fixed order by the convert kernel.
#include <hip/hip_runtime.h>

#include "../../include/rw.h"
#include "rw_device.hpp"
#include "rw_internal.hpp"

namespace rw {

// LDS table per medium (12 floats):
// {flight = ln2 / sigma_t, albedo, g, hq}, {sigma_t, nu0, lam log2(e), hgk},
// {1 / nu0, 1 / (2 pi lam), cumulative weight, (1 - g)^2}
constexpr int kDwFloats = 12;

// nu0 of an albedo clamped to [0.3, 1 - 1e-7]: bisection on x = 1/nu in
// (0, 1), where atanh(x) / x rises from 1 to infinity, in FP64.
__device__ double dwivedi_nu0(double alpha) {
  const double a = fmin(fmax(alpha, 0.3), 1.0 - 1e-7);
  double lo = 0.0, hi = 1.0;
  for (int i = 0; i < 200; ++i) {
    const double x = 0.5 * (lo + hi);
    if (x <= lo || x >= hi) break;
    const double f = atanh(x) / x;
    if (a * f < 1.0) lo = x;
    else hi = x;
  }
  return 2.0 / (lo + hi);
}

struct DwPath {
  float x, y, z, ux, uy, uz, W, A;
  int k;
  bool mixed;  // the current flight's direction was sampled (not the entry, not a reflection)
  bool dw;     // ... by the Dwivedi technique
  float p_hg, p_d, mu_s, sig_d;
};

// Load and check unit u's media into the wave's LDS table (lane k stages
// medium k).  Returns false (and raises the flag) for an invalid unit.
template <int K>
__device__ __forceinline__ bool stage_dwivedi(const DwivediArgs& a, int64_t u, float* tab,
                                              int lane) {
  const UnitParams<K> up = load_unit<K>(a.w, u);
  if (lane < K) {
    float s = up.sigma_t[0], al = up.alb[0], g = up.g[0], c = up.cum[0];
#pragma unroll
    for (int j = 1; j < K; ++j) {
      s = (lane == j) ? up.sigma_t[j] : s;
      al = (lane == j) ? up.alb[j] : al;
      g = (lane == j) ? up.g[j] : g;
      c = (lane == j) ? up.cum[j] : c;
    }
    const Medium m = make_medium(s, al, g);
    // nu0 and its derived constants, computed once per unit and medium
    const float4 dn = reinterpret_cast<const float4*>(a.nu)[u * K + lane];
    float* e = tab + lane * kDwFloats;
    e[0] = m.flight; e[1] = al; e[2] = g; e[3] = m.hq;
    e[4] = s;
    e[5] = dn.x;
    e[6] = dn.y;
    e[7] = (1.0f - g * g) * 0.07957747154594767f;  // (1 - g^2) / (4 pi)
    e[8] = dn.z;
    e[9] = dn.w;
    e[10] = c;
    e[11] = (1.0f - g) * (1.0f - g);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (!up.ok && lane == 0) atomicOr(a.w.flags, RW_FLAG_BAD_PARAMS);
  return up.ok;
}

// Per unit and medium: (nu0, lam log2(e), 1 / nu0, 1 / (2 pi lam)) of its
// albedo, [n_units][K] float4 (an invalid albedo gets the clamp's value; the
// walk kernel flags the unit)
template <int K>
__global__ void __launch_bounds__(256) dwivedi_nu_kernel(const DwivediArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n_units * K) return;
  const int64_t u = i / K;
  const int k = int(i - u * K);
  const float al = a.w.albedo[k * a.w.k_stride + u];
  const double nu = dwivedi_nu0(al == al ? double(al) : 0.5);
  const double lam = log((nu + 1.0) / (nu - 1.0));
  reinterpret_cast<float4*>(a.nu)[i] =
      make_float4(float(nu), float(lam * 1.4426950408889634), float(1.0 / nu),
                  float(1.0 / (2.0 * 3.141592653589793 * lam)));
}

// Henyey-Greenstein density per steradian from b = 1 + g^2 - 2 g cos(theta)
__device__ __forceinline__ float hg_density(float hgk, float b) {
  return hgk * __builtin_amdgcn_rcpf(b * __builtin_amdgcn_sqrtf(b));
}

// A path whose weight leaves [0, 2^64] (the FP32 range guard of the product of
// MIS factors, each at most 1 / (1 - q)) ends here and scores 0
constexpr int EV_WEIGHT_CAP = EV_CAP + 1;
constexpr float kDwWeightCap = 1.8446744e19f;

// One vertex (v >= 1) of a Dwivedi path.  Returns the vertex event.
__device__ __forceinline__ int dwivedi_step(DwPath& p, uint4 w, const float* tab, float q,
                                            const WalkGeom& geo) {
  const float* e = tab + p.k * kDwFloats;
  const float sig = e[4], nu0 = e[5], inv_nu0 = e[8];
  // flight: -ln(u0) / sigma (sigma' after a Dwivedi direction)
  const float fl = p.dw ? 0.69314718055994531f * __builtin_amdgcn_rcpf(p.sig_d) : e[0];
  const float s = -__builtin_amdgcn_logf(u01(w.x)) * fl;
  const float zn = fmaf(s, p.uz, p.z);
  const bool top = (p.uz < 0.0f) && (zn <= 0.0f);
  const bool bottom = geo.slab && (p.uz > 0.0f) && (zn >= geo.slab_mm);
  const bool hit = top || bottom;
  // The move and the MIS factor are the same arithmetic for a flight that
  // reaches a surface after l = db and one that collides after l = s, so all
  // lanes evaluate them together: true density over the mixture, divided
  // through by the plain technique's e^{-sigma l} (times sigma for a
  // collision), p_hg / (q p_d f e^{sigma mu_s l / nu0} + (1 - q) p_hg) with
  // f = sigma' / sigma after a collision and 1 at a surface
  const float zs = top ? 0.0f : geo.slab_mm;
  const float l = hit ? (zs - p.z) * __builtin_amdgcn_rcpf(p.uz) : s;
  p.x = fmaf(l, p.ux, p.x);
  p.y = fmaf(l, p.uy, p.y);
  p.z = hit ? zs : zn;
  if (p.mixed) {
    const float ex = __builtin_amdgcn_exp2f(sig * p.mu_s * l * inv_nu0 * 1.4426950408889634f);
    const float f = hit ? 1.0f : p.sig_d * __builtin_amdgcn_rcpf(sig);
    p.W *= p.p_hg * __builtin_amdgcn_rcpf(fmaf(q * p.p_d * f, ex, (1.0f - q) * p.p_hg));
    if (!(p.W <= kDwWeightCap)) return EV_WEIGHT_CAP;
  }
  if (hit) {
    p.mixed = false;
    p.dw = false;
    if (!geo.index_matched) {
      const float F = fresnel(fabsf(p.uz), geo.n_rel, geo.n_rel2);
      if (u01(w.w) < F) {
        p.uz = -p.uz;
        return EV_REFLECT;
      }
    }
    return top ? EV_EXIT_TOP : EV_EXIT_BOTTOM;
  }
  const float alb = e[1];
  p.A = fmaf(p.W, 1.0f - alb, p.A);
  p.W *= alb;
  if (p.W < geo.rr_weight) {
    if (u01(w.w) < geo.rr_survive) p.W *= geo.rr_boost;
    else return EV_RR_KILL;
  }
  // the technique of the next flight: the low 9 bits of the fourth word (the
  // roulette and Fresnel uniform uses its top 23)
  const float ut = (float(w.w & 0x1FFu) + 0.5f) * 0.001953125f;
  p.dw = ut < q;
  const float g = e[2];
  // Both techniques turn a reference direction by a polar cosine mu and an
  // azimuth: Henyey-Greenstein about the old direction, Dwivedi about the
  // outward normal (0, 0, -1) with cosine m = mu_s (there the frame of rotate
  // has the tangents (1, 0, 0) and (0, -1, 0), so the sine term changes sign
  // to give (st cos, st sin, -m)).  Only the cosine differs per technique; the
  // square root, the azimuth's sine and cosine, the turn and the
  // Henyey-Greenstein density are shared, so a wave with lanes of both
  // techniques evaluates them once.
  float mu, st2, omm = 0.0f;
  if (p.dw) {
    mu = nu0 - (nu0 + 1.0f) * __builtin_amdgcn_exp2f(-u01(w.y) * e[6]);
    st2 = fmaxf(0.0f, fmaf(-mu, mu, 1.0f));
  } else {
    float den;
    omm = hg_omm(g, e[3], u01(w.y), den);
    mu = 1.0f - omm;
    st2 = omm * (2.0f - omm);
  }
  const float st = __builtin_amdgcn_sqrtf(st2);
  const float u2 = u01(w.z);
  const float sp = st * __builtin_amdgcn_cosf(u2), sq = st * __builtin_amdgcn_sinf(u2);
  const float ox = p.ux, oy = p.uy, oz = p.uz;
  float nx = p.dw ? 0.0f : ox, ny = p.dw ? 0.0f : oy, nz = p.dw ? -1.0f : oz;
  rotate(nx, ny, nz, mu, sp, p.dw ? -sq : sq);
  // 1 + g^2 - 2 g cos(theta): from the turn's cosine for Henyey-Greenstein,
  // as (1 - g)^2 + 2 g (1 - mu) (no cancellation near mu = 1); from the cosine
  // between the old and the new direction for Dwivedi
  const float c = fmaf(nx, ox, fmaf(ny, oy, nz * oz));
  const float b = p.dw ? fmaf(-2.0f * g, c, fmaf(g, g, 1.0f)) : fmaf(2.0f * g, omm, e[11]);
  p.p_hg = hg_density(e[7], b);
  p.ux = nx;
  p.uy = ny;
  p.uz = nz;
  p.mu_s = -p.uz;
  p.p_d = e[9] * __builtin_amdgcn_rcpf(nu0 - p.mu_s);
  p.sig_d = sig * fmaf(-p.mu_s, inv_nu0, 1.0f);
  p.mixed = true;
  return EV_COLLIDE;
}

__device__ __forceinline__ void lds_addd(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// per-wave LDS: the medium table (K x 12 floats, padded to 8-byte words), then
// the sums [bins (n_bins+2) x (sum x, sum x^2) | sum x, sum x^2, T, A], then a
// ring of kDwRing top exits (radius, weight) tallied kWave at a time
inline __host__ __device__ int dwivedi_acc_words(int n_bins) { return 2 * (n_bins + 2) + 4; }
constexpr int kDwTableWords = kMaxMedia * kDwFloats / 2;
constexpr int kDwRing = kWave;

template <int K>
__global__ void __launch_bounds__(256) dwivedi_walk_kernel(const DwivediArgs a) {
  extern __shared__ double dw_lds[];
  const int lane = __lane_id();
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t item = int64_t(blockIdx.x) * (blockDim.x / kWave) + wid;
  if (item >= a.n_items) return;  // whole waves
  const int nb = a.w.geo.n_bins;
  const int acc_words = dwivedi_acc_words(nb);
  double* base = dw_lds + int64_t(wid) * (kDwTableWords + acc_words + kDwRing);
  float* tab = reinterpret_cast<float*>(base);
  double* acc = base + kDwTableWords;
  float2* ring = reinterpret_cast<float2*>(acc + acc_words);
  const int64_t ul = item / a.chunks_per_unit;
  const int64_t c = item - ul * a.chunks_per_unit;
  const int64_t u = ul;  // the call's units start at 0 of the media view
  const uint32_t pb = uint32_t(c * a.chunk);
  const uint32_t pe = uint32_t(min(int64_t(pb) + a.chunk, a.w.map.paths_uniform));
  for (int i = lane; i < acc_words; i += kWave) acc[i] = 0.0;
  double* slot = a.slots + item * int64_t(acc_words + 1);
  if (!stage_dwivedi<K>(a, u, tab, lane)) {
    for (int i = lane; i <= acc_words; i += kWave) slot[i] = 0.0;
    return;  // an invalid unit keeps zero tallies
  }
  const PhiloxKey ks = philox_schedule(a.w.key0, a.w.key1);
  const uint32_t ctr3 = uint32_t(uint64_t(a.w.unit_base) + uint64_t(u));
  const WalkGeom geo = a.w.geo;
  const float q = a.q;
  double* bins = acc;

  DwPath p;
  bool alive = false, capped = false, wcapped = false;
  uint32_t path = 0, v = 0, cursor = pb;
  uint64_t verts = 0;
  // per-lane sums of the item (x, x^2 of top exits, T, A); the radial bins
  // go to LDS (spread over the bins, so few lanes meet on one word)
  double rx = 0.0, rx2 = 0.0, rt = 0.0, ra = 0.0;
  // top exits wait in the ring and are tallied a full wave at a time: the
  // bin's logarithm and the FP64 sums then run on all lanes instead of on the
  // few that leave in a given step
  uint32_t rn = 0;
  auto flush_ring = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (uint32_t(lane) < rn) {
      const float2 r = ring[lane];
      const int b = radial_slot_r(r.x, geo);
      const double x = double(r.y);
      lds_addd(&bins[2 * b], x);
      lds_addd(&bins[2 * b + 1], x * x);
      rx += x;
      rx2 += x * x;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    rn = 0;
  };
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
        }
      }
      const uint32_t next = cursor + uint32_t(__popcll(idle));
      cursor = next < pe ? next : pe;
    }
    if (__ballot(alive) == 0) break;
    bool top_end = false;
    float top_r = 0.0f, top_w = 0.0f;
    // three vertex steps per pass of the regeneration and the ring (one,
    // two and four measured 5 %, 1 % and 1 % slower); a lane whose path ends
    // in an earlier step sits out the later ones
#pragma unroll
    for (int rep = 0; rep < 3; ++rep) {
      if (alive) {
        const uint4 w = philox(v, path, a.w.tag, ctr3, ks);
        if (v == 0) {
          // medium by the cumulative weights; pencil beam entering at r = 0
          const float u0 = u01(w.x);
          int k = 0;
#pragma unroll
          for (int j = 0; j < K - 1; ++j) k += (u0 >= tab[j * kDwFloats + 10]) ? 1 : 0;
          p.k = k;
          p.x = 0.0f; p.y = 0.0f; p.z = 0.0f;
          p.ux = 0.0f; p.uy = 0.0f; p.uz = 1.0f;
          p.W = geo.entry_weight;
          p.A = 0.0f;
          p.mixed = false;
          p.dw = false;
          p.p_hg = 0.0f; p.p_d = 0.0f; p.mu_s = 0.0f; p.sig_d = 0.0f;
          v = 1;
        } else {
          int ev = dwivedi_step(p, w, tab, q, geo);
          if (ev < EV_EXIT_TOP && v >= geo.max_vertices) {
            ev = EV_CAP;
            capped = true;
          }
          if (ev >= EV_EXIT_TOP) {
            alive = false;
            verts += v;
            wcapped |= ev == EV_WEIGHT_CAP;
            if (ev == EV_EXIT_TOP) {
              top_end = true;
              top_r = exit_radius(p.x, p.y);
              top_w = p.W;
            } else if (ev == EV_EXIT_BOTTOM) {
              rt += double(p.W);
            }
            ra += double(p.A);
          } else {
            ++v;
          }
        }
      }
    }
    const uint64_t tm = __ballot(top_end);
    if (tm != 0) {
      const uint32_t nt = uint32_t(__popcll(tm));
      if (rn + nt > uint32_t(kDwRing)) flush_ring();
      if (top_end)
        ring[rn + __builtin_amdgcn_mbcnt_hi(uint32_t(tm >> 32),
                                            __builtin_amdgcn_mbcnt_lo(uint32_t(tm), 0u))] =
            make_float2(top_r, top_w);
      rn += nt;
    }
  }
  flush_ring();
  // the item's sums to its slot (the lanes' sums reduced in a fixed order); the
  // vertex count after them
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int i = lane; i < 2 * (nb + 2); i += kWave) slot[i] = bins[i];
  uint64_t tv = verts;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    tv += __shfl_xor(tv, off, kWave);
    rx += __shfl_xor(rx, off, kWave);
    rx2 += __shfl_xor(rx2, off, kWave);
    rt += __shfl_xor(rt, off, kWave);
    ra += __shfl_xor(ra, off, kWave);
  }
  if (lane == 0) {
    slot[2 * (nb + 2)] = rx;
    slot[2 * (nb + 2) + 1] = rx2;
    slot[2 * (nb + 2) + 2] = rt;
    slot[2 * (nb + 2) + 3] = ra;
    slot[acc_words] = double(tv);
  }
  if (__any(capped) && lane == 0) atomicOr(a.w.flags, RW_FLAG_VERTEX_CAP);
  if (__any(wcapped) && lane == 0) atomicOr(a.w.flags, RW_FLAG_WEIGHT_CAP);
}

// Per unit: its items' slots added in a fixed order; R = (sum x, sum x^2, T,
// A), bins, vertices.  A block takes kDwConvWords words of one unit: thread
// (j, i) adds the unit's items c = i, i + kDwConvParts, ... for word j (loads of
// kDwConvWords consecutive words per item), and the kDwConvParts partial sums of a
// word are then added in i order.  Grid stride over (unit, word group).
constexpr int kDwConvWords = 32;
constexpr int kDwConvParts = 8;

__global__ void __launch_bounds__(kDwConvWords * kDwConvParts)
    dwivedi_convert_kernel(const DwivediArgs a) {
  __shared__ double part[kDwConvParts][kDwConvWords];
  const int nb2 = 2 * (a.w.geo.n_bins + 2);
  const int acc_words = nb2 + 4;
  const int64_t stride = acc_words + 1;
  const int64_t groups = (stride + kDwConvWords - 1) / kDwConvWords;
  const int j = threadIdx.x % kDwConvWords, i = threadIdx.x / kDwConvWords;
  for (int64_t bg = blockIdx.x; bg < a.n_units * groups; bg += gridDim.x) {
    const int64_t u = bg / groups;
    const int64_t wd = (bg - u * groups) * kDwConvWords + j;
    double s = 0.0;
    if (wd < stride) {
      const double* col = a.slots + u * a.chunks_per_unit * stride + wd;
      int64_t c = i;
      // four independent loads in flight, added in c order
      for (; c + 3 * kDwConvParts < a.chunks_per_unit; c += 4 * kDwConvParts) {
        const double x0 = col[c * stride], x1 = col[(c + kDwConvParts) * stride];
        const double x2 = col[(c + 2 * kDwConvParts) * stride];
        const double x3 = col[(c + 3 * kDwConvParts) * stride];
        s += x0;
        s += x1;
        s += x2;
        s += x3;
      }
      for (; c < a.chunks_per_unit; c += kDwConvParts) s += col[c * stride];
    }
    part[i][j] = s;
    __syncthreads();
    if (i == 0 && wd < stride) {
      double t = part[0][j];
#pragma unroll
      for (int k = 1; k < kDwConvParts; ++k) t += part[k][j];
      if (wd < nb2) a.w.out_bins[u * nb2 + wd] = t;
      else if (wd < acc_words) a.w.out_R[u * 4 + (wd - nb2)] = t;
      else a.w.out_vertices[u] = int64_t(t);
    }
    __syncthreads();
  }
}

int dwivedi_lds_bytes(int n_bins, int waves_per_wg) {
  return waves_per_wg * (kDwTableWords + dwivedi_acc_words(n_bins) + kDwRing) *
         int(sizeof(double));
}

int64_t dwivedi_slot_words(int n_bins) { return dwivedi_acc_words(n_bins) + 1; }

template <int K>
static hipError_t launch_dwivedi_k(const DwivediArgs& a, int wpw, hipStream_t s) {
  // the walk kernel is built for at most 256 threads per workgroup
  if (wpw < 1 || wpw * kWave > 256) return hipErrorInvalidValue;
  const int64_t blocks = (a.n_items + wpw - 1) / wpw;
  const size_t lds = size_t(dwivedi_lds_bytes(a.w.geo.n_bins, wpw));
  if (a.n_units > 0)
    hipLaunchKernelGGL(dwivedi_nu_kernel<K>, dim3(unsigned((a.n_units * K + 255) / 256)),
                       dim3(256), 0, s, a);
  if (blocks > 0)
    hipLaunchKernelGGL(dwivedi_walk_kernel<K>, dim3(unsigned(blocks)), dim3(wpw * kWave), lds, s,
                       a);
  if (a.n_units > 0) {
    const int64_t groups = (dwivedi_slot_words(a.w.geo.n_bins) + kDwConvWords - 1) / kDwConvWords;
    const int64_t n = a.n_units * groups;
    const unsigned g = unsigned(n < (int64_t(1) << 20) ? n : (int64_t(1) << 20));
    hipLaunchKernelGGL(dwivedi_convert_kernel, dim3(g), dim3(kDwConvWords * kDwConvParts), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_dwivedi(const DwivediArgs& a, int K, int waves_per_wg, hipStream_t s) {
  switch (K) {
    case 1: return launch_dwivedi_k<1>(a, waves_per_wg, s);
    case 2: return launch_dwivedi_k<2>(a, waves_per_wg, s);
    case 3: return launch_dwivedi_k<3>(a, waves_per_wg, s);
    case 4: return launch_dwivedi_k<4>(a, waves_per_wg, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rw
