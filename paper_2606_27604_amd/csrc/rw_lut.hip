// Lookup-table fit (Sec. 4.2): the K-media profile of eq. mixture from the
// scale-independent tables R(alpha, g) and P_d(r | alpha, g) at sigma_t = 1,
// the per-unit loss of eq. joint_loss, its analytic gradient and an Adam step,
// fused in one kernel.  The shape term compares P_hat = sum_k w_k P_k, as
// defined after eq. refl_loss, or (shape_form = mixture) the normalised
// profile of eq. mixture, sum_k w_k R_k P_k / R_hat.
//
// One wavefront per unit; lanes stride over the evaluation radii.  Every
// per-radius term of the gradient is linear in the shape term's per-unit
// scale 1 / (n_bins_used * shape), so a single pass over the radii
// accumulates unscaled sums, which one set of wave reductions turns into the
// loss and the gradient (no per-radius storage, each table entry read once).
//
// Interpolation as a piecewise-linear function: the cell is the floor of the
// grid coordinate clamped to [0, n - 1] (and to n - 2 for the lower corner);
// the coordinate passes gradient only inside [0, n - 1].  The radial
// coordinate of sigma_t r is (log sigma_t + log r - log r_min) / step - 1/2
// (bin centres), and P is 0 off the table (half a bin beyond the outer
// centres, with a 1e-3 margin).
#include <hip/hip_runtime.h>

#include "../../include/rw.h"
#include "rw_internal.hpp"

namespace rw {

struct Cell {
  int i;       // lower corner
  float f;     // weight of the upper corner
  float dt;    // d coordinate / d input (0 where the coordinate was clamped)
};

__device__ __forceinline__ Cell grid_cell(float x, float scale, int n) {
  // coordinate t = x * scale on a grid of n points
  const float t = x * scale;
  const float hi = float(n - 1);
  Cell c;
  c.dt = (t >= 0.0f && t <= hi) ? scale : 0.0f;
  const float tc = fminf(fmaxf(t, 0.0f), hi);
  int i = int(floorf(tc));
  i = i < 0 ? 0 : (i > n - 2 ? n - 2 : i);
  c.i = i;
  c.f = tc - float(i);
  return c;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

template <int K>
__global__ void __launch_bounds__(256) lut_fit_kernel(const LutArgs a) {
  const int lane = __lane_id();
  const int64_t u = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (u >= a.n_units) return;  // whole waves
  const int64_t n = a.n_units;
  constexpr int P = 4 * K - 1;

  // physical parameters from the raw ones (identical in every lane)
  float la[K], sig[K], alb[K], sg[K], g[K], w[K];
  float lmax = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    la[k] = a.params[k * n + u];
    sig[k] = __expf(la[k]);
    alb[k] = 1.0f / (1.0f + __expf(-a.params[(K + k) * n + u]));
    sg[k] = 1.0f / (1.0f + __expf(-a.params[(2 * K + k) * n + u]));
    g[k] = 0.99f * sg[k];
    w[k] = k < K - 1 ? a.params[(3 * K + k) * n + u] : 0.0f;
    lmax = fmaxf(lmax, w[k]);
  }
  float wsum = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    w[k] = __expf(w[k] - lmax);
    wsum += w[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] /= wsum;

  // (alpha, g) cells, R_k by bilinear interpolation and its derivatives
  Cell ca[K], cg[K];
  float Rk[K], dRa[K], dRg[K];
  const float sa = float(a.n_alpha - 1) / a.alpha_max, sgc = float(a.n_g - 1) / a.g_max;
  float R_hat = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ca[k] = grid_cell(alb[k], sa, a.n_alpha);
    cg[k] = grid_cell(g[k], sgc, a.n_g);
    const float* T = a.R + int64_t(ca[k].i) * a.n_g + cg[k].i;
    const float r00 = T[0], r01 = T[1], r10 = T[a.n_g], r11 = T[a.n_g + 1];
    const float fa = ca[k].f, fg = cg[k].f;
    const float lo = (1.0f - fg) * r00 + fg * r01, hi = (1.0f - fg) * r10 + fg * r11;
    Rk[k] = (1.0f - fa) * lo + fa * hi;
    dRa[k] = (hi - lo) * ca[k].dt;                                   // d R_k / d alpha_k
    dRg[k] = ((1.0f - fa) * (r01 - r00) + fa * (r11 - r10)) * cg[k].dt;  // d R_k / d g_k
    R_hat += w[k] * Rk[k];
  }
  const float Rc = fmaxf(R_hat, 1e-12f);
  const float inv_Rc = 1.0f / Rc;
  // profile weights of the media: w_k (paper form) or w_k R_k / R_hat (mixture)
  const bool mix = a.shape_form == RW_LUT_SHAPE_MIXTURE;
  const float pnorm = mix ? inv_Rc : 1.0f;
  float cw[K];
#pragma unroll
  for (int k = 0; k < K; ++k) cw[k] = mix ? w[k] * Rk[k] : w[k];

  // one pass over the radii: loss sums and unscaled gradient sums
  float sum_d2 = 0.0f, cnt = 0.0f, s_rd = 0.0f;
  float A[K], Ba[K], Bb[K], Bc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) A[k] = Ba[k] = Bb[k] = Bc[k] = 0.0f;
  const int nb = a.n_bins;
  const int64_t plane = nb;
  for (int j = lane; j < a.n_r; j += kWave) {
    const float lr = __logf(a.r_mm[j]);
    float Pk[K], dPa[K], dPb[K], dPc[K];
    float Rd = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      // radial coordinate of sigma_t r among the bin centres
      const float tb = (la[k] + lr - a.log_rmin) * a.inv_step - 0.5f;
      const bool inside = tb >= -0.5f - 1e-3f && tb <= float(nb) - 0.5f + 1e-3f;
      const Cell cb = grid_cell(tb, 1.0f, nb);
      const float* Q = a.Pd + (int64_t(ca[k].i) * a.n_g + cg[k].i) * plane + cb.i;
      const float* Qa = Q + int64_t(a.n_g) * plane;  // alpha + 1
      const float p000 = Q[0], p001 = Q[1], p010 = Q[plane], p011 = Q[plane + 1];
      const float p100 = Qa[0], p101 = Qa[1], p110 = Qa[plane], p111 = Qa[plane + 1];
      const float fb = cb.f, fa = ca[k].f, fg = cg[k].f;
      const float c00 = (1.0f - fb) * p000 + fb * p001, c01 = (1.0f - fb) * p010 + fb * p011;
      const float c10 = (1.0f - fb) * p100 + fb * p101, c11 = (1.0f - fb) * p110 + fb * p111;
      const float lo = (1.0f - fg) * c00 + fg * c01, hi = (1.0f - fg) * c10 + fg * c11;
      const float val = (1.0f - fa) * lo + fa * hi;
      const float d00 = p001 - p000, d01 = p011 - p010, d10 = p101 - p100, d11 = p111 - p110;
      const float dfb = (1.0f - fa) * ((1.0f - fg) * d00 + fg * d01) + fa * ((1.0f - fg) * d10 + fg * d11);
      const float dfa = hi - lo;
      const float dfg = (1.0f - fa) * (c01 - c00) + fa * (c11 - c10);
      const float s2 = inside ? sig[k] * sig[k] : 0.0f;
      Pk[k] = s2 * val;
      // P = sigma^2 val(tb(log sigma)): d/d(log sigma) = sigma^2 (2 val + dval/dtb / step)
      dPa[k] = s2 * (2.0f * val + dfb * cb.dt * a.inv_step);
      dPb[k] = s2 * dfa * ca[k].dt;   // per unit of alpha
      dPc[k] = s2 * dfg * cg[k].dt;   // per unit of g
      Rd += cw[k] * Pk[k];
    }
    const float Pd = Rd * pnorm;
    const int64_t tj = u * a.n_r + j;
    float q = 0.0f;
    if (a.t_mass[tj] >= a.min_mass) {
      const float pt = a.t_Pd[tj];
      const float f = a.shape_floor * pt + 1e-12f;
      const float den = Pd + f;
      const float d = __logf(den) - __logf(pt + f);
      sum_d2 += d * d;
      cnt += 1.0f;
      q = d / den;
    }
    const float uq = q * pnorm;
    s_rd += q * Rd;  // the mixture form's dependence on R_hat
#pragma unroll
    for (int k = 0; k < K; ++k) {
      A[k] += uq * Pk[k];
      Ba[k] += uq * dPa[k];
      Bb[k] += uq * dPb[k];
      Bc[k] += uq * dPc[k];
    }
  }
  sum_d2 = wave_sum(sum_d2);
  cnt = wave_sum(cnt);
  s_rd = wave_sum(s_rd);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    A[k] = wave_sum(A[k]);
    Ba[k] = wave_sum(Ba[k]);
    Bb[k] = wave_sum(Bb[k]);
    Bc[k] = wave_sum(Bc[k]);
  }
  const float ncnt = fmaxf(cnt, 1.0f);
  const float shape = sqrtf(sum_d2 / ncnt + 1e-30f);
  const float scale = 1.0f / (ncnt * shape);
  const float dR = R_hat - a.t_R[u];
  const float loss = shape + a.lambda_R * dR * dR;
  // d L / d R_hat: the reflectance term, and in the mixture form the
  // normalisation of P_hat
  const float gRh =
      2.0f * a.lambda_R * dR - (mix && R_hat > 1e-12f ? scale * s_rd * inv_Rc * inv_Rc : 0.0f);

  float gr[P];
  float gw[K], wgw = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float sA = scale * A[k];
    // d L / d w_k and d L / d R_k; wr: d L / d P_k per unit of the radial sums
    gw[k] = (mix ? Rk[k] * sA : sA) + gRh * Rk[k];
    const float gRk = (mix ? w[k] * sA : 0.0f) + gRh * w[k];
    const float wr = cw[k] * scale;
    gr[k] = wr * Ba[k];                                                   // log sigma_t
    gr[K + k] = (wr * Bb[k] + gRk * dRa[k]) * alb[k] * (1.0f - alb[k]);   // logit alpha
    gr[2 * K + k] = (wr * Bc[k] + gRk * dRg[k]) * 0.99f * sg[k] * (1.0f - sg[k]);  // logit(g/0.99)
    wgw += w[k] * gw[k];
  }
#pragma unroll
  for (int k = 0; k < K - 1; ++k) gr[3 * K + k] = w[k] * (gw[k] - wgw);

  if (lane == 0 && a.loss) a.loss[u] = loss;
  if (a.grad) {
#pragma unroll
    for (int p = 0; p < P; ++p)
      if (lane == p) a.grad[p * n + u] = gr[p];
  }
  if (a.adam) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f / (1.0f - powf(b1, float(a.step)));
    const float c2 = 1.0f / (1.0f - powf(b2, float(a.step)));
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (lane == p) {
        const int64_t i = p * n + u;
        const float m = b1 * a.adam_m[i] + (1.0f - b1) * gr[p];
        const float v = b2 * a.adam_v[i] + (1.0f - b2) * gr[p] * gr[p];
        a.adam_m[i] = m;
        a.adam_v[i] = v;
        a.params_out[i] = a.params[i] - a.lr * (m * c1) / (sqrtf(v * c2) + eps);
      }
    }
  }
}

hipError_t launch_lut(const LutArgs& a, int K, hipStream_t s) {
  if (a.n_units <= 0) return hipSuccess;
  const int64_t blocks = (a.n_units * kWave + 255) / 256;
  const dim3 grid = dim3(unsigned(blocks)), block = dim3(256);
  switch (K) {
    case 1: hipLaunchKernelGGL(lut_fit_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(lut_fit_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(lut_fit_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(lut_fit_kernel<4>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rw
