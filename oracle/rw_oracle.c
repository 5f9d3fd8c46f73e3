/*
 * rw_oracle.c - FP64 CPU reference ("oracle") for the random-walk subsurface
 * transport through a mixture of K homogeneous media.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP implementation; both sides
 * implement the same written estimator independently.
 *
 * What is computed (paper, Sec. 4.1 "Subsurface Scattering by
 * Mixtures-of-Media"): the BSSRDF of a K-medium mixture is the w_k-weighted sum
 * of the per-medium path integrals (second form of eq. sss), and a random walk
 * realises it by choosing the medium once, before the walk starts, with
 * probability w_k (same section, last paragraph; Sec. 7 "Results", which also
 * states that the pdf of that choice cancels the weight).  Each per-medium walk
 * samples the path-integral contribution of eq. sss: transmittance
 * T = exp(-sigma_t s) between vertices and the phase function scaled by the
 * albedo at every scattering vertex.  Under normal incidence the result is the
 * radial profile R_d(r) = R * P_d(r) of eq. radsss, tallied here as the total
 * diffuse reflectance R and a histogram of exit radii.  The boundary is a
 * smooth Fresnel interface (Sec. 8, "Limitations").
 *
 * The paper fixes no walk details.  The readings used (written conventions,
 * identical on the GPU side):
 *   - pencil beam at r = 0 along +z (z = depth), path weight starts at
 *     1 - F(0); specular F(0) is not part of R.  Variant (the cosine-weighted
 *     lobe of Sec. 8): at r = 0, cos(theta_i) = sqrt(u1), phi = 2 pi u2 of
 *     vertex 0, refracted by Snell's law, weight 1 - F(theta_i);
 *   - medium k = first index with u0 < c_k (c = cumulative weights, c_{K-1}=1);
 *   - free flight s = -ln(u0)/sigma_t;  top hit when uz < 0 and z + s*uz <= 0;
 *   - boundary: unpolarised Fresnel, total internal reflection when
 *     n*sin(theta_i) >= 1, reflect when u3 < F (specular, uz -> -uz);
 *   - collision: W *= alpha (implicit capture), Russian roulette when
 *     W < rr_weight (survive when u3 < rr_survive, W /= rr_survive);
 *   - Henyey-Greenstein cos(theta) by inversion of its CDF with u1, azimuth
 *     phi = 2*pi*u2 measured from the first tangent of the Duff et al. (2017)
 *     orthonormal frame of the current direction;
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (vertex, path, stream tag, unit), one block of four words per
 *     vertex, word -> ((w >> 9) + 0.5) * 2^-23 in (0, 1);
 *   - exit radius binned in n_bins log-spaced bins over [r_min, r_max) with an
 *     underflow slot 0 and an overflow slot n_bins + 1.
 * The adjoint uses the score-function (likelihood-ratio) estimator of the
 * path density, evaluated by replaying the same random numbers.
 *
 * The same estimator also runs in the two-layer tissue of the paper's data
 * generator (Sec. 3: a top layer of given thickness over a semi-infinite
 * bottom layer, per-layer sigma_t, albedo, g and refractive index), see
 * walk_layers() for its readings at the interface.  Its adjoint scores each
 * layer with the flights, collisions and scatterings a path had in that
 * layer (the path density factorises over the vertices, and each factor
 * depends on one layer's parameters only).
 *
 * Dwivedi sampling (the variance reduction the paper names beside hero
 * wavelengths in Sec. 2; the zero-variance-based scheme of Krivanek and
 * d'Eon, "A zero-variance-based sampling scheme for Monte Carlo subsurface
 * scattering", SIGGRAPH 2014 Talks, after Dwivedi 1982) runs as a variant of
 * the mixture walk: see dwivedi_nu0() and walk() for its readings.
 *
 * Everything is FP64.  Threads split the paths of a unit into fixed ranges;
 * partial sums are merged in range order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_K 4
#define ORC_RANGE 16384 /* paths per task: fixed, so merging is deterministic */

/* ------------------------------------------------------------------------- */
/* Public structs (mirrored by oracle/oracle.py with ctypes)                  */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_media;      /* K, 1..4 */
  int32_t n_bins;       /* radial bins (slots 0 and n_bins+1 are under/overflow) */
  double n_rel;         /* refractive index of the medium over the outside */
  double slab_mm;       /* thickness; <= 0 means semi-infinite */
  double r_min_mm, r_max_mm;
  double rr_weight;     /* Russian roulette threshold; <= 0 disables it */
  double rr_survive;    /* survival probability of the roulette */
  int64_t max_vertices; /* vertex cap per path */
  int32_t analog;       /* 1: analog absorption, unit weights, no roulette */
  int32_t order_filter; /* > 0: tally only paths with this many collisions */
  int32_t incidence;    /* 0: normal pencil beam; 1: cosine-weighted lobe at r = 0 */
} orc_geometry;

/* per-unit tally layout of orc_forward: 8 doubles */
enum {
  T_SUMX = 0,    /* sum of contributions exiting the top surface */
  T_SUMX2 = 1,   /* sum of their squares */
  T_SUMT = 2,    /* weight leaving through the bottom of a slab */
  T_SUMA = 3,    /* absorbed weight */
  T_SPEC = 4,    /* analog mode: paths specularly reflected at entry */
  T_CAPPED = 5,  /* paths that hit the vertex cap */
  T_KILLED = 6,  /* paths ended by roulette */
  T_NEXIT = 7,   /* number of paths tallied at the top */
  T_NSLOTS = 8
};

/* path end kinds (also written to traces) */
enum {
  END_NONE = 0,
  END_EXIT_TOP = 1,
  END_EXIT_BOTTOM = 2,
  END_RR_KILLED = 3,
  END_CAPPED = 4,
  END_ABSORBED = 5,   /* analog only */
  END_SPECULAR = 6,   /* analog only */
  END_NO_BLOCKS = 7   /* traces that ran out of blocks */
};

/* trace event codes */
enum {
  EV_START = 0,
  EV_COLLIDE = 1,
  EV_REFLECT = 2,
  EV_EXIT_TOP = 3,
  EV_EXIT_BOTTOM = 4,
  EV_RR_KILL = 5,
  EV_CAP = 6,
  EV_ABSORB = 7,
  EV_CROSS = 8        /* two-layer walk: transmitted through the interface */
};

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 products with the    */
/* published multipliers, key bumped by the published Weyl constants.         */
/* ------------------------------------------------------------------------- */
static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* word -> uniform in (0,1): odd multiples of 2^-24, exact in FP32 and FP64 */
static double u01(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }

/* ------------------------------------------------------------------------- */
/* Physics pieces                                                              */
/* ------------------------------------------------------------------------- */

/* Unpolarised Fresnel reflectance for light inside the medium (index n
 * relative to the outside) hitting the surface with cos(theta_i) = cos_i.
 * Average of the s and p amplitude-squared coefficients; returns 1 under total
 * internal reflection (n*sin(theta_i) >= 1). */
static double fresnel(double cos_i, double n) {
  double sin_i2 = 1.0 - cos_i * cos_i;
  if (sin_i2 < 0.0) sin_i2 = 0.0;
  double sin_t2 = n * n * sin_i2;
  if (sin_t2 >= 1.0) return 1.0;
  double cos_t = sqrt(1.0 - sin_t2);
  double rs = (n * cos_i - cos_t) / (n * cos_i + cos_t);
  double rp = (cos_i - n * cos_t) / (cos_i + n * cos_t);
  return 0.5 * (rs * rs + rp * rp);
}

/* Henyey-Greenstein: cos(theta) by inverting the CDF of
 * p(mu) = (1 - g^2) / (2 (1 + g^2 - 2 g mu)^{3/2}) at u (textbook form). */
static double hg_cos(double g, double u) {
  double mu;
  if (fabs(g) < 1e-9) {
    mu = 2.0 * u - 1.0;
  } else {
    double t = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
    mu = (1.0 + g * g - t * t) / (2.0 * g);
  }
  if (mu > 1.0) mu = 1.0;
  if (mu < -1.0) mu = -1.0;
  return mu;
}

/* d ln p_HG(mu; g) / d g */
static double hg_dlog_dg(double g, double mu) {
  return -2.0 * g / (1.0 - g * g) + 3.0 * (mu - g) / (1.0 + g * g - 2.0 * g * mu);
}

/* Orthonormal frame (t1, t2, d) of a unit vector d (Duff, Burgess, Christensen,
 * Hery, Kensler, Liani, Villemin, "Building an Orthonormal Basis, Revisited",
 * JCGT 6(1), 2017). */
static void frame(const double d[3], double t1[3], double t2[3]) {
  double s = copysign(1.0, d[2]);
  double a = -1.0 / (s + d[2]);
  double b = d[0] * d[1] * a;
  t1[0] = 1.0 + s * d[0] * d[0] * a;
  t1[1] = s * b;
  t1[2] = -s * d[0];
  t2[0] = b;
  t2[1] = s + d[1] * d[1] * a;
  t2[2] = -d[1];
}

/* new direction at polar cosine mu from d and azimuth phi (radians) from t1 */
static void scatter_dir(double d[3], double mu, double phi) {
  double t1[3], t2[3];
  frame(d, t1, t2);
  double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  double a = st * cos(phi), b = st * sin(phi);
  double nd[3];
  for (int i = 0; i < 3; ++i) nd[i] = a * t1[i] + b * t2[i] + mu * d[i];
  d[0] = nd[0]; d[1] = nd[1]; d[2] = nd[2];
}

/* specular reflection off a plane z = const */
static void reflect(double d[3]) { d[2] = -d[2]; }

/* distance of a surface point from the entry point r = 0 */
static double exit_radius(const double p[3]) { return sqrt(p[0] * p[0] + p[1] * p[1]); }

/* radial slot: 0 underflow, 1..n_bins log bins, n_bins+1 overflow */
static int bin_slot(double r, const orc_geometry* g) {
  if (!(r >= g->r_min_mm)) return 0;
  if (r >= g->r_max_mm) return g->n_bins + 1;
  double t = log(r / g->r_min_mm) / log(g->r_max_mm / g->r_min_mm);
  int b = (int)floor(t * g->n_bins);
  if (b < 0) b = 0;
  if (b > g->n_bins - 1) b = g->n_bins - 1;
  return b + 1;
}

/* ------------------------------------------------------------------------- */
/* Dwivedi sampling                                                            */
/* ------------------------------------------------------------------------- */
/* Readings (Krivanek and d'Eon 2014; the paper only names the technique):
 *   - mu_s = -d_z, the cosine of a direction with the outward normal of the
 *     top surface (positive towards the surface);
 *   - nu0(alpha) > 1 is the root of alpha nu atanh(1/nu) = 1, the decay
 *     constant of the asymptotic (diffusion-regime) solution of isotropic
 *     transport in a half-space; computed from the single-scattering albedo
 *     clamped to [DW_ALB_MIN, DW_ALB_MAX] (the estimator stays unbiased for
 *     every nu0 > 1; the clamp only keeps the pdf below representable);
 *   - Dwivedi direction pdf (per steradian) p_D = 1 / (2 pi lam (nu0 - mu_s)),
 *     lam = ln((nu0 + 1) / (nu0 - 1)), sampled by inverting its CDF:
 *     mu_s = nu0 - (nu0 + 1) exp(-u1 lam), azimuth 2 pi u2 about the normal;
 *   - with it the flight is sampled against sigma' = sigma_t (1 - mu_s / nu0)
 *     (longer flights towards the surface, shorter away from it);
 *   - at every scattering one of two techniques is chosen: Dwivedi
 *     (direction and flight as above) with probability q, else the plain walk
 *     (Henyey-Greenstein direction, flight against sigma_t); the technique
 *     uniform comes from the low 9 bits of the vertex's fourth word, which the
 *     roulette and Fresnel uniform (its top 23 bits) does not use;
 *   - one-sample MIS with the balance heuristic: at the end of that flight the
 *     weight is multiplied by the true density of (direction, flight) over
 *     the two techniques' mixture,
 *       p_HG T / (q p_D T' + (1 - q) p_HG T),
 *     T = sigma_t e^{-sigma_t s}, T' = sigma' e^{-sigma' s} for a collision
 *     after s, and T = e^{-sigma_t l}, T' = e^{-sigma' l} for a flight that
 *     reaches a surface after l; so each factor is at most 1 / (1 - q);
 *   - the entry flight and flights after a surface reflection are plain
 *     (their direction is not sampled) and keep their weight. */
#define DW_ALB_MIN 0.3
#define DW_ALB_MAX (1.0 - 1e-7)

/* nu0 of the albedo, by bisection on x = 1/nu in (0, 1), where
 * atanh(x) / x rises from 1 to infinity */
static double dwivedi_nu0(double alpha) {
  const double a = fmin(fmax(alpha, DW_ALB_MIN), DW_ALB_MAX);
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

/* Henyey-Greenstein phase function per steradian at cos(theta) = c */
static double hg_pdf(double g, double c) {
  const double b = 1.0 + g * g - 2.0 * g * c;
  return (1.0 - g * g) / (4.0 * M_PI * b * sqrt(b));
}

/* Dwivedi direction pdf per steradian at mu_s */
static double dwivedi_pdf(double nu0, double lam, double mu_s) {
  return 1.0 / (2.0 * M_PI * lam * (nu0 - mu_s));
}

/* ------------------------------------------------------------------------- */
/* One path                                                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
  int K;
  double sigma_t[ORC_MAX_K], albedo[ORC_MAX_K], g[ORC_MAX_K], w[ORC_MAX_K];
  double cum[ORC_MAX_K];
  /* Dwivedi walk: nu0 of each medium and ln((nu0 + 1) / (nu0 - 1)) */
  double nu0[ORC_MAX_K], lam[ORC_MAX_K];
} unit_params;

typedef struct {
  /* Philox source */
  uint32_t key[2];
  uint32_t path, unit, tag;
  /* injected source (traces): words[v*4 + i] */
  const uint32_t* words;
  int64_t n_blocks; /* blocks available to the path (either source) */
} block_source;

typedef struct {
  int end;
  int k;
  int slot;
  double x;        /* contribution when the path leaves the top (or bottom) */
  double r;
  double absorbed;
  int64_t n_vert;
  int64_t n_coll;
  double L;        /* total length of all flight segments */
  double Sg;       /* sum of d ln p_HG / d g over the scattering vertices */
  /* two-layer walk: the same three sums per layer (0 top, 1 bottom) */
  int64_t n_coll_l[2];
  double L_l[2];
  double Sg_l[2];
} path_result;

/* fetch block v; returns 0 when an injected source has run out.  w3, when
 * not NULL, receives the raw fourth word (its low 9 bits, which u01 drops,
 * choose the sampling technique of the Dwivedi walk) */
static int get_block_w(const block_source* src, int64_t v, double u[4], uint32_t* w3) {
  uint32_t w[4];
  if (v >= src->n_blocks) return 0;
  if (src->words) {
    for (int i = 0; i < 4; ++i) w[i] = src->words[v * 4 + i];
  } else {
    uint32_t ctr[4] = {(uint32_t)v, src->path, src->tag, src->unit};
    philox4x32_10(ctr, src->key, w);
  }
  for (int i = 0; i < 4; ++i) u[i] = u01(w[i]);
  if (w3) *w3 = w[3];
  return 1;
}

static int get_block(const block_source* src, int64_t v, double u[4]) {
  return get_block_w(src, v, u, NULL);
}

static void put_event(double* ev, int64_t max_ev, int64_t idx, int code,
                      const double p[3], const double d[3], double W) {
  if (!ev || idx >= max_ev) return;
  double* e = ev + idx * 8;
  e[0] = code; e[1] = p[0]; e[2] = p[1]; e[3] = p[2];
  e[4] = d[0]; e[5] = d[1]; e[6] = d[2]; e[7] = W;
}

/* Entry at r = 0 through a surface of relative index n, from the words of
 * vertex 0: normal incidence transmits 1 - F(0); the cosine-weighted lobe
 * (Sec. 8, Limitations) draws cos(theta_i) = sqrt(u1), phi = 2 pi u2 outside,
 * refracts by Snell's law and transmits 1 - F(theta_i), where the Fresnel
 * reflectance of the entry equals that of the reverse crossing from inside at
 * the refracted angle.  Sets the direction d and the starting weight *W;
 * returns 1 when the analog estimator reflects the path specularly. */
static int enter(const orc_geometry* geo, double n, const double u[4], double d[3], double* W) {
  d[0] = 0.0; d[1] = 0.0; d[2] = 1.0;
  double F_in = ((n - 1.0) / (n + 1.0)) * ((n - 1.0) / (n + 1.0));
  if (geo->incidence == 1) {
    const double sin2_t = (1.0 - u[1]) / (n * n);
    if (sin2_t >= 1.0) {
      F_in = 1.0;
    } else {
      const double ct = sqrt(1.0 - sin2_t), st = sqrt(sin2_t);
      const double phi = 2.0 * M_PI * u[2];
      F_in = fresnel(ct, n);
      d[0] = st * cos(phi); d[1] = st * sin(phi); d[2] = ct;
    }
  }
  if (geo->analog) {
    *W = 1.0;
    return (geo->incidence == 1 ? u[3] : u[1]) < F_in;
  }
  *W = 1.0 - F_in;
  return 0;
}

/* Absorption at a collision with a medium of albedo alb: implicit capture
 * with Russian roulette, or the analog survival test.  Returns END_NONE when
 * the path goes on, else how it ended. */
static int absorb(const orc_geometry* geo, double alb, const double u[4], double* Wp,
                  path_result* res) {
  double W = *Wp;
  res->n_coll += 1;
  if (geo->analog) {
    if (!(u[3] < alb)) {
      res->absorbed += 1.0;
      return END_ABSORBED;
    }
  } else {
    res->absorbed += W * (1.0 - alb);
    W *= alb;
    if (geo->rr_weight > 0.0 && W < geo->rr_weight) {
      if (u[3] < geo->rr_survive) {
        W /= geo->rr_survive;
      } else {
        *Wp = 0.0;
        return END_RR_KILLED;
      }
    }
  }
  *Wp = W;
  return END_NONE;
}

/* A collision with a medium of albedo alb and anisotropy g: absorption, then
 * Henyey-Greenstein scattering of the direction d.  Returns END_NONE when the
 * path goes on, else how it ended. */
/* Henyey-Greenstein scattering of d by the words u1 (cosine) and u2
 * (azimuth); returns the cosine */
static double hg_scatter(double g, const double u[4], double d[3]) {
  const double mu = hg_cos(g, u[1]);
  scatter_dir(d, mu, 2.0 * M_PI * u[2]);
  return mu;
}

static int collide(const orc_geometry* geo, double alb, double g, const double u[4], double d[3],
                   double* Wp, path_result* res) {
  const int end = absorb(geo, alb, u, Wp, res);
  if (end != END_NONE) return end;
  const double mu = hg_scatter(g, u, d);
  res->Sg += hg_dlog_dg(g, mu);
  return END_NONE;
}

/* One path of the mixture walk.  dw_q > 0: Dwivedi sampling with technique
 * probability dw_q (the readings above; up->nu0/lam set); dw_q = 0: the plain
 * walk. */
/* A collision of the Dwivedi walk: implicit capture and roulette as in
 * collide(), then the technique choice and the new direction with the two
 * techniques' densities of it and the flight extinction sig_d of the next
 * flight (used when *dw). */
static int dwivedi_collide(const orc_geometry* geo, const unit_params* up, int k, double q,
                           const double u[4], uint32_t w3, double d[3], double* Wp,
                           path_result* res, int* dw, double* p_hg, double* p_d, double* mu_s,
                           double* sig_d) {
  const double g = up->g[k], nu0 = up->nu0[k], lam = up->lam[k];
  const int end = absorb(geo, up->albedo[k], u, Wp, res);
  if (end != END_NONE) return end;
  const double ut = ((double)(w3 & 0x1FFu) + 0.5) / 512.0;
  *dw = ut < q;
  if (*dw) {
    const double m = nu0 - (nu0 + 1.0) * exp(-u[1] * lam);
    const double phi = 2.0 * M_PI * u[2];
    const double st = sqrt(fmax(0.0, 1.0 - m * m));
    const double nd[3] = {st * cos(phi), st * sin(phi), -m};
    const double c = nd[0] * d[0] + nd[1] * d[1] + nd[2] * d[2];
    *p_hg = hg_pdf(g, c);
    d[0] = nd[0]; d[1] = nd[1]; d[2] = nd[2];
  } else {
    *p_hg = hg_pdf(g, hg_scatter(g, u, d));
  }
  *mu_s = -d[2];
  *p_d = dwivedi_pdf(nu0, lam, *mu_s);
  *sig_d = up->sigma_t[k] * (1.0 - *mu_s / nu0);
  return END_NONE;
}

static void walk(const unit_params* up, const orc_geometry* geo,
                 const block_source* src, path_result* res,
                 double* events, int64_t max_events, double dw_q) {
  const double n = geo->n_rel;
  const int slab = geo->slab_mm > 0.0;
  double u[4];
  uint32_t w3 = 0;
  memset(res, 0, sizeof(*res));
  res->slot = -1;

  /* vertex 0: medium choice (and the entry direction and analog specular test) */
  if (!get_block(src, 0, u)) { res->end = END_NO_BLOCKS; return; }
  int k = up->K - 1;
  for (int j = 0; j < up->K; ++j) {
    if (u[0] < up->cum[j]) { k = j; break; }
  }
  res->k = k;
  const double sig = up->sigma_t[k], alb = up->albedo[k], g = up->g[k];
  /* Dwivedi state of the current flight: mixed = its direction was sampled
   * (0 for the entry and after a reflection); dw = by the Dwivedi technique;
   * p_hg, p_d = both techniques' densities of that direction; mu_s, sig_d */
  int mixed = 0, dw = 0;
  double p_hg = 0.0, p_d = 0.0, mu_s = 0.0, sig_d = sig;

  double p[3] = {0.0, 0.0, 0.0};
  double d[3];
  double W;
  if (enter(geo, n, u, d, &W)) {
    res->end = END_SPECULAR;
    put_event(events, max_events, 0, EV_START, p, d, 0.0);
    return;
  }
  put_event(events, max_events, 0, EV_START, p, d, W);

  for (int64_t v = 1;; ++v) {
    if (v > geo->max_vertices) {
      res->end = END_CAPPED;
      put_event(events, max_events, v, EV_CAP, p, d, W);
      return;
    }
    if (!get_block_w(src, v, u, &w3)) { res->end = END_NO_BLOCKS; return; }
    res->n_vert = v;
    double s = -log(u[0]) / (dw ? sig_d : sig);

    /* boundary crossings along this flight */
    int hit = 0; /* 1 top, 2 bottom */
    double db = 0.0;
    if (d[2] < 0.0 && p[2] + s * d[2] <= 0.0) {
      hit = 1;
      db = -p[2] / d[2];
    } else if (slab && d[2] > 0.0 && p[2] + s * d[2] >= geo->slab_mm) {
      hit = 2;
      db = (geo->slab_mm - p[2]) / d[2];
    }

    if (hit) {
      res->L += db;
      p[0] += db * d[0];
      p[1] += db * d[1];
      p[2] = (hit == 1) ? 0.0 : geo->slab_mm;
      if (mixed) {
        /* the flight passed db: e^{-sigma_t db} over the mixture */
        W *= p_hg / (dw_q * p_d * exp(sig * mu_s * db / up->nu0[k]) + (1.0 - dw_q) * p_hg);
        mixed = 0;
        dw = 0;
      }
      double F = fresnel(fabs(d[2]), n);
      if (u[3] < F) {
        reflect(d);
        put_event(events, max_events, v, EV_REFLECT, p, d, W);
        continue;
      }
      res->x = W;
      if (hit == 1) {
        res->end = END_EXIT_TOP;
        res->r = exit_radius(p);
        res->slot = bin_slot(res->r, geo);
        put_event(events, max_events, v, EV_EXIT_TOP, p, d, W);
      } else {
        res->end = END_EXIT_BOTTOM;
        put_event(events, max_events, v, EV_EXIT_BOTTOM, p, d, W);
      }
      return;
    }

    /* collision */
    res->L += s;
    for (int i = 0; i < 3; ++i) p[i] += s * d[i];
    if (mixed) {
      /* a collision after s: sigma_t e^{-sigma_t s} over the mixture */
      W *= p_hg / (dw_q * p_d * (sig_d / sig) * exp(sig * mu_s * s / up->nu0[k]) +
                   (1.0 - dw_q) * p_hg);
    }
    if (dw_q > 0.0) {
      const int end = dwivedi_collide(geo, up, k, dw_q, u, w3, d, &W, res, &dw, &p_hg, &p_d,
                                      &mu_s, &sig_d);
      mixed = 1;
      if (end != END_NONE) {
        res->end = end;
        put_event(events, max_events, v, EV_RR_KILL, p, d, 0.0);
        return;
      }
      put_event(events, max_events, v, EV_COLLIDE, p, d, W);
      continue;
    }
    const int end = collide(geo, alb, g, u, d, &W, res);
    if (end != END_NONE) {
      res->end = end;
      put_event(events, max_events, v, end == END_ABSORBED ? EV_ABSORB : EV_RR_KILL, p, d,
                end == END_ABSORBED ? W : 0.0);
      return;
    }
    put_event(events, max_events, v, EV_COLLIDE, p, d, W);
  }
}

/* ------------------------------------------------------------------------- */
/* Two-layer tissue (Sec. 3): a top layer of thickness d over a bottom layer  */
/* that is semi-infinite (or ends at slab_mm for tests)                        */
/* ------------------------------------------------------------------------- */
typedef struct {
  double sigma_t[2], albedo[2], g[2]; /* layer 0 = top, 1 = bottom */
  double d;                           /* top-layer thickness, mm (> 0) */
  double n[2];                        /* indices relative to the outside */
} layer_params;

/* ------------------------------------------------------------------------- */
/* Hero wavelengths: one path serves a group of C wavelengths of one tissue     */
/* ------------------------------------------------------------------------- */
#define ORC_MAX_HERO 16

/* log of the Henyey-Greenstein density of mu = cos(theta) */
static double hg_log_pdf(double g, double mu) {
  return log(0.5 * (1.0 - g * g)) - 1.5 * log(1.0 + g * g - 2.0 * g * mu);
}

/* Hero-wavelength spectral sampling (Wilkie et al. 2014, the "hero
 * wavelength" tracking named in Sec. 2; Sec. 3's simulator propagates all its
 * wavelengths together) in the two-layer walk.  Group member `hero` samples
 * the path with its own optics: free flights from its sigma_t, scattering from
 * its Henyey-Greenstein g (the Fresnel and interface decisions depend on the
 * indices alone, which the group shares).  Every member i carries its own
 * weight x_i, multiplied by its albedo at each collision; Russian roulette
 * decides on the largest weight (a decision that does not depend on i, so it
 * leaves every weight unbiased) and boosts all of them.  The path density
 * under member i's optics is
 *   p_i = prod over layers of sigma_i^n_coll exp(-sigma_i L)
 *         x prod over scatterings of p_HG(mu; g_i)
 * times factors shared by all members, and with the hero chosen uniformly
 * (path index mod C) the one-sample balance-heuristic estimator of member i's
 * tally is F_i = C x_i p_i / sum_j p_j.  walk_layers runs this when given a
 * hero_walk; with C = 1 it is the plain walk. */
typedef struct {
  const layer_params* lps; /* the C members */
  int C, hero;
  double x[ORC_MAX_HERO];  /* weights */
  double hg[ORC_MAX_HERO]; /* sums of ln p_HG(mu; g_i) over the scatterings */
  double F[ORC_MAX_HERO];  /* contributions of a path that leaves (else 0) */
} hero_walk;

/* A collision in `layer` of a hero path: every member's weight times its
 * albedo, roulette on the largest weight, the hero's Henyey-Greenstein
 * scattering and every member's log phase density of it. */
static int collide_hero(const orc_geometry* geo, hero_walk* hw, int layer, const double u[4],
                        double d[3], path_result* res) {
  res->n_coll += 1;
  double xmax = 0.0;
  for (int i = 0; i < hw->C; ++i) {
    hw->x[i] *= hw->lps[i].albedo[layer];
    if (hw->x[i] > xmax) xmax = hw->x[i];
  }
  if (geo->rr_weight > 0.0 && xmax < geo->rr_weight) {
    if (u[3] < geo->rr_survive) {
      for (int i = 0; i < hw->C; ++i) hw->x[i] /= geo->rr_survive;
    } else {
      return END_RR_KILLED;
    }
  }
  const double mu = hg_cos(hw->lps[hw->hero].g[layer], u[1]);
  for (int i = 0; i < hw->C; ++i) hw->hg[i] += hg_log_pdf(hw->lps[i].g[layer], mu);
  const double phi = 2.0 * M_PI * u[2];
  scatter_dir(d, mu, phi);
  return END_NONE;
}

/* A hero path leaves: the balance-heuristic contributions of all members. */
static void exit_hero(hero_walk* hw, const path_result* res) {
  double lp[ORC_MAX_HERO], m = -INFINITY;
  for (int i = 0; i < hw->C; ++i) {
    lp[i] = hw->hg[i];
    for (int l = 0; l < 2; ++l)
      lp[i] += (double)res->n_coll_l[l] * log(hw->lps[i].sigma_t[l]) -
               hw->lps[i].sigma_t[l] * res->L_l[l];
    if (lp[i] > m) m = lp[i];
  }
  double S = 0.0;
  for (int i = 0; i < hw->C; ++i) S += exp(lp[i] - m);
  for (int i = 0; i < hw->C; ++i) hw->F[i] = (double)hw->C * hw->x[i] * exp(lp[i] - m) / S;
}

/* The same estimator as walk(), in layers.  Readings (identical on the GPU
 * side): the path enters the top layer through the surface of index n[0]; a
 * flight that reaches the interface z = d stops there (a vertex); the
 * interface reflects with the unpolarised Fresnel reflectance of the relative
 * index n_from / n_to (u3 < F), else the path crosses, refracted by Snell's
 * law, and the next flight is drawn afresh in the other layer (the free-flight
 * distribution is memoryless, so stopping at the interface does not change
 * the path density).  The bottom layer's lower face (slab tests) has index
 * n[1] over the outside.  For the adjoint the flight lengths, collisions and
 * g-score terms are also kept per layer (n_coll_l, L_l, Sg_l).  Given a
 * hero_walk (hw non-NULL), lp is its hero member and the collisions and the
 * exit follow the hero-wavelength estimator (collide_hero, exit_hero). */
static void walk_layers(const layer_params* lp, const orc_geometry* geo,
                        const block_source* src, path_result* res,
                        double* events, int64_t max_events, hero_walk* hw) {
  const int slab = geo->slab_mm > 0.0;
  double u[4];
  memset(res, 0, sizeof(*res));
  res->slot = -1;
  if (!get_block(src, 0, u)) { res->end = END_NO_BLOCKS; return; }
  double p[3] = {0.0, 0.0, 0.0};
  double d[3];
  double W;
  int layer = 0;
  res->k = layer;
  if (enter(geo, lp->n[0], u, d, &W)) {
    res->end = END_SPECULAR;
    put_event(events, max_events, 0, EV_START, p, d, 0.0);
    return;
  }
  if (hw) {
    for (int i = 0; i < hw->C; ++i) {
      hw->x[i] = W;
      hw->hg[i] = 0.0;
      hw->F[i] = 0.0;
    }
  }
  put_event(events, max_events, 0, EV_START, p, d, W);

  for (int64_t v = 1;; ++v) {
    if (v > geo->max_vertices) {
      res->end = END_CAPPED;
      put_event(events, max_events, v, EV_CAP, p, d, W);
      return;
    }
    if (!get_block(src, v, u)) { res->end = END_NO_BLOCKS; return; }
    res->n_vert = v;
    const double flight = -log(u[0]) / lp->sigma_t[layer];
    const double zn = p[2] + flight * d[2];

    /* which face of the current layer the flight reaches, if any:
     * 1 top surface, 2 interface, 3 bottom face of a slab */
    int face = 0;
    double zf = 0.0;
    if (layer == 0) {
      if (d[2] < 0.0 && zn <= 0.0) { face = 1; zf = 0.0; }
      else if (d[2] > 0.0 && zn >= lp->d) { face = 2; zf = lp->d; }
    } else {
      if (d[2] < 0.0 && zn <= lp->d) { face = 2; zf = lp->d; }
      else if (slab && d[2] > 0.0 && zn >= geo->slab_mm) { face = 3; zf = geo->slab_mm; }
    }

    if (face) {
      const double db = (zf - p[2]) / d[2];
      res->L_l[layer] += db;
      p[0] += db * d[0];
      p[1] += db * d[1];
      p[2] = zf;
      if (face == 2) {
        const double rel = lp->n[layer] / lp->n[1 - layer];
        if (u[3] < fresnel(fabs(d[2]), rel)) {
          reflect(d);
          put_event(events, max_events, v, EV_REFLECT, p, d, W);
          continue;
        }
        /* Snell: the tangential components scale by rel, the normal one
         * keeps its sign */
        const double sin2_t = rel * rel * (1.0 - d[2] * d[2]);
        const double ct = sqrt(fmax(0.0, 1.0 - sin2_t));
        d[0] *= rel;
        d[1] *= rel;
        d[2] = d[2] > 0.0 ? ct : -ct;
        layer = 1 - layer;
        res->k = layer;
        put_event(events, max_events, v, EV_CROSS, p, d, W);
        continue;
      }
      const double F = fresnel(fabs(d[2]), lp->n[layer]);
      if (u[3] < F) {
        reflect(d);
        put_event(events, max_events, v, EV_REFLECT, p, d, W);
        continue;
      }
      if (hw) {
        exit_hero(hw, res);
        W = hw->F[hw->hero];
      }
      res->x = W;
      if (face == 1) {
        res->end = END_EXIT_TOP;
        res->r = exit_radius(p);
        res->slot = bin_slot(res->r, geo);
        put_event(events, max_events, v, EV_EXIT_TOP, p, d, W);
      } else {
        res->end = END_EXIT_BOTTOM;
        put_event(events, max_events, v, EV_EXIT_BOTTOM, p, d, W);
      }
      return;
    }

    for (int i = 0; i < 3; ++i) p[i] += flight * d[i];
    res->L_l[layer] += flight;
    const int64_t nc0 = res->n_coll;
    const double sg0 = res->Sg;
    int end;
    if (hw) {
      end = collide_hero(geo, hw, layer, u, d, res);
      W = end == END_NONE ? hw->x[hw->hero] : 0.0;
    } else {
      end = collide(geo, lp->albedo[layer], lp->g[layer], u, d, &W, res);
    }
    res->n_coll_l[layer] += res->n_coll - nc0;
    res->Sg_l[layer] += res->Sg - sg0;
    if (end != END_NONE) {
      res->end = end;
      put_event(events, max_events, v, end == END_ABSORBED ? EV_ABSORB : EV_RR_KILL, p, d,
                end == END_ABSORBED ? W : 0.0);
      return;
    }
    put_event(events, max_events, v, EV_COLLIDE, p, d, W);
  }
}

/* ------------------------------------------------------------------------- */
/* Work split                                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
  const orc_geometry* geo;
  int K;
  const double *sigma_t, *albedo, *g, *w;
  int64_t n_units;
  const int64_t* paths;
  uint64_t seed;
  uint32_t tag;
  uint32_t unit_base; /* counter index of unit 0 (unit u draws as unit_base + u) */
  /* two-layer walk: thickness[n_units] of the top layer, index of the bottom
   * layer (the top layer's is geo->n_rel); sigma_t/albedo/g are [2][n_units] */
  int layered;
  const double* thickness;
  double n_bottom;
  /* hero-wavelength walk: groups of `hero` consecutive units (0: off); the
   * task table then runs over groups */
  int hero;
  /* Dwivedi walk: technique probability q (0: the plain walk) */
  double dwivedi;
  /* adjoint inputs (NULL for the forward) */
  int adjoint;
  const double* cot_R;
  const double* cot_bins;
  int want_jac;
  /* task table */
  int64_t n_tasks;
  int64_t* task_unit;
  int64_t* task_begin;
  int64_t* task_end;
  double* part;        /* n_tasks * part_len */
  int64_t part_len;
  int64_t next_task;
  pthread_mutex_t lock;
  int status;
} job_t;

static int load_unit(const job_t* job, int64_t u, unit_params* up) {
  int K = job->K;
  up->K = K;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    up->sigma_t[k] = job->sigma_t[(int64_t)k * job->n_units + u];
    up->albedo[k] = job->albedo[(int64_t)k * job->n_units + u];
    up->g[k] = job->g[(int64_t)k * job->n_units + u];
    up->w[k] = job->w[(int64_t)k * job->n_units + u];
    acc += up->w[k];
    up->cum[k] = acc;
  }
  up->cum[K - 1] = 1.0;
  for (int k = 0; k < K; ++k) {
    if (!(up->sigma_t[k] > 0.0) || !(up->albedo[k] >= 0.0) || !(up->albedo[k] <= 1.0) ||
        !(fabs(up->g[k]) < 1.0) || !(up->w[k] >= 0.0))
      return -1;
    if (job->dwivedi > 0.0) {
      up->nu0[k] = dwivedi_nu0(up->albedo[k]);
      up->lam[k] = log((up->nu0[k] + 1.0) / (up->nu0[k] - 1.0));
    }
  }
  if (!(fabs(acc - 1.0) <= 1e-5)) return -1;
  return 0;
}

static int load_layers(const job_t* job, int64_t u, layer_params* lp) {
  for (int k = 0; k < 2; ++k) {
    lp->sigma_t[k] = job->sigma_t[(int64_t)k * job->n_units + u];
    lp->albedo[k] = job->albedo[(int64_t)k * job->n_units + u];
    lp->g[k] = job->g[(int64_t)k * job->n_units + u];
    if (!(lp->sigma_t[k] > 0.0) || !(lp->albedo[k] >= 0.0) || !(lp->albedo[k] <= 1.0) ||
        !(fabs(lp->g[k]) < 1.0))
      return -1;
  }
  lp->d = job->thickness[u];
  lp->n[0] = job->geo->n_rel;
  lp->n[1] = job->n_bottom;
  if (!(lp->d > 0.0) || !(lp->d < 1e30)) return -1;
  if (job->geo->slab_mm > 0.0 && !(job->geo->slab_mm > lp->d)) return -1;
  return 0;
}

/* partial layout per task:
 *   forward: [T_NSLOTS] + bins[(nb+2)*2] + vertices(1)
 *   adjoint: grad[4K] + sumsq[4K] + (jac: jacR[4K] + jacB[(nb+2)*4K])      */
static void run_hero_task(job_t* job, int64_t t);

static void run_task(job_t* job, int64_t t) {
  if (job->hero > 0) {
    run_hero_task(job, t);
    return;
  }
  const orc_geometry* geo = job->geo;
  const int nb = geo->n_bins;
  const int K = job->K;
  const int P = 4 * K;
  int64_t u = job->task_unit[t];
  double* part = job->part + t * job->part_len;
  unit_params up;
  layer_params lp;
  if (job->layered ? load_layers(job, u, &lp) != 0 : load_unit(job, u, &up) != 0) {
    pthread_mutex_lock(&job->lock);
    job->status |= 1;
    pthread_mutex_unlock(&job->lock);
    return;
  }
  block_source src;
  memset(&src, 0, sizeof(src));
  src.key[0] = (uint32_t)job->seed;
  src.key[1] = (uint32_t)(job->seed >> 32);
  src.unit = (uint32_t)((uint64_t)job->unit_base + (uint64_t)u);
  src.tag = job->tag;
  src.n_blocks = INT64_MAX;
  double score[4 * ORC_MAX_K];
  for (int64_t pth = job->task_begin[t]; pth < job->task_end[t]; ++pth) {
    path_result r;
    src.path = (uint32_t)pth;
    if (job->layered) walk_layers(&lp, geo, &src, &r, NULL, 0, NULL);
    else walk(&up, geo, &src, &r, NULL, 0, job->dwivedi);
    int tallied_top = (r.end == END_EXIT_TOP) &&
                      (geo->order_filter <= 0 || r.n_coll == geo->order_filter);
    if (!job->adjoint) {
      double* tal = part;
      double* bins = part + T_NSLOTS;
      double* vert = bins + (int64_t)(nb + 2) * 2;
      if (tallied_top) {
        tal[T_SUMX] += r.x;
        tal[T_SUMX2] += r.x * r.x;
        tal[T_NEXIT] += 1.0;
        bins[r.slot * 2 + 0] += r.x;
        bins[r.slot * 2 + 1] += r.x * r.x;
      }
      if (r.end == END_EXIT_BOTTOM) tal[T_SUMT] += r.x;
      tal[T_SUMA] += r.absorbed;
      if (r.end == END_SPECULAR) tal[T_SPEC] += 1.0;
      if (r.end == END_CAPPED) tal[T_CAPPED] += 1.0;
      if (r.end == END_RR_KILLED) tal[T_KILLED] += 1.0;
      vert[0] += (double)r.n_vert;
    } else {
      if (!tallied_top || r.x == 0.0) continue;
      for (int j = 0; j < P; ++j) score[j] = 0.0;
      if (job->layered) {
        /* each layer scores the flights, collisions and scatterings the path
         * had in it; no mixture weights */
        for (int l = 0; l < 2; ++l) {
          score[l] = (double)r.n_coll_l[l] / lp.sigma_t[l] - r.L_l[l];
          score[K + l] = (r.n_coll_l[l] == 0) ? 0.0 : (double)r.n_coll_l[l] / lp.albedo[l];
          score[2 * K + l] = r.Sg_l[l];
        }
      } else {
        int k = r.k;
        score[k] = (double)r.n_coll / up.sigma_t[k] - r.L;
        score[K + k] = (r.n_coll == 0) ? 0.0 : (double)r.n_coll / up.albedo[k];
        score[2 * K + k] = r.Sg;
        for (int j = 0; j < K; ++j) score[3 * K + j] = (j == k ? 1.0 : 0.0) - up.w[j];
      }
      double cot = job->cot_R ? job->cot_R[u] : 0.0;
      if (job->cot_bins) cot += job->cot_bins[u * (nb + 2) + r.slot];
      double* grad = part;
      double* sumsq = part + P;
      for (int j = 0; j < P; ++j) {
        double c = r.x * cot * score[j];
        grad[j] += c;
        sumsq[j] += c * c;
      }
      if (job->want_jac) {
        double* jacR = part + 2 * P;
        double* jacB = jacR + P;
        for (int j = 0; j < P; ++j) {
          jacR[j] += r.x * score[j];
          jacB[(int64_t)r.slot * P + j] += r.x * score[j];
        }
      }
    }
  }
}

/* partial layout of a hero task (group q): per member i,
 *   [T_NSLOTS] + bins[(nb+2)*2] + vertices(1)
 * with the vertices of the paths whose hero member i was */
static void run_hero_task(job_t* job, int64_t t) {
  const orc_geometry* geo = job->geo;
  const int nb = geo->n_bins;
  const int C = job->hero;
  const int64_t q = job->task_unit[t];
  const int64_t stride = T_NSLOTS + (int64_t)(nb + 2) * 2 + 1;
  double* part = job->part + t * job->part_len;
  layer_params lps[ORC_MAX_HERO];
  for (int i = 0; i < C; ++i) {
    if (load_layers(job, q * C + i, &lps[i]) != 0 || lps[i].d != lps[0].d) {
      pthread_mutex_lock(&job->lock);
      job->status |= 1;
      pthread_mutex_unlock(&job->lock);
      return;
    }
  }
  block_source src;
  memset(&src, 0, sizeof(src));
  src.key[0] = (uint32_t)job->seed;
  src.key[1] = (uint32_t)(job->seed >> 32);
  src.unit = (uint32_t)((uint64_t)job->unit_base + (uint64_t)q);
  src.tag = job->tag;
  src.n_blocks = INT64_MAX;
  hero_walk hw;
  hw.lps = lps;
  hw.C = C;
  const double* F = hw.F;
  for (int64_t pth = job->task_begin[t]; pth < job->task_end[t]; ++pth) {
    path_result r;
    src.path = (uint32_t)pth;
    const int hero = (int)(pth % C);
    hw.hero = hero;
    walk_layers(&lps[hero], geo, &src, &r, NULL, 0, &hw);
    for (int i = 0; i < C; ++i) {
      double* tal = part + i * stride;
      double* bins = tal + T_NSLOTS;
      if (r.end == END_EXIT_TOP) {
        tal[T_SUMX] += F[i];
        tal[T_SUMX2] += F[i] * F[i];
        tal[T_NEXIT] += 1.0;
        bins[r.slot * 2 + 0] += F[i];
        bins[r.slot * 2 + 1] += F[i] * F[i];
      } else if (r.end == END_EXIT_BOTTOM) {
        tal[T_SUMT] += F[i];
      }
    }
    double* th = part + hero * stride;
    if (r.end == END_CAPPED) th[T_CAPPED] += 1.0;
    if (r.end == END_RR_KILLED) th[T_KILLED] += 1.0;
    th[T_NSLOTS + (nb + 2) * 2] += (double)r.n_vert;
  }
}

static void* worker(void* arg) {
  job_t* job = (job_t*)arg;
  for (;;) {
    pthread_mutex_lock(&job->lock);
    int64_t t = job->next_task++;
    pthread_mutex_unlock(&job->lock);
    if (t >= job->n_tasks) break;
    run_task(job, t);
  }
  return NULL;
}

/* Split the paths of n_owners owners (units, or groups of a hero walk) into
 * tasks of at most ORC_RANGE paths and run them on n_threads threads. */
static int run_job_groups(job_t* job, int64_t n_owners, int n_threads) {
  int64_t n_tasks = 0;
  for (int64_t u = 0; u < n_owners; ++u) {
    if (job->paths[u] < 0) return -1;
    n_tasks += (job->paths[u] + ORC_RANGE - 1) / ORC_RANGE;
  }
  job->n_tasks = n_tasks;
  job->task_unit = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_tasks + 1));
  job->task_begin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_tasks + 1));
  job->task_end = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_tasks + 1));
  job->part = (double*)calloc((size_t)(n_tasks + 1) * (size_t)job->part_len, sizeof(double));
  if (!job->task_unit || !job->task_begin || !job->task_end || !job->part) {
    free(job->task_unit); free(job->task_begin); free(job->task_end); free(job->part);
    return -2;
  }
  int64_t t = 0;
  for (int64_t u = 0; u < n_owners; ++u) {
    for (int64_t b = 0; b < job->paths[u]; b += ORC_RANGE) {
      job->task_unit[t] = u;
      job->task_begin[t] = b;
      job->task_end[t] = (b + ORC_RANGE < job->paths[u]) ? b + ORC_RANGE : job->paths[u];
      ++t;
    }
  }
  job->next_task = 0;
  job->status = 0;
  pthread_mutex_init(&job->lock, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  int started = 0;
  for (int i = 1; i < n_threads; ++i) {
    if (pthread_create(&th[i], NULL, worker, job) != 0) break;
    started = i;
  }
  worker(job);
  for (int i = 1; i <= started; ++i) pthread_join(th[i], NULL);
  pthread_mutex_destroy(&job->lock);
  return job->status ? -3 : 0;
}

static int run_job(job_t* job, int n_threads) { return run_job_groups(job, job->n_units, n_threads); }

static void free_job(job_t* job) {
  free(job->task_unit); free(job->task_begin); free(job->task_end); free(job->part);
}

static int check_geometry(const orc_geometry* g) {
  if (!g) return -1;
  if (g->n_media < 1 || g->n_media > ORC_MAX_K) return -1;
  if (g->n_bins < 1 || g->n_bins > 4096) return -1;
  if (!(g->r_min_mm > 0.0) || !(g->r_max_mm > g->r_min_mm)) return -1;
  if (!(g->n_rel > 0.0)) return -1;
  if (g->max_vertices < 1) return -1;
  if (g->incidence != 0 && g->incidence != 1) return -1;
  if (!g->analog && g->rr_weight > 0.0 && !(g->rr_survive > 0.0 && g->rr_survive <= 1.0))
    return -1;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Exported API                                                               */
/* ------------------------------------------------------------------------- */

/* Forward tallies.  Parameters are SoA [K][n_units].  Outputs (zero-filled
 * here):  tally[n_units][8] (layout T_*), bins[n_units][n_bins+2][2] (sum x,
 * sum x^2), vertices[n_units].  Returns 0, -1 bad arguments, -2 no memory,
 * -3 invalid unit parameters. */
int orc_forward(const orc_geometry* geo, const double* sigma_t, const double* albedo,
                const double* g, const double* w, int64_t n_units, const int64_t* paths,
                uint64_t seed, uint32_t tag, uint32_t unit_base, int n_threads, double* tally,
                double* bins, int64_t* vertices) {
  if (check_geometry(geo) || !sigma_t || !albedo || !g || !w || !paths || n_units < 0 ||
      !tally || !bins || !vertices)
    return -1;
  const int nb = geo->n_bins;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.geo = geo; job.K = geo->n_media;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g; job.w = w;
  job.n_units = n_units; job.paths = paths; job.seed = seed; job.tag = tag;
  job.unit_base = unit_base;
  job.part_len = T_NSLOTS + (int64_t)(nb + 2) * 2 + 1;
  int rc = run_job(&job, n_threads);
  if (rc == -1 || rc == -2) return rc;
  memset(tally, 0, sizeof(double) * (size_t)n_units * T_NSLOTS);
  memset(bins, 0, sizeof(double) * (size_t)n_units * (size_t)(nb + 2) * 2);
  for (int64_t u = 0; u < n_units; ++u) vertices[u] = 0;
  for (int64_t t = 0; t < job.n_tasks; ++t) {
    int64_t u = job.task_unit[t];
    const double* part = job.part + t * job.part_len;
    for (int i = 0; i < T_NSLOTS; ++i) tally[u * T_NSLOTS + i] += part[i];
    for (int i = 0; i < (nb + 2) * 2; ++i) bins[u * (nb + 2) * 2 + i] += part[T_NSLOTS + i];
    vertices[u] += (int64_t)part[T_NSLOTS + (nb + 2) * 2];
  }
  free_job(&job);
  return rc;
}

/* The forward of the mixture walk with Dwivedi sampling (technique
 * probability 0 < q < 1; see the readings above dwivedi_nu0).  Same tallies
 * and layout as orc_forward; the weights of the exiting paths now vary from
 * path to path.  Normal incidence, implicit capture only (no analog mode).
 * Returns as orc_forward. */
int orc_dwivedi_forward(const orc_geometry* geo, const double* sigma_t, const double* albedo,
                        const double* g, const double* w, int64_t n_units, const int64_t* paths,
                        uint64_t seed, uint32_t tag, uint32_t unit_base, double q, int n_threads,
                        double* tally, double* bins, int64_t* vertices) {
  if (check_geometry(geo) || geo->analog || geo->incidence != 0 || !(q > 0.0) || !(q <= 1.0) ||
      !sigma_t || !albedo || !g || !w || !paths || n_units < 0 || !tally || !bins || !vertices)
    return -1;
  const int nb = geo->n_bins;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.geo = geo; job.K = geo->n_media;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g; job.w = w;
  job.n_units = n_units; job.paths = paths; job.seed = seed; job.tag = tag;
  job.unit_base = unit_base;
  job.dwivedi = q;
  job.part_len = T_NSLOTS + (int64_t)(nb + 2) * 2 + 1;
  int rc = run_job(&job, n_threads);
  if (rc == -1 || rc == -2) return rc;
  memset(tally, 0, sizeof(double) * (size_t)n_units * T_NSLOTS);
  memset(bins, 0, sizeof(double) * (size_t)n_units * (size_t)(nb + 2) * 2);
  for (int64_t u = 0; u < n_units; ++u) vertices[u] = 0;
  for (int64_t t = 0; t < job.n_tasks; ++t) {
    int64_t u = job.task_unit[t];
    const double* part = job.part + t * job.part_len;
    for (int i = 0; i < T_NSLOTS; ++i) tally[u * T_NSLOTS + i] += part[i];
    for (int i = 0; i < (nb + 2) * 2; ++i) bins[u * (nb + 2) * 2 + i] += part[T_NSLOTS + i];
    vertices[u] += (int64_t)part[T_NSLOTS + (nb + 2) * 2];
  }
  free_job(&job);
  return rc;
}

/* nu0 of an albedo (the Dwivedi walk's constant), for tests */
double orc_dwivedi_nu0(double alpha) { return dwivedi_nu0(alpha); }

/* Score-function gradient of the cotangent-weighted top tallies:
 *   grad[u][j] = sum over paths of x * (cot_R[u] + cot_bins[u][slot]) * score_j
 * with score layout [sigma_t(K) | albedo(K) | g(K) | logits(K)] (logits of a
 * softmax that reproduces w).  grad_sumsq holds the sum of squares of the
 * per-path terms.  cot_bins may be NULL.  When jac_R / jac_bins are non-NULL
 * they receive the per-unit Jacobian sums sum x*score_j, for the total and per
 * slot ([n_units][4K] and [n_units][n_bins+2][4K]).  All sums are raw (not
 * divided by the path count). */
int orc_adjoint(const orc_geometry* geo, const double* sigma_t, const double* albedo,
                const double* g, const double* w, int64_t n_units, const int64_t* paths,
                uint64_t seed, uint32_t tag, uint32_t unit_base, int n_threads,
                const double* cot_R, const double* cot_bins, double* grad, double* grad_sumsq,
                double* jac_R, double* jac_bins) {
  if (check_geometry(geo) || !sigma_t || !albedo || !g || !w || !paths || n_units < 0 ||
      !grad || !grad_sumsq)
    return -1;
  if ((jac_R == NULL) != (jac_bins == NULL)) return -1;
  const int nb = geo->n_bins;
  const int P = 4 * geo->n_media;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.geo = geo; job.K = geo->n_media;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g; job.w = w;
  job.n_units = n_units; job.paths = paths; job.seed = seed; job.tag = tag;
  job.unit_base = unit_base;
  job.adjoint = 1; job.cot_R = cot_R; job.cot_bins = cot_bins;
  job.want_jac = jac_R != NULL;
  job.part_len = 2 * P + (job.want_jac ? P + (int64_t)(nb + 2) * P : 0);
  int rc = run_job(&job, n_threads);
  if (rc == -1 || rc == -2) return rc;
  memset(grad, 0, sizeof(double) * (size_t)n_units * P);
  memset(grad_sumsq, 0, sizeof(double) * (size_t)n_units * P);
  if (job.want_jac) {
    memset(jac_R, 0, sizeof(double) * (size_t)n_units * P);
    memset(jac_bins, 0, sizeof(double) * (size_t)n_units * (size_t)(nb + 2) * P);
  }
  for (int64_t t = 0; t < job.n_tasks; ++t) {
    int64_t u = job.task_unit[t];
    const double* part = job.part + t * job.part_len;
    for (int j = 0; j < P; ++j) {
      grad[u * P + j] += part[j];
      grad_sumsq[u * P + j] += part[P + j];
    }
    if (job.want_jac) {
      for (int j = 0; j < P; ++j) jac_R[u * P + j] += part[2 * P + j];
      for (int i = 0; i < (nb + 2) * P; ++i)
        jac_bins[u * (int64_t)(nb + 2) * P + i] += part[3 * P + i];
    }
  }
  free_job(&job);
  return rc;
}

/* Per-path replay with injected Philox output words (or Philox itself when
 * words == NULL, then path index p of unit `unit`); either way a path draws
 * at most n_blocks blocks and ends "out of blocks" after that.  One unit (parameters
 * sigma_t[K], albedo[K], g[K], w[K]).  words: [n_paths][n_blocks][4].
 * events: [n_paths][n_blocks][8] = (code, x, y, z, ux, uy, uz, W) per vertex,
 * zero-filled here; path_out: [n_paths][8] = (end, k, slot, x, r, n_vert,
 * n_coll, absorbed); path_adj: [n_paths][2] = (L, Sg) or NULL. */
int orc_trace(const orc_geometry* geo, const double* sigma_t, const double* albedo,
              const double* g, const double* w, const uint32_t* words, int64_t n_paths,
              int64_t n_blocks, uint64_t seed, uint32_t unit, uint32_t tag, double* events,
              double* path_out, double* path_adj, double dw_q) {
  if (check_geometry(geo) || !sigma_t || !albedo || !g || !w || n_paths < 0 ||
      n_blocks < 1 || !path_out || !(dw_q >= 0.0) || !(dw_q <= 1.0) ||
      (dw_q > 0.0 && (geo->analog || geo->incidence != 0)))
    return -1;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.K = geo->n_media; job.n_units = 1;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g; job.w = w;
  job.dwivedi = dw_q;
  unit_params up;
  if (load_unit(&job, 0, &up) != 0) return -3;
  if (events) memset(events, 0, sizeof(double) * (size_t)n_paths * (size_t)n_blocks * 8);
  for (int64_t p = 0; p < n_paths; ++p) {
    block_source src;
    memset(&src, 0, sizeof(src));
    src.key[0] = (uint32_t)seed;
    src.key[1] = (uint32_t)(seed >> 32);
    src.path = (uint32_t)p;
    src.unit = unit;
    src.tag = tag;
    src.n_blocks = n_blocks;
    if (words) src.words = words + p * n_blocks * 4;
    path_result r;
    walk(&up, geo, &src, &r, events ? events + p * n_blocks * 8 : NULL, n_blocks, dw_q);
    double* o = path_out + p * 8;
    o[0] = r.end; o[1] = r.k; o[2] = r.slot; o[3] = r.x; o[4] = r.r;
    o[5] = (double)r.n_vert; o[6] = (double)r.n_coll; o[7] = r.absorbed;
    if (path_adj) {
      path_adj[p * 2 + 0] = r.L;
      path_adj[p * 2 + 1] = r.Sg;
    }
  }
  return 0;
}

/* Two-layer forward tallies (Sec. 3 geometry), same outputs as orc_forward.
 * sigma_t/albedo/g: [2][n_units] (top, bottom); thickness: [n_units] top-layer
 * thickness in mm (> 0, below slab_mm when the bottom is a slab); n_bottom:
 * index of the bottom layer relative to the outside (the top layer's is
 * geo->n_rel; geo->n_media must be 2). */
int orc_layered_forward(const orc_geometry* geo, const double* sigma_t, const double* albedo,
                        const double* g, const double* thickness, double n_bottom,
                        int64_t n_units, const int64_t* paths, uint64_t seed, uint32_t tag,
                        uint32_t unit_base, int n_threads, double* tally, double* bins,
                        int64_t* vertices) {
  if (check_geometry(geo) || geo->n_media != 2 || !(n_bottom > 0.0) || !sigma_t || !albedo ||
      !g || !thickness || !paths || n_units < 0 || !tally || !bins || !vertices)
    return -1;
  const int nb = geo->n_bins;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.geo = geo; job.K = 2;
  job.layered = 1; job.thickness = thickness; job.n_bottom = n_bottom;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g;
  job.n_units = n_units; job.paths = paths; job.seed = seed; job.tag = tag;
  job.unit_base = unit_base;
  job.part_len = T_NSLOTS + (int64_t)(nb + 2) * 2 + 1;
  int rc = run_job(&job, n_threads);
  if (rc == -1 || rc == -2) return rc;
  memset(tally, 0, sizeof(double) * (size_t)n_units * T_NSLOTS);
  memset(bins, 0, sizeof(double) * (size_t)n_units * (size_t)(nb + 2) * 2);
  for (int64_t u = 0; u < n_units; ++u) vertices[u] = 0;
  for (int64_t t = 0; t < job.n_tasks; ++t) {
    int64_t u = job.task_unit[t];
    const double* part = job.part + t * job.part_len;
    for (int i = 0; i < T_NSLOTS; ++i) tally[u * T_NSLOTS + i] += part[i];
    for (int i = 0; i < (nb + 2) * 2; ++i) bins[u * (nb + 2) * 2 + i] += part[T_NSLOTS + i];
    vertices[u] += (int64_t)part[T_NSLOTS + (nb + 2) * 2];
  }
  free_job(&job);
  return rc;
}

/* Hero-wavelength two-layer walk: units in groups of C consecutive units
 * (u = q C + i; the members of a group share the top-layer thickness, and the
 * indices are the call's), paths[q] paths per group (a multiple of C), path p
 * of group q drawing from Philox counter (v, p, tag, unit_base + q) with hero
 * member p mod C.  Outputs per unit as orc_layered_forward (tally[T_SUMA] is
 * 0; vertices[u] counts the paths whose hero u was).  Returns -1 for bad
 * arguments (C outside 1..16, a path count not a multiple of C, analog mode),
 * -3 when a group's layers are invalid or their thicknesses differ. */
int orc_layered_hero_forward(const orc_geometry* geo, const double* sigma_t, const double* albedo,
                             const double* g, const double* thickness, double n_bottom,
                             int64_t n_units, int C, const int64_t* paths, uint64_t seed,
                             uint32_t tag, uint32_t unit_base, int n_threads, double* tally,
                             double* bins, int64_t* vertices) {
  if (check_geometry(geo) || geo->n_media != 2 || geo->analog || !(n_bottom > 0.0) || !sigma_t ||
      !albedo || !g || !thickness || !paths || n_units < 0 || !tally || !bins || !vertices ||
      C < 1 || C > ORC_MAX_HERO || n_units % C != 0)
    return -1;
  const int64_t n_groups = n_units / C;
  for (int64_t q = 0; q < n_groups; ++q)
    if (paths[q] % C != 0) return -1;
  const int nb = geo->n_bins;
  const int64_t stride = T_NSLOTS + (int64_t)(nb + 2) * 2 + 1;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.geo = geo; job.K = 2;
  job.layered = 1; job.thickness = thickness; job.n_bottom = n_bottom;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g;
  /* the task table runs over groups; load_layers reads unit q C + i of the
   * full arrays, so the SoA stride is the unit count */
  job.n_units = n_units;
  job.hero = C;
  job.paths = paths; job.seed = seed; job.tag = tag;
  job.unit_base = unit_base;
  job.part_len = (int64_t)C * stride;
  int rc = run_job_groups(&job, n_groups, n_threads);
  if (rc == -1 || rc == -2) return rc;
  memset(tally, 0, sizeof(double) * (size_t)n_units * T_NSLOTS);
  memset(bins, 0, sizeof(double) * (size_t)n_units * (size_t)(nb + 2) * 2);
  for (int64_t u = 0; u < n_units; ++u) vertices[u] = 0;
  for (int64_t t = 0; t < job.n_tasks; ++t) {
    const int64_t q = job.task_unit[t];
    const double* part = job.part + t * job.part_len;
    for (int i = 0; i < C; ++i) {
      const int64_t u = q * C + i;
      const double* pi = part + i * stride;
      for (int k = 0; k < T_NSLOTS; ++k) tally[u * T_NSLOTS + k] += pi[k];
      for (int k = 0; k < (nb + 2) * 2; ++k) bins[u * (nb + 2) * 2 + k] += pi[T_NSLOTS + k];
      vertices[u] += (int64_t)pi[T_NSLOTS + (nb + 2) * 2];
    }
  }
  free_job(&job);
  return rc;
}

/* Score-function gradient of the two-layer walk, the layered counterpart of
 * orc_adjoint: grad[n_units][8] = (sigma_t top, bottom, albedo top, bottom,
 * g top, bottom, 0, 0), raw sums over the paths leaving the top of
 * x * (cot_R + cot_bins[slot]) * score, each layer scored with the flights,
 * collisions and scatterings the path had in it. */
int orc_layered_adjoint(const orc_geometry* geo, const double* sigma_t, const double* albedo,
                        const double* g, const double* thickness, double n_bottom,
                        int64_t n_units, const int64_t* paths, uint64_t seed, uint32_t tag,
                        uint32_t unit_base, int n_threads, const double* cot_R,
                        const double* cot_bins, double* grad, double* grad_sumsq) {
  if (check_geometry(geo) || geo->n_media != 2 || !(n_bottom > 0.0) || !sigma_t || !albedo ||
      !g || !thickness || !paths || n_units < 0 || !grad || !grad_sumsq)
    return -1;
  const int P = 8;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.geo = geo; job.K = 2;
  job.layered = 1; job.thickness = thickness; job.n_bottom = n_bottom;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g;
  job.n_units = n_units; job.paths = paths; job.seed = seed; job.tag = tag;
  job.unit_base = unit_base;
  job.adjoint = 1; job.cot_R = cot_R; job.cot_bins = cot_bins;
  job.part_len = 2 * P;
  int rc = run_job(&job, n_threads);
  if (rc == -1 || rc == -2) return rc;
  memset(grad, 0, sizeof(double) * (size_t)n_units * P);
  memset(grad_sumsq, 0, sizeof(double) * (size_t)n_units * P);
  for (int64_t t = 0; t < job.n_tasks; ++t) {
    int64_t u = job.task_unit[t];
    const double* part = job.part + t * job.part_len;
    for (int j = 0; j < P; ++j) {
      grad[u * P + j] += part[j];
      grad_sumsq[u * P + j] += part[P + j];
    }
  }
  free_job(&job);
  return rc;
}

/* Per-path replay of one two-layer unit, as orc_trace (path_out[1] is the
 * layer the path ended in; EV_CROSS marks interface transmissions). */
int orc_layered_trace(const orc_geometry* geo, const double* sigma_t, const double* albedo,
                      const double* g, double thickness, double n_bottom, const uint32_t* words,
                      int64_t n_paths, int64_t n_blocks, uint64_t seed, uint32_t unit,
                      uint32_t tag, double* events, double* path_out) {
  if (check_geometry(geo) || geo->n_media != 2 || !(n_bottom > 0.0) || !sigma_t || !albedo ||
      !g || n_paths < 0 || n_blocks < 1 || !path_out)
    return -1;
  job_t job;
  memset(&job, 0, sizeof(job));
  job.geo = geo; job.K = 2; job.n_units = 1;
  job.layered = 1; job.thickness = &thickness; job.n_bottom = n_bottom;
  job.sigma_t = sigma_t; job.albedo = albedo; job.g = g;
  layer_params lp;
  if (load_layers(&job, 0, &lp) != 0) return -3;
  if (events) memset(events, 0, sizeof(double) * (size_t)n_paths * (size_t)n_blocks * 8);
  for (int64_t p = 0; p < n_paths; ++p) {
    block_source src;
    memset(&src, 0, sizeof(src));
    src.key[0] = (uint32_t)seed;
    src.key[1] = (uint32_t)(seed >> 32);
    src.path = (uint32_t)p;
    src.unit = unit;
    src.tag = tag;
    src.n_blocks = n_blocks;
    if (words) src.words = words + p * n_blocks * 4;
    path_result r;
    walk_layers(&lp, geo, &src, &r, events ? events + p * n_blocks * 8 : NULL, n_blocks, NULL);
    double* o = path_out + p * 8;
    o[0] = r.end; o[1] = r.k; o[2] = r.slot; o[3] = r.x; o[4] = r.r;
    o[5] = (double)r.n_vert; o[6] = (double)r.n_coll; o[7] = r.absorbed;
  }
  return 0;
}

/* Building blocks exported for their own pins. */
void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}
double orc_u01(uint32_t w) { return u01(w); }
double orc_fresnel(double cos_i, double n) { return fresnel(cos_i, n); }
double orc_hg_cos(double g, double u) { return hg_cos(g, u); }
double orc_hg_dlog_dg(double g, double mu) { return hg_dlog_dg(g, mu); }
void orc_frame(const double* d, double* t1, double* t2) { frame(d, t1, t2); }
void orc_scatter_dir(double* d, double mu, double phi) { scatter_dir(d, mu, phi); }
int orc_bin_slot(double r, const orc_geometry* geo) { return bin_slot(r, geo); }
