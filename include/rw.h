/*
 * rw.h - C ABI of the MI355X (gfx950) random-walk subsurface transport through
 * a mixture of K homogeneous media.
 *
 * The operation (paper Sec. 4.1, "Subsurface Scattering by Mixtures-of-Media"):
 * the BSSRDF of a mixture is the w_k-weighted sum of the per-medium path
 * integrals (second form of eq. sss); a random walk realises it by choosing
 * the medium k with probability w_k once, before the walk starts (same
 * section, and Sec. 7 "Results": the choice pdf cancels the weight).  Under
 * normal incidence the BSSRDF is radial, R_d(r) = R * P_d(r) (eq. radsss),
 * so each (parameter set, wavelength) "unit" yields the total diffuse
 * reflectance R and a radial histogram.  The per-wavelength parameters are
 * theta(lambda) = {alpha_k, g_k, sigma_t_k, w_k} (Sec. 5.1, eq.
 * decoder_output); the boundary is a smooth Fresnel interface (Sec. 8,
 * "Limitations").
 *
 * Walk conventions (the paper fixes none; identical in the FP64 oracle):
 *   z is depth, the medium fills z >= 0 (and z <= slab_mm for a slab); the
 *   beam enters at r = 0 along +z with weight 1 - F(0), F(0) = ((n-1)/(n+1))^2
 *   (the specular part is not in R).  Per path, Philox4x32-10 (Salmon et al.,
 *   SC'11) with key = seed and counter = (vertex, path, stream tag, unit)
 *   gives one block of four words per vertex; word w -> ((w >> 9) + 0.5) 2^-23.
 *   Vertex 0: medium = first k with u0 < cumulative weight.  Vertex v >= 1:
 *   flight s = -ln(u0)/sigma_t; when it crosses the surface the photon moves
 *   there and reflects (uz -> -uz) with the unpolarised Fresnel probability
 *   (u3 < F, total internal reflection when n sin(theta_i) >= 1), else
 *   leaves and its weight is tallied at r = hypot(x, y); otherwise it
 *   collides: W *= alpha, Russian roulette when W < rr_weight (survive when
 *   u3 < rr_survive, W /= rr_survive), Henyey-Greenstein cosine from u1 and
 *   azimuth 2 pi u2 measured from the first tangent of the Duff et al. (2017)
 *   frame of the current direction.  One loop iteration is one "vertex".
 *   Radial slots: 0 for r < r_min, 1..n_bins for log-spaced bins over
 *   [r_min, r_max), n_bins + 1 for r >= r_max.
 *
 * All entry points are asynchronous on the given HIP stream (passed as
 * void*, i.e. a hipStream_t; NULL is the null stream) and return once the
 * work is enqueued; back-to-back batched calls with the same launch shape
 * replay a ring of graph instantiations and do not wait for each other.  The
 * exceptions: rw_check synchronises by definition; the first batched call
 * with autotune = 1 on a new shape times candidate launches; a call that
 * needs more workspace than the context holds waits for the device before it
 * frees the smaller buffer.  Host-side argument checks return RW_E_INVALID before
 * anything is enqueued.  Per-unit parameter checks run on the device and set
 * bits in flags[0] (RW_FLAG_*); rw_check() synchronises and reports them.
 * Device pointers are caller-owned; the library never allocates caller-visible
 * memory.  A context owns its workspace, tuned launch shapes and captured
 * graphs; one context per stream, not thread-safe.
 */
#ifndef RW_H
#define RW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RW_OK = 0,
  RW_E_INVALID = 1,     /* bad argument (null pointer, size, geometry) */
  RW_E_HIP = 2,         /* a HIP runtime call failed */
  RW_E_NOMEM = 3,       /* workspace allocation failed */
  RW_E_UNSUPPORTED = 4, /* valid but not supported (e.g. K > 4) */
  RW_E_DEVICE_FLAG = 5  /* a device-side check raised a flag (rw_check) */
} rw_status;

/* device flag bits written to flags[0] */
#define RW_FLAG_BAD_PARAMS 1   /* a unit had sigma_t <= 0, alpha not in [0,1], |g| >= 1,
                                  a negative weight, weights not summing to 1 (+-1e-5)
                                  or a NaN; that unit is left with zero tallies */
#define RW_FLAG_VERTEX_CAP 2   /* some path hit max_vertices; it scored 0 */
#define RW_FLAG_WEIGHT_CAP 4   /* rw_dwivedi_forward: a path's weight exceeded 2^64 (FP32
                                  range guard); it was ended and scored 0 */

typedef struct rw_context rw_context;

/* Create a context on HIP device `hip_device` (allocates its small workspace).
 * *out is set to NULL on failure. */
rw_status rw_create(rw_context** out, int hip_device);
/* Release a context and everything it owns; NULL is accepted. */
rw_status rw_destroy(rw_context* ctx);
/* Message of the last non-OK status returned on this context ("" if none). */
const char* rw_last_error(const rw_context* ctx);
/* Static name of a status code. */
const char* rw_status_string(rw_status s);

/* Geometry and estimator constants, copied by value into kernel arguments. */
typedef struct {
  int32_t n_media;      /* K, 1..4 */
  int32_t n_bins;       /* radial bins, 1..4096 (plus under/overflow slots); the
                           walk keeps a per-wave histogram in LDS, so with many
                           bins it runs fewer waves per workgroup */
  float n_rel;          /* refractive index of the medium over the outside, > 0;
                           1 = index-matched */
  float slab_mm;        /* <= 0: semi-infinite; > 0: slab of this thickness (T tallied) */
  float r_min_mm;       /* > 0, first bin edge */
  float r_max_mm;       /* > r_min_mm, last bin edge */
  float rr_weight;      /* roulette threshold (<= 0 disables roulette) */
  float rr_survive;     /* roulette survival probability, (0, 1] */
  int64_t max_vertices; /* per-path vertex cap, 1..2^31 */
  int32_t incidence;    /* RW_INCIDENCE_NORMAL: pencil beam at r = 0 along the normal
                           (Sec. 4.1, eq. radsss); RW_INCIDENCE_COSINE: the
                           cosine-weighted lobe of Sec. 8 at r = 0, with
                           cos(theta_i) = sqrt(u1), phi = 2 pi u2 of vertex 0,
                           refracted by Snell's law, weight 1 - F(theta_i) */
} rw_geometry;

#define RW_INCIDENCE_NORMAL 0
#define RW_INCIDENCE_COSINE 1

/* Media parameters: DEVICE pointers, SoA [K][n_units] FP32, caller-owned,
 * unit = set * n_wl + wavelength index (the wavelength list of the paper's
 * per-wavelength parameters; the walk itself depends on lambda only through
 * the parameters). */
typedef struct {
  const float* sigma_t;       /* extinction, mm^-1, > 0 */
  const float* albedo;        /* single-scattering albedo, [0, 1] */
  const float* g;             /* Henyey-Greenstein anisotropy, (-1, 1) */
  const float* weight;        /* mixture weights (sum 1 per unit), or logits */
  int32_t weights_are_logits; /* 1: weight holds logits, w = softmax over K */
  int64_t n_sets;             /* parameter sets */
  int64_t n_wl;               /* wavelengths per set */
  const float* wavelength_nm; /* [n_wl] labels, may be NULL; not read by the walk */
  int64_t k_stride;           /* elements between media k and k+1 in each array;
                                 0 means n_sets * n_wl (a sub-range of a larger SoA
                                 array passes the full array's unit count) */
  int64_t unit_base;          /* index of this call's first unit in the random-number
                                 counter (unit u draws with index unit_base + u, mod
                                 2^32), so a call on a sub-range of a larger set draws
                                 the same random numbers as the call on the whole set;
                                 0 for a call on a whole set */
} rw_media;

/* Raw FP64 sums, DEVICE pointers, caller-owned.  The library overwrites them
 * (it clears them first), so a tally holds exactly one call's result. */
typedef struct {
  double* R;          /* [n_units][4]: sum x, sum x^2 (top exits), sum T (bottom
                         exits of a slab), sum A (absorbed weight) */
  double* bins;       /* [n_units][n_bins + 2][2]: per slot sum x, sum x^2 */
  int64_t* vertices;  /* [n_units]: exact vertex counts */
  int32_t* flags;     /* [1]: RW_FLAG_* bits (cleared by each call) */
} rw_tally;

/* Forward walk (the mixture walk of Sec. 4.1: medium chosen once by its
 * weight, eq. sss sampled per medium; tallies of eq. radsss), plain form:
 * one launch over a static grid of
 * (unit, chunk of paths) work items, one item per wavefront; every unit runs
 * `paths_per_unit` paths (0..2^31).  Sums are exact (per path, 32-bit fixed
 * point; per unit, 64-bit integer sums, converted to FP64 at the end), so
 * results are bit-identical for the same seed whatever the launch shape or
 * scheduling.  A call with more than one work item per unit uses a device
 * workspace of (n_bins + 2) * 16 + 40 bytes per work item (2048 paths, grown
 * so that the workspace stays within 1 GiB). */
rw_status rw_forward(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                     int64_t paths_per_unit, uint64_t seed, rw_tally* out, void* stream);

/* Allocation-free variant of rw_forward, for callers that cannot allocate
 * device memory during the call: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, launches and
 * results as rw_forward (bit-identical tallies for the same seed), but it
 * calls no hipMalloc, hipFree or other allocating routine, on the device or
 * the host: the forward slot sums of a call whose units span several work
 * items live in a fixed 64 MiB device array that the library holds on every
 * device it runs on until the process ends (its address is looked up once
 * per device by rw_create).  The plan is rw_forward's, except that work items
 * grow (doubling from 2048 paths, at most 65 536) until n_items *
 * ((n_bins + 2) * 16 + 40) bytes fit the array; a call that still does not
 * fit returns RW_E_UNSUPPORTED before anything is enqueued (e.g. more than
 * 1 023 work items of 65 536 paths at 4 096 bins).  Every call on a device
 * shares that array, so calls that overlap on one device (two streams, two
 * contexts, two threads) race; callers serialise them.  The array is cleared
 * by each call, on its stream, with kernels (no memset nodes). */
rw_status rw_forward_noalloc(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                             int64_t paths_per_unit, uint64_t seed, rw_tally* out, void* stream);

/* Batched persistent form of the forward walk (not in the paper, which
 * batches wavelengths in its simulator, Sec. 3; here a launch form for many
 * parameter sets x wavelengths with uneven work): a persistent grid pulls
 * (unit, chunk) work items from a device queue, units with the longest
 * estimated paths first, and wavefronts move on to further items without
 * waiting for an item's slowest path.  Items hold 2048 paths, or the shape the
 * autotuner chose; without a tuned shape, a call with fewer items than about
 * twice the device's resident wavefronts halves them (down to 512 paths) so
 * that the device stays busy.  `paths_per_unit` is a DEVICE int32
 * array [n_units] (uneven counts allowed, 0 allowed; entries above
 * paths_uniform are clamped to it) or NULL, in which case every unit runs
 * `paths_uniform` paths.  Same random numbers per path as rw_forward, hence
 * bit-identical tallies for the same seed and path counts. */
typedef struct {
  int32_t use_graph;            /* build the launch sequence as a hipGraph and replay it */
  int32_t autotune;             /* time candidate launch shapes on first use, cache them */
  int64_t unit_begin, unit_end; /* resume window [begin, end) of units; end <= 0: all.
                                   Units outside the window are left untouched. */
  uint32_t* path_mask;          /* DEVICE [n_units][ceil(paths_uniform / 32)] words, or NULL.
                                   A forward call clears the window's words and sets bit
                                   (p mod 32) of word [u][p / 32] for every path p of unit u
                                   that leaves the top surface (the only paths a gradient
                                   sum can see: a path ended by roulette, the vertex cap or
                                   a slab bottom adds nothing).  An adjoint call given the
                                   mask of the forward with the same seed, path counts and
                                   units replays only those paths, and its vertex counts are
                                   the vertices it replayed.  A mask of another forward gives
                                   a wrong gradient; the library cannot tell. */
} rw_batch_opts;

rw_status rw_batch_forward(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                           const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                           rw_tally* out, const rw_batch_opts* opts, void* stream);

/* Adjoint by path replay (not in the paper, which fits through look-up
 * tables, Sec. 4.2): re-runs the forward walk on the same random numbers
 * (same seed, same path counts) and returns the score-function gradient
 *   grad[u][j] = sum over paths leaving the top of
 *                x * (cot_R[u] + cot_bins[u][slot]) * score_j
 * with the score of the path density: for the chosen medium k,
 *   sigma_t_k: n_coll / sigma_t_k - L   (L = total flight length),
 *   alpha_k:   n_coll / alpha_k,
 *   g_k:       sum over scatterings of d ln p_HG(mu) / d g,
 *   logit_j:   [k == j] - w_j          (w = softmax of the logits),
 * i.e. the gradient of sum_u (cot_R[u] * R_sum[u] + sum_s cot_bins[u][s] * bins[u][s][0]).
 * Output layout grad[n_units][4K] = (sigma_t[K], alpha[K], g[K], logit[K]);
 * raw sums (divide by the path count for the gradient of the means), summed
 * in FP64: the same seed gives the same per-path terms whatever the launch
 * shape, and the sums agree to FP64 rounding (their order follows the
 * schedule, so they are reproducible to rounding, not bitwise).
 * cot_R: DEVICE float [n_units] or NULL (zero); cot_bins: DEVICE float
 * [n_units][n_bins + 2] or NULL (zero).  grad_sumsq (DEVICE double
 * [n_units][4K] or NULL) receives the sums of squares of the per-path terms.
 * vertices (DEVICE int64 [n_units] or NULL) receives the replayed vertex
 * counts; flags (DEVICE int32 [1], required) as for the forward.
 * rw_adjoint uses the plain static grid; rw_batch_adjoint the persistent
 * queue with the same options as rw_batch_forward. */
rw_status rw_adjoint(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                     int64_t paths_per_unit, uint64_t seed, const float* cot_R,
                     const float* cot_bins, double* grad, double* grad_sumsq, int64_t* vertices,
                     int32_t* flags, void* stream);

rw_status rw_batch_adjoint(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                           const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                           const float* cot_R, const float* cot_bins, double* grad,
                           double* grad_sumsq, int64_t* vertices, int32_t* flags,
                           const rw_batch_opts* opts, void* stream);

/* Two-layer tissue, the geometry of the paper's data generator (Sec. 3): a
 * top layer (the epidermis, 50-350 um) of thickness d over a bottom layer that
 * is semi-infinite (rw_geometry.slab_mm <= 0) or ends at slab_mm (tests), each
 * with its own sigma_t, albedo and g.  DEVICE pointers, caller-owned, SoA
 * [2][k_stride] FP32 (row 0 top, row 1 bottom).  The top layer's refractive
 * index over the outside is rw_geometry.n_rel, the bottom layer's
 * n_rel_bottom; rw_geometry.n_media must be 2. */
typedef struct {
  const float* sigma_t;      /* extinction, mm^-1, > 0 */
  const float* albedo;       /* [0, 1] */
  const float* g;            /* (-1, 1) */
  const float* thickness_mm; /* [k_stride]: top-layer thickness d, 0 < d (< slab_mm) */
  float n_rel_bottom;        /* bottom layer's index over the outside, > 0 */
  int64_t n_units;
  int64_t k_stride;          /* 0 means n_units */
  int64_t unit_base;         /* random-number counter index of unit 0, as in rw_media */
} rw_layers;

/* Forward walk through two layers, batched persistent form (options and
 * outputs as rw_batch_forward; the same exact integer tallies).  The path
 * enters the top layer through the surface; a flight that reaches the
 * interface stops there (a vertex), where the path is reflected with the
 * unpolarised Fresnel reflectance of n_from / n_to or else crosses, refracted
 * by Snell's law, and draws its next flight in the other layer.  Units whose
 * layers are invalid (including d <= 0, or d >= slab_mm for a slab) keep zero
 * tallies and raise RW_FLAG_BAD_PARAMS.  rw_layered_adjoint replays it. */
rw_status rw_layered_forward(rw_context* ctx, const rw_layers* layers, const rw_geometry* geom,
                             const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                             rw_tally* out, const rw_batch_opts* opts, void* stream);

/* Adjoint of the two-layer walk by path replay (not in the paper): the same
 * random numbers as rw_layered_forward (same seed and path counts), and the
 * score-function gradient of sum_u (cot_R[u] R_sum[u] + sum_s cot_bins[u][s]
 * bins[u][s][0]) with respect to each layer's sigma_t, albedo and g (not the
 * thickness, which moves the interface).  A path scores each layer with the
 * flights, collisions and scatterings it had there:
 *   sigma_t_l: n_coll_l / sigma_t_l - L_l   (L_l = length travelled in layer l),
 *   alpha_l:   n_coll_l / alpha_l,
 *   g_l:       sum over scatterings in layer l of d ln p_HG(mu) / d g.
 * Output layout as rw_batch_adjoint with K = 2 layers, grad[n_units][8] =
 * (sigma_t[2], alpha[2], g[2], 0, 0) (top, bottom; the last two columns, the
 * mixture logits of rw_adjoint, are 0), raw FP64 sums; grad_sumsq, vertices
 * and flags as there.  Options as rw_batch_forward. */
rw_status rw_layered_adjoint(rw_context* ctx, const rw_layers* layers, const rw_geometry* geom,
                             const int32_t* paths_per_unit, int64_t paths_uniform, uint64_t seed,
                             const float* cot_R, const float* cot_bins, double* grad,
                             double* grad_sumsq, int64_t* vertices, int32_t* flags,
                             const rw_batch_opts* opts, void* stream);

/* Hero-wavelength form of the two-layer walk (Wilkie et al. 2014's hero
 * wavelength, named in Sec. 2; Sec. 3's simulator propagates all its
 * wavelengths together): one path serves a group of n_hero wavelengths of one
 * tissue.  Units come in groups of n_hero consecutive units (u = q n_hero + i,
 * e.g. a tone's wavelengths); members of a group must share the top-layer
 * thickness (else the group keeps zero tallies and RW_FLAG_BAD_PARAMS is
 * raised); the indices are the call's.  Path p of group q draws Philox counter
 * (v, p, 0, unit_base + q) and is sampled with the optics of member p mod
 * n_hero (its flights from that member's sigma_t, its scatterings from its
 * g); every member carries its own albedo weight, Russian roulette decides on
 * the largest weight, and a path that leaves contributes to member i the
 * one-sample balance-heuristic estimate n_hero x_i p_i / sum_j p_j, where
 * p_j is the path's density under member j's optics.  With n_hero = 1 this
 * is rw_layered_forward's walk.  n_hero: 1, 2, 3, 4, 8 or 9;
 * paths_per_group: a multiple of n_hero in [0, 2^31] (each member then was
 * hero of the same number of paths); every unit's estimate is a mean over its
 * group's paths_per_group paths (finalize with that count).  Outputs per unit
 * as rw_layered_forward's exact sums, except sum A = 0 (absorbed weight is
 * not estimated) and vertices[u] = the vertices of the paths unit u was hero
 * of.  A device workspace of 8 n_hero (2 n_bins + 6) bytes per work item of
 * 2048 paths (grown so that it stays within 1 GiB). */
rw_status rw_layered_hero_forward(rw_context* ctx, const rw_layers* layers,
                                  const rw_geometry* geom, int32_t n_hero,
                                  int64_t paths_per_group, uint64_t seed, rw_tally* out,
                                  void* stream);

/* Dwivedi sampling in the mixture walk (the second variance reduction named in
 * Sec. 2; the zero-variance-based scheme of Krivanek and d'Eon 2014, after
 * Dwivedi 1982).  The walk of rw_forward (same media, geometry, Philox
 * counters (v, p, 0, unit_base + u) and tally layout), except that at every
 * scattering it takes, with probability q (0 < q <= 1), the Dwivedi
 * technique: a direction of density 1 / (2 pi lam (nu0 - mu_s)) in the cosine
 * mu_s with the top surface's outward normal and a flight against
 * sigma_t (1 - mu_s / nu0), with nu0 > 1 the root of a nu atanh(1/nu) = 1 for
 * the medium's albedo a clamped to [0.3, 1 - 1e-7] and
 * lam = ln((nu0 + 1) / (nu0 - 1)); otherwise the plain technique.  The flight's
 * end multiplies the weight by the true density of the sampled direction and
 * flight over the two techniques' mixture (one-sample MIS, balance heuristic),
 * so the estimate stays unbiased; the technique uniform is the low 9 bits of
 * the vertex's fourth Philox word.  Exit weights vary from path to path and
 * may exceed 1: the sums are FP64 (per work item, then added in a fixed order),
 * and R[u] = (sum x, sum x^2, T, A) and bins as rw_forward's.  With q = 1 in
 * an isotropic medium the weights telescope (every exit weight depends only on
 * the first collision's depth and the exit cosine); with strongly forward
 * scattering media the weights become heavy-tailed and the plain walk is the
 * better estimator.  A path whose weight exceeds 2^64 ends with score 0 and
 * raises RW_FLAG_WEIGHT_CAP.  Normal incidence only (RW_E_UNSUPPORTED otherwise); no
 * adjoint.  A device workspace of 8 (2 n_bins + 9) bytes per work item of up
 * to 2048 paths (512-2048, smaller when the call has few items; grown so that
 * it stays within 1 GiB) plus 16 K bytes per unit.
 * Asynchronous on `stream`. */
rw_status rw_dwivedi_forward(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                             int64_t paths_per_unit, uint64_t seed, float q, rw_tally* out,
                             void* stream);

/* Finalize (eq. radsss): per unit, from the raw sums of a forward tally and the
 * path count N the walk ran: with a DEVICE int32 paths_per_unit [n_units],
 * N = min(max(paths_per_unit[u], 0), paths_uniform) (the clamp of
 * rw_batch_forward; paths_uniform must then be > 0), else N = paths_uniform:
 *   R_mean = sum x / N,  R_se = sqrt((sum x^2 - (sum x)^2 / N) / (N (N - 1))),
 *   Rr[b]  = bins sum / (N * pi (r_{b+1}^2 - r_b^2))  [mm^-2], b = 0..n_bins-1,
 *   Rr_se  likewise from the per-slot sums of squares,
 *   Pd[b]  = Rr[b] / R_mean (0 when R_mean = 0).
 * Outputs are DEVICE double arrays: R_mean, R_se [n_units]; Rr, Rr_se, Pd
 * [n_units][n_bins] (any of them may be NULL).  Units with N = 0 give zeros. */
rw_status rw_finalize(rw_context* ctx, const rw_geometry* geom, int64_t n_units,
                      const int32_t* paths_per_unit, int64_t paths_uniform, const rw_tally* tally,
                      double* R_mean, double* R_se, double* Rr, double* Rr_se, double* Pd,
                      void* stream);

/* ---------------------------------------------------------------------------
 * Lookup-table fit (Sec. 4.2): the K-media profile from the scale-independent
 * tables R(alpha, g) and P_d(r | alpha, g) at sigma_t = 1 (eq. mixture, with
 * eq. separability for sigma_t: P(r | alpha, g, sigma_t) =
 * sigma_t^2 P_d(sigma_t r | alpha, g)), R bilinear in (alpha, g) and P
 * trilinear in (alpha, g, log r) between bin centres, 0 off the table; the
 * loss of eq. joint_loss per unit; its gradient; one Adam step.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* R;        /* DEVICE [n_alpha][n_g] total diffuse reflectance */
  const float* Pd;       /* DEVICE [n_alpha][n_g][n_bins] profile, mm^-2 at sigma_t = 1 */
  int32_t n_alpha, n_g, n_bins;   /* n_alpha, n_g >= 2, n_bins >= 2 */
  float alpha_max, g_max;         /* uniform grids over [0, alpha_max] and [0, g_max] */
  float r_min_mm, r_max_mm;       /* n_bins log-spaced bins over [r_min, r_max) */
} rw_lut;

typedef struct {
  const float* R;        /* DEVICE [n_units] target total reflectance */
  const float* Pd;       /* DEVICE [n_units][n_r] target normalised profile R(r)/R, mm^-2 */
  const float* mass;     /* DEVICE [n_units][n_r] target exit probability per bin */
  const float* r_mm;     /* DEVICE [n_r] evaluation radii (bin centres) */
  int32_t n_r;           /* 1..512 */
  float lambda_R;        /* weight of (R_hat - R_t)^2 (the paper's 5) */
  float min_mass;        /* bins with mass < min_mass stay out of the shape term */
  float shape_floor;     /* relative floor f: the shape term compares
                            log(P + f P_t) with log(P_t + f P_t) */
  int32_t shape_form;    /* RW_LUT_SHAPE_PAPER: P_hat = sum_k w_k P_k, as Sec. 4.2
                            defines it after eq. refl_loss; RW_LUT_SHAPE_MIXTURE:
                            the normalised profile of eq. mixture,
                            P_hat = sum_k w_k R_k P_k / max(R_hat, 1e-12) */
} rw_lut_targets;

#define RW_LUT_SHAPE_PAPER 0
#define RW_LUT_SHAPE_MIXTURE 1

/* Loss and gradient of eq. joint_loss for K media per unit (K = 1..4):
 *   L = sqrt(mean over bins with mass >= min_mass of
 *            (log(P_hat + f P_t + 1e-12) - log(P_t + f P_t + 1e-12))^2 + 1e-30)
 *       + lambda_R (R_hat - R_t)^2,
 * R_hat = sum_k w_k R(alpha_k, g_k), P_hat as targets->shape_form selects.
 * params: DEVICE float [4K - 1][n_units] raw parameters (row-major by
 * parameter): log sigma_t (K rows), logit alpha (K), logit(g / 0.99) (K) and
 * the first K - 1 softmax logits of the weights (the last logit is 0).
 * grad (DEVICE float, same layout, or NULL) receives dL/dparams; loss (DEVICE
 * float [n_units], or NULL) receives L.  Interpolation follows the cell of the
 * floor of the grid coordinate, clamped to the grid, as a piecewise-linear
 * function is differentiated; coordinates outside a table's range clamp and
 * pass no gradient.  Returns RW_E_INVALID for bad sizes or NULL tables. */
rw_status rw_lut_loss_grad(rw_context* ctx, const rw_lut* lut, const rw_lut_targets* targets,
                           int64_t n_units, int32_t n_media, const float* params, float* grad,
                           float* loss, void* stream);

/* One Adam step (the paper's optimiser, Sec. 4.2 "Optimization") on the same
 * loss, in place: m = b1 m + (1 - b1) grad, v = b2 v + (1 - b2) grad^2,
 * params -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) with
 * b1 = 0.9, b2 = 0.999, eps = 1e-8 and t = step (>= 1).  adam_m, adam_v:
 * DEVICE float, same layout as params, zero before the first step.  loss
 * (or NULL) receives the loss before the step.  A schedule passes its lr per
 * step. */
rw_status rw_lut_fit_step(rw_context* ctx, const rw_lut* lut, const rw_lut_targets* targets,
                          int64_t n_units, int32_t n_media, float* params, float* adam_m,
                          float* adam_v, int32_t step, float lr, float* loss, void* stream);

/* Synchronise `stream`, read flags[0] into *out_flags (may be NULL) and
 * return RW_E_DEVICE_FLAG when it is nonzero. */
rw_status rw_check(rw_context* ctx, const int32_t* flags, int32_t* out_flags, void* stream);

/* Per-path replay for tests: runs n_paths paths of ONE unit (media with
 * n_sets = n_wl = 1) with the random words taken from `words` (DEVICE uint32
 * [n_paths][n_blocks][4], block v of path p) or, when words is NULL, from
 * Philox with counter (v, p, 0, unit_index).  Writes per vertex
 * events[p][v][8] = (code, x, y, z, ux, uy, uz, W) with code 0 start,
 * 1 collision, 2 reflection, 3 top exit, 4 bottom exit, 5 roulette kill,
 * 6 vertex cap (state after the vertex; zero-filled beyond the path end), and
 * path_out[p][8] = (end, k, slot, x, r, n_vert, n_coll, absorbed) with end 1
 * top exit, 2 bottom exit, 3 roulette kill, 4 cap, 7 out of words;
 * path_adj[p][2] = (L, sum d ln p_HG / d g) or NULL.  All DEVICE float. */
rw_status rw_debug_trace(rw_context* ctx, const rw_media* media, const rw_geometry* geom,
                         const uint32_t* words, int64_t n_paths, int64_t n_blocks, uint64_t seed,
                         uint32_t unit_index, float* events, float* path_out, float* path_adj,
                         void* stream);

/* The same replay for one two-layer unit (layers->n_units == 1); path_out[1]
 * is the layer the path ended in, event code 8 marks an interface crossing. */
rw_status rw_debug_trace_layered(rw_context* ctx, const rw_layers* layers,
                                 const rw_geometry* geom, const uint32_t* words, int64_t n_paths,
                                 int64_t n_blocks, uint64_t seed, uint32_t unit_index,
                                 float* events, float* path_out, void* stream);

/* Philox4x32-10 blocks for tests: out[i][0..3] = Philox(ctr[i], key); DEVICE
 * uint32 arrays [n][4]. */
rw_status rw_debug_philox(rw_context* ctx, const uint32_t* ctr, uint64_t key, int64_t n,
                          uint32_t* out, void* stream);

/* Library version string. */
const char* rw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RW_H */
