"""Checks that pin the FP64 oracle's random walk to things other than itself.

Each ``check_*`` returns (ok: bool, detail: str) so that the same battery runs
at full size in test_oracle_transport.py and at small size against copies of
the oracle with planted mistakes in test_oracle_mutations.py.

What pins what:
  plane albedo     - total R against Chandrasekhar's 1 - H(1) sqrt(1-alpha)
  second moment    - sum x^2 / N against R(alpha^2) (x = alpha^n_coll without
                     roulette, so E[x^2](alpha) = R(alpha^2)), SE from R(alpha^4)
  single scatter   - order-1 tallies (total and per annulus) against the 1-D
                     quadrature for any g and Fresnel index
  energy           - slab without roulette: R + T + A = 1 - F(0) per path
  analog/weighted  - two different estimators of the same R agree
  Beer-Lambert     - purely absorbing slab: T = exp(-sigma_t d), R = 0
  mixture          - R_mix = sum_k w_k R(alpha_k) (paper Sec. 4.1, eq. sss)
  special case     - w = (1, 0, 0) reproduces the one-medium walk bit for bit
  scale invariance - sigma_t -> c sigma_t on the same random numbers leaves R
                     unchanged and divides every exit radius by c (eq. separability)
  trace invariants - reflection law, straight flights, exponential first flight,
                     Henyey-Greenstein scattering cosines, uniform azimuth
  adjoint          - closed-form dR/dalpha, dR/dsigma_t = 0, mixture gradients,
                     and common-random-number central differences of the forward
  brute force      - a deterministic grid of injected words averages to the
                     single-scattering closed form
  adding-doubling  - totals of multiply-scattering media with g != 0 and a
                     Fresnel boundary (semi-infinite, slab R and T, two layers,
                     normal and cosine incidence) against the deterministic
                     adding-doubling solution, itself pinned to closed forms
  two layers       - Beer-Lambert through two absorbing layers; identical
                     layers and a vanishing top layer reproduce the
                     plane albedo; an absorbing non-scattering top layer over an
                     isotropic bottom follows Chandrasekhar's exit law times
                     e^(-tau/mu); a non-scattering stack follows the incoherent
                     adding of its three Fresnel interfaces (R and T, normal and
                     cosine incidence, with and without total internal
                     reflection at the interface); analog and weighted agree;
                     traces obey Snell's law at every crossing
  Dwivedi walk     - nu0 against a library root finder and its diffusion
                     limit; in isotropic index-matched media with technique
                     probability 1 every exit weight equals its closed form
                     alpha e^(-sigma_t z1 / nu0) lam (nu0 - mu_exit) / 2 (the
                     weights telescope); R against Chandrasekhar's closed
                     form (probabilities 1 and 0.5) and, with anisotropy and
                     a Fresnel surface, against adding-doubling; an isotropic
                     three-medium mixture agrees with the plain walk in R and
                     the radial histogram
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, stats

from oracle import closed_forms as cf
from oracle import oracle as O
from tests._stats import accept_histogram, histogram_z, mean_se


def _r(ok, detail):
    return bool(ok), detail


def check_plane_albedo(alphas=(0.5, 0.7, 0.9, 0.99), paths=1 << 18, seed=1, k=3.0, rel=None):
    alphas = np.asarray(alphas, np.float64)
    n = alphas.size
    geo = O.Geometry(n_media=1, n_rel=1.0)
    tal, _, _ = O.forward(geo, np.ones(n), alphas, np.zeros(n), np.ones(n), paths, seed)
    m, se = mean_se(tal[:, 0], tal[:, 1], paths)
    ref = np.array([cf.R_plane(a) for a in alphas])
    z = (m - ref) / se
    ok = np.all(np.abs(z) <= k)
    if rel is not None:
        ok = ok and np.all(np.abs(m - ref) <= rel * ref)
    return _r(ok, f"z={np.round(z, 2)} rel={np.round((m - ref) / ref, 5)}")


def check_second_moment(alpha=0.8, paths=1 << 18, seed=2, k=3.0):
    # without roulette the walk only ends at the surface and path lengths are
    # heavy-tailed; a path still inside after 4096 vertices carries
    # x <= alpha^4095, which is 0 in FP64 for alpha <= 0.8, so the cap (which
    # scores 0) does not bias E[x^2]
    geo = O.Geometry(n_media=1, n_rel=1.0, rr_weight=0.0, max_vertices=4096)
    tal, _, _ = O.forward(geo, [1.0], [alpha], [0.0], [1.0], paths, seed)
    m2 = tal[0, 1] / paths
    ref = cf.R_plane(alpha * alpha)
    se = math.sqrt(max(cf.R_plane(alpha ** 4) - ref * ref, 0.0) / paths)
    z = (m2 - ref) / se
    return _r(abs(z) <= k, f"E[x^2] z={z:.2f}")


def check_single_scatter(g=0.5, n=1.4, sigma_t=2.0, alpha=0.9, paths=1 << 18, seed=3, k=3.0,
                         n_bins=64):
    geo = O.Geometry(n_media=1, n_rel=n, order_filter=1, n_bins=n_bins)
    tal, bins, _ = O.forward(geo, [sigma_t], [alpha], [g], [1.0], paths, seed)
    m, se = mean_se(tal[0, 0], tal[0, 1], paths)
    ref = cf.R1_total(alpha, g, n)
    z = (m - ref) / se
    slots = cf.R1_slots(alpha, g, n, sigma_t, n_bins, geo.r_min_mm, geo.r_max_mm)
    bm, bse = mean_se(bins[0, :, 0], bins[0, :, 1], paths)
    hits = bins[0, :, 0] ** 2 / np.maximum(bins[0, :, 1], 1e-300)  # effective hit count
    zb = histogram_z(bm, bse, slots, 0.0, mask=hits >= 30)
    okh, chi2, lim = accept_histogram(zb)
    return _r(abs(z) <= k and okh, f"total z={z:.2f}; bins chi2={chi2:.1f}/{lim:.1f} "
              f"n={zb.size} max|z|={np.max(np.abs(zb)) if zb.size else 0:.2f}")


def check_energy_exact(paths=1 << 14, seed=4):
    n = 1.4
    geo = O.Geometry(n_media=1, n_rel=n, slab_mm=2.0, rr_weight=0.0)
    tal, _, _ = O.forward(geo, [1.5], [0.9], [0.8], [1.0], paths, seed)
    F0 = ((n - 1) / (n + 1)) ** 2
    tot = (tal[0, 0] + tal[0, 2] + tal[0, 3]) / paths
    capped = tal[0, 5]
    return _r(abs(tot - (1 - F0)) < 1e-10 and capped == 0, f"R+T+A={tot!r} vs {1 - F0!r}")


def check_analog_vs_weighted(paths=1 << 18, seed=5, k=3.0):
    n = 1.4
    base = dict(n_media=1, n_rel=n, slab_mm=3.0)
    args = ([2.0], [0.95], [0.6], [1.0], paths)
    ta, _, _ = O.forward(O.Geometry(analog=True, **base), *args, seed)
    tw, _, _ = O.forward(O.Geometry(**base), *args, seed + 100)
    counts = ta[0, 0] + ta[0, 2] + ta[0, 3] + ta[0, 4] + ta[0, 5]
    pa = ta[0, 0] / paths
    sa = math.sqrt(pa * (1 - pa) / paths)
    mw, sw = mean_se(tw[0, 0], tw[0, 1], paths)
    z = (pa - mw) / math.hypot(sa, sw)
    pt = ta[0, 2] / paths
    mt = tw[0, 2] / paths
    return _r(abs(z) <= k and counts == paths and abs(pt - mt) < 5 * math.sqrt(pt / paths),
              f"R analog={pa:.5f} weighted={mw:.5f} z={z:.2f}; T {pt:.5f}/{mt:.5f}; counts={counts}")


def check_spherical_albedo(paths=1 << 18, seed=15, k=3.0):
    """Cosine-weighted incidence, isotropic scattering, n = 1: R against the
    spherical albedo 1 - 2 sqrt(1 - alpha) int mu H(mu) dmu."""
    al = np.array([0.5, 0.8, 0.95, 0.99])
    geo = O.Geometry(n_media=1, n_rel=1.0, incidence=1)
    tal, _, _ = O.forward(geo, np.ones(4), al, np.zeros(4), np.ones(4), paths, seed)
    m, se = mean_se(tal[:, 0], tal[:, 1], paths)
    ref = np.array([cf.R_spherical(float(a)) for a in al])
    z = (m - ref) / se
    return _r(bool(np.all(np.abs(z) <= k)), f"z={np.round(z, 2)}")


def check_analog_vs_weighted_cosine(paths=1 << 18, seed=16, k=3.0):
    """Both estimators under the cosine-weighted lobe with a Fresnel boundary."""
    n = 1.4
    base = dict(n_media=1, n_rel=n, slab_mm=3.0, incidence=1)
    args = ([2.0], [0.95], [0.6], [1.0], paths)
    ta, _, _ = O.forward(O.Geometry(analog=True, **base), *args, seed)
    tw, _, _ = O.forward(O.Geometry(**base), *args, seed + 100)
    pa = ta[0, 0] / paths
    sa = math.sqrt(pa * (1 - pa) / paths)
    mw, sw = mean_se(tw[0, 0], tw[0, 1], paths)
    z = (pa - mw) / math.hypot(sa, sw)
    spec = ta[0, 4] / paths
    # the mean entry reflectance of a cosine lobe at n = 1.4 (hemispherical
    # average of the Fresnel reflectance, about 0.09)
    return _r(abs(z) <= k and 0.07 < spec < 0.11, f"R analog={pa:.5f} weighted={mw:.5f} "
              f"z={z:.2f}; specular {spec:.4f}")


def check_beer_lambert(paths=1 << 18, seed=6, k=3.0):
    geo = O.Geometry(n_media=1, n_rel=1.0, slab_mm=1.0)
    tal, _, _ = O.forward(geo, [1.3], [0.0], [0.0], [1.0], paths, seed)
    p = cf.beer_lambert(1.3, 1.0)
    T = tal[0, 2] / paths
    z = (T - p) / math.sqrt(p * (1 - p) / paths)
    return _r(abs(z) <= k and tal[0, 0] == 0.0, f"T={T:.5f} vs {p:.5f} z={z:.2f} R={tal[0, 0]}")


def check_mixture_linearity(paths=1 << 18, seed=7, k=3.0):
    al = np.array([[0.6], [0.9], [0.99]])
    w = np.array([[0.2], [0.5], [0.3]])
    geo = O.Geometry(n_media=3, n_rel=1.0)
    tal, _, _ = O.forward(geo, [[1.0], [3.0], [0.5]], al, np.zeros((3, 1)), w, paths, seed)
    m, se = mean_se(tal[0, 0], tal[0, 1], paths)
    ref = sum(w[i, 0] * cf.R_plane(al[i, 0]) for i in range(3))
    z = (m - ref) / se
    return _r(abs(z) <= k, f"R_mix={m:.5f} vs {ref:.5f} z={z:.2f}")


def check_single_medium_special_case(paths=1 << 14, seed=8):
    one = O.Geometry(n_media=1, n_rel=1.4)
    three = O.Geometry(n_media=3, n_rel=1.4)
    t1, b1, v1 = O.forward(one, [2.0], [0.9], [0.7], [1.0], paths, seed)
    t3, b3, v3 = O.forward(three, [[2.0], [5.0], [0.3]], [[0.9], [0.5], [0.99]],
                           [[0.7], [0.1], [0.2]], [[1.0], [0.0], [0.0]], paths, seed)
    ok = np.array_equal(t1, t3) and np.array_equal(b1, b3) and np.array_equal(v1, v3)
    return _r(ok, "K=3 with w=(1,0,0) vs K=1")


def check_scale_invariance(paths=1 << 14, seed=9, c=3.7):
    geo = O.Geometry(n_media=1, n_rel=1.4)
    ta, _, _ = O.forward(geo, [1.0], [0.95], [0.6], [1.0], paths, seed)
    tb, _, _ = O.forward(geo, [c], [0.95], [0.6], [1.0], paths, seed)
    okR = abs(ta[0, 0] - tb[0, 0]) <= 1e-9 * abs(ta[0, 0])
    _, oa, _ = O.trace(geo, [1.0], [0.95], [0.6], [1.0], n_paths=512, n_blocks=4096, seed=seed)
    _, ob, _ = O.trace(geo, [c], [0.95], [0.6], [1.0], n_paths=512, n_blocks=4096, seed=seed)
    top = (oa[:, 0] == O.END_EXIT_TOP) & (ob[:, 0] == O.END_EXIT_TOP)
    okr = np.allclose(oa[top, 4], ob[top, 4] * c, rtol=1e-9, atol=1e-12) and top.sum() > 100
    return _r(okR and okr, f"R {ta[0, 0]!r} vs {tb[0, 0]!r}; radii scale ok={okr}")


def check_trace_invariants(n_paths=4000, seed=10, g=0.6, n=1.4, sigma_t=2.5, alpha=0.95):
    geo = O.Geometry(n_media=1, n_rel=n)
    ev, out, _ = O.trace(geo, [sigma_t], [alpha], [g], [1.0], n_paths=n_paths, n_blocks=2048,
                         seed=seed)
    nv = out[:, 5].astype(np.int64)
    vidx = np.arange(1, ev.shape[1])[None, :]
    live = vidx <= nv[:, None]                      # [paths, vertices-1] pairs (v-1, v)
    prev, cur = ev[:, :-1][live], ev[:, 1:][live]
    code = cur[:, 0].astype(int)
    fails = []
    dpos = cur[:, 1:4] - prev[:, 1:4]
    cross = np.linalg.norm(np.cross(dpos, prev[:, 4:7]), axis=1)
    if np.any(cross > 1e-9 * np.maximum(1.0, np.linalg.norm(dpos, axis=1))):
        fails.append("flight not along direction")
    if np.any(np.einsum("ij,ij->i", dpos, prev[:, 4:7]) < -1e-12):
        fails.append("flight backwards")
    bnd = (code == O.EV_REFLECT) | (code == O.EV_EXIT_TOP)
    if np.any(cur[bnd, 3] != 0.0):
        fails.append("boundary event off the surface")
    refl = code == O.EV_REFLECT
    if not (np.array_equal(cur[refl, 4], prev[refl, 4]) and np.array_equal(cur[refl, 5], prev[refl, 5])
            and np.array_equal(cur[refl, 6], -prev[refl, 6])):
        fails.append("reflection law")
    if not np.array_equal(cur[refl, 7], prev[refl, 7]):
        fails.append("weight changed at reflection")
    col = code == O.EV_COLLIDE
    if np.any(np.abs(np.linalg.norm(cur[col, 4:7], axis=1) - 1.0) > 1e-12):
        fails.append("direction not unit")
    ratio = cur[col, 7] / prev[col, 7]
    okw = (np.abs(ratio - alpha) < 1e-12 * alpha) | (
        np.abs(ratio - alpha / geo.rr_survive) < 1e-9 * alpha / geo.rr_survive)
    if not np.all(okw):
        fails.append("weight update")
    cosines = np.einsum("ij,ij->i", cur[col, 4:7], prev[col, 4:7])
    first = ev[:, 1][ev[:, 1, 0] == O.EV_COLLIDE]   # first vertex, entered along +z
    first_depth = first[:, 3]
    first_phi = np.arctan2(first[:, 5], first[:, 4])
    exits = out[:, 0] == O.END_EXIT_TOP
    last = ev[np.arange(n_paths), nv][exits]
    if np.any(np.abs(out[exits, 4] - np.hypot(last[:, 1], last[:, 2]))
              > 1e-12 * np.maximum(1.0, out[exits, 4])):
        fails.append("exit radius")
    if not np.array_equal(last[:, 7], out[exits, 3]):
        fails.append("exit weight")
    # first flight from the surface along +z: depth ~ Exp(sigma_t)
    ks_depth = stats.kstest(first_depth, lambda z: 1.0 - np.exp(-sigma_t * np.asarray(z))).pvalue
    # scattering cosines ~ HG(g): CDF by integrating the closed-form density
    grid = np.linspace(-1, 1, 400001)
    cdf_grid = integrate.cumulative_trapezoid(cf.hg_pdf(grid, g), grid, initial=0.0)
    ks_cos = stats.kstest(cosines[:20000], lambda m: np.interp(m, grid, cdf_grid)).pvalue
    ks_phi = stats.kstest(first_phi, "uniform", args=(-math.pi, 2 * math.pi)).pvalue
    n_reflect = int(refl.sum())
    ok = not fails and ks_depth > 1e-4 and ks_cos > 1e-4 and ks_phi > 1e-4 and n_reflect > 0
    return _r(ok, f"fails={fails[:4]} ks depth={ks_depth:.3g} cos={ks_cos:.3g} "
              f"phi={ks_phi:.3g} reflections={n_reflect}")


def check_brute_force_single_scatter(m=48, alpha=0.7, g=0.0):
    """Deterministic grid over (first flight u0, scattering u1, azimuth u2, second
    flight u0'), index-matched: the grid mean of the order-1 tally converges to
    alpha (1 - ln 2)/2 (g = 0).  The words encode the grid points exactly."""
    geo = O.Geometry(n_media=1, n_rel=1.0, rr_weight=0.0, order_filter=0)
    pts = (np.arange(m) + 0.5) / m

    def word(u):  # the word whose uniform is the grid point rounded to 2^-23
        return (np.floor(u * (1 << 23)).astype(np.uint64) << 9).astype(np.uint32)

    a, b, c = np.meshgrid(pts, pts, pts, indexing="ij")
    n = a.size
    words = np.zeros((n, 3, 4), np.uint32)
    words[:, 0, 0] = word(np.full(n, 0.5))
    words[:, 1, 0] = word(a.ravel())
    words[:, 1, 1] = word(b.ravel())
    words[:, 1, 2] = word(np.full(n, 0.25))
    words[:, 2, 0] = word(c.ravel())
    words[:, 2, 3] = word(np.full(n, 0.5))
    _, out, _ = O.trace(geo, [1.0], [alpha], [g], [1.0], words=words)
    order1 = (out[:, 0] == O.END_EXIT_TOP) & (out[:, 6] == 1)
    est = float(np.sum(out[order1, 3])) / n
    ref = cf.R1_total(alpha, g, 1.0)
    return _r(abs(est - ref) < 0.02 * ref, f"grid mean {est:.6f} vs {ref:.6f}")


def check_adjoint_plane(alphas=(0.6, 0.9), paths=1 << 18, seed=11, k=3.0):
    alphas = np.asarray(alphas, np.float64)
    n = alphas.size
    geo = O.Geometry(n_media=1, n_rel=1.0)
    grad, sq = O.adjoint(geo, np.full(n, 2.0), alphas, np.zeros(n), np.ones(n), paths, seed,
                         cot_R=np.ones(n))
    ga, sa = mean_se(grad[:, 1], sq[:, 1], paths)
    gs, ss = mean_se(grad[:, 0], sq[:, 0], paths)
    gl, _ = mean_se(grad[:, 3], sq[:, 3], paths)
    ref = np.array([cf.dR_plane_dalpha(a) for a in alphas])
    za = (ga - ref) / sa
    zs = gs / ss
    ok = np.all(np.abs(za) <= k) and np.all(np.abs(zs) <= k) and np.all(np.abs(gl) < 1e-12)
    return _r(ok, f"dR/dalpha z={np.round(za, 2)}; dR/dsigma z={np.round(zs, 2)}")


def check_adjoint_mixture(paths=1 << 18, seed=12, k=3.0):
    al = np.array([0.6, 0.9, 0.99])
    w = np.array([0.2, 0.5, 0.3])
    geo = O.Geometry(n_media=3, n_rel=1.0)
    grad, sq = O.adjoint(geo, np.array([1.0, 3.0, 0.5]), al, np.zeros(3), w, paths, seed,
                         cot_R=[1.0])
    g, se = mean_se(grad[0], sq[0], paths)
    Rk = np.array([cf.R_plane(a) for a in al])
    Rmix = float(w @ Rk)
    ref_l = w * (Rk - Rmix)
    ref_a = w * np.array([cf.dR_plane_dalpha(a) for a in al])
    z = np.concatenate([(g[9:12] - ref_l) / se[9:12], (g[3:6] - ref_a) / se[3:6], g[0:3] / se[0:3]])
    return _r(np.all(np.abs(z) <= k), f"z={np.round(z, 2)}")


def check_adjoint_vs_crn_fd(paths=1 << 15, reps=8, seed=13, k=3.5):
    """VJP with random cotangents against central differences of the cotangent-weighted
    forward tallies on common random numbers, with replica means for the SE."""
    geo = O.Geometry(n_media=3, n_rel=1.4, n_bins=32, r_min_mm=1e-2, r_max_mm=20.0)
    sig = np.array([1.0, 4.0, 0.5])
    alb = np.array([0.9, 0.6, 0.97])
    gg = np.array([0.5, 0.2, 0.8])
    logits = np.array([0.3, -0.4, 0.0])
    rng = np.random.default_rng(seed)
    cotB = rng.standard_normal(geo.n_bins + 2)
    cotR = 1.0

    def weights(l):
        e = np.exp(l - l.max())
        return e / e.sum()

    def J(s, a, g_, l, sd):
        tal, bins, _ = O.forward(geo, s, a, g_, weights(l), paths, sd)
        return (cotR * tal[0, 0] + bins[0, :, 0] @ cotB) / paths

    P = 12
    adj = np.zeros((reps, P))
    fd = np.zeros((reps, P))
    for r in range(reps):
        sd = seed * 1000 + r
        grad, _ = O.adjoint(geo, sig, alb, gg, weights(logits), paths, sd, cot_R=[cotR],
                            cot_bins=cotB[None, :])
        adj[r] = grad[0] / paths
        for j in range(P):
            s, a, g_, l = sig.copy(), alb.copy(), gg.copy(), logits.copy()
            grp, i = divmod(j, 3)
            if grp == 0:
                h = 1e-3 * s[i]
                s[i] += h; Jp = J(s, a, g_, l, sd); s[i] -= 2 * h; Jm = J(s, a, g_, l, sd)
            elif grp == 1:
                h = 1e-3 * a[i]
                a[i] += h; Jp = J(s, a, g_, l, sd); a[i] -= 2 * h; Jm = J(s, a, g_, l, sd)
            elif grp == 2:
                h = 1e-3
                g_[i] += h; Jp = J(s, a, g_, l, sd); g_[i] -= 2 * h; Jm = J(s, a, g_, l, sd)
            else:
                # a logit step moves the medium-choice thresholds, so only paths
                # whose u0 lies within ~h*w of a threshold change; a larger step keeps
                # the difference from resting on a handful of paths (the mixture is
                # smooth in the logits, so the O(h^2) error stays far below the SE)
                h = 1e-2
                l[i] += h; Jp = J(s, a, g_, l, sd); l[i] -= 2 * h; Jm = J(s, a, g_, l, sd)
            fd[r, j] = (Jp - Jm) / (2 * h)
    ma, sa = adj.mean(0), adj.std(0, ddof=1) / math.sqrt(reps)
    mf, sf = fd.mean(0), fd.std(0, ddof=1) / math.sqrt(reps)
    z = (ma - mf) / np.sqrt(sa ** 2 + sf ** 2 + 1e-30)
    return _r(np.all(np.abs(z) <= k), f"z={np.round(z, 2)}")


def check_jacobian(paths=1 << 13, seed=14, rtol=1e-9):
    """The Jacobian output of the oracle's adjoint (per unit, the score sums of
    the total and of every radial slot), pinned without re-deriving it:
    (i) contracted with any cotangents it gives the gradient the adjoint
        returns for those cotangents (a vector-Jacobian product is the
        Jacobian's transpose applied to the cotangent), for K = 1..4 on two
        units, with a Fresnel boundary and g != 0;
    (ii) its slots add up to its total row (every top exit lands in one slot);
    (iii) on single-scattering paths (order filter 1, eq. sss with one
        scattering vertex) the exit weight is linear in the albedo, so the
        albedo column of every slot equals that slot's forward sum divided by
        the albedo, and the logit columns of each slot sum to zero (the
        softmax weights sum to one)."""
    rng = np.random.default_rng(seed)
    for K in (1, 2, 3, 4):
        n_units = 2
        geo = O.Geometry(n_media=K, n_rel=1.4, n_bins=12, r_min_mm=1e-2, r_max_mm=20.0)
        sig = 10 ** rng.uniform(-0.5, 1.0, (K, n_units))
        alb = rng.uniform(0.5, 0.97, (K, n_units))
        gg = rng.uniform(-0.3, 0.9, (K, n_units))
        w = rng.dirichlet(np.ones(K), n_units).T
        cotR = rng.standard_normal(n_units)
        cotB = rng.standard_normal((n_units, geo.n_bins + 2))
        grad, _, jR, jB = O.adjoint(geo, sig, alb, gg, w, paths, seed + K, cot_R=cotR,
                                    cot_bins=cotB, jacobian=True)
        vjp = cotR[:, None] * jR + np.einsum("us,usj->uj", cotB, jB)
        scale = np.abs(cotR)[:, None] * np.abs(jR) + np.einsum("us,usj->uj", np.abs(cotB),
                                                               np.abs(jB)) + 1e-300
        err = np.abs(vjp - grad) / scale
        if not np.all(err <= rtol):
            return _r(False, f"K={K}: contraction differs from the gradient, max rel {err.max():.2e}")
        if not np.allclose(jB.sum(1), jR, rtol=1e-12, atol=1e-12 * np.abs(jR).max()):
            return _r(False, f"K={K}: slots do not add up to the total row")
        if not np.any(np.abs(jB) > 0):
            return _r(False, f"K={K}: empty Jacobian")
    # (iii) single scattering, K = 1 (albedo column) and K = 3 (logit columns)
    for K in (1, 3):
        geo = O.Geometry(n_media=K, n_rel=1.4, n_bins=12, r_min_mm=1e-2, r_max_mm=20.0,
                         order_filter=1)
        sig = np.array([2.0, 0.7, 5.0][:K])
        alb = np.array([0.8, 0.6, 0.95][:K])
        gg = np.array([0.5, 0.1, 0.8][:K])
        w = np.array([0.5, 0.2, 0.3][:K]) if K == 3 else np.ones(1)
        _, bins, _ = O.forward(geo, sig, alb, gg, w, paths * 4, seed + 10)
        _, _, jR, jB = O.adjoint(geo, sig, alb, gg, w, paths * 4, seed + 10, cot_R=[1.0],
                                 jacobian=True)
        if K == 1:
            want = bins[0, :, 0] / alb[0]
            if not np.allclose(jB[0, :, 1], want, rtol=1e-12, atol=1e-15):
                return _r(False, "single-scatter albedo column != slot sum / albedo")
            if not np.any(want > 0):
                return _r(False, "no single-scatter exits")
        else:
            lsum = jB[0, :, 9:12].sum(1)
            if not np.all(np.abs(lsum) <= 1e-12 * (np.abs(jB[0, :, 9:12]).sum(1) + 1e-300)):
                return _r(False, "logit columns of a slot do not sum to zero")
    return _r(True, "")


# ---- two-layer tissue ------------------------------------------------------
def _layered(geo, top, bot, d, n_bottom, paths, seed, n=1):
    """top/bot = (sigma_t, albedo, g) of each layer, repeated over n units.
    Raises when a path hits the vertex cap (these set-ups never come near
    it), so that a walk that stops making progress fails fast."""
    s = np.array([[top[0]] * n, [bot[0]] * n], np.float64)
    a = np.array([[top[1]] * n, [bot[1]] * n], np.float64)
    g = np.array([[top[2]] * n, [bot[2]] * n], np.float64)
    geo = O.Geometry(**{**geo.__dict__, "max_vertices": min(geo.max_vertices, 1 << 14)})
    tal, bins, vert = O.layered_forward(geo, s, a, g, np.full(n, d), n_bottom, paths, seed)
    if np.any(tal[:, O.T_CAPPED] > 0):
        raise ValueError("paths reached the vertex cap")
    return tal, bins, vert


def check_two_layer_beer_lambert(paths=1 << 18, seed=25, k=3.0):
    """Two purely absorbing layers (albedo 0) in a slab, n = 1: the unscattered
    beam leaves the bottom with probability exp(-sigma_1 d - sigma_2 (L - d))."""
    geo = O.Geometry(n_media=2, n_rel=1.0, slab_mm=1.0)
    s1, s2, d = 1.7, 0.6, 0.3
    tal, _, _ = _layered(geo, (s1, 0.0, 0.0), (s2, 0.0, 0.0), d, 1.0, paths, seed)
    p = math.exp(-s1 * d - s2 * (1.0 - d))
    T = tal[0, 2] / paths
    z = (T - p) / math.sqrt(p * (1 - p) / paths)
    return _r(abs(z) <= k and tal[0, 0] == 0.0, f"T={T:.5f} vs {p:.5f} z={z:.2f} R={tal[0, 0]}")


def check_layers_reduce_to_plane(paths=1 << 18, seed=20, k=3.0):
    """Two identical isotropic layers, and a top layer too thin to interact
    (d = 1e-7 mm with other optics), both reproduce 1 - H(1) sqrt(1 - alpha)."""
    geo = O.Geometry(n_media=2, n_rel=1.0)
    zs = []
    for al, top, d in ((0.9, (2.0, 0.9, 0.0), 0.3), (0.7, (5.0, 0.2, 0.8), 1e-7)):
        tal, _, _ = _layered(geo, top, (2.0, al, 0.0), d, 1.0, paths, seed)
        m, se = mean_se(tal[0, 0], tal[0, 1], paths)
        zs.append((m - cf.R_plane(al)) / se)
    return _r(all(abs(z) <= k for z in zs), f"z={np.round(zs, 2)}")


def check_absorbing_top_layer(paths=1 << 18, seed=21, k=3.0):
    """Non-scattering absorbing top layer (albedo 0) of optical thickness tau
    over an isotropic bottom, n = 1: R = e^-tau int dR/dmu e^(-tau/mu) dmu."""
    geo = O.Geometry(n_media=2, n_rel=1.0)
    zs = []
    for tau, al in ((0.2, 0.95), (1.0, 0.8)):
        d = 0.25
        tal, _, _ = _layered(geo, (tau / d, 0.0, 0.0), (3.0, al, 0.0), d, 1.0, paths, seed)
        m, se = mean_se(tal[0, 0], tal[0, 1], paths)
        zs.append((m - cf.R_absorbing_top(al, tau)) / se)
    return _r(all(abs(z) <= k for z in zs), f"z={np.round(zs, 2)}")


def check_layered_adjoint_absorbing_top(paths=1 << 18, seed=26, k=3.0):
    """Two-layer adjoint against the derivatives of the absorbing-top closed
    form (non-scattering top layer of optical thickness tau = sigma_top d over
    an isotropic bottom of albedo alpha, n = 1): dR/dsigma_top = d dR/dtau,
    dR/dalpha_bottom = dR/dalpha, and dR/dsigma_bottom = 0 (the bottom's
    reflectance does not depend on its length scale).  The derivatives of the
    closed form are central differences of the quadrature, far below the
    statistical error."""
    geo = O.Geometry(n_media=2, n_rel=1.0)
    zs = []
    for tau, al in ((0.3, 0.95), (1.0, 0.8)):
        d = 0.25
        s = np.array([[tau / d], [3.0]])
        a = np.array([[0.0], [al]])
        g = np.zeros((2, 1))
        grad, sq = O.layered_adjoint(geo, s, a, g, [d], 1.0, paths, seed, cot_R=[1.0])
        m, se = mean_se(grad[0], sq[0], paths)
        h = 1e-5
        dtau = (cf.R_absorbing_top(al, tau + h) - cf.R_absorbing_top(al, tau - h)) / (2 * h)
        dal = (cf.R_absorbing_top(al + h, tau) - cf.R_absorbing_top(al - h, tau)) / (2 * h)
        zs += [(m[0] - d * dtau) / se[0], (m[3] - dal) / se[3], m[1] / se[1]]
        if np.any(grad[0, 6:] != 0.0):
            return _r(False, "logit columns of the two-layer adjoint must be 0")
    return _r(all(abs(z) <= k for z in zs), f"z={np.round(zs, 2)}")


def check_layered_adjoint_vs_crn_fd(paths=1 << 14, reps=8, seed=27, k=3.5):
    """Two-layer VJP with random bin cotangents against central differences
    of the cotangent-weighted forward tallies on common random numbers (each
    layer's sigma_t, albedo and g, an index step at the interface), replica
    means for the SE."""
    geo = O.Geometry(n_media=2, n_rel=1.4, n_bins=32, r_min_mm=1e-2, r_max_mm=20.0)
    sig = np.array([6.0, 1.5])
    alb = np.array([0.85, 0.95])
    gg = np.array([0.7, 0.5])
    d, n_bot = 0.15, 1.36
    rng = np.random.default_rng(seed)
    cotB = rng.standard_normal(geo.n_bins + 2)

    def J(s, a, g_, sd):
        tal, bins, _ = O.layered_forward(geo, s[:, None], a[:, None], g_[:, None], [d], n_bot,
                                         paths, sd)
        return (tal[0, 0] + bins[0, :, 0] @ cotB) / paths

    adj = np.zeros((reps, 6))
    fd = np.zeros((reps, 6))
    for r in range(reps):
        sd = seed * 1000 + r
        grad, _ = O.layered_adjoint(geo, sig[:, None], alb[:, None], gg[:, None], [d], n_bot,
                                    paths, sd, cot_R=[1.0], cot_bins=cotB[None, :])
        adj[r] = grad[0, :6] / paths
        for j in range(6):
            s, a, g_ = sig.copy(), alb.copy(), gg.copy()
            grp, i = divmod(j, 2)
            v = (s, a, g_)[grp]
            h = 1e-3 * (v[i] if grp < 2 else 1.0)
            v[i] += h
            Jp = J(s, a, g_, sd)
            v[i] -= 2 * h
            Jm = J(s, a, g_, sd)
            fd[r, j] = (Jp - Jm) / (2 * h)
    ma, sa = adj.mean(0), adj.std(0, ddof=1) / math.sqrt(reps)
    mf, sf = fd.mean(0), fd.std(0, ddof=1) / math.sqrt(reps)
    z = (ma - mf) / np.sqrt(sa ** 2 + sf ** 2 + 1e-30)
    return _r(np.all(np.abs(z) <= k), f"z={np.round(z, 2)}")


def check_transparent_stack(paths=1 << 17, seed=22, k=3.5):
    """Non-scattering stack outside | n0 | n1 | outside (slab bottom): top and
    bottom exits against the incoherent adding of the three Fresnel
    interfaces; normal and cosine incidence; n1 < n0 / ... includes total
    internal reflection at the interface."""
    zs = []
    for n0, n1, inc in ((1.4, 1.6, 0), (1.4, 1.3, 1), (1.4, 0.8, 1)):
        geo = O.Geometry(n_media=2, n_rel=n0, slab_mm=2.0, incidence=inc, rr_weight=0.0)
        tal, _, _ = _layered(geo, (1e-12, 1.0, 0.0), (1e-12, 1.0, 0.0), 0.7, n1, paths, seed)
        R_ref, T_ref = cf.stack_RT(n0, n1, "cosine" if inc else "normal")
        mR, seR = mean_se(tal[0, 0], tal[0, 1], paths)
        # T: a path leaves the bottom with its entry weight
        W0 = ((1.0 - ((n0 - 1) / (n0 + 1)) ** 2) if not inc else None)
        T = tal[0, 2] / paths
        seT = math.sqrt(max(T * (1 - T), 1e-12) / paths) if inc else \
            W0 * math.sqrt(max(T / W0 * (1 - T / W0), 1e-12) / paths)
        zs += [(mR - R_ref) / max(seR, 1e-9), (T - T_ref) / max(seT, 1e-9)]
    return _r(all(abs(z) <= k for z in zs), f"z={np.round(zs, 2)}")


def check_layers_analog_vs_weighted(paths=1 << 18, seed=23, k=3.0):
    """Analog and weighted estimators agree on a scattering two-layer slab with
    an index step at the interface; the analog one conserves energy exactly."""
    base = dict(n_media=2, n_rel=1.45, slab_mm=2.0)
    args = ((8.0, 0.7, 0.8), (2.0, 0.97, 0.6), 0.2, 1.35, paths)
    ta, _, _ = _layered(O.Geometry(analog=True, **base), *args, seed)
    tw, _, _ = _layered(O.Geometry(**base), *args, seed + 100)
    pa = ta[0, 0] / paths
    sa = math.sqrt(pa * (1 - pa) / paths)
    mw, sw = mean_se(tw[0, 0], tw[0, 1], paths)
    z = (pa - mw) / math.hypot(sa, sw)
    energy = ta[0, 0] + ta[0, 2] + ta[0, 3] + ta[0, 4]
    return _r(abs(z) <= k and energy == paths, f"z={z:.2f} analog energy {energy} of {paths}")


def check_layer_trace_invariants(n_paths=3000, seed=24):
    """Every interface crossing happens at z = d and obeys Snell's law
    (n_from sin_from = n_to sin_to, azimuth kept, unit direction, the normal
    component keeps its sign); interface reflections flip uz only; the layer
    reported at the end matches the last depth."""
    n0, n1, d = 1.45, 1.3, 0.15
    geo = O.Geometry(n_media=2, n_rel=n0)
    ev, out = O.layered_trace(geo, [6.0, 1.5], [0.9, 0.95], [0.7, 0.5], d, n1, n_paths=n_paths,
                              n_blocks=1024, seed=seed)
    nv = out[:, 5].astype(np.int64)
    vidx = np.arange(1, ev.shape[1])[None, :]
    live = vidx <= nv[:, None]
    prev, cur = ev[:, :-1][live], ev[:, 1:][live]
    code = cur[:, 0].astype(int)
    fails = []
    cr = code == O.EV_CROSS
    if not np.all(cur[cr, 3] == d):
        fails.append("crossing off the interface")
    down = prev[cr, 6] > 0
    n_from = np.where(down, n0, n1)
    n_to = np.where(down, n1, n0)
    s_from = np.hypot(prev[cr, 4], prev[cr, 5])
    s_to = np.hypot(cur[cr, 4], cur[cr, 5])
    if np.any(np.abs(n_from * s_from - n_to * s_to) > 1e-12):
        fails.append("Snell")
    if np.any(np.abs(np.arctan2(cur[cr, 5], cur[cr, 4]) - np.arctan2(prev[cr, 5], prev[cr, 4]))
              > 1e-9 * (s_from > 1e-6)):
        fails.append("azimuth at crossing")
    if np.any(np.sign(cur[cr, 6]) != np.sign(prev[cr, 6])):
        fails.append("crossing reversed")
    if np.any(np.abs(np.linalg.norm(cur[cr, 4:7], axis=1) - 1.0) > 1e-12):
        fails.append("direction not unit after crossing")
    rf = (code == O.EV_REFLECT) & (cur[:, 3] == d)
    if not (np.array_equal(cur[rf, 4], prev[rf, 4]) and np.array_equal(cur[rf, 6], -prev[rf, 6])):
        fails.append("interface reflection law")
    # the layer at the end: a path that ends by an exit or collision at depth z
    last = ev[np.arange(n_paths), nv]
    z_end = last[:, 3]
    ended = out[:, 0] == O.END_RR_KILLED
    exp_layer = (z_end[ended] > d).astype(float)
    if not np.array_equal(out[ended, 1], exp_layer):
        fails.append("layer index")
    n_cross = int(cr.sum())
    n_if_refl = int(rf.sum())
    ok = not fails and n_cross > 100 and n_if_refl > 10
    return _r(ok, f"fails={fails} crossings={n_cross} interface reflections={n_if_refl}")


# ---- multiple scattering with g != 0 and Fresnel: adding-doubling ------------
def _hero(geo, members, d, n_bottom, C, paths, seed):
    """members: list over units of ((sigma_t, albedo, g) top, (...) bottom)."""
    s = np.array([[m[0][0] for m in members], [m[1][0] for m in members]], np.float64)
    a = np.array([[m[0][1] for m in members], [m[1][1] for m in members]], np.float64)
    g = np.array([[m[0][2] for m in members], [m[1][2] for m in members]], np.float64)
    geo = O.Geometry(**{**geo.__dict__, "max_vertices": min(geo.max_vertices, 1 << 16)})
    return O.layered_hero_forward(geo, s, a, g, np.full(len(members), d), n_bottom, C, paths,
                                  seed)


def check_hero_reduces_to_the_plain_walk(paths=1 << 13, seed=40):
    """Hero-wavelength groups in the two-layer walk, two exact reductions:
    (i) a group of one (C = 1) is the plain walk itself, bit for bit (same
        streams, same weights and roulette), with an index step at the
        interface and both incidence modes;
    (ii) a group of C identical members gives every member the plain walk of
        that group's stream (the balance weights are 1/C each), to rounding."""
    rng = np.random.default_rng(seed)
    n = 6
    for inc, n0, n1 in ((0, 1.4, 1.4), (1, 1.4, 1.33)):
        geo = O.Geometry(n_media=2, n_rel=n0, incidence=inc, n_bins=24, r_min_mm=1e-2,
                         r_max_mm=20.0)
        s = np.stack([rng.uniform(5, 40, n), rng.uniform(0.5, 5, n)])
        a = np.stack([rng.uniform(0.3, 0.9, n), rng.uniform(0.8, 0.995, n)])
        g = np.stack([rng.uniform(0.0, 0.9, n), rng.uniform(0.0, 0.9, n)])
        d = rng.uniform(0.05, 0.3, n)
        t1, b1, v1 = O.layered_hero_forward(geo, s, a, g, d, n1, 1, paths, seed)
        t0, b0, v0 = O.layered_forward(geo, s, a, g, d, n1, paths, seed)
        if not (np.array_equal(t1[:, :3], t0[:, :3]) and np.array_equal(b1, b0) and
                np.array_equal(v1, v0)):
            return _r(False, f"C = 1 differs from the plain walk (incidence {inc})")
        # (ii) three copies of unit 2 as one group (group 0 draws unit 0's stream)
        C = 3
        N = paths - paths % C  # a multiple of C: every member is hero equally often
        rep = lambda x: np.repeat(x[:, 2:3], C, axis=1)  # noqa: E731
        th, bh, _ = O.layered_hero_forward(geo, rep(s), rep(a), rep(g), np.full(C, d[2]), n1, C,
                                           N, seed)
        tp, bp, _ = O.layered_forward(geo, s[:, 2:3], a[:, 2:3], g[:, 2:3], d[2:3], n1, N,
                                      seed)
        for i in range(C):
            if not (np.allclose(th[i, :3], tp[0, :3], rtol=1e-12, atol=0) and
                    np.allclose(bh[i], bp[0], rtol=1e-12, atol=0)):
                return _r(False, f"identical members differ from the plain walk (member {i})")
    return _r(True, "")


def check_hero_against_closed_forms(paths=1 << 17, seed=41, k=3.5):
    """Members that differ from the hero are reweighted by their path-density
    ratios; their estimates must match closed forms of their own optics:
    (i) an absorbing non-scattering top layer over an isotropic bottom (n = 1)
        with members differing in the top layer's sigma_t (optical thickness
        0.2, 0.5, 0.9) and the bottom's albedo, against
        e^-tau int dR/dmu e^(-tau/mu) dmu;
    (ii) two scattering layers with a Fresnel surface whose members differ in
        g, sigma_t and albedo of both layers, against adding-doubling."""
    from oracle import adding_doubling as AD

    zs = []
    paths -= paths % 3  # a multiple of the group size
    geo = O.Geometry(n_media=2, n_rel=1.0)
    d = 0.25
    taus, als = (0.2, 0.5, 0.9), (0.95, 0.9, 0.8)
    mem = [((t / d, 0.0, 0.0), (3.0, al, 0.0)) for t, al in zip(taus, als)]
    tal, _, _ = _hero(geo, mem, d, 1.0, 3, paths, seed)
    for i, (t, al) in enumerate(zip(taus, als)):
        m, se = mean_se(tal[i, 0], tal[i, 1], paths)
        zs.append((m - cf.R_absorbing_top(al, t)) / se)
    geo = O.Geometry(n_media=2, n_rel=1.4)
    d = 0.1
    tops = ((8.0, 0.7, 0.8), (7.0, 0.75, 0.7), (9.0, 0.65, 0.85))
    bots = ((2.0, 0.97, 0.6), (1.8, 0.95, 0.7), (2.3, 0.98, 0.5))
    tal, _, _ = _hero(geo, list(zip(tops, bots)), d, 1.4, 3, paths, seed + 1)
    for i, (tp, bt) in enumerate(zip(tops, bots)):
        m, se = mean_se(tal[i, 0], tal[i, 1], paths)
        zs.append((m - AD.two_layer_R((tp[1], tp[2], tp[0] * d), (bt[1], bt[2]), 1.4)) / se)
    return _r(all(abs(z) <= k for z in zs), f"z={np.round(zs, 2)}")


def check_adding_doubling(paths=1 << 18, seed=30, k=3.0):
    """Totals of multiply-scattering media with anisotropic scattering and a
    Fresnel boundary against the deterministic adding-doubling solution
    (oracle/adding_doubling.py): semi-infinite media under a normal beam and a
    cosine lobe, R and T of a slab, and a two-layer medium."""
    from oracle import adding_doubling as AD

    zs = []
    for al, g, n, inc in ((0.9, 0.8, 1.4, 0), (0.97, 0.5, 1.33, 1), (0.6, -0.3, 1.0, 0)):
        geo = O.Geometry(n_media=1, n_rel=n, incidence=inc)
        tal, _, _ = O.forward(geo, [2.0], [al], [g], [1.0], paths, seed)
        m, se = mean_se(tal[0, 0], tal[0, 1], paths)
        zs.append((m - AD.R_semi_infinite(al, g, n, "cosine" if inc else "normal")) / se)
    # slab of optical thickness 2 with Fresnel faces: R and T
    geo = O.Geometry(n_media=1, n_rel=1.4, slab_mm=1.0)
    tal, _, _ = O.forward(geo, [2.0], [0.95], [0.6], [1.0], paths, seed + 1)
    R_ref, T_ref = AD.slab_RT(0.95, 0.6, 1.4, 2.0)
    m, se = mean_se(tal[0, 0], tal[0, 1], paths)
    T = tal[0, 2] / paths
    zs += [(m - R_ref) / se, (T - T_ref) / math.sqrt(T_ref * (1 - T_ref) / paths)]
    # two layers (matched interface): top tau = 0.8 over a semi-infinite bottom
    geo = O.Geometry(n_media=2, n_rel=1.4)
    tal, _, _ = O.layered_forward(geo, [[8.0], [2.0]], [[0.7], [0.97]], [[0.8], [0.6]], [0.1],
                                  1.4, paths, seed + 2)
    m, se = mean_se(tal[0, 0], tal[0, 1], paths)
    zs.append((m - AD.two_layer_R((0.7, 0.8, 0.8), (0.97, 0.6), 1.4)) / se)
    return _r(all(abs(z) <= k for z in zs), f"z={np.round(zs, 2)}")


def check_dwivedi_nu0():
    """nu0 (root > 1 of alpha nu atanh(1/nu) = 1) against scipy's brentq on the
    same equation, its diffusion limit nu0 sqrt(3 (1 - alpha)) -> 1, and the
    clamp of the albedo to [0.3, 1 - 1e-7]."""
    from scipy import optimize

    errs = []
    for al in (0.3, 0.5, 0.7, 0.9, 0.99, 0.999):
        ref = optimize.brentq(lambda v: al * v * math.atanh(1.0 / v) - 1.0, 1.0 + 1e-14, 1e7,
                              xtol=1e-15, rtol=1e-15)
        errs.append(abs(O.dwivedi_nu0(al) / ref - 1.0))
    lim = O.dwivedi_nu0(0.99999) * math.sqrt(3 * 1e-5)
    clamp = O.dwivedi_nu0(0.1) == O.dwivedi_nu0(0.3)
    ok = max(errs) < 1e-12 and abs(lim - 1.0) < 1e-3 and clamp
    return _r(ok, f"rel errs {max(errs):.1e} limit {lim:.6f} clamp {clamp}")


def check_dwivedi_weights_telescope(n_paths=1500, seed=31):
    """Isotropic, index-matched, technique probability 1: the weight factor of
    a collision is alpha lam nu0 / 2 e^(sigma_t dz / nu0) = e^(sigma_t dz / nu0)
    (nu0's equation), so an exiting path carries exactly
    alpha e^(-sigma_t z1 / nu0) lam (nu0 - mu_exit) / 2, z1 the depth of its
    first collision (the entry flight is plain), mu_exit the cosine of its exit
    direction with the outward normal."""
    worst, n_exit = 0.0, 0
    for al, sig in ((0.99, 2.0), (0.8, 0.7)):
        nu = O.dwivedi_nu0(al)
        lam = math.log((nu + 1.0) / (nu - 1.0))
        geo = O.Geometry(n_media=1, n_rel=1.0)
        ev, out, _ = O.trace(geo, [sig], [al], [0.0], [1.0], n_paths=n_paths, n_blocks=2048,
                             seed=seed, dwivedi_q=1.0)
        for p in np.where(out[:, 0] == 1)[0]:
            nv = int(out[p, 5])
            if nv < 2:
                continue
            pred = al * math.exp(-sig * ev[p, 1, 3] / nu) * lam * (nu + ev[p, nv, 6]) / 2.0
            worst = max(worst, abs(out[p, 3] / pred - 1.0))
            n_exit += 1
    return _r(worst < 1e-10 and n_exit > n_paths, f"worst rel {worst:.1e} over {n_exit} exits")


def check_dwivedi_closed_forms(paths=1 << 17, seed=32, k=3.5):
    """The Dwivedi walk is unbiased: (i) isotropic index-matched half-spaces
    against Chandrasekhar's 1 - H(1) sqrt(1 - alpha), technique probability 1
    and 0.5; (ii) anisotropic media, some with a Fresnel surface, against
    adding-doubling (probabilities 0.2-1), forward-peaked ones (g = 0.9) among
    them at albedos where the weights' variance stays finite."""
    from oracle import adding_doubling as AD

    zs = []
    geo = O.Geometry(n_media=1, n_rel=1.0)
    al = np.array([0.5, 0.9, 0.99])
    for q in (1.0, 0.5):
        tal, _, _ = O.dwivedi_forward(geo, np.ones(3), al, np.zeros(3), np.ones(3), paths, seed, q)
        m, se = mean_se(tal[:, 0], tal[:, 1], paths)
        zs += list((m - np.array([cf.R_plane(a) for a in al])) / se)
    for a, g, n, q in ((0.7, 0.5, 1.4, 0.5), (0.9, 0.3, 1.4, 0.3), (0.6, -0.3, 1.0, 1.0),
                       (0.9, 0.9, 1.4, 0.2), (0.95, 0.9, 1.0, 0.2)):
        geo = O.Geometry(n_media=1, n_rel=n)
        tal, _, _ = O.dwivedi_forward(geo, [2.0], [a], [g], [1.0], paths, seed + 1, q)
        m, se = mean_se(tal[0, 0], tal[0, 1], paths)
        zs.append((m - AD.R_semi_infinite(a, g, n, "normal")) / se)
    return _r(all(abs(z) <= k for z in zs), f"z={np.round(zs, 2)}")


def check_dwivedi_vs_plain(paths=1 << 17, seed=33, k=3.5):
    """An isotropic three-medium mixture under a Fresnel surface (n = 1.4):
    the Dwivedi walk (probability 1) and the plain walk estimate the same R and
    radial histogram (independent streams; combined standard errors)."""
    K = 3
    geo = O.Geometry(n_media=K, n_rel=1.4, n_bins=32, r_min_mm=1e-2, r_max_mm=20.0)
    s = np.array([[0.5, 3.0], [4.0, 1.0], [20.0, 8.0]])
    a = np.array([[0.95, 0.7], [0.999, 0.9], [0.6, 0.99]])
    g = np.zeros((K, 2))
    w = np.array([[0.2, 0.5], [0.5, 0.3], [0.3, 0.2]])
    td, bd, _ = O.dwivedi_forward(geo, s, a, g, w, paths, seed, 1.0)
    tp, bp, _ = O.forward(geo, s, a, g, w, paths, seed + 1)
    md, sd = mean_se(td[:, 0], td[:, 1], paths)
    mp, sp = mean_se(tp[:, 0], tp[:, 1], paths)
    z = (md - mp) / np.hypot(sd, sp)
    ok = bool(np.all(np.abs(z) <= k))
    for u in range(2):
        m1, s1 = mean_se(bd[u, :, 0], bd[u, :, 1], paths)
        m2, s2 = mean_se(bp[u, :, 0], bp[u, :, 1], paths)
        zb = histogram_z(m1, s1, m2, s2, mask=(m1 > 0) & (m2 > 0))
        hok, chi2, lim = accept_histogram(zb)
        ok = ok and hok
    return _r(ok, f"z={np.round(z, 2)}")


BATTERY_SMALL = [
    ("plane", lambda: check_plane_albedo(alphas=(0.5, 0.9), paths=1 << 16, k=4.0)),
    ("second_moment", lambda: check_second_moment(paths=1 << 16, k=4.0)),
    ("single_scatter", lambda: check_single_scatter(paths=1 << 16, k=4.0, n_bins=32)),
    ("energy", lambda: check_energy_exact(paths=1 << 12)),
    ("analog", lambda: check_analog_vs_weighted(paths=1 << 16, k=4.0)),
    ("beer", lambda: check_beer_lambert(paths=1 << 16, k=4.0)),
    ("mixture", lambda: check_mixture_linearity(paths=1 << 16, k=4.0)),
    ("special", lambda: check_single_medium_special_case(paths=1 << 12)),
    ("scale", lambda: check_scale_invariance(paths=1 << 12)),
    ("trace", lambda: check_trace_invariants(n_paths=1500)),
    ("brute", lambda: check_brute_force_single_scatter(m=32)),
    ("adj_plane", lambda: check_adjoint_plane(paths=1 << 16, k=4.0)),
    ("adj_mixture", lambda: check_adjoint_mixture(paths=1 << 16, k=4.0)),
    ("jacobian", lambda: check_jacobian(paths=1 << 11)),
    ("spherical", lambda: check_spherical_albedo(paths=1 << 16, k=4.0)),
    ("analog_cosine", lambda: check_analog_vs_weighted_cosine(paths=1 << 16, k=4.0)),
    ("layers_beer", lambda: check_two_layer_beer_lambert(paths=1 << 16, k=4.0)),
    ("layers_plane", lambda: check_layers_reduce_to_plane(paths=1 << 16, k=4.0)),
    ("layers_absorbing_top", lambda: check_absorbing_top_layer(paths=1 << 16, k=4.0)),
    ("layers_adj_absorbing_top",
     lambda: check_layered_adjoint_absorbing_top(paths=1 << 16, k=4.0)),
    ("layers_stack", lambda: check_transparent_stack(paths=1 << 15, k=4.0)),
    ("layers_analog", lambda: check_layers_analog_vs_weighted(paths=1 << 16, k=4.0)),
    ("layers_trace", lambda: check_layer_trace_invariants(n_paths=1500)),
    ("adding_doubling", lambda: check_adding_doubling(paths=1 << 16, k=4.0)),
    ("hero_reductions", lambda: check_hero_reduces_to_the_plain_walk(paths=1 << 11)),
    ("hero_closed_forms", lambda: check_hero_against_closed_forms(paths=1 << 16, k=4.0)),
    ("dwivedi_nu0", check_dwivedi_nu0),
    ("dwivedi_telescope", lambda: check_dwivedi_weights_telescope(n_paths=300)),
    ("dwivedi_closed_forms", lambda: check_dwivedi_closed_forms(paths=1 << 15, k=4.0)),
    ("dwivedi_vs_plain", lambda: check_dwivedi_vs_plain(paths=1 << 15, k=4.0)),
]
