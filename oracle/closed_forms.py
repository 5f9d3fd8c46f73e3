"""Closed forms and quadratures that pin the oracle.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

None of these come from the random walk itself; each is an independent
mathematical statement about the quantity the walk estimates:

* Isotropic scattering, index-matched boundary, normal incidence on a
  semi-infinite homogeneous medium: the plane albedo is
  R = 1 - H(1) * sqrt(1 - alpha), with Chandrasekhar's H-function
  (S. Chandrasekhar, *Radiative Transfer*, 1950/1960, ch. V).  H is computed two
  independent ways (the non-linear integral equation iterated on Gauss-Legendre
  nodes, and the explicit integral representation), which must agree.
* dR/dalpha from the explicit representation.
* The single-scattering term (exactly one collision before the path leaves the
  top surface), as a 1-D quadrature for any Henyey-Greenstein g and any
  relative index n (smooth Fresnel boundary, paper Sec. 8 "Limitations"), in
  total and per radial annulus.
* Fresnel reflectance in Hecht's sine/tangent form (a different formula for the
  same quantity as the amplitude form the oracle uses).
* Beer-Lambert transmission of a purely absorbing slab.

The paper's own relation used as a pin elsewhere: scale separability
(Sec. 4.2, eq. separability) - R does not depend on sigma_t, the profile
rescales with 1/sigma_t.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


# --------------------------------------------------------------------------
# Chandrasekhar H-function for isotropic scattering with albedo w
# --------------------------------------------------------------------------
def _gauss_legendre_01(n: int):
    x, wt = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * wt


def H_iterative(mu, w: float, n_nodes: int = 400, tol: float = 1e-14, max_iter: int = 200000):
    """H(mu) from 1/H(mu) = sqrt(1-w) + (w/2) int_0^1 mu' H(mu') / (mu + mu') dmu',
    iterated on Gauss-Legendre nodes (valid for w < 1)."""
    if not (0.0 <= w < 1.0):
        raise ValueError("iterative form needs 0 <= w < 1")
    x, wt = _gauss_legendre_01(n_nodes)
    H = np.ones_like(x)
    s = math.sqrt(1.0 - w)
    K = x[None, :] * wt[None, :] / (x[:, None] + x[None, :])
    for _ in range(max_iter):
        Hn = 1.0 / (s + 0.5 * w * (K @ H))
        if np.max(np.abs(Hn - H)) < tol:
            H = Hn
            break
        H = Hn
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    Km = x[None, :] * wt[None, :] / (mu[:, None] + x[None, :])
    out = 1.0 / (s + 0.5 * w * (Km @ H))
    return out if out.size > 1 else float(out[0])


def _theta_cot(t):
    return t / math.tan(t) if t > 0.0 else 1.0


def _one_minus_theta_cot(t):
    """1 - theta cot(theta), by its Taylor series where it cancels."""
    if t < 1e-3:
        t2 = t * t
        return t2 / 3.0 + t2 * t2 / 45.0 + 2.0 * t2 * t2 * t2 / 945.0
    return 1.0 - t / math.tan(t)


def H_explicit(mu: float, w: float) -> float:
    """H(mu) = exp( -(mu/pi) int_0^{pi/2} ln(1 - w theta cot theta)
    / (cos^2 theta + mu^2 sin^2 theta) dtheta )."""
    def f(t):
        return math.log((1.0 - w) + w * _one_minus_theta_cot(t)) / (
            math.cos(t) ** 2 + (mu * math.sin(t)) ** 2)

    val, _ = integrate.quad(f, 0.0, 0.5 * math.pi, limit=400, epsabs=1e-14, epsrel=1e-13)
    return math.exp(-mu / math.pi * val)


def H_moment0(w: float) -> float:
    """int_0^1 H(mu) dmu = (2/w)(1 - sqrt(1 - w))."""
    return 2.0 / w * (1.0 - math.sqrt(1.0 - w))


def R_plane(alpha: float) -> float:
    """Total diffuse reflectance, isotropic scattering, n = 1, normal incidence."""
    return 1.0 - H_explicit(1.0, alpha) * math.sqrt(1.0 - alpha)


def H_moment1(w: float, form: str = "explicit") -> float:
    """First moment int_0^1 mu H(mu) dmu, by quadrature of either H form."""
    if form == "explicit":
        val, _ = integrate.quad(lambda m: m * H_explicit(m, w), 0.0, 1.0, limit=200,
                                epsabs=1e-13, epsrel=1e-12)
        return val
    x, wt = _gauss_legendre_01(400)
    return float(np.sum(wt * x * H_iterative(x, w)))


def R_spherical(alpha: float) -> float:
    """Total diffuse reflectance under cosine-weighted (diffuse) incidence,
    isotropic scattering, n = 1: the cosine-weighted average of the plane
    albedo, 2 int_0^1 mu (1 - H(mu) sqrt(1 - alpha)) dmu."""
    return 1.0 - 2.0 * math.sqrt(1.0 - alpha) * H_moment1(alpha)


def dlnH1_dw(w: float) -> float:
    def f(t):
        return _theta_cot(t) / ((1.0 - w) + w * _one_minus_theta_cot(t))

    val, _ = integrate.quad(f, 0.0, 0.5 * math.pi, limit=400, epsabs=1e-14, epsrel=1e-13)
    return val / math.pi


def dR_plane_dalpha(alpha: float) -> float:
    H1 = H_explicit(1.0, alpha)
    s = math.sqrt(1.0 - alpha)
    return -H1 * (dlnH1_dw(alpha) * s - 0.5 / s)


# --------------------------------------------------------------------------
# Fresnel (Hecht's form) and single scattering
# --------------------------------------------------------------------------
def fresnel_hecht(cos_i: float, n: float) -> float:
    """Unpolarised reflectance, light inside index n going out to index 1:
    R = (sin^2(ti - tt)/sin^2(ti + tt) + tan^2(ti - tt)/tan^2(ti + tt)) / 2,
    with Snell sin(tt) = n sin(ti); 1 under total internal reflection; normal
    incidence ((n-1)/(n+1))^2."""
    cos_i = min(max(cos_i, 0.0), 1.0)
    ti = math.acos(cos_i)
    st = n * math.sin(ti)
    if st >= 1.0:
        return 1.0
    if ti < 1e-7:
        return ((n - 1.0) / (n + 1.0)) ** 2
    tt = math.asin(st)
    if abs(ti - tt) < 1e-300:
        return 0.0
    a = math.sin(ti - tt) ** 2 / math.sin(ti + tt) ** 2
    b = math.tan(ti - tt) ** 2 / math.tan(ti + tt) ** 2 if abs(ti + tt - 0.5 * math.pi) > 1e-12 else 0.0
    return 0.5 * (a + b)


def hg_pdf(mu, g: float):
    """Henyey-Greenstein density in mu = cos(theta), normalised on [-1, 1]."""
    return 0.5 * (1.0 - g * g) / (1.0 + g * g - 2.0 * g * np.asarray(mu)) ** 1.5


def R1_total(alpha: float, g: float, n: float) -> float:
    """Mean contribution of paths that leave the top after exactly one collision:
    (1 - F0) alpha int_0^1 p_HG(-mu) (1 - F(mu)) mu / (1 + mu) dmu."""
    F0 = ((n - 1.0) / (n + 1.0)) ** 2

    def f(mu):
        return float(hg_pdf(-mu, g)) * (1.0 - fresnel_hecht(mu, n)) * mu / (1.0 + mu)

    pts = []
    if n > 1.0:
        pts = [math.sqrt(1.0 - 1.0 / (n * n))]  # critical angle kink
    val, _ = integrate.quad(f, 0.0, 1.0, points=pts or None, limit=400, epsabs=1e-13, epsrel=1e-12)
    return (1.0 - F0) * alpha * val


def R1_annulus(alpha: float, g: float, n: float, sigma_t: float, r_a: float, r_b: float) -> float:
    """Single-scattering mean contribution that exits with radius in [r_a, r_b).

    A collision at depth z followed by an upward direction with cosine mu exits
    at radius z * sqrt(1 - mu^2) / mu; integrating the depth analytically gives
    (mu/(1+mu)) [exp(-c r_a) - exp(-c r_b)] with c = sigma_t (1 + mu) / sqrt(1 - mu^2)."""
    F0 = ((n - 1.0) / (n + 1.0)) ** 2

    def f(mu):
        s = math.sqrt(max(1.0 - mu * mu, 0.0))
        if s == 0.0:
            c = math.inf
        else:
            c = sigma_t * (1.0 + mu) / s
        ea = 1.0 if r_a == 0.0 else (math.exp(-c * r_a) if c < math.inf else 0.0)
        eb = 0.0 if r_b == math.inf else (math.exp(-c * r_b) if c < math.inf else 0.0)
        return float(hg_pdf(-mu, g)) * (1.0 - fresnel_hecht(mu, n)) * mu / (1.0 + mu) * (ea - eb)

    pts = [math.sqrt(1.0 - 1.0 / (n * n))] if n > 1.0 else None
    val, _ = integrate.quad(f, 0.0, 1.0, points=pts, limit=800, epsabs=1e-15, epsrel=1e-11)
    return (1.0 - F0) * alpha * val


def bin_edges(n_bins: int, r_min: float, r_max: float) -> np.ndarray:
    """Edges of the log-spaced radial bins: r_i = r_min (r_max/r_min)^(i/n_bins)."""
    return r_min * (r_max / r_min) ** (np.arange(n_bins + 1) / n_bins)


def R1_slots(alpha: float, g: float, n: float, sigma_t: float, n_bins: int, r_min: float,
             r_max: float) -> np.ndarray:
    """Single-scattering contribution per slot (0 underflow, 1..n_bins, overflow)."""
    e = bin_edges(n_bins, r_min, r_max)
    edges = np.concatenate([[0.0], e, [math.inf]])
    return np.array([R1_annulus(alpha, g, n, sigma_t, edges[i], edges[i + 1])
                     for i in range(n_bins + 2)])


def beer_lambert(sigma_t: float, d: float) -> float:
    return math.exp(-sigma_t * d)


# --------------------------------------------------------------------------
# Two-layer tissue (the paper's data-generation geometry, Sec. 3)
# --------------------------------------------------------------------------
def exit_cosine_density(mu: float, alpha: float) -> float:
    """Chandrasekhar's law of diffuse reflection for a semi-infinite isotropic
    scatterer under normal incidence (ch. IV, mu0 = 1), as a density of the
    exit cosine: dR/dmu = (alpha/2) mu H(mu) H(1) / (1 + mu).  Its integral over
    [0, 1] is the plane albedo."""
    return 0.5 * alpha * mu * H_explicit(mu, alpha) * H_explicit(1.0, alpha) / (1.0 + mu)


def R_absorbing_top(alpha: float, tau: float) -> float:
    """Total reflectance of an isotropic semi-infinite bottom layer (albedo
    alpha) under a non-scattering absorbing top layer of optical thickness tau,
    n = 1 everywhere, normal incidence: the beam reaches the bottom with
    probability e^-tau, and light leaving the bottom at cosine mu crosses the
    top with e^(-tau/mu) (what collides in the top layer is absorbed):
    R = e^-tau int_0^1 dR/dmu e^(-tau/mu) dmu."""
    if tau == 0.0:
        return R_plane(alpha)
    val, _ = integrate.quad(lambda m: exit_cosine_density(m, alpha) * math.exp(-tau / m),
                            0.0, 1.0, limit=200, epsabs=1e-13, epsrel=1e-11)
    return math.exp(-tau) * val


def _stack_at(mu_out: float, n0: float, n1: float):
    """Top exits R (specular excluded) and bottom exits T of a non-scattering
    stack outside | top (n0) | bottom (n1) | outside, for light entering at
    outside cosine mu_out: three parallel interfaces, added incoherently.  The
    polar angle in each layer follows Snell's law (sin is conserved times n);
    each interface reflects the same fraction from both sides at conjugate
    angles (reciprocity), so the adding rule for two interfaces,
    R_ab = R_a + T_a^2 R_b / (1 - R_a R_b),  T_ab = T_a T_b / (1 - R_a R_b),
    applies twice."""
    s2 = 1.0 - mu_out * mu_out
    c0 = math.sqrt(max(0.0, 1.0 - s2 / (n0 * n0)))       # cosine in the top layer
    RA = fresnel_hecht(c0, n0)                           # surface
    RB = fresnel_hecht(c0, n0 / n1)                      # interface, from the top
    if RB >= 1.0:                                        # total internal reflection
        RC, c1 = 0.0, 0.0
    else:
        c1 = math.sqrt(max(0.0, 1.0 - s2 / (n1 * n1)))   # cosine in the bottom layer
        RC = fresnel_hecht(c1, n1)                       # bottom face
    TA, TB, TC = 1.0 - RA, 1.0 - RB, 1.0 - RC
    # surface + interface, seen from the outside and from the bottom layer
    den = 1.0 - RA * RB
    R_ab = RA + TA * TA * RB / den
    T_ab = TA * TB / den
    R_ba = RB + TB * TB * RA / den
    den2 = 1.0 - R_ba * RC
    R_tot = R_ab + T_ab * T_ab * RC / den2
    T_tot = T_ab * TC / den2
    return R_tot - RA, T_tot


def stack_RT(n0: float, n1: float, incidence: str = "normal"):
    """(R, T) of the non-scattering two-layer stack of _stack_at under a normal
    pencil beam or a cosine-weighted lobe (density 2 mu_out)."""
    if incidence == "normal":
        return _stack_at(1.0, n0, n1)
    R, _ = integrate.quad(lambda m: 2.0 * m * _stack_at(m, n0, n1)[0], 0.0, 1.0, limit=400,
                          epsabs=1e-13, epsrel=1e-11)
    T, _ = integrate.quad(lambda m: 2.0 * m * _stack_at(m, n0, n1)[1], 0.0, 1.0, limit=400,
                          epsabs=1e-13, epsrel=1e-11)
    return R, T
