"""Adding-doubling solution of the plane-parallel transport problem, as an
independent deterministic reference for the random walk's totals.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

The random walk estimates the total diffuse reflectance R (and, for a slab,
the transmittance T) of a homogeneous medium with albedo alpha,
Henyey-Greenstein anisotropy g and a smooth Fresnel boundary of relative index
n (Sec. 4.1, eq. sss; Sec. 8 for the boundary).  For azimuthally symmetric
illumination (a normal pencil beam or a cosine lobe) the totals depend only on
the azimuthally averaged radiance, which the adding-doubling method computes on
a quadrature in mu = cos(theta) (van de Hulst, "Multiple Light Scattering",
1980; Prahl, "The adding-doubling method", in Optical-Thermal Response of
Laser-Irradiated Tissue, 1995):

* Directions: per hemisphere, Gauss-Legendre nodes on [0, mu_c] and
  Gauss-Radau nodes on [mu_c, 1] with the node mu = 1 (the normal beam),
  mu_c = sqrt(1 - 1/n^2) the critical cosine inside (where the boundary's
  reflectance has its kink and the refracted cone ends); one Radau interval
  when n <= 1.
* Operators act on flux-normalised radiance v_i = sqrt(c_i) L_i, with
  c_i = 2 mu_i w_i, so that layers combine by ordinary matrix products.
* Phase function: the azimuthal average of Henyey-Greenstein is
  h(mu, mu') = sum_l (2l + 1) g^l P_l(mu) P_l(mu'), a polynomial that the
  quadrature integrates exactly for the degrees used (truncated where g^l is
  below 1e-17).
* A layer of optical thickness dtau (2^-32) starts from single scattering:
  R_ij = alpha dtau h(-mu_i, mu_j) sqrt(w_i w_j / (mu_i mu_j)) / 2, the same with
  h(mu_i, mu_j) plus exp(-dtau / mu_i) on the diagonal for T.  Doubling,
  R2 = R + T (I - R R)^-1 R T and T2 = T (I - R R)^-1 T, reaches the slab
  thickness (or 2^12 for a semi-infinite medium, far beyond the diffusion
  length of the albedos tested).
* The smooth boundary reflects specularly with the unpolarised Fresnel
  reflectance F(mu_i) seen from inside (diagonal); what it transmits leaves.
  Light entering refracts into the cone mu >= mu_c, carrying 1 - F.

Pinned in tests against closed forms: the plane albedo and the spherical
albedo for g = 0, n = 1; the single-scattering term for any g and n as
alpha -> 0; Beer-Lambert with Fresnel faces for a non-scattering slab; energy
conservation for alpha = 1; for two layers, identical layers, a vanishing top
layer and an absorbing top layer over an isotropic bottom (Chandrasekhar's
exit law).
"""
from __future__ import annotations

import math

import numpy as np

from . import closed_forms as cf

DTAU0 = 2.0 ** -32


def _gauss(n: int, a: float, b: float):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _radau_upper(n: int, a: float, b: float):
    """Gauss-Radau nodes and weights on [a, b] with the fixed node b.  On
    [-1, 1] with the fixed node -1 the other nodes are the roots of
    (P_{n-1}(x) + P_n(x)) / (1 + x), weights 2/n^2 at -1 and
    (1 - x) / (n^2 P_{n-1}(x)^2) elsewhere; x -> b - (b - a)(x + 1)/2 maps
    -1 to b."""
    Pn1 = np.polynomial.legendre.Legendre.basis(n - 1)
    Pn = np.polynomial.legendre.Legendre.basis(n)
    q = (Pn1 + Pn)
    # divide by (1 + x): roots of q other than -1
    roots = np.sort(np.real(q.roots()))
    roots = roots[np.abs(roots + 1.0) > 1e-10]
    x = np.concatenate([[-1.0], roots])
    w = np.empty(n)
    w[0] = 2.0 / n ** 2
    w[1:] = (1.0 - roots) / (n ** 2 * Pn1(roots) ** 2)
    mu = b - (b - a) * (x + 1.0) / 2.0
    return mu, w * (b - a) / 2.0


def quadrature(n_rel: float, n_nodes: int = 64):
    """Nodes mu (descending from 1) and weights on (0, 1] for a medium of
    relative index n_rel: split at the critical cosine when n_rel > 1."""
    if n_rel > 1.0:
        mu_c = math.sqrt(1.0 - 1.0 / (n_rel * n_rel))
        m1, w1 = _radau_upper(n_nodes, mu_c, 1.0)
        m2, w2 = _gauss(n_nodes, 0.0, mu_c)
        mu, w = np.concatenate([m1, m2[::-1]]), np.concatenate([w1, w2[::-1]])
    else:
        mu, w = _radau_upper(2 * n_nodes, 0.0, 1.0)
    return mu, w


def _legendre_table(x: np.ndarray, L: int) -> np.ndarray:
    """P_l(x) for l = 0..L by the three-term recurrence; shape [L + 1, len(x)]."""
    P = np.zeros((L + 1, x.size))
    P[0] = 1.0
    if L >= 1:
        P[1] = x
    for l in range(1, L):
        P[l + 1] = ((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1)
    return P


def redistribution(mu: np.ndarray, g: float):
    """Azimuthally averaged HG phase function between the nodes:
    (h(mu_i, mu_j), h(-mu_i, mu_j)), normalised so that
    (1/2) int_-1^1 h(mu, mu') dmu' = 1."""
    if g == 0.0:
        one = np.ones((mu.size, mu.size))
        return one, one
    L = max(1, int(math.ceil(math.log(1e-17) / math.log(abs(g)))))
    P = _legendre_table(mu, L)
    l = np.arange(L + 1)
    coef = (2 * l + 1) * g ** l
    same = (P * coef[:, None]).T @ P                 # sum_l (2l+1) g^l P_l(mu_i) P_l(mu_j)
    opp = (P * (coef * (-1.0) ** l)[:, None]).T @ P  # P_l(-mu) = (-1)^l P_l(mu)
    return same, opp


def layer(alpha: float, g: float, tau: float, mu: np.ndarray, w: np.ndarray):
    """(R, T) of a homogeneous layer of optical thickness tau (flux-normalised
    operators, symmetric layer: the same from both sides)."""
    same, opp = redistribution(mu, g)
    s = np.sqrt(w / mu)
    S = np.outer(s, s) / 2.0
    k = 0
    while DTAU0 * 2.0 ** k < tau:
        k += 1
    dtau = tau / 2.0 ** k
    R = alpha * dtau * opp * S
    T = alpha * dtau * same * S + np.diag(np.exp(-dtau / mu))
    I = np.eye(mu.size)
    for _ in range(k):
        A = np.linalg.solve(I - R @ R, np.eye(mu.size))
        TA = T @ A
        R, T = R + TA @ R @ T, TA @ T
    return R, T


def _fresnel_inside(mu: np.ndarray, n_rel: float) -> np.ndarray:
    return np.array([cf.fresnel_hecht(float(m), n_rel) for m in mu])


def _entry(mu, w, n_rel, incidence):
    """Flux-normalised radiance entering the medium per unit incident flux,
    and the specular part.  Normal: 1 - F(1) into mu = 1 (node 0).  Cosine
    lobe: inside, the flux density per dmu_in is 2 n^2 mu_in (1 - F) on the
    refracted cone mu_in >= mu_c (change of variables of 2 mu_out dmu_out)."""
    c = 2.0 * mu * w
    F = _fresnel_inside(mu, n_rel)
    v = np.zeros(mu.size)
    if incidence == "normal":
        v[0] = (1.0 - F[0]) / math.sqrt(c[0])
        return v, F[0]
    mu_c = math.sqrt(1.0 - 1.0 / n_rel ** 2) if n_rel > 1.0 else 0.0
    inside = mu >= mu_c - 1e-15
    flux = np.where(inside, n_rel ** 2 * c * (1.0 - F), 0.0)
    v = flux / np.sqrt(c)
    return v, 1.0 - flux.sum()


def slab_RT(alpha: float, g: float, n_rel: float, tau: float | None = None,
            incidence: str = "normal", n_nodes: int = 64):
    """Total diffuse reflectance R (specular excluded) and transmittance T of a
    homogeneous slab of optical thickness tau (None: semi-infinite) with
    smooth Fresnel faces of relative index n_rel on both sides."""
    mu, w = quadrature(n_rel, n_nodes)
    semi = tau is None
    R, T = layer(alpha, g, 2.0 ** 12 if semi else tau, mu, w)
    F = np.diag(_fresnel_inside(mu, n_rel))
    Tout = np.eye(mu.size) - F
    v_in, _ = _entry(mu, w, n_rel, incidence)
    c = 2.0 * mu * w
    I = np.eye(mu.size)
    if semi:
        # up-going light at the top: (I - R F)^-1 R v_in
        up = np.linalg.solve(I - R @ F, R @ v_in)
        return float(np.sqrt(c) @ (Tout @ up)), 0.0
    # Slab between two specular faces F.  Unknowns: a = the downward radiance
    # entering the medium at the top (incident light plus what the top face
    # reflects back), b = the upward radiance entering it at the bottom:
    #   up at the top = R a + T b,   down at the bottom = T a + R b,
    #   a = v_in + F (R a + T b),    b = F (T a + R b).
    n = mu.size
    M = np.block([[I - F @ R, -F @ T], [-F @ T, I - F @ R]])
    rhs = np.concatenate([v_in, np.zeros(n)])
    ab = np.linalg.solve(M, rhs)
    a, b = ab[:n], ab[n:]
    up_top = R @ a + T @ b
    down_bottom = T @ a + R @ b
    Rt = float(np.sqrt(c) @ (Tout @ up_top))
    Tt = float(np.sqrt(c) @ (Tout @ down_bottom))
    return Rt, Tt


def R_semi_infinite(alpha: float, g: float, n_rel: float, incidence: str = "normal",
                    n_nodes: int = 64) -> float:
    return slab_RT(alpha, g, n_rel, None, incidence, n_nodes)[0]


def two_layer_R(top, bottom, n_rel: float, incidence: str = "normal", n_nodes: int = 64) -> float:
    """Total diffuse reflectance of a top layer (alpha, g, tau) over a
    semi-infinite bottom layer (alpha, g), both of relative index n_rel (an
    index-matched interface: the layers add without reflection between them),
    under a smooth Fresnel surface.  Homogeneous layers reflect alike from both
    sides, so adding gives R = R1 + T1 (I - R2 R1)^-1 R2 T1."""
    mu, w = quadrature(n_rel, n_nodes)
    R1, T1 = layer(top[0], top[1], top[2], mu, w)
    R2, _ = layer(bottom[0], bottom[1], 2.0 ** 12, mu, w)
    I = np.eye(mu.size)
    R = R1 + T1 @ np.linalg.solve(I - R2 @ R1, R2 @ T1)
    F = np.diag(_fresnel_inside(mu, n_rel))
    v_in, _ = _entry(mu, w, n_rel, incidence)
    c = 2.0 * mu * w
    up = np.linalg.solve(I - R @ F, R @ v_in)
    return float(np.sqrt(c) @ ((I - F) @ up))


def entry_specular(n_rel: float, incidence: str = "normal", n_nodes: int = 64) -> float:
    """The part of the incident flux reflected at entry (excluded from R)."""
    mu, w = quadrature(n_rel, n_nodes)
    return _entry(mu, w, n_rel, incidence)[1]
