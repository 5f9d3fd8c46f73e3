"""Pins of the closed forms themselves (CPU only).

The closed forms in oracle/closed_forms.py pin the oracle; here they are pinned
against textbook values, identities and each other (two independent
computations of Chandrasekhar's H-function, its moments, a tabulated value,
numerical differentiation, and an elementary integral)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("w", [0.3, 0.5, 0.9, 0.99, 0.999])
def test_H_two_independent_forms_agree(w):
    for mu in (0.05, 0.3, 1.0):
        assert abs(cf.H_iterative(mu, w) - cf.H_explicit(mu, w)) < 1e-10


@pytest.mark.parametrize("w", [0.5, 0.9, 1.0])
def test_H_zeroth_moment_identity(w):
    m0, _ = integrate.quad(lambda m: cf.H_explicit(m, w), 0.0, 1.0, epsabs=1e-12)
    assert abs(m0 - cf.H_moment0(w)) < 1e-9


def test_H_conservative_table_value_and_first_moment():
    with open(os.path.join(GOLDEN, "chandrasekhar_h.json")) as f:
        gold = json.load(f)
    H1 = cf.H_explicit(1.0, 1.0)
    assert abs(H1 - gold["H_at_1"]) < 0.5 * 10.0 ** (-gold["H_at_1_digits"])
    m1, _ = integrate.quad(lambda m: m * cf.H_explicit(m, 1.0), 0.0, 1.0, epsabs=1e-12)
    assert abs(m1 - gold["moment1"]) < 1e-8


@pytest.mark.parametrize("a", [0.5, 0.7, 0.9, 0.99])
def test_dR_dalpha_matches_numerical_derivative(a):
    h = 1e-5
    fd = (cf.R_plane(a + h) - cf.R_plane(a - h)) / (2 * h)
    assert abs(cf.dR_plane_dalpha(a) - fd) < 1e-6 * max(1.0, abs(fd))


def test_plane_albedo_limits():
    # alpha -> 0: no scattering, nothing comes back; alpha -> 1: everything does
    assert abs(cf.R_plane(1e-9)) < 1e-8
    assert abs(cf.R_plane(1.0 - 1e-12) - 1.0) < 1e-5


def test_single_scatter_isotropic_index_matched_is_elementary():
    # alpha * int_0^1 mu / (2 (1 + mu)) dmu = alpha (1 - ln 2) / 2
    for a in (0.3, 1.0):
        assert abs(cf.R1_total(a, 0.0, 1.0) - a * (1.0 - math.log(2.0)) / 2.0) < 1e-12


@pytest.mark.parametrize("g,n", [(0.0, 1.0), (0.5, 1.4), (0.9, 1.4)])
def test_single_scatter_annuli_sum_to_total(g, n):
    slots = cf.R1_slots(0.8, g, n, 2.0, 64, 1e-3, 50.0)
    assert abs(slots.sum() - cf.R1_total(0.8, g, n)) < 1e-9


def test_single_scatter_annulus_scales_with_sigma_t():
    # eq. separability: the profile rescales with 1/sigma_t
    a = cf.R1_annulus(0.9, 0.3, 1.4, 1.0, 0.2, 0.5)
    b = cf.R1_annulus(0.9, 0.3, 1.4, 4.0, 0.05, 0.125)
    assert abs(a - b) < 1e-12


def test_fresnel_hecht_limits():
    assert cf.fresnel_hecht(1.0, 1.4) == pytest.approx((0.4 / 2.4) ** 2, abs=1e-15)
    assert cf.fresnel_hecht(0.3, 1.0) == 0.0
    crit = math.sqrt(1.0 - 1.0 / 1.4 ** 2)
    assert cf.fresnel_hecht(crit * 0.999, 1.4) == 1.0
    assert cf.fresnel_hecht(crit * 1.001, 1.4) < 1.0


def test_golden_files_regenerate():
    with open(os.path.join(GOLDEN, "plane_albedo_16.json")) as f:
        plane = json.load(f)
    for a, R, d in zip(plane["alpha"], plane["R"], plane["dR_dalpha"]):
        assert abs(cf.R_plane(a) - R) < 1e-12
        assert abs(cf.dR_plane_dalpha(a) - d) < 1e-9
    with open(os.path.join(GOLDEN, "single_scatter.json")) as f:
        ss = json.load(f)
    for c in ss["cases"]:
        assert abs(cf.R1_total(1.0, c["g"], c["n"]) - c["R1"]) < 1e-12


def test_H_first_moment_two_forms_and_spherical_albedo_limits():
    for w in (0.3, 0.7, 0.95, 0.999):
        assert abs(cf.H_moment1(w, "explicit") - cf.H_moment1(w, "iterative")) < 1e-10
    assert abs(cf.R_spherical(1e-9)) < 1e-8          # no scattering: nothing returns
    assert abs(cf.R_spherical(1.0) - 1.0) < 1e-12     # conservative: everything returns
    # diffuse light penetrates less deeply than a normal beam: higher albedo
    for a in (0.5, 0.9, 0.99):
        assert cf.R_spherical(a) > cf.R_plane(a)
    # the cosine-weighted mean of the plane albedo over incidence angles
    import numpy as np
    x, w = np.polynomial.legendre.leggauss(64)
    mu = 0.5 * (x + 1.0)
    for a in (0.6, 0.9):
        avg = float(np.sum(0.5 * w * 2 * mu * (1 - np.array([cf.H_explicit(m, a) for m in mu])
                                                     * np.sqrt(1 - a))))
        assert abs(avg - cf.R_spherical(a)) < 1e-9


def test_two_layer_closed_forms_limits():
    # Chandrasekhar's exit law integrates to the plane albedo
    for a in (0.5, 0.9, 0.99):
        val, _ = integrate.quad(lambda m: cf.exit_cosine_density(m, a), 0.0, 1.0, limit=200,
                                epsabs=1e-13)
        assert abs(val - cf.R_plane(a)) < 1e-10
    # an absorbing top layer of vanishing thickness changes nothing; a thick one blocks
    assert abs(cf.R_absorbing_top(0.9, 1e-10) - cf.R_plane(0.9)) < 1e-8
    assert cf.R_absorbing_top(0.9, 30.0) < 1e-14
    # stack: index-matched is fully transparent; equal layers are one slab,
    # T = (1 - F)/(1 + F) at normal incidence; energy R + T + F = 1
    assert cf.stack_RT(1.0, 1.0) == (0.0, 1.0)
    F = (0.4 / 2.4) ** 2
    R, T = cf.stack_RT(1.4, 1.4)
    assert abs(T - (1 - F) / (1 + F)) < 1e-14 and abs(R + T + F - 1.0) < 1e-14
    R, T = cf.stack_RT(1.4, 1.7)
    assert abs(R + T + F - 1.0) < 1e-14
    # cosine incidence: R + T + the lobe-averaged entry reflectance = 1
    Fbar, _ = integrate.quad(
        lambda m: 2 * m * cf.fresnel_hecht(math.sqrt(1 - (1 - m * m) / 1.96), 1.4), 0, 1)
    for n1 in (1.3, 0.8):
        R, T = cf.stack_RT(1.4, n1, "cosine")
        assert abs(R + T + Fbar - 1.0) < 1e-9


def test_adding_doubling_against_closed_forms():
    from oracle import adding_doubling as AD
    # g = 0, n = 1: plane albedo (normal) and spherical albedo (cosine lobe)
    for a in (0.5, 0.9, 0.99):
        assert abs(AD.R_semi_infinite(a, 0.0, 1.0) - cf.R_plane(a)) < 2e-6
    for a in (0.5, 0.9):
        assert abs(AD.R_semi_infinite(a, 0.0, 1.0, "cosine") - cf.R_spherical(a)) < 2e-6
    # alpha -> 0: the single-scattering term, any g and Fresnel index
    a = 1e-4
    for g, n in ((0.0, 1.4), (0.8, 1.4), (0.5, 1.0), (-0.3, 1.33)):
        r1 = cf.R1_total(a, g, n)
        assert abs(AD.R_semi_infinite(a, g, n) - r1) < 5e-4 * r1
    # non-scattering slab with Fresnel faces (normal incidence)
    n, tau = 1.4, 0.7
    F, e = ((n - 1) / (n + 1)) ** 2, math.exp(-0.7)
    R, T = AD.slab_RT(0.0, 0.0, n, tau)
    assert abs(T - (1 - F) ** 2 * e / (1 - F * F * e * e)) < 1e-6
    assert abs(R - (1 - F) ** 2 * F * e * e / (1 - F * F * e * e)) < 1e-7
    # energy: alpha = 1 slab, R + T + specular = 1, both incidences
    for g in (0.0, 0.8):
        for inc in ("normal", "cosine"):
            R, T = AD.slab_RT(1.0, g, 1.4, 2.0, inc)
            assert abs(R + T + AD.entry_specular(1.4, inc) - 1.0) < 1e-6
    # two layers: identical layers, a vanishing top layer, an absorbing top
    assert abs(AD.two_layer_R((0.9, 0.8, 0.7), (0.9, 0.8), 1.4) -
               AD.R_semi_infinite(0.9, 0.8, 1.4)) < 1e-8
    assert abs(AD.two_layer_R((0.2, 0.5, 1e-9), (0.95, 0.7), 1.4, "cosine") -
               AD.R_semi_infinite(0.95, 0.7, 1.4, "cosine")) < 1e-8
    assert abs(AD.two_layer_R((0.0, 0.0, 0.5), (0.8, 0.0), 1.0) -
               cf.R_absorbing_top(0.8, 0.5)) < 1e-7
