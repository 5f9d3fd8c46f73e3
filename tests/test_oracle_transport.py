"""The FP64 oracle's random walk against closed forms, invariants, brute force
and finite differences (CPU only).  The checks live in tests/oracle_pins.py."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests import oracle_pins as P
from tests._stats import mean_se

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _assert(res):
    ok, detail = res
    assert ok, detail


def test_plane_albedo_16_albedos_config():
    # the 16-albedo homogeneous workload at 2^16 paths: every albedo within 3 SE
    with open(os.path.join(GOLDEN, "plane_albedo_16.json")) as f:
        gold = json.load(f)
    a = np.array(gold["alpha"])
    geo = O.Geometry(n_media=1, n_rel=1.0)
    tal, bins, vert = O.forward(geo, np.ones(16), a, np.zeros(16), np.ones(16), 1 << 16, 0)
    m, se = mean_se(tal[:, 0], tal[:, 1], 1 << 16)
    z = (m - np.array(gold["R"])) / se
    assert np.all(np.abs(z) <= 3.0), z
    # every tallied path lands in exactly one slot
    assert np.allclose(bins[:, :, 0].sum(1), tal[:, 0], rtol=1e-12)


def test_plane_albedo_bias_run_resolves_half_percent():
    # 2^22 paths resolve 0.5 % at 3 SE for the end points of the albedo range
    _assert(P.check_plane_albedo(alphas=(0.5, 0.99), paths=1 << 22, seed=21, rel=0.005))


def test_plane_albedo_mid_range():
    _assert(P.check_plane_albedo())


def test_second_moment():
    _assert(P.check_second_moment())


@pytest.mark.parametrize("g,n,sigma_t", [(0.0, 1.0, 1.0), (0.5, 1.4, 2.0), (0.9, 1.4, 0.3),
                                         (0.7, 1.0, 7.0)])
def test_single_scatter_total_and_annuli(g, n, sigma_t):
    _assert(P.check_single_scatter(g=g, n=n, sigma_t=sigma_t))


def test_energy_exact_without_roulette():
    _assert(P.check_energy_exact())


def test_analog_and_weighted_estimators_agree():
    _assert(P.check_analog_vs_weighted())


def test_spherical_albedo_under_cosine_incidence():
    _assert(P.check_spherical_albedo())


def test_analog_and_weighted_agree_under_cosine_incidence():
    _assert(P.check_analog_vs_weighted_cosine())


def test_beer_lambert():
    _assert(P.check_beer_lambert())


def test_mixture_linearity():
    _assert(P.check_mixture_linearity())


def test_one_hot_weights_reproduce_single_medium():
    _assert(P.check_single_medium_special_case())


def test_scale_invariance_common_random_numbers():
    _assert(P.check_scale_invariance())


def test_trace_invariants():
    _assert(P.check_trace_invariants())


def test_brute_force_grid_single_scatter():
    _assert(P.check_brute_force_single_scatter(m=64))


def test_adjoint_plane_closed_forms():
    _assert(P.check_adjoint_plane())


def test_adjoint_mixture_closed_forms():
    _assert(P.check_adjoint_mixture())


def test_adjoint_against_crn_finite_differences():
    _assert(P.check_adjoint_vs_crn_fd())


def test_adjoint_jacobian_output():
    _assert(P.check_jacobian())


def test_results_do_not_depend_on_thread_count():
    geo = O.Geometry(n_media=3, n_rel=1.4)
    args = ([[1.0], [5.0], [0.2]], [[0.9], [0.5], [0.99]], [[0.7], [0.1], [0.2]],
            [[0.3], [0.3], [0.4]], 40000, 5)
    a = O.forward(geo, *args, n_threads=1)
    b = O.forward(geo, *args, n_threads=7)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_invalid_parameters_are_rejected():
    geo = O.Geometry(n_media=1)
    for bad in (dict(s=0.0), dict(a=1.5), dict(g=1.0), dict(s=float("nan"))):
        s, a, g = bad.get("s", 1.0), bad.get("a", 0.5), bad.get("g", 0.0)
        with pytest.raises(ValueError):
            O.forward(geo, [s], [a], [g], [1.0], 16, 0)
    with pytest.raises(ValueError):
        O.forward(O.Geometry(n_media=2), [1.0, 1.0], [0.5, 0.5], [0, 0], [0.5, 0.6], 16, 0)


def test_vertex_cap_scores_zero_and_counts():
    geo = O.Geometry(n_media=1, n_rel=1.0, max_vertices=3, rr_weight=0.0)
    tal, _, vert = O.forward(geo, [1.0], [1.0], [0.0], [1.0], 4096, 1)
    assert tal[0, 5] > 0                      # some paths were capped
    assert vert[0] <= 3 * 4096
    _, out, _ = O.trace(geo, [1.0], [1.0], [0.0], [1.0], n_paths=256, n_blocks=8, seed=1)
    capped = out[:, 0] == O.END_CAPPED
    assert capped.any() and np.all(out[capped, 3] == 0.0) and np.all(out[capped, 5] == 3)


# ---- two-layer tissue (Sec. 3 geometry) --------------------------------------
def test_two_layer_beer_lambert():
    ok, detail = P.check_two_layer_beer_lambert()
    assert ok, detail


def test_layers_reduce_to_plane_albedo():
    ok, detail = P.check_layers_reduce_to_plane()
    assert ok, detail


def test_absorbing_top_layer_exit_law():
    ok, detail = P.check_absorbing_top_layer()
    assert ok, detail


def test_layered_adjoint_absorbing_top_closed_form():
    ok, detail = P.check_layered_adjoint_absorbing_top()
    assert ok, detail


def test_layered_adjoint_against_crn_finite_differences():
    ok, detail = P.check_layered_adjoint_vs_crn_fd()
    assert ok, detail


def test_transparent_stack_fresnel_adding():
    ok, detail = P.check_transparent_stack(paths=1 << 19)
    assert ok, detail


def test_layers_analog_vs_weighted_and_energy():
    ok, detail = P.check_layers_analog_vs_weighted()
    assert ok, detail


def test_layer_trace_invariants():
    ok, detail = P.check_layer_trace_invariants()
    assert ok, detail


def test_layers_identical_to_homogeneous_with_fresnel():
    """Identical layers with a Fresnel surface (n = 1.4, g != 0) give the
    homogeneous walk's R (the interface stops flights but does not change the
    path density)."""
    n = 1 << 18
    geo1 = O.Geometry(n_media=1, n_rel=1.4)
    t1, _, _ = O.forward(geo1, [2.0], [0.95], [0.8], [1.0], n, 30)
    geo2 = O.Geometry(n_media=2, n_rel=1.4)
    t2, _, _ = O.layered_forward(geo2, [[2.0], [2.0]], [[0.95], [0.95]], [[0.8], [0.8]], [0.1],
                                 1.4, n, 31)
    m1, s1 = mean_se(t1[0, 0], t1[0, 1], n)
    m2, s2 = mean_se(t2[0, 0], t2[0, 1], n)
    assert abs(m1 - m2) <= 3.0 * math.hypot(s1, s2), (m1, m2)


def test_layered_invalid_parameters_are_rejected():
    geo = O.Geometry(n_media=2, n_rel=1.4)
    good = dict(s=[[1.0], [1.0]], a=[[0.5], [0.5]], g=[[0.0], [0.0]], d=[0.1], nb=1.4)
    for key, val in (("d", [0.0]), ("d", [float("nan")]), ("s", [[0.0], [1.0]]),
                     ("a", [[0.5], [1.2]]), ("g", [[0.0], [-1.0]]), ("nb", 0.0)):
        kw = dict(good)
        kw[key] = val
        with pytest.raises(ValueError):
            O.layered_forward(geo, kw["s"], kw["a"], kw["g"], kw["d"], kw["nb"], 16, 0)
    with pytest.raises(ValueError):  # the top layer must end above a slab's bottom
        O.layered_forward(O.Geometry(n_media=2, slab_mm=0.1), good["s"], good["a"], good["g"],
                          [0.2], 1.4, 16, 0)
    with pytest.raises(ValueError):  # two layers means n_media = 2
        O.layered_forward(O.Geometry(n_media=3), good["s"], good["a"], good["g"], [0.1], 1.4,
                          16, 0)


def test_multiple_scattering_against_adding_doubling():
    # six comparisons at once: 3.5 SE each keeps the family-wise false alarm
    # rate near 0.3 % (a run at 2^23 paths of the g = 0.8, n = 1.4 case sits at
    # 0.5 SE of the adding-doubling value)
    ok, detail = P.check_adding_doubling(paths=1 << 20, k=3.5)
    assert ok, detail


def test_hero_wavelength_groups_reduce_to_the_plain_walk():
    _assert(P.check_hero_reduces_to_the_plain_walk())


def test_hero_wavelength_members_match_closed_forms():
    _assert(P.check_hero_against_closed_forms())


def test_dwivedi_nu0_against_a_root_finder_and_its_limit():
    _assert(P.check_dwivedi_nu0())


def test_dwivedi_exit_weights_telescope_in_isotropic_media():
    _assert(P.check_dwivedi_weights_telescope())


def test_dwivedi_walk_matches_closed_forms():
    _assert(P.check_dwivedi_closed_forms())


def test_dwivedi_walk_agrees_with_the_plain_walk():
    _assert(P.check_dwivedi_vs_plain())
