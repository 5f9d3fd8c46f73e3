"""The FP64 oracle's random walk against closed forms, invariants, brute force
and finite differences (CPU only).  The checks live in tests/oracle_pins.py."""
import json
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
