"""CPU pins of the FP64 look-up-table oracle (oracle/lut_oracle.py), the
reference of the fused LUT-fit kernel (Sec. 4.2: eq. separability, eq.
mixture, eq. joint_loss, Adam).

Each pin checks the oracle against something other than its own formulas:
tables whose interpolation is exact, a profile family with a closed-form
rescaling and normalisation, reductions of the mixture to one medium, the
loss at the parameters that generated its targets, central differences of the
loss, the closed-form first Adam step and the round trip of the parameter
maps.  A battery of planted mistakes (each a plausible slip in one line of the
oracle) must each fail at least one pin."""
import math
import types

import numpy as np
import pytest

from oracle import lut_oracle
from tests import lut_tables as T


def _grid(tab):
    return (np.linspace(0.0, tab.alpha_max, tab.n_alpha), np.linspace(0.0, tab.g_max, tab.n_g))


def _centres(tab):
    return np.exp(math.log(tab.r_min) + (np.arange(tab.n_bins) + 0.5) * tab.log_step)


# ---- pins, each taking the oracle module so that mutants can be run -------
def pin_cell_stays_on_grid(LO):
    for n in (2, 9, 256, 800):
        t = np.array([-5.0, 0.0, 0.5, n - 1.5, n - 1 - 1e-9, n - 1.0, n + 3.0])
        i, f, inside = LO.cell(t, n)
        assert i.min() >= 0 and i.max() + 1 <= n - 1, (n, i)
        assert np.all((f >= 0) & (f <= 1)), f
        assert list(inside) == [0, 1, 1, 1, 1, 1, 0]


def pin_grid_points_reproduce_tables(LO):
    tab, _ = T.smooth_table(mod=LO)
    al, gg = _grid(tab)
    ia = np.array([0, 5, 31, tab.n_alpha - 1])
    ig = np.array([0, 7, 20, tab.n_g - 1])
    R, _, _ = LO.lookup_R(tab, al[ia], gg[ig])
    np.testing.assert_allclose(R, tab.R[ia, ig], rtol=1e-12, atol=1e-15)
    rc = _centres(tab)
    P = LO.lookup_P(tab, al[ia], gg[ig], np.ones(4), rc)[0]
    # a centre's coordinate lands on the grid up to rounding (~1e-13 of the
    # neighbouring bin leaks in)
    np.testing.assert_allclose(P, tab.Pd[ia, ig], rtol=1e-9, atol=1e-12 * tab.Pd.max())


def pin_linear_tables_interpolate_exactly(LO):
    c, d = (0.3, 0.5, -0.2, 0.1), (2.0, 0.4, -0.3, 0.05)
    tab = T.linear_table(c=c, d=d, mod=LO)
    rng = np.random.default_rng(1)
    a = rng.uniform(0.0, tab.alpha_max, 50)
    g = rng.uniform(0.0, tab.g_max, 50)
    R, dRa, dRg = LO.lookup_R(tab, a, g)
    np.testing.assert_allclose(R, c[0] + c[1] * a + c[2] * g + c[3] * a * g, rtol=1e-12)
    np.testing.assert_allclose(dRa, c[1] + c[3] * g, rtol=1e-9)
    np.testing.assert_allclose(dRg, c[2] + c[3] * a, rtol=1e-9)
    # sigma_t = e^(k step) moves bin centre b to b + k and scales by sigma_t^2
    rc = _centres(tab)
    for k in (0, 3, -2):
        s = math.exp(k * tab.log_step)
        b = np.arange(max(0, -k), min(tab.n_bins, tab.n_bins - k))
        P, dls, dPa, dPg = LO.lookup_P(tab, a[:5], g[:5], np.full(5, s), rc[b])
        V = d[0] + d[1] * a[:5, None] + d[2] * g[:5, None] + d[3] * (b + k)[None, :]
        np.testing.assert_allclose(P, s * s * V, rtol=1e-9)
        np.testing.assert_allclose(dPa, s * s * d[1] * np.ones_like(V), rtol=1e-9)
        np.testing.assert_allclose(dPg, s * s * d[2] * np.ones_like(V), rtol=1e-9)
        # between the outer centres P is smooth in log sigma_t: 2 P + sigma^2 d3 / step
        inner = (b + k > 0) & (b + k < tab.n_bins - 1)
        np.testing.assert_allclose(dls[:, inner], (2 * s * s * V + s * s * d[3] / tab.log_step)[:, inner],
                                   rtol=1e-9)


def pin_separability_of_a_profile_family(LO):
    """f(rho) = exp(-rho) / (2 pi) per unit area integrates to 1 over the plane;
    a medium of extinction sigma_t has sigma_t^2 f(sigma_t r), which integrates
    to 1 as well.  A table of f at sigma_t = 1 must reproduce both."""
    # linear interpolation in log r errs by about step^2 / 8 (rho^2 - rho)
    # relative: 8e-6 per unit at 2 000 bins, below 1e-3 up to rho = sigma_t r = 8
    nb, r_min, r_max = 2000, 1e-4, 1e3
    tab = LO.Table(np.ones((2, 2)), np.zeros((2, 2, nb)), 0.9, 0.9, r_min, r_max)
    rc = np.exp(math.log(r_min) + (np.arange(nb) + 0.5) * tab.log_step)
    tab.Pd[:] = np.exp(-rc) / (2 * math.pi)
    for s in (0.5, 2.0, 7.0):
        r = np.exp(np.linspace(math.log(1e-2), math.log(8.0 / s), 200))
        P = LO.lookup_P(tab, np.array([0.3]), np.array([0.2]), np.array([s]), r)[0][0]
        ref = s * s * np.exp(-s * r) / (2 * math.pi)
        np.testing.assert_allclose(P, ref, rtol=2e-3)
        # normalisation over a fine log grid covering the profile
        rr = np.exp(np.linspace(math.log(1e-4 / s), math.log(60.0 / s), 4000))
        Pf = LO.lookup_P(tab, np.array([0.3]), np.array([0.2]), np.array([s]), rr)[0][0]
        integral = np.trapezoid(Pf * 2 * math.pi * rr * rr, np.log(rr))
        assert abs(integral - 1.0) < 2e-3, (s, integral)


def pin_radial_range(LO):
    tab = T.linear_table(mod=LO)  # positive over the whole table
    far = np.array([tab.r_min * 0.9, tab.r_min * 1.001, tab.r_max * 0.999, tab.r_max * 1.1])
    P = LO.lookup_P(tab, np.array([0.5]), np.array([0.3]), np.ones(1), far)[0][0]
    assert P[0] == 0.0 and P[3] == 0.0 and P[1] > 0.0 and P[2] > 0.0
    # between the first bin's edge and its centre the value is the centre's
    rc0 = _centres(tab)[0]
    P2 = LO.lookup_P(tab, np.array([0.5]), np.array([0.3]), np.ones(1),
                     np.array([tab.r_min * 1.001, rc0]))[0][0]
    assert P2[0] == P2[1]


def pin_mixture_reduces_to_one_medium(LO):
    tab, r = T.smooth_table(mod=LO)
    rng = np.random.default_rng(2)
    s, a, g, w = T.random_params(rng, 3, 8)
    one = np.zeros_like(w)
    one[1] = 1.0
    Rh, Rd = LO.mixture(tab, s, a, g, one, r)
    R1, _, _ = LO.lookup_R(tab, a[1], g[1])
    P1 = LO.lookup_P(tab, a[1], g[1], s[1], r)[0]
    np.testing.assert_allclose(Rh, R1, rtol=1e-12)
    np.testing.assert_allclose(Rd, R1[:, None] * P1, rtol=1e-12, atol=1e-300)
    # three identical media with any weights are that medium
    same = [np.repeat(x[:1], 3, 0) for x in (s, a, g)]
    Rh3, Rd3 = LO.mixture(tab, *same, w, r)
    R0, _, _ = LO.lookup_R(tab, a[0], g[0])
    P0 = LO.lookup_P(tab, a[0], g[0], s[0], r)[0]
    np.testing.assert_allclose(Rh3, R0, rtol=1e-12)
    np.testing.assert_allclose(Rd3, R0[:, None] * P0, rtol=1e-12, atol=1e-300)


def _targets(LO, tab, r, theta, form):
    """Targets built from the lookups directly: R_hat and the form's P_hat."""
    s, a, g, w = theta
    Rk = np.stack([LO.lookup_R(tab, a[k], g[k])[0] for k in range(len(s))])
    Pk = np.stack([LO.lookup_P(tab, a[k], g[k], s[k], r)[0] for k in range(len(s))])
    R_t = (w * Rk).sum(0)
    if form == LO.SHAPE_PAPER:
        P_t = (w[..., None] * Pk).sum(0)
    else:
        P_t = ((w * Rk)[..., None] * Pk).sum(0) / R_t[:, None]
    return R_t, P_t


def pin_loss_vanishes_at_the_truth(LO):
    tab, r = T.smooth_table(mod=LO)
    rng = np.random.default_rng(3)
    for form in (LO.SHAPE_PAPER, LO.SHAPE_MIXTURE):
        for K in (1, 3):
            theta = T.random_params(rng, K, 6)
            R_t, P_t = _targets(LO, tab, r, theta, form)
            raw = LO.raw_from_physical(*theta)
            loss, grad = LO.loss_and_grad(tab, raw, K, R_t, P_t, T.annulus_mass(P_t, r), r,
                                          shape_form=form)
            assert np.all(loss < 1e-9), (form, K, loss)
            # away from the truth the loss is positive
            loss2, _ = LO.loss_and_grad(tab, raw + 0.3, K, R_t, P_t, T.annulus_mass(P_t, r), r,
                                        shape_form=form)
            assert np.all(loss2 > 1e-3), (form, K, loss2)


def pin_gradient_matches_central_differences(LO):
    tab, r = T.smooth_table(mod=LO)
    rng = np.random.default_rng(4)
    for form in (LO.SHAPE_PAPER, LO.SHAPE_MIXTURE):
        for K, floor, min_mass in ((1, 0.0, 0.0), (2, 0.01, 1e-3), (3, 0.0, 0.0), (4, 0.01, 1e-3)):
            truth = T.random_params(rng, K, 5)
            R_t, P_t = _targets(LO, tab, r, truth, form)
            mass = T.annulus_mass(P_t, r)
            raw = LO.raw_from_physical(*T.random_params(rng, K, 5))
            args = (K, R_t, P_t, mass, r, 5.0, min_mass, floor, form)
            _, grad = LO.loss_and_grad(tab, raw, *args)
            h = 1e-6
            fd = np.zeros_like(raw)
            for i in range(raw.shape[0]):
                e = np.zeros_like(raw)
                e[i] = h
                fd[i] = (LO.loss_and_grad(tab, raw + e, *args)[0]
                         - LO.loss_and_grad(tab, raw - e, *args)[0]) / (2 * h)
            scale = np.abs(fd).max(0, keepdims=True) + 1e-12
            np.testing.assert_allclose(grad, fd, rtol=1e-4, atol=1e-5 * float(scale.max()),
                                       err_msg=f"form {form}, K {K}")


def pin_first_adam_step(LO):
    """With zero moments the bias-corrected first step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p = rng.standard_normal((7, 9))
    g = rng.standard_normal((7, 9))
    p1, m1, v1 = LO.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, 0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # a constant gradient keeps the step at lr (both moments track it exactly)
    q, m, v = p, np.zeros_like(p), np.zeros_like(p)
    for t in range(1, 6):
        q_new, m, v = LO.adam_step(q, g, m, v, t, 0.01)
        np.testing.assert_allclose(q - q_new, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        q = q_new


def pin_parameter_maps_round_trip(LO):
    rng = np.random.default_rng(6)
    for K in (1, 2, 3, 4):
        theta = T.random_params(rng, K, 10)
        s, a, g, w, _ = LO.physical(LO.raw_from_physical(*theta), K)
        for x, y in zip((s, a, g, w), theta):
            np.testing.assert_allclose(x, y, rtol=1e-10)


def pin_fit_lowers_the_loss(LO):
    tab, r = T.smooth_table(mod=LO)
    rng = np.random.default_rng(7)
    K, n = 3, 12
    truth = T.random_params(rng, K, n)
    R_t, P_t = _targets(LO, tab, r, truth, LO.SHAPE_PAPER)
    start = LO.raw_from_physical(*T.random_params(rng, K, n))
    p, hist = LO.fit(tab, R_t, P_t, T.annulus_mass(P_t, r), start, K, r, iters=80, lr=5e-2,
                     schedule="cosine", init_k1_iters=40)
    k1 = [h for h in hist if h[0] == "k1"]
    mix = [h for h in hist if h[0] == "mix"]
    assert k1[-1][2] < 0.5 * k1[0][2], hist
    assert mix[-1][2] < mix[0][2], hist
    s, a, g, w, _ = LO.physical(p, K)
    assert np.allclose(w.sum(0), 1.0)


PINS = [pin_cell_stays_on_grid, pin_grid_points_reproduce_tables,
        pin_linear_tables_interpolate_exactly, pin_separability_of_a_profile_family,
        pin_radial_range, pin_mixture_reduces_to_one_medium, pin_loss_vanishes_at_the_truth,
        pin_gradient_matches_central_differences, pin_first_adam_step,
        pin_parameter_maps_round_trip, pin_fit_lowers_the_loss]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_lut_oracle_pin(pin):
    pin(lut_oracle)


MUTATIONS = [
    ("separability_sigma_not_squared", "s2 = np.where(inb, sigma_t ** 2, 0.0)",
     "s2 = np.where(inb, sigma_t, 0.0)"),
    ("separability_radius_divided", "np.log(sigma_t) + np.log(r)", "np.log(r) - np.log(sigma_t)"),
    ("bin_edges_not_centres", "/ tab.log_step - 0.5", "/ tab.log_step"),
    ("bilinear_weights_swapped", "val = (1 - fa) * lo + fa * hi", "val = (1 - fg) * lo + fg * hi"),
    ("cell_cap_off_by_one", "np.minimum(np.floor(tc), n - 2)", "np.minimum(np.floor(tc), n - 1)"),
    ("dR_dg_wrong_corners", "d_g = ((1 - fa) * (r01 - r00) + fa * (r11 - r10)) * sg * ing",
     "d_g = ((1 - fa) * (r10 - r00) + fa * (r11 - r01)) * sg * ing"),
    ("dlogsigma_factor_dropped", "2.0 * V + dV_dtb", "V + dV_dtb"),
    ("paper_form_weighted_by_R", "P_hat = (w[..., None] * Pk).sum(0)",
     "P_hat = ((w * Rk)[..., None] * Pk).sum(0)"),
    ("shape_not_a_root", "shape = np.sqrt((d * d).sum(1) / n_used + 1e-30)",
     "shape = (d * d).sum(1) / n_used + 1e-30"),
    ("mixture_normalisation_not_differentiated",
     "gRh = gR - np.where(R_hat > 1e-12, (q * N).sum(1) / Rc ** 2, 0.0)", "gRh = gR"),
    ("g_chain_without_scale", "grad[2 * K:3 * K] = d_g * 0.99 * sgm * (1 - sgm)",
     "grad[2 * K:3 * K] = d_g * sgm * (1 - sgm)"),
    ("alpha_chain_incomplete", "grad[K:2 * K] = d_alpha * alpha * (1 - alpha)",
     "grad[K:2 * K] = d_alpha * alpha"),
    ("softmax_gradient_no_baseline", "grad[3 * K:] = (w * (gw - wg[None]))[:K - 1]",
     "grad[3 * K:] = (w * gw)[:K - 1]"),
    ("adam_no_bias_correction", "mh = m / (1 - b1 ** step)", "mh = m"),
    ("raw_logits_not_relative", "lw[:K - 1] - lw[K - 1:]], 0)", "lw[:K - 1]], 0)"),
    ("floor_outside_target_log", "d = (np.log(P_hat + f) - np.log(Pd_t + f)) * use",
     "d = (np.log(P_hat + f) - np.log(Pd_t)) * use"),
]


def _mutant(old, new):
    import inspect
    src = inspect.getsource(lut_oracle)
    assert src.count(old) == 1, old
    import sys
    name = "lut_oracle_mutant"
    mod = types.ModuleType(name)
    sys.modules[name] = mod  # the dataclass decorator looks its module up
    try:
        exec(compile(src.replace(old, new), name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def _caught(mod):
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except Exception:
            return True
    return False


def test_planted_mistakes_fail_a_pin():
    survivors = [name for name, old, new in MUTATIONS if not _caught(_mutant(old, new))]
    assert not survivors, f"planted mistakes not caught: {survivors}"
