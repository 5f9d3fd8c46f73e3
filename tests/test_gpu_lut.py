"""GPU: lookup tables from the batched walk (Sec. 4.2) and the fused LUT-fit
kernel, checked against the FP64 LUT oracle (oracle/lut_oracle.py).

Tables: with n = 1 and g = 0 the table's R(alpha) is the plane albedo
1 - H(1) sqrt(1 - alpha) (closed form); eq. separability (a sigma_t = 2 walk
against the oracle's sigma_t^2 P_d(sigma_t r) prediction from the table).
Kernel: loss and gradient of eq. joint_loss (both definitions of P_hat, with
and without the mass threshold and floor), three Adam steps, and a whole fit
with the paper's schedule, each against the oracle on the same FP32 inputs;
the fit lowers the loss on a table made by the walk."""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import lut_oracle as LO

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2606_27604_amd import rw  # noqa: E402
from tests import lut_tables as T  # noqa: E402
from tests.gpu_common import ctx, np64  # noqa: E402

FORMS = {"paper": LO.SHAPE_PAPER, "mixture": LO.SHAPE_MIXTURE}


def _oracle_table(t):
    """The oracle's view of a product table (the same FP32 values, in FP64)."""
    return LO.Table(np64(t.R), np64(t.Pd), float(t.alpha[-1]), float(t.g[-1]), t.r_min, t.r_max)


def _product_table(tab):
    from paper_2606_27604_amd import lut as L
    f32 = lambda x: torch.tensor(np.asarray(x, np.float32), device="cuda")  # noqa: E731
    return L.LUT(f32(np.linspace(0.0, tab.alpha_max, tab.n_alpha)),
                 f32(np.linspace(0.0, tab.g_max, tab.n_g)), f32(tab.R), f32(tab.Pd), tab.r_min,
                 tab.r_max, 1.4, 1)


def _r_centres(n_bins, r_min, r_max):
    step = (math.log(r_max) - math.log(r_min)) / n_bins
    return np.exp(math.log(r_min) + (np.arange(n_bins) + 0.5) * step)


def test_table_R_matches_plane_albedo_and_separability():
    from paper_2606_27604_amd import api, lut
    N = 1 << 20
    t = lut.generate(ctx(), 9, 2, N, n_rel=1.0, alpha_max=0.99, g_max=0.5)
    al = np64(t.alpha)
    R0 = np64(t.R)[:, 0]  # g = 0 column
    ref = np.array([cf.R_plane(float(a)) if a > 0 else 0.0 for a in al])
    se = np.sqrt(np.maximum(ref * (1 - ref), 1e-12) / N)  # upper bound of the per-path SD
    assert np.all(np.abs(R0 - ref) <= 4 * se + 1e-12), (R0 - ref) / se
    # eq. separability: a walk at sigma_t = 2 against sigma_t^2 P_d(sigma_t r) of the table
    a, g = float(t.alpha[6]), float(t.g[1])
    m = rw.Media(torch.full((1, 1), 2.0, device="cuda"), torch.full((1, 1), a, device="cuda"),
                 torch.full((1, 1), g, device="cuda"), torch.ones((1, 1), device="cuda"), 1, 1)
    geom = rw.Geometry(n_media=1, n_rel=1.0)
    res = api.forward(ctx(), m, geom, 1 << 20, 3)
    # the walk's own bins (256 over [1e-3, 50] mm), predicted from the wider table
    nb = geom.n_bins
    r = _r_centres(nb, geom.r_min_mm, geom.r_max_mm)
    pr = LO.lookup_P(_oracle_table(t), np.array([a]), np.array([g]), np.array([2.0]), r)[0][0]
    got = np64(res.Pd[0])
    # compare where both sides expect >= 400 exits in the bin (relative noise
    # <= 5 %): mass per bin = P x annulus area (the sigma_t^2 of the rescaling
    # cancels against the area of the scaled annulus)
    step = (math.log(geom.r_max_mm) - math.log(geom.r_min_mm)) / nb
    edges = geom.r_min_mm * np.exp(np.arange(nb + 1) * step)
    area = np.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    Rw, Rt = float(res.R[0]), float(t.R[6, 1])
    ok = (got * area * Rw * (1 << 20) >= 400) & (pr * area * Rt * N >= 400)
    rel = np.abs(got[ok] - pr[ok]) / pr[ok]
    assert ok.sum() > 40 and np.median(rel) < 0.05, (ok.sum(), np.median(rel))


def _problem(K, n, seed, form):
    """The smooth synthetic table, targets from the oracle's model at random
    parameters, a random start; FP32 copies for the kernel and the same values
    in FP64 for the oracle."""
    tab, r = T.smooth_table()
    # the kernel reads the grid bounds in FP32
    tab.alpha_max, tab.g_max = float(np.float32(tab.alpha_max)), float(np.float32(tab.g_max))
    r = np.asarray(r, np.float32).astype(np.float64)
    rng = np.random.default_rng(seed)
    s, a, g, w = T.random_params(rng, K, n)
    Rk = np.stack([LO.lookup_R(tab, a[k], g[k])[0] for k in range(K)])
    Pk = np.stack([LO.lookup_P(tab, a[k], g[k], s[k], r)[0] for k in range(K)])
    R_t = (w * Rk).sum(0)
    if form == LO.SHAPE_PAPER:
        P_t = (w[..., None] * Pk).sum(0)
    else:
        P_t = ((w * Rk)[..., None] * Pk).sum(0) / R_t[:, None]
    mass = T.annulus_mass(P_t, r)
    f32 = lambda x: np.asarray(x, np.float32).astype(np.float64)  # noqa: E731
    R_t, P_t, mass = f32(R_t), f32(P_t), f32(mass)
    start = LO.raw_from_physical(*T.random_params(rng, K, n)).astype(np.float32)
    return tab, r, R_t, P_t, mass, start


def _native(tab, r, R_t, P_t, mass, lambda_R, form, min_mass, floor):
    from paper_2606_27604_amd import lut as L
    cuda = lambda x: torch.tensor(np.asarray(x, np.float32), device="cuda")  # noqa: E731
    pt = _product_table(tab)
    tabs = L._native_tables(pt)
    tg = L._native_targets(cuda(R_t), cuda(P_t), cuda(mass), cuda(r), lambda_R, form, min_mass,
                           floor)
    return pt, tabs, tg


@pytest.mark.parametrize("form", ["paper", "mixture"])
@pytest.mark.parametrize("K,min_mass,floor", [(1, 0.0, 0.0), (3, 0.0, 0.0), (3, 1e-3, 1e-2),
                                              (4, 1e-3, 1e-2)])
def test_lut_kernel_loss_and_gradient_match_oracle(form, K, min_mass, floor):
    tab, r, R_t, P_t, mass, start = _problem(K, 64, 10 + K, FORMS[form])
    n = R_t.size
    _, tabs, tg = _native(tab, r, R_t, P_t, mass, 5.0, form, min_mass, floor)
    params = torch.tensor(start, device="cuda")
    grad = torch.zeros_like(params)
    loss = torch.zeros(n, dtype=torch.float32, device="cuda")
    rw.rw_lut_loss_grad(ctx(), tabs[0], tg[0], n, K, params, grad, loss)
    torch.cuda.synchronize()
    mm = float(np.float32(min_mass))
    ref_loss, ref_grad = LO.loss_and_grad(tab, start.astype(np.float64), K, R_t, P_t, mass, r,
                                          5.0, mm, float(np.float32(floor)), FORMS[form])
    np.testing.assert_allclose(np64(loss), ref_loss, rtol=2e-4, atol=1e-6)
    G = np64(grad)
    scale = np.abs(ref_grad).max()
    np.testing.assert_allclose(G, ref_grad, rtol=3e-3, atol=1e-3 * scale)


@pytest.mark.parametrize("form", ["paper", "mixture"])
def test_lut_kernel_adam_steps_match_oracle(form):
    K = 3
    tab, r, R_t, P_t, mass, start = _problem(K, 32, 5, FORMS[form])
    n = R_t.size
    _, tabs, tg = _native(tab, r, R_t, P_t, mass, 5.0, form, 0.0, 0.0)
    params = torch.tensor(start, device="cuda")
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    p = start.astype(np.float64)
    pm, pv = np.zeros_like(p), np.zeros_like(p)
    for step in (1, 2, 3):
        rw.rw_lut_fit_step(ctx(), tabs[0], tg[0], n, K, params, m, v, step, 1e-2)
        _, gr = LO.loss_and_grad(tab, p, K, R_t, P_t, mass, r, 5.0, 0.0, 0.0, FORMS[form])
        p, pm, pv = LO.adam_step(p, gr, pm, pv, step, 1e-2)
        torch.cuda.synchronize()
        # each Adam step moves a parameter by at most ~lr; the two agree to a
        # small fraction of that (tiny gradients, whose step is eps-limited,
        # may differ)
        d = np.abs(np64(params) - p)
        assert np.quantile(d, 0.98) <= 1e-3 * step, np.quantile(d, 0.98)


def test_native_fit_follows_the_oracle_fit():
    """lut.fit (one fused kernel per Adam step) against the oracle's fit with the
    paper's schedule: the K = 1 profile-only start, then all components, cosine
    learning rate."""
    from paper_2606_27604_amd import lut as L
    K, n = 3, 48
    tab, r, R_t, P_t, mass, start = _problem(K, n, 6, LO.SHAPE_PAPER)
    cuda = lambda x: torch.tensor(np.asarray(x, np.float32), device="cuda")  # noqa: E731
    pt = _product_table(tab)
    st = tuple(torch.tensor(x, device="cuda") for x in LO.physical(start.astype(np.float64), K)[:4])
    from paper_2606_27604_amd.fit import MIN_BIN_MASS, SHAPE_FLOOR
    _, h1 = L.fit(pt, cuda(R_t), cuda(P_t), cuda(mass), st, cuda(r), iters=60, lr=2e-2,
                  schedule="cosine", init_k1_iters=30, ctx=ctx())
    _, h2 = LO.fit(tab, R_t, P_t, mass, start, K, r, iters=60, lr=2e-2, schedule="cosine",
                   init_k1_iters=30, min_mass=float(np.float32(MIN_BIN_MASS)),
                   shape_floor=float(np.float32(SHAPE_FLOOR)))
    assert [h[:2] for h in h1] == [h[:2] for h in h2]
    l1 = np.array([h[2] for h in h1])
    l2 = np.array([h[2] for h in h2])
    np.testing.assert_allclose(l1, l2, rtol=5e-2)
    assert l1[-1] < l1[[i for i, h in enumerate(h1) if h[0] == "mix"][0]]


@pytest.mark.parametrize("form", ["paper", "mixture"])
def test_lut_fit_lowers_the_loss_on_a_walk_table(form):
    """A 33 x 33 table from the batched walk; targets from the oracle's model on
    that table; the native fit from another start lowers the loss."""
    from paper_2606_27604_amd import lut as L
    t = L.generate(ctx(), 33, 33, 1 << 12)
    tab = _oracle_table(t)
    r = _r_centres(256, 1e-3, 50.0).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(3)
    K, n = 3, 64
    s, a, g, w = (10 ** rng.uniform(-0.5, 1, (K, n)), rng.uniform(0.5, 0.98, (K, n)),
                  rng.uniform(0.0, 0.9, (K, n)), rng.dirichlet(np.ones(K), n).T.copy())
    Rk = np.stack([LO.lookup_R(tab, a[k], g[k])[0] for k in range(K)])
    Pk = np.stack([LO.lookup_P(tab, a[k], g[k], s[k], r)[0] for k in range(K)])
    R_t = (w * Rk).sum(0)
    P_t = ((w[..., None] if form == "paper" else (w * Rk)[..., None]) * Pk).sum(0)
    if form == "mixture":
        P_t = P_t / R_t[:, None]
    step = (math.log(50.0) - math.log(1e-3)) / 256
    edges = 1e-3 * np.exp(np.arange(257) * step)
    mass = P_t * np.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    cuda = lambda x: torch.tensor(np.asarray(x, np.float32), device="cuda")  # noqa: E731
    st = tuple(cuda(x) for x in (10 ** rng.uniform(-0.5, 1, (K, n)), rng.uniform(0.5, 0.98, (K, n)),
                                 rng.uniform(0.0, 0.9, (K, n)), rng.dirichlet(np.ones(K), n).T.copy()))
    _, hist = L.fit(t, cuda(R_t), cuda(P_t), cuda(mass), st, cuda(r), iters=150, lr=2e-2,
                    shape_form=form, ctx=ctx())
    assert hist[-1][2] < 0.5 * hist[0][2], hist
    _, hist = L.fit(t, cuda(R_t), cuda(P_t), cuda(mass), st, cuda(r), iters=150, lr=2e-2,
                    schedule="cosine", init_k1_iters=60, shape_form=form, ctx=ctx())
    k1 = [h for h in hist if h[0] == "k1"]
    mix = [h for h in hist if h[0] == "mix"]
    assert k1[-1][2] < k1[0][2] and mix[-1][2] < mix[0][2], hist
