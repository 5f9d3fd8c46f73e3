"""GPU: lookup tables from the batched walk (Sec. 4.2) and the LUT-based fit.

Pins: with n = 1 and g = 0 the table's R(alpha) is the plane albedo
1 - H(1) sqrt(1 - alpha) (closed form); eq. separability (a sigma_t = 2 walk
against the table's sigma_t^2 P_d(sigma_t r) prediction); eq. mixture with a
one-hot weight reproduces the single-medium table row; the LUT fit lowers
eq. joint_loss on targets drawn from the table model itself."""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_common import ctx, np64  # noqa: E402


def test_table_R_matches_plane_albedo_and_separability():
    from paper_2606_27604_amd import api, lut, rw
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
    step = (math.log(geom.r_max_mm) - math.log(geom.r_min_mm)) / nb
    r = torch.exp(math.log(geom.r_min_mm) +
                  (torch.arange(nb, device="cuda", dtype=torch.float32) + 0.5) * step)
    pred = lut.lookup_P(t, t.alpha[6:7], t.g[1:2], torch.full((1,), 2.0, device="cuda"), r)[0]
    got = np64(res.Pd[0])
    pr = np64(pred)
    # compare where both sides expect >= 400 exits in the bin (relative noise
    # <= 5 %): mass per bin = P x annulus area (the sigma_t^2 of the rescaling
    # cancels against the area of the scaled annulus)
    edges = geom.r_min_mm * np.exp(np.arange(nb + 1) * step)
    area = np.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    Rw, Rt = float(res.R[0]), float(t.R[6, 1])
    ok = (got * area * Rw * (1 << 20) >= 400) & (pr * area * Rt * N >= 400)
    rel = np.abs(got[ok] - pr[ok]) / pr[ok]
    assert ok.sum() > 40 and np.median(rel) < 0.05, (ok.sum(), np.median(rel))


def test_mixture_one_hot_and_lut_fit_lowers_loss():
    from paper_2606_27604_amd import fit, lut
    t = lut.generate(ctx(), 33, 33, 1 << 12)
    nb = t.n_bins
    step = (math.log(t.r_max) - math.log(t.r_min)) / nb
    r = torch.exp(math.log(t.r_min) + (torch.arange(nb, device="cuda", dtype=torch.float32) + 0.5) * step)
    # one-hot weights reproduce the table at a grid point (sigma_t = 1)
    K, n = 3, 1
    s = torch.ones((K, n), device="cuda")
    al = torch.stack([t.alpha[20], t.alpha[5], t.alpha[7]])[:, None]
    gg = torch.stack([t.g[10], t.g[3], t.g[4]])[:, None]
    w = torch.tensor([[1.0], [0.0], [0.0]], device="cuda")
    R_hat, Rd = lut.mixture_profile(t, s, al, gg, w, r)
    assert abs(float(R_hat[0]) - float(t.R[20, 10])) < 1e-6
    # the FP32 grid coordinate of a grid point is within ~1e-5 of an integer, so
    # that share of a neighbouring cell of the (noisy) table can leak in
    nbr = float(t.Pd[19:22, 9:12].max())
    np.testing.assert_allclose(np64(Rd[0]) / float(t.R[20, 10]), np64(t.Pd[20, 10]), rtol=1e-4,
                               atol=1e-4 * nbr)
    # targets from the table model, fit from another start: the loss drops
    gen = np.random.default_rng(3)
    n = 64
    tr = [torch.tensor(x, device="cuda") for x in (
        (10 ** gen.uniform(-0.5, 1, (K, n))).astype(np.float32),
        gen.uniform(0.5, 0.98, (K, n)).astype(np.float32),
        gen.uniform(0.0, 0.9, (K, n)).astype(np.float32),
        gen.dirichlet(np.ones(K), n).T.astype(np.float32).copy())]
    R_t, Rd_t = lut.mixture_profile(t, *tr, r)
    Pd_t = (Rd_t / R_t[:, None]).double()
    area = fit.bin_areas(type("G", (), {"n_bins": nb, "r_min_mm": t.r_min, "r_max_mm": t.r_max})(),
                         "cuda")
    mass = Pd_t * area
    start = [torch.tensor(x, device="cuda") for x in (
        (10 ** gen.uniform(-0.5, 1, (K, n))).astype(np.float32),
        gen.uniform(0.5, 0.98, (K, n)).astype(np.float32),
        gen.uniform(0.0, 0.9, (K, n)).astype(np.float32),
        gen.dirichlet(np.ones(K), n).T.astype(np.float32).copy())]
    _, hist = lut.fit(t, R_t.double(), Pd_t, mass, start, r, iters=150, lr=2e-2)
    assert hist[-1][2] < 0.5 * hist[0][2], hist
    # the paper's schedule: K = 1 profile-only start, cosine-annealed Adam
    _, hist = lut.fit(t, R_t.double(), Pd_t, mass, start, r, iters=150, lr=2e-2,
                      schedule="cosine", init_k1_iters=60)
    k1 = [h for h in hist if h[0] == "k1"]
    mix = [h for h in hist if h[0] == "mix"]
    assert k1[-1][2] < k1[0][2] and mix[-1][2] < mix[0][2], hist
