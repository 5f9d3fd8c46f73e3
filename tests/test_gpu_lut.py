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
from paper_2606_27604_amd import rw  # noqa: E402
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


def _smooth_problem(K=3, n=64, seed=4):
    """A smooth synthetic table on the GPU, targets from its own model at
    random parameters, and a random raw start (tests.test_lut_cpu's table)."""
    from paper_2606_27604_amd import lut as L
    from tests.test_lut_cpu import _smooth_table
    t, r = _smooth_table()
    t = L.LUT(t.alpha.cuda(), t.g.cuda(), t.R.cuda(), t.Pd.cuda(), t.r_min, t.r_max, t.n_rel,
              t.paths)
    r = r.cuda()
    gen = torch.Generator(device="cuda").manual_seed(seed)
    truth = (10 ** (torch.rand((K, n), generator=gen, device="cuda") - 0.5),
             0.5 + 0.45 * torch.rand((K, n), generator=gen, device="cuda"),
             0.8 * torch.rand((K, n), generator=gen, device="cuda"),
             torch.softmax(torch.randn((K, n), generator=gen, device="cuda"), 0))
    R_t, Rd_t = L.mixture_profile(t, *truth, r)
    Pd_t = (Rd_t / R_t[:, None]).double()
    lr_ = torch.log(r.double())
    h = float(lr_[1] - lr_[0])
    edges = torch.exp(torch.cat([lr_ - 0.5 * h, lr_[-1:] + 0.5 * h]))
    mass = Pd_t * math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    start = (10 ** (torch.rand((K, n), generator=gen, device="cuda") - 0.5),
             0.5 + 0.45 * torch.rand((K, n), generator=gen, device="cuda"),
             0.8 * torch.rand((K, n), generator=gen, device="cuda"),
             torch.softmax(torch.randn((K, n), generator=gen, device="cuda"), 0))
    return t, r, R_t.double(), Pd_t, mass, start


@pytest.mark.parametrize("K", [1, 3])
def test_lut_kernel_loss_and_gradient_match_autograd(K):
    from paper_2606_27604_amd import lut as L
    from tests.lut_reference import loss_reference
    t, r, R_t, Pd_t, mass, start = _smooth_problem(K=K)
    n = R_t.numel()
    params = L.raw_from_physical(*start)
    tabs = L._native_tables(t)
    tg = L._native_targets(R_t, Pd_t, mass, r, 5.0)
    grad = torch.zeros_like(params)
    loss = torch.zeros(n, dtype=torch.float32, device="cuda")
    rw.rw_lut_loss_grad(ctx(), tabs[0], tg[0], n, K, params, grad, loss)
    torch.cuda.synchronize()
    p64 = params.double().clone().requires_grad_(True)
    ref = loss_reference(t, p64, K, R_t, Pd_t, mass, r)
    ref.sum().backward()
    np.testing.assert_allclose(np64(loss), np64(ref.detach()), rtol=2e-4, atol=1e-6)
    G, Gr = np64(grad), np64(p64.grad)
    scale = np.abs(Gr).max(axis=0, keepdims=True)
    np.testing.assert_allclose(G, Gr, rtol=3e-3, atol=1e-3 * float(scale.max()))


def test_lut_kernel_adam_steps_match_torch_adam():
    from paper_2606_27604_amd import lut as L
    from tests.lut_reference import loss_reference
    K = 3
    t, r, R_t, Pd_t, mass, start = _smooth_problem(K=K, n=32, seed=5)
    n = R_t.numel()
    params = L.raw_from_physical(*start)
    ref = params.double().clone().requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=1e-2)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    tabs = L._native_tables(t)
    tg = L._native_targets(R_t, Pd_t, mass, r, 5.0)
    for step in (1, 2, 3):
        rw.rw_lut_fit_step(ctx(), tabs[0], tg[0], n, K, params, m, v, step, 1e-2)
        opt.zero_grad()
        loss_reference(t, ref, K, R_t, Pd_t, mass, r).sum().backward()
        opt.step()
        torch.cuda.synchronize()
        # each Adam step moves a parameter by at most ~lr; the two agree to a
        # small fraction of that (tiny gradients, whose step is eps-limited,
        # may differ)
        d = np.abs(np64(params) - np64(ref.detach()))
        assert np.quantile(d, 0.98) <= 1e-3 * step, np.quantile(d, 0.98)


def test_native_fit_follows_the_reference_fit():
    from paper_2606_27604_amd import lut as L
    from tests.lut_reference import fit_reference
    t, r, R_t, Pd_t, mass, start = _smooth_problem(K=3, n=48, seed=6)
    (s1, a1, g1, w1), h1 = L.fit(t, R_t, Pd_t, mass, start, r, iters=60, lr=2e-2,
                                 schedule="cosine", init_k1_iters=30, ctx=ctx())
    (s2, a2, g2, w2), h2 = fit_reference(t, R_t, Pd_t, mass, start, r, iters=60, lr=2e-2,
                                         schedule="cosine", init_k1_iters=30)
    l1 = np.array([h[2] for h in h1])
    l2 = np.array([h[2] for h in h2])
    assert [h[:2] for h in h1] == [h[:2] for h in h2]
    np.testing.assert_allclose(l1, l2, rtol=5e-2)
    assert l1[-1] < l1[[i for i, h in enumerate(h1) if h[0] == "mix"][0]]
