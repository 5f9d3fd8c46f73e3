"""CPU checks of the LUT interpolation (torch on CPU tensors: an index out of
range raises here instead of touching memory): grid points reproduce the
table, the interpolation is linear between them, the edges of the (alpha, g)
grid and of the radial range are handled, and sigma_t rescales the radial
axis as eq. separability states."""
import math

import pytest

torch = pytest.importorskip("torch")

from paper_2606_27604_amd import lut as L  # noqa: E402


def _table(na=800, ng=7, nb=256):
    alpha = torch.linspace(0.0, 0.999, na)
    g = torch.linspace(0.0, 0.99, ng)
    R = alpha[:, None] * 0.5 + g[None, :] * 0.25
    b = torch.arange(nb, dtype=torch.float32)
    Pd = (1.0 + alpha[:, None, None]) * (1.0 + g[None, :, None]) * torch.exp(-0.01 * b)[None, None, :]
    return L.LUT(alpha, g, R, Pd.contiguous(), 1e-3, 50.0, 1.4, 1)


def test_cell_never_leaves_the_grid():
    for n in (2, 9, 256, 800, 1001):
        t = torch.tensor([-5.0, 0.0, 0.5, n - 1.5, n - 1 - 1e-6, n - 1.0, n + 3.0, float("nan")])
        i, w = L._cell(t, n)
        assert int(i.min()) >= 0 and int(i.max()) + 1 <= n - 1, (n, i)
        ok = ~torch.isnan(t)
        assert bool(((w[ok] >= 0) & (w[ok] <= 1.0 + 1e-6)).all())


def test_bilinear_R_grid_points_linear_and_edges():
    t = _table()
    a, g = t.alpha[[0, 10, 799]], t.g[[0, 3, 6]]
    assert torch.allclose(L.lookup_R(t, a, g), t.R[[0, 10, 799], [0, 3, 6]], atol=1e-6)
    # the table is linear in both axes, so bilinear interpolation is exact
    aa = torch.tensor([0.1234, 0.999, 1.5, -0.2])
    gg = torch.tensor([0.5, 0.99, 2.0, -1.0])
    ref = aa.clamp(0, 0.999) * 0.5 + gg.clamp(0, 0.99) * 0.25
    assert torch.allclose(L.lookup_R(t, aa, gg), ref, atol=1e-5)


def test_trilinear_P_radial_scaling_and_range():
    t = _table()
    nb = t.n_bins
    step = (math.log(t.r_max) - math.log(t.r_min)) / nb
    centres = torch.exp(math.log(t.r_min) + (torch.arange(nb, dtype=torch.float32) + 0.5) * step)
    a = t.alpha[[5]]
    g = t.g[[2]]
    # sigma_t = 1 at bin centres returns the table
    p1 = L.lookup_P(t, a, g, torch.ones(1), centres)[0]
    assert torch.allclose(p1, t.Pd[5, 2], rtol=1e-4)
    # eq. separability: sigma_t = e^(k step) shifts the bins by k and scales by sigma_t^2
    k = 7
    s = math.exp(k * step)
    p2 = L.lookup_P(t, a, g, torch.full((1,), s), centres)[0]
    assert torch.allclose(p2[: nb - k], s * s * t.Pd[5, 2, k:], rtol=1e-3)
    # radii beyond the table's range give 0, radii at its edges stay in range
    far = torch.tensor([1e-6, t.r_min, t.r_max * 0.999, 1e3])
    pf = L.lookup_P(t, a, g, torch.ones(1), far)[0]
    assert float(pf[0]) == 0.0 and float(pf[3]) == 0.0 and float(pf[1]) > 0 and float(pf[2]) > 0


def _smooth_table(na=64, ng=32, nb=160):
    """A table with the qualitative behaviour of the real one: R rises with
    alpha and falls with g, the profile widens with alpha and g and its tail
    stretches with g.  The table spans [1e-4, 1e3] mm, evaluation radii
    [1e-2, 20] mm, so sigma_t in [0.1, 50] stays on the table."""
    alpha = torch.linspace(0.0, 0.999, na, dtype=torch.float64)
    g = torch.linspace(0.0, 0.99, ng, dtype=torch.float64)
    R = alpha[:, None] ** 2 * (1.0 - 0.5 * g[None, :])
    r_min, r_max = 1e-4, 1e3
    step = (math.log(r_max) - math.log(r_min)) / nb
    rc = torch.exp(math.log(r_min) + (torch.arange(nb, dtype=torch.float64) + 0.5) * step)
    width = (0.3 + 2.0 * alpha[:, None, None])
    p = 1.0 - 0.5 * g[None, :, None]
    Pd = torch.exp(-(rc[None, None, :] / width) ** p) / (2 * math.pi * width ** 2)
    r = torch.exp(torch.linspace(math.log(1e-2), math.log(20.0), 48, dtype=torch.float64))
    return L.LUT(alpha.float(), g.float(), R.float(), Pd.float().contiguous(), r_min, r_max, 1.4,
                 1), r.float()


def test_fit_k1_start_and_cosine_schedule_lower_the_loss():
    """The fit's schedule and K = 1 start, on the autograd reference that the
    GPU kernel is checked against."""
    from tests.lut_reference import fit_reference

    t, r = _smooth_table()
    gen = torch.Generator().manual_seed(4)
    K, n = 3, 16
    truth = (10 ** (torch.rand((K, n), generator=gen) - 0.5), 0.5 + 0.45 * torch.rand((K, n), generator=gen),
             0.8 * torch.rand((K, n), generator=gen), torch.full((K, n), 1.0 / K))
    R_t, Rd_t = L.mixture_profile(t, *truth, r)
    Pd_t = (Rd_t / R_t[:, None]).double()
    # annulus areas of the evaluation radii (log-spaced, as the data's bins)
    lr = torch.log(r.double())
    h = float(lr[1] - lr[0])
    edges = torch.exp(torch.cat([lr - 0.5 * h, lr[-1:] + 0.5 * h]))
    mass = Pd_t * math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    start = tuple(x.clone() for x in truth)
    (s, a, g, w), hist = fit_reference(t, R_t.double(), Pd_t, mass, start, r, iters=80, lr=5e-2,
                                       schedule="cosine", init_k1_iters=40)
    k1 = [h for h in hist if h[0] == "k1"]
    mix = [h for h in hist if h[0] == "mix"]
    assert k1[-1][2] < 0.5 * k1[0][2], hist
    assert mix[-1][2] < mix[0][2], hist
    # the K = 1 start ignores the given start: components share alpha and g,
    # with extinctions in the ratio 0.5 : 1 : 2 before the mixture stage
    assert s.shape == (K, n) and torch.all(w.sum(0).sub(1.0).abs() < 1e-9)
