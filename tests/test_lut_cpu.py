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
