"""GPU: the live-path mask of the batched forward and the adjoint that replays
only the paths it marks (rw_batch_opts.path_mask).

A path ended by roulette, the vertex cap or a slab bottom adds nothing to any
gradient sum, so skipping it leaves the gradient unchanged: the masked replay
must give the full replay's gradient to FP64 rounding (its sums are taken in
another order) while walking fewer vertices.  The mask itself must mark
exactly the paths that left the top: on the same random streams its
popcount per unit is the oracle's count of top exits."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_27604_amd import api, rw, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_common import ctx, geoms, media, np64  # noqa: E402


def _popcount(mask):
    m = mask.cpu().numpy().view(np.uint32)
    return np.unpackbits(m.view(np.uint8), axis=-1).sum(-1)


def _close(a, b, rel=1e-9):
    """Equal to FP64 rounding: per entry, relative to the entry and to its
    column's largest magnitude."""
    a, b = np64(a), np64(b)
    scale = np.abs(b) + np.abs(b).max(0, keepdims=True) + 1e-300
    return float((np.abs(a - b) / scale).max()) <= rel


def _skip_vs_full(m, g, N, seed, cR, cB, n_units, paths_per_unit=None, **kw):
    mask = rw.new_path_mask(n_units, N)
    mask.fill_(-1)  # garbage: the forward must clear it
    res = api.forward(ctx(), m, g, N, seed, path_mask=mask, paths_per_unit=paths_per_unit)
    assert rw.rw_check(ctx(), res.tally.flags) == 0
    full = api.adjoint(ctx(), m, g, N, seed, cot_R=cR, cot_bins=cB,
                       paths_per_unit=paths_per_unit, **kw)
    skip = api.adjoint(ctx(), m, g, N, seed, cot_R=cR, cot_bins=cB, path_mask=mask,
                       paths_per_unit=paths_per_unit, **kw)
    assert rw.rw_check(ctx(), full[3]) == 0 and rw.rw_check(ctx(), skip[3]) == 0
    return res, mask, full, skip


def test_masked_adjoint_equals_full_replay_on_the_mixture_workload():
    wl = workloads.config2(paths=1 << 16)
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, og = geoms(3, wl.n_rel)
    N = wl.paths_per_unit
    rng = np.random.default_rng(8)
    cR = torch.ones(wl.n_units, dtype=torch.float32, device="cuda")
    cB = torch.from_numpy(rng.standard_normal((wl.n_units, g.n_bins + 2)).astype(np.float32)).cuda()
    res, mask, full, skip = _skip_vs_full(m, g, N, 5, cR, cB, wl.n_units)
    assert _close(skip[0], full[0]), "gradient sums differ"
    assert _close(skip[1], full[1]), "sums of squares differ"
    fv, sv, rv = np64(full[2]), np64(skip[2]), np64(res.vertices)
    # the full replay walks the forward's vertices; the masked one fewer
    assert np.array_equal(fv, rv), np.abs(fv - rv).max()
    assert np.all(sv < fv) and sv.sum() < 0.8 * fv.sum(), (sv.sum() / fv.sum())
    # the mask marks the top exits: the oracle's count on the same streams
    tal, _, _ = O.forward(og, wl.sigma_t, wl.albedo, wl.g, wl.weight, N, 5)
    n_top = tal[:, 7]
    pc = _popcount(mask)
    assert np.all(np.abs(pc - n_top) <= 1e-3 * n_top + 2), np.abs(pc - n_top).max()
    # bits beyond the path count stay clear (N is a multiple of 32 here)
    assert mask.shape[1] == N // 32


@pytest.mark.parametrize("K", [1, 2, 4])
def test_masked_adjoint_random_mixtures_and_incidence(K):
    rng = np.random.default_rng(300 + K)
    n = 24
    s = rng.uniform(0.5, 40, (K, n)).astype(np.float32)
    a = rng.uniform(0.5, 0.999, (K, n)).astype(np.float32)
    gg = rng.uniform(-0.5, 0.95, (K, n)).astype(np.float32)
    w = rng.dirichlet(np.ones(K), n).T.astype(np.float32)
    m = media(s, a, gg, w)
    g, _ = geoms(K, float(rng.uniform(1.0, 1.6)), incidence=K % 2)
    N = 3000  # not a multiple of 32: the last word is partial
    cR = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
    cB = torch.from_numpy(rng.standard_normal((n, g.n_bins + 2)).astype(np.float32)).cuda()
    res, mask, full, skip = _skip_vs_full(m, g, N, 11, cR, cB, n)
    assert _close(skip[0], full[0]) and _close(skip[1], full[1])
    assert np.all(np64(skip[2]) <= np64(full[2]))
    tail = mask[:, -1].cpu().numpy().view(np.uint32)
    assert np.all(tail >> (N % 32) == 0), "bits beyond the last path are set"


def test_masked_adjoint_with_uneven_counts_window_and_small_units():
    """Per-unit path counts (0 included), many small units per wave (paths of a
    unit still running after the wave moved on) and a unit window: only the
    window's mask words are written, and the masked gradient of the window
    equals the full replay's."""
    rng = np.random.default_rng(71)
    K, n = 3, 4096
    s = rng.uniform(0.5, 5.0, (K, n))
    a = rng.uniform(0.5, 0.999, (K, n))
    gg = rng.uniform(0.0, 0.9, (K, n))
    w = rng.dirichlet(np.ones(K), n).T
    m = media(s, a, gg, w)
    g, _ = geoms(K, 1.4, n_bins=32)
    P = 96
    counts = torch.from_numpy(rng.integers(0, P + 1, n).astype(np.int32)).cuda()
    counts[5] = 0
    cR = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
    cB = torch.from_numpy(rng.standard_normal((n, g.n_bins + 2)).astype(np.float32)).cuda()
    res, mask, full, skip = _skip_vs_full(m, g, P, 23, cR, cB, n, paths_per_unit=counts)
    assert _close(skip[0], full[0]) and _close(skip[1], full[1])
    assert int(_popcount(mask)[5]) == 0
    # a window: words outside it are left as they were
    mask2 = torch.full_like(mask, -1)
    t = rw.Tally(n, g.n_bins)
    rw.rw_batch_forward(ctx(), m, g, counts, P, 23, t, unit_begin=1000, unit_end=3000,
                        path_mask=mask2)
    torch.cuda.synchronize()
    assert bool((mask2[:1000] == -1).all()) and bool((mask2[3000:] == -1).all())
    assert torch.equal(mask2[1000:3000], mask[1000:3000])
    G = torch.zeros((n, 4 * K), dtype=torch.float64, device="cuda")
    S = torch.zeros_like(G)
    V = torch.zeros(n, dtype=torch.int64, device="cuda")
    F = torch.zeros(1, dtype=torch.int32, device="cuda")
    rw.rw_batch_adjoint(ctx(), m, g, counts, P, 23, cR, cB, G, S, V, F, unit_begin=1000,
                        unit_end=3000, path_mask=mask2)
    torch.cuda.synchronize()
    assert _close(G[1000:3000], full[0][1000:3000])


@pytest.mark.parametrize("chunk", [1024, 8192])
def test_masked_adjoint_with_other_item_sizes(tmp_path, monkeypatch, chunk):
    """Items of 1 024 and 8 192 paths (set through the tune cache): an item of
    8 192 paths spans 256 mask words, so the replay refills its LDS window of
    64 words four times per item.  Vertex counts equal the default shape's
    and the gradient its value to FP64 rounding."""
    wl = workloads.config2(paths=1 << 15)
    sub = wl.subset(np.arange(12))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, _ = geoms(3, sub.n_rel)
    N, n = sub.paths_per_unit, sub.n_units
    rng = np.random.default_rng(31)
    cR = torch.ones(n, dtype=torch.float32, device="cuda")
    cB = torch.from_numpy(rng.standard_normal((n, g.n_bins + 2)).astype(np.float32)).cuda()
    res, mask, full, skip = _skip_vs_full(m, g, N, 41, cR, cB, n)
    cache = tmp_path / "tune.txt"
    cache.write_text(f"gfx950 K3 adj persistent nb{g.n_bins} p{N} m1|{chunk} 4 0\n")
    monkeypatch.setenv("RW_AUTOTUNE_CACHE", str(cache))
    c2 = rw.Context(0)  # reads the cache at its first batched call
    other = api.adjoint(c2, m, g, N, 41, cot_R=cR, cot_bins=cB, path_mask=mask)
    assert rw.rw_check(c2, other[3]) == 0
    assert torch.equal(other[2], skip[2])
    assert _close(other[0], skip[0]) and _close(other[1], skip[1])


def test_masked_adjoint_of_one_small_unit():
    """One unit of 100 paths: one work item for a workgroup of four waves, so
    three waves take no item at all."""
    m = media(np.full((3, 1), 2.0), np.full((3, 1), 0.9), np.full((3, 1), 0.5),
              np.full((3, 1), 1.0 / 3))
    g, _ = geoms(3, 1.4)
    cR = torch.ones(1, dtype=torch.float32, device="cuda")
    cB = torch.ones((1, g.n_bins + 2), dtype=torch.float32, device="cuda")
    res, mask, full, skip = _skip_vs_full(m, g, 100, 3, cR, cB, 1)
    assert _close(skip[0], full[0]) and _close(skip[1], full[1])
    assert 0 < int(_popcount(mask)[0]) <= 100


def test_masked_layered_adjoint_equals_full_replay():
    wl = workloads.layered_tones(8, paths=1 << 14)
    L = rw.Layers.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.thickness_mm, wl.n_rel_bottom)
    g = rw.Geometry(n_media=2, n_rel=wl.n_rel, n_bins=wl.n_bins)
    N = wl.paths_per_unit
    rng = np.random.default_rng(9)
    n = L.n_units
    cR = torch.ones(n, dtype=torch.float32, device="cuda")
    cB = torch.from_numpy(rng.standard_normal((n, g.n_bins + 2)).astype(np.float32)).cuda()
    mask = rw.new_path_mask(n, N)
    res = api.layered_forward(ctx(), L, g, N, 4, path_mask=mask)
    assert rw.rw_check(ctx(), res.tally.flags) == 0
    full = api.layered_adjoint(ctx(), L, g, N, 4, cot_R=cR, cot_bins=cB)
    skip = api.layered_adjoint(ctx(), L, g, N, 4, cot_R=cR, cot_bins=cB, path_mask=mask)
    assert _close(skip[0], full[0]) and _close(skip[1], full[1])
    assert np.all(np64(skip[2]) < np64(full[2]))


def test_autograd_wrapper_uses_the_mask():
    """RWReflectance keeps the forward's mask: its gradient equals the full
    replay's."""
    K, n = 3, 6
    rng = np.random.default_rng(13)
    s = torch.tensor((10 ** rng.uniform(-0.5, 1, (K, n))).astype(np.float32), device="cuda",
                     requires_grad=True)
    a = torch.tensor(rng.uniform(0.5, 0.99, (K, n)).astype(np.float32), device="cuda",
                     requires_grad=True)
    gg = torch.tensor(rng.uniform(0.0, 0.9, (K, n)).astype(np.float32), device="cuda",
                      requires_grad=True)
    lg = torch.tensor(rng.normal(0, 0.5, (K, n)).astype(np.float32), device="cuda",
                      requires_grad=True)
    g, _ = geoms(K, 1.4)
    N = 1 << 15
    R, B = api.RWReflectance.apply(s, a, gg, lg, ctx(), g, N, 19, n, 1)
    (R.sum() + 0.3 * B[:, 90:150].sum()).backward()
    cot_R = torch.full((n,), 1.0 / N, dtype=torch.float32, device="cuda")
    cot_B = torch.zeros((n, g.n_bins + 2), dtype=torch.float32, device="cuda")
    cot_B[:, 90:150] = 0.3 / N
    m = rw.Media(s.detach(), a.detach(), gg.detach(), lg.detach(), n, 1, weights_are_logits=True)
    grad, _, _, _ = api.adjoint(ctx(), m, g, N, 19, cot_R, cot_B)
    gr = np64(grad)
    for i, t in enumerate((s, a, gg, lg)):
        ref = gr[:, i * K:(i + 1) * K].T
        np.testing.assert_allclose(np64(t.grad), ref, rtol=1e-5,
                                   atol=1e-6 * np.abs(ref).max() + 1e-12)
