"""GPU parity: the HIP walk (through the C ABI) against the FP64 oracle.

Both sides consume the same Philox4x32-10 streams (each implements the
generator from its published definition), so besides the statistical
acceptance rule (|diff| <= 3 combined standard errors, and 0.5 % relative where
the statistics resolve it) the per-path replays can be compared event by event.
FP32 path arithmetic on the GPU versus FP64 in the oracle can flip a rare
threshold decision (a Fresnel or roulette draw, a boundary test, a bin edge)
within about 1e-6 of its threshold; such a flip makes that one path diverge,
which the tolerances below allow for explicitly."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import oracle as O
from paper_2606_27604_amd import rw, workloads
from tests._stats import SAME_STREAM_Z, accept_histogram, histogram_z, mean_se

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_common import ctx, geoms, gpu_forward, media, np64  # noqa: E402


def test_philox_bit_exact_against_oracle():
    rng = np.random.default_rng(1)
    n = 1 << 20
    ctr = rng.integers(0, 1 << 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4096] = np.stack(np.meshgrid(np.arange(16), np.arange(16), np.arange(16), [0],
                                      indexing="ij"), -1).reshape(-1, 4)
    key = 0x0123456789ABCDEF
    out = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    c = torch.from_numpy(ctr.view(np.int32)).cuda()
    rw.rw_debug_philox(ctx(), c, key, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    ref = O.philox(ctr, [key & 0xFFFFFFFF, key >> 32])
    assert np.array_equal(got, ref)


def _trace_gpu(m, g, words, n_paths, n_blocks, seed=0, unit=0):
    ev = torch.zeros((n_paths, n_blocks, 8), dtype=torch.float32, device="cuda")
    out = torch.zeros((n_paths, 8), dtype=torch.float32, device="cuda")
    adj = torch.zeros((n_paths, 2), dtype=torch.float32, device="cuda")
    w = None if words is None else torch.from_numpy(np.ascontiguousarray(words).view(np.int32)).cuda()
    rw.rw_debug_trace(ctx(), m, g, w, n_paths, n_blocks, seed, unit, ev, out, adj)
    torch.cuda.synchronize()
    return np64(ev), np64(out), np64(adj)


def _compare_traces(ev_g, out_g, ev_o, out_o, tol=2e-4):
    """Fraction of paths whose event codes agree at every vertex and whose
    states agree within tol (relative to the path's scale)."""
    n = out_g.shape[0]
    same = np.zeros(n, bool)
    for p in range(n):
        nv = int(out_o[p, 5])
        if int(out_g[p, 5]) != nv or out_g[p, 0] != out_o[p, 0]:
            continue
        cg, co = ev_g[p, :nv + 1], ev_o[p, :nv + 1]
        if not np.array_equal(cg[:, 0], co[:, 0]):
            continue
        scale = 1.0 + np.max(np.abs(co[:, 1:4]))
        if np.max(np.abs(cg[:, 1:4] - co[:, 1:4])) > tol * scale:
            continue
        if np.max(np.abs(cg[:, 4:7] - co[:, 4:7])) > tol * 10:
            continue
        if np.max(np.abs(cg[:, 7] - co[:, 7]) / np.maximum(np.abs(co[:, 7]), 1e-30)) > tol:
            continue
        same[p] = True
    return same


@pytest.mark.parametrize("K,n_rel,g", [(1, 1.0, 0.0), (1, 1.4, 0.8), (3, 1.4, 0.5)])
def test_trace_injected_words_match_oracle(K, n_rel, g):
    sig = [2.0, 0.7, 9.0][:K]
    alb = [0.95, 0.6, 0.99][:K]
    gg = [g, 0.1, 0.9][:K]
    w = [0.5, 0.3, 0.2][:K] if K == 3 else [1.0]
    m = media(np.array(sig)[:, None], np.array(alb)[:, None], np.array(gg)[:, None],
              np.array(w)[:, None])
    gg_, og = geoms(K, n_rel)
    words = workloads.random_words(2048, 160, seed=K * 10 + int(n_rel * 10))
    ev_g, out_g, adj_g = _trace_gpu(m, gg_, words, 2048, 160)
    ev_o, out_o, adj_o = O.trace(og, np.float32(sig), np.float32(alb), np.float32(gg),
                                 np.float32(w), words=words)
    same = _compare_traces(ev_g, out_g, ev_o, out_o)
    assert same.mean() >= 0.995, f"only {same.mean():.4f} of replayed paths agree"
    # medium choice identical on every path (vertex 0 uses no FP arithmetic but a compare)
    assert np.mean(out_g[:, 1] == out_o[:, 1]) >= 0.999
    # score bookkeeping of the agreeing paths: D = n_coll/sigma_t - L and the g score
    ok = same & (out_o[:, 0] == O.END_EXIT_TOP)
    k = out_o[ok, 1].astype(int)
    D_o = out_o[ok, 6] / np.asarray(sig, np.float64)[k] - adj_o[ok, 0]
    assert np.allclose(adj_g[ok, 0], D_o, rtol=1e-3, atol=2e-3 * (1 + np.sqrt(out_o[ok, 6])))
    assert np.allclose(adj_g[ok, 1], adj_o[ok, 1], rtol=1e-3, atol=1e-3 * (1 + out_o[ok, 6]))


def test_trace_philox_stream_matches_oracle():
    m = media([[1.5]], [[0.97]], [[0.7]], [[1.0]])
    g, og = geoms(1, 1.4)
    ev_g, out_g, _ = _trace_gpu(m, g, None, 4096, 256, seed=77, unit=5)
    ev_o, out_o, _ = O.trace(og, [1.5], [np.float32(0.97)], [np.float32(0.7)], [1.0],
                             n_paths=4096, n_blocks=256, seed=77, unit=5)
    same = _compare_traces(ev_g, out_g, ev_o, out_o)
    assert same.mean() >= 0.99, f"only {same.mean():.4f} of Philox-driven paths agree"


def test_forward_homogeneous_closed_form_and_oracle():
    wl = workloads.config1()
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, og = geoms(1, 1.0)
    res, flags = gpu_forward(m, g, wl.paths_per_unit, wl.seed)
    assert flags == 0
    R, se = np64(res.R), np64(res.R_se)
    ref = np.array([cf.R_plane(float(a)) for a in wl.albedo[0]])
    z = (R - ref) / se
    assert np.all(np.abs(z) <= 3.0), z
    tal, bins, vert = O.forward(og, wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.paths_per_unit,
                                wl.seed)
    oR, ose = mean_se(tal[:, 0], tal[:, 1], wl.paths_per_unit)
    zc = (R - oR) / np.hypot(se, ose)
    assert np.all(np.abs(zc) <= 3.0), zc
    # same random numbers: the two estimates are far closer than their SE
    assert np.all(np.abs(R - oR) <= 0.25 * se), (R - oR) / se
    # vertex counts agree to the rare diverging path
    assert np.all(np.abs(np64(res.vertices) - vert) <= 1e-3 * vert)


def test_forward_homogeneous_bias_run_2_22_paths():
    """The 16 homogeneous units (K = 1, g = 0, n = 1) at 2^22 paths each, a
    standard error about 8x smaller than at 2^16: the estimates must still sit
    on the closed-form plane albedo (Chandrasekhar's H function), so any bias
    of the FP32 walk above ~1e-4 would show."""
    wl = workloads.config1()
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, _ = geoms(1, 1.0)
    res, flags = gpu_forward(m, g, 1 << 22, 1234)
    assert flags == 0
    R, se = np64(res.R), np64(res.R_se)
    ref = np.array([cf.R_plane(float(a)) for a in wl.albedo[0]])
    z = (R - ref) / se
    assert np.all(np.abs(z) <= 3.5), z
    assert np.all(se < 3e-4)


def test_forward_mixture_81_wavelengths_vs_oracle():
    wl = workloads.config2(paths=1 << 16)
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, og = geoms(3, wl.n_rel)
    res, flags = gpu_forward(m, g, wl.paths_per_unit, 5)
    assert flags == 0
    tal, bins, vert = O.forward(og, wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.paths_per_unit, 5)
    N = wl.paths_per_unit
    R, se = np64(res.R), np64(res.R_se)
    oR, ose = mean_se(tal[:, 0], tal[:, 1], N)
    z = (R - oR) / np.hypot(se, ose)
    assert np.all(np.abs(z) <= 3.0), z
    # 0.5 % relative wherever 3 combined SE resolve it
    res_ok = 3 * np.hypot(se, ose) <= 0.005 * oR
    assert np.all(np.abs(R - oR)[res_ok] <= 0.005 * oR[res_ok])
    # radial histograms, slot by slot
    gb = np64(res.tally.bins)
    worst = worst_big = 0.0
    for u in range(wl.n_units):
        mg, sg = mean_se(gb[u, :, 0], gb[u, :, 1], N)
        mo, so = mean_se(bins[u, :, 0], bins[u, :, 1], N)
        hits = np.minimum(bins[u, :, 0] ** 2 / np.maximum(bins[u, :, 1], 1e-300),
                          gb[u, :, 0] ** 2 / np.maximum(gb[u, :, 1], 1e-300))
        zb = histogram_z(mg, sg, mo, so, mask=hits >= 30)
        ok, chi2, lim = accept_histogram(zb)
        assert ok, f"unit {u}: chi2 {chi2:.1f} > {lim:.1f} or max|z| {np.max(np.abs(zb)):.2f}"
        # same random numbers: a slot differs only by the paths whose FP32 and
        # FP64 replays part at a threshold, each moving it by about
        # 1/sqrt(hits) of its SE; slots with >= 100 hits agree to a quarter of
        # their SE, slots with 30-100 hits to half of it
        zall = np.abs(histogram_z(mg, sg, mo, so, mask=hits >= 30))
        zbig = np.abs(histogram_z(mg, sg, mo, so, mask=hits >= 100))
        worst = max(worst, float(np.max(zall, initial=0.0)))
        worst_big = max(worst_big, float(np.max(zbig, initial=0.0)))
    assert worst_big <= 0.25, f"largest per-slot |difference| {worst_big:.3f} SE (>= 100 hits)"
    assert worst <= 0.5, f"largest per-slot |difference| {worst:.3f} SE (>= 30 hits)"
    assert np.all(np.abs(np64(res.vertices) - vert) <= 2e-3 * vert)


def test_plain_and_batched_agree():
    wl = workloads.config2(paths=1 << 15)
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, _ = geoms(3, wl.n_rel)
    a, _ = gpu_forward(m, g, wl.paths_per_unit, 9, batched=False)
    b, _ = gpu_forward(m, g, wl.paths_per_unit, 9, batched=True)
    c, _ = gpu_forward(m, g, wl.paths_per_unit, 9, batched=True, use_graph=False)
    # exact integer accumulation: bit-identical whatever the schedule
    for x in (b, c):
        assert torch.equal(a.tally.vertices, x.tally.vertices)
        assert torch.equal(a.tally.R, x.tally.R)
        assert torch.equal(a.tally.bins, x.tally.bins)


def test_same_seed_is_bit_identical_and_seed_changes_result():
    wl = workloads.config2(paths=1 << 14)
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, _ = geoms(3, wl.n_rel)
    a, _ = gpu_forward(m, g, wl.paths_per_unit, 3)
    b, _ = gpu_forward(m, g, wl.paths_per_unit, 3)
    c, _ = gpu_forward(m, g, wl.paths_per_unit, 4)
    assert torch.equal(a.tally.R, b.tally.R) and torch.equal(a.tally.bins, b.tally.bins)
    assert not torch.equal(a.tally.R, c.tally.R)


def test_adjoint_vs_oracle_and_closed_forms():
    # homogeneous, isotropic, index-matched: dR/dalpha closed form, dR/dsigma_t = 0
    al = np.array([0.6, 0.9, 0.99], np.float32)
    m = media(np.full((1, 3), 2.0), al[None], np.zeros((1, 3)), np.ones((1, 3)))
    g, og = geoms(1, 1.0)
    N = 1 << 18
    from paper_2606_27604_amd import api
    cot = torch.ones(3, dtype=torch.float32, device="cuda")
    grad, sq, vert, flags = api.adjoint(ctx(), m, g, N, 21, cot_R=cot)
    assert rw.rw_check(ctx(), flags) == 0
    gr, s2 = np64(grad), np64(sq)
    mean, se = mean_se(gr, s2, N)
    ref = np.array([cf.dR_plane_dalpha(float(a)) for a in al])
    assert np.all(np.abs((mean[:, 1] - ref) / se[:, 1]) <= 3.0), (mean[:, 1] - ref) / se[:, 1]
    assert np.all(np.abs(mean[:, 0] / se[:, 0]) <= 3.0)
    # mixture, Fresnel, anisotropic: against the oracle's FP64 score gradient with
    # random bin cotangents
    wl = workloads.config2(paths=1 << 16)
    sub = wl.subset(np.arange(12))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, og = geoms(3, sub.n_rel)
    rng = np.random.default_rng(0)
    cR = np.ones(sub.n_units, np.float32)
    cB = rng.standard_normal((sub.n_units, g.n_bins + 2)).astype(np.float32)
    grad, sq, vert, flags = api.adjoint(ctx(), m, g, sub.paths_per_unit, 8,
                                        cot_R=torch.from_numpy(cR).cuda(),
                                        cot_bins=torch.from_numpy(cB).cuda())
    assert rw.rw_check(ctx(), flags) == 0
    og_, osq = O.adjoint(og, sub.sigma_t, sub.albedo, sub.g, sub.weight, sub.paths_per_unit, 8,
                         cot_R=cR, cot_bins=cB)
    Np = sub.paths_per_unit
    mg, sg = mean_se(np64(grad), np64(sq), Np)
    mo, so = mean_se(og_, osq, Np)
    z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2 + 1e-300)
    assert np.all(np.abs(z) <= SAME_STREAM_Z), np.abs(z).max()
    # logit gradients sum to zero (softmax), on both sides
    assert np.allclose(np64(grad)[:, 9:12].sum(1), 0.0, atol=1e-6 * np.abs(np64(grad)).max())
