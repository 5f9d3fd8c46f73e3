"""More GPU parity and behaviour tests, all through the C ABI.

Schedules and launch forms (graph replay, uneven path counts, unit windows,
sub-range views) must give bit-identical forward tallies: every path draws the
same Philox numbers whatever the schedule, and the forward sums are exact
integers.  Physics against the FP64 oracle and closed forms: K = 1, 2, 4
mixtures, finite slabs (energy balance, Beer-Lambert), the vertex cap, invalid
parameters, the finalize formulas of eq. radsss, the autograd wrapper, the
adjoint against common-random-number central differences, and the full-size
81-wavelength workload in the benchmark's launch form on sampled units.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_27604_amd import api, rw, workloads
from tests._stats import SAME_STREAM_Z, mean_se

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_common import ctx, geoms, gpu_forward, media, np64  # noqa: E402


def _same_tally(a, b):
    return (torch.equal(a.vertices, b.vertices) and torch.equal(a.R, b.R)
            and torch.equal(a.bins, b.bins))


def _run(m, g, paths, seed, batched=True, **kw):
    t = rw.Tally(m.n_units, g.n_bins)
    if batched:
        rw.rw_batch_forward(ctx(), m, g, kw.pop("paths_per_unit", None), paths, seed, t, **kw)
    else:
        rw.rw_forward(ctx(), m, g, paths, seed, t)
    torch.cuda.synchronize()
    return t


def test_graph_replays_match_eager():
    """The graph form, replayed with new seeds and with eager work in between,
    gives the eager result every time."""
    wl = workloads.config2(paths=1 << 13)
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, _ = geoms(3, wl.n_rel)
    for seed in (11, 12, 11, 13):
        ref = _run(m, g, wl.paths_per_unit, seed, use_graph=False)
        _run(m, g, wl.paths_per_unit, seed + 100, batched=False)  # eager work between replays
        got = _run(m, g, wl.paths_per_unit, seed, use_graph=True)
        assert _same_tally(ref, got), f"graph replay with seed {seed} differs"


def test_back_to_back_graph_replays_do_not_wait():
    """Three batched calls of one launch shape (one graph key) with different
    seeds, enqueued with no synchronisation in between: the host returns from
    the last while the GPU is still busy with them (no wait between replays),
    and each tally equals the eager launch of its seed."""
    wl = workloads.config2()
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, _ = geoms(3, wl.n_rel)
    P = wl.paths_per_unit
    _run(m, g, P, 1)  # builds the graph
    outs = [rw.Tally(m.n_units, g.n_bins) for _ in range(3)]
    torch.cuda.synchronize()
    for seed, t in zip((2, 3, 4), outs):
        rw.rw_batch_forward(ctx(), m, g, None, P, seed, t)
    pending = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    assert pending, "the third call returned only after the GPU had finished"
    for seed, t in zip((2, 3, 4), outs):
        assert _same_tally(t, _run(m, g, P, seed, use_graph=False)), seed


def test_uneven_path_counts_and_zero_units():
    """Per-unit path counts (zero included) give, unit by unit, the tallies of a
    uniform call with that unit's count."""
    wl = workloads.config2(paths=1 << 12)
    sub = wl.subset(np.arange(10))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, _ = geoms(3, sub.n_rel)
    counts = np.array([0, 1, 63, 64, 65, 4095, 4096, 777, 0, 2048], np.int32)
    P = int(counts.max())
    t = _run(m, g, P, 5, paths_per_unit=torch.from_numpy(counts).cuda())
    for u in range(sub.n_units):
        if counts[u] == 0:
            assert int(t.vertices[u]) == 0 and float(t.R[u].abs().sum()) == 0.0
            continue
        one = _run(m.unit_range(u, 1), g, int(counts[u]), 5, use_graph=False)
        assert torch.equal(one.vertices[0], t.vertices[u]), u
        assert torch.equal(one.R[0], t.R[u]) and torch.equal(one.bins[0], t.bins[u]), u


def test_unit_window_resume_and_subrange_views():
    """A window [b, e) fills exactly those units, equal to the full call; plain
    per-set calls on sub-range views reproduce the batched call."""
    wl = workloads.config3(n_sets=8)
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, _ = geoms(3, wl.n_rel)
    P = 1024
    full = _run(m, g, P, 7)
    t = rw.Tally(m.n_units, g.n_bins)
    t.R.fill_(-1.0)
    rw.rw_batch_forward(ctx(), m, g, None, P, 7, t, unit_begin=20, unit_end=50)
    torch.cuda.synchronize()
    assert torch.equal(t.R[20:50], full.R[20:50]) and torch.equal(t.bins[20:50], full.bins[20:50])
    assert bool((t.R[:20] == -1.0).all()) and bool((t.R[50:] == -1.0).all())
    for s in range(wl.n_sets):
        v = m.unit_range(s * wl.n_wl, wl.n_wl)
        one = _run(v, g, P, 7, batched=False)
        sl = slice(s * wl.n_wl, (s + 1) * wl.n_wl)
        assert torch.equal(one.R, full.R[sl]) and torch.equal(one.bins, full.bins[sl]), s


def test_finalize_matches_definition():
    """rw_finalize against eq. radsss written out from the raw sums."""
    wl = workloads.config2(paths=1 << 14)
    sub = wl.subset(np.arange(6))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, _ = geoms(3, sub.n_rel)
    res, _ = gpu_forward(m, g, sub.paths_per_unit, 3)
    N = float(sub.paths_per_unit)
    Rs, bins = np64(res.tally.R), np64(res.tally.bins)
    mean = Rs[:, 0] / N
    se = np.sqrt(np.maximum(Rs[:, 1] - Rs[:, 0] ** 2 / N, 0) / (N * (N - 1)))
    edges = 1e-3 * (5e4 ** (np.arange(g.n_bins + 1) / g.n_bins))
    area = np.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    Rr = bins[:, 1:-1, 0] / (N * area)
    Rr_se = np.sqrt(np.maximum(bins[:, 1:-1, 1] - bins[:, 1:-1, 0] ** 2 / N, 0)
                    / (N * (N - 1))) / area
    np.testing.assert_allclose(np64(res.R), mean, rtol=1e-12)
    np.testing.assert_allclose(np64(res.R_se), se, rtol=1e-9)
    np.testing.assert_allclose(np64(res.Rr), Rr, rtol=2e-6)  # FP32 bin edges on the device
    np.testing.assert_allclose(np64(res.Rr_se), Rr_se, rtol=2e-6, atol=1e-300)
    np.testing.assert_allclose(np64(res.Pd), Rr / mean[:, None], rtol=2e-6)
    # every top exit lands in one slot: the slots add up to the total
    np.testing.assert_allclose(bins[:, :, 0].sum(1), Rs[:, 0], rtol=1e-12)


def test_finalize_clamps_path_counts_like_the_walk():
    """A per-unit count above paths_uniform runs paths_uniform paths (the walk's
    clamp), and finalize divides by that same count: R, its SE and the profile
    equal those of a uniform call at paths_uniform.  A negative count runs no
    path and finalizes to zeros."""
    wl = workloads.config2(paths=1 << 12)
    sub = wl.subset(np.arange(4))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, _ = geoms(3, sub.n_rel)
    P = 2048
    counts = torch.tensor([5000, P, 1 << 30, -3], dtype=torch.int32, device="cuda")
    got = api.forward(ctx(), m, g, P, 9, paths_per_unit=counts)
    ref = api.forward(ctx(), m, g, P, 9)
    torch.cuda.synchronize()
    for u in (0, 1, 2):
        assert torch.equal(got.tally.R[u], ref.tally.R[u]), u
        assert torch.equal(got.R[u], ref.R[u]) and torch.equal(got.R_se[u], ref.R_se[u]), u
        assert torch.equal(got.Rr[u], ref.Rr[u]) and torch.equal(got.Pd[u], ref.Pd[u]), u
    assert float(got.R[3]) == 0.0 and float(got.R_se[3]) == 0.0
    assert float(got.Rr[3].abs().sum()) == 0.0 and int(got.vertices[3]) == 0


@pytest.mark.parametrize("K", [1, 2, 4])
def test_mixtures_of_other_sizes_vs_oracle(K):
    rng = np.random.default_rng(40 + K)
    n = 8
    s = (10 ** rng.uniform(-1, 2, (K, n))).astype(np.float32)
    a = rng.uniform(0.3, 0.99, (K, n)).astype(np.float32)
    gg = rng.uniform(0, 0.9, (K, n)).astype(np.float32)
    w = rng.dirichlet(np.ones(K), n).T.astype(np.float32)
    w /= w.sum(0, keepdims=True)
    m = media(s, a, gg, w)
    g, og = geoms(K, 1.4)
    N = 1 << 15
    res, flags = gpu_forward(m, g, N, 17)
    assert flags == 0
    tal, _, vert = O.forward(og, s, a, gg, w, N, 17)
    oR, ose = mean_se(tal[:, 0], tal[:, 1], N)
    R, se = np64(res.R), np64(res.R_se)
    assert np.all(np.abs(R - oR) <= 3 * np.hypot(se, ose)), (R - oR) / np.hypot(se, ose)
    # same random numbers: much closer than the statistical error
    assert np.all(np.abs(R - oR) <= 0.3 * se + 1e-12)
    assert np.all(np.abs(np64(res.vertices) - vert) <= 2e-3 * vert)


def test_slab_energy_balance_and_beer_lambert():
    # alpha = 0, n = 1: no scattering, T = exp(-sigma_t d), R = 0
    d = 0.7
    sig = np.array([[0.5, 1.0, 3.0]], np.float32)
    m = media(sig, np.zeros((1, 3)), np.zeros((1, 3)), np.ones((1, 3)))
    g, og = geoms(1, 1.0, slab_mm=d)
    N = 1 << 18
    t = _run(m, g, N, 2)
    T = np64(t.R)[:, 2] / N
    ref = np.exp(-sig[0].astype(np.float64) * np.float32(d))
    se = np.sqrt(ref * (1 - ref) / N)
    assert np.all(np.abs(T - ref) <= 3 * se), (T - ref) / se
    assert float(t.R[:, 0].abs().sum()) == 0.0
    # scattering slab with a Fresnel boundary: R + T + A = 1 - F(0) in expectation
    sig = np.array([[2.0, 1.0, 4.0]], np.float32)
    al = np.array([[0.9, 0.5, 0.99]], np.float32)
    gg = np.array([[0.5, 0.0, 0.8]], np.float32)
    m = media(sig, al, gg, np.ones((1, 3)))
    g, og = geoms(1, 1.4, slab_mm=1.0)
    t = _run(m, g, N, 4)
    Rs = np64(t.R) / N
    total = Rs[:, 0] + Rs[:, 2] + Rs[:, 3]
    F0 = ((1.4 - 1) / 2.4) ** 2
    tal, _, _ = O.forward(og, sig, al, gg, np.ones((1, 3)), N, 4)
    ot = (tal[:, 0] + tal[:, 2] + tal[:, 3]) / N
    # roulette makes the balance hold in expectation only; the spread of the
    # per-path total is at most the roulette boost x its weight threshold
    assert np.all(np.abs(total - (1 - F0)) <= 5e-3), total
    assert np.all(np.abs(total - ot) <= 1e-3), (total, ot)


def test_vertex_cap_raises_flag_and_scores_zero():
    m = media([[1.0]], [[0.999]], [[0.9]], [[1.0]])
    g, og = geoms(1, 1.4, max_vertices=16)
    N = 1 << 14
    res, flags = gpu_forward(m, g, N, 6)
    assert flags & rw.RW_FLAG_VERTEX_CAP
    tal, _, vert = O.forward(og, [[1.0]], [[np.float32(0.999)]], [[np.float32(0.9)]], [[1.0]], N, 6)
    oR, ose = mean_se(tal[:, 0], tal[:, 1], N)
    R, se = np64(res.R), np64(res.R_se)
    assert np.all(np.abs(R - oR) <= 3 * np.hypot(se, ose))
    # no path goes past the cap
    assert int(res.vertices[0]) <= 16 * N


def test_invalid_parameters_flag_and_zero_only_that_unit():
    s = np.array([[1.0, -1.0, 1.0, 1.0, 1.0]], np.float32)
    a = np.array([[0.9, 0.9, 1.5, 0.9, 0.9]], np.float32)
    gg = np.array([[0.5, 0.5, 0.5, 1.0, 0.5]], np.float32)
    w = np.ones((1, 5), np.float32)
    m = media(s, a, gg, w)
    g, _ = geoms(1, 1.4)
    t = _run(m, g, 4096, 1)
    flags = int(t.flags.item())
    assert flags & rw.RW_FLAG_BAD_PARAMS
    assert float(t.R[1:4].abs().sum()) == 0.0 and int(t.vertices[1:4].sum()) == 0
    good = _run(m.unit_range(4, 1), g, 4096, 1)
    assert torch.equal(good.R[0], t.R[4]) and int(t.vertices[0]) > 0
    # weights that do not sum to one
    m2 = media(np.ones((2, 2)), np.full((2, 2), 0.9), np.zeros((2, 2)),
               np.array([[0.5, 0.7], [0.5, 0.7]]))
    g2, _ = geoms(2, 1.4)
    t2 = _run(m2, g2, 1024, 1)
    assert int(t2.flags.item()) & rw.RW_FLAG_BAD_PARAMS
    assert int(t2.vertices[0]) > 0 and int(t2.vertices[1]) == 0


def test_logits_equal_weights_statistically():
    wl = workloads.config2(paths=1 << 14)
    sub = wl.subset(np.arange(8))
    g, _ = geoms(3, sub.n_rel)
    a, _ = gpu_forward(media(sub.sigma_t, sub.albedo, sub.g, sub.weight), g,
                       sub.paths_per_unit, 4)
    lg = np.log(np.maximum(sub.weight, 1e-30))
    b, _ = gpu_forward(media(sub.sigma_t, sub.albedo, sub.g, lg, logits=True), g,
                       sub.paths_per_unit, 4)
    # softmax(log w) reproduces w to FP32 rounding, so at most a path whose u0
    # lies within rounding of a cumulative weight changes medium
    assert np.all(np.abs(np64(a.R) - np64(b.R)) <= 0.05 * np64(a.R_se))


def test_autograd_function_matches_adjoint_and_finite_differences():
    K, n = 3, 4
    rng = np.random.default_rng(3)
    s = torch.tensor((10 ** rng.uniform(-0.5, 1, (K, n))).astype(np.float32), device="cuda",
                     requires_grad=True)
    a = torch.tensor(rng.uniform(0.5, 0.95, (K, n)).astype(np.float32), device="cuda",
                     requires_grad=True)
    gg = torch.tensor(rng.uniform(0.0, 0.8, (K, n)).astype(np.float32), device="cuda",
                      requires_grad=True)
    lg = torch.tensor(rng.normal(0, 0.5, (K, n)).astype(np.float32), device="cuda",
                      requires_grad=True)
    g, _ = geoms(K, 1.4)
    N = 1 << 17
    R, B = api.RWReflectance.apply(s, a, gg, lg, ctx(), g, N, 31, n, 1)
    loss = R.sum() + 0.5 * B[:, 100:140].sum()
    loss.backward()
    cot_R = torch.ones(n, dtype=torch.float32, device="cuda") / N
    cot_B = torch.zeros((n, g.n_bins + 2), dtype=torch.float32, device="cuda")
    cot_B[:, 100:140] = 0.5 / N
    m = rw.Media(s.detach(), a.detach(), gg.detach(), lg.detach(), n, 1, weights_are_logits=True)
    grad, sq, _, _ = api.adjoint(ctx(), m, g, N, 31, cot_R, cot_B)
    gr = np64(grad)
    for i, t in enumerate((s, a, gg, lg)):
        np.testing.assert_allclose(np64(t.grad).T, gr[:, i * K:(i + 1) * K].astype(np.float32),
                                   rtol=1e-5, atol=1e-7)
    # common-random-number central differences of the same objective in albedo
    h = 1e-3
    for k in range(K):
        ap, am = a.detach().clone(), a.detach().clone()
        ap[k] += h * ap[k]
        am[k] -= h * am[k]
        vals = []
        for aa in (ap, am):
            Rp, Bp = api.RWReflectance.apply(s.detach(), aa, gg.detach(), lg.detach(), ctx(), g, N,
                                             31, n, 1)
            vals.append(np64(Rp) + 0.5 * np64(Bp[:, 100:140]).sum(1))
        fd = (vals[0] - vals[1]) / (2 * h * np64(a.detach()[k]))
        est = gr[:, K + k]
        sd = np.sqrt(np.maximum(np64(sq)[:, K + k] - est ** 2 / N, 0))  # SE of the raw sum
        assert np.all(np.abs(est - fd) <= 4 * sd + 1e-3 * np.abs(fd)), (k, est, fd, sd)


def test_adjoint_against_crn_central_differences_every_parameter():
    """The adjoint's vector-Jacobian product (v_R = 1, random bin cotangents)
    against common-random-number central differences of the same
    cotangent-weighted forward sums on the device, for every column: sigma_t
    (h = 1e-3 sigma_t), albedo (h = 1e-3 alpha), g (h = 1e-3) and the softmax
    logits (h = 1e-2: a logit step moves the medium-choice thresholds, so a
    smaller one would rest on a handful of paths).  Units are independent, so
    one pair of forward launches perturbs a medium of every unit at once.
    Replica means over 8 seeds give the standard errors."""
    K, n = 3, 4
    rng = np.random.default_rng(12)
    s = (10 ** rng.uniform(-0.5, 1, (K, n))).astype(np.float32)
    a = rng.uniform(0.5, 0.95, (K, n)).astype(np.float32)
    gg = rng.uniform(0.0, 0.8, (K, n)).astype(np.float32)
    lg = rng.normal(0, 0.5, (K, n)).astype(np.float32)
    g, _ = geoms(K, 1.4, n_bins=32, r_min=1e-2, r_max=20.0)
    N = 1 << 15
    cotB = rng.standard_normal((n, g.n_bins + 2)).astype(np.float32)
    cR = torch.ones(n, dtype=torch.float32, device="cuda")
    cB = torch.from_numpy(cotB).cuda()

    def J(p4, seed):
        res, flags = gpu_forward(media(*p4, logits=True), g, N, seed)
        assert flags == 0
        return (np64(res.tally.R)[:, 0] + (np64(res.tally.bins)[:, :, 0] * cotB).sum(1)) / N

    reps, P = 8, 4 * K
    adj = np.zeros((reps, n, P))
    fd = np.zeros((reps, n, P))
    for r in range(reps):
        seed = 900 + r
        grad, _, _, flags = api.adjoint(ctx(), media(s, a, gg, lg, logits=True), g, N, seed,
                                        cot_R=cR, cot_bins=cB)
        assert rw.rw_check(ctx(), flags) == 0
        adj[r] = np64(grad) / N
        for j in range(P):
            grp, i = divmod(j, K)
            base = [s, a, gg, lg]
            x = base[grp]
            h = (1e-3 * x[i], 1e-3 * x[i], np.full(n, 1e-3, np.float32),
                 np.full(n, 1e-2, np.float32))[grp]
            xp, xm = x.copy(), x.copy()
            xp[i] = x[i] + h
            xm[i] = x[i] - h
            step = xp[i].astype(np.float64) - xm[i].astype(np.float64)  # the FP32 step taken
            Jp = J([xp if q == grp else base[q] for q in range(4)], seed)
            Jm = J([xm if q == grp else base[q] for q in range(4)], seed)
            fd[r, :, j] = (Jp - Jm) / step
    ma, sa = adj.mean(0), adj.std(0, ddof=1) / np.sqrt(reps)
    mf, sf = fd.mean(0), fd.std(0, ddof=1) / np.sqrt(reps)
    z = (ma - mf) / np.sqrt(sa ** 2 + sf ** 2 + 1e-30)
    assert np.all(np.abs(z) <= 3.5), np.round(z, 2)
    # most columns are resolved by the differences: the check is not vacuous
    assert np.mean(np.abs(mf) > 2 * sf) > 0.5, np.round(mf / sf, 1)


def test_full_size_81_wavelengths_sampled_units_vs_oracle():
    """The benchmark's workload and launch form (81 wavelengths x 2^20 paths,
    persistent graph launch) against the oracle on sampled units."""
    wl = workloads.config2()
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, og = geoms(3, wl.n_rel, n_bins=wl.n_bins)
    res, flags = gpu_forward(m, g, wl.paths_per_unit, 2)
    assert flags == 0
    sample = np.array([1, 17, 40, 63, 80])
    sub = wl.subset(sample)
    R, se = np64(res.R)[sample], np64(res.R_se)[sample]
    for i, u in enumerate(sample):
        tal, bins, vert = O.forward(og, sub.sigma_t[:, i:i + 1], sub.albedo[:, i:i + 1],
                                    sub.g[:, i:i + 1], sub.weight[:, i:i + 1], wl.paths_per_unit,
                                    2, unit_base=int(u))
        oR, ose = mean_se(tal[0, 0], tal[0, 1], wl.paths_per_unit)
        zc = (R[i] - oR) / np.hypot(se[i], ose)
        assert abs(zc) <= 3.0, (u, zc)
        assert abs(R[i] - oR) <= 0.005 * oR, (u, R[i], oR)
        assert abs(R[i] - oR) <= 0.25 * se[i], (u, (R[i] - oR) / se[i])  # same random numbers
        assert abs(float(res.vertices[u]) - vert[0]) <= 1e-3 * vert[0]
    # properties that hold at any size: slots add up to the total, R in (0, 1)
    bins = np64(res.tally.bins)
    np.testing.assert_allclose(bins[:, :, 0].sum(1), np64(res.tally.R)[:, 0], rtol=1e-12)
    assert np.all((np64(res.R) > 0) & (np64(res.R) < 1))


def test_full_size_81_wavelengths_adjoint_sampled_units_vs_oracle():
    """The benchmark's adjoint (81 wavelengths x 2^20 paths, persistent graph
    launch, v_R = 1, v_bins ~ N(0, 1)) against the oracle's FP64 score gradient
    on sampled units, which draw the same random numbers (unit_base)."""
    wl = workloads.config2()
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, og = geoms(3, wl.n_rel, n_bins=wl.n_bins)
    rng = np.random.default_rng(2024)
    cR = np.ones(wl.n_units, np.float32)
    cB = rng.standard_normal((wl.n_units, g.n_bins + 2)).astype(np.float32)
    N = wl.paths_per_unit
    grad, sq, vert, flags = api.adjoint(ctx(), m, g, N, 3, cot_R=torch.from_numpy(cR).cuda(),
                                        cot_bins=torch.from_numpy(cB).cuda())
    assert rw.rw_check(ctx(), flags) == 0
    G, S = np64(grad), np64(sq)
    sample = np.array([0, 33, 80])
    sub = wl.subset(sample)
    zs = []
    for i, u in enumerate(sample):
        og_, osq = O.adjoint(og, sub.sigma_t[:, i:i + 1], sub.albedo[:, i:i + 1], sub.g[:, i:i + 1],
                             sub.weight[:, i:i + 1], N, 3, cot_R=cR[u:u + 1],
                             cot_bins=cB[u:u + 1], unit_base=int(u))
        mg, sg = mean_se(G[u], S[u], N)
        mo, so = mean_se(og_[0], osq[0], N)
        z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2 + 1e-300)
        assert np.all(np.abs(z) <= SAME_STREAM_Z), (u, z)
        zs += list(np.abs(z))
    # same random numbers: far inside the statistical error
    assert np.median(zs) <= 0.05, np.median(zs)
    # properties at any size: the logit gradients of every unit sum to zero
    K = 3
    assert np.allclose(G[:, 3 * K:].sum(1), 0.0, atol=1e-6 * np.abs(G).max())


def test_adjoint_plain_batched_graph_agree_and_sigma_invariance():
    wl = workloads.config2(paths=1 << 14)
    sub = wl.subset(np.arange(9))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, _ = geoms(3, sub.n_rel)
    cR = torch.ones(sub.n_units, dtype=torch.float32, device="cuda")
    outs = [api.adjoint(ctx(), m, g, sub.paths_per_unit, 9, cot_R=cR, batched=b, use_graph=ug)
            for b, ug in ((False, False), (True, False), (True, True))]
    ref = np64(outs[0][0])
    for o in outs[1:]:
        np.testing.assert_allclose(np64(o[0]), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
        assert torch.equal(o[2], outs[0][2])
    # scale invariance of the total (eq. separability): sum_k sigma_k dR/dsigma_k = 0
    N = sub.paths_per_unit
    gs = ref[:, :3] * sub.sigma_t.T.astype(np.float64)
    sq = np64(outs[0][1])[:, :3] * sub.sigma_t.T.astype(np.float64) ** 2
    tot, tot_se = gs.sum(1), np.sqrt(sq.sum(1))
    assert np.all(np.abs(tot) <= 4 * tot_se + 1e-9), tot / tot_se


@pytest.mark.parametrize("n_bins", [1, 4096])
def test_extreme_bin_counts(n_bins):
    """1 and 4 096 bins, the range the ABI accepts; at 4 096 the per-wave
    histogram exceeds a four-wave workgroup's LDS and the launch uses fewer
    waves per workgroup.  The totals are exact integer sums of the same
    per-path values as with 256 bins, so they agree bit for bit, and the slots
    add up to them."""
    wl = workloads.config2(paths=1 << 14)
    sub = wl.subset(np.arange(0, 81, 10))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g256, _ = geoms(3, sub.n_rel, n_bins=256)
    g4k, _ = geoms(3, sub.n_rel, n_bins=n_bins)
    for use_graph in (True, False):
        a = _run(m, g256, sub.paths_per_unit, 31, use_graph=use_graph)
        b = _run(m, g4k, sub.paths_per_unit, 31, use_graph=use_graph)
        assert rw.rw_check(ctx(), a.flags) == 0 and rw.rw_check(ctx(), b.flags) == 0
        assert torch.equal(a.R, b.R) and torch.equal(a.vertices, b.vertices)
        bins = np64(b.bins)
        np.testing.assert_allclose(bins[:, :, 0].sum(1), np64(b.R)[:, 0], rtol=1e-12)
    plain = _run(m, g4k, sub.paths_per_unit, 31, batched=False)
    assert _same_tally(plain, b)
    # the adjoint's LDS does not grow with the bins: same gradient of R
    cR = torch.ones(sub.n_units, dtype=torch.float32, device="cuda")
    ga = api.adjoint(ctx(), m, g256, sub.paths_per_unit, 31, cot_R=cR)
    gb = api.adjoint(ctx(), m, g4k, sub.paths_per_unit, 31, cot_R=cR)
    ref = np64(ga[0])
    np.testing.assert_allclose(np64(gb[0]), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("n,paths", [(24576, 64), (12288, 4096)])
def test_forward_paths_outliving_their_wave_visit(n, paths):
    """Forward counterpart of the test below: many units per wave, so that
    paths end after their wave moved on and add to their own unit's slot
    from global memory (one item per unit: the output rows themselves; two
    items per unit: the slot workspace).  Batched tallies must equal the static
    launch's bit for bit, unit by unit."""
    rng = np.random.default_rng(62 + paths)
    K = 3
    m = media(rng.uniform(0.5, 5.0, (K, n)), rng.uniform(0.5, 0.999, (K, n)),
              rng.uniform(0.0, 0.9, (K, n)), rng.dirichlet(np.ones(K), n).T)
    g, _ = geoms(K, 1.4, n_bins=32)
    ref = _run(m, g, paths, 23, batched=False)
    for use_graph in (True, False):
        got = _run(m, g, paths, 23, use_graph=use_graph)
        assert _same_tally(got, ref)


def test_adjoint_paths_outliving_their_wave_visit():
    """Many small units, so that each wave of the persistent launch takes
    several of them and paths of a unit are still running when the wave moves
    on to the next: those paths tally straight into their own unit's slot.
    The batched gradient must equal the static launch's (one unit per wave,
    no such paths) to FP64 rounding, unit by unit and with bin cotangents, and
    sampled units must match the oracle on the same streams."""
    rng = np.random.default_rng(61)
    K, n = 3, 24576
    s = rng.uniform(0.5, 5.0, (K, n))
    a = rng.uniform(0.5, 0.999, (K, n))
    gg = rng.uniform(0.0, 0.9, (K, n))
    w = rng.dirichlet(np.ones(K), n).T
    m = media(s, a, gg, w)
    g, og = geoms(K, 1.4, n_bins=32)
    cR = rng.standard_normal(n).astype(np.float32)
    cB = rng.standard_normal((n, g.n_bins + 2)).astype(np.float32)
    kw = dict(cot_R=torch.from_numpy(cR).cuda(), cot_bins=torch.from_numpy(cB).cuda())
    N = 64
    ref = api.adjoint(ctx(), m, g, N, 21, batched=False, **kw)
    for use_graph in (True, False):
        got = api.adjoint(ctx(), m, g, N, 21, use_graph=use_graph, **kw)
        assert rw.rw_check(ctx(), got[3]) == 0
        assert torch.equal(got[2], ref[2])
        G, R = np64(got[0]), np64(ref[0])
        ratio = np.abs(G - R) / (1e-9 * (np.abs(R) + np.abs(R).max(0)))
        assert ratio.max() <= 1.0, (ratio.max(), np.unravel_index(ratio.argmax(), R.shape))
        np.testing.assert_allclose(np64(got[1]), np64(ref[1]), rtol=1e-9)
    f = lambda x: x.astype(np.float32)  # noqa: E731
    for u in (0, 1, 777, 12345, n - 1):
        og_, osq = O.adjoint(og, f(s[:, u]), f(a[:, u]), f(gg[:, u]), f(w[:, u]), N, 21,
                             cot_R=cR[u:u + 1], cot_bins=cB[u:u + 1], unit_base=u)
        mg, sg = mean_se(np64(ref[0])[u], np64(ref[1])[u], N)
        mo, so = mean_se(og_[0], osq[0], N)
        z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2 + 1e-300)
        assert np.all(np.abs(z) <= SAME_STREAM_Z), (u, z)


def test_adjoint_workload_subset_vs_oracle_gradient():
    """Sets of the adjoint workload (K = 3, 81 wavelengths, 2^14 paths, v_R = 1,
    v_bins ~ N(0, 1)) against the oracle's FP64 score gradient, same streams."""
    wl = workloads.config4(n_sets=2)
    m = media(wl.sigma_t, wl.albedo, wl.g, wl.weight)
    g, og = geoms(3, wl.n_rel)
    cR, cB = wl.extra["cot_R"], wl.extra["cot_bins"]
    grad, sq, vert, flags = api.adjoint(ctx(), m, g, wl.paths_per_unit, 13,
                                        cot_R=torch.from_numpy(cR).cuda(),
                                        cot_bins=torch.from_numpy(cB).cuda())
    assert rw.rw_check(ctx(), flags) == 0
    og_, osq = O.adjoint(og, wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.paths_per_unit, 13,
                         cot_R=cR, cot_bins=cB)
    N = wl.paths_per_unit
    mg, sg = mean_se(np64(grad), np64(sq), N)
    mo, so = mean_se(og_, osq, N)
    z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2 + 1e-300)
    assert np.all(np.abs(z) <= SAME_STREAM_Z), np.abs(z).max()
    # same random numbers: far inside the statistical error
    assert np.median(np.abs(z)) <= 0.05, np.median(np.abs(z))


def test_full_size_batched_sweep_sampled_units_vs_oracle():
    """The batched sweep as the benchmark times it (65,536 sets x 16
    wavelengths x 4,096 paths, one persistent graph launch) against the oracle
    on sampled units, which draw the same random numbers (unit_base)."""
    wl = workloads.config3()
    m = rw.Media.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.n_sets, wl.n_wl)
    g, og = geoms(3, wl.n_rel, n_bins=wl.n_bins)
    res, flags = gpu_forward(m, g, wl.paths_per_unit, 7)
    assert flags == 0
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(wl.n_units, 24, replace=False))
    sub = wl.subset(sample)
    N = wl.paths_per_unit
    R, se = np64(res.R)[sample], np64(res.R_se)[sample]
    for i, u in enumerate(sample):
        tal, _, vert = O.forward(og, sub.sigma_t[:, i:i + 1], sub.albedo[:, i:i + 1],
                                 sub.g[:, i:i + 1], sub.weight[:, i:i + 1], N, 7,
                                 unit_base=int(u))
        oR, ose = mean_se(tal[0, 0], tal[0, 1], N)
        assert abs(R[i] - oR) <= 3.0 * np.hypot(se[i], ose), u
        assert abs(R[i] - oR) <= 0.25 * se[i] + 1e-12, (u, (R[i] - oR) / se[i])
        assert abs(float(res.vertices[u]) - vert[0]) <= 2e-3 * vert[0]
    Rall = np64(res.R)
    assert np.all((Rall > 0) & (Rall < 1))
    bins = np64(res.tally.bins)
    np.testing.assert_allclose(bins[:, :, 0].sum(1), np64(res.tally.R)[:, 0], rtol=1e-12)


def test_full_size_adjoint_sweep_sampled_units_vs_oracle():
    """The adjoint sweep as the benchmark times it (1,024 sets x 81
    wavelengths x 2^14 paths, v_R = 1, v_bins ~ N(0, 1), persistent graph
    launch) against the oracle's FP64 gradient on sampled units."""
    wl = workloads.config4()
    m = rw.Media.from_numpy(wl.sigma_t, wl.albedo, wl.g, wl.weight, wl.n_sets, wl.n_wl)
    g, og = geoms(3, wl.n_rel)
    cR, cB = wl.extra["cot_R"], wl.extra["cot_bins"]
    grad, sq, vert, flags = api.adjoint(ctx(), m, g, wl.paths_per_unit, 41,
                                        cot_R=torch.from_numpy(cR).cuda(),
                                        cot_bins=torch.from_numpy(cB).cuda())
    assert rw.rw_check(ctx(), flags) == 0
    rng = np.random.default_rng(6)
    sample = np.sort(rng.choice(wl.n_units, 12, replace=False))
    sub = wl.subset(sample)
    N = wl.paths_per_unit
    G, S = np64(grad)[sample], np64(sq)[sample]
    zs = []
    for i, u in enumerate(sample):
        og_, osq = O.adjoint(og, sub.sigma_t[:, i:i + 1], sub.albedo[:, i:i + 1],
                             sub.g[:, i:i + 1], sub.weight[:, i:i + 1], N, 41,
                             cot_R=cR[u:u + 1], cot_bins=cB[u:u + 1], unit_base=int(u))
        mg, sg = mean_se(G[i:i + 1], S[i:i + 1], N)
        mo, so = mean_se(og_, osq, N)
        zs.append(((mg - mo) / np.sqrt(sg ** 2 + so ** 2 + 1e-300)).ravel())
    z = np.concatenate(zs)
    assert np.all(np.abs(z) <= SAME_STREAM_Z), np.abs(z).max()
    # same random numbers: far inside the statistical error (a path whose FP32
    # and FP64 replays part at a threshold moves one unit's gradient by a
    # fraction of its SE, hence a median over the 144 sampled values)
    assert np.median(np.abs(z)) <= 0.08, np.median(np.abs(z))
    # the softmax logits' gradients sum to zero in every unit
    gr = np64(grad)
    assert np.allclose(gr[:, 9:12].sum(1), 0.0, atol=1e-6 * np.abs(gr).max())


def test_per_slot_jacobian_matches_oracle():
    """The full per-slot Jacobian (n_bins + 2 slots x 12 parameters) from
    one-hot-cotangent replays against the oracle's FP64 Jacobian on the same
    streams; its slot sum is the total-R gradient."""
    wl = workloads.config2(paths=1 << 16)
    sub = wl.subset(np.array([3, 40]))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, og = geoms(3, sub.n_rel, n_bins=32)
    N = sub.paths_per_unit
    J = np64(api.jacobian(ctx(), m, g, N, 17))
    _, _, jR, jB = O.adjoint(og, sub.sigma_t, sub.albedo, sub.g, sub.weight, N, 17,
                             cot_R=np.zeros(2), jacobian=True)
    assert J.shape == jB.shape == (2, 34, 12)
    # same random numbers: every entry agrees to a small fraction of the entry
    # scale of its unit and parameter (a rare FP32/FP64 parting moves a few paths)
    scale = np.abs(jB).max(axis=1, keepdims=True) + 1e-300
    assert np.quantile(np.abs(J - jB) / scale, 0.99) <= 2e-3
    np.testing.assert_allclose(J.sum(1), jR, rtol=2e-3, atol=2e-3 * np.abs(jR).max())
    cR = torch.ones(2, dtype=torch.float32, device="cuda")
    grad, _, _, _ = api.adjoint(ctx(), m, g, N, 17, cot_R=cR)
    np.testing.assert_allclose(J.sum(1), np64(grad), rtol=1e-9, atol=1e-9 * np.abs(J).max())


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_mixture_random_parameters_vs_oracle(K):
    """Forward and adjoint over random mixtures spanning the parameter space
    (sigma_t 0.5-40 /mm, albedo 0.5-0.999, g -0.5-0.95, Dirichlet weights,
    n 1.0-1.6, normal and cosine incidence) against the oracle on the same
    streams; the adjoint walks the forward's vertices."""
    rng = np.random.default_rng(2000 + K)
    n = 24
    s = rng.uniform(0.5, 40, (K, n)).astype(np.float32)
    a = rng.uniform(0.5, 0.999, (K, n)).astype(np.float32)
    g = rng.uniform(-0.5, 0.95, (K, n)).astype(np.float32)
    w = rng.dirichlet(np.ones(K), n).T.astype(np.float32)
    m = media(s, a, g, w)
    gg, og = geoms(K, float(rng.uniform(1.0, 1.6)), incidence=K % 2)
    N = 1 << 13
    seed = 70 + K
    cR = np.ones(n, np.float32)
    cB = rng.standard_normal((n, gg.n_bins + 2)).astype(np.float32)
    grad, sq, vert, flags = api.adjoint(ctx(), m, gg, N, seed, cot_R=torch.from_numpy(cR).cuda(),
                                        cot_bins=torch.from_numpy(cB).cuda())
    assert rw.rw_check(ctx(), flags) == 0
    ogr, osq = O.adjoint(og, s, a, g, w, N, seed, cot_R=cR, cot_bins=cB)
    mg, sg = mean_se(np64(grad), np64(sq), N)
    mo, so = mean_se(ogr, osq, N)
    z = np.abs(mg - mo) / np.sqrt(sg ** 2 + so ** 2 + 1e-300)
    assert z.max() <= SAME_STREAM_Z and np.median(z) <= 0.05, (z.max(), np.median(z))
    res, f2 = gpu_forward(m, gg, N, seed)
    assert f2 == 0
    tal, _, _ = O.forward(og, s, a, g, w, N, seed)
    R, se = np64(res.R), np64(res.R_se)
    oR, ose = mean_se(tal[:, 0], tal[:, 1], N)
    assert np.all(np.abs(R - oR) <= 0.25 * np.hypot(se, ose) + 1e-12)
    fv, av = np64(res.vertices), np64(vert)
    assert np.all(np.abs(fv - av) <= 1e-3 * fv)
