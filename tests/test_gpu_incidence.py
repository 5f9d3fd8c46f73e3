"""GPU parity of the cosine-weighted entry lobe (Sec. 8 variant) against the
oracle and the spherical-albedo closed form.

The lobe draws cos(theta_i) = sqrt(u1) and azimuth 2 pi u2 from the words of
vertex 0, refracts by Snell's law and carries 1 - F(theta_i).  With n = 1 and
isotropic scattering the total reflectance is the spherical albedo of the
half-space, 1 - 2 sqrt(1 - alpha) int mu H(mu) dmu."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import oracle as O
from paper_2606_27604_amd import api, rw, workloads
from tests._stats import SAME_STREAM_Z, mean_se

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_common import ctx, geoms, gpu_forward, media, np64  # noqa: E402
from tests.test_gpu_parity import _compare_traces, _trace_gpu  # noqa: E402


@pytest.mark.parametrize("K,n_rel", [(1, 1.0), (3, 1.4)])
def test_trace_cosine_entry_injected_words(K, n_rel):
    sig = [2.0, 0.7, 9.0][:K]
    alb = [0.95, 0.6, 0.99][:K]
    gg = [0.6, 0.1, 0.9][:K]
    w = [0.5, 0.3, 0.2][:K] if K == 3 else [1.0]
    m = media(np.array(sig)[:, None], np.array(alb)[:, None], np.array(gg)[:, None],
              np.array(w)[:, None])
    g, og = geoms(K, n_rel, incidence=1)
    words = workloads.random_words(2048, 160, seed=500 + K)
    ev_g, out_g, _ = _trace_gpu(m, g, words, 2048, 160)
    ev_o, out_o, _ = O.trace(og, np.float32(sig), np.float32(alb), np.float32(gg),
                             np.float32(w), words=words)
    # vertex 0 carries the refracted direction and the entry weight
    d_g, d_o = ev_g[:, 0, 4:7], ev_o[:, 0, 4:7]
    assert np.max(np.abs(d_g - d_o)) <= 2e-6
    assert np.max(np.abs(ev_g[:, 0, 7] - ev_o[:, 0, 7])) <= 2e-6
    if n_rel > 1.0:
        # directions inside the refraction cone, weights below 1 - F(0)
        assert np.all(d_o[:, 2] >= np.sqrt(1.0 - 1.0 / n_rel ** 2) - 1e-6)
    same = _compare_traces(ev_g, out_g, ev_o, out_o)
    assert same.mean() >= 0.995, f"only {same.mean():.4f} of replayed paths agree"


def test_cosine_forward_spherical_albedo_and_oracle():
    al = np.array([0.5, 0.8, 0.95, 0.99], np.float32)
    n = len(al)
    m = media(np.ones((1, n)), al[None], np.zeros((1, n)), np.ones((1, n)))
    g, og = geoms(1, 1.0, incidence=1)
    N = 1 << 18
    res, flags = gpu_forward(m, g, N, 31)
    assert flags == 0
    R, se = np64(res.R), np64(res.R_se)
    ref = np.array([cf.R_spherical(float(a)) for a in al])
    z = (R - ref) / se
    assert np.all(np.abs(z) <= 3.0), z
    tal, _, vert = O.forward(og, np.ones((1, n)), al[None].astype(np.float64), np.zeros((1, n)),
                             np.ones((1, n)), N, 31)
    oR, ose = mean_se(tal[:, 0], tal[:, 1], N)
    # same random numbers: far closer than the standard error
    assert np.all(np.abs(R - oR) <= 0.25 * se), (R - oR) / se
    assert np.all(np.abs(np64(res.vertices) - vert) <= 1e-3 * vert)
    # the lobe differs from the pencil beam: R_spherical > R_plane for alpha < 1
    gn, _ = geoms(1, 1.0)
    rn, _ = gpu_forward(m, gn, N, 31)
    assert np.all(R - np64(rn.R) > 3 * np.hypot(se, np64(rn.R_se)))


def test_cosine_mixture_forward_and_adjoint_vs_oracle():
    wl = workloads.config2(paths=1 << 15)
    sub = wl.subset(np.arange(16))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, og = geoms(3, sub.n_rel, incidence=1)
    N = sub.paths_per_unit
    res, flags = gpu_forward(m, g, N, 12)
    assert flags == 0
    tal, bins, vert = O.forward(og, sub.sigma_t, sub.albedo, sub.g, sub.weight, N, 12)
    R, se = np64(res.R), np64(res.R_se)
    oR, ose = mean_se(tal[:, 0], tal[:, 1], N)
    assert np.all(np.abs(R - oR) <= 3.0 * np.hypot(se, ose))
    assert np.all(np.abs(R - oR) <= 0.25 * se), (R - oR) / se
    gb = np64(res.tally.bins)
    mg, _ = mean_se(gb[..., 0], gb[..., 1], N)
    mo, so = mean_se(bins[..., 0], bins[..., 1], N)
    hit = bins[..., 0] ** 2 / np.maximum(bins[..., 1], 1e-300) >= 30
    assert np.all(np.abs(mg - mo)[hit] <= 0.25 * so[hit] + 1e-12)
    assert np.all(np.abs(np64(res.vertices) - vert) <= 2e-3 * vert)
    rng = np.random.default_rng(3)
    cR = np.ones(sub.n_units, np.float32)
    cB = rng.standard_normal((sub.n_units, g.n_bins + 2)).astype(np.float32)
    grad, sq, _, flags = api.adjoint(ctx(), m, g, N, 13, cot_R=torch.from_numpy(cR).cuda(),
                                     cot_bins=torch.from_numpy(cB).cuda())
    assert rw.rw_check(ctx(), flags) == 0
    og_, osq = O.adjoint(og, sub.sigma_t, sub.albedo, sub.g, sub.weight, N, 13, cot_R=cR,
                         cot_bins=cB)
    mg, sg = mean_se(np64(grad), np64(sq), N)
    mo, so = mean_se(og_, osq, N)
    z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2 + 1e-300)
    assert np.all(np.abs(z) <= SAME_STREAM_Z), np.abs(z).max()
    # same random numbers: the two gradients are far closer than their SE
    close = np.abs(mg - mo) <= 0.25 * sg + 1e-9 * np.abs(mo).max()
    assert close.mean() >= 0.99, close.mean()


def test_incidence_rejects_unknown_mode():
    m = media([[1.0]], [[0.9]], [[0.0]], [[1.0]])
    g, _ = geoms(1, 1.0, incidence=2)
    with pytest.raises(RuntimeError, match="incidence"):
        api.forward(ctx(), m, g, 64, 0)
