"""Pins of the oracle's building blocks (CPU only).

Each piece is checked against something other than itself: rocRAND's own
Philox4x32-10 engine, Hecht's form of the Fresnel equations and the Stokes
energy identity, the Henyey-Greenstein density integrated numerically, the
definition of an orthonormal frame, and the bin edges of the log grid."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import closed_forms as cf
from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference helper")
    exe = str(tmp_path_factory.mktemp("rr") / "rr_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_ref.cpp")],
                          cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def _rocrand_blocks(exe, ctrs, keys):
    lines = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctrs, keys))
    out = subprocess.run([exe], input=lines + "\n", capture_output=True, text=True, check=True).stdout
    return np.array([[int(t) for t in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(11)
    n = 20000
    ctrs = rng.integers(0, 1 << 32, size=(n, 4), dtype=np.uint64)
    # also the structured counters the walk uses: small vertex / path / unit indices
    ctrs[:64] = [[v, p, u, 0] for v in range(4) for p in range(4) for u in range(4)]
    ctrs[64:70] = [[0xFFFFFFFF] * 4, [0] * 4, [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]]
    keys = rng.integers(0, 1 << 32, size=(n, 2), dtype=np.uint64)
    keys[:70] = [0, 0]
    ref = _rocrand_blocks(rocrand_ref, ctrs, keys)
    got = np.concatenate([O.philox(ctrs[i:i + 1], keys[i]) for i in range(n)])
    assert np.array_equal(got.astype(np.uint64), ref)


def test_philox_output_is_uniform():
    ctr = np.zeros((1 << 16, 4), np.uint32)
    ctr[:, 1] = np.arange(1 << 16)
    w = O.philox(ctr, [7, 9]).ravel()
    counts = np.bincount((w >> 28).astype(np.int64), minlength=16)
    assert stats.chisquare(counts).pvalue > 1e-4


def test_u01_map_open_interval_and_exact_in_fp32():
    lo, hi = O.u01(0), O.u01(0xFFFFFFFF)
    assert lo == 2.0 ** -24 and hi == 1.0 - 2.0 ** -24
    for w in (0, 1, 511, 512, 0x7FFFFFFF, 0x80000000, 0xFFFFFE00, 0xFFFFFFFF):
        u = O.u01(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exactly representable in FP32
        assert float(np.float32(1.0) - np.float32(u)) == 1.0 - u


@pytest.mark.parametrize("n", [1.0, 1.33, 1.4, 1.6, 0.8])
def test_fresnel_matches_hecht_form(n):
    for c in np.linspace(0.0, 1.0, 201):
        assert abs(O.fresnel(c, n) - cf.fresnel_hecht(c, n)) < 1e-12


@pytest.mark.parametrize("n", [1.33, 1.4, 1.6])
def test_fresnel_stokes_energy_identity(n):
    # R + T = 1 with T from the transmission amplitudes (inside index n -> 1)
    for c in np.linspace(0.05, 1.0, 50):
        s2 = n * n * (1 - c * c)
        if s2 >= 1.0:
            assert O.fresnel(c, n) == 1.0
            continue
        ct = math.sqrt(1 - s2)
        ts = 2 * n * c / (n * c + ct)
        tp = 2 * n * c / (c + n * ct)
        T = 0.5 * (ts * ts + tp * tp) * ct / (n * c)
        assert abs(O.fresnel(c, n) + T - 1.0) < 1e-12


def test_fresnel_special_values():
    assert O.fresnel(1.0, 1.4) == pytest.approx((0.4 / 2.4) ** 2, abs=1e-15)
    # index-matched: zero up to rounding, far below the smallest uniform 2^-24, so
    # the reflect/transmit decision never reflects
    assert abs(O.fresnel(0.2, 1.0)) < 1e-25
    assert O.fresnel(0.0, 1.4) == 1.0


@pytest.mark.parametrize("g", [0.0, 0.3, 0.7, 0.95, -0.5])
def test_hg_sampler_inverts_the_density(g):
    # P(mu' <= hg_cos(g, u)) = u, with the probability computed by integrating the
    # closed-form density numerically
    for u in (0.01, 0.2, 0.5, 0.8, 0.99):
        mu = O.hg_cos(g, u)
        p, _ = integrate.quad(lambda m: float(cf.hg_pdf(m, g)), -1.0, mu, epsabs=1e-13)
        assert abs(p - u) < 1e-9


@pytest.mark.parametrize("g", [0.0, 0.4, 0.9])
def test_hg_sampler_mean_cosine_is_g(g):
    u = (np.arange(200000) + 0.5) / 200000
    m = np.mean([O.hg_cos(g, x) for x in u[::10]])
    assert abs(m - g) < 2e-4


@pytest.mark.parametrize("g", [0.1, 0.5, 0.9])
def test_hg_score_is_derivative_of_log_density(g):
    h = 1e-6
    for mu in (-0.9, 0.0, 0.5, 0.99):
        fd = (math.log(cf.hg_pdf(mu, g + h)) - math.log(cf.hg_pdf(mu, g - h))) / (2 * h)
        assert abs(O.hg_dlog_dg(g, mu) - fd) < 1e-6 * max(1, abs(fd))


def test_frame_is_right_handed_orthonormal():
    rng = np.random.default_rng(3)
    dirs = rng.standard_normal((500, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    dirs[:4] = [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1e-9, -1]]
    dirs[:4] /= np.linalg.norm(dirs[:4], axis=1, keepdims=True)
    for d in dirs:
        t1, t2 = O.frame(d)
        M = np.stack([t1, t2, d])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(t1, t2), d, atol=1e-12)


def test_scatter_direction_polar_and_azimuth():
    rng = np.random.default_rng(5)
    for _ in range(300):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        mu = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * np.pi)
        nd = O.scatter_dir(d, mu, phi)
        t1, t2 = O.frame(d)
        st = math.sqrt(1 - mu * mu)
        assert abs(np.linalg.norm(nd) - 1.0) < 1e-12
        assert abs(nd @ d - mu) < 1e-12
        assert abs(nd @ t1 - st * math.cos(phi)) < 1e-12
        assert abs(nd @ t2 - st * math.sin(phi)) < 1e-12


def test_bin_slots_follow_log_edges():
    geo = O.Geometry(n_bins=256)
    e = cf.bin_edges(256, 1e-3, 50.0)
    assert O.bin_slot(0.0, geo) == 0
    assert O.bin_slot(0.999e-3, geo) == 0
    assert O.bin_slot(50.0, geo) == 257
    assert O.bin_slot(1e9, geo) == 257
    for i in range(256):
        mid = math.sqrt(e[i] * e[i + 1])
        assert O.bin_slot(mid, geo) == i + 1
        assert O.bin_slot(e[i] * (1 + 1e-9), geo) == i + 1
        assert O.bin_slot(e[i + 1] * (1 - 1e-9), geo) == i + 1
