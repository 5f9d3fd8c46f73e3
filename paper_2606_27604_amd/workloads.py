"""Seeded synthetic inputs for the random-walk workloads.

This module only draws parameters (numpy, no transport arithmetic).  Both the
HIP path and the FP64 oracle are fed from here, so they see bit-identical
FP32 parameter values.

The paper's data (skin-tone dataset, trained decoder, captured albedos) is not
available, so the workloads are synthetic stand-ins shaped like the paper's:
per-wavelength K = 3 media parameters theta(lambda) = {alpha_k, g_k, sigma_t_k,
w_k} (Sec. 5.1, eq. decoder_output), a smooth Fresnel boundary (Sec. 8), the
mixture chosen per path (Sec. 4.1), radial tallies in log-spaced bins (the
paper's simulator uses 512 log bins to 5 cm, Sec. 3; these use 256 bins over
[1e-3, 50] mm).

Layout: every parameter array is SoA float32 of shape [K, n_units], with
unit = set_index * n_wavelengths + wavelength_index.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

N_BINS = 256
R_MIN_MM = 1e-3
R_MAX_MM = 50.0


@dataclass
class Workload:
    name: str
    n_media: int
    n_sets: int
    n_wl: int
    sigma_t: np.ndarray  # [K, n_units] float32, mm^-1
    albedo: np.ndarray   # [K, n_units] float32
    g: np.ndarray        # [K, n_units] float32
    weight: np.ndarray   # [K, n_units] float32, sums to 1 over K
    wavelength_nm: np.ndarray  # [n_wl] float32 labels
    paths_per_unit: int
    n_rel: float
    seed: int
    n_bins: int = N_BINS
    r_min_mm: float = R_MIN_MM
    r_max_mm: float = R_MAX_MM
    extra: dict = field(default_factory=dict)

    @property
    def n_units(self) -> int:
        return self.n_sets * self.n_wl

    def subset(self, units) -> "Workload":
        """Workload restricted to the given unit indices (same values)."""
        units = np.asarray(units)
        return Workload(
            name=f"{self.name}[subset {units.size}]", n_media=self.n_media, n_sets=units.size,
            n_wl=1, sigma_t=np.ascontiguousarray(self.sigma_t[:, units]),
            albedo=np.ascontiguousarray(self.albedo[:, units]),
            g=np.ascontiguousarray(self.g[:, units]),
            weight=np.ascontiguousarray(self.weight[:, units]),
            wavelength_nm=self.wavelength_nm, paths_per_unit=self.paths_per_unit,
            n_rel=self.n_rel, seed=self.seed, n_bins=self.n_bins, r_min_mm=self.r_min_mm,
            r_max_mm=self.r_max_mm, extra=dict(self.extra))


def _draw_mixture(rng: np.random.Generator, n_units: int, K: int = 3):
    """Per (unit, medium): sigma_t log-uniform in [0.1, 100] mm^-1, alpha uniform in
    [0.30, 0.999], g uniform in [0, 0.95]; per unit: weights ~ Dirichlet(1, ..., 1)."""
    sigma_t = (10.0 ** rng.uniform(-1.0, 2.0, size=(K, n_units))).astype(np.float32)
    albedo = rng.uniform(0.30, 0.999, size=(K, n_units)).astype(np.float32)
    g = rng.uniform(0.0, 0.95, size=(K, n_units)).astype(np.float32)
    w = rng.dirichlet(np.ones(K), size=n_units).T.astype(np.float32)  # [K, n_units]
    # re-normalise in FP32 so that the stored weights sum to 1 within FP32 rounding
    w = (w / w.sum(axis=0, keepdims=True, dtype=np.float64)).astype(np.float32)
    return sigma_t, albedo, g, w


def config1(paths: int = 1 << 16, seed: int = 0) -> Workload:
    """Single homogeneous semi-infinite medium, g = 0, n = 1, normal incidence,
    16 albedos linearly spaced in [0.50, 0.99], sigma_t = 1 mm^-1."""
    n = 16
    albedo = np.linspace(0.5, 0.99, n).astype(np.float32)[None, :]
    return Workload(
        name="plain-homogeneous-16-albedos", n_media=1, n_sets=n, n_wl=1,
        sigma_t=np.ones((1, n), np.float32), albedo=np.ascontiguousarray(albedo),
        g=np.zeros((1, n), np.float32), weight=np.ones((1, n), np.float32),
        wavelength_nm=np.array([550.0], np.float32), paths_per_unit=paths, n_rel=1.0, seed=seed)


def wavelengths_81() -> np.ndarray:
    return np.arange(380.0, 781.0, 5.0, dtype=np.float32)


def config2(paths: int = 1 << 20, seed: int = 2) -> Workload:
    """Three-medium mixture per wavelength: 81 wavelengths 380-780 nm (5 nm),
    n = 1.4, 256 log bins over [1e-3, 50] mm."""
    rng = np.random.default_rng(seed)
    wl = wavelengths_81()
    s, a, g, w = _draw_mixture(rng, wl.size)
    return Workload(name="mixture3-81wl", n_media=3, n_sets=1, n_wl=wl.size, sigma_t=s,
                    albedo=a, g=g, weight=w, wavelength_nm=wl, paths_per_unit=paths,
                    n_rel=1.4, seed=seed)


def config3(n_sets: int = 65536, n_wl: int = 16, paths: int = 4096, seed: int = 3) -> Workload:
    """Batched sweep: n_sets random three-medium sets x n_wl wavelengths, drawn as in
    the 81-wavelength mixture; wavelength labels linspace(380, 780, n_wl)."""
    rng = np.random.default_rng(seed)
    s, a, g, w = _draw_mixture(rng, n_sets * n_wl)
    return Workload(name=f"batched-{n_sets}x{n_wl}", n_media=3, n_sets=n_sets, n_wl=n_wl,
                    sigma_t=s, albedo=a, g=g, weight=w,
                    wavelength_nm=np.linspace(380.0, 780.0, n_wl).astype(np.float32),
                    paths_per_unit=paths, n_rel=1.4, seed=seed)


def config4(n_sets: int = 1024, paths: int = 1 << 14, seed: int = 4) -> Workload:
    """Adjoint workload: n_sets three-medium sets x 81 wavelengths; cotangents
    v_R = 1 and v_bins ~ N(0, 1) (seeded) in extra."""
    rng = np.random.default_rng(seed)
    wl = wavelengths_81()
    n_units = n_sets * wl.size
    s, a, g, w = _draw_mixture(rng, n_units)
    cot_R = np.ones(n_units, np.float32)
    cot_bins = rng.standard_normal((n_units, N_BINS + 2)).astype(np.float32)
    return Workload(name=f"adjoint-{n_sets}x81", n_media=3, n_sets=n_sets, n_wl=wl.size,
                    sigma_t=s, albedo=a, g=g, weight=w, wavelength_nm=wl,
                    paths_per_unit=paths, n_rel=1.4, seed=seed,
                    extra={"cot_R": cot_R, "cot_bins": cot_bins})


def uneven_paths(n_units: int, base: int, seed: int = 7) -> np.ndarray:
    """Per-unit path counts varying over [base/4, 2*base] (for uneven batches)."""
    rng = np.random.default_rng(seed)
    return rng.integers(base // 4, 2 * base + 1, size=n_units).astype(np.int32)


def random_words(n_paths: int, n_blocks: int, seed: int) -> np.ndarray:
    """Injected 32-bit random words [n_paths, n_blocks, 4] for per-path replays."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 32, size=(n_paths, n_blocks, 4), dtype=np.uint64).astype(np.uint32)


@dataclass
class LayeredWorkload:
    """Two-layer tissue units (Sec. 3 geometry): per (tone, wavelength) the
    top and bottom layers' sigma_t, albedo, g ([2, n_units] float32) and the
    tone's top-layer thickness ([n_units] float32, mm)."""
    name: str
    n_sets: int
    n_wl: int
    sigma_t: np.ndarray
    albedo: np.ndarray
    g: np.ndarray
    thickness_mm: np.ndarray
    wavelength_nm: np.ndarray
    paths_per_unit: int
    n_rel: float          # top layer over the outside
    n_rel_bottom: float   # bottom layer over the outside
    seed: int
    n_bins: int = N_BINS
    r_min_mm: float = R_MIN_MM
    r_max_mm: float = R_MAX_MM

    @property
    def n_units(self) -> int:
        return self.n_sets * self.n_wl

    def subset(self, units) -> "LayeredWorkload":
        units = np.asarray(units)
        c = lambda a: np.ascontiguousarray(a[..., units])  # noqa: E731
        return LayeredWorkload(f"{self.name}[subset {units.size}]", units.size, 1, c(self.sigma_t),
                               c(self.albedo), c(self.g), c(self.thickness_mm),
                               self.wavelength_nm, self.paths_per_unit, self.n_rel,
                               self.n_rel_bottom, self.seed, self.n_bins, self.r_min_mm,
                               self.r_max_mm)


def layered_tones(n_tones: int = 64, paths: int = 1 << 16, seed: int = 6, n_rel: float = 1.4,
                  n_rel_bottom: float = 1.4) -> LayeredWorkload:
    """Synthetic two-layer "skin tones" x 81 wavelengths (380-780 nm).  The
    paper's chromophore spectra are not available; these are smooth stand-ins
    with the structure Sec. 3 describes: a thin top layer (thickness uniform in
    [0.05, 0.35] mm) whose absorption is dominated by a melanin-like term
    falling steeply with wavelength (scaled by a per-tone fraction), over a
    bottom layer with a blood-like absorption (bands near 420 and 550 nm,
    scaled by a per-tone fraction) and a small baseline; scattering falls as a
    power of wavelength in both layers; g(lambda) = 0.62 + 0.00029 lambda/nm in
    both layers (the paper's epidermal phase function)."""
    rng = np.random.default_rng(seed)
    wl = wavelengths_81().astype(np.float64)
    n = n_tones * wl.size
    d = rng.uniform(0.05, 0.35, n_tones)
    f_mel = rng.uniform(0.01, 0.40, n_tones)
    f_blood = rng.uniform(0.002, 0.07, n_tones)
    s_top = rng.uniform(15.0, 40.0, n_tones)   # mm^-1 at 500 nm
    s_bot = rng.uniform(8.0, 25.0, n_tones)
    L = wl[None, :] / 500.0
    mua_top = f_mel[:, None] * 40.0 * L ** -3.3 + 0.02
    blood = 30.0 * np.exp(-((wl - 420.0) / 18.0) ** 2) + 3.5 * np.exp(-((wl - 555.0) / 28.0) ** 2)
    mua_bot = f_blood[:, None] * (blood[None, :] + 0.3) + 0.01
    mus_top = s_top[:, None] * L ** -1.1
    mus_bot = s_bot[:, None] * L ** -1.4
    g = np.broadcast_to(0.62 + 0.00029 * wl[None, :], (n_tones, wl.size))

    def soa(top, bot):
        return np.ascontiguousarray(np.stack([top.reshape(n), bot.reshape(n)]).astype(np.float32))

    st = soa(mua_top + mus_top, mua_bot + mus_bot)
    al = soa(mus_top / (mua_top + mus_top), mus_bot / (mua_bot + mus_bot))
    gg = soa(g, g)
    th = np.ascontiguousarray(np.repeat(d, wl.size).astype(np.float32))
    return LayeredWorkload(f"layered-{n_tones}x81", n_tones, wl.size, st, al, gg, th,
                           wl.astype(np.float32), paths, n_rel, n_rel_bottom, seed)
