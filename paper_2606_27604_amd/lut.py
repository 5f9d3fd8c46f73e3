"""Scale-independent lookup tables and the LUT-based K-media fit (Sec. 4.2).

Generation (Sec. 4.2, "Scale-independent lookup table").  For a homogeneous
semi-infinite medium the normalised profile depends on (alpha, g) only, and
sigma_t rescales the radial axis (eq. separability):
    P_d(r | alpha, g, sigma_t) = sigma_t^2 P_d(sigma_t r | alpha, g, 1).
So one batched walk over an (alpha, g) grid at sigma_t = 1 gives R(alpha, g) and
P_d(r | alpha, g) for every sigma_t.  Each grid cell is a K = 1 unit of the
batched forward launch; the paper uses an 800 x 800 grid at 10^6 photons per
cell.

Fit (Sec. 4.2, eq. mixture, eq. joint_loss, "Optimization").  The K-media
profile is
    R_d_fit(r) = sum_k w_k R(alpha_k, g_k) P(r | alpha_k, g_k, sigma_t_k),
with R bilinear in (alpha, g) and P trilinear in (alpha, g, log r), the radial
coordinate scaled by sigma_t as above.  The loss is eq. joint_loss (lambda_R =
5) and the optimiser Adam.  Each optimisation step is one fused HIP kernel
(rw_lut_fit_step: the lookups, the loss, its analytic gradient and the Adam
update, one wavefront per unit); the tables come from the walk kernel.  The
shape term compares P_hat = sum_k w_k P_k, the definition after eq.
refl_loss (shape_form "paper", the default), or the normalised profile of
eq. mixture, sum_k w_k R_k P_k / R_hat (shape_form "mixture").

Readings: the grid is uniform in alpha over [0, alpha_max] and in g over
[0, g_max] (the paper gives the size, not the spacing); radial interpolation is
linear in log r between bin centres, and P is 0 outside the table's radial
range (beyond it the table holds only its under/overflow slots).  Since
sigma_t rescales the radius, a table evaluated at radii r for extinctions
sigma_t must cover sigma_t r: the default range [1e-5, 1e5] mm in 512 log bins
(50 per decade) covers target radii in [1e-3, 50] mm for sigma_t in
[0.01, 1000] mm^-1, and the far tail of high-albedo, forward-scattering cells
at sigma_t = 1.  (A table no wider than the targets would put part of every
profile off the table as soon as sigma_t differs from 1, and the log-shape loss
would see cliffs there.)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import api, rw


@dataclass
class LUT:
    alpha: torch.Tensor  # [Na] grid
    g: torch.Tensor      # [Ng] grid
    R: torch.Tensor      # [Na, Ng] total diffuse reflectance
    Pd: torch.Tensor     # [Na, Ng, n_bins] normalised profile (mm^-2 at sigma_t = 1)
    r_min: float
    r_max: float
    n_rel: float
    paths: int

    @property
    def n_bins(self) -> int:
        return self.Pd.shape[-1]


LUT_BINS, LUT_R_MIN, LUT_R_MAX = 512, 1e-5, 1e5


def generate(ctx: rw.Context, n_alpha: int, n_g: int, paths: int, n_rel: float = 1.4,
             n_bins: int = LUT_BINS, r_min: float = LUT_R_MIN, r_max: float = LUT_R_MAX,
             alpha_max: float = 0.999, g_max: float = 0.99, seed: int = 17,
             max_units_per_call: int = 1 << 17, stream=None, on_batch=None) -> LUT:
    """Tables over a uniform (alpha, g) grid at sigma_t = 1, one K = 1 unit per
    cell, batched forward launches of at most max_units_per_call cells.
    on_batch(begin, end, result), if given, is called after each launch has been
    enqueued (for progress and timing)."""
    dev = torch.device("cuda")
    alpha = torch.linspace(0.0, alpha_max, n_alpha, dtype=torch.float32, device=dev)
    g = torch.linspace(0.0, g_max, n_g, dtype=torch.float32, device=dev)
    A, G = torch.meshgrid(alpha, g, indexing="ij")
    n = n_alpha * n_g
    sig = torch.ones((1, n), dtype=torch.float32, device=dev)
    media = rw.Media(sig, A.reshape(1, n).contiguous(), G.reshape(1, n).contiguous(),
                     torch.ones((1, n), dtype=torch.float32, device=dev), n, 1)
    geom = rw.Geometry(n_media=1, n_rel=n_rel, n_bins=n_bins, r_min_mm=r_min, r_max_mm=r_max)
    R = torch.empty(n, dtype=torch.float64, device=dev)
    Pd = torch.empty((n, n_bins), dtype=torch.float32, device=dev)
    for b in range(0, n, max_units_per_call):
        e = min(n, b + max_units_per_call)
        sub = media.unit_range(b, e - b)
        res = api.forward(ctx, sub, geom, paths, seed, stream=stream)
        if on_batch is not None:
            on_batch(b, e, res)
        R[b:e] = res.R
        Pd[b:e] = res.Pd.float()
    return LUT(alpha, g, R.float().reshape(n_alpha, n_g), Pd.reshape(n_alpha, n_g, n_bins),
               r_min, r_max, n_rel, paths)


# Components of the K = 1 initialisation: extinction factors around the K = 1 fit
K1_SPREAD = (0.5, 1.0, 2.0, 4.0)


def _native_tables(lut: LUT):
    """rw_lut view of the tables (float32, contiguous; the tensors are kept in
    the returned tuple)."""
    R = lut.R.float().contiguous()
    Pd = lut.Pd.float().contiguous()
    c = rw.RwLutC(R.data_ptr(), Pd.data_ptr(), lut.alpha.numel(), lut.g.numel(), lut.n_bins,
                  float(lut.alpha[-1]), float(lut.g[-1]), lut.r_min, lut.r_max)
    return c, (R, Pd)


SHAPE_FORMS = {"paper": rw.RW_LUT_SHAPE_PAPER, "mixture": rw.RW_LUT_SHAPE_MIXTURE}


def _native_targets(R_t, Pd_t, mass_t, r, lambda_R: float, shape_form: str = "paper",
                    min_mass: float | None = None, shape_floor: float | None = None):
    from .fit import MIN_BIN_MASS, SHAPE_FLOOR

    R = R_t.float().contiguous()
    Pd = Pd_t.float().contiguous()
    mass = mass_t.float().contiguous()
    rr = r.float().contiguous()
    c = rw.RwLutTargetsC(R.data_ptr(), Pd.data_ptr(), mass.data_ptr(), rr.data_ptr(), rr.numel(),
                         float(lambda_R), MIN_BIN_MASS if min_mass is None else float(min_mass),
                         SHAPE_FLOOR if shape_floor is None else float(shape_floor),
                         SHAPE_FORMS[shape_form])
    return c, (R, Pd, mass, rr)


def raw_from_physical(sigma_t, albedo, g, w) -> torch.Tensor:
    """Raw parameters [4K - 1, n] float32 of rw_lut_fit_step: log sigma_t,
    logit alpha, logit(g / 0.99), K - 1 logits (the last is 0); the same
    parameterisation and clamps as fit.Params."""
    K = sigma_t.shape[0]
    al = albedo.double().clamp(1e-4, 1 - 1e-4)
    gg = (g.double() / 0.99).clamp(1e-4, 1 - 1e-4)
    lw = torch.log(w.double().clamp_min(1e-8))
    rows = [torch.log(sigma_t.double()), torch.log(al / (1 - al)), torch.log(gg / (1 - gg)),
            lw[:K - 1] - lw[K - 1:]]
    return torch.cat(rows, 0).float().contiguous()


def physical_from_raw(params: torch.Tensor, K: int):
    p = params.double()
    logits = torch.cat([p[3 * K:], torch.zeros_like(p[:1])], 0)
    return (torch.exp(p[:K]), torch.sigmoid(p[K:2 * K]), 0.99 * torch.sigmoid(p[2 * K:3 * K]),
            torch.softmax(logits, 0))


def _adam_native(ctx, tabs, tg, params, K, iters, lr, schedule, hist, tag):
    n = params.shape[1]
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.empty(n, dtype=torch.float32, device=params.device)
    for it in range(iters):
        lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * it / iters)) if schedule == "cosine" else lr
        rw.rw_lut_fit_step(ctx, tabs[0], tg[0], n, K, params, m, v, it + 1, lr_t, loss)
        if it == 0 or it == iters - 1 or it % 20 == 0:
            hist.append((tag, it, float(loss.double().mean())))


def fit(lut: LUT, R_t: torch.Tensor, Pd_t: torch.Tensor, mass_t: torch.Tensor,
        start, r: torch.Tensor, iters: int = 200, lr: float = 1e-2, schedule: str = "constant",
        init_k1_iters: int = 0, ctx: rw.Context | None = None, shape_form: str = "paper"):
    """Adam over (log sigma_t, logit alpha, logit g / 0.99, K - 1 free logits)
    per unit on eq. joint_loss with the LUT model (Sec. 4.2, "Optimization"),
    one fused HIP kernel launch per step (rw_lut_fit_step: lookups, loss,
    analytic gradient and the Adam update).

    start: (sigma_t, albedo, g, w) [K, n], used as given when init_k1_iters = 0.
    schedule "cosine" anneals the learning rate as 0.5 lr (1 + cos(pi t / T)).
    init_k1_iters > 0 first fits a single medium to the profile alone (the
    shape term, lambda_R = 0) from alpha = 0.9, g = 0.5, sigma_t = 1 mm^-1, as
    the paper initialises its fit; the K components then start at that medium
    with sigma_t scaled by 0.5, 1, 2 (, 4) and equal weights, since identical
    components would stay identical under a symmetric loss.
    shape_form selects P_hat of the shape term ("paper" or "mixture", see the
    module docstring).
    Returns the fitted physical parameters and the loss history
    [(stage, iteration, mean loss before the step)]."""
    from .fit import LAMBDA_R

    dev = R_t.device
    if ctx is None:
        ctx = rw.Context(dev.index or 0)
    tabs = _native_tables(lut)
    hist = []
    K, n = start[0].shape
    if init_k1_iters > 0:
        one = torch.ones((1, n), dtype=torch.float64, device=dev)
        p1 = raw_from_physical(one, 0.9 * one, 0.5 * one, one)
        tg1 = _native_targets(R_t, Pd_t, mass_t, r, 0.0, shape_form)
        _adam_native(ctx, tabs, tg1, p1, 1, init_k1_iters, lr, schedule, hist, "k1")
        s1, a1, g1, _ = physical_from_raw(p1, 1)
        f = torch.tensor(K1_SPREAD[:K], dtype=torch.float64, device=dev)[:, None]
        start = (s1 * f, a1.expand(K, n), g1.expand(K, n),
                 torch.full((K, n), 1.0 / K, dtype=torch.float64, device=dev))
    params = raw_from_physical(*start)
    tg = _native_targets(R_t, Pd_t, mass_t, r, LAMBDA_R, shape_form)
    _adam_native(ctx, tabs, tg, params, K, iters, lr, schedule, hist, "mix")
    return physical_from_raw(params, K), hist
