"""Convenience layer over the C-ABI binding: allocate outputs, call the entry
points, return tensors.  Every numerical step runs in the HIP library.

The per-wavelength parameter layout of the paper is
theta(lambda) = {alpha_k, g_k, sigma_t_k, w_k}_{k=1..K} (Sec. 5.1, eq.
decoder_output); ``media_from_theta`` converts a tensor [S, L, K, 4] in that
order to the library's SoA layout.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import rw
from .rw import Context, Geometry, Media, Tally


@dataclass
class ForwardResult:
    tally: Tally
    R: torch.Tensor        # [n_units] mean total diffuse reflectance
    R_se: torch.Tensor     # [n_units]
    Rr: torch.Tensor       # [n_units, n_bins] radial density, mm^-2
    Rr_se: torch.Tensor
    Pd: torch.Tensor       # [n_units, n_bins] normalised profile Rr / R
    vertices: torch.Tensor  # [n_units] int64


def media_from_theta(theta: torch.Tensor, weights_are_logits: bool = False) -> Media:
    """theta: float32 [S, L, K, 4] with (alpha, g, sigma_t, w) per medium."""
    S, L, K, four = theta.shape
    assert four == 4
    soa = theta.permute(3, 2, 0, 1).reshape(4, K, S * L).contiguous().float()
    return Media(soa[2].contiguous(), soa[0].contiguous(), soa[1].contiguous(),
                 soa[3].contiguous(), S, L, weights_are_logits)


def finalize(ctx: Context, geom: Geometry, tally: Tally, n_units: int, paths_uniform: int,
             paths_per_unit=None, stream=None) -> ForwardResult:
    dev = tally.R.device
    nb = geom.n_bins
    R = torch.empty(n_units, dtype=torch.float64, device=dev)
    R_se = torch.empty_like(R)
    Rr = torch.empty((n_units, nb), dtype=torch.float64, device=dev)
    Rr_se = torch.empty_like(Rr)
    Pd = torch.empty_like(Rr)
    rw.rw_finalize(ctx, geom, n_units, paths_per_unit, paths_uniform, tally, R, R_se, Rr, Rr_se, Pd,
                   stream=stream)
    return ForwardResult(tally, R, R_se, Rr, Rr_se, Pd, tally.vertices)


def forward(ctx: Context, media: Media, geom: Geometry, paths: int, seed: int, batched: bool = True,
            paths_per_unit=None, use_graph: bool = True, autotune: bool = False,
            stream=None, path_mask=None) -> ForwardResult:
    """Forward walk + finalize.  batched=False uses the plain static launch.
    path_mask (batched only, rw.new_path_mask) receives the live-path mask
    that lets the adjoint of the same seed skip paths that add nothing."""
    tally = Tally(media.n_units, geom.n_bins, device=media.sigma_t.device)
    if batched:
        rw.rw_batch_forward(ctx, media, geom, paths_per_unit, paths, seed, tally,
                            use_graph=use_graph, autotune=autotune, stream=stream,
                            path_mask=path_mask)
    else:
        rw.rw_forward(ctx, media, geom, paths, seed, tally, stream=stream)
    return finalize(ctx, geom, tally, media.n_units, paths, paths_per_unit, stream=stream)


def layered_forward(ctx: Context, layers, geom: Geometry, paths: int, seed: int,
                    paths_per_unit=None, use_graph: bool = True, stream=None,
                    path_mask=None) -> ForwardResult:
    """Two-layer forward walk (rw_layered_forward) + finalize."""
    tally = Tally(layers.n_units, geom.n_bins, device=layers.sigma_t.device)
    rw.rw_layered_forward(ctx, layers, geom, paths_per_unit, paths, seed, tally,
                          use_graph=use_graph, stream=stream, path_mask=path_mask)
    return finalize(ctx, geom, tally, layers.n_units, paths, paths_per_unit, stream=stream)


def layered_hero_forward(ctx: Context, layers, geom: Geometry, n_hero: int, paths: int,
                         seed: int, stream=None) -> ForwardResult:
    """Hero-wavelength two-layer walk (rw_layered_hero_forward) + finalize:
    units in groups of n_hero wavelengths sharing paths, `paths` per group."""
    tally = Tally(layers.n_units, geom.n_bins, device=layers.sigma_t.device)
    rw.rw_layered_hero_forward(ctx, layers, geom, n_hero, paths, seed, tally, stream=stream)
    return finalize(ctx, geom, tally, layers.n_units, paths, stream=stream)


def dwivedi_forward(ctx: Context, media: Media, geom: Geometry, paths: int, seed: int,
                    q: float = 1.0, stream=None) -> ForwardResult:
    """Mixture walk with Dwivedi sampling (rw_dwivedi_forward, technique
    probability q) + finalize."""
    tally = Tally(media.n_units, geom.n_bins, device=media.sigma_t.device)
    rw.rw_dwivedi_forward(ctx, media, geom, paths, seed, q, tally, stream=stream)
    return finalize(ctx, geom, tally, media.n_units, paths, stream=stream)


def layered_adjoint(ctx: Context, layers, geom: Geometry, paths: int, seed: int, cot_R=None,
                    cot_bins=None, paths_per_unit=None, use_graph: bool = True, stream=None,
                    path_mask=None):
    """Gradient sums of the two-layer walk (raw, see rw_layered_adjoint): columns
    (sigma_t top, bottom, albedo top, bottom, g top, bottom, 0, 0).  Returns
    (grad, grad_sumsq, vertices, flags)."""
    dev = layers.sigma_t.device
    n = layers.n_units
    grad = torch.empty((n, 8), dtype=torch.float64, device=dev)
    sumsq = torch.empty_like(grad)
    vert = torch.empty(n, dtype=torch.int64, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    rw.rw_layered_adjoint(ctx, layers, geom, paths_per_unit, paths, seed, cot_R, cot_bins, grad,
                          sumsq, vert, flags, use_graph=use_graph, stream=stream,
                          path_mask=path_mask)
    return grad, sumsq, vert, flags


def adjoint(ctx: Context, media: Media, geom: Geometry, paths: int, seed: int, cot_R=None,
            cot_bins=None, batched: bool = True, paths_per_unit=None, use_graph: bool = True,
            stream=None, path_mask=None):
    """Gradient sums (raw, see rw_adjoint).  Returns (grad, grad_sumsq, vertices, flags).
    path_mask (batched only): the live-path mask of the forward with the same
    seed; the replay then skips the paths that add nothing."""
    dev = media.sigma_t.device
    n, P = media.n_units, 4 * geom.n_media
    grad = torch.empty((n, P), dtype=torch.float64, device=dev)
    sumsq = torch.empty_like(grad)
    vert = torch.empty(n, dtype=torch.int64, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    if batched:
        rw.rw_batch_adjoint(ctx, media, geom, paths_per_unit, paths, seed, cot_R, cot_bins, grad,
                            sumsq, vert, flags, use_graph=use_graph, stream=stream,
                            path_mask=path_mask)
    else:
        rw.rw_adjoint(ctx, media, geom, paths, seed, cot_R, cot_bins, grad, sumsq, vert, flags,
                      stream=stream)
    return grad, sumsq, vert, flags


def jacobian(ctx: Context, media: Media, geom: Geometry, paths: int, seed: int,
             batched: bool = True, stream=None):
    """Per-slot Jacobian of the forward sums: J[u][s][j] = d(sum of x over the
    paths of unit u that exit in slot s)/d theta_j (raw sums, layout of
    rw_adjoint's gradient), one path replay per slot with a one-hot bin
    cotangent (batched: only the paths that leave the top, from one forward's
    live-path mask).  The total-R row is J.sum(1)."""
    n, nb2, P = media.n_units, geom.n_bins + 2, 4 * geom.n_media
    dev = media.sigma_t.device
    J = torch.empty((n, nb2, P), dtype=torch.float64, device=dev)
    cot = torch.zeros((n, nb2), dtype=torch.float32, device=dev)
    mask = None
    if batched:
        mask = rw.new_path_mask(n, paths, dev)
        forward(ctx, media, geom, paths, seed, stream=stream, path_mask=mask)
    for s in range(nb2):
        cot.zero_()
        cot[:, s] = 1.0
        grad, _, _, flags = adjoint(ctx, media, geom, paths, seed, cot_bins=cot, batched=batched,
                                    stream=stream, path_mask=mask)
        J[:, s, :] = grad
    return J


class RWReflectance(torch.autograd.Function):
    """Differentiable mixture-of-media reflectance.

    forward(sigma_t, albedo, g, logits [K, n_units] float32 on the GPU) ->
    (R [n_units], bins [n_units, n_bins + 2]) as per-path means (bins not per
    area).  backward replays the same random numbers (same seed) in the
    adjoint kernel and returns d/d(sigma_t, albedo, g, logits); the weights are
    w = softmax(logits) over the K media.  The forward keeps its live-path
    mask, so the replay walks only the paths that left the top surface (the
    others add nothing to any gradient).
    """

    @staticmethod
    def forward(fctx, sigma_t, albedo, g, logits, ctx, geom, paths, seed, n_sets, n_wl):
        media = Media(sigma_t.contiguous(), albedo.contiguous(), g.contiguous(),
                      logits.contiguous(), n_sets, n_wl, weights_are_logits=True)
        tally = Tally(media.n_units, geom.n_bins, device=sigma_t.device)
        mask = rw.new_path_mask(media.n_units, paths, sigma_t.device)
        rw.rw_batch_forward(ctx, media, geom, None, paths, seed, tally, path_mask=mask)
        fctx.save_for_backward(sigma_t, albedo, g, logits)
        fctx.meta = (ctx, geom, paths, seed, n_sets, n_wl)
        fctx.mask = mask
        return tally.R[:, 0] / paths, tally.bins[:, :, 0] / paths

    @staticmethod
    def backward(fctx, gR, gB):
        sigma_t, albedo, g, logits = fctx.saved_tensors
        ctx, geom, paths, seed, n_sets, n_wl = fctx.meta
        media = Media(sigma_t.contiguous(), albedo.contiguous(), g.contiguous(),
                      logits.contiguous(), n_sets, n_wl, weights_are_logits=True)
        cot_R = None if gR is None else (gR / paths).float().contiguous()
        cot_B = None if gB is None else (gB / paths).float().contiguous()
        grad, _, _, _ = adjoint(ctx, media, geom, paths, seed, cot_R, cot_B, path_mask=fctx.mask)
        K = geom.n_media
        gr = grad.t().reshape(4, K, -1).float()
        return gr[0], gr[1], gr[2], gr[3], None, None, None, None, None, None


class RWLayeredReflectance(torch.autograd.Function):
    """Differentiable two-layer reflectance (the Sec. 3 tissue geometry).

    forward(sigma_t, albedo, g [2, n_units] float32 on the GPU (row 0 top
    layer), thickness_mm [n_units]) -> (R [n_units], bins [n_units, n_bins + 2])
    as per-path means (bins not per area).  backward replays the same random
    numbers in the two-layer adjoint and returns d/d(sigma_t, albedo, g) of both
    layers.  The thickness gets no gradient: moving the interface moves the
    paths' support, which a score function does not capture."""

    @staticmethod
    def forward(fctx, sigma_t, albedo, g, thickness_mm, ctx, geom, paths, seed, n_rel_bottom):
        layers = rw.Layers(sigma_t.contiguous(), albedo.contiguous(), g.contiguous(),
                           thickness_mm.contiguous(), n_rel_bottom)
        tally = Tally(layers.n_units, geom.n_bins, device=sigma_t.device)
        mask = rw.new_path_mask(layers.n_units, paths, sigma_t.device)
        rw.rw_layered_forward(ctx, layers, geom, None, paths, seed, tally, path_mask=mask)
        fctx.save_for_backward(sigma_t, albedo, g, thickness_mm)
        fctx.meta = (ctx, geom, paths, seed, n_rel_bottom)
        fctx.mask = mask
        return tally.R[:, 0] / paths, tally.bins[:, :, 0] / paths

    @staticmethod
    def backward(fctx, gR, gB):
        sigma_t, albedo, g, thickness_mm = fctx.saved_tensors
        ctx, geom, paths, seed, n_rel_bottom = fctx.meta
        layers = rw.Layers(sigma_t.contiguous(), albedo.contiguous(), g.contiguous(),
                           thickness_mm.contiguous(), n_rel_bottom)
        cot_R = None if gR is None else (gR / paths).float().contiguous()
        cot_B = None if gB is None else (gB / paths).float().contiguous()
        grad, _, _, _ = layered_adjoint(ctx, layers, geom, paths, seed, cot_R, cot_B,
                                        path_mask=fctx.mask)
        gr = grad[:, :6].t().reshape(3, 2, -1).float()
        return gr[0], gr[1], gr[2], None, None, None, None, None, None
