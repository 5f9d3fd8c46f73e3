"""Shared helpers of the GPU tests: context, media upload and oracle geometry.

The GPU side is always called through the C ABI (paper_2606_27604_amd.rw);
the oracle side through oracle/oracle.py.  Inputs come from
paper_2606_27604_amd.workloads, which only draws parameters."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2606_27604_amd import api, rw  # noqa: E402

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        _CTX = rw.Context(0)
    return _CTX


def media(sigma_t, albedo, g, w, logits=False):
    K = np.asarray(sigma_t).reshape(-1, np.asarray(sigma_t).shape[-1]).shape[0]
    s = np.asarray(sigma_t, np.float32).reshape(K, -1)
    return rw.Media.from_numpy(s, np.asarray(albedo, np.float32).reshape(K, -1),
                               np.asarray(g, np.float32).reshape(K, -1),
                               np.asarray(w, np.float32).reshape(K, -1), s.shape[1],
                               weights_are_logits=logits)


def geoms(K, n_rel, n_bins=256, slab_mm=0.0, r_min=1e-3, r_max=50.0, rr_weight=1e-4,
          max_vertices=1 << 20, incidence=0):
    g = rw.Geometry(n_media=K, n_rel=n_rel, slab_mm=slab_mm, n_bins=n_bins, r_min_mm=r_min,
                    r_max_mm=r_max, rr_weight=rr_weight, max_vertices=max_vertices,
                    incidence=incidence)
    o = O.Geometry(n_media=K, n_rel=float(np.float32(n_rel)), slab_mm=float(np.float32(slab_mm)),
                   n_bins=n_bins, r_min_mm=float(np.float32(r_min)),
                   r_max_mm=float(np.float32(r_max)), rr_weight=float(np.float32(rr_weight)),
                   rr_survive=float(np.float32(0.1)), max_vertices=max_vertices,
                   incidence=incidence)
    return g, o


def gpu_forward(m, g, paths, seed, batched=True, **kw):
    res = api.forward(ctx(), m, g, paths, seed, batched=batched, **kw)
    flags = rw.rw_check(ctx(), res.tally.flags)
    return res, flags


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)
