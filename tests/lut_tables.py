"""Synthetic look-up tables for the LUT tests (NumPy, no model arithmetic):
a table with the qualitative behaviour of the walk's tables, and tables that
are exactly linear in their coordinates."""
from __future__ import annotations

import math

import numpy as np

from oracle import lut_oracle as LO


def smooth_table(na=64, ng=32, nb=160, alpha_max=0.999, g_max=0.99, r_min=1e-4, r_max=1e3,
                 mod=LO):
    """R rises with alpha and falls with g; the profile widens with alpha and
    its tail stretches with g.  The table spans [1e-4, 1e3] mm; the evaluation
    radii returned span [1e-2, 20] mm, so sigma_t in [0.1, 50] stays on it."""
    alpha = np.linspace(0.0, alpha_max, na)
    g = np.linspace(0.0, g_max, ng)
    R = alpha[:, None] ** 2 * (1.0 - 0.5 * g[None, :])
    step = (math.log(r_max) - math.log(r_min)) / nb
    rc = np.exp(math.log(r_min) + (np.arange(nb) + 0.5) * step)
    width = 0.3 + 2.0 * alpha[:, None, None]
    p = 1.0 - 0.5 * g[None, :, None]
    Pd = np.exp(-(rc[None, None, :] / width) ** p) / (2 * math.pi * width ** 2)
    r = np.exp(np.linspace(math.log(1e-2), math.log(20.0), 48))
    return mod.Table(R.astype(np.float32).astype(np.float64),
                     Pd.astype(np.float32).astype(np.float64), alpha_max, g_max, r_min, r_max), r


def linear_table(na=9, ng=7, nb=40, alpha_max=0.9, g_max=0.8, r_min=1e-2, r_max=1e2,
                 c=(0.3, 0.5, -0.2, 0.1), d=(2.0, 0.4, -0.3, 0.05), mod=LO):
    """R = c0 + c1 alpha + c2 g + c3 alpha g and P_d = d0 + d1 alpha + d2 g +
    d3 t_b at bin centre t_b: bilinear and trilinear interpolation reproduce
    them exactly inside the grid."""
    alpha = np.linspace(0.0, alpha_max, na)
    g = np.linspace(0.0, g_max, ng)
    R = c[0] + c[1] * alpha[:, None] + c[2] * g[None, :] + c[3] * alpha[:, None] * g[None, :]
    tb = np.arange(nb, dtype=np.float64)
    Pd = (d[0] + d[1] * alpha[:, None, None] + d[2] * g[None, :, None] + d[3] * tb[None, None, :])
    return mod.Table(R, Pd, alpha_max, g_max, r_min, r_max)


def annulus_mass(Pd, r):
    """Exit probability per evaluation radius: P_d times the annulus area of a
    log-spaced bin centred (in log r) on each radius."""
    lr = np.log(r)
    h = lr[1] - lr[0]
    edges = np.exp(np.concatenate([lr - 0.5 * h, lr[-1:] + 0.5 * h]))
    return Pd * math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)


def random_params(rng, K, n):
    """(sigma_t, alpha, g, w) [K, n] inside the smooth table's useful range."""
    return (10 ** rng.uniform(-0.5, 0.5, (K, n)), rng.uniform(0.5, 0.95, (K, n)),
            rng.uniform(0.0, 0.8, (K, n)), rng.dirichlet(np.ones(K), n).T.copy())
