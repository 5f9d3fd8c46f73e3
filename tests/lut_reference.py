"""Plain PyTorch reference of the LUT fit (autograd through the interpolation
of paper_2606_27604_amd.lut and the loss of paper_2606_27604_amd.fit), for the
tests of the fused HIP kernel and of the fit's schedule and K = 1 start.
Test infrastructure only."""
from __future__ import annotations

import math

import torch

from paper_2606_27604_amd import lut as L
from paper_2606_27604_amd.fit import LAMBDA_R, Params, joint_loss


def loss_reference(table, params_raw: torch.Tensor, K: int, R_t, Pd_t, mass_t, r,
                   lambda_R: float = LAMBDA_R):
    """Per-unit eq. joint_loss of the LUT model at raw parameters [4K - 1, n]
    (the layout of rw_lut_fit_step), differentiable in params_raw."""
    p = params_raw
    s = torch.exp(p[:K])
    a = torch.sigmoid(p[K:2 * K])
    g = 0.99 * torch.sigmoid(p[2 * K:3 * K])
    w = torch.softmax(torch.cat([p[3 * K:], torch.zeros_like(p[:1])], 0), 0)
    R_hat, Rd = L.mixture_profile(table, s, a, g, w, r)
    Pd = Rd / R_hat.clamp_min(1e-12)[:, None]
    return joint_loss(R_hat, Pd, R_t, Pd_t, mass_t, lambda_R=lambda_R)


def _adam(table, P, R_t, Pd_t, mass_t, r, iters, lr, schedule, lambda_R, hist, tag):
    opt = torch.optim.Adam(P.parameters(), lr=lr)
    for it in range(iters):
        if schedule == "cosine":
            for grp in opt.param_groups:
                grp["lr"] = 0.5 * lr * (1.0 + math.cos(math.pi * it / iters))
        opt.zero_grad(set_to_none=True)
        s, a, gg, lg = P.physical()
        w = torch.softmax(lg, 0)
        R_hat, Rd = L.mixture_profile(table, s.float(), a.float(), gg.float(), w.float(), r)
        Pd = Rd / R_hat.clamp_min(1e-12)[:, None]
        loss_u = joint_loss(R_hat.double(), Pd.double(), R_t, Pd_t, mass_t, lambda_R=lambda_R)
        loss_u.sum().backward()
        opt.step()
        if it == 0 or it == iters - 1 or it % 20 == 0:
            hist.append((tag, it, float(loss_u.detach().mean())))


def fit_reference(table, R_t, Pd_t, mass_t, start, r, iters=200, lr=1e-2, schedule="constant",
                  init_k1_iters=0):
    """The same fit as lut.fit (schedule, K = 1 profile start, component
    spread) with torch.optim.Adam on autograd gradients."""
    dev = R_t.device
    hist = []
    if init_k1_iters > 0:
        K, n = start[0].shape
        one = torch.ones((1, n), dtype=torch.float64, device=dev)
        P1 = Params(one, 0.9 * one, 0.5 * one, one).to(dev)
        _adam(table, P1, R_t, Pd_t, mass_t, r, init_k1_iters, lr, schedule, 0.0, hist, "k1")
        with torch.no_grad():
            s1, a1, g1, _ = P1.physical()
            f = torch.tensor(L.K1_SPREAD[:K], dtype=torch.float64, device=dev)[:, None]
            start = (s1 * f, a1.expand(K, n).clone(), g1.expand(K, n).clone(),
                     torch.full((K, n), 1.0 / K, dtype=torch.float64, device=dev))
    P = Params(*start).to(dev)
    _adam(table, P, R_t, Pd_t, mass_t, r, iters, lr, schedule, LAMBDA_R, hist, "mix")
    with torch.no_grad():
        s, a, gg, lg = P.physical()
        return (s, a, gg, torch.softmax(lg, 0)), hist
