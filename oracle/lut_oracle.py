"""FP64 reference ("oracle") of the look-up-table fit of Sec. 4.2.

TEST INFRASTRUCTURE ONLY: imported by the test-suite alone.  It shares no
code with the HIP kernel or the package; it evaluates the same written model
in plain NumPy, FP64, vectorised over units.

What is computed (paper, Sec. 4.2):
  * "Scale-independent lookup table": tables R(alpha, g) and P_d(r | alpha, g)
    at sigma_t = 1; extinction rescales the radial axis (eq. separability),
        P(r | alpha, g, sigma_t) = sigma_t^2 P_d(sigma_t r | alpha, g).
  * eq. mixture: R_d_fit(r) = sum_k w_k R(alpha_k, g_k) P(r | alpha_k, g_k,
    sigma_t_k), R bilinear in (alpha, g) and P trilinear in (alpha, g, r).
  * eq. joint_loss = L_shape + lambda_R L_R with L_shape = RMSE over radii of
    log P_hat - log P_target (eq. shape_loss) and L_R = (R_hat - R_target)^2
    (eq. refl_loss), R_hat = sum_k w_k R_k.  The text after eq. refl_loss
    defines P_hat = sum_k w_k P_k ("paper" form); the normalised profile of
    eq. mixture, sum_k w_k R_k P_k / R_hat, is the "mixture" form.
  * "Optimization": Adam (lr 1e-2, cosine schedule), started by a K = 1 fit of
    the profile alone; sigma_t = exp(raw).

Readings (the paper gives the grid size, not its layout):
  * alpha on a uniform grid over [0, alpha_max], g over [0, g_max]; the table
    has n_bins log-spaced radial bins over [r_min, r_max); P is linear in
    log r between bin centres and 0 outside [r_min, r_max) after the
    rescaling; between the outer bin centres and the table edges it is held
    at the outer centre's value.
  * Interpolation is a piecewise-linear function: the cell of a coordinate t
    on a grid of n points is floor(t) of t clamped to [0, n - 1], capped at
    n - 2; its derivative is the cell's slope inside [0, n - 1] and 0 where
    the coordinate was clamped.
  * Loss over the radii whose target exit probability (mass) is at least
    min_mass, with a relative floor f inside the logarithms:
        d_j = log(P_hat_j + f P_t,j + 1e-12) - log(P_t,j + f P_t,j + 1e-12),
        L_shape = sqrt(sum_j d_j^2 / max(n_used, 1) + 1e-30).
    min_mass = 0 and f = 0 give eq. shape_loss itself.
  * Raw parameters per unit, rows [4K - 1][n_units]: log sigma_t (K),
    logit alpha (K), logit(g / 0.99) (K), the first K - 1 softmax logits of the
    weights (the last logit is 0).
  * Adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction
    (Kingma & Ba 2015, Algorithm 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SHAPE_PAPER = 0     # P_hat = sum_k w_k P_k (the definition after eq. refl_loss)
SHAPE_MIXTURE = 1   # P_hat = sum_k w_k R_k P_k / R_hat (eq. mixture, normalised)


@dataclass
class Table:
    R: np.ndarray        # [n_alpha, n_g]
    Pd: np.ndarray       # [n_alpha, n_g, n_bins], mm^-2 at sigma_t = 1
    alpha_max: float
    g_max: float
    r_min: float
    r_max: float

    @property
    def n_alpha(self):
        return self.R.shape[0]

    @property
    def n_g(self):
        return self.R.shape[1]

    @property
    def n_bins(self):
        return self.Pd.shape[2]

    @property
    def log_step(self):
        return (math.log(self.r_max) - math.log(self.r_min)) / self.n_bins


def cell(t, n):
    """Piecewise-linear cell of grid coordinate t on n points: (index, weight of
    the upper point, 1 where t lies inside [0, n - 1] else 0)."""
    t = np.asarray(t, np.float64)
    tc = np.clip(t, 0.0, n - 1.0)
    i = np.minimum(np.floor(tc), n - 2).astype(np.int64)
    i = np.maximum(i, 0)
    inside = ((t >= 0.0) & (t <= n - 1.0)).astype(np.float64)
    return i, tc - i, inside


def lookup_R(tab: Table, alpha, g):
    """Bilinear R(alpha, g) and its derivatives d/dalpha, d/dg."""
    sa = (tab.n_alpha - 1) / tab.alpha_max
    sg = (tab.n_g - 1) / tab.g_max
    ia, fa, ina = cell(np.asarray(alpha) * sa, tab.n_alpha)
    ig, fg, ing = cell(np.asarray(g) * sg, tab.n_g)
    r00 = tab.R[ia, ig]
    r01 = tab.R[ia, ig + 1]
    r10 = tab.R[ia + 1, ig]
    r11 = tab.R[ia + 1, ig + 1]
    lo = (1 - fg) * r00 + fg * r01
    hi = (1 - fg) * r10 + fg * r11
    val = (1 - fa) * lo + fa * hi
    d_alpha = (hi - lo) * sa * ina
    d_g = ((1 - fa) * (r01 - r00) + fa * (r11 - r10)) * sg * ing
    return val, d_alpha, d_g


def lookup_P(tab: Table, alpha, g, sigma_t, r):
    """eq. separability with a trilinear table: P(r | alpha, g, sigma_t) =
    sigma_t^2 P_d(sigma_t r | alpha, g).  alpha, g, sigma_t: [...]; r: [n_r].
    Returns P [..., n_r] and its derivatives with respect to log sigma_t,
    alpha and g (same shape)."""
    alpha = np.asarray(alpha, np.float64)[..., None]
    g = np.asarray(g, np.float64)[..., None]
    sigma_t = np.asarray(sigma_t, np.float64)[..., None]
    r = np.asarray(r, np.float64)
    nb = tab.n_bins
    sa = (tab.n_alpha - 1) / tab.alpha_max
    sg = (tab.n_g - 1) / tab.g_max
    ia, fa, ina = cell(alpha * sa, tab.n_alpha)
    ig, fg, ing = cell(g * sg, tab.n_g)
    # radial grid coordinate of sigma_t r among the bin centres
    tb = (np.log(sigma_t) + np.log(r) - math.log(tab.r_min)) / tab.log_step - 0.5
    inb = (tb >= -0.5) & (tb <= nb - 0.5)
    ib, fb, inr = cell(tb, nb)
    ia, ig = np.broadcast_to(ia, ib.shape), np.broadcast_to(ig, ib.shape)

    def radial(da, dg):
        lo = tab.Pd[ia + da, ig + dg, ib]
        hi = tab.Pd[ia + da, ig + dg, ib + 1]
        return (1 - fb) * lo + fb * hi, hi - lo

    c00, e00 = radial(0, 0)
    c01, e01 = radial(0, 1)
    c10, e10 = radial(1, 0)
    c11, e11 = radial(1, 1)
    lo = (1 - fg) * c00 + fg * c01
    hi = (1 - fg) * c10 + fg * c11
    V = (1 - fa) * lo + fa * hi
    dV_dtb = (1 - fa) * ((1 - fg) * e00 + fg * e01) + fa * ((1 - fg) * e10 + fg * e11)
    dV_da = (hi - lo) * sa * ina
    dV_dg = ((1 - fa) * (c01 - c00) + fa * (c11 - c10)) * sg * ing
    s2 = np.where(inb, sigma_t ** 2, 0.0)
    P = s2 * V
    # d/d(log sigma_t): the factor sigma_t^2 and the shift of the coordinate
    dP_dlogs = s2 * (2.0 * V + dV_dtb * inr / tab.log_step)
    return P, dP_dlogs, s2 * dV_da, s2 * dV_dg


def physical(params, K):
    """Raw parameters [4K - 1, n] -> sigma_t, alpha, g, w (each [K, n]) and the
    sigmoid of the g row (for its derivative)."""
    p = np.asarray(params, np.float64)
    sigma_t = np.exp(p[:K])
    alpha = 1.0 / (1.0 + np.exp(-p[K:2 * K]))
    sgm = 1.0 / (1.0 + np.exp(-p[2 * K:3 * K]))
    g = 0.99 * sgm
    logits = np.concatenate([p[3 * K:], np.zeros((1, p.shape[1]))], 0)
    e = np.exp(logits - logits.max(0, keepdims=True))
    w = e / e.sum(0, keepdims=True)
    return sigma_t, alpha, g, w, sgm


def raw_from_physical(sigma_t, alpha, g, w):
    """Inverse of physical() with the clamps of the fit's start: alpha and
    g / 0.99 in [1e-4, 1 - 1e-4], weights >= 1e-8."""
    K = np.asarray(sigma_t).shape[0]
    a = np.clip(np.asarray(alpha, np.float64), 1e-4, 1 - 1e-4)
    gg = np.clip(np.asarray(g, np.float64) / 0.99, 1e-4, 1 - 1e-4)
    lw = np.log(np.maximum(np.asarray(w, np.float64), 1e-8))
    return np.concatenate([np.log(np.asarray(sigma_t, np.float64)), np.log(a / (1 - a)),
                           np.log(gg / (1 - gg)), lw[:K - 1] - lw[K - 1:]], 0)


def mixture(tab: Table, sigma_t, alpha, g, w, r):
    """eq. mixture: R_hat [n] and R_d_fit(r) [n, n_r] for parameters [K, n]."""
    Rk, _, _ = lookup_R(tab, alpha, g)
    Pk = lookup_P(tab, alpha, g, sigma_t, r)[0]
    w = np.asarray(w, np.float64)
    return (w * Rk).sum(0), ((w * Rk)[..., None] * Pk).sum(0)


def loss_and_grad(tab: Table, params, K, R_t, Pd_t, mass_t, r, lambda_R=5.0, min_mass=0.0,
                  shape_floor=0.0, shape_form=SHAPE_PAPER):
    """eq. joint_loss per unit and its gradient with respect to the raw
    parameters [4K - 1, n] (chain rule written out step by step)."""
    params = np.asarray(params, np.float64)
    n = params.shape[1]
    sigma_t, alpha, g, w, sgm = physical(params, K)
    Rk, dRk_da, dRk_dg = lookup_R(tab, alpha, g)                  # [K, n]
    Pk, dPk_dls, dPk_da, dPk_dg = lookup_P(tab, alpha, g, sigma_t, r)  # [K, n, n_r]
    R_hat = (w * Rk).sum(0)                                        # [n]
    if shape_form == SHAPE_PAPER:
        P_hat = (w[..., None] * Pk).sum(0)                          # [n, n_r]
    else:
        Rc = np.maximum(R_hat, 1e-12)
        N = ((w * Rk)[..., None] * Pk).sum(0)
        P_hat = N / Rc[:, None]
    Pd_t = np.asarray(Pd_t, np.float64)
    use = (np.asarray(mass_t, np.float64) >= min_mass).astype(np.float64)
    f = shape_floor * Pd_t + 1e-12
    d = (np.log(P_hat + f) - np.log(Pd_t + f)) * use
    n_used = np.maximum(use.sum(1), 1.0)
    shape = np.sqrt((d * d).sum(1) / n_used + 1e-30)
    dR = R_hat - np.asarray(R_t, np.float64)
    loss = shape + lambda_R * dR * dR

    # dL/dP_hat per radius, and dL/dR_hat through the reflectance term
    q = d / (n_used * shape)[:, None] / (P_hat + f)                # [n, n_r]
    gR = 2.0 * lambda_R * dR                                       # [n]
    if shape_form == SHAPE_PAPER:
        gP = w[..., None] * q[None]                                 # dL/dP_k   [K, n, n_r]
        gw = (q[None] * Pk).sum(2) + gR[None] * Rk                  # dL/dw_k   [K, n]
        gRk = gR[None] * w                                          # dL/dR_k   [K, n]
    else:
        gN = q / Rc[:, None]                                        # dL/dN_j
        gRh = gR - np.where(R_hat > 1e-12, (q * N).sum(1) / Rc ** 2, 0.0)
        gP = (w * Rk)[..., None] * gN[None]
        gw = Rk * ((gN[None] * Pk).sum(2) + gRh[None])
        gRk = w * ((gN[None] * Pk).sum(2) + gRh[None])
    grad = np.zeros_like(params)
    grad[:K] = (gP * dPk_dls).sum(2)
    d_alpha = (gP * dPk_da).sum(2) + gRk * dRk_da
    d_g = (gP * dPk_dg).sum(2) + gRk * dRk_dg
    grad[K:2 * K] = d_alpha * alpha * (1 - alpha)
    grad[2 * K:3 * K] = d_g * 0.99 * sgm * (1 - sgm)
    # softmax: dL/dl_j = w_j (dL/dw_j - sum_k w_k dL/dw_k), free logits j < K - 1
    wg = (w * gw).sum(0)
    grad[3 * K:] = (w * (gw - wg[None]))[:K - 1]
    return loss, grad


def adam_step(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); returns new arrays."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# K = 1 start of the fit: the components begin at the K = 1 medium with these
# extinction factors and equal weights (identical components would stay
# identical under the symmetric loss)
K1_SPREAD = (0.5, 1.0, 2.0, 4.0)


def fit(tab: Table, R_t, Pd_t, mass_t, start_raw, K, r, iters, lr, schedule="constant",
        init_k1_iters=0, lambda_R=5.0, min_mass=0.0, shape_floor=0.0, shape_form=SHAPE_PAPER):
    """Adam on eq. joint_loss per unit ("Optimization" of Sec. 4.2).
    schedule "cosine": lr_t = lr (1 + cos(pi t / T)) / 2.  init_k1_iters > 0
    first fits one medium to the shape term alone (lambda_R = 0) from
    alpha = 0.9, g = 0.5, sigma_t = 1; the K components then start from it with
    sigma_t scaled by K1_SPREAD and equal weights.  Returns the raw parameters
    and the history [(stage, step, mean loss before the step)] at steps 0,
    every 20th and the last."""
    n = np.asarray(R_t).shape[0]
    hist = []

    def run(p, KK, steps, lam, tag):
        m = np.zeros_like(p)
        v = np.zeros_like(p)
        for it in range(steps):
            lr_t = 0.5 * lr * (1 + math.cos(math.pi * it / steps)) if schedule == "cosine" else lr
            loss, gr = loss_and_grad(tab, p, KK, R_t, Pd_t, mass_t, r, lam, min_mass,
                                     shape_floor, shape_form)
            if it == 0 or it == steps - 1 or it % 20 == 0:
                hist.append((tag, it, float(loss.mean())))
            p, m, v = adam_step(p, gr, m, v, it + 1, lr_t)
        return p

    p = np.asarray(start_raw, np.float64).copy()
    if init_k1_iters > 0:
        one = np.ones((1, n))
        p1 = run(raw_from_physical(one, 0.9 * one, 0.5 * one, one), 1, init_k1_iters, 0.0, "k1")
        s1, a1, g1, _, _ = physical(p1, 1)
        f = np.asarray(K1_SPREAD[:K])[:, None]
        p = raw_from_physical(s1 * f, np.repeat(a1, K, 0), np.repeat(g1, K, 0),
                              np.full((K, n), 1.0 / K))
    p = run(p, K, iters, lambda_R, "mix")
    return p, hist
