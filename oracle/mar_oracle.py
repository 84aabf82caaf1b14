"""FP64 CPU oracle of the MAR initialisation (Section 2.2, Fig. 1, Eq. 4) for
2D fan-beam full scans.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never calls it, and it
shares no code with it.  Plain numpy in FP64; the only step taken from the
C oracle is the system operator (the forward projection of the prior image
and of the metal image), which the initialisation uses as Fig. 1 draws it.

The steps, in the order of the flowchart:
    line_integrals  p_j = -ln(max(d_j, 1) / sum_E I0_j(E)) (counts below one
                    photon are taken as one)
    fbp             equiangular fan-beam filtered backprojection of a full
                    scan (Kak & Slaney, Sec. 3.4.2): pre-weight sid cos(gamma),
                    convolution with the sampled ramp kernel
                        g(0) = 1/(8 a^2), g(n a) = 0 (n even),
                        g(n a) = -1 / (2 pi^2 sin^2(n a)) (n odd),   a = dgamma,
                    times a, then f(x) = (2 pi / n_views) sum_v Q_v(gamma') / L^2
                    with gamma' and L the angle and distance of x seen from the
                    source and linear interpolation between channels (zero
                    outside the detector)
    metal_image     M = [mu_H >= metal_frac * water_H] on the uncorrected FBP
    prior           per spectrum j: 0 where mu_j < air_frac water_j, water_j
                    where mu_j < bone_frac water_j or on M, mu_j elsewhere (air,
                    soft tissue and metal flattened, bone kept)
    nmar            per view: p / (H prior + eps) interpolated linearly across
                    the trace along the channels (nearest value beyond the
                    detector ends), times (H prior + eps); unchanged off the
                    trace (normalised metal artifact reduction, Meyer et al.)
    decompose       Eq. 4: c = Mt^-1 (mu_L, mu_H) with
                    Mt[j][i] = sum_E I0_j mu_i / sum_E I0_j
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def _check_full_fan(g):
    if g.kind != 0 or g.n_rows != 1:
        raise ValueError("the MAR initialisation is defined for 2D fan-beam scans")
    if abs(g.n_views * 2.0 * math.pi / g.views_per_rot - 2.0 * math.pi) > 1e-9:
        raise ValueError("the fan-beam FBP needs one full rotation")


def line_integrals(d, I0):
    """p_j(y) = -ln(max(d_j(y), 1) / sum_E I0_j(E)), shape (2, R)."""
    d = np.asarray(d, dtype=np.float64)
    tot = np.asarray(I0, dtype=np.float64).sum(axis=1)
    return -np.log(np.maximum(d, 1.0) / tot[:, None])


def ramp_kernel(n_cols, dgamma):
    """g(m a) for m = -(n_cols-1) .. n_cols-1 (Kak & Slaney's equiangular kernel)."""
    m = np.arange(-(n_cols - 1), n_cols)
    g = np.zeros(m.shape)
    g[m == 0] = 1.0 / (8.0 * dgamma * dgamma)
    odd = (m % 2) != 0
    g[odd] = -1.0 / (2.0 * math.pi ** 2 * np.sin(m[odd] * dgamma) ** 2)
    return g


def channel_angles(g):
    k = np.arange(g.n_cols)
    return (k - 0.5 * (g.n_cols - 1) - g.col_offset) * g.dgamma


def fan_filter(g, p):
    """Filtered projections Q (n_ch, R) of line integrals p (n_ch, R)."""
    _check_full_fan(g)
    p = np.asarray(p, dtype=np.float64).reshape(-1, g.n_views, g.n_cols)
    kern = ramp_kernel(g.n_cols, g.dgamma)
    w = g.sid * np.cos(channel_angles(g))
    Q = np.zeros_like(p)
    n = g.n_cols
    for c in range(p.shape[0]):
        for v in range(g.n_views):
            full = np.convolve(p[c, v] * w, kern)          # length 3n - 2
            Q[c, v] = g.dgamma * full[n - 1:2 * n - 1]
    return Q.reshape(p.shape[0], -1)


def fan_backproject(g, Q):
    """f(x) = (2 pi / n_views) sum_v Q_v(gamma'(x)) / L(x)^2, shape (n_ch, V)."""
    _check_full_fan(g)
    Q = np.asarray(Q, dtype=np.float64).reshape(-1, g.n_views, g.n_cols)
    x = -0.5 * g.nx * g.dx + (np.arange(g.nx) + 0.5) * g.dx
    y = -0.5 * g.ny * g.dy + (np.arange(g.ny) + 0.5) * g.dy
    X, Y = np.meshgrid(x, y, indexing="xy")               # (ny, nx): x fastest
    kc = 0.5 * (g.n_cols - 1) + g.col_offset
    out = np.zeros((Q.shape[0], g.ny, g.nx))
    for v in range(g.n_views):
        beta = g.beta0 + 2.0 * math.pi * v / g.views_per_rot
        cb, sb = math.cos(beta), math.sin(beta)
        vx, vy = X - g.sid * cb, Y - g.sid * sb            # source -> pixel
        ux, uy = -cb, -sb                                   # central ray
        gam = np.arctan2(ux * vy - uy * vx, ux * vx + uy * vy)
        L2 = vx * vx + vy * vy
        kf = gam / g.dgamma + kc
        k0 = np.floor(kf).astype(np.int64)
        fr = kf - k0
        for c in range(Q.shape[0]):
            q = np.concatenate([[0.0], Q[c, v], [0.0]])     # zero outside the detector
            i0 = np.clip(k0 + 1, 0, g.n_cols + 1)
            i1 = np.clip(k0 + 2, 0, g.n_cols + 1)
            inside = (k0 >= -1) & (k0 <= g.n_cols - 1)
            val = np.where(inside, (1.0 - fr) * q[i0] + fr * q[i1], 0.0)
            out[c] += val / L2
    return (2.0 * math.pi / g.n_views) * out.reshape(Q.shape[0], -1)


def fbp(g, p):
    return fan_backproject(g, fan_filter(g, p))


def effective_mu(I0, mu):
    """Mt[j][i] = sum_E I0_j(E) mu_i(E) / sum_E I0_j(E) (Eq. 4's weights)."""
    I0 = np.asarray(I0, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    return (I0 @ mu.T) / I0.sum(axis=1)[:, None]


def decompose(mu_img, I0, mu):
    """Eq. 4: c (2, V) from the FBP images mu_img (2, V) = (mu_L, mu_H)."""
    return np.linalg.solve(effective_mu(I0, mu), np.asarray(mu_img, dtype=np.float64))


def metal_image(mu_img, prm):
    return (np.asarray(mu_img)[1] >= prm["metal_frac"] * prm["water"][1]).astype(np.uint8)


def prior(mu_img, M, prm):
    """Prior images (2, V): air -> 0, soft tissue and metal -> water_j, bone kept."""
    mu_img = np.asarray(mu_img, dtype=np.float64)
    out = np.empty_like(mu_img)
    for j in range(2):
        wj = prm["water"][j]
        m = mu_img[j]
        out[j] = np.where(m < prm["air_frac"] * wj, 0.0, np.where(m < prm["bone_frac"] * wj, wj, m))
        out[j][np.asarray(M) != 0] = wj
    return out


def nmar(g, p, mask, p_prior, eps):
    """Normalised interpolation across the trace, per view and spectrum."""
    p = np.asarray(p, dtype=np.float64).reshape(-1, g.n_views, g.n_cols)
    pp = np.asarray(p_prior, dtype=np.float64).reshape(p.shape)
    mk = np.asarray(mask).reshape(g.n_views, g.n_cols) != 0
    out = p.copy()
    k = np.arange(g.n_cols)
    for v in range(g.n_views):
        bad = mk[v]
        if not bad.any() or bad.all():
            continue
        for c in range(p.shape[0]):
            den = pp[c, v] + eps
            pn = p[c, v] / den
            out[c, v, bad] = np.interp(k[bad], k[~bad], pn[~bad]) * den[bad]
    return out.reshape(p.shape[0], -1)


def mar_init(g, I0, mu, d, prm):
    """The whole initialisation (Fig. 1).  Returns a dict with the basis
    images c (2, V), the metal image M, the trace mask, and the intermediate
    images and sinograms."""
    p = line_integrals(d, I0)
    mu0 = fbp(g, p)
    M = metal_image(mu0, prm)
    mask, T = O.metal_trace(g, M, prm["t"])
    pri = prior(mu0, M, prm)
    pp = O.forward(g, pri)
    pc = nmar(g, p, mask, pp, prm["eps"])
    mu1 = fbp(g, pc)
    c = decompose(mu1, I0, mu)
    return dict(c=c, M=M, mask=mask, T=T, p=p, mu0=mu0, prior=pri, p_prior=pp, p_corr=pc,
                mu1=mu1)
