"""Chain rule from screen-space gradients to the Gaussian parameters.

Differentiates exactly the forward of ``project`` (EWA projection, sigmoid
opacity, SH colour with the zero clamp), hand-derived, in float64:

* conic (A, B, C) = (c, -b, a) / D with D = a c - b^2, differentiated through
  the scalar entries a, b, c of Sigma2;
* Sigma2 = T Sigma3 T^T with T = J R (rows T0, T1): dSigma3 = ga T0 T0^T +
  gb T0 T1^T + gc T1 T1^T, dT0 = 2 ga Sigma3 T0 + gb Sigma3 T1,
  dT1 = gb Sigma3 T0 + 2 gc Sigma3 T1;
* J entries fx/tz, -fx u/tz, fy/tz, -fy v/tz with u = clamp(tx/tz) (zero
  derivative while clamped);
* Sigma3 = M M^T, M = R(q/|q|) diag(exp(s)); the rotation of a unit
  quaternion differentiated entry by entry, then the normalisation;
* mean2D = (fx tx/tz + cx, fy ty/tz + cy); t = R mu + t_cam;
* SH: d rgb_c / d sh_jc = Y_j(d) where unclamped, and the view direction
  d = (mu - c)/|mu - c| feeds back into mu;
* opacity = sigmoid(logit).
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh


def param_grads(proj, params, cam, acc):
    """Parameter gradients (dict of float64 arrays, same layout as params)."""
    n = proj["m"].shape[1]
    ok = proj["touched"]
    gm = np.where(ok, acc["m"], 0.0)
    gcon = np.where(ok, acc["conic"], 0.0)
    gop = np.where(ok, acc["opacity"], 0.0)
    grgb = np.where(ok, acc["rgb"], 0.0)
    R = np.asarray(cam["R"], np.float64)
    fx, fy = cam["fx"], cam["fy"]
    tx, ty = proj["t"][0], proj["t"][1]
    tz = np.where(ok, proj["t"][2], 1.0)

    # opacity
    o = proj["opacity"]
    g_logit = gop * o * (1 - o)

    # SH colour
    deg = proj["sh_degree"]
    nb = (deg + 1) ** 2
    live = np.where(proj["clamped"], 0.0, grgb)                # (3, N)
    shc = np.asarray(params["sh"], np.float64)
    g_sh = np.zeros((nb * 3, n))
    for c in range(3):
        g_sh[c::3] = proj["Y"] * live[c][None, :]
    dY = _sh.basis_grad(proj["dhat"], deg)                     # (nb, 3, N)
    g_d = np.zeros((3, n))
    for c in range(3):
        g_d += (shc[c::3][:nb][:, None, :] * dY).sum(0) * live[c][None, :]
    dh = proj["dhat"]
    g_dir = (g_d - dh * (dh * g_d).sum(0)[None, :]) / proj["dlen"][None, :]
    g_mu = g_dir.copy()

    # conic -> (a, b, c)
    a, b, c = proj["cov2"]
    D = np.where(ok, proj["det"], 1.0)
    gA, gB, gC = gcon
    gD = -(gA * c - gB * b + gC * a) / (D * D)
    ga = gC / D + gD * c
    gb = -gB / D - 2.0 * gD * b
    gc = gA / D + gD * a

    # Sigma2 = T Sigma3 T^T
    T = proj["T"]
    Sig = proj["Sig"]
    T0, T1 = T[0], T[1]                                         # (3, N)
    G_sig = (ga[None, None] * T0[:, None] * T0[None, :]
             + gb[None, None] * T0[:, None] * T1[None, :]
             + gc[None, None] * T1[:, None] * T1[None, :])
    S0 = np.einsum("ijn,jn->in", Sig, T0)
    S1 = np.einsum("ijn,jn->in", Sig, T1)
    gT0 = 2 * ga * S0 + gb * S1
    gT1 = gb * S0 + 2 * gc * S1
    gT = np.stack([gT0, gT1], 0)                                # (2, 3, N)

    # T = J R  ->  dJ = dT R^T
    gJ = np.einsum("ikn,jk->ijn", gT, R)
    u, v = proj["u"], proj["v"]
    g_t = np.zeros((3, n))
    g_t[2] += (gJ[0, 0] * (-fx / (tz * tz)) + gJ[1, 1] * (-fy / (tz * tz))
               + gJ[0, 2] * (fx * u / (tz * tz)) + gJ[1, 2] * (fy * v / (tz * tz)))
    gu = gJ[0, 2] * (-fx / tz)
    gv = gJ[1, 2] * (-fy / tz)
    free_u = (proj["xz"] >= -proj["limx"]) & (proj["xz"] <= proj["limx"])
    free_v = (proj["yz"] >= -proj["limy"]) & (proj["yz"] <= proj["limy"])
    g_t[0] += np.where(free_u, gu / tz, 0.0)
    g_t[2] += np.where(free_u, -gu * tx / (tz * tz), 0.0)
    g_t[1] += np.where(free_v, gv / tz, 0.0)
    g_t[2] += np.where(free_v, -gv * ty / (tz * tz), 0.0)

    # mean2D
    g_t[0] += gm[0] * fx / tz
    g_t[1] += gm[1] * fy / tz
    g_t[2] += -(gm[0] * fx * tx + gm[1] * fy * ty) / (tz * tz)
    g_mu += R.T @ g_t

    # Sigma3 = M M^T
    M = proj["M"]
    Gs = G_sig + np.transpose(G_sig, (1, 0, 2))
    gM = np.einsum("ikn,kjn->ijn", Gs, M)
    s = proj["s"]
    Rq = proj["Rq"]
    gR = gM * s[None, :, :]
    g_s = (gM * Rq).sum(0)
    g_ls = g_s * s

    # rotation of a unit quaternion
    w, x, y, z = proj["qn"]
    g = gR
    gw = 2 * (-z * g[0, 1] + y * g[0, 2] + z * g[1, 0] - x * g[1, 2] - y * g[2, 0] + x * g[2, 1])
    gx = 2 * (y * g[0, 1] + z * g[0, 2] + y * g[1, 0] - 2 * x * g[1, 1] - w * g[1, 2]
              + z * g[2, 0] + w * g[2, 1] - 2 * x * g[2, 2])
    gy = 2 * (-2 * y * g[0, 0] + x * g[0, 1] + w * g[0, 2] + x * g[1, 0] + z * g[1, 2]
              - w * g[2, 0] + z * g[2, 1] - 2 * y * g[2, 2])
    gz = 2 * (-2 * z * g[0, 0] - w * g[0, 1] + x * g[0, 2] + w * g[1, 0] - 2 * z * g[1, 1]
              + y * g[1, 2] + x * g[2, 0] + y * g[2, 1])
    gqn = np.stack([gw, gx, gy, gz], 0)
    qn = proj["qn"]
    g_q = (gqn - qn * (qn * gqn).sum(0)[None, :]) / proj["qnorm"][None, :]

    zero = ~ok
    return {
        "means": np.where(zero, 0.0, g_mu),
        "log_scales": np.where(zero, 0.0, g_ls),
        "quats": np.where(zero, 0.0, g_q),
        "opacity_logits": np.where(zero, 0.0, g_logit),
        "sh": np.where(zero, 0.0, g_sh),
    }
