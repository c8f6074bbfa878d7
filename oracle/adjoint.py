"""Analytic FP64 gradient of the oracle's per-ray render.

The paper optimises site positions, density parameters and both texture maps
with Adam (Sec. 5.5) but prints no adjoint; this is the plain chain rule of
the forward model in ``render`` (Sec. 3.2 compositing, Sec. 3.1 bisector
crossings), written term by term:

Compositing.  With tau_k = sigma_k delta_k, T_k = exp(-sum_{j<k} tau_j) and
w_k = T_k - T_{k+1}:
    dC/dtau_k       = T_{k+1} c_k - sum_{j>k} w_j c_j
    dT_final/dtau_k = -T_final
    dC/dc_k         = w_k
so for L = g . C + g_T T_final:
    dL/dtau_k = g . (T_{k+1} c_k - S_k) - g_T T_final,   S_k = sum_{j>k} w_j c_j
    dL/dsigma_{i_k} += dL/dtau_k * delta_k
    dL/dtexel_q     += w_k * b_q * g      (b_q: bilinear weight of tap q)

Segment ends.  delta_k = t_exit - t_entry (when positive).  Its exit end is
the bisector crossing out of i_k unless clipped at tmax; its entry end is the
crossing that last advanced t (none for the first segment).  Each end moves
with the sites: for the bisector of (a, b) crossed at t, with n = p_b - p_a,
beta = n . w and x = o + t w,
    dt/dp_b = (p_b - x) / beta,   dt/dp_a = (x - p_a) / beta.
Stopping decisions, the start cell and the cell sequence are piecewise
constant: no gradient flows through tmax, early termination or max_steps.

Under sigma = exp(rho) (Sec. 5.4) the caller's autograd multiplies by sigma,
giving dL/drho = dL/dalpha (1 - alpha) ln(1/(1 - alpha)) per segment.

Full appearance model (Sec. 5.2), c = sigmoid(l), l = T_vi(oct(d)) + T_vd(oct(-w)):
    dL/dl           = w_k g * c (1 - c)                       (per channel)
    dL/dtexel_q     += b_q dL/dl   for the taps of both maps
    dL/dd           = sum_ch dL/dl_ch (dl_ch/du grad u + dl_ch/dv grad v)
with (u, v) the octahedral coordinates of d and the taps held fixed.  With
d = (x - p_i)/r, r = |x - p_i|, the hit point x = o + t_hit w gives
    dL/dx = (I - d d^T) dL/dd / r,   dL/dp_i -= dL/dx,   dL/dt_hit = dL/dx . w,
and t_hit moves with the crossing that defines it (the entry face, or the
start cell's exit face), through the same dt/dp as above.

Distortion loss (Sec. 5.3), L += g_dist L_dist, with G_k = dL_dist/dw_k and
the interval-end partials from ``distortion.distortion_partials``: since
w_k = T_k - T_{k+1} and T_k = exp(-sum_{j<k} tau_j),
    dL_dist/dtau_j = G_j T_{j+1} - sum_{k>j} G_k w_k,
and the interval ends t_k (entry) and t_k + delta_k (exit, unless clipped
at tmax) move with their crossings like the segment ends above.
"""
from __future__ import annotations

import numpy as np

from . import appearance, distortion, walk


def face_dt_dsites(sites, a, b, o, w, t):
    """(dt/dp_a, dt/dp_b) for the bisector of sites a, b crossed at parameter t."""
    p = walk.as64(sites)
    o = walk.as64(o)
    w = walk.as64(w)
    n = p[b] - p[a]
    beta = float(n @ w)
    x = o + t * w
    return (x - p[a]) / beta, (p[b] - x) / beta


def grad_ray(sites, density, texels, o, w, tmax, rec, g_rgb, g_T, g_sites, g_density,
             g_texels, g_dist=0.0):
    """Accumulate dL/d(sites, density, texels) of one ray into the dense arrays, for
    L = g_rgb . C + g_T T_final + g_dist L_dist.

    ``rec`` is the oracle forward record of this ray (render.render_ray).
    """
    sig = walk.as64(density)
    g = np.asarray(g_rgb, np.float64)
    gT = float(g_T)
    w = walk.as64(w)
    res = texels.shape[1]
    C = np.asarray(rec.rgb, np.float64)
    Tf = float(rec.T)
    K = rec.K
    app = getattr(rec, "appearance", 0)
    if app == 1:
        res = texels.shape[2]
        taps = appearance.bilinear_weights(-w, res)
    else:
        taps = appearance.bilinear_weights(w, res)
    p64 = walk.as64(sites)
    o64 = walk.as64(o)
    gdist = float(g_dist)
    if gdist != 0.0:
        t_ends = [a + b for a, b in zip(rec.t_in, rec.delta)]
        Gw, Gt0, Gt1 = distortion.distortion_partials(rec.weight, rec.t_in, t_ends)
        Gw_suffix = np.zeros(K + 1)          # sum_{k>=j} G_k w_k
        for k in range(K - 1, -1, -1):
            Gw_suffix[k] = Gw_suffix[k + 1] + Gw[k] * rec.weight[k]
    else:
        Gw = Gt0 = Gt1 = np.zeros(K)
        Gw_suffix = np.zeros(K + 1)
    # suffix sums S_k = C - sum_{j<=k} w_j c_j
    prefix = np.zeros(3)
    entry_face = None  # (a, b, t) of the crossing that set the current entry
    for k in range(K):
        i = rec.cells[k]
        wk = rec.weight[k]
        ck = rec.color[k]
        prefix = prefix + wk * ck
        S = C - prefix
        T_next = rec.T_before[k] * np.exp(-sig[i] * rec.delta[k])
        dtau = float(g @ (T_next * ck - S)) - gT * Tf
        dtau += gdist * (Gw[k] * T_next - Gw_suffix[k + 1])
        g_density[i] += dtau * rec.delta[k]
        if not rec.skipped[k] and app == 0:
            for r, col, bw in taps:
                g_texels[i, r, col, :3] += wk * bw * g
        if not rec.skipped[k] and app == 1:
            gl = wk * g * ck * (1.0 - ck)
            d_surf = rec.surf_dir[k]
            for r, col, bw in appearance.bilinear_weights(d_surf, res):
                g_texels[i, 0, r, col, :3] += bw * gl
            for r, col, bw in taps:
                g_texels[i, 1, r, col, :3] += bw * gl
            x = o64 + rec.t_hit[k] * w
            rr = float(np.linalg.norm(x - p64[i]))
            if rr > 0.0:
                dcu, dcv = appearance.lookup_grad_uv(texels[i, 0], d_surf)
                ju, jv = appearance.octahedral_jacobian(d_surf)
                gd = float(gl @ dcu) * ju + float(gl @ dcv) * jv
                gx = (gd - d_surf * float(d_surf @ gd)) / rr
                g_sites[i] -= gx
                dldt = float(gx @ w)
                face = None
                if k == 0:
                    if rec.exit[0] < tmax and rec.nxt[0] >= 0:
                        face = (i, rec.nxt[0], rec.exit[0])
                elif entry_face is not None:
                    face = entry_face
                if face is not None:
                    a, b, t = face
                    da, db = face_dt_dsites(sites, a, b, o, w, t)
                    g_sites[a] += dldt * da
                    g_sites[b] += dldt * db
        if rec.delta[k] > 0.0:
            ddelta = sig[i] * dtau
            if entry_face is not None:
                a, b, t = entry_face
                da, db = face_dt_dsites(sites, a, b, o, w, t)
                c_in = gdist * Gt0[k] - ddelta
                g_sites[a] += c_in * da
                g_sites[b] += c_in * db
            ex = rec.exit[k]
            if ex < tmax and rec.nxt[k] >= 0:
                da, db = face_dt_dsites(sites, i, rec.nxt[k], o, w, ex)
                c_out = ddelta + gdist * Gt1[k]
                g_sites[i] += c_out * da
                g_sites[rec.nxt[k]] += c_out * db
                entry_face = (i, rec.nxt[k], ex)


def grad_rays(sites, density, texels, origins, dirs, tmax, recs, g_rgb, g_T, g_dist=None):
    """Dense FP64 gradients summed over rays: (g_sites[N,3], g_density[N], g_texels
    shaped like texels: [N,R,R,4], or [N,2,R,R,4] for the full appearance model)."""
    N = len(sites)
    gs = np.zeros((N, 3))
    gd = np.zeros(N)
    gt = np.zeros(np.shape(texels))
    tm = np.broadcast_to(np.asarray(tmax, np.float64), (len(origins),))
    for r, rec in enumerate(recs):
        if rec is None:
            continue
        grad_ray(sites, density, texels, origins[r], dirs[r], tm[r], rec, g_rgb[r], g_T[r],
                 gs, gd, gt, 0.0 if g_dist is None else g_dist[r])
    return gs, gd, gt
