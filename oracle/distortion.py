"""Distortion loss of one ray (Sec. 5.3, eq. distortion-loss), FP64.

Test infrastructure only.  With the ray's segments [t_k, t_{k+1}] and
compositing weights w_k, depth is mapped to s(t) = 1 - 1/(1+t) (written
t/(1+t)), and with sbar_k = (s(t_k) + s(t_{k+1}))/2, ds_k = s(t_{k+1}) - s(t_k):

    L_dist = sum_{k,l} w_k w_l |sbar_k - sbar_l| + (1/3) sum_k w_k^2 ds_k

evaluated here as written, a double sum over all pairs.  The partial
derivatives are those of this expression with the weights and interval
ends as independent variables; ``adjoint`` chains them through w_k and the
crossing parameters.
"""
from __future__ import annotations

import numpy as np


def s_of_t(t):
    t = np.asarray(t, np.float64)
    return t / (1.0 + t)


def ds_dt(t):
    t = np.asarray(t, np.float64)
    return 1.0 / ((1.0 + t) * (1.0 + t))


def distortion(w, t0, t1) -> float:
    """L_dist for weights w_k on intervals [t0_k, t1_k]."""
    w = np.asarray(w, np.float64)
    s0, s1 = s_of_t(t0), s_of_t(t1)
    sb = 0.5 * (s0 + s1)
    pair = 0.0
    for k in range(len(w)):
        for l in range(len(w)):
            pair += w[k] * w[l] * abs(sb[k] - sb[l])
    return float(pair + np.sum(w * w * (s1 - s0)) / 3.0)


def distortion_partials(w, t0, t1):
    """(dL/dw_k, dL/dt0_k, dL/dt1_k) of ``distortion`` (|x| differentiated as sign x, sign 0 = 0)."""
    w = np.asarray(w, np.float64)
    t0 = np.asarray(t0, np.float64)
    t1 = np.asarray(t1, np.float64)
    s0, s1 = s_of_t(t0), s_of_t(t1)
    sb = 0.5 * (s0 + s1)
    K = len(w)
    gw = np.zeros(K)
    gsb = np.zeros(K)
    for k in range(K):
        for l in range(K):
            gw[k] += 2.0 * w[l] * abs(sb[k] - sb[l])
            gsb[k] += 2.0 * w[k] * w[l] * np.sign(sb[k] - sb[l])
    gw += 2.0 / 3.0 * w * (s1 - s0)
    gds = w * w / 3.0
    g0 = (0.5 * gsb - gds) * ds_dt(t0)
    g1 = (0.5 * gsb + gds) * ds_dt(t1)
    return gw, g0, g1
