"""Spherical-harmonic cell colour (Sec. 3.3, the appearance model that the
octahedral textures replace), FP64.  Test infrastructure only.

c(w) = sum_{l<=3} sum_{m=-l..l} k_lm Y_l^m(w), with the real, orthonormal
spherical harmonics

    Y_l^0  = N_l0 P_l(cos theta)
    Y_l^m  = sqrt(2) N_lm P_l^m(cos theta) cos(m phi)      (m > 0)
    Y_l^-m = sqrt(2) N_lm P_l^m(cos theta) sin(m phi)      (m > 0)
    N_lm   = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)

theta the polar angle from +z, phi = atan2(y, x), and P_l^m the associated
Legendre function without the Condon-Shortley phase.  Coefficient i =
l^2 + l + m holds k_lm (RGB): 16 per channel, 48 values per cell, stored
[N, 48] as (coefficient, channel).  Readings: the colour is the sum itself
(the paper's equation has no activation), evaluated at the ray direction.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import lpmv

L_MAX = 3
N_COEFF = (L_MAX + 1) ** 2


def real_sh(d) -> np.ndarray:
    """The 16 real SH values Y_i(d), i = l^2 + l + m, at a direction d (normalised here)."""
    d = np.asarray(d, np.float64)
    x, y, z = d / np.linalg.norm(d)
    ct = max(-1.0, min(1.0, z))
    phi = math.atan2(y, x)
    out = np.zeros(N_COEFF)
    for l in range(L_MAX + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am)
                             / math.factorial(l + am))
            p = (-1) ** am * lpmv(am, l, ct)          # remove the Condon-Shortley phase
            if m == 0:
                v = norm * p
            elif m > 0:
                v = math.sqrt(2.0) * norm * p * math.cos(m * phi)
            else:
                v = math.sqrt(2.0) * norm * p * math.sin(am * phi)
            out[l * l + l + m] = v
    return out


def sh_colour(coeffs_cell, d) -> np.ndarray:
    """RGB of one cell's [48] coefficients (coefficient-major) at direction d."""
    k = np.asarray(coeffs_cell, np.float64).reshape(N_COEFF, 3)
    return real_sh(d) @ k
