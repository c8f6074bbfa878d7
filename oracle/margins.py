"""Degeneracy margins of an oracle ray record (test infrastructure).

A ray is epsilon-degenerate when FP32 rounding may legitimately change its
cell sequence or step count: near-tied exits (readings of the tie rule,
Sec. 3.1), near-zero segments, exits next to tmax, or a transmittance next to
the early-stop threshold (Sec. 3.2).  Their colours still must match; only
their sequences are excluded from exact comparison.
"""
from __future__ import annotations

import math

# The GPU re-decides exits whose FP32 gap is within 1e-6 max(1,|t|) in FP64;
# FP32 crossing errors are ~1e-7 per unit t, so an FP64 gap of 4x the window
# is decided identically by both sides.
EPS_SEQ = 4e-6      # FP64 gap (relative to max(1,|t|)) below which a step is a near tie
EPS_DELTA = 1e-7    # segments shorter than this are crossings next to a cell edge
EPS_TMAX = 1e-5     # exits this close to tmax may end the ray one step earlier or later
EPS_TSTOP = 1e-4    # relative margin of T_k to t_stop (FP32 T carries ~K*1e-7)


def degenerate(rec, t_stop=1e-4, tmax=None) -> bool:
    if rec is None:
        return False
    if rec.start_gap < 1e-9:
        return True
    for k in range(rec.K):
        t = rec.exit[k]
        if rec.gaps[k] < EPS_SEQ * max(1.0, abs(t) if math.isfinite(t) else 1.0):
            return True
        if rec.delta[k] < EPS_DELTA and k + 1 < rec.K:
            return True
        if tmax is not None and math.isfinite(t) and abs(t - tmax) < EPS_TMAX:
            return True
        Tk = rec.T_before[k + 1] if k + 1 < rec.K else rec.T
        if t_stop > 0 and abs(Tk - t_stop) < EPS_TSTOP * t_stop:
            return True
    return False
