"""Degeneracy margins of an oracle ray record (test infrastructure).

A ray is epsilon-degenerate when FP32 rounding may legitimately change its
cell sequence or step count: near-tied exits (readings of the tie rule,
Sec. 3.1), near-zero segments, exits next to tmax, or a transmittance next to
the early-stop threshold (Sec. 3.2).  Their colours still must match; only
their sequences are excluded from exact comparison.
"""
from __future__ import annotations

import math

# The GPU re-decides exits whose FP32 gap is within W = 1e-6 max(1,|t|) in
# FP64.  With FP32 crossing errors E ~ 1e-7 per unit t (up to ~1e-6 for
# grazing faces), every decision whose true gap exceeds E comes out the same,
# and so does every one whose FP32 gap falls inside W; a margin of 2W covers
# the remaining grazing cases.
EPS_SEQ = 2e-6      # FP64 gap (relative to max(1,|t|)) below which a step is a near tie
EPS_DELTA = 1e-7    # segments shorter than this are crossings next to a cell edge
EPS_TMAX = 1e-5     # exits this close to tmax may end the ray one step earlier or later
EPS_TSTOP = 1e-4    # relative margin of T_k to t_stop (FP32 T carries ~K*1e-7)


def stop_degenerate(rec, t_stop=1e-4) -> bool:
    """T lands next to t_stop: FP32 may stop one segment earlier or later, which
    changes the colour by up to t_stop (all other degeneracies change it by the
    length of a near-zero segment only)."""
    if rec is None or t_stop <= 0:
        return False
    for k in range(rec.K):
        Tk = rec.T_before[k + 1] if k + 1 < rec.K else rec.T
        if abs(Tk - t_stop) < EPS_TSTOP * t_stop:
            return True
    return False


def degenerate(rec, t_stop=1e-4, tmax=None) -> bool:
    """Any step whose decision FP32 may take differently (sequence comparison)."""
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
    return stop_degenerate(rec, t_stop)
