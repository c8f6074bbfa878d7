"""Shared helpers of the GPU parity tests (seeded inputs, oracle margins)."""
from __future__ import annotations

import math

import numpy as np

EPS_SEQ = 1e-5      # FP64 gap (relative to max(1,|t|)) below which a step is a near tie
EPS_DELTA = 1e-5    # segments shorter than this are near-degenerate crossings
EPS_TSTOP = 1e-4    # relative margin of T_k to t_stop (FP32 T carries ~K*1e-7)


def degenerate(rec, t_stop=1e-4, tmax=None) -> bool:
    """True when FP32 rounding may legitimately change the cell sequence or the
    step count of this ray (readings of the near-tie and stop rules)."""
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
        if tmax is not None and math.isfinite(t) and abs(t - tmax) < 1e-5:
            return True
        Tk = rec.T_before[k + 1] if k + 1 < rec.K else rec.T
        if t_stop > 0 and abs(Tk - t_stop) < EPS_TSTOP * t_stop:
            return True
    return False


def f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
