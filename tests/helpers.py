"""Shared helpers of the GPU parity tests."""
from __future__ import annotations

import numpy as np

from oracle.margins import degenerate, stop_degenerate  # noqa: F401


def f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
