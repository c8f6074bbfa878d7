"""Shared helpers of the GPU parity tests."""
from __future__ import annotations

import numpy as np

from oracle.margins import degenerate, stop_degenerate  # noqa: F401


def f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))


def seq_hash(cells) -> int:
    """64-bit digest of a visited-cell sequence (cell ids in the scene's own numbering)."""
    import hashlib
    b = np.ascontiguousarray(np.asarray(cells, dtype="<i8")).tobytes()
    return int.from_bytes(hashlib.blake2b(b, digest_size=8).digest(), "little")


def scene_fingerprint(scene) -> str:
    """Digest of a scene's float32 sites, densities and texels (the oracle's inputs)."""
    import hashlib
    h = hashlib.blake2b(digest_size=16)
    for a in (scene.sites, scene.density, scene.texels):
        h.update(np.ascontiguousarray(a, np.float32).tobytes())
    return h.hexdigest()
