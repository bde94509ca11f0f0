"""Digests of the integer state of a run (test infrastructure).

The same function summarises the oracle's state (when the stored values
are written) and the GPU library's state (when a test compares against
them): per patch, the per-bucket counts, a SHA-256 over every bucket's bin
grid dimensions and histogram, and a SHA-256 of the patch's particle
multiset in canonical order (rows sorted lexicographically over all ten
integer columns).  Both sides expose the same readouts (``counts``,
``tile_dims``, ``tiles``, ``particles``), so equal digests mean bit-equal
integer state.  No arithmetic of the method is done here.
"""
from __future__ import annotations

import hashlib

import numpy as np


def canonical(P: np.ndarray) -> np.ndarray:
    P = np.ascontiguousarray(P, dtype=np.int64).reshape(-1, 10)
    if P.shape[0] == 0:
        return P
    return P[np.lexsort(P.T[::-1])]


def _sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
    return h.hexdigest()


def state_digest(ocean, n_patches: int, n_buckets: int) -> dict:
    """Counts (live, injected, emitted, subdivided, died per bucket), the
    histogram digest and the particle-multiset digest of every patch."""
    P = np.asarray(ocean.particles(), dtype=np.int64).reshape(-1, 10)
    order = np.argsort(P[:, 0], kind="stable")
    P = P[order]
    starts = np.searchsorted(P[:, 0], np.arange(n_patches + 1))
    out = {"n_particles": int(P.shape[0]), "counts": [], "hist_sha": [], "particles_sha": []}
    for p in range(n_patches):
        c = np.asarray(ocean.counts(p), dtype=np.int64)[:, :5]
        out["counts"].append(c.tolist())
        parts = []
        for b in range(n_buckets):
            parts.append(np.asarray(ocean.tile_dims(p, b), dtype=np.int64))
            parts.append(np.asarray(ocean.tiles(p, b), dtype=np.int64).ravel())
        out["hist_sha"].append(_sha(*parts))
        out["particles_sha"].append(_sha(canonical(P[starts[p]:starts[p + 1]])))
    return out
