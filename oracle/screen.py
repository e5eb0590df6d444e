"""Conjunction screening oracle: TEST INFRASTRUCTURE ONLY.

The definition written out by brute force (every pair at every sample time),
for checking the library's screening kernel; only the tests may call it.

At each sample time k, a pair of satellites i < j is an event when both
points are valid (three finite position components; code 0 or 6 when codes
are given) and
    d2 = (dx*dx + dy*dy) + dz*dz < D*D,   dx = x_j - x_i, ...
in float64 from the stored positions (numpy evaluates the expression as
written, with no fused multiply-add); the event carries d = sqrt(d2).
"""
from __future__ import annotations

import numpy as np


def screen_step(r_k: np.ndarray, valid: np.ndarray, D: float, rows: int = 1024):
    """Events at one time: r_k float [3, n]; returns (i, j, d) arrays, i < j,
    sorted by (i, j).  Rows of the pair matrix are taken in blocks of `rows`
    (only to bound memory)."""
    x = np.asarray(r_k, dtype=np.float64)
    idx = np.flatnonzero(valid)
    p = x[:, idx]
    m = idx.size
    D2 = D * D
    out_i, out_j, out_d = [], [], []
    for a0 in range(0, m, rows):
        a1 = min(m, a0 + rows)
        dx = p[0][None, :] - p[0][a0:a1, None]
        dy = p[1][None, :] - p[1][a0:a1, None]
        dz = p[2][None, :] - p[2][a0:a1, None]
        d2 = (dx * dx + dy * dy) + dz * dz
        a, b = np.nonzero(d2 < D2)
        a = a + a0
        keep = b > a
        a, b = a[keep], b[keep]
        out_i.append(idx[a]); out_j.append(idx[b]); out_d.append(np.sqrt(d2[a - a0, b]))
    if not out_i:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    i, j, d = np.concatenate(out_i), np.concatenate(out_j), np.concatenate(out_d)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    order = np.lexsort((hi, lo))
    return lo[order], hi[order], d[order]


def valid_points(r: np.ndarray, err=None):
    """r [3, n, T] -> bool [n, T]."""
    ok = np.all(np.isfinite(r), axis=0)
    if err is not None:
        ok &= (err == 0) | (err == 6)
    return ok


def screen(r: np.ndarray, D: float, err=None, times=None):
    """Events over the sample times `times` (default all): int64 [m, 3] of
    (i, j, k) sorted by (k, i, j) and float64 [m] distances."""
    r = np.asarray(r)
    ok = valid_points(r, err)
    T = r.shape[2]
    ks = range(T) if times is None else times
    ev, dd = [], []
    for k in ks:
        i, j, d = screen_step(r[:, :, k], ok[:, k], D)
        ev.append(np.stack([i, j, np.full(i.size, k, dtype=np.int64)], axis=1))
        dd.append(d)
    if not ev:
        return np.zeros((0, 3), np.int64), np.zeros(0)
    return np.concatenate(ev), np.concatenate(dd)
