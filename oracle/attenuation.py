"""Accumulated attenuation factor, Eq. (1) (Sec. II-A).

With the rotated attenuation map mu_t[i, j, k] and the plane j = ny-1 (0-based)
nearest the detector,

  mubar[i, j, k] = exp(-dy * (mu_t[i, j, k] / 2 + sum_{s=j+1}^{ny-1} mu_t[i, s, k]))

i.e. half a voxel of self-attenuation plus everything between the voxel and
the detector.  dy is the voxel size along y in the length unit of 1/mu.
"""
from __future__ import annotations

import numpy as np


def mubar(mu_t: np.ndarray, dy: float) -> np.ndarray:
    """mu_t has shape (nx, ny, nz) in paper order; returns the same shape."""
    mu_t = np.asarray(mu_t, dtype=np.float64)
    ny = mu_t.shape[1]
    out = np.empty_like(mu_t)
    beyond = np.zeros((mu_t.shape[0], mu_t.shape[2]))   # sum over s > j
    for j in range(ny - 1, -1, -1):
        out[:, j, :] = np.exp(-dy * (0.5 * mu_t[:, j, :] + beyond))
        beyond = beyond + mu_t[:, j, :]
    return out
