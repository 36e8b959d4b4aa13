"""Forward projector (Alg. 1) and its exact adjoint back projector
(Eq. (2), Alg. 2), FP64.

Forward, for every view l:
  x_t   = R_l x              rotate the activity by theta_l
  mu_t  = R_l mu             rotate the attenuation map by theta_l
  mubar = Eq. (1) of mu_t
  w     = x_t * mubar
  v[:, :, l] = sum_j conv(w[:, j, :], p[:, :, j, l])

Back (the transpose of each step, composed in reverse order):
  g[i, j, k] = v[i, k, l] for every j        (transpose of the depth sum)
  u = conv^T(g)                              (with the replicate-padding fold)
  x += R_l^T (u * mubar)                     (mubar from the forward mu_t)

Inputs arrive in the C-ABI storage layout and are cast to float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry, rotation, attenuation, convolution


@dataclass
class Geometry:
    nx: int
    ny: int
    nz: int
    nview: int
    px: int
    pz: int
    dy: float = 1.0
    angles: object = None          # None -> theta_l = 2 pi l / nview
    rotation: str = "3pass"        # "3pass" (three 1-D shears) or "bilinear" (Sec. II-A)
    splits: list = field(init=False)

    def __post_init__(self):
        if self.nx != self.ny:
            raise ValueError("rotation about z needs nx == ny")
        if self.px % 2 == 0 or self.pz % 2 == 0:
            raise ValueError("PSF sizes must be odd")
        if self.rotation not in rotation.METHODS:
            raise ValueError("rotation must be '3pass' or 'bilinear'")
        self.splits = geometry.view_splits(self.nview, self.angles)


def rotate_view(f, geom: Geometry, l: int):
    return rotation.METHODS[geom.rotation][0](f, geom.splits[l])


def rotate_view_T(g, geom: Geometry, l: int):
    return rotation.METHODS[geom.rotation][1](g, geom.splits[l])


def vol_to_paper(x):             # [nz][ny][nx] -> x[i, j, k]
    return np.asarray(x, dtype=np.float64).transpose(2, 1, 0)


def vol_from_paper(x):           # x[i, j, k] -> [nz][ny][nx]
    return np.ascontiguousarray(np.asarray(x).transpose(2, 1, 0))


def psf_view_paper(psf, l):      # [nview][ny][pz][px] -> p[a, b, j] for view l
    return np.asarray(psf[l], dtype=np.float64).transpose(2, 1, 0)


def mubar_view(mu_p, geom: Geometry, l: int):
    """Eq. (1) for view l; mu_p in paper order (nx, ny, nz)."""
    return attenuation.mubar(rotate_view(mu_p, geom, l), geom.dy)


def forward(x, mu, psf, geom: Geometry, views=None, conv="direct") -> np.ndarray:
    """Alg. 1.  x, mu: [nz][ny][nx]; psf: [nview][ny][pz][px].
    Returns v as [nview][nz][nx] (rows for views not in ``views`` are 0)."""
    xp = vol_to_paper(x)
    mup = vol_to_paper(mu)
    v = np.zeros((geom.nview, geom.nz, geom.nx))
    for l in (range(geom.nview) if views is None else views):
        w = rotate_view(xp, geom, l) * mubar_view(mup, geom, l)
        p = psf_view_paper(psf, l)
        if conv == "direct":
            v2 = convolution.conv_planes(w, p).sum(axis=1)           # depth sum
        else:
            v2 = convolution.conv_sum_fft(w, p)
        v[l] = v2.T                                                  # (nx, nz) -> [nz][nx]
    return v


def back(v, mu, psf, geom: Geometry, views=None, conv="direct") -> np.ndarray:
    """Alg. 2 (exact transpose of ``forward``).  v: [nview][nz][nx].
    Returns x as [nz][ny][nx]."""
    v = np.asarray(v, dtype=np.float64)
    mup = vol_to_paper(mu)
    x = np.zeros((geom.nx, geom.ny, geom.nz))
    for l in (range(geom.nview) if views is None else views):
        g2 = v[l].T                                                  # (nx, nz)
        p = psf_view_paper(psf, l)
        if conv == "direct":
            g = np.repeat(g2[:, None, :], geom.ny, axis=1)          # transpose of depth sum
            u = convolution.conv_planes_T(g, p)
        else:
            u = convolution.conv_planes_T_fft(g2, p)
        x += rotate_view_T(u * mubar_view(mup, geom, l), geom, l)
    return vol_from_paper(x)
