"""Explicit system matrices for tiny problems (Sec. III-A-3: the paper forms
the (nx nz nview) x (nx ny nz) matrix of the forward projector for an
8x8x6 volume with 7 views and compares its transpose with the back
projector).

A column of A is the forward projection of a unit voxel; a column of the
back-projector matrix B is the back projection of a unit detector bin.  Both
use the storage layout order (C order of [nz][ny][nx] and [nview][nz][nx]).
"""
from __future__ import annotations

import numpy as np

from .projector import forward, back


def forward_matrix(mu, psf, geom, conv="direct") -> np.ndarray:
    n_in = geom.nx * geom.ny * geom.nz
    n_out = geom.nview * geom.nz * geom.nx
    A = np.zeros((n_out, n_in))
    e = np.zeros(n_in)
    for c in range(n_in):
        e[:] = 0.0
        e[c] = 1.0
        A[:, c] = forward(e.reshape(geom.nz, geom.ny, geom.nx), mu, psf, geom, conv=conv).ravel()
    return A


def back_matrix(mu, psf, geom, conv="direct") -> np.ndarray:
    n_in = geom.nview * geom.nz * geom.nx
    n_out = geom.nx * geom.ny * geom.nz
    B = np.zeros((n_out, n_in))
    e = np.zeros(n_in)
    for c in range(n_in):
        e[:] = 0.0
        e[c] = 1.0
        B[:, c] = back(e.reshape(geom.nview, geom.nz, geom.nx), mu, psf, geom, conv=conv).ravel()
    return B
