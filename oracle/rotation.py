"""Image rotation about the z axis by theta_l and its exact transpose
(Sec. II-A; the adjoint of interpolation is needed because the transpose of
a discrete rotation is not the rotation by -theta).

All functions act on arrays f[i, j, ...] (i along x, j along y; any trailing
axes, e.g. k, are carried along).  Grid is n x n with centre c = (n-1)/2.

Forward (gather) form, for one view with split (m, phi):
  P_m   exact quarter turn:  out(p) = in(R(m pi/2)^-1 (p - c) + c)
  pass1 out[i, j] = L(in[:, j], +t (j - c))[i]
  pass2 out[i, j] = L(in[i, :], -s (i - c))[j]
  pass3 = pass1
with L(row, d)[i] = (1 - f) row[q] + f row[q + 1], q = floor(i + d),
f = i + d - q and row[.] = 0 outside [0, n) (zero-padding boundary).
Rotation = pass3 . pass2 . pass1 . P_m.

The transposes below are written as the literal adjoint of each gather
(scatter-add of the same weights), not as a rotation by -theta.

The 2-D bilinear alternative (also Sec. II-A) is at the end of the file.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- quarter turns

def quarter_turn_source(n: int, m: int):
    """Index arrays (si, sj) with P_m f = f[si, sj] (gather).

    Derived from out(p) = in(R^-1 (p - c) + c) with R = R(m * 90 deg),
    R(a) = [[cos a, -sin a], [sin a, cos a]] acting on (i, j):
      m=1: (di, dj) -> ( dj, -di)   m=2: -> (-di, -dj)   m=3: -> (-dj, di)
    evaluated in integers (c = (n-1)/2 so c + d is an integer)."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m %= 4
    if m == 0:
        return i, j
    if m == 1:
        return j, n - 1 - i
    if m == 2:
        return n - 1 - i, n - 1 - j
    return n - 1 - j, i


def quarter_turn(f: np.ndarray, m: int) -> np.ndarray:
    n = f.shape[0]
    assert f.shape[1] == n
    si, sj = quarter_turn_source(n, m)
    return f[si, sj]


def quarter_turn_T(g: np.ndarray, m: int) -> np.ndarray:
    """Transpose of quarter_turn: scatter out-values back to their sources."""
    n = g.shape[0]
    si, sj = quarter_turn_source(n, m)
    out = np.zeros_like(g)
    out[si, sj] = g          # a permutation: every source is hit exactly once
    return out


# ---------------------------------------------------------------- 1-D shears

def _lerp_taps(n: int, shifts: np.ndarray):
    """For each line index r and sample i: (q, f) with pos = i + shifts[r],
    q = floor(pos), f = pos - q.  Returns q, f of shape (n_lines, n)."""
    pos = np.arange(n)[None, :] + np.asarray(shifts, dtype=np.float64)[:, None]
    q = np.floor(pos)
    return q.astype(np.int64), pos - q


def shear_lines(f: np.ndarray, shifts: np.ndarray) -> np.ndarray:
    """Gather shear along axis 0: out[i, r, ...] = L(f[:, r, ...], shifts[r])[i]."""
    n = f.shape[0]
    q, w = _lerp_taps(n, shifts)             # (lines, n)
    out = np.zeros(f.shape, dtype=np.float64)
    for r in range(f.shape[1]):
        for tap, wt in ((q[r], 1.0 - w[r]), (q[r] + 1, w[r])):
            ok = (tap >= 0) & (tap < n)
            out[ok, r, ...] += wt[ok].reshape((-1,) + (1,) * (f.ndim - 2)) * f[tap[ok], r, ...]
    return out


def shear_lines_T(g: np.ndarray, shifts: np.ndarray) -> np.ndarray:
    """Transpose of shear_lines: every output sample scatters its two
    weights back onto the input samples it read."""
    n = g.shape[0]
    q, w = _lerp_taps(n, shifts)
    out = np.zeros(g.shape, dtype=np.float64)
    for r in range(g.shape[1]):
        for tap, wt in ((q[r], 1.0 - w[r]), (q[r] + 1, w[r])):
            ok = (tap >= 0) & (tap < n)
            np.add.at(out[:, r, ...], tap[ok],
                      wt[ok].reshape((-1,) + (1,) * (g.ndim - 2)) * g[ok, r, ...])
    return out


def _pass_shifts(n: int, split):
    c = (n - 1) / 2.0
    idx = np.arange(n) - c
    return split.t * idx, -split.s * idx      # pass 1/3 (per j), pass 2 (per i)


def rotate(f: np.ndarray, split) -> np.ndarray:
    """Rotate f[i, j, ...] by theta = m*90deg + phi (forward, gather)."""
    n = f.shape[0]
    d13, d2 = _pass_shifts(n, split)
    g = quarter_turn(np.asarray(f, dtype=np.float64), split.m)
    g = shear_lines(g, d13)                                        # pass 1, along i
    g = np.swapaxes(shear_lines(np.swapaxes(g, 0, 1), d2), 0, 1)   # pass 2, along j
    g = shear_lines(g, d13)                                        # pass 3, along i
    return g


def rotate_T(g: np.ndarray, split) -> np.ndarray:
    """Exact transpose of rotate: pass3^T, pass2^T, pass1^T, then P_m^T."""
    n = g.shape[0]
    d13, d2 = _pass_shifts(n, split)
    h = shear_lines_T(np.asarray(g, dtype=np.float64), d13)
    h = np.swapaxes(shear_lines_T(np.swapaxes(h, 0, 1), d2), 0, 1)
    h = shear_lines_T(h, d13)
    return quarter_turn_T(h, split.m)


# ---------------------------------------------------------------- 2-D bilinear
# Sec. II-A implements, beside the 3-pass shears, rotation by 2-D bilinear
# interpolation with zero padding.  Reading: the same exact quarter turn P_m
# first, then the gather out(p) = sum over the four grid neighbours q of
# s(p) = R(phi)^-1 (p - c) + c of the bilinear weights times (P_m f)(q), with
# (P_m f) = 0 outside the grid.  P_m is a symmetry of the grid, so this is
# bilinear interpolation of f at R(theta)^-1 (p - c) + c.

def bilinear_taps(n: int, phi: float):
    """Source position s(p) of every output pixel p = (i, j) for the residual
    angle phi: integer parts (qi, qj) and fractions (fi, fj), each (n, n)."""
    c = (n - 1) / 2.0
    u, v = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    co, sn = math.cos(phi), math.sin(phi)
    si = c + co * u + sn * v               # R(phi)^-1 = [[cos, sin], [-sin, cos]]
    sj = c - sn * u + co * v
    qi, qj = np.floor(si), np.floor(sj)
    return qi.astype(np.int64), qj.astype(np.int64), si - qi, sj - qj


def _bilinear_corners(n: int, phi: float):
    qi, qj, fi, fj = bilinear_taps(n, phi)
    for di, wi in ((0, 1.0 - fi), (1, fi)):
        for dj, wj in ((0, 1.0 - fj), (1, fj)):
            a, b = qi + di, qj + dj
            ok = (a >= 0) & (a < n) & (b >= 0) & (b < n)
            yield a, b, wi * wj, ok


def rotate_bilinear(f: np.ndarray, split) -> np.ndarray:
    """Rotate f[i, j, ...] by theta = m*90deg + phi with bilinear interpolation."""
    n = f.shape[0]
    g = quarter_turn(np.asarray(f, dtype=np.float64), split.m)
    out = np.zeros(g.shape, dtype=np.float64)
    trail = (1,) * (g.ndim - 2)
    for a, b, w, ok in _bilinear_corners(n, split.phi):
        out[ok] += w[ok].reshape((-1,) + trail) * g[a[ok], b[ok]]
    return out


def rotate_bilinear_T(g: np.ndarray, split) -> np.ndarray:
    """Exact transpose of rotate_bilinear: every output pixel scatters its
    four weights back onto the samples it read, then P_m^T."""
    n = g.shape[0]
    g = np.asarray(g, dtype=np.float64)
    h = np.zeros(g.shape, dtype=np.float64)
    trail = (1,) * (g.ndim - 2)
    for a, b, w, ok in _bilinear_corners(n, split.phi):
        np.add.at(h, (a[ok], b[ok]), w[ok].reshape((-1,) + trail) * g[ok])
    return quarter_turn_T(h, split.m)


METHODS = {"3pass": (rotate, rotate_T), "bilinear": (rotate_bilinear, rotate_bilinear_T)}


def shear_shift_rows(n: int, split):
    """(pass-1/3 shifts per j, pass-2 shifts per i); exposed for tests."""
    return _pass_shifts(n, split)


__all__ = ["quarter_turn", "quarter_turn_T", "quarter_turn_source", "shear_lines",
           "shear_lines_T", "rotate", "rotate_T", "bilinear_taps", "rotate_bilinear",
           "rotate_bilinear_T", "METHODS", "shear_shift_rows", "math"]
