"""Depth- and view-dependent PSF convolution with replicate padding and its
exact transpose (Sec. II-A: each (x, z) plane j of the rotated, attenuated
volume is convolved with p(:, :, j, l), replicate padding in i and k; Alg. 1;
adjoint: the convolution's transpose together with the adjoint of replicate
padding, Alg. 2).

Definition (true convolution, odd kernel px x pz, ha = (px-1)/2,
hb = (pz-1)/2, replicate padding = clamping the source index):

  c[i, k] = sum_{a<px} sum_{b<pz} p[a, b] * w[clamp(i - a + ha, 0, nx-1),
                                              clamp(k - b + hb, 0, nz-1)]

The transpose scatters each output back through the same clamped indices,
which sums the padded border onto the edge rows / columns.  The paper assumes
symmetric PSFs to shortcut this; the literal transpose below needs no such
assumption.

Planes are arrays w[i, j, k] (paper order) with kernels p[a, b, j]; every
depth plane j has its own kernel.  ``conv_planes_fft`` is the FFT form the
paper uses (edge-pad, linear convolution, crop): the same operator.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

# Threads scipy.fft may use in the FFT form (None -> scipy's default of 1).
FFT_WORKERS = None


def _clamp_index(n: int, h: int, taps: int):
    """idx[t, o] = clamp(o - t + h, 0, n-1): source of output o for tap t."""
    o = np.arange(n)[None, :]
    t = np.arange(taps)[:, None]
    return np.clip(o - t + h, 0, n - 1)


def conv_planes(w: np.ndarray, p: np.ndarray) -> np.ndarray:
    """c[i, j, k] = sum_{a,b} p[a, b, j] w[clamp(i-a+ha), j, clamp(k-b+hb)].

    w: (nx, ny, nz); p: (px, pz, ny).  Direct sum, loop over taps."""
    w = np.asarray(w, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    nx, ny, nz = w.shape
    px, pz, _ = p.shape
    assert px % 2 == 1 and pz % 2 == 1
    ia = _clamp_index(nx, (px - 1) // 2, px)
    kb = _clamp_index(nz, (pz - 1) // 2, pz)
    c = np.zeros_like(w)
    for a in range(px):
        wa = w[ia[a], :, :]
        for b in range(pz):
            c += p[a, b, :][None, :, None] * wa[:, :, kb[b]]
    return c


def conv_planes_T(g: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Exact transpose of conv_planes: for every tap, scatter-add
    p[a, b, j] * g[i, j, k] onto w-index (clamp(i-a+ha), j, clamp(k-b+hb))."""
    g = np.asarray(g, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    nx, ny, nz = g.shape
    px, pz, _ = p.shape
    ia = _clamp_index(nx, (px - 1) // 2, px)
    kb = _clamp_index(nz, (pz - 1) // 2, pz)
    u = np.zeros_like(g)
    for a in range(px):
        # scatter along i for tap a: rows of g go to rows ia[a]
        ga = np.zeros_like(g)
        np.add.at(ga, ia[a], g)
        for b in range(pz):
            contrib = p[a, b, :][None, :, None] * ga
            ub = np.zeros_like(g)
            np.add.at(ub.transpose(2, 0, 1), kb[b], contrib.transpose(2, 0, 1))
            u += ub
    return u


# ---------------------------------------------------------------- FFT form

def _fft_shape(nx, nz, px, pz):
    return (scipy.fft.next_fast_len(nx + 2 * ((px - 1) // 2) + px - 1, real=True),
            scipy.fft.next_fast_len(nz + 2 * ((pz - 1) // 2) + pz - 1, real=True))


def conv_sum_fft(w: np.ndarray, p: np.ndarray, workers=None) -> np.ndarray:
    """sum_j conv_planes(w, p)[:, j, :] via FFT, summing depths in the
    frequency domain (edge-padded linear convolution, then crop).

    Padded w: W[q] = w[clamp(q - ha)], q in [0, nx + 2 ha).  The linear
    convolution full[s] = sum_a p[a] W[s - a] equals c[i] at s = i + 2 ha."""
    workers = FFT_WORKERS if workers is None else workers
    w = np.asarray(w, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    nx, ny, nz = w.shape
    px, pz, _ = p.shape
    ha, hb = (px - 1) // 2, (pz - 1) // 2
    shape = _fft_shape(nx, nz, px, pz)
    wp = np.pad(w, ((ha, ha), (0, 0), (hb, hb)), mode="edge")       # (nx+2ha, ny, nz+2hb)
    Fw = scipy.fft.rfft2(wp, s=shape, axes=(0, 2), workers=workers)
    Fp = scipy.fft.rfft2(p.transpose(0, 2, 1), s=shape, axes=(0, 2), workers=workers)  # (px, ny, pz)
    full = scipy.fft.irfft2((Fw * Fp).sum(axis=1), s=shape, axes=(0, 1), workers=workers)
    return full[2 * ha: 2 * ha + nx, 2 * hb: 2 * hb + nz]


def conv_planes_T_fft(g2: np.ndarray, p: np.ndarray, workers=None) -> np.ndarray:
    """Transpose of conv_sum_fft applied to a projection g2[i, k]: returns
    u[i, j, k] = (conv_planes^T of g broadcast to every j).

    Adjoint of the linear convolution w.r.t. the padded input is the
    correlation U[q] = sum_i g[i] p[i + 2 ha - q] = (g * flip(p))[q]; the
    adjoint of the edge padding then folds the border rows/columns of U onto
    the edge rows/columns."""
    workers = FFT_WORKERS if workers is None else workers
    g2 = np.asarray(g2, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    nx, nz = g2.shape
    px, pz, ny = p.shape
    ha, hb = (px - 1) // 2, (pz - 1) // 2
    shape = _fft_shape(nx, nz, px, pz)
    Fg = scipy.fft.rfft2(g2, s=shape, axes=(0, 1), workers=workers)
    Fq = scipy.fft.rfft2(p[::-1, ::-1, :], s=shape, axes=(0, 1), workers=workers)
    U = scipy.fft.irfft2(Fg[:, :, None] * Fq, s=shape, axes=(0, 1), workers=workers)
    U = U[: nx + 2 * ha, : nz + 2 * hb, :]                         # (nx+2ha, nz+2hb, ny)
    # fold the padding (adjoint of replicate padding)
    Ui = U[ha: ha + nx].copy()
    Ui[0] += U[:ha].sum(axis=0)
    Ui[-1] += U[ha + nx:].sum(axis=0)
    Uk = Ui[:, hb: hb + nz].copy()
    Uk[:, 0] += Ui[:, :hb].sum(axis=1)
    Uk[:, -1] += Ui[:, hb + nz:].sum(axis=1)
    return Uk.transpose(0, 2, 1)                                   # (nx, ny, nz)
