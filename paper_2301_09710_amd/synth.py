"""Seeded synthetic inputs for the SPECT projector: activity phantoms,
attenuation maps, depth/view-dependent Gaussian PSFs and Poisson draws.

This module holds no projector arithmetic (no rotation, attenuation factor,
convolution or depth sum).  It only draws inputs, so that the GPU path and the
FP64 reference can be fed identical data.  All arrays are float32 in the
storage layout of the C ABI:

  volumes      [nz][ny][nx]          (i = x fastest, j = y = depth, k = z)
  projections  [nview][nz][nx]
  PSFs         [nview][ny][pz][px]   (a along x fastest, b along z)

Shapes and value ranges follow the paper's workloads (Sec. II-C: 128x128x80
at 4.8 mm, 128 views, lesions of 5-100 mL, 2-D Gaussian PSF fits per
distance).  The paper's XCAT / patient phantoms are not available; these
generators stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "ellipsoid_phantom", "cylinder_mu", "body_phantom", "gaussian_psf",
    "random_psf", "random_volume", "poisson_counts", "config_inputs",
]


def _grid(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.astype(np.float64), j.astype(np.float64), k.astype(np.float64)


def ellipsoid_phantom(nx, ny, nz, n_ellipsoids=6, seed=0, support=0.6):
    """Sum of random solid ellipsoids with U(0,1) intensity.

    Centres lie within ``support * n/2`` of the rotation axis in the (x, y)
    plane and away from the z ends; semi-axes are U[2, 6] voxels (scaled down
    for small grids)."""
    rng = np.random.default_rng(seed)
    i, j, k = _grid(nx, ny, nz)
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    x = np.zeros((nz, ny, nx))
    amax = max(2.0, min(6.0, min(nx, ny) / 6.0))
    for _ in range(n_ellipsoids):
        r = support * min(nx, ny) / 2.0 * np.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * np.pi)
        x0, y0 = cx + r * np.cos(ang), cy + r * np.sin(ang)
        z0 = rng.uniform(min(3, nz / 4), max(nz - 4, 3 * nz / 4))
        ax, ay, az = rng.uniform(min(2.0, amax), amax, size=3)
        val = rng.uniform(0.0, 1.0)
        inside = ((i - x0) / ax) ** 2 + ((j - y0) / ay) ** 2 + ((k - z0) / az) ** 2 <= 1.0
        x[inside] += val
    return x.astype(np.float32)


def cylinder_mu(nx, ny, nz, value=0.015, ax_frac=0.4, ay_frac=0.3):
    """Attenuation map: ``value`` inside a centred elliptic cylinder along z
    (semi-axes ax_frac*nx, ay_frac*ny), zero outside."""
    i, j, _ = _grid(nx, ny, nz)
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    inside = ((i - cx) / (ax_frac * nx)) ** 2 + ((j - cy) / (ay_frac * ny)) ** 2 <= 1.0
    return np.where(inside, value, 0.0).astype(np.float32)


def body_phantom(nx=128, ny=128, nz=80, seed=0):
    """Ellipsoidal body (activity 1) with 3-6 hot spherical lesions (contrast
    4-10, radius 2.2-6.0 voxels = 5-100 mL at 4.8 mm) and a matching
    attenuation map in mm^-1: soft tissue 0.011, two lungs 0.003, a posterior
    spine cylinder 0.02.  Sizes scale with the grid (semi-axes 38, 27, 38 at
    128x128x80)."""
    rng = np.random.default_rng(seed)
    i, j, k = _grid(nx, ny, nz)
    cx, cy, cz = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    sx, sy = nx / 128.0, ny / 128.0
    sz = nz / 80.0
    ax, ay, az = 38.0 * sx, 27.0 * sy, 38.0 * sz
    body = ((i - cx) / ax) ** 2 + ((j - cy) / ay) ** 2 + ((k - cz) / az) ** 2 <= 1.0
    x = np.where(body, 1.0, 0.0)
    mu = np.where(body, 0.011, 0.0)
    # lungs
    for side in (-1.0, 1.0):
        lung = (((i - (cx + side * 14.0 * sx)) / (10.0 * sx)) ** 2
                + ((j - cy) / (8.0 * sy)) ** 2
                + ((k - (cz + 8.0 * sz)) / (15.0 * sz)) ** 2) <= 1.0
        mu = np.where(lung & body, 0.003, mu)
    # spine: posterior cylinder along z (posterior = low j side)
    spine = ((i - cx) ** 2 + (j - (cy - 18.0 * sy)) ** 2) <= (4.0 * min(sx, sy)) ** 2
    mu = np.where(spine & body, 0.02, mu)
    nles = int(rng.integers(3, 7))
    placed = 0
    tries = 0
    while placed < nles and tries < 1000:
        tries += 1
        rad = rng.uniform(2.2, 6.0) * min(sx, sy, sz)
        p = np.array([rng.uniform(cx - ax, cx + ax), rng.uniform(cy - ay, cy + ay),
                      rng.uniform(cz - az, cz + az)])
        # keep the whole sphere inside the body
        if ((abs(p[0] - cx) + rad) / ax) ** 2 + ((abs(p[1] - cy) + rad) / ay) ** 2 \
                + ((abs(p[2] - cz) + rad) / az) ** 2 > 1.0:
            continue
        contrast = rng.uniform(4.0, 10.0)
        sph = (i - p[0]) ** 2 + (j - p[1]) ** 2 + (k - p[2]) ** 2 <= rad ** 2
        x = np.where(sph, contrast, x)
        placed += 1
    return x.astype(np.float32), mu.astype(np.float32)


def gaussian_psf(px, pz, ny, nview, sigma_min, sigma_max, view_wobble=0.0):
    """Point-sampled 2-D Gaussian exp(-(a^2+b^2)/(2 sigma^2)) on the integer
    grid, normalised to sum 1 per (depth, view).  sigma is linear in depth:
    sigma_min at j = ny-1 (the plane nearest the detector) to sigma_max at
    j = 0.  ``view_wobble`` multiplies sigma by (1 + view_wobble *
    sin(2 pi l / nview)) so that the (j, l) indexing of the kernels can be
    told apart in tests."""
    ha, hb = (px - 1) // 2, (pz - 1) // 2
    a = np.arange(px) - ha
    b = np.arange(pz) - hb
    out = np.empty((nview, ny, pz, px), dtype=np.float64)
    for l in range(nview):
        f = 1.0 + view_wobble * np.sin(2 * np.pi * l / nview)
        for jj in range(ny):
            t = (ny - 1 - jj) / (ny - 1) if ny > 1 else 0.0
            s = (sigma_min + (sigma_max - sigma_min) * t) * f
            g = np.exp(-(b[:, None] ** 2 + a[None, :] ** 2) / (2 * s * s))
            out[l, jj] = g / g.sum()
    return out.astype(np.float32)


def gaussian_psf_factors(px, pz, ny, nview, sigma_min, sigma_max, view_wobble=0.0):
    """The 1-D factors of ``gaussian_psf``: fz [nview][ny][pz] and fx
    [nview][ny][px], each exp(-t^2 / (2 sigma^2)) normalised to sum 1, so that
    their outer product fz[b] fx[a] is the normalised 2-D Gaussian."""
    ha, hb = (px - 1) // 2, (pz - 1) // 2
    a = np.arange(px) - ha
    b = np.arange(pz) - hb
    fz = np.empty((nview, ny, pz), dtype=np.float64)
    fx = np.empty((nview, ny, px), dtype=np.float64)
    for l in range(nview):
        f = 1.0 + view_wobble * np.sin(2 * np.pi * l / nview)
        for jj in range(ny):
            t = (ny - 1 - jj) / (ny - 1) if ny > 1 else 0.0
            s = (sigma_min + (sigma_max - sigma_min) * t) * f
            gz = np.exp(-(b ** 2) / (2 * s * s))
            gx = np.exp(-(a ** 2) / (2 * s * s))
            fz[l, jj] = gz / gz.sum()
            fx[l, jj] = gx / gx.sum()
    return fz.astype(np.float32), fx.astype(np.float32)


def random_psf(px, pz, ny, nview, seed=0, symmetric=True):
    """Random nonnegative PSFs normalised to sum 1.  ``symmetric`` makes each
    kernel symmetric in both a and b (the paper's adjoint test uses random
    symmetric PSFs)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, 1.0, size=(nview, ny, pz, px))
    if symmetric:
        p = p + p[..., ::-1, :]
        p = p + p[..., :, ::-1]
    p = p / p.sum(axis=(2, 3), keepdims=True)
    return p.astype(np.float32)


def random_volume(nx, ny, nz, seed=0, low=0.0, high=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=(nz, ny, nx)).astype(np.float32)


def poisson_counts(mean, seed=0):
    """Poisson draw with the given mean array (float32 result)."""
    rng = np.random.default_rng(seed)
    return rng.poisson(np.maximum(np.asarray(mean, dtype=np.float64), 0.0)).astype(np.float32)


# Workloads (sizes, PSF widths, units) -------------------------------------------

CONFIGS = {
    # tiny: 32x32x20, 16 views, 7x7 PSF, sigma 0.5 -> 2, mu = 0.015 per voxel, dy = 1
    "tiny": dict(nx=32, ny=32, nz=20, nview=16, px=7, pz=7, sigma=(0.5, 2.0), dy=1.0),
    # paper scale: 128x128x80 at 4.8 mm, 128 views, 37x37 PSF, sigma 1 -> 6, mu in mm^-1
    "paper": dict(nx=128, ny=128, nz=80, nview=128, px=37, pz=37, sigma=(1.0, 6.0), dy=4.8),
    # serving mix members
    "serve64": dict(nx=64, ny=64, nz=40, nview=64, px=19, pz=19, sigma=(0.5, 3.0), dy=9.6),
    "serve96": dict(nx=96, ny=96, nz=64, nview=120, px=29, pz=29, sigma=(0.75, 4.5), dy=6.4),
    # precision workload: 256x256x160 at 2.4 mm, 128 views, 37x37
    "large": dict(nx=256, ny=256, nz=160, nview=128, px=37, pz=37, sigma=(1.0, 6.0), dy=2.4),
}


def config_inputs(name, seed=0, view_wobble=0.0):
    """(x, mu, psf, dy) for a named workload."""
    c = CONFIGS[name]
    nx, ny, nz, nv = c["nx"], c["ny"], c["nz"], c["nview"]
    if name == "tiny":
        x = ellipsoid_phantom(nx, ny, nz, 6, seed=seed)
        mu = cylinder_mu(nx, ny, nz, 0.015)
    else:
        x, mu = body_phantom(nx, ny, nz, seed=seed)
    psf = gaussian_psf(c["px"], c["pz"], ny, nv, c["sigma"][0], c["sigma"][1], view_wobble)
    return x, mu, psf, c["dy"]
