"""Pins of the oracle's 2-D bilinear rotation (Sec. II-A names bilinear
interpolation with zero padding as the alternative to the 3-pass shears)
against facts that do not come from the oracle: scipy's order-1 spline
interpolation with constant zero padding at the rotated coordinates, exact
reproduction of linear functions, the quarter turns at phi = 0, a
brute-force transpose, agreement with the 3-pass rotation on a smooth blob
(same sense and centre), and the projector-level dense adjoint."""
import math

import numpy as np
import pytest
import scipy.ndimage

import oracle
from oracle import geometry, rotation
from oracle.projector import Geometry
from paper_2301_09710_amd import synth


def rotated_coords(n, theta):
    """R(theta)^-1 (p - c) + c for every output pixel p = (i, j)."""
    c = (n - 1) / 2.0
    u, v = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    co, sn = math.cos(theta), math.sin(theta)
    return c + co * u + sn * v, c - sn * u + co * v


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_phi_zero_is_the_quarter_turn(m):
    f = np.random.default_rng(m).uniform(size=(9, 9, 2))
    split = geometry.ViewSplit(m, 0.0, 0.0, 0.0)
    np.testing.assert_array_equal(rotation.rotate_bilinear(f, split), rotation.quarter_turn(f, m))


@pytest.mark.parametrize("n", [9, 12])
@pytest.mark.parametrize("theta", [0.3, 1.9, -2.5, 4.0, math.pi / 4, 3 * math.pi / 4 + 1e-3])
def test_matches_scipy_order1_zero_padding(n, theta):
    rng = np.random.default_rng(n)
    f = rng.uniform(size=(n, n, 2))
    got = rotation.rotate_bilinear(f, geometry.split_angle(theta))
    si, sj = rotated_coords(n, theta)
    for k in range(2):
        ref = scipy.ndimage.map_coordinates(f[:, :, k], [si, sj], order=1, mode="grid-constant",
                                            cval=0.0)
        np.testing.assert_allclose(got[:, :, k], ref, rtol=0, atol=1e-12)


def test_linear_function_reproduced_inside_the_grid():
    n, theta = 16, 0.37
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = 0.7 * i - 1.3 * j + 5.0
    got = rotation.rotate_bilinear(f, geometry.split_angle(theta))
    si, sj = rotated_coords(n, theta)
    inside = (si >= 0) & (si <= n - 1) & (sj >= 0) & (sj <= n - 1)
    assert inside.sum() > n * n // 2
    np.testing.assert_allclose(got[inside], (0.7 * si - 1.3 * sj + 5.0)[inside], rtol=0, atol=1e-12)


@pytest.mark.parametrize("theta", [0.0, 0.5, 2.2, -1.0, math.pi / 4])
def test_transpose_brute_force(theta):
    n, t = 6, 2
    split = geometry.split_angle(theta)
    N = n * n * t
    A = np.zeros((N, N))
    B = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        A[:, c] = rotation.rotate_bilinear(e.reshape(n, n, t), split).ravel()
        B[:, c] = rotation.rotate_bilinear_T(e.reshape(n, n, t), split).ravel()
    np.testing.assert_allclose(B, A.T, rtol=0, atol=1e-15)


def test_same_sense_and_centre_as_three_pass():
    n, theta = 48, 0.7
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = np.exp(-((i - 30.0) ** 2 + (j - 19.0) ** 2) / (2 * 3.0 ** 2))[:, :, None]
    split = geometry.split_angle(theta)
    a = rotation.rotate(f, split)[:, :, 0]
    b = rotation.rotate_bilinear(f, split)[:, :, 0]

    def centroid(g):
        return np.array([(g * i).sum(), (g * j).sum()]) / g.sum()

    # the blob's centre moves by R(theta) about c
    c = (n - 1) / 2.0
    co, sn = math.cos(theta), math.sin(theta)
    expect = np.array([c + co * (30.0 - c) - sn * (19.0 - c), c + sn * (30.0 - c) + co * (19.0 - c)])
    np.testing.assert_allclose(centroid(a), expect, atol=0.05)
    np.testing.assert_allclose(centroid(b), expect, atol=0.05)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 0.03


@pytest.mark.parametrize("case", [(6, 3, 3, 3, 3), (5, 2, 4, 3, 1)])
def test_bilinear_projector_dense_adjoint(case):
    nx, nz, nview, px, pz = case
    mu = synth.random_volume(nx, nx, nz, seed=11, high=0.3)
    psf = synth.random_psf(px, pz, nx, nview, seed=12, symmetric=False)
    g = Geometry(nx, nx, nz, nview, px, pz, 1.3, rotation="bilinear")
    A = oracle.dense.forward_matrix(mu, psf, g)
    B = oracle.dense.back_matrix(mu, psf, g)
    np.testing.assert_allclose(B, A.T, rtol=0, atol=1e-13 * np.abs(A).max())


def test_bilinear_quarter_views_are_line_sums():
    """mu = 0, delta PSF, views at multiples of 90 degrees: every rotation is
    an exact quarter turn, so the projection is the plain depth sum of the
    quarter-turned volume (the same as with the 3-pass shears)."""
    n, nz = 8, 3
    x = synth.random_volume(n, n, nz, seed=3).astype(np.float64)
    mu = np.zeros_like(x)
    psf = np.ones((4, n, 1, 1))
    g = Geometry(n, n, nz, 4, 1, 1, 1.0, rotation="bilinear")
    v = oracle.forward(x, mu, psf, g)
    xp = x.transpose(2, 1, 0)                       # x[i, j, k]
    for l in range(4):
        ref = rotation.quarter_turn(xp, l).sum(axis=1).T
        np.testing.assert_allclose(v[l], ref, rtol=0, atol=1e-12)
