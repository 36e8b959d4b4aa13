"""Pins of the oracle's EM derivatives (Sec. II-B: unrolled EM trained by
backpropagation through the projector) against central finite differences
in FP64 -- brute force that shares nothing with the chain-rule code.

The finite-difference case follows the differentiation workload: a
16x16x8 volume, 8 views, 5x5 PSFs, FP64 throughout.
"""
import numpy as np
import pytest

import oracle
from oracle import em
from oracle.projector import Geometry
from paper_2301_09710_amd import synth


def _problem(nx=16, nz=8, nview=8, p=5, seed=0):
    x, mu = synth.body_phantom(nx, nx, nz, seed=seed)
    psf = synth.gaussian_psf(p, p, nx, nview, 0.5, 1.5, view_wobble=0.1)
    g = Geometry(nx, nx, nz, nview, p, p, 4.8 * 128 / nx)

    def A(v):
        return oracle.forward(np.asarray(v).reshape(nz, nx, nx), mu, psf, g)

    def At(v):
        return oracle.back(v, mu, psf, g)

    xt = x.astype(np.float64) + 0.1
    sens = At(np.ones((nview, nz, nx)))
    yc = A(xt)
    r = np.full(yc.shape, 0.05 * yc.mean())
    y = synth.poisson_counts(yc * 20 + r, seed=seed + 3).astype(np.float64) + 0.5
    return xt, y, r, sens, A, At


def _central(f, z, d, eps):
    return (f(z + eps * d) - f(z - eps * d)) / (2 * eps)


def test_mlem_step_vjp_matches_finite_differences():
    xt, y, r, sens, A, At = _problem()
    rng = np.random.default_rng(1)
    x = np.ones_like(xt) * xt.mean() * rng.uniform(0.5, 1.5, size=xt.shape)
    g = rng.normal(size=xt.shape)
    gx, gy = em.mlem_step_vjp(x, y, r, sens, g, A, At)

    def L_x(z):
        return float((g * em.mlem_step(z, y, r, sens, A, At)).sum())

    def L_y(z):
        return float((g * em.mlem_step(x, z, r, sens, A, At)).sum())

    for k in range(3):
        dx = rng.normal(size=x.shape) * x.mean()
        fd = _central(L_x, x, dx, 1e-6)
        assert abs(fd - (gx * dx).sum()) <= 1e-7 * abs(fd) + 1e-12
        dy = rng.normal(size=y.shape) * y.mean()
        fd = _central(L_y, y, dy, 1e-6)
        assert abs(fd - (gy * dy).sum()) <= 1e-7 * abs(fd) + 1e-12


def test_vjp_drops_a_term_fails():
    """The finite-difference check above is sharp enough to see each term of
    the chain rule: removing the ybar path changes the x-gradient well beyond
    the tolerance."""
    xt, y, r, sens, A, At = _problem(nx=10, nz=4, nview=4, p=3)
    rng = np.random.default_rng(2)
    x = xt * rng.uniform(0.5, 1.5, size=xt.shape)
    g = rng.normal(size=xt.shape)
    gx, _ = em.mlem_step_vjp(x, y, r, sens, g, A, At)
    ybar = A(x) + r
    b = At(y / ybar)
    direct = g * b / sens
    dx = rng.normal(size=x.shape)
    fd = _central(lambda z: float((g * em.mlem_step(z, y, r, sens, A, At)).sum()), x, dx, 1e-6)
    assert abs(fd - (gx * dx).sum()) <= 1e-7 * abs(fd)
    assert abs(fd - (direct * dx).sum()) > 1e-3 * abs(fd)


def test_unrolled_gradient_matches_finite_differences():
    xt, y, r, sens, A, At = _problem()
    iters = 10
    x0 = np.full_like(xt, xt.mean())

    def loss_grad(xk):
        d = xk - xt
        return float((d * d).mean()), 2.0 * d / d.size

    xK, loss, gx0, gy = em.unrolled_mlem_grad(x0, y, r, sens, A, At, iters, loss_grad)

    def L(x0_, y_):
        z = x0_
        for _ in range(iters):
            z = em.mlem_step(z, y_, r, sens, A, At)
        return loss_grad(z)[0]

    assert abs(L(x0, y) - loss) <= 1e-12 * loss
    rng = np.random.default_rng(3)
    dx = rng.normal(size=x0.shape) * x0.mean()
    fd = _central(lambda z: L(z, y), x0, dx, 1e-5)
    assert abs(fd - (gx0 * dx).sum()) <= 1e-6 * abs(fd)
    dy = rng.normal(size=y.shape) * y.mean()
    fd = _central(lambda z: L(x0, z), y, dy, 1e-5)
    assert abs(fd - (gy * dy).sum()) <= 1e-6 * abs(fd)


def test_unrolled_gradient_zero_at_fixed_point_data():
    """With noiseless data y = A x_true (r = 0) and x0 = x_true, every iterate
    equals x_true, so the MSE loss and its gradients vanish."""
    xt, _, _, sens, A, At = _problem(nx=10, nz=4, nview=4, p=3)
    y = A(xt)

    def loss_grad(xk):
        d = xk - xt
        return float((d * d).mean()), 2.0 * d / d.size

    xK, loss, gx0, gy = em.unrolled_mlem_grad(xt, y, None, sens, A, At, 3, loss_grad)
    assert loss <= 1e-24
    assert np.abs(gx0).max() <= 1e-12 and np.abs(gy).max() <= 1e-12
