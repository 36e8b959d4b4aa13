"""Poisson model and EM updates (Sec. II-B).

  y ~ Poisson(A x + r)                                   Eq. (3)
  f(x) = 1'(A x + r) - y' log(A x + r)                   Eq. (4)
  e(x) = A'(y / (A x + r)),  d(beta) = A'1 - beta u      Eq. (8)
  x_hat = (-d + sqrt(d^2 + 4 beta x e)) / (2 beta)       Eq. (7)

beta -> 0 gives the plain ML-EM update x+ = x * e / A'1.  The paper does not
say what to do with zero denominators; the reading here: the ratio is 0 where
A x + r <= 0 and the update is 0 where A'1 <= 0.

For beta > 0 and d > 0 the root of Eq. (7) is evaluated in the equivalent
cancellation-free form 2 x e / (d + sqrt(d^2 + 4 beta x e)).
"""
from __future__ import annotations

import numpy as np


def neg_log_likelihood(ybar, y):
    """Eq. (4) without the constant, for ybar = A x + r > 0."""
    ybar = np.asarray(ybar, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(ybar.sum() - (y * np.log(ybar)).sum())


def ratio(y, ybar):
    y = np.asarray(y, dtype=np.float64)
    ybar = np.asarray(ybar, dtype=np.float64)
    out = np.zeros_like(ybar)
    ok = ybar > 0
    out[ok] = y[ok] / ybar[ok]
    return out


def mlem_step(x, y, r, sens, A, At):
    """One ML-EM update; A, At are callables (forward / back projector)."""
    x = np.asarray(x, dtype=np.float64)
    ybar = A(x) + (0.0 if r is None else np.asarray(r, dtype=np.float64))
    e = At(ratio(y, ybar))
    sens = np.asarray(sens, dtype=np.float64)
    out = np.zeros_like(x)
    ok = sens > 0
    out[ok] = x[ok] * e[ok] / sens[ok]
    return out


def reg_em_update(x, e, sens, u, beta):
    """Eq. (7) with d = sens - beta u, for beta > 0."""
    x = np.asarray(x, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    d = np.asarray(sens, dtype=np.float64) - beta * np.asarray(u, dtype=np.float64)
    disc = np.sqrt(d * d + 4.0 * beta * x * e)
    return np.where(d > 0, 2.0 * x * e / np.where(d > 0, d + disc, 1.0),
                    (-d + disc) / (2.0 * beta))


def mlem_step_vjp(x, y, r, sens, g, A, At, ybar=None, b=None):
    """Reverse-mode derivative of ``mlem_step`` (the unrolled EM iterations of
    Sec. II-B are trained by backpropagation).  For x+ = x * b / s with
    b = At(rho), rho = y / ybar, ybar = A x + r and upstream g = dL/dx+, the
    chain rule gives, away from the guarded branches (which are constant):

      dL/db   = g x / s                 dL/dx (direct) = g b / s
      dL/drho = A(dL/db)                (b = At rho, and At's adjoint is A)
      dL/dy   = dL/drho / ybar
      dL/dybar = -dL/drho * y / ybar^2
      dL/dx  += At(dL/dybar)            (ybar = A x + r)

    Returns (dL/dx, dL/dy).  A and At are callables; FP64 throughout.
    ``ybar`` and ``b``, when given, are the step's own A x + r and
    At(y / ybar) (as the forward step computed them); otherwise they are
    recomputed from x."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    sens = np.asarray(sens, dtype=np.float64)
    if ybar is None:
        ybar = A(x) + (0.0 if r is None else np.asarray(r, dtype=np.float64))
    if b is None:
        b = At(ratio(y, ybar))
    okx = sens > 0
    g_b = np.zeros_like(x)
    g_b[okx] = g[okx] * x[okx] / sens[okx]
    gx = np.zeros_like(x)
    gx[okx] = g[okx] * b[okx] / sens[okx]
    g_rho = A(g_b)
    oky = ybar > 0
    gy = np.zeros_like(ybar)
    gy[oky] = g_rho[oky] / ybar[oky]
    g_ybar = np.zeros_like(ybar)
    g_ybar[oky] = -g_rho[oky] * y[oky] / ybar[oky] ** 2
    gx = gx + At(g_ybar)
    return gx, gy


def unrolled_mlem_grad(x0, y, r, sens, A, At, iters, loss_grad):
    """x_K after ``iters`` ML-EM updates from x0, and the gradients of a loss
    L(x_K) with respect to x0 and y.  ``loss_grad(x_K)`` returns
    (L, dL/dx_K).  Plain reverse accumulation over the stored iterates; each
    step's A x + r and At(y / (A x + r)) are kept from the forward sweep, so
    the backward sweep projects only the two new directions per step."""
    rr = 0.0 if r is None else np.asarray(r, dtype=np.float64)
    xs = [np.asarray(x0, dtype=np.float64)]
    saved = []
    s64 = np.asarray(sens, dtype=np.float64)
    for _ in range(iters):
        x = xs[-1]
        ybar = A(x) + rr
        b = At(ratio(y, ybar))
        out = np.zeros_like(x)
        ok = s64 > 0
        out[ok] = x[ok] * b[ok] / s64[ok]
        saved.append((ybar, b))
        xs.append(out)
    loss, g = loss_grad(xs[-1])
    gy = np.zeros_like(np.asarray(y, dtype=np.float64))
    for k in range(iters - 1, -1, -1):
        g, gyk = mlem_step_vjp(xs[k], y, r, sens, g, A, At, ybar=saved[k][0], b=saved[k][1])
        gy = gy + gyk
    return xs[-1], loss, g, gy


def osem_subsets(nview, nsub):
    """Ordered subsets of the views (Sec. III-A compares OSEM reconstructions):
    subset s holds the views l with l mod nsub = s, visited for s = 0..nsub-1.
    The paper does not say how its subsets are formed; interleaved subsets
    are the usual choice."""
    return [list(range(s, nview, nsub)) for s in range(nsub)]


def osem(x0, y, r, A_sub, At_sub, nview, nsub, iters):
    """OSEM: each iteration runs one ML-EM update per subset, with the
    subset's own projector A_s, back projector At_s and sensitivity At_s 1.
    A_sub(s, x) returns the projections of subset s ([len(s)][nz][nx]);
    At_sub(s, v) back-projects them.  y, r: full sinograms [nview][nz][nx]."""
    subs = osem_subsets(nview, nsub)
    y = np.asarray(y, dtype=np.float64)
    r = None if r is None else np.asarray(r, dtype=np.float64)
    sens = [At_sub(s, np.ones((len(v),) + y.shape[1:])) for s, v in enumerate(subs)]
    x = np.asarray(x0, dtype=np.float64)
    for _ in range(iters):
        for s, views in enumerate(subs):
            x = mlem_step(x, y[views], None if r is None else r[views], sens[s],
                          lambda z, s=s: A_sub(s, z), lambda v, s=s: At_sub(s, v))
    return x
