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
