"""View angles and the split of a rotation into an exact quarter turn and a
residual handled by three 1-D shears (Sec. II-A: each view rotates the
volume about the z axis by theta_l, typically 2*pi*l/nview for 0-based l,
using 3-pass 1-D linear interpolation).

The paper cites the 3-pass method without stating range reduction or the
shear order; the reading used here:

  theta = M * (pi/2) + phi,  M = floor(theta / (pi/2) + 1/2),  m = M mod 4,
  phi in [-pi/4, pi/4)  (a tie phi = +pi/4 rounds up to the next quarter).

For the default angles theta_l = 2*pi*l/nview the split is done in exact
integer arithmetic: M = floor((8 l + nview) / (2 nview)) and
phi = (pi/2) (4 l - M nview) / nview, so ties at 45 degrees are exact.

Rotation by phi about c is R(phi) and the gather needs R(phi)^-1 =
R(-phi) = X(t) Y(-s) X(t), t = tan(phi/2), s = sin(phi), where
X(a) = [[1, a], [0, 1]] and Y(b) = [[1, 0], [b, 1]] act on (i, j).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class ViewSplit:
    m: int        # quarter turns, 0..3
    phi: float    # residual angle in [-pi/4, pi/4)
    t: float      # tan(phi/2): shift per unit j in passes 1 and 3
    s: float      # sin(phi):  shift per unit i in pass 2 is -s


def default_angles(nview: int) -> np.ndarray:
    return np.array([2.0 * math.pi * l / nview for l in range(nview)])


def split_default(l: int, nview: int) -> ViewSplit:
    M = (8 * l + nview) // (2 * nview)
    phi = (math.pi / 2.0) * (4 * l - M * nview) / nview
    return ViewSplit(M % 4, phi, math.tan(phi / 2.0), math.sin(phi))


def split_angle(theta: float) -> ViewSplit:
    q = theta / (math.pi / 2.0)
    M = math.floor(q + 0.5)
    phi = theta - M * (math.pi / 2.0)
    return ViewSplit(int(M) % 4, phi, math.tan(phi / 2.0), math.sin(phi))


def view_splits(nview: int, angles=None) -> list[ViewSplit]:
    if angles is None:
        return [split_default(l, nview) for l in range(nview)]
    angles = np.asarray(angles, dtype=np.float64)
    assert angles.shape == (nview,)
    return [split_angle(float(a)) for a in angles]
