"""The plain FP32 convolution kernels (csrc/conv.hip), which a plan selects
when the PSF is taller than the matrix-core tiles hold (pz >= 67): forward
(Sec. II-A, Alg. 1, replicate padding by clamped source indices) and its
exact transpose with the fold of the padding (Eq. (2), Alg. 2), through the
C ABI against the FP64 oracle.

Bars: forward and back within 1e-5 relative L2 of the oracle; the GPU
adjoint identity within 1e-5; the explicit matrices B = A^T and A = the
oracle's matrix within 1e-6 (the paper's adjoint check, Sec. III-A).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle.projector import Geometry
from paper_2301_09710_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2301_09710_amd import spect  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [
    # nx, nz, nview, px, pz, angles
    (32, 80, 16, 9, 69, None),                       # 32x32x80, 16 views, 9x69
    (17, 3, 5, 5, 71, [0.3, -1.1, 2.0, 4.0, 7.5]),   # kernel taller than the volume, odd n
    (24, 70, 8, 1, 67, None),                        # z-only kernel, 45-degree ties
]


@pytest.mark.parametrize("case", CASES)
def test_direct_parity(case):
    nx, nz, nview, px, pz, angles = case
    say(f"direct {case}")
    seed = 7 * nx + pz
    x = synth.random_volume(nx, nx, nz, seed=seed)
    mu = synth.random_volume(nx, nx, nz, seed=seed + 1, high=0.05)
    psf = synth.random_psf(px, pz, nx, nview, seed=seed + 2, symmetric=False)
    dy = 1.5
    g = Geometry(nx, nx, nz, nview, px, pz, dy, angles=angles)
    for cache in (False, True):
        plan = spect.Plan(to_dev(mu), to_dev(psf), dy, angles=angles, cache_mubar=cache)
        assert plan.describe()["conv"] == "fp32-direct", plan.describe()
        ef = rel_l2(host(plan.forward(to_dev(x))), oracle.forward(x, mu, psf, g, conv="fft"))
        y = synth.random_volume(nx, nz, nview, seed=seed + 3)
        eb = rel_l2(host(plan.back(to_dev(y))), oracle.back(y, mu, psf, g, conv="fft"))
        say(f"  cache={cache}: forward {ef:.2e}, back {eb:.2e}")
        assert ef <= TOL and eb <= TOL
        lhs = spect.dot_f64(plan.forward(to_dev(x)), to_dev(y))
        rhs = spect.dot_f64(to_dev(x), plan.back(to_dev(y)))
        assert abs(lhs - rhs) <= TOL * abs(lhs)
        plan.close()


def test_direct_dense_adjoint():
    """Explicit A and B on 6x6x5 / 3 views with 3x67 PSFs (taller than the
    volume, so every edge fold sums a run of rows)."""
    nx, nz, nview, px, pz = 6, 5, 3, 3, 67
    N, M = nx * nx * nz, nview * nz * nx
    eyeN = torch.eye(N, device=DEV).reshape(N, nz, nx, nx)
    eyeM = torch.eye(M, device=DEV).reshape(M, nview, nz, nx)
    worst_t = worst_o = 0.0
    for rep in range(3):
        mu = synth.random_volume(nx, nx, nz, seed=50 + rep, high=0.3)
        psf = synth.random_psf(px, pz, nx, nview, seed=60 + rep, symmetric=False)
        plan = spect.Plan(to_dev(mu), to_dev(psf), 1.0)
        assert plan.describe()["conv"] == "fp32-direct"
        At = torch.empty(N, nview, nz, nx, device=DEV)
        B = torch.empty(M, nz, nx, nx, device=DEV)
        for c in range(N):
            plan.forward(eyeN[c], out=At[c])
        for c in range(M):
            plan.back(eyeM[c], out=B[c])
        torch.cuda.synchronize()
        A = At.reshape(N, M).double().T.cpu().numpy()
        Bm = B.reshape(M, N).double().T.cpu().numpy()
        Aref = oracle.dense.forward_matrix(mu, psf, Geometry(nx, nx, nz, nview, px, pz, 1.0))
        worst_t = max(worst_t, np.linalg.norm(A.T - Bm) / np.linalg.norm(A))
        worst_o = max(worst_o, np.linalg.norm(A - Aref) / np.linalg.norm(Aref))
        plan.close()
    say(f"direct dense: ||A^T - B|| / ||A|| = {worst_t:.2e}, vs oracle {worst_o:.2e}")
    assert worst_t <= 1e-6 and worst_o <= 1e-6
