"""GPU projector pair with 2-D bilinear rotation (SPECT_ROT_BILINEAR, the
alternative Sec. II-A names beside the 3-pass shears) against the FP64
oracle's bilinear projector: the same 1e-5 relative L2 bar as the 3-pass
path, the adjoint identity within 1e-5, the paper's explicit-matrix check
within 1e-6, slices above the LDS limit (global working slices), and the
paper-size workload on sampled views."""
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
    # nx, nz, nview, px, pz, angles, cache
    (32, 20, 16, 7, 7, None, False),
    (32, 20, 16, 7, 7, None, True),
    (37, 13, 10, 9, 5, None, False),                              # odd n
    (16, 1, 3, 41, 3, None, True),                                # one slice, wide kernel
    (20, 9, 8, 3, 7, None, False),                                # 45-degree ties
    (12, 7, 5, 5, 5, [0.1, -2.0, 3.9, 7.5, math.pi / 4], False),  # explicit angles
    (144, 4, 5, 5, 7, None, True),                                # above the LDS slice limit
    (144, 4, 5, 5, 7, None, False),
]


@pytest.mark.parametrize("case", CASES)
def test_bilinear_parity(case):
    nx, nz, nview, px, pz, angles, cache = case
    say(f"bilinear {case}")
    seed = 5 * nx + nz + nview
    x = synth.random_volume(nx, nx, nz, seed=seed)
    mu = synth.random_volume(nx, nx, nz, seed=seed + 1, high=0.06)
    psf = synth.random_psf(px, pz, nx, nview, seed=seed + 2, symmetric=False)
    dy = 1.5
    g = Geometry(nx, nx, nz, nview, px, pz, dy, angles=angles, rotation="bilinear")
    plan = spect.Plan(to_dev(mu), to_dev(psf), dy, angles=angles, cache_mubar=cache,
                      rotation="bilinear")
    v = host(plan.forward(to_dev(x)))
    ef = rel_l2(v, oracle.forward(x, mu, psf, g))
    y = synth.random_volume(nx, nz, nview, seed=seed + 3)
    b = host(plan.back(to_dev(y)))
    eb = rel_l2(b, oracle.back(y, mu, psf, g))
    say(f"  forward {ef:.2e}, back {eb:.2e}")
    assert ef <= TOL and eb <= TOL


def test_bilinear_differs_from_three_pass():
    """The flag selects a different operator (guards against a silently
    ignored flag): the two GPU projections differ by far more than the bar."""
    x, mu, psf, dy = synth.config_inputs("tiny", seed=2)
    a = spect.Plan(to_dev(mu), to_dev(psf), dy, rotation="3pass")
    b = spect.Plan(to_dev(mu), to_dev(psf), dy, rotation="bilinear")
    va, vb = host(a.forward(to_dev(x))), host(b.forward(to_dev(x)))
    assert rel_l2(va, vb) > 1e-3


def test_bilinear_dense_adjoint():
    """Sec. III-A-3 with bilinear rotation: explicit A and B at 8x8x6, 7 views."""
    nx, nz, nview, px = 8, 6, 7, 3
    N, M = nx * nx * nz, nview * nz * nx
    eyeN = torch.eye(N, device=DEV).reshape(N, nz, nx, nx)
    eyeM = torch.eye(M, device=DEV).reshape(M, nview, nz, nx)
    worst_t = worst_o = 0.0
    for rep in range(5):
        mu = synth.random_volume(nx, nx, nz, seed=700 + rep, high=0.3)
        psf = synth.random_psf(px, px, nx, nview, seed=800 + rep, symmetric=True)
        plan = spect.Plan(to_dev(mu), to_dev(psf), 1.0, rotation="bilinear")
        At = torch.empty(N, nview, nz, nx, device=DEV)
        B = torch.empty(M, nz, nx, nx, device=DEV)
        for c in range(N):
            plan.forward(eyeN[c], out=At[c])
        for c in range(M):
            plan.back(eyeM[c], out=B[c])
        torch.cuda.synchronize()
        A = At.reshape(N, M).double().T.cpu().numpy()
        Bm = B.reshape(M, N).double().T.cpu().numpy()
        worst_t = max(worst_t, np.linalg.norm(A.T - Bm) / np.linalg.norm(A))
        if rep < 2:
            g = Geometry(nx, nx, nz, nview, px, px, 1.0, rotation="bilinear")
            Aref = oracle.dense.forward_matrix(mu, psf, g)
            worst_o = max(worst_o, np.linalg.norm(A - Aref) / np.linalg.norm(Aref))
    say(f"bilinear dense: ||A^T - B|| / ||A|| = {worst_t:.2e}, vs oracle {worst_o:.2e}")
    assert worst_t <= 1e-6 and worst_o <= 1e-6


def test_bilinear_paper_size_sampled_views():
    """128x128x80, 128 views, 37x37 PSFs with bilinear rotation (the projector
    the paper times): forward on sampled views, the back projection of a
    projection nonzero on those views only, and the full-size adjoint
    identity."""
    say("bilinear paper size")
    x, mu, psf, dy = synth.config_inputs("paper", seed=0, view_wobble=0.1)
    g = Geometry(128, 128, 80, 128, 37, 37, dy, rotation="bilinear")
    views = [0, 16, 77]
    plan = spect.Plan(to_dev(mu), to_dev(psf), dy, cache_mubar=True, rotation="bilinear")
    xd = to_dev(x)
    v = host(plan.forward(xd))
    v_ref = oracle.forward(x, mu, psf, g, views=views, conv="fft")
    ef = max(rel_l2(v[l], v_ref[l]) for l in views)
    y = np.zeros((128, 80, 128), np.float32)
    y[views] = np.random.default_rng(6).uniform(0.0, 1.0, size=(len(views), 80, 128))
    b = host(plan.back(to_dev(y)))
    eb = rel_l2(b, oracle.back(y, mu, psf, g, views=views, conv="fft"))
    yd = to_dev(np.random.default_rng(7).uniform(0.0, 1.0, (128, 80, 128)))
    lhs = spect.dot_f64(plan.forward(xd), yd)
    rhs = spect.dot_f64(xd, plan.back(yd))
    gap = abs(lhs - rhs) / abs(lhs)
    say(f"  forward {ef:.2e}, back {eb:.2e}, adjoint gap {gap:.2e}")
    assert ef <= TOL and eb <= TOL and gap <= TOL
