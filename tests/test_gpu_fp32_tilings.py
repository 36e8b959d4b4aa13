"""The two FP32 tilings of the PSF convolution, each forced at plan creation
through the SPECT_TILING_* flags: 16x16x4 Toeplitz blocks ("16x16") and 4x4x1
blocks ("4x4", which pairs mirror-image taps when the PSF rows are symmetric
in x; "4x4/all-taps" turns the pairing off through SPECT_PSF_ALL_TAPS),
against the FP64 oracle.

The plan picks a tiling per shape from its cost model (4x4 blocks at the
paper's 128x128x80 / 37x37 workload, 16x16 blocks on most small shapes), so
without the override most small cases would exercise one tiling only.  Cases
cover ragged tiles along z and x, a kernel wider than the plane, one slice,
asymmetric PSFs, several z tiles, and the paper-size workload on sampled
views; the explicit-matrix adjoint check runs on both.
"""
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
TILINGS = ["4x4", "4x4/all-taps", "16x16"]


def force(tiling):
    """Plan keywords selecting a tiling (and whether the 4x4 kernels may pair
    mirror-image taps)."""
    return dict(tiling=tiling.split("/")[0],
                mirror="off" if tiling.endswith("/all-taps") else "auto")


def check_selection(plan, tiling, symmetric):
    d = plan.describe()
    assert d["conv"] == ("fp32-16x16" if tiling == "16x16" else "fp32-4x4"), d
    assert d["mirror"] == ("1" if tiling == "4x4" and symmetric else "0"), d


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
    # nx, nz, nview, px, pz, symmetric PSF
    (32, 20, 6, 7, 7, True),
    (37, 13, 5, 9, 5, False),
    (16, 1, 3, 41, 3, True),      # kernel wider than the plane, one slice
    (48, 41, 4, 19, 21, False),   # z tile boundary, asymmetric PSF
    (70, 85, 3, 11, 13, False),   # two z tiles
    (9, 4, 2, 1, 1, True),
]


@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("case", CASES)
def test_tiling_parity(case, tiling):
    nx, nz, nview, px, pz, sym = case
    say(f"tiling {tiling} {case}")
    seed = 7 * nx + nz
    x = synth.random_volume(nx, nx, nz, seed=seed)
    mu = synth.random_volume(nx, nx, nz, seed=seed + 1, high=0.05)
    psf = synth.random_psf(px, pz, nx, nview, seed=seed + 2, symmetric=sym)
    dy = 1.5
    g = Geometry(nx, nx, nz, nview, px, pz, dy)
    plan = spect.Plan(to_dev(mu), to_dev(psf), dy, **force(tiling))
    check_selection(plan, tiling, sym)
    v = host(plan.forward(to_dev(x)))
    ef = rel_l2(v, oracle.forward(x, mu, psf, g))
    y = synth.random_volume(nx, nz, nview, seed=seed + 3)
    b = host(plan.back(to_dev(y)))
    eb = rel_l2(b, oracle.back(y, mu, psf, g))
    say(f"  forward {ef:.2e}, back {eb:.2e}")
    assert ef <= TOL and eb <= TOL


@pytest.mark.parametrize("tiling", TILINGS)
def test_tiling_dense_adjoint(tiling):
    """Explicit A and B on 8x8x6 / 7 views: B = A^T to 1e-6 relative."""
    nx, nz, nview, px = 8, 6, 7, 3
    N, M = nx * nx * nz, nview * nz * nx
    eyeN = torch.eye(N, device=DEV).reshape(N, nz, nx, nx)
    eyeM = torch.eye(M, device=DEV).reshape(M, nview, nz, nx)
    worst = 0.0
    for rep in range(5):
        mu = synth.random_volume(nx, nx, nz, seed=300 + rep, high=0.3)
        psf = synth.random_psf(px, px, nx, nview, seed=400 + rep, symmetric=False)
        plan = spect.Plan(to_dev(mu), to_dev(psf), 1.0, **force(tiling))
        At = torch.empty(N, nview, nz, nx, device=DEV)
        B = torch.empty(M, nz, nx, nx, device=DEV)
        for c in range(N):
            plan.forward(eyeN[c], out=At[c])
        for c in range(M):
            plan.back(eyeM[c], out=B[c])
        torch.cuda.synchronize()
        A = At.reshape(N, M).double().T.cpu().numpy()
        Bm = B.reshape(M, N).double().T.cpu().numpy()
        worst = max(worst, np.linalg.norm(A.T - Bm) / np.linalg.norm(A))
    say(f"tiling {tiling}: ||A^T - B|| / ||A|| = {worst:.2e}")
    assert worst <= 1e-6


@pytest.fixture(scope="module")
def paper():
    x, mu, psf, dy = synth.config_inputs("paper", seed=1)
    g = Geometry(128, 128, 80, 128, 37, 37, dy)
    views = [3, 90]
    say("paper: oracle on sampled views")
    v_ref = oracle.forward(x, mu, psf, g, views=views, conv="fft")
    y = np.zeros((128, 80, 128), np.float32)
    y[views] = np.random.default_rng(4).uniform(0.0, 1.0, size=(len(views), 80, 128))
    b_ref = oracle.back(y, mu, psf, g, views=views, conv="fft")
    return dict(x=x, mu=mu, psf=psf, dy=dy, views=views, v_ref=v_ref, y=y, b_ref=b_ref)


@pytest.mark.parametrize("tiling", TILINGS)
def test_tiling_paper_sampled(paper, tiling):
    say(f"tiling {tiling}: paper size")
    plan = spect.Plan(to_dev(paper["mu"]), to_dev(paper["psf"]), paper["dy"], cache_mubar=True,
                      **force(tiling))
    check_selection(plan, tiling, True)
    xd = to_dev(paper["x"])
    v = host(plan.forward(xd))
    ef = max(rel_l2(v[l], paper["v_ref"][l]) for l in paper["views"])
    b = host(plan.back(to_dev(paper["y"])))
    eb = rel_l2(b, paper["b_ref"])
    yd = to_dev(np.random.default_rng(5).uniform(0.0, 1.0, (128, 80, 128)))
    lhs = spect.dot_f64(plan.forward(xd), yd)
    rhs = spect.dot_f64(xd, plan.back(yd))
    gap = abs(lhs - rhs) / abs(lhs)
    say(f"  forward {ef:.2e}, back {eb:.2e}, adjoint gap {gap:.2e}")
    assert ef <= TOL and eb <= TOL and gap <= TOL
