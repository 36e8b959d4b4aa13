"""Method variants on the GPU against the FP64 oracle: the regularised EM
update of Eq. (7)-(8) (beta > 0, target image u)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import em
from oracle.projector import Geometry
from paper_2301_09710_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2301_09710_amd import spect  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.mark.parametrize("beta", [0.0, 1e-3, 0.05, 2.0])
def test_regularized_em_step_parity(beta):
    print(f"reg em beta={beta}", flush=True)
    x_true, mu, psf, dy = synth.config_inputs("tiny", seed=0, view_wobble=0.1)
    g = Geometry(32, 32, 20, 16, 7, 7, dy)
    A = lambda v: oracle.forward(np.asarray(v).reshape(20, 32, 32), mu, psf, g)
    At = lambda v: oracle.back(v, mu, psf, g)
    rng = np.random.default_rng(4)
    yc = A(x_true)
    r = np.full(yc.shape, 0.05 * yc.mean(), dtype=np.float32)
    y = synth.poisson_counts(yc * 30 + r, seed=6).astype(np.float32)
    x = (x_true + 0.2 * rng.uniform(size=x_true.shape)).astype(np.float32)
    u = (x_true * rng.uniform(0.5, 1.5, size=x_true.shape)).astype(np.float32)
    sens = At(np.ones(yc.shape)).astype(np.float32)
    e = At(em.ratio(y, A(x) + r))
    ref = (em.mlem_step(x, y, r, sens, A, At) if beta == 0.0
           else em.reg_em_update(x, e, sens, u, beta))
    plan = spect.Plan(to_dev(mu), to_dev(psf), dy)
    xd = to_dev(x)
    plan.reg_em_step(xd, to_dev(y), to_dev(sens), to_dev(u), beta, to_dev(r))
    torch.cuda.synchronize()
    err = rel_l2(xd.cpu().numpy(), ref)
    print(f"reg em beta={beta}: rel L2 {err:.2e}", flush=True)
    assert err <= TOL


def test_osem_parity():
    """OSEM, 4 subsets x 2 iterations (the paper's comparisons use 4 subsets)."""
    import math
    from paper_2301_09710_amd.osem import OSEM
    print("osem", flush=True)
    x_true, mu, psf, dy = synth.config_inputs("tiny", seed=0, view_wobble=0.1)
    nview, nsub = 16, 4
    g = Geometry(32, 32, 20, nview, 7, 7, dy)
    yc = oracle.forward(x_true, mu, psf, g)
    r = np.full(yc.shape, 0.05 * yc.mean(), dtype=np.float32)
    y = synth.poisson_counts(yc * 30 + r, seed=8).astype(np.float32)
    subs = em.osem_subsets(nview, nsub)

    def geom(s):
        return Geometry(32, 32, 20, len(subs[s]), 7, 7, dy,
                        angles=[2 * math.pi * l / nview for l in subs[s]])

    A_sub = lambda s, z: oracle.forward(np.asarray(z).reshape(20, 32, 32), mu, psf[subs[s]], geom(s))
    At_sub = lambda s, v: oracle.back(v, mu, psf[subs[s]], geom(s))
    ref = em.osem(np.ones_like(x_true), y, r, A_sub, At_sub, nview, nsub, 2)
    os_ = OSEM(to_dev(mu), to_dev(psf), dy, nsub)
    x = torch.ones(os_.plans[0].vol_shape, device=DEV)
    os_.run(x, to_dev(y), to_dev(r), iters=2)
    torch.cuda.synchronize()
    err = rel_l2(x.cpu().numpy(), ref)
    print(f"osem 4x2: rel L2 {err:.2e}", flush=True)
    assert err <= TOL
