"""GPU against the FP64 oracle at the sizes of the differentiation and
precision workloads, through the C ABI.

Sec. II-B trains unrolled EM by backpropagating through the projector and
its exact adjoint; Eq. (7)-(8) with beta -> 0 is the ML-EM update.  The
problems follow the differentiation workload: the body phantom as x_true,
y ~ Poisson(A x_true + r) with r = 5% of the mean of A x_true (uniform),
x0 uniform at the mean of x_true, 10 EM iterations, MSE loss against
x_true.  The oracle runs the FFT form of its projector over a process pool
of views (the same operator, pinned to the direct form to 1e-12), and its
chain rule is pinned by finite differences on the CPU.

Bars.
* FP32 GPU: x_10, dL/dx0 and dL/dy within 1e-5 relative L2 of the oracle
  (the projector's bar; the GPU chain is four FP32 projector directions per
  step, each about 1e-7 from the oracle).
* 10-iteration EM images per convolution precision, each precision's plan
  computing its own sensitivity A'1: FP32 within 1e-5; BF16 and FP16 within
  10u (u = 2^-8, 2^-11).  Each product has two rounded operands (2u
  relative at most), so one projector direction is within 2u and an EM
  update, a ratio of projections times a back projection divided by the
  sensitivity, moves by at most a few u per iteration; the rounding errors
  of different taps are independent and mostly cancel in the sums, and the
  EM map damps perturbations of the iterate, so 10u over 10 iterations is a
  stated bound with margin, not a tight one.
* Split BF16 (a = a1 + a2, a1 = bf16(a), a2 = bf16(a - a1), so
  |a - a1 - a2| <= 2^-16 |a|; products a1 b1 + a1 b2 + a2 b1): each product
  is within 3 * 2^-16 of a b (two representation errors and the dropped
  a2 b2).  The PSF's representation error is the same for every voxel a
  tap meets, so it does not cancel in the sums: one projector direction is
  within 3 * 2^-16 and the EM images within 5 times that (the ratio of the
  per-direction and EM bounds of the plain formats).
"""
import os
import sys

import numpy as np
import pytest

from oracle import em, precision
from oracle.pool import OraclePool
from oracle.projector import Geometry
from paper_2301_09710_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2301_09710_amd import autograd as sag  # noqa: E402
from paper_2301_09710_amd import spect  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5
ITERS = 10
SPLIT = 3 * 2.0 ** -16        # split BF16, one projector direction


def em_bound(prec):
    if prec == "fp32":
        return TOL
    if prec == "bf16x3":
        return 5 * SPLIT
    return 10 * precision.unit_roundoff(prec)


def direction_bound(prec):
    if prec == "fp32":
        return TOL
    if prec == "bf16x3":
        return SPLIT
    return 2 * precision.unit_roundoff(prec)


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
    return t.detach().cpu().numpy()


def _oracle_problem(name, seed=0):
    """Inputs (FP32-representable) and the oracle's unrolled-EM results."""
    c = synth.CONFIGS[name]
    x, mu, psf, dy = synth.config_inputs(name, seed=seed)
    g = Geometry(c["nx"], c["ny"], c["nz"], c["nview"], c["px"], c["pz"], dy)
    P = dict(name=name, x=x, mu=mu, psf=psf, dy=dy, g=g)
    with OraclePool(mu, psf, g, conv="fft") as pool:
        say(f"{name}: oracle over {pool.workers} processes")
        yc = pool.forward(x)
        r = np.full(yc.shape, 0.05 * yc.mean(), dtype=np.float32)
        y = synth.poisson_counts(yc + r, seed=seed + 3)
        sens = pool.back(np.ones(yc.shape)).astype(np.float32)
        x0 = np.full(x.shape, x.mean(), dtype=np.float32)
        xt = x.astype(np.float64)

        def loss_grad(xk):
            d = xk - xt
            return float((d * d).mean()), 2.0 * d / d.size

        xK, loss, gx0, gy = em.unrolled_mlem_grad(x0, y, r, sens, pool.forward, pool.back,
                                                  ITERS, loss_grad)
        P.update(yc=yc, r=r, y=y, sens=sens, x0=x0, xK=xK, loss=loss, gx0=gx0, gy=gy)
        say(f"{name}: oracle done")
    return P


@pytest.fixture(scope="module", params=[
    pytest.param("serve64", id="64x64x40"),
    pytest.param("paper", id="128x128x80", marks=[pytest.mark.slow, pytest.mark.timeout(1200)]),
])
def prob(request):
    return _oracle_problem(request.param)


@pytest.mark.timeout(1200)
def test_unrolled_em_gradient_vs_oracle(prob):
    """x_10, dL/dx0 and dL/dy of 10 unrolled EM iterations (autograd through
    spect_em_step / spect_em_step_vjp, the plan the benchmark times) against
    the oracle's chain rule."""
    say(f"unrolled gradient {prob['name']}")
    plan = spect.Plan(to_dev(prob["mu"]), to_dev(prob["psf"]), prob["dy"], cache_mubar=True)
    x0d = to_dev(prob["x0"]).requires_grad_(True)
    yd = to_dev(prob["y"]).requires_grad_(True)
    xK = sag.unrolled_mlem(plan, x0d, yd, to_dev(prob["sens"]), to_dev(prob["r"]), iters=ITERS)
    loss = ((xK - to_dev(prob["x"])) ** 2).mean()
    loss.backward()
    e_x = rel_l2(host(xK), prob["xK"])
    e_gx = rel_l2(host(x0d.grad), prob["gx0"])
    e_gy = rel_l2(host(yd.grad), prob["gy"])
    e_l = abs(float(loss.detach()) - prob["loss"]) / prob["loss"]
    say(f"{prob['name']} unrolled x{ITERS}: x_K {e_x:.2e}, loss {e_l:.2e}, dx0 {e_gx:.2e}, "
        f"dy {e_gy:.2e}")
    assert e_x <= TOL and e_l <= TOL
    assert e_gx <= TOL and e_gy <= TOL
    plan.close()


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3"])
def test_em_ten_iterations_vs_oracle(prob, prec):
    """10-iteration EM image of each convolution precision against the FP64
    oracle's (Eq. (7)-(8), beta -> 0), each plan with its own A'1."""
    plan = spect.Plan(to_dev(prob["mu"]), to_dev(prob["psf"]), prob["dy"], cache_mubar=True,
                      precision=prec)
    sens = plan.back(torch.ones(plan.proj_shape, device=DEV))
    xd = to_dev(prob["x0"])
    yd, rd = to_dev(prob["y"]), to_dev(prob["r"])
    for _ in range(ITERS):
        plan.em_step(xd, yd, sens, rd)
    e = rel_l2(host(xd), prob["xK"])
    bound = em_bound(prec)
    say(f"{prob['name']} {prec} EM x{ITERS} vs oracle: {e:.2e} (bound {bound:.2e})")
    assert e <= bound
    plan.close()


@pytest.mark.slow
@pytest.mark.timeout(3000)
@pytest.mark.skipif(os.environ.get("SPECT_ORACLE_LARGE") != "1",
                    reason="the 256x256x160 oracle references take about three minutes on "
                           "16 host cores; run with SPECT_ORACLE_LARGE=1")
def test_large_precision_vs_oracle():
    """The 256x256x160 / 128-view / 37x37 precision workload: forward of x_true,
    back of y and the 10-iteration EM image, each precision against the FP64
    oracle (full volumes and sinograms)."""
    c = synth.CONFIGS["large"]
    x, mu, psf, dy = synth.config_inputs("large", seed=0)
    g = Geometry(c["nx"], c["ny"], c["nz"], c["nview"], c["px"], c["pz"], dy)
    with OraclePool(mu, psf, g, conv="fft") as pool:
        say(f"large: oracle over {pool.workers} processes")
        yc = pool.forward(x)
        r = np.full(yc.shape, 0.05 * yc.mean(), dtype=np.float32)
        y = synth.poisson_counts(yc + r, seed=3)
        b_ref = pool.back(y)
        sens = pool.back(np.ones(yc.shape))
        xk = np.full(x.shape, x.mean(), dtype=np.float32).astype(np.float64)
        for it in range(ITERS):
            xk = em.mlem_step(xk, y, r, sens, pool.forward, pool.back)
            say(f"large: oracle EM iteration {it + 1}")
    x0 = np.full(x.shape, x.mean(), dtype=np.float32)
    worst = {}
    for prec in ("fp32", "bf16", "fp16", "bf16x3"):
        plan = spect.Plan(to_dev(mu), to_dev(psf), dy, cache_mubar=True, precision=prec)
        ef = rel_l2(host(plan.forward(to_dev(x))), yc)
        eb = rel_l2(host(plan.back(to_dev(y))), b_ref)
        s = plan.back(torch.ones(plan.proj_shape, device=DEV))
        xd, yd, rd = to_dev(x0), to_dev(y), to_dev(r)
        for _ in range(ITERS):
            plan.em_step(xd, yd, s, rd)
        ee = rel_l2(host(xd), xk)
        bound = em_bound(prec)
        fb_bound = direction_bound(prec)
        say(f"large {prec} vs oracle: forward {ef:.2e}, back {eb:.2e}, EM x{ITERS} {ee:.2e}")
        worst[prec] = (ef, eb, ee, fb_bound, bound)
        plan.close()
        del plan, s, xd
        torch.cuda.empty_cache()
    for prec, (ef, eb, ee, fb, b) in worst.items():
        assert ef <= fb and eb <= fb and ee <= b, prec
