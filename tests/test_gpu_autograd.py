"""GPU differentiation through the projector and unrolled EM (Sec. II-B:
the unrolled EM network is trained by backpropagation through the exact
adjoint), through the C ABI, against the FP64 oracle's chain rule (itself
pinned by finite differences in test_oracle_grad_pins.py).

Tolerances.  Projector gradients are one projector direction: the 1e-5
relative-L2 bar of the projector applies.  The EM vector-Jacobian product
chains four FP32 projector directions (each about 1e-7 relative L2 here)
with divisions by ybar = A x + r; through 10 unrolled iterations the
gradients stay within a few 1e-6, and GRAD_TOL holds them to the same 1e-5
bar as the projector.
"""
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

from paper_2301_09710_amd import autograd as sag  # noqa: E402
from paper_2301_09710_amd import spect  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5
GRAD_TOL = 1e-5


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


def _problem(nx, nz, nview, p, seed=0, counts=20.0):
    """Body phantom, Poisson data with 5% uniform background; FP32-representable."""
    x, mu = synth.body_phantom(nx, nx, nz, seed=seed)
    psf = synth.gaussian_psf(p, p, nx, nview, 0.5, 1.5, view_wobble=0.1)
    dy = 4.8 * 128 / nx
    g = Geometry(nx, nx, nz, nview, p, p, dy)
    xt = (x + 0.1).astype(np.float32)
    yc = oracle.forward(xt, mu, psf, g)
    r = np.full(yc.shape, 0.05 * yc.mean(), dtype=np.float32)
    y = synth.poisson_counts(yc * counts + r, seed=seed + 3).astype(np.float32)
    return dict(xt=xt, mu=mu, psf=psf, dy=dy, g=g, y=y, r=r)


def _oracle_ops(P):
    def A(v):
        return oracle.forward(np.asarray(v).reshape(P["g"].nz, P["g"].ny, P["g"].nx),
                              P["mu"], P["psf"], P["g"])

    def At(v):
        return oracle.back(v, P["mu"], P["psf"], P["g"])
    return A, At


@pytest.fixture(scope="module", params=[(16, 8, 8, 5), (32, 20, 16, 7)], ids=["16x16x8", "tiny"])
def prob(request):
    nx, nz, nview, p = request.param
    say(f"autograd problem {request.param}")
    P = _problem(nx, nz, nview, p)
    P["plan"] = spect.Plan(to_dev(P["mu"]), to_dev(P["psf"]), P["dy"])
    A, At = _oracle_ops(P)
    P["A"], P["At"] = A, At
    P["sens"] = At(np.ones(P["y"].shape)).astype(np.float32)
    return P


def test_project_backward_is_back_projector(prob):
    plan = prob["plan"]
    x = to_dev(prob["xt"]).requires_grad_(True)
    w = np.random.default_rng(5).uniform(0.5, 1.5, size=prob["y"].shape).astype(np.float32)
    loss = (sag.project(plan, x) * to_dev(w)).sum()
    loss.backward()
    gx = host(x.grad)
    np.testing.assert_array_equal(gx, host(plan.back(to_dev(w))))
    assert rel_l2(gx, prob["At"](w)) <= TOL
    v = to_dev(w).requires_grad_(True)
    (sag.backproject(plan, v) * to_dev(prob["xt"])).sum().backward()
    assert rel_l2(host(v.grad), prob["A"](prob["xt"])) <= TOL


def test_em_step_forward_and_vjp_parity(prob):
    plan, A, At = prob["plan"], prob["A"], prob["At"]
    rng = np.random.default_rng(7)
    x = (prob["xt"].mean() * rng.uniform(0.5, 1.5, size=prob["xt"].shape)).astype(np.float32)
    g = rng.normal(size=x.shape).astype(np.float32)
    xd = to_dev(x).requires_grad_(True)
    yd = to_dev(prob["y"]).requires_grad_(True)
    out = sag.em_step(plan, xd, yd, to_dev(prob["sens"]), to_dev(prob["r"]))
    ref = em.mlem_step(x, prob["y"], prob["r"], prob["sens"], A, At)
    e_fwd = rel_l2(host(out), ref)
    out.backward(to_dev(g))
    gx_ref, gy_ref = em.mlem_step_vjp(x, prob["y"], prob["r"], prob["sens"], g, A, At)
    e_gx, e_gy = rel_l2(host(xd.grad), gx_ref), rel_l2(host(yd.grad), gy_ref)
    say(f"em step rel L2: forward {e_fwd:.2e}, dx {e_gx:.2e}, dy {e_gy:.2e}")
    assert e_fwd <= TOL
    assert e_gx <= GRAD_TOL and e_gy <= GRAD_TOL


def test_unrolled_mlem_gradient_parity(prob):
    plan, A, At = prob["plan"], prob["A"], prob["At"]
    iters = 10
    xt = prob["xt"]
    x0 = np.full_like(xt, xt.mean())

    def loss_grad(xk):
        d = xk - xt
        return float((d * d).mean()), 2.0 * d / d.size

    xK_ref, loss_ref, gx0_ref, gy_ref = em.unrolled_mlem_grad(
        x0, prob["y"], prob["r"], prob["sens"], A, At, iters, loss_grad)
    x0d = to_dev(x0).requires_grad_(True)
    yd = to_dev(prob["y"]).requires_grad_(True)
    xK = sag.unrolled_mlem(plan, x0d, yd, to_dev(prob["sens"]), to_dev(prob["r"]), iters=iters)
    loss = ((xK - to_dev(xt)) ** 2).mean()
    loss.backward()
    e_x = rel_l2(host(xK), xK_ref)
    e_gx, e_gy = rel_l2(host(x0d.grad), gx0_ref), rel_l2(host(yd.grad), gy_ref)
    say(f"unrolled x10 rel L2: x_K {e_x:.2e}, loss {abs(float(loss) - loss_ref) / loss_ref:.2e}, "
        f"dx0 {e_gx:.2e}, dy {e_gy:.2e}")
    assert e_x <= GRAD_TOL
    assert abs(float(loss) - loss_ref) <= GRAD_TOL * loss_ref
    assert e_gx <= GRAD_TOL and e_gy <= GRAD_TOL


def test_em_step_vjp_in_place_gradient_buffer(prob):
    """d_gx may equal d_g: the in-place call gives the same result."""
    plan = prob["plan"]
    rng = np.random.default_rng(9)
    x = to_dev(prob["xt"])
    y, sens, r = to_dev(prob["y"]), to_dev(prob["sens"]), to_dev(prob["r"])
    g = to_dev(rng.normal(size=prob["xt"].shape))
    gx, gy = plan.em_step_vjp(x, y, sens, g, r)
    g2 = g.clone()
    spect.spect_em_step_vjp(plan._plan, x.data_ptr(), y.data_ptr(), r.data_ptr(), sens.data_ptr(),
                            g2.data_ptr(), g2.data_ptr(), None,
                            torch.cuda.current_stream(DEV).cuda_stream)
    np.testing.assert_array_equal(host(g2), host(gx))


def test_unrolled_gradient_paper_size_directional():
    """128x128x80, 128 views, 37x37 PSFs, 3 unrolled iterations: the GPU
    gradient against a central finite difference of the GPU loss along a
    random direction (a property that holds at any size; FP32 loss
    evaluations limit the agreement to about 1e-3)."""
    say("paper-size unrolled gradient")
    x, mu, psf, dy = synth.config_inputs("paper", seed=0)
    plan = spect.Plan(to_dev(mu), to_dev(psf), dy, cache_mubar=True)
    xt = to_dev(x)
    with torch.no_grad():
        yc = plan.forward(xt)
        r = torch.full_like(yc, 0.05 * float(yc.mean()))
        y = torch.poisson((yc * 5.0 + r).clamp_min(0.0))
        sens = plan.back(torch.ones_like(yc))
    x0 = torch.full_like(xt, float(xt.mean()))

    def loss_of(z0):
        with torch.no_grad():
            z = sag.unrolled_mlem(plan, z0, y, sens, r, iters=3)
            return float(((z.double() - xt.double()) ** 2).mean())

    x0g = x0.clone().requires_grad_(True)
    zK = sag.unrolled_mlem(plan, x0g, y, sens, r, iters=3)
    ((zK - xt) ** 2).mean().backward()
    gen = torch.Generator(device=DEV).manual_seed(11)
    d = torch.randn(x0.shape, device=DEV, generator=gen) * float(x0.mean())
    eps = 1e-2
    fd = (loss_of(x0 + eps * d) - loss_of(x0 - eps * d)) / (2 * eps)
    an = float((x0g.grad.double() * d.double()).sum())
    say(f"paper-size directional derivative: fd {fd:.6e} analytic {an:.6e}")
    assert abs(fd - an) <= 1e-2 * abs(fd)
