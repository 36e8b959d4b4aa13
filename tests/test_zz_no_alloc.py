"""spect_forward_static, the forward projection that allocates nothing (its
workspace is the library's static device array), through the C ABI against
spect_forward on a plan of the same geometry and against the FP64 oracle,
on calls in a row whose inputs shrink (the array keeps the previous call's
contents), and with every plan-choice flag it honours.

Bar: 1e-5 relative L2 (the FP32 projector's bar against the oracle); the
rotation tables are computed on the device here and on the host for a plan,
from the same FP64 formulas.
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
SCRATCH = 64 << 20


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def fitting_view_batch(nx, nz, nview, px, pz, dy, flags):
    """The largest view batch whose workspace fits the static array."""
    for vb in range(nview, 0, -1):
        g, _ = spect.make_geom(nx, nx, nz, nview, px, pz, dy, flags=flags, view_batch=vb)
        if spect.spect_workspace_bytes(g) <= SCRATCH:
            return vb
    raise AssertionError("no view batch fits")


def static_forward(x, mu, psf, dy, flags, view_batch):
    nz, ny, nx = x.shape
    nview, _, pz, px = psf.shape
    g, _ = spect.make_geom(nx, ny, nz, nview, px, pz, dy, flags=flags, view_batch=view_batch)
    xd, mud, psfd = to_dev(x), to_dev(mu), to_dev(psf)
    v = torch.full((nview, nz, nx), float("nan"), device=DEV)
    say(f"spect_forward_static {nx}x{ny}x{nz} views {nview} psf {px}x{pz} flags {flags:#x} "
        f"view_batch {view_batch}")
    spect.spect_forward_static(g, mud.data_ptr(), psfd.data_ptr(), xd.data_ptr(), v.data_ptr(),
                               torch.cuda.current_stream(DEV).cuda_stream)
    torch.cuda.synchronize()
    return v.cpu().numpy()


def plan_forward(x, mu, psf, dy, **kw):
    plan = spect.Plan(to_dev(mu), to_dev(psf), dy, **kw)
    v = plan.forward(to_dev(x))
    torch.cuda.synchronize()
    out = v.cpu().numpy()
    plan.close()
    return out


CASES = [
    # name, x/mu/psf maker, plan keywords, flags
    ("serve64-symmetric", "serve64", dict(mirror="assume"), spect.SPECT_PSF_SYMMETRIC_X),
    ("tiny-all-taps", "tiny", dict(mirror="off"), 0),
    ("16x16x8-asymmetric", "small", dict(mirror="off"), 0),
    ("tiny-bilinear", "tiny", dict(mirror="assume", rotation="bilinear"),
     spect.SPECT_PSF_SYMMETRIC_X | spect.SPECT_ROT_BILINEAR),
    ("tiny-fft", "tiny", dict(method="fft"), spect.SPECT_CONV_FFT),
    ("16x16x8-fft", "small", dict(method="fft"), spect.SPECT_CONV_FFT),
    ("serve64-fft-real", "serve64-16", dict(method="fft", mirror="assume", symmetric_z=True),
     spect.SPECT_CONV_FFT | spect.SPECT_PSF_SYMMETRIC_X | spect.SPECT_PSF_SYMMETRIC_Z),
]


def _inputs(which):
    if which == "serve64-16":      # the 64x64x40 / 19x19 size (90 x 60 transforms), 16 views
        x, mu, psf, dy = synth.config_inputs("serve64", seed=1)
        return x, mu, np.ascontiguousarray(psf[::4]), dy
    if which == "small":
        x = synth.random_volume(16, 16, 8, seed=3)
        mu = synth.random_volume(16, 16, 8, seed=4, high=0.05)
        psf = synth.random_psf(5, 5, 16, 8, seed=5, symmetric=False)
        return x, mu, psf, 1.5
    return synth.config_inputs(which, seed=1)


def test_static_forward_matches_plan_and_oracle_on_shrinking_calls():
    """Calls in a row, largest first: each must match the plan's forward and
    the oracle whatever the previous call left in the array."""
    for name, which, kw, flags in CASES:
        x, mu, psf, dy = _inputs(which)
        nz, ny, nx = x.shape
        nview, _, pz, px = psf.shape
        vb = fitting_view_batch(nx, nz, nview, px, pz, dy, flags)
        v = static_forward(x, mu, psf, dy, flags, vb)
        assert np.isfinite(v).all(), name
        ref_plan = plan_forward(x, mu, psf, dy, **kw)
        rot = "bilinear" if flags & spect.SPECT_ROT_BILINEAR else "3pass"
        g = Geometry(nx, ny, nz, nview, px, pz, dy, rotation=rot)
        ref = oracle.forward(x, mu, psf, g, conv="fft" if nx >= 64 else "direct")
        ep, eo = rel_l2(v, ref_plan), rel_l2(v, ref)
        say(f"{name}: view_batch {vb}, vs plan {ep:.2e}, vs oracle {eo:.2e}")
        assert ep <= TOL and eo <= TOL, name


def test_static_forward_twice_smaller_second():
    """The same two geometries twice in a row, the second call smaller: the
    results repeat bit for bit (deterministic kernels, nothing carried over)."""
    first = _inputs("tiny")
    second = _inputs("small")
    f1 = static_forward(*first, 0, 0)
    s1 = static_forward(*second, 0, 0)
    f2 = static_forward(*first, 0, 0)
    s2 = static_forward(*second, 0, 0)
    assert np.array_equal(f1, f2) and np.array_equal(s1, s2)
    assert rel_l2(s1, plan_forward(*second, mirror="off")) <= TOL
