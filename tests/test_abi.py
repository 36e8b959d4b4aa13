"""C-ABI checks that need no GPU: the library loads, exports every function
include/spect.h declares, and rejects bad arguments synchronously, before
any HIP call (so these run on a machine without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2301_09710_amd import spect

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spect.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spect_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = spect.load()
    names = declared_functions()
    assert {"spect_plan_create", "spect_forward", "spect_back", "spect_em_step"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(spect.EXPORTED)
    assert "gfx950" in spect.spect_version()


def test_plan_describe_rejects_null():
    lib = spect.load()
    buf = ctypes.create_string_buffer(64)
    assert lib.spect_plan_describe(None, buf, 64) == 1
    assert lib.spect_plan_describe(ctypes.c_void_p(1), None, 64) == 1


def test_status_strings():
    lib = spect.load()
    for s in range(8):
        assert lib.spect_status_string(s)
    assert lib.spect_status_string(0) == b"ok"


@pytest.mark.parametrize("kw,status", [
    (dict(ny=30), 2),                 # nx != ny
    (dict(px=6), 2),                  # even PSF
    (dict(pz=0), 2),
    (dict(nz=0), 2),
    (dict(nview=0), 2),
    (dict(dy=0.0), 3),
    (dict(dy=float("nan")), 3),
    (dict(flags=0x200), 3),           # unknown flag bit
    (dict(flags=0x18), 3),            # all taps and stated symmetry together
    (dict(flags=0x60), 3),            # both FP32 tilings together
    (dict(flags=0x4, conv_precision=1), 5),   # separable PSFs: FP32 only
    (dict(view_batch=-1), 3),
    (dict(nx=300, ny=300), 5),        # in-plane size above the largest supported (256)
])
def test_workspace_bytes_validation(kw, status):
    args = dict(nx=32, ny=32, nz=20, nview=16, px=7, pz=7, dy=1.0, angles=None, flags=0, view_batch=0)
    args.update(kw)
    g, _keep = spect.make_geom(**args)
    with pytest.raises(spect.SpectError) as e:
        spect.spect_workspace_bytes(g)
    assert e.value.status == status


def test_rotation_flag_accepted_with_the_same_workspace():
    """SPECT_ROT_BILINEAR only changes the rotation tables' meaning: the
    workspace is the same size, alone and with the attenuation cache."""
    ws = lambda f: spect.spect_workspace_bytes(spect.make_geom(32, 32, 20, 16, 7, 7, 1.0, flags=f)[0])
    assert ws(spect.SPECT_ROT_BILINEAR) == ws(0)
    assert ws(spect.SPECT_ROT_BILINEAR | spect.SPECT_CACHE_MUBAR) == ws(spect.SPECT_CACHE_MUBAR)


def test_nonfinite_angle_rejected():
    g, _keep = spect.make_geom(8, 8, 6, 3, 3, 3, 1.0, angles=[0.0, float("inf"), 1.0])
    with pytest.raises(spect.SpectError) as e:
        spect.spect_workspace_bytes(g)
    assert e.value.status == 3


def test_workspace_grows_with_cache_and_shrinks_with_batch():
    """The attenuation cache holds every view; without it a buffer for one view
    batch is kept instead.  Smaller view batches shrink the per-batch buffers."""
    N = 128 * 128 * 80 * 4
    ws = lambda **kw: spect.spect_workspace_bytes(spect.make_geom(128, 128, 80, 128, 37, 37, 4.8, **kw)[0])
    b_all = ws()
    b_all_cache = ws(flags=spect.SPECT_CACHE_MUBAR)
    b16 = ws(view_batch=16)
    b16_cache = ws(view_batch=16, flags=spect.SPECT_CACHE_MUBAR)
    assert b_all_cache == b_all                    # batch = all views: same size either way
    assert b16_cache - b16 == (128 - 16) * N       # cache of 128 views replaces a 16-view batch
    assert b16 < b_all - 200 * N                   # W and mubar batch buffers both shrink
    assert all(b % 256 == 0 for b in (b_all, b_all_cache, b16, b16_cache))


def test_plan_create_rejects_before_any_gpu_call():
    lib = spect.load()
    g, _ = spect.make_geom(32, 32, 20, 16, 7, 7, 1.0)
    need = spect.spect_workspace_bytes(g)
    fake = 1 << 40                      # never dereferenced: validation fails first
    plan = ctypes.c_void_p(0)
    # null pointers
    assert lib.spect_plan_create(ctypes.byref(plan), ctypes.byref(g), None, fake, fake, need, None) == 1
    assert lib.spect_plan_create(None, ctypes.byref(g), fake, fake, fake, need, None) == 1
    # workspace too small
    assert lib.spect_plan_create(ctypes.byref(plan), ctypes.byref(g), fake, fake, fake,
                                 need - 1, None) == 4
    # misaligned workspace / mu
    assert lib.spect_plan_create(ctypes.byref(plan), ctypes.byref(g), fake, fake, fake + 16,
                                 need, None) == 7
    assert lib.spect_plan_create(ctypes.byref(plan), ctypes.byref(g), fake + 2, fake, fake,
                                 need, None) == 7
    # bad geometry
    gb, _ = spect.make_geom(32, 32, 20, 16, 8, 7, 1.0)
    assert lib.spect_plan_create(ctypes.byref(plan), ctypes.byref(gb), fake, fake, fake,
                                 need, None) == 2
    assert plan.value is None


def test_entry_points_reject_null():
    lib = spect.load()
    fake = 1 << 40
    assert lib.spect_forward(None, fake, fake, None) == 1
    assert lib.spect_back(None, fake, fake, None) == 1
    assert lib.spect_em_step(None, fake, fake, None, fake, None) == 1
    assert lib.spect_reg_em_step(None, fake, fake, None, fake, fake, 0.5, None) == 1
    assert lib.spect_em_step_vjp(None, fake, fake, None, fake, fake, fake, None, None) == 1
    # a non-null fake plan pointer is never dereferenced before argument checks
    assert lib.spect_reg_em_step(fake, fake, fake, None, fake, None, 0.5, None) == 1
    assert lib.spect_reg_em_step(fake, fake, fake, None, fake, fake, -1.0, None) == 3
    assert lib.spect_reg_em_step(fake, fake, fake, None, fake, fake, float("nan"), None) == 3
    assert lib.spect_em_step_vjp(fake, fake, fake, None, fake, fake, None, None, None) == 1
    assert lib.spect_plan_destroy(None) == 1
    assert lib.spect_dot_f64(None, fake, 4, fake, None) == 1
    assert lib.spect_dot_f64(fake, fake, 4, fake + 4, None) == 7


def test_conv_precision_validation():
    for prec in (0, 1, 2, 3):
        g, _ = spect.make_geom(32, 32, 20, 16, 7, 7, 1.0, conv_precision=prec)
        assert spect.spect_workspace_bytes(g) > 0
    for bad in (-1, 4, 99):
        g, _ = spect.make_geom(32, 32, 20, 16, 7, 7, 1.0, conv_precision=bad)
        with pytest.raises(spect.SpectError) as e:
            spect.spect_workspace_bytes(g)
        assert e.value.status == 3


def test_plan_choice_flags_keep_the_workspace():
    """The tap-pairing and tiling flags only change kernel selection."""
    ws = lambda f: spect.spect_workspace_bytes(spect.make_geom(32, 32, 20, 16, 7, 7, 1.0, flags=f)[0])
    for f in (spect.SPECT_PSF_ALL_TAPS, spect.SPECT_PSF_SYMMETRIC_X, spect.SPECT_TILING_4X4,
              spect.SPECT_TILING_16X16, spect.SPECT_PSF_SYMMETRIC_X | spect.SPECT_TILING_4X4):
        assert ws(f) == ws(0)


def test_direct_convolution_shape_is_accepted_in_fp32_only():
    """PSFs taller than the matrix-core tiles hold (pz >= 67) run on the plain
    FP32 kernels; the reduced-precision forms need the tiles."""
    g, _ = spect.make_geom(32, 32, 80, 16, 9, 69, 1.0)
    assert spect.spect_workspace_bytes(g) > 0
    for prec in (1, 2, 3):
        g, _ = spect.make_geom(32, 32, 80, 16, 9, 69, 1.0, conv_precision=prec)
        with pytest.raises(spect.SpectError) as e:
            spect.spect_workspace_bytes(g)
        assert e.value.status == 5


def test_static_forward_rejects_before_any_gpu_call():
    """spect_forward_static validates the geometry and checks that its
    workspace fits the library's static array before touching a device."""
    lib = spect.load()
    fake = 1 << 40
    g, _ = spect.make_geom(128, 128, 80, 128, 37, 37, 4.8)          # 1.4 GiB of workspace
    assert lib.spect_forward_static(ctypes.byref(g), fake, fake, fake, fake, None) == 4
    g, _keep = spect.make_geom(16, 16, 8, 3, 3, 3, 1.0, angles=[0.0, 1.0, 2.0])
    assert lib.spect_forward_static(ctypes.byref(g), fake, fake, fake, fake, None) == 5
    g, _ = spect.make_geom(16, 16, 8, 3, 4, 3, 1.0)                   # even PSF
    assert lib.spect_forward_static(ctypes.byref(g), fake, fake, fake, fake, None) == 2
    g, _ = spect.make_geom(16, 16, 8, 3, 3, 3, 1.0)
    assert lib.spect_forward_static(ctypes.byref(g), None, fake, fake, fake, None) == 1
    assert lib.spect_forward_static(ctypes.byref(g), fake, fake, fake + 2, fake, None) == 7


def test_fft_flag_validation_and_workspace():
    """SPECT_CONV_FFT: FP32 only, not with separable PSFs; the plan keeps the
    PSF spectra, so the workspace grows by at least nview * ny spectra."""
    base, _ = spect.make_geom(128, 128, 80, 128, 37, 37, 4.8)
    fft, _ = spect.make_geom(128, 128, 80, 128, 37, 37, 4.8, flags=spect.SPECT_CONV_FFT)
    b0, b1 = spect.spect_workspace_bytes(base), spect.spect_workspace_bytes(fft)
    # 180 x 120 transforms: 89 x 120 + 2 x 61 complex slots per PSF
    assert b1 - b0 >= 128 * 128 * (89 * 120 + 122) * 8
    for kw in (dict(conv_precision=1), dict(conv_precision=3),
               dict(flags=spect.SPECT_CONV_FFT | spect.SPECT_PSF_SEPARABLE)):
        args = dict(flags=spect.SPECT_CONV_FFT)
        args.update(kw)
        g, _ = spect.make_geom(32, 32, 20, 16, 7, 7, 1.0, **args)
        with pytest.raises(spect.SpectError) as e:
            spect.spect_workspace_bytes(g)
        assert e.value.status == 5
    g, _ = spect.make_geom(256, 256, 160, 128, 37, 37, 2.4, flags=spect.SPECT_CONV_FFT)
    with pytest.raises(spect.SpectError) as e:      # 300 x 200 transforms exceed LDS
        spect.spect_workspace_bytes(g)
    assert e.value.status == 5


def test_fft_real_spectra_workspace():
    """SPECT_PSF_SYMMETRIC_X | SPECT_PSF_SYMMETRIC_Z with SPECT_CONV_FFT on a
    compiled-in transform size keeps one float per spectrum bin: the
    workspace shrinks by exactly half the spectra; on a run-time size (or
    with one of the two flags) nothing changes; without SPECT_CONV_FFT the
    flag is accepted and changes nothing."""
    sym = spect.SPECT_PSF_SYMMETRIC_X | spect.SPECT_PSF_SYMMETRIC_Z
    def ws(nx, nz, nview, p, flags):
        g, _ = spect.make_geom(nx, nx, nz, nview, p, p, 4.8, flags=flags)
        return spect.spect_workspace_bytes(g)
    F = spect.SPECT_CONV_FFT
    full, real = ws(128, 80, 128, 37, F), ws(128, 80, 128, 37, F | sym)
    spectra = 128 * 128 * (89 * 120 + 122) * 8                # complex, 256-byte aligned
    assert abs((full - real) - spectra // 2) <= 512
    assert ws(128, 80, 128, 37, F | spect.SPECT_PSF_SYMMETRIC_X) == full
    assert ws(128, 80, 128, 37, F | spect.SPECT_PSF_SYMMETRIC_Z) == full
    assert ws(32, 20, 16, 7, F | sym) == ws(32, 20, 16, 7, F)  # 40 x 30: run-time sizes
    assert ws(32, 20, 16, 7, spect.SPECT_PSF_SYMMETRIC_Z) == ws(32, 20, 16, 7, 0)
