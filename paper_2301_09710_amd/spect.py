"""ctypes binding of libspect (include/spect.h).

Argument marshalling only: every step of the projector runs in the HIP
kernels of libspect.so.  PyTorch supplies device memory and the stream.
The functions ``spect_*`` mirror the C ABI one to one (raw device pointers
as ints); ``Plan`` wraps them for torch tensors.

If libspect.so is missing this module raises at first use: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_size_t, c_uint32, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspect.so")

SPECT_OK = 0
SPECT_CACHE_MUBAR = 0x1
SPECT_ROT_BILINEAR = 0x2
SPECT_PSF_SEPARABLE = 0x4
SPECT_PSF_ALL_TAPS = 0x8
SPECT_PSF_SYMMETRIC_X = 0x10
SPECT_TILING_4X4 = 0x20
SPECT_TILING_16X16 = 0x40
SPECT_CONV_FFT = 0x80
SPECT_PSF_SYMMETRIC_Z = 0x100
METHODS = {"direct": 0, "fft": SPECT_CONV_FFT}
MIRRORS = {"auto": 0, "off": SPECT_PSF_ALL_TAPS, "assume": SPECT_PSF_SYMMETRIC_X}
TILINGS = {"auto": 0, "4x4": SPECT_TILING_4X4, "16x16": SPECT_TILING_16X16}
ROTATIONS = {"3pass": 0, "bilinear": SPECT_ROT_BILINEAR}
SPECT_CONV_FP32, SPECT_CONV_BF16, SPECT_CONV_FP16, SPECT_CONV_BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp32": SPECT_CONV_FP32, "bf16": SPECT_CONV_BF16, "fp16": SPECT_CONV_FP16,
              "bf16x3": SPECT_CONV_BF16X3}
STATUS_NAMES = {
    0: "SPECT_OK", 1: "SPECT_ERR_NULL", 2: "SPECT_ERR_SHAPE", 3: "SPECT_ERR_VALUE",
    4: "SPECT_ERR_WORKSPACE", 5: "SPECT_ERR_UNSUPPORTED", 6: "SPECT_ERR_HIP", 7: "SPECT_ERR_ALIGN",
}
EXPORTED = ("spect_workspace_bytes", "spect_plan_create", "spect_forward", "spect_back",
            "spect_em_step", "spect_reg_em_step", "spect_em_step_vjp", "spect_plan_destroy", "spect_status_string", "spect_dot_f64",
            "spect_profile_start", "spect_profile_stop", "spect_version", "spect_plan_describe",
            "spect_forward_static")


class SpectError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} "
                         f"({_lib().spect_status_string(status).decode()})")


class spect_geom(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("nview", c_int32),
                ("px", c_int32), ("pz", c_int32), ("dy", c_double),
                ("angles", POINTER(c_double)), ("flags", c_uint32), ("view_batch", c_int32),
                ("conv_precision", c_int32)]


class spect_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_int32), ("total_ms", c_double),
                ("min_ms", c_double), ("max_ms", c_double)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2301_09710_amd.build`"
                               " (there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        lib.spect_workspace_bytes.argtypes = [POINTER(spect_geom), POINTER(c_size_t)]
        lib.spect_plan_create.argtypes = [POINTER(c_void_p), POINTER(spect_geom), c_void_p, c_void_p,
                                          c_void_p, c_size_t, c_void_p]
        lib.spect_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        lib.spect_back.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        lib.spect_em_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        lib.spect_em_step_vjp.argtypes = [c_void_p] * 9
        lib.spect_reg_em_step.argtypes = [c_void_p] * 6 + [ctypes.c_float, c_void_p]
        lib.spect_plan_destroy.argtypes = [c_void_p]
        lib.spect_dot_f64.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]
        lib.spect_profile_start.argtypes = [c_void_p, c_int32]
        lib.spect_profile_stop.argtypes = [c_void_p, POINTER(spect_kernel_time), c_int32,
                                           POINTER(c_int32)]
        for name in ("spect_workspace_bytes", "spect_plan_create", "spect_forward", "spect_back",
                     "spect_em_step", "spect_reg_em_step", "spect_em_step_vjp", "spect_plan_destroy", "spect_dot_f64",
                     "spect_profile_start", "spect_profile_stop"):
            getattr(lib, name).restype = c_int
        lib.spect_status_string.argtypes = [c_int]
        lib.spect_status_string.restype = c_char_p
        lib.spect_version.argtypes = []
        lib.spect_version.restype = c_char_p
        lib.spect_plan_describe.argtypes = [c_void_p, ctypes.c_char_p, c_size_t]
        lib.spect_plan_describe.restype = c_int
        lib.spect_forward_static.argtypes = [POINTER(spect_geom), c_void_p, c_void_p, c_void_p,
                                             c_void_p, c_void_p]
        lib.spect_forward_static.restype = c_int
        _LIB = lib
    return _LIB


def load():
    """Load libspect.so (raises if it is not built)."""
    return _lib()


def make_geom(nx, ny, nz, nview, px, pz, dy, angles=None, flags=0, view_batch=0,
              conv_precision=SPECT_CONV_FP32):
    """Build a spect_geom; returns (geom, keepalive) -- keep the second item
    alive while the geom is in use (it owns the angles array)."""
    g = spect_geom(nx, ny, nz, nview, px, pz, float(dy), None, flags, view_batch, conv_precision)
    keep = None
    if angles is not None:
        keep = (c_double * nview)(*[float(a) for a in angles])
        g.angles = ctypes.cast(keep, POINTER(c_double))
    return g, keep


# ---------------------------------------------------------------- raw C ABI

def spect_workspace_bytes(geom: spect_geom) -> int:
    out = c_size_t(0)
    st = _lib().spect_workspace_bytes(ctypes.byref(geom), ctypes.byref(out))
    if st != SPECT_OK:
        raise SpectError(st, "spect_workspace_bytes")
    return out.value


def spect_plan_create(geom, d_mu: int, d_psf: int, d_ws: int, ws_bytes: int, stream: int) -> int:
    plan = c_void_p(0)
    st = _lib().spect_plan_create(ctypes.byref(plan), ctypes.byref(geom), d_mu, d_psf, d_ws,
                                  ws_bytes, stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_plan_create")
    return plan.value


def spect_forward(plan: int, d_x: int, d_v: int, stream: int) -> None:
    st = _lib().spect_forward(plan, d_x, d_v, stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_forward")


def spect_back(plan: int, d_v: int, d_x: int, stream: int) -> None:
    st = _lib().spect_back(plan, d_v, d_x, stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_back")


def spect_em_step(plan: int, d_x: int, d_y: int, d_r, d_sens: int, stream: int) -> None:
    st = _lib().spect_em_step(plan, d_x, d_y, d_r, d_sens, stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_em_step")


def spect_reg_em_step(plan: int, d_x: int, d_y: int, d_r, d_sens: int, d_u: int, beta: float,
                      stream: int) -> None:
    st = _lib().spect_reg_em_step(plan, d_x, d_y, d_r, d_sens, d_u, float(beta), stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_reg_em_step")


def spect_em_step_vjp(plan: int, d_x: int, d_y: int, d_r, d_sens: int, d_g: int, d_gx: int,
                      d_gy, stream: int) -> None:
    st = _lib().spect_em_step_vjp(plan, d_x, d_y, d_r, d_sens, d_g, d_gx, d_gy, stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_em_step_vjp")


def spect_forward_static(geom: spect_geom, d_mu: int, d_psf: int, d_x: int, d_v: int,
                         stream: int) -> None:
    st = _lib().spect_forward_static(ctypes.byref(geom), d_mu, d_psf, d_x, d_v, stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_forward_static")


def spect_plan_destroy(plan: int) -> None:
    st = _lib().spect_plan_destroy(plan)
    if st != SPECT_OK:
        raise SpectError(st, "spect_plan_destroy")


def spect_dot_f64(d_a: int, d_b: int, n: int, d_out: int, stream: int) -> None:
    st = _lib().spect_dot_f64(d_a, d_b, n, d_out, stream)
    if st != SPECT_OK:
        raise SpectError(st, "spect_dot_f64")


def spect_profile_start(plan: int, max_launches: int) -> None:
    st = _lib().spect_profile_start(plan, max_launches)
    if st != SPECT_OK:
        raise SpectError(st, "spect_profile_start")


def spect_profile_stop(plan: int) -> dict:
    """Returns {kernel name: dict(launches, total_ms, min_ms, max_ms)}."""
    out = (spect_kernel_time * 16)()
    n = c_int32(0)
    st = _lib().spect_profile_stop(plan, out, 16, ctypes.byref(n))
    if st != SPECT_OK:
        raise SpectError(st, "spect_profile_stop")
    return {out[i].name.decode(): dict(launches=out[i].launches, total_ms=out[i].total_ms,
                                       min_ms=out[i].min_ms, max_ms=out[i].max_ms)
            for i in range(n.value)}


def spect_version() -> str:
    return _lib().spect_version().decode()


def spect_plan_describe(plan: int) -> dict:
    """The plan's kernel selection as a dict of strings (host only)."""
    buf = ctypes.create_string_buffer(256)
    st = _lib().spect_plan_describe(plan, buf, len(buf))
    if st != 0:
        raise SpectError(st, "spect_plan_describe")
    return dict(kv.split("=", 1) for kv in buf.value.decode().split())


# ---------------------------------------------------------------- torch wrapper

def _stream(torch, device):
    return torch.cuda.current_stream(device).cuda_stream


def _check(t, shape, name, device):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device != device:
        raise ValueError(f"{name} must be contiguous float32 on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """A projector plan over torch tensors (borrowed mu / psf, owned workspace).

    x: [nz][ny][nx], v: [nview][nz][nx], mu: [nz][ny][nx], psf: [nview][ny][pz][px],
    or for separable PSFs p[b][a] = fz[b] fx[a] the pair (fz, fx) with
    fz: [nview][ny][pz] and fx: [nview][ny][px] (packed here into the
    [nview][ny][pz + px] layout of SPECT_PSF_SEPARABLE).

    mirror: "auto" (pair mirror-image taps when the device check finds every
    PSF row symmetric in x), "off" (SPECT_PSF_ALL_TAPS) or "assume"
    (SPECT_PSF_SYMMETRIC_X: the caller states the symmetry; no check, no
    wait).  tiling: "auto", "4x4" or "16x16" (the FP32 convolution's blocks).
    method: "direct" (the convolution sum on the matrix cores) or "fft"
    (SPECT_CONV_FFT: FP32 FFTs, the same operator).  symmetric_z: the caller
    states that every PSF column is symmetric in z (SPECT_PSF_SYMMETRIC_Z);
    with method="fft" and mirror="assume" the plan keeps real PSF spectra.
    """

    def __init__(self, mu, psf, dy, angles=None, cache_mubar=False, view_batch=0,
                 precision="fp32", rotation="3pass", mirror="auto", tiling="auto",
                 method="direct", symmetric_z=False):
        import torch
        self.device = mu.device
        if self.device.type != "cuda":
            raise ValueError("mu must live on a GPU")
        nz, ny, nx = mu.shape
        sep = isinstance(psf, (tuple, list))
        if sep:
            fz, fx = psf
            nview, ny2, pz = fz.shape
            px = fx.shape[2]
            if ny2 != ny:
                raise ValueError("psf depth does not match mu")
            _check(fz, (nview, ny, pz), "fz", self.device)
            _check(fx, (nview, ny, px), "fx", self.device)
            psf = torch.cat([fz, fx], dim=2).contiguous()      # owned by the plan
        else:
            nview, ny2, pz, px = psf.shape
            if ny2 != ny:
                raise ValueError("psf depth does not match mu")
            _check(psf, (nview, ny, pz, px), "psf", self.device)
        _check(mu, (nz, ny, nx), "mu", self.device)
        self.separable = sep
        self.shape = (nx, ny, nz, nview, px, pz)
        self.nx, self.ny, self.nz, self.nview, self.px, self.pz = self.shape
        if rotation not in ROTATIONS:
            raise ValueError(f"rotation must be one of {sorted(ROTATIONS)}")
        self.rotation = rotation
        if mirror not in MIRRORS:
            raise ValueError(f"mirror must be one of {sorted(MIRRORS)}")
        if tiling not in TILINGS:
            raise ValueError(f"tiling must be one of {sorted(TILINGS)}")
        if method not in METHODS:
            raise ValueError(f"method must be one of {sorted(METHODS)}")
        self.method = method
        flags = ((SPECT_CACHE_MUBAR if cache_mubar else 0) | ROTATIONS[rotation] |
                 (SPECT_PSF_SEPARABLE if sep else 0) | MIRRORS[mirror] | TILINGS[tiling] |
                 METHODS[method] | (SPECT_PSF_SYMMETRIC_Z if symmetric_z else 0))
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self.precision = precision
        self._geom, self._keep = make_geom(nx, ny, nz, nview, px, pz, dy, angles, flags, view_batch,
                                           PRECISIONS[precision])
        self.ws_bytes = spect_workspace_bytes(self._geom)
        self._mu, self._psf = mu, psf
        self._ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self._plan = spect_plan_create(self._geom, mu.data_ptr(), psf.data_ptr(),
                                       self._ws.data_ptr(), self.ws_bytes,
                                       _stream(torch, self.device))

    def describe(self) -> dict:
        """Kernels this plan selected (conv, mirror, rotation, view_batch, nchunk)."""
        return spect_plan_describe(self._plan)

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (self.nview, self.nz, self.nx)

    def forward(self, x, out=None):
        import torch
        _check(x, self.vol_shape, "x", self.device)
        if out is None:
            out = torch.empty(self.proj_shape, dtype=torch.float32, device=self.device)
        _check(out, self.proj_shape, "out", self.device)
        spect_forward(self._plan, x.data_ptr(), out.data_ptr(), _stream(torch, self.device))
        return out

    def back(self, v, out=None):
        import torch
        _check(v, self.proj_shape, "v", self.device)
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float32, device=self.device)
        _check(out, self.vol_shape, "out", self.device)
        spect_back(self._plan, v.data_ptr(), out.data_ptr(), _stream(torch, self.device))
        return out

    def em_step(self, x, y, sens, r=None):
        import torch
        _check(x, self.vol_shape, "x", self.device)
        _check(y, self.proj_shape, "y", self.device)
        _check(sens, self.vol_shape, "sens", self.device)
        if r is not None:
            _check(r, self.proj_shape, "r", self.device)
        spect_em_step(self._plan, x.data_ptr(), y.data_ptr(), None if r is None else r.data_ptr(),
                      sens.data_ptr(), _stream(torch, self.device))
        return x

    def reg_em_step(self, x, y, sens, u, beta, r=None):
        """Regularised EM update of Eq. (7)-(8) in place (target u, weight beta)."""
        import torch
        _check(x, self.vol_shape, "x", self.device)
        _check(y, self.proj_shape, "y", self.device)
        _check(sens, self.vol_shape, "sens", self.device)
        _check(u, self.vol_shape, "u", self.device)
        if r is not None:
            _check(r, self.proj_shape, "r", self.device)
        spect_reg_em_step(self._plan, x.data_ptr(), y.data_ptr(), None if r is None else r.data_ptr(),
                          sens.data_ptr(), u.data_ptr(), beta, _stream(torch, self.device))
        return x

    def em_step_vjp(self, x, y, sens, g, r=None, need_gy=True):
        """(dL/dx, dL/dy or None) of one em_step at input x for dL/dx+ = g."""
        import torch
        _check(x, self.vol_shape, "x", self.device)
        _check(y, self.proj_shape, "y", self.device)
        _check(sens, self.vol_shape, "sens", self.device)
        _check(g, self.vol_shape, "g", self.device)
        if r is not None:
            _check(r, self.proj_shape, "r", self.device)
        gx = torch.empty(self.vol_shape, dtype=torch.float32, device=self.device)
        gy = torch.empty(self.proj_shape, dtype=torch.float32, device=self.device) if need_gy else None
        spect_em_step_vjp(self._plan, x.data_ptr(), y.data_ptr(),
                          None if r is None else r.data_ptr(), sens.data_ptr(), g.data_ptr(),
                          gx.data_ptr(), None if gy is None else gy.data_ptr(),
                          _stream(torch, self.device))
        return gx, gy

    def profile_start(self, max_launches=4096):
        spect_profile_start(self._plan, max_launches)

    def profile_stop(self):
        return spect_profile_stop(self._plan)

    def close(self):
        if getattr(self, "_plan", None):
            spect_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dot_f64(a, b) -> float:
    """FP64 inner product of two float32 device tensors, on the GPU."""
    import torch
    if a.numel() != b.numel():
        raise ValueError("size mismatch")
    a = a.contiguous()
    b = b.contiguous()
    out = torch.empty(1, dtype=torch.float64, device=a.device)
    spect_dot_f64(a.data_ptr(), b.data_ptr(), a.numel(), out.data_ptr(), _stream(torch, a.device))
    return float(out.item())
