"""Rounding of FP32 values to the 16-bit formats of the reduced-precision
convolution (the precision study of the projector: BF16 / FP16 operands,
FP32 accumulation).  TEST INFRASTRUCTURE ONLY, like the rest of the oracle.

Both are round-to-nearest, ties to even, as IEEE 754 defines for a
narrowing conversion:
  bf16: 8 significant bits (7 stored), the FP32 exponent range;
  fp16: 11 significant bits (10 stored), exponent range of binary16
        (overflow to infinity above 65504, subnormals below 2^-14).
The result is returned widened to float64 so that the oracle can use it in
its own arithmetic.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x):
    """Nearest-even BF16 value of each FP32 value of x (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round_fp16(x):
    """Nearest-even FP16 value of each FP32 value of x."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def rounder(precision):
    return {"bf16": round_bf16, "fp16": round_fp16,
            "fp32": lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)}[precision]


def unit_roundoff(precision):
    """Half the spacing of the format at 1: 2^-p for p significant bits."""
    return {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp32": 2.0 ** -24}[precision]
