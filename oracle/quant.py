"""ORACLE (test infrastructure only): storage formats of the precision form.

Written from the format definitions (IEEE 754 binary16; bfloat16 = the upper
half of binary32; OCP 8-bit floating point E4M3 "FN" variant: bias 7, no
infinities, only S.1111.111 is NaN, largest finite 448).  Rounding is to
nearest, ties to even; values beyond the largest finite saturate (the
path's scales guarantee |x| <= max, so saturation never decides a result).

Parity status: pinned against PyTorch's CPU conversions (a library routine)
on exhaustive code tables and random values.
"""
from __future__ import annotations

import numpy as np

# name: (mantissa bits, minimum normal exponent, largest finite value, bytes)
FORMATS = {
    "bf16": (7, -126, (2.0 - 2.0 ** -7) * 2.0 ** 127, 2),
    "f16": (10, -14, 65504.0, 2),
    "f8e4m3": (3, -6, 448.0, 1),
}


def quantize(x, fmt: str) -> np.ndarray:
    """Nearest representable value of `fmt` (ties to even), as float64."""
    p, emin, vmax, _ = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    _, E = np.frexp(x[nz])
    e = np.maximum(E - 1, emin)             # exponent of the binade (or subnormal range)
    quantum = np.ldexp(1.0, e - p)
    q = np.rint(x[nz] / quantum) * quantum  # np.rint rounds half to even
    out[nz] = np.clip(q, -vmax, vmax)
    return out


def spacing(x, fmt: str) -> np.ndarray:
    """Distance between consecutive representable values around |x|."""
    p, emin, _, _ = FORMATS[fmt]
    x = np.abs(np.asarray(x, dtype=np.float64))
    _, E = np.frexp(np.where(x > 0, x, 1.0))
    e = np.where(x > 0, np.maximum(E - 1, emin), emin)
    return np.ldexp(1.0, e - p)


def decode(bits, fmt: str) -> np.ndarray:
    """Value of each stored code (uint16 for bf16/f16, uint8 for f8e4m3)."""
    b = np.asarray(bits).astype(np.int64)
    if fmt == "bf16":
        with np.errstate(invalid="ignore"):
            return (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    if fmt == "f16":
        s, e, m = (b >> 15) & 1, (b >> 10) & 0x1F, b & 0x3FF
        mag = np.where(e == 0, np.ldexp(m / 1024.0, -14),
                       np.ldexp(1.0 + m / 1024.0, e - 15))
        mag = np.where(e == 31, np.where(m == 0, np.inf, np.nan), mag)
        return np.where(s == 1, -mag, mag)
    if fmt == "f8e4m3":
        s, e, m = (b >> 7) & 1, (b >> 3) & 0xF, b & 0x7
        mag = np.where(e == 0, np.ldexp(m / 8.0, -6), np.ldexp(1.0 + m / 8.0, e - 7))
        mag = np.where((e == 15) & (m == 7), np.nan, mag)
        return np.where(s == 1, -mag, mag)
    raise ValueError(fmt)


def encode(x, fmt: str) -> np.ndarray:
    """Code of the nearest representable value (RNE, saturating)."""
    q = quantize(x, fmt)
    if fmt == "bf16":
        return (q.astype(np.float32).view(np.uint32) >> np.uint32(16)).astype(np.uint16)
    p, emin, _, nbytes = FORMATS[fmt]
    ebias = 1 - emin
    neg = np.signbit(q)
    a = np.abs(q)
    _, E = np.frexp(np.where(a > 0, a, 1.0))
    e = E - 1
    normal = (a > 0) & (e >= emin)
    field_e = np.where(normal, e + ebias, 0)
    frac = np.where(normal, a / np.ldexp(1.0, e) - 1.0, a / np.ldexp(1.0, emin))
    field_m = np.rint(frac * (1 << p)).astype(np.int64)
    code = (field_e.astype(np.int64) << p) | field_m
    code = code | (neg.astype(np.int64) << (8 * nbytes - 1))
    return code.astype(np.uint8 if nbytes == 1 else np.uint16)


# Per-step relative Frobenius bounds of one stored product (teacher forced):
# storage rounding u = 2^-(p+1) times a small margin for the FP32 accumulation.
STEP_BOUND = {"f32": 1e-5, "f16": 5e-4, "bf16": 4e-3, "f8e4m3": 6.3e-2}
