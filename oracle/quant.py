"""16-bit storage of the kernel library with per-depth power-of-two scales.

Test infrastructure only (see ``oracle/__init__``).

The paper stores its operator in single-precision complex form (Sec. 4);
the 16-bit forms are precision variants the paper does not have.  For each depth l,
s_l = 2^(e - ceil(log2 max_{k,n} |H^[k,l,n]|)) with e = 0 for bfloat16 and
e = 15 for float16; the stored value is H_q = round16(round32(H^ * s_l)),
both roundings to nearest-even, and the dequantised value H_q / s_l is
exact because s_l is a power of two.
"""
from __future__ import annotations

import math

import numpy as np

EXPONENT = {"bf16": 0, "f16": 15}


def ceil_log2(v: float) -> int:
    """ceil(log2 v) for v > 0, exact for powers of two."""
    f, e = math.frexp(v)          # v = f * 2^e with 0.5 <= f < 1
    return e - 1 if f == 0.5 else e


def depth_scales(Hk: np.ndarray, kind: str) -> np.ndarray:
    """s_l for H^ given as [..., Nz, Nt] (all transverse frequencies)."""
    nz = Hk.shape[-2]
    amax = np.abs(Hk).reshape(-1, nz, Hk.shape[-1]).max(axis=(0, 2))
    out = np.empty(nz)
    for l in range(nz):
        out[l] = 1.0 if amax[l] == 0.0 else math.ldexp(1.0, EXPONENT[kind] - ceil_log2(float(amax[l])))
    return out


def round_bf16(a32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 (round to nearest even), returned as the float32
    value of the bfloat16 number."""
    u = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def quantise(Hk: np.ndarray, kind: str, scales: np.ndarray | None = None):
    """Returns (dequantised H^ in float64, scales).  Works on [..., Nz, Nt]."""
    if scales is None:
        scales = depth_scales(Hk, kind)
    s = scales[:, None]
    a32 = (Hk * s).astype(np.float32)
    if kind == "bf16":
        q = round_bf16(a32).astype(np.float64)
    elif kind == "f16":
        q = a32.astype(np.float16).astype(np.float64)
    else:
        raise ValueError(kind)
    return q / s, scales
