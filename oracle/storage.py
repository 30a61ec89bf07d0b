"""Reduced-precision storage of the population deviations.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The state is stored as the deviation g_i = f_i - w_i rho0 (the delta-rho form of the
equilibrium, Section 2, which the paper adopts to limit round-off). At reduced precision each
stored value is the FP32 value rounded to nearest, ties to even, in IEEE binary16 (FP16) or
in bfloat16 (the upper 16 bits of binary32). Loading widens exactly. These are the reference
roundings for the codec; the pins check them against two independent library conversions.
"""
from __future__ import annotations

import numpy as np


def round_to_f16(x) -> np.ndarray:
    """FP32 -> binary16 (round to nearest even, subnormals kept) -> FP32, as float32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def round_to_bf16(x) -> np.ndarray:
    """FP32 -> bfloat16 -> FP32, as float32, for finite inputs. Round to nearest even on the
    bit pattern: add 0x7FFF plus the lowest kept bit, then clear the 16 dropped bits (the
    carry into the exponent is the correct rounding up to the next binade, or to infinity)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep_lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = (b + np.uint64(0x7FFF) + keep_lsb) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32)


def round_storage(x, storage: str) -> np.ndarray:
    if storage == "f32":
        return np.asarray(x, dtype=np.float32)
    if storage == "f16":
        return round_to_f16(x)
    if storage == "bf16":
        return round_to_bf16(x)
    raise ValueError(storage)
