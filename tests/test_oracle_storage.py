"""Pins of the reference storage roundings (oracle/storage.py): against numpy's and torch's
own conversions, on random values over many binades, exact ties, subnormals and the largest
finite values."""
import numpy as np
import torch

from oracle import storage


def _values(seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=20000) * 10.0 ** rng.uniform(-9, 4, size=20000)
    return x.astype(np.float32)


def _ties_f16(seed):
    """FP32 values exactly halfway between adjacent binary16 values (normal and subnormal)."""
    rng = np.random.default_rng(seed)
    bits = rng.integers(1, 0x7BFF, size=4000, dtype=np.uint16)
    lo = bits.view(np.float16).astype(np.float64)
    hi = (bits + 1).view(np.float16).astype(np.float64)
    mid = ((lo + hi) / 2).astype(np.float32)
    assert np.all(mid.astype(np.float64) == (lo + hi) / 2)  # exactly representable in FP32
    sign = np.where(rng.random(4000) < 0.5, -1.0, 1.0).astype(np.float32)
    return mid * sign


def _ties_bf16(seed):
    rng = np.random.default_rng(seed)
    hi16 = rng.integers(0x0080, 0x7F7F, size=4000, dtype=np.uint32)
    sign = rng.integers(0, 2, size=4000, dtype=np.uint32) << np.uint32(31)
    return ((hi16 << np.uint32(16)) | np.uint32(0x8000) | sign).view(np.float32)


def test_f16_matches_torch():
    for x in (_values(1), _ties_f16(2), np.array([6.1e-5, -5.96e-8, 2.98e-8, 65504.0, 65519.0, 0.0, -0.0],
                                                 dtype=np.float32)):
        ref = torch.from_numpy(x).to(torch.float16).to(torch.float32).numpy()
        assert np.array_equal(storage.round_to_f16(x).view(np.uint32), ref.view(np.uint32))


def test_bf16_matches_torch():
    for x in (_values(3), _ties_bf16(4), np.array([1e-40, -3e-39, 3.3895e38, 0.0, -0.0], dtype=np.float32)):
        ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
        assert np.array_equal(storage.round_to_bf16(x).view(np.uint32), ref.view(np.uint32))


def test_ties_go_to_even_and_rounding_is_within_half_an_ulp():
    t = _ties_bf16(5)
    r = storage.round_to_bf16(t).view(np.uint32)
    assert np.all((r >> 16) & 1 == 0)
    x = _values(6)
    x = x[(np.abs(x) > 1e-30) & (np.abs(x) < 1e30)]
    for f, u in ((storage.round_to_bf16, 2.0 ** -8), (storage.round_to_f16, 2.0 ** -11)):
        xx = x if f is storage.round_to_bf16 else x[(np.abs(x) > 6.2e-5) & (np.abs(x) < 6.5e4)]
        r = f(xx).astype(np.float64)
        assert np.all(np.abs(r - xx) <= u * np.abs(xx))
        assert np.array_equal(f(f(xx)), f(xx))  # idempotent
