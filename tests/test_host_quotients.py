"""The leading DE step takes small integer quotients (k = 256 / P, a
thread's member and part, a thread's tile count) from an FP32 reciprocal
instead of the integer division sequence (kernels.h: div_small, div_mid).
These checks emulate both on the CPU with the reciprocal rounded to FP32 and
then moved by one unit in the last place either way (the hardware
reciprocal's stated accuracy), and compare with exact integer division over
the ranges the kernel uses them on."""
import numpy as np


def _rcp_variants(b):
    r = (np.float32(1.0) / b.astype(np.float32)).astype(np.float32)
    return [r, np.nextafter(r, np.float32(np.inf)), np.nextafter(r, np.float32(0))]


def div_small(a, b, r):
    # floor((a + 1/2) * rcp(b)) in FP32 arithmetic
    return np.trunc((a.astype(np.float32) + np.float32(0.5)) * r).astype(np.int64)


def div_mid(a, b, r):
    q = np.trunc(a.astype(np.float32) * r).astype(np.int64)
    rem = a - q * b
    return q + (rem >= b) - (rem < 0)


def test_div_small_exact_up_to_4096():
    a, b = np.meshgrid(np.arange(0, 4097, dtype=np.int64), np.arange(1, 4097, dtype=np.int64), indexing="ij")
    a, b = a.ravel(), b.ravel()
    want = a // b
    for r in _rcp_variants(b):
        assert np.array_equal(div_small(a, b, r), want)


def test_div_mid_exact_below_2_23():
    rng = np.random.default_rng(3)
    # every divisor a thread count can be (1 .. 256) against numerators up to
    # 2^23: random, near multiples of the divisor, and the top of the range
    b = np.repeat(np.arange(1, 257, dtype=np.int64), 4000)
    a = rng.integers(0, 1 << 23, size=b.size, dtype=np.int64)
    mult = (a // b) * b
    cases = np.concatenate([a, np.clip(mult - 1, 0, None), mult, np.minimum(mult + 1, (1 << 23) - 1),
                            np.full(256, (1 << 23) - 1, dtype=np.int64)])
    bb = np.concatenate([b, b, b, b, np.arange(1, 257, dtype=np.int64)])
    want = cases // bb
    for r in _rcp_variants(bb):
        assert np.array_equal(div_mid(cases, bb, r), want)


def test_div_mid_guards_its_estimate():
    # an estimate off by one either way is corrected
    a = np.array([999, 1000, 1001, 8388607], dtype=np.int64)
    b = np.array([10, 10, 10, 7], dtype=np.int64)
    exact = (np.float32(1.0) / b.astype(np.float32)).astype(np.float32)
    for scale in (np.float32(1.0 + 2.0 ** -20), np.float32(1.0 - 2.0 ** -20)):
        assert np.array_equal(div_mid(a, b, (exact * scale).astype(np.float32)), a // b)
