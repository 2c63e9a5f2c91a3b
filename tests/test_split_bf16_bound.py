"""Host check of the error bound behind the split-BF16 tolerances (no GPU):
with hi = bf16(x) and lo = bf16(x - hi) (round to nearest even, as the
kernels round; BF16 keeps 8 significant bits, unit roundoff 2^-8), hi + lo
represents an FP32 x to within 2^-8 * 2^-8 |x| = 2^-16 |x|, and the three-term
product lo_a hi_b + hi_a lo_b + hi_a hi_b is within 3 * 2^-16 |a b| of a b.  The emulation rounds by the
same bit operation the kernels use, on FP32 inputs drawn over many binades (Henry, Tang and Heinecke, 2019)."""
import numpy as np


def bf16(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, np.float32)
    hi = bf16(x)
    d = (x - hi).astype(np.float32)
    # x - hi is exact in FP32 (hi is x rounded to 8 significant bits)
    assert np.array_equal(d.astype(np.float64), x.astype(np.float64) - hi.astype(np.float64))
    return hi, bf16(d)


def test_split_represents_fp32_to_2_pow_minus_16():
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(200000) * np.exp2(rng.integers(-40, 40, 200000))).astype(np.float32)
    hi, lo = split(x)
    err = np.abs(hi.astype(np.float64) + lo.astype(np.float64) - x.astype(np.float64))
    assert np.all(err <= 2.0 ** -16 * np.abs(x.astype(np.float64)))
    # plain BF16 alone is off by up to 2^-8, as the single-MFMA path is
    e1 = np.abs(hi.astype(np.float64) - x.astype(np.float64)) / np.abs(x.astype(np.float64))
    assert e1.max() <= 2.0 ** -8 and e1.max() > 2.0 ** -9


def test_three_term_product_bound():
    rng = np.random.default_rng(8)
    a = (rng.standard_normal(200000) * np.exp2(rng.integers(-20, 20, 200000))).astype(np.float32)
    b = (rng.standard_normal(200000) * np.exp2(rng.integers(-20, 20, 200000))).astype(np.float32)
    ah, al = (v.astype(np.float64) for v in split(a))
    bh, bl = (v.astype(np.float64) for v in split(b))
    exact = a.astype(np.float64) * b.astype(np.float64)
    # products of BF16 values are exact in FP64 (8 + 8 significant bits)
    three = al * bh + ah * bl + ah * bh
    rel = np.abs(three - exact) / np.abs(exact)
    assert rel.max() <= 3 * 2.0 ** -16
    # with the dropped term lo_a lo_b put back, only the two representation errors remain
    assert (np.abs(three + al * bl - exact) / np.abs(exact)).max() <= 2 * 2.0 ** -16 + 2.0 ** -32
