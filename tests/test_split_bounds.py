"""The error bounds the matrix-core split schemes rest on, checked on the CPU by
emulating the splits with IEEE round-to-nearest-even conversions (numpy float16, and
bfloat16 by rounding the FP32 bit pattern):

* two-part FP16: v = h1 + h2 + r with |r| <= max(2^-22 |v|, 2^-25) for |v| <= 65504,
  and (a1 + a2)(b1 + b2) - a2 b2 within 3 x 2^-22 |ab| of ab for normal operands;
* three-part bf16: v = p1 + p2 + p3 + r with |r| <= 2^-24 |v| while the three parts
  are normal numbers (|v| >= 2^-110; below, r is bounded by the bf16 subnormal
  spacing 2^-133 instead), and the six products with i + j <= 4 within
  6 x 2^-24 |ab| of ab.
"""
import numpy as np

RNG = np.random.default_rng(27)


def _f16_split(v):
    v = v.astype(np.float32)
    h1 = v.astype(np.float16)
    r = (v - h1.astype(np.float32)).astype(np.float32)  # exact in FP32
    h2 = r.astype(np.float16)
    return h1.astype(np.float64), h2.astype(np.float64)


def _bf16(v):
    b = v.astype(np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32)


def _bf16_split(v):
    v = v.astype(np.float32)
    p1 = _bf16(v)
    r1 = (v - p1).astype(np.float32)
    p2 = _bf16(r1)
    r2 = (r1 - p2).astype(np.float32)
    p3 = _bf16(r2)
    return [p.astype(np.float64) for p in (p1, p2, p3)]


def _values(lo_exp, hi_exp, n=200000):
    mag = 2.0 ** RNG.uniform(lo_exp, hi_exp, n)
    return (mag * RNG.choice([-1.0, 1.0], n)).astype(np.float32)


def test_fp16_two_part_residual():
    v = np.r_[_values(-30, 15.99), np.float32(65504.0), np.float32(2.0 ** -25)]
    h1, h2 = _f16_split(v)
    r = np.abs(v.astype(np.float64) - h1 - h2)
    assert np.all(np.isfinite(h1)) and np.all(np.isfinite(h2))
    assert np.all(r <= np.maximum(2.0 ** -22 * np.abs(v.astype(np.float64)), 2.0 ** -25))


def test_fp16_three_products():
    # operands as the kernels scale them: largest near 2^15, normal FP16 parts
    a, b = _values(-2, 15), _values(-2, 15)
    a1, a2 = _f16_split(a)
    b1, b2 = _f16_split(b)
    ab = a.astype(np.float64) * b.astype(np.float64)
    approx = a1 * b1 + a1 * b2 + a2 * b1
    assert np.all(np.abs(approx - ab) <= 3 * 2.0 ** -22 * np.abs(ab))


def test_bf16_three_part_residual_and_six_products():
    v = _values(-110, 120)
    p1, p2, p3 = _bf16_split(v)
    r = np.abs(v.astype(np.float64) - p1 - p2 - p3)
    assert np.all(r <= 2.0 ** -24 * np.abs(v.astype(np.float64)))
    # below that range the third part is subnormal: an absolute bound instead
    t = _values(-140, -110)
    q1, q2, q3 = _bf16_split(t)
    assert np.all(np.abs(t.astype(np.float64) - q1 - q2 - q3) <= 2.0 ** -133)
    a, b = _values(-60, 60), _values(-60, 60)
    pa, pb = _bf16_split(a), _bf16_split(b)
    ab = a.astype(np.float64) * b.astype(np.float64)
    approx = sum(pa[i] * pb[j] for i in range(3) for j in range(3) if i + j <= 2)
    assert np.all(np.abs(approx - ab) <= 6 * 2.0 ** -24 * np.abs(ab))
