"""The arithmetic of the split-BF16 products (tp_gemm_mode(2)) on the host: a model of the operand
split with round-to-nearest-even BF16 conversions, checked against the error bounds the library
documents.  The GPU tests check the kernel against the oracle; this pins the bounds themselves."""
import numpy as np


def bf16_rne(x):
    """FP32 -> BF16 (8 significant bits) with ties to even, returned as FP32 values."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne((x - hi).astype(np.float32))
    return hi, lo


def _samples(n, seed, lim=1e30):
    rng = np.random.default_rng(seed)
    mag = np.exp(rng.uniform(-np.log(lim), np.log(lim), n))
    return (mag * rng.choice([-1.0, 1.0], n)).astype(np.float32)


def test_bf16_rounding_is_nearest_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even significand (1.0)
    assert bf16_rne(np.float32(1.0 + 2.0 ** -8)) == np.float32(1.0)
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: ties go to 1 + 2^-6
    assert bf16_rne(np.float32(1.0 + 3 * 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)
    x = _samples(100000, 1)
    h = bf16_rne(x).astype(np.float64)
    # representable in 8 significant bits, and the nearest such value
    assert np.all(np.abs(h - x) <= 2.0 ** -8 * np.abs(x.astype(np.float64)))


def test_split_remainder_bound():
    """x = hi + lo + r with |r| <= 2^-16 |x| (each of hi, lo has 8 significant bits)."""
    x = _samples(200000, 2)
    hi, lo = split(x)
    r = x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64)
    assert np.all(np.abs(r) <= 2.0 ** -16 * np.abs(x.astype(np.float64)))
    # the subtraction x - hi is exact in FP32 (no extra rounding before the second conversion)
    assert np.all((x - hi).astype(np.float64) == x.astype(np.float64) - hi.astype(np.float64))


def test_split_product_bound():
    """hi hi' + hi lo' + lo hi' differs from x y by at most about 3 * 2^-16 |x y|; the three terms
    are exact in FP32 (8 x 8 significant bits)."""
    x, y = _samples(200000, 3, 1e15), _samples(200000, 4, 1e15)   # x y inside the FP32 range
    xh, xl = split(x)
    yh, yl = split(y)
    exact = [xh.astype(np.float64) * yh, xh.astype(np.float64) * yl, xl.astype(np.float64) * yh]
    for t, e in zip([xh * yh, xh * yl, xl * yh], exact):
        ok = np.abs(e) > 1e-30          # away from FP32 underflow
        assert np.all(t[ok].astype(np.float64) == e[ok])
    p = exact[0] + exact[1] + exact[2]
    xy = x.astype(np.float64) * y.astype(np.float64)
    rel = np.abs(p - xy) / np.abs(xy)
    assert rel.max() <= 3.01 * 2.0 ** -16
    # far below the bound on average, and well above the FP32 product's 2^-24 at worst
    assert np.median(rel) < 2.0 ** -17
    assert rel.max() > 2.0 ** -20
