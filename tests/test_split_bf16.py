"""The arithmetic behind the archive update on BF16 matrix cores, checked on
the host: a float32 value cut by truncation into three bfloat16 parts is
reproduced exactly, and the six part products with i + j <= 2 give the
product to float32 accuracy.  (The GPU kernel itself is checked against the
oracle by the parity tests.)"""
import numpy as np


def _split3(x):
    """x (float32) -> three float32 arrays holding bfloat16 values, by
    truncation of the lower 16 bits, as the kernel cuts its operands."""
    m = np.uint32(0xFFFF0000)
    x0 = (x.view(np.uint32) & m).view(np.float32)
    r1 = (x - x0).astype(np.float32)
    x1 = (r1.view(np.uint32) & m).view(np.float32)
    x2 = (r1 - x1).astype(np.float32)
    return x0, x1, x2


def _operands(rng, n):
    # normal floats over a wide exponent range, both signs, and exact zeros
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n))).astype(np.float32)
    x[::97] = 0.0
    return x


def test_split_is_exact_and_each_part_is_bfloat16():
    rng = np.random.default_rng(5)
    x = _operands(rng, 200_000)
    x0, x1, x2 = _split3(x)
    for p in (x0, x1, x2):
        assert not np.any(p.view(np.uint32) & np.uint32(0xFFFF)), "a part has bits below bfloat16"
    # exact in float64 (no rounding anywhere)
    assert np.array_equal(x0.astype(np.float64) + x1.astype(np.float64) + x2.astype(np.float64),
                          x.astype(np.float64))
    # each part carries 8 significand bits: the residuals shrink by 2^-8 at least
    nz = x != 0
    assert np.all(np.abs(x1[nz]) <= np.abs(x[nz]) * 2.0**-7)
    assert np.all(np.abs(x2[nz]) <= np.abs(x[nz]) * 2.0**-15)


def test_six_part_products_have_float32_accuracy():
    rng = np.random.default_rng(6)
    n, k = 4096, 64
    q = _operands(rng, n * k).reshape(n, k)
    c = (rng.standard_normal(k) * 1e-5).astype(np.float32)
    qs, cs = _split3(q), _split3(c)
    exact = q.astype(np.float64) @ c.astype(np.float64)
    # part products are exact in float32 (8 x 8 significand bits); accumulate
    # them the way the kernel does, in float32, smallest terms first
    pairs = [(2, 0), (1, 1), (0, 2), (1, 0), (0, 1), (0, 0)]
    acc = np.zeros(n, dtype=np.float32)
    for j in range(k):
        for a, b in pairs:
            acc = (acc + (cs[a][j] * qs[b][:, j]).astype(np.float32)).astype(np.float32)
    scale = np.abs(q).astype(np.float64) @ np.abs(c).astype(np.float64)
    err = np.abs(acc.astype(np.float64) - exact)
    # float32 accumulation of 6 k terms: a few units of 2^-24 per term at worst
    assert np.all(err <= 6 * k * 2.0**-24 * scale)
    # the three dropped products: |x1| < 2^-7 |x|, |x2| < 2^-15 |x| bound them
    # by 2^-22 (twice) and 2^-30
    dropped = sum(np.abs(cs[a][None, :] * qs[b]).astype(np.float64) for a, b in [(1, 2), (2, 1), (2, 2)])
    assert np.all(dropped <= 3 * 2.0**-22 * np.abs(q) * np.abs(c)[None, :] + 1e-300)
    # the plain bfloat16 product (one part each) is not accurate enough
    plain = qs[0].astype(np.float64) @ cs[0].astype(np.float64)
    assert np.max(np.abs(plain - exact) / np.maximum(scale, 1e-300)) > 2.0**-12
