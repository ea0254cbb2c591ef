"""P19: the error bound of the BF16x3 product, on the CPU.

A double x is split as x = hi + lo + e with hi = bf16(x), lo = bf16(x - hi)
(round to nearest even on the FP32 value), |e| <= u^2 |x|, u = 2^-8 the unit
roundoff of an 8-bit significand.  The product of two such splits keeps the
three terms hi.hi + hi.lo + lo.hi (each exact in FP32) and drops lo.lo, so a
sum of K products accumulated in FP32 over chunks of kc terms, the chunks
then added in FP64, differs from the exact sum by at most
    (3 u^2 (1 + 2u) + kc 2^-24) sum_k |a_k b_k|
(three dropped or rounded terms of u^2 |ab| each, and the FP32 accumulation
of a chunk, a standard bound on recursive summation).  The test emulates
the split and the accumulation bit for bit and checks the bound on random
and on cancelling data, and that dropping a cross term breaks it."""
import numpy as np

U = 2.0 ** -8


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float32."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> 16) & 1
    r = ((f + 0x7FFF + lsb) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32)


def split(x):
    hi = bf16(x.astype(np.float32))
    lo = bf16((x - hi.astype(np.float64)).astype(np.float32))
    return hi, lo


def bf16x3_dot(a, b, kc, terms=3):
    ah, al = split(a)
    bh, bl = split(b)
    p = ah.astype(np.float64) * bh
    if terms >= 2:
        p = p + ah.astype(np.float64) * bl
    if terms >= 3:
        p = p + al.astype(np.float64) * bh
    total = 0.0
    for c0 in range(0, len(a), kc):
        acc = np.float32(0.0)
        for v in p[c0:c0 + kc].astype(np.float32):
            acc = np.float32(acc + v)
        total += float(acc)
    return total


def bound(a, b, kc):
    return (3 * U * U * (1 + 2 * U) + kc * 2.0 ** -24) * float(np.abs(a * b).sum())


def test_split_is_exact_to_u_squared():
    rng = np.random.default_rng(0)
    x = rng.normal(size=20000) * np.exp(rng.normal(size=20000))
    hi, lo = split(x)
    err = np.abs(x - hi.astype(np.float64) - lo.astype(np.float64))
    assert (err <= U * U * np.abs(x) * (1 + U)).all()
    assert err.max() > 0


def test_bf16x3_product_within_bound():
    rng = np.random.default_rng(1)
    for K, kc in ((1000, 256), (4096, 1024)):
        a = rng.normal(size=K)
        b = rng.normal(size=K) / (1 + np.arange(K) / 100.0)
        exact = float(np.dot(a, b))
        got = bf16x3_dot(a, b, kc)
        assert abs(got - exact) <= bound(a, b, kc)
        # cancelling data: the sum is tiny against sum |ab|
        b2 = b.copy()
        b2[K // 2:] = -a[:K // 2] * b[:K // 2] / a[K // 2:]
        got2 = bf16x3_dot(a, b2, kc)
        assert abs(got2 - float(np.dot(a, b2))) <= bound(a, b2, kc)


def test_dropping_a_cross_term_breaks_the_bound():
    # values just above 1 whose BF16 rounding is 1 (spacing 2^-7): every lo
    # part is positive, so the dropped term cannot average out
    rng = np.random.default_rng(2)
    a = 1.0 + 2.0 ** -9 * (1.0 + 0.4 * rng.random(2048))
    b = np.abs(rng.normal(size=2048))
    exact = float(np.dot(a, b))
    assert abs(bf16x3_dot(a, b, 256) - exact) <= bound(a, b, 256)
    assert abs(bf16x3_dot(a, b, 256, terms=2) - exact) > bound(a, b, 256)
