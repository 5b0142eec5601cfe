"""Host-side checks of the error model behind the GPU tolerances for
three-term BF16 exponents (tests/gpu_util.py): each FP32 operand v is split
into BF16 terms h + m + l, and six of the nine cross products (hh, hm, mh, hl,
lh, mm) are summed.  BF16 rounding is emulated with integer operations
(round to nearest, ties to even, on the upper 16 bits of the FP32 pattern)."""
import numpy as np

U32 = 2.0 ** -24


def bf16(x):
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def split3(v):
    v = np.asarray(v, dtype=np.float32)
    h = bf16(v)
    r1 = v - h  # exact in FP32
    m = bf16(r1)
    lo = bf16(r1 - m)
    return h, m, lo


def _operands(n, seed):
    rng = np.random.default_rng(seed)
    mant = rng.uniform(-1.0, 1.0, n)
    expo = rng.integers(-30, 30, n)
    return (mant * 2.0 ** expo).astype(np.float32)


def test_bf16_emulation_rounds_to_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even pattern 1
    assert bf16(np.float32(1 + 2.0 ** -8)) == np.float32(1.0)
    assert bf16(np.float32(1 + 3 * 2.0 ** -8)) == np.float32(1 + 2.0 ** -6)
    v = _operands(4096, 1)
    hv = bf16(v)
    assert np.all(hv.view(np.uint32) & 0xFFFF == 0)
    # 8 significant bits: rounding within 2^-8 of |v|
    assert np.all(np.abs(v.astype(np.float64) - hv) <= 2.0 ** -8 * np.abs(v))


def test_split_is_exact_with_term_sizes():
    # v - h leaves at most 16 significant bits and (v - h) - m at most 8, so
    # for normal FP32 values the three terms hold v exactly; |m| <= 2^-8 |v|,
    # |l| <= 2^-16 |v|
    v = _operands(20000, 2)
    h, m, lo = split3(v)
    v64 = v.astype(np.float64)
    assert np.all(v64 - h.astype(np.float64) - m.astype(np.float64) - lo.astype(np.float64) == 0.0)
    assert np.all(np.abs(m) <= 2.0 ** -8 * np.abs(v64))
    assert np.all(np.abs(lo) <= 2.0 ** -16 * np.abs(v64))


def test_term_products_exact_in_fp32():
    x, y = _operands(20000, 3), _operands(20000, 4)
    for a in split3(x):
        for b in split3(y):
            p32 = (a * b).astype(np.float64)
            p64 = a.astype(np.float64) * b.astype(np.float64)
            nz = p64 != 0.0
            # exact unless the product leaves FP32's normal range
            ok = ~nz | ((np.abs(p64) >= 2.0 ** -126) & (np.abs(p64) < 2.0 ** 127))
            assert np.all(p32[ok] == p64[ok])


def test_six_products_within_2u_of_the_product():
    # the dropped products ml, lm, ll are at most (2 x 2^-24 + 2^-32) |x y|
    x, y = _operands(20000, 5), _operands(20000, 6)
    hx, mx, lx = (t.astype(np.float64) for t in split3(x))
    hy, my, ly = (t.astype(np.float64) for t in split3(y))
    six = hx * hy + hx * my + mx * hy + hx * ly + lx * hy + mx * my
    exact = x.astype(np.float64) * y.astype(np.float64)
    bound = (2 * U32 + 2.0 ** -32) * np.abs(exact)
    assert np.all(np.abs(exact - six) <= bound)
    # every kept product matters: dropping hl (2^-16 of the product) breaks it
    five = six - hx * ly
    assert np.any(np.abs(exact - five) > bound)


def _split_dot_fp32(x, y):
    """Dot product of FP32 vectors from three-term BF16 splits: the six kept
    cross products of each coordinate pair, exact in FP32, summed one after
    the other in FP32 (the worst order for the bound)."""
    hx, mx, lx = split3(x)
    hy, my, ly = split3(y)
    acc = np.float32(0.0)
    for k in range(x.shape[0]):
        for a, b in ((hx, hy), (hx, my), (mx, hy), (hx, ly), (lx, hy), (mx, my)):
            acc = np.float32(acc + np.float32(a[k] * b[k]))
    return float(acc)


def test_split_dot_product_unit_count():
    # The unit count the GPU tolerances use for a dot product of n FP32 terms
    # formed from three-term BF16 splits: 6 n + 2 units of sum |x_k y_k|
    # (6 n exact products summed in FP32, dropped cross terms 2 u each).
    rng = np.random.default_rng(7)
    worst = 0.0
    for n in (3, 10, 18, 54):
        for _ in range(300):
            x = rng.standard_normal(n).astype(np.float32)
            y = rng.standard_normal(n).astype(np.float32)
            exact = float(np.dot(x.astype(np.float64), y.astype(np.float64)))
            mag = float(np.abs(x.astype(np.float64) * y.astype(np.float64)).sum())
            err = abs(_split_dot_fp32(x, y) - exact)
            assert err <= (6 * n + 2) * U32 * mag
            worst = max(worst, err / (U32 * mag))
    # the count is not vacuous: the sums do lose several units
    assert worst > 1.0
