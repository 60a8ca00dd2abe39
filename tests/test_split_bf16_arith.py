"""The arithmetic of the FP32 64 x 64 products, checked on the host.

Those products split every FP32 operand x into three bf16 parts (h = bf16(x),
m = bf16(x - h), l = bf16(x - h - m), round to nearest even) and sum the six
part products hh, hm, mh, mm, hl, lh in FP32 accumulators.  The claims behind
that form: both differences are exact in FP32, |m| <= 2^-8 |x| and
|l| <= 2^-16 |x|, the dropped ml + lm + ll is below 2^-23 |x y|, and a dot
product built this way is as accurate as an FP32 one.  This emulates the
arithmetic in numpy (bf16 rounding on the bit pattern, FP32 sums in order)
and checks each claim against float64 references; it does not run the
kernel, whose results the GPU transform and batch tests compare with the
oracle.
"""
import numpy as np


def bf16_rne(x):
    """float32 -> nearest bf16 (ties to even), returned as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split3(x):
    x = np.asarray(x, dtype=np.float32)
    h = bf16_rne(x)
    r1 = (x - h).astype(np.float32)
    m = bf16_rne(r1)
    r2 = (r1 - m).astype(np.float32)
    l = bf16_rne(r2)
    return h, m, l, r1, r2


def sample(n, seed):
    rng = np.random.default_rng(seed)
    # signs, and magnitudes over a wide exponent range (no subnormals)
    return (rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n))).astype(np.float32)


def test_parts_exact_and_bounded():
    x = sample(200000, 1)
    h, m, l, r1, r2 = split3(x)
    x64 = x.astype(np.float64)
    # both differences are exact in FP32
    assert np.array_equal(r1.astype(np.float64), x64 - h.astype(np.float64))
    assert np.array_equal(r2.astype(np.float64), r1.astype(np.float64) - m.astype(np.float64))
    ax = np.abs(x64)
    assert np.all(np.abs(m.astype(np.float64)) <= 2.0 ** -8 * ax)
    assert np.all(np.abs(l.astype(np.float64)) <= 2.0 ** -16 * ax)
    # what the three parts miss of x
    resid = np.abs(x64 - h.astype(np.float64) - m.astype(np.float64) - l.astype(np.float64))
    assert np.all(resid <= 2.0 ** -24 * ax)


def test_part_products_exact_and_dropped_terms_small():
    x, y = sample(100000, 2), sample(100000, 3)
    hx, mx, lx, _, _ = split3(x)
    hy, my, ly, _, _ = split3(y)
    for a, b in ((hx, hy), (hx, my), (mx, hy), (mx, my), (hx, ly), (lx, hy)):
        # a bf16 x bf16 product has at most 16 significant bits: exact in FP32
        p32 = (a * b).astype(np.float64)
        assert np.array_equal(p32, a.astype(np.float64) * b.astype(np.float64))
    dropped = (mx.astype(np.float64) * ly + lx.astype(np.float64) * my + lx.astype(np.float64) * ly)
    assert np.all(np.abs(dropped) <= 2.0 ** -23 * np.abs(x.astype(np.float64) * y))


def split_dot(x, y):
    """sum_k x_k y_k as the kernel forms it: per k the six part products,
    smallest first, into one FP32 accumulator."""
    hx, mx, lx, _, _ = split3(x)
    hy, my, ly, _, _ = split3(y)
    acc = np.float32(0)
    for k in range(len(x)):
        for a, b in ((mx, my), (hx, ly), (lx, hy), (hx, my), (mx, hy), (hx, hy)):
            acc = np.float32(acc + np.float32(a[k] * b[k]))
    return acc


def fp32_dot(x, y):
    acc = np.float32(0)
    for k in range(len(x)):
        acc = np.float32(acc + np.float32(x[k] * y[k]))
    return acc


def test_dot_as_accurate_as_fp32():
    rng = np.random.default_rng(4)
    worst_split, worst_fp32 = 0.0, 0.0
    for trial in range(40):
        n = 512
        x = rng.standard_normal(n).astype(np.float32)
        y = rng.standard_normal(n).astype(np.float32)
        ref = np.dot(x.astype(np.float64), y.astype(np.float64))
        scale = np.dot(np.abs(x).astype(np.float64), np.abs(y).astype(np.float64))
        worst_split = max(worst_split, abs(float(split_dot(x, y)) - ref) / scale)
        worst_fp32 = max(worst_fp32, abs(float(fp32_dot(x, y)) - ref) / scale)
    # both at the FP32 accumulation level (n eps / 2 bound: 512 * 2^-24 = 3e-5;
    # typical far below), and the split form no worse than twice plain FP32
    assert worst_split <= 512 * 2.0 ** -24
    assert worst_split <= 2.0 * worst_fp32 + 2.0 ** -24
