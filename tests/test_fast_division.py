"""CPU check of the division by a grid extent that every kernel uses to turn a
node index into coordinates (FastDiv in the library's internal header):

    s = ceil(log2 d),  m = floor(2^(31 + s) / d) + 1  (32 bits),
    n / d = umulhi(n, m) >> (s - 1)        for d >= 2,  n itself for d = 1.

A context accepts up to 2^31 - 1 nodes, so the quotient must be exact for
every n < 2^31.  The argument: m d - 2^(31+s) = e with 0 < e <= d, so
n m / 2^(31+s) = n / d + n e / (d 2^(31+s)), and the last term is below
2^31 d / (d 2^(31+s)) = 2^-s <= 1/d, too small to carry n / d past the next
integer.  The test checks it by brute force where it can fail first: around
every multiple of d near the top of the range, at the range ends, and at
random points, for the divisors of the workloads (nx, nx ny) and random ones.
"""
import numpy as np
import pytest

TOP = (1 << 31) - 1


def fastdiv_set(d):
    if d <= 1:
        return 0, 0
    s = 0
    while (1 << s) < d:
        s += 1
    m = ((1 << (31 + s)) // d) + 1
    assert m < (1 << 32)
    return m, s


def fastdiv(n, d, m, s):
    if d == 1:
        return n
    return ((n * m) >> 32) >> (s - 1)


DIVISORS = [1, 2, 3, 5, 7, 62, 63, 64, 65, 127, 128, 129, 255, 256, 257, 512, 1000, 1024, 1025, 4096,
            23200, 23232, 816, 816 * 816, 256 * 256, 46340, 46341, 65535, 65536, 65537, 1 << 20,
            (1 << 20) + 1, 40000 * 40000, (1 << 30) + 1, TOP]


@pytest.mark.parametrize("d", DIVISORS + [int(v) for v in np.random.default_rng(21).integers(2, 1 << 31, 40)])
def test_quotient_exact_below_2_31(d):
    m, s = fastdiv_set(d)
    rng = np.random.default_rng(d % 1000003)
    ns = {0, 1, TOP, TOP - 1, d - 1, d, d + 1}
    # around the multiples of d nearest to the top of the range
    q = TOP // d
    for k in range(max(q - 64, 0), q + 1):
        for delta in (-2, -1, 0, 1, 2):
            v = k * d + delta
            if 0 <= v <= TOP:
                ns.add(v)
    ns.update(int(v) for v in rng.integers(0, TOP + 1, 2000))
    for n in ns:
        assert fastdiv(n, d, m, s) == n // d, (n, d)


def test_largest_square_grid_and_its_coordinates():
    """The largest square D2Q9 grid a context accepts: every node's (x, y)
    from the division, at the last rows."""
    nx = 46340                      # 46340^2 < 2^31 <= 46341^2
    ny = TOP // nx
    assert nx * ny <= TOP
    m, s = fastdiv_set(nx)
    for n in range(nx * ny - 3 * nx, nx * ny):
        y = fastdiv(n, nx, m, s)
        assert y == n // nx and 0 <= n - y * nx < nx
