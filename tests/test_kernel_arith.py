"""Integer identities the HIP kernels rely on, checked exhaustively on the host.

The sampler places AES block lb of an 8 x n segment (n/8 blocks per row) in row lb / (n/8)
without a division: it takes the high word of 2 lb * magic, magic = floor(2^32 / (2 n/8)) + 1.
That quotient is exact when 2 lb * (magic * 2 n/8 - 2^32) < 2^32; here every registrable n
(multiples of 8 up to 32768) and every block lb < n is checked directly."""
import numpy as np


def test_sampler_row_reciprocal_exact_for_every_n():
    for n in range(8, 32768 + 1, 8):
        nb = n // 8
        magic = np.uint64(0xFFFFFFFF // (2 * nb) + 1)
        assert int(magic) < 1 << 32, n  # fits the kernel's 32-bit register
        lb = np.arange(n, dtype=np.uint64)
        row = ((np.uint64(2) * lb * magic) >> np.uint64(32)).astype(np.int64)
        assert np.array_equal(row, np.arange(n) // nb), n
        col = 8 * (np.arange(n) - row * nb)
        assert col.min() == 0 and col.max() == n - 8, n
