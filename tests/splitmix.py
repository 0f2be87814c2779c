"""SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), written out from its definition with Python
integers: the reference for the batch draw of po_draw_batch."""

M64 = (1 << 64) - 1


def splitmix64(seed: int, k: int) -> int:
    """Element k (from 0) of the sequence of `seed`."""
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def draw_rows(seed: int, first: int, n: int, n_src: int) -> list:
    """Rows floor(z * n_src / 2^64) of elements first .. first + n - 1."""
    return [(splitmix64(seed, first + i) * n_src) >> 64 for i in range(n)]
