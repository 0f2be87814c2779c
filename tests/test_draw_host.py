"""The reference batch generator against published SplitMix64 outputs, and
the uniformity of its row draw (CPU)."""
import numpy as np

from splitmix import draw_rows, splitmix64


def test_splitmix64_published_values():
    # the first outputs of the reference generator for seeds 0 and 1234567
    assert splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert splitmix64(1234567, 0) == 6457827717110365317
    assert splitmix64(1234567, 1) == 3203168211198807973


def test_draw_rows_uniform():
    # 200,000 draws over 50 rows: every row within 5 sigma of n / 50, and
    # consecutive ranges of the sequence continue one another
    n, m = 200_000, 50
    rows = np.array(draw_rows(7, 0, n, m))
    assert rows.min() == 0 and rows.max() == m - 1
    cnt = np.bincount(rows, minlength=m)
    sd = np.sqrt(n / m * (1 - 1 / m))
    assert np.all(np.abs(cnt - n / m) < 5 * sd)
    assert draw_rows(7, 1000, 10, m) == list(rows[1000:1010])
