"""Pins for the oracle's codebook compression (App. B.2): median-cut
quantisation of each basis function's RGB coefficients, float16 codebooks and
16-bit indices.

The float16 rounding is checked against NumPy's IEEE conversion; the median
cut against answers its definition fixes (a line of points, separated
clusters, as many boxes as distinct points, one box), against properties any
correct run has (every point's colour lies in its box, the representative is
the rounded mean of the box, a run with more boxes refines one with fewer and
does not raise the squared error) and against the edge cases.
"""
import numpy as np
import pytest


def test_half_bits_match_ieee(oracle_mod):
    rng = np.random.default_rng(0)
    xs = list(rng.standard_normal(2000) * 10.0 ** rng.integers(-9, 6, 2000))
    xs += [0.0, -0.0, 1.0, 65504.0, 65519.99, 65520.0, 1e9, -1e9, 2.0 ** -14, 2.0 ** -24, 2.0 ** -25,
           3 * 2.0 ** -26, 6e-8, float("inf"), -float("inf")]
    # exact halfway cases between neighbouring float16 values (ties to even)
    h = np.arange(0, 0x7bff, 97, dtype=np.uint16).view(np.float16).astype(np.float64)
    xs += list(0.5 * (h[:-1] + np.nextafter(h[:-1].astype(np.float16), np.float16(np.inf)).astype(np.float64)))
    for x in xs:
        with np.errstate(over="ignore"):
            want = int(np.array(x, np.float64).astype(np.float16).view(np.uint16))
        assert oracle_mod.half_bits(x) == want, x
    assert oracle_mod.half_bits(float("nan")) & 0x7c00 == 0x7c00


def test_line_of_points(oracle_mod):
    # 0..7 on the x axis, 4 boxes: {0..3} keeps box 0 and {4..7} becomes box 1;
    # then box 0 (first of two equal extents) splits into {0,1} and box 2 = {2,3};
    # then box 1 splits into {4,5} and box 3 = {6,7}
    pts = np.column_stack([np.arange(8.0), np.zeros(8), np.zeros(8)])
    idx, cb, nb = oracle_mod.median_cut(pts, 4)
    assert nb == 4
    assert list(idx) == [0, 0, 2, 2, 1, 1, 3, 3]
    np.testing.assert_array_equal(cb[:, 0].astype(np.float64), [0.5, 4.5, 2.5, 6.5])
    # an odd count: the lower half is the floor
    idx, cb, nb = oracle_mod.median_cut(pts[:7], 2)
    assert list(idx) == [0, 0, 0, 1, 1, 1, 1]
    # the longest side decides the axis: points spread along y, out of index order
    ys = np.array([3.0, 0.0, 7.0, 1.0, 6.0, 2.0, 5.0, 4.0])
    idx, cb, nb = oracle_mod.median_cut(np.column_stack([np.full(8, 0.5), ys, np.zeros(8)]), 2)
    assert list(idx) == [0, 0, 1, 0, 1, 0, 1, 1]
    # a median inside a run of equal coordinates: ties go by point index
    xs = np.array([0.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 2.0])
    idx, cb, nb = oracle_mod.median_cut(np.column_stack([xs, np.zeros(8), np.zeros(8)]), 2)
    assert list(idx) == [0, 0, 0, 0, 1, 1, 1, 1]


def test_separated_clusters(oracle_mod):
    rng = np.random.default_rng(1)
    # equal counts: the median split falls in the gap between the clusters
    a = rng.normal(0.0, 0.01, (250, 3)).astype(np.float32)
    b = rng.normal(5.0, 0.01, (250, 3)).astype(np.float32)
    pts = np.concatenate([a, b]).astype(np.float64)
    idx, cb, nb = oracle_mod.median_cut(pts, 2)
    assert nb == 2
    assert list(idx) == [0] * 250 + [1] * 250
    np.testing.assert_allclose(cb[0].astype(np.float64), a.astype(np.float64).mean(0), atol=1e-3)
    np.testing.assert_allclose(cb[1].astype(np.float64), b.astype(np.float64).mean(0), atol=4e-3)


def test_enough_boxes_is_exact(oracle_mod):
    rng = np.random.default_rng(2)
    # distinct points: every split separates points, so 40 points end in 40 boxes
    uniq = rng.standard_normal((40, 3)).astype(np.float32).astype(np.float64)
    idx, cb, nb = oracle_mod.median_cut(uniq, 64)
    assert nb == 40 and sorted(idx) == list(range(40))
    np.testing.assert_array_equal(cb[idx], uniq.astype(np.float16))
    # repeated points: a median may fall inside a run of equal points, but
    # with as many boxes as points every box ends with a single value
    pts = uniq[rng.integers(0, 40, 500)]
    idx, cb, nb = oracle_mod.median_cut(pts, 500)
    assert 40 <= nb <= 500
    np.testing.assert_array_equal(cb[idx], pts.astype(np.float16))


@pytest.mark.parametrize("M", [16, 256])
def test_box_properties(oracle_mod, M):
    rng = np.random.default_rng(3)
    pts = (rng.standard_normal((4000, 3)) * [0.5, 1.0, 0.2]).astype(np.float32).astype(np.float64)
    idx, cb, nb = oracle_mod.median_cut(pts, M)
    assert nb == M and idx.min() == 0 and idx.max() == M - 1
    for b in range(nb):
        mem = pts[idx == b]
        assert len(mem) > 0
        mean = mem.mean(0)
        got = cb[b].astype(np.float64)
        # the representative is the mean, rounded to float16 (half an ulp of slack)
        ulp = np.abs(mean.astype(np.float16).astype(np.float64) -
                     np.nextafter(mean.astype(np.float16), np.float16(np.inf)).astype(np.float64))
        assert np.all(np.abs(got - mean) <= 0.5 * ulp * (1 + 1e-9) + 1e-300)
        # and lies in the box's bounding box (up to the rounding)
        assert np.all(got >= mem.min(0) - ulp) and np.all(got <= mem.max(0) + ulp)
    # the sizes after the first split are floor / ceil of n
    idx2, _, _ = oracle_mod.median_cut(pts, 2)
    assert sorted(np.bincount(idx2)) == [2000, 2000]


def test_more_boxes_refine(oracle_mod):
    rng = np.random.default_rng(4)
    pts = rng.standard_normal((3000, 3)).astype(np.float32).astype(np.float64)
    prev_idx, prev_cb, _ = oracle_mod.median_cut(pts, 8)
    prev_sse = np.sum((prev_cb[prev_idx].astype(np.float64) - pts) ** 2)
    for M in (16, 64, 200):
        idx, cb, _ = oracle_mod.median_cut(pts, M)
        # every new box lies inside one old box, and keeps the old numbering of its lower part
        for b in range(M):
            assert len(set(prev_idx[idx == b])) == 1
        assert np.all(idx[prev_idx < len(prev_cb)] >= 0)
        sse = np.sum((cb[idx].astype(np.float64) - pts) ** 2)
        assert sse <= prev_sse * (1 + 1e-6)
        prev_idx, prev_cb, prev_sse = idx, cb, sse


def test_edge_cases(oracle_mod):
    idx, cb, nb = oracle_mod.median_cut(np.zeros((0, 3)), 16)
    assert nb == 0 and len(idx) == 0
    idx, cb, nb = oracle_mod.median_cut(np.array([[0.25, -1.5, 3.0]]), 16)
    assert nb == 1 and list(idx) == [0]
    np.testing.assert_array_equal(cb[0], np.array([0.25, -1.5, 3.0], np.float16))
    pts = np.random.default_rng(5).standard_normal((100, 3)).astype(np.float32).astype(np.float64)
    idx, cb, nb = oracle_mod.median_cut(pts, 1)
    assert nb == 1 and np.all(idx == 0)
    np.testing.assert_array_equal(cb[0], pts.mean(0).astype(np.float16))


def test_codebook_of_leaves(oracle_mod):
    rng = np.random.default_rng(6)
    sh = rng.normal(0, 0.5, (2000, 3, 9)).astype(np.float32)
    idx, books = oracle_mod.codebook(sh, 128)
    assert idx.shape == (2000, 9) and len(books) == 9
    dec = oracle_mod.codebook_decode(idx, books)
    err = np.abs(dec - sh.astype(np.float64))
    # each basis function is quantised on its own: a finer codebook is closer
    idx2, books2 = oracle_mod.codebook(sh, 1024)
    err2 = np.abs(oracle_mod.codebook_decode(idx2, books2) - sh.astype(np.float64))
    assert err2.mean() < 0.6 * err.mean()
    for k in range(9):
        i_k, cb_k, _ = oracle_mod.median_cut(sh[:, :, k], 128)
        assert np.array_equal(idx[:, k], i_k) and np.array_equal(books[k].view(np.uint16), cb_k.view(np.uint16))
