"""Pins for the oracle's visibility filter (Sec. 4.2, "Filtering"): the
largest ray weight each leaf receives over the rays of alpha renders.

Closed forms on one leaf, the telescoping sum of contributions along a single
ray (they add up to the opacity 1 - T), the longest chord through each leaf
when nothing stops the rays, the removal of voxels hidden behind an opaque
wall by the early stop, and invariance under reordering the rays.
"""
import numpy as np
import pytest

from paper_2103_14024_amd import scenes


def _tree(oracle_mod, depth, cells, sigma, lmax=1):
    K = (lmax + 1) ** 2
    sh = np.zeros((len(cells), 3, K))
    return oracle_mod.OracleTree(depth, lmax, (0, 0, 0), 1.0, np.asarray(cells, np.int32), np.asarray(sigma), sh)


def test_single_leaf_closed_form(oracle_mod):
    # leaf (2; 1,1,1) spans [-0.5, 0)^3; an x-parallel ray crosses 0.5 of it
    cells = [[2, 1, 1, 1], [2, 0, 1, 1]]
    tree = _tree(oracle_mod, 2, cells, [3.0, 0.7])
    o = np.array([[-3.0, -0.3, -0.2]])
    d = np.array([[1.0, 0.0, 0.0]])
    w0 = tree.leaf_weights(o, d, mode=0)
    w1 = tree.leaf_weights(o, d, mode=1)
    a_front, a_back = 1 - np.exp(-0.7 * 0.5), 1 - np.exp(-3.0 * 0.5)
    assert abs(w0[1] - a_front) < 1e-15 and abs(w0[0] - a_back) < 1e-15
    assert abs(w1[1] - a_front) < 1e-15
    assert abs(w1[0] - np.exp(-0.7 * 0.5) * a_back) < 1e-15
    # a ray missing both leaves leaves the weights at zero
    assert np.all(tree.leaf_weights(np.array([[-3.0, 0.5, 0.5]]), d) == 0.0)


def test_single_ray_contributions_sum_to_opacity(oracle_mod):
    sc = scenes.scene_small()
    tree = oracle_mod.OracleTree(sc["depth"], sc["sh_degree"], sc["center"], sc["half"], sc["cells"],
                                 sc["sigma"], sc["sh"])
    o, d = scenes.random_rays(400, 31)
    _, T, ns, _ = tree.render_rays(o, d)
    checked = 0
    for r in np.flatnonzero(ns > 0)[:60]:
        w = tree.leaf_weights(o[r:r + 1], d[r:r + 1], mode=1)
        # a ray crosses a (convex) cell once, so every leaf holds one contribution
        assert abs(w.sum() - (1.0 - T[r])) < 1e-12
        checked += 1
    assert checked == 60


def test_alpha_weight_is_longest_chord(oracle_mod):
    sc = scenes.scene_small()
    tree = oracle_mod.OracleTree(sc["depth"], sc["sh_degree"], sc["center"], sc["half"], sc["cells"],
                                 sc["sigma"], sc["sh"])
    o, d = scenes.random_rays(400, 32)
    w = tree.leaf_weights(o, d, gamma=0.0, mode=0)
    # without early stop every crossed leaf counts; alpha grows with the chord
    chord = np.zeros(tree.n_leaves)
    for r in range(len(o)):
        a, b, leaf = tree.segments(o[r], d[r])
        for ai, bi, li in zip(a, b, leaf):
            if li >= 0:
                chord[li] = max(chord[li], bi - ai)
    sig = np.maximum(np.asarray(sc["sigma"], np.float64), 0.0)
    np.testing.assert_allclose(w, -np.expm1(-sig * chord), rtol=0, atol=1e-15)
    assert np.count_nonzero(w) > 100


def _wall_scene(oracle_mod):
    # depth 3 (8^3): an opaque wall at x-cell 2 over the whole y-z range and a
    # thin layer behind it at x-cell 5
    cells, sigma = [], []
    for j in range(8):
        for k in range(8):
            cells.append([3, 2, j, k])
            sigma.append(1e4)
            cells.append([3, 5, j, k])
            sigma.append(1.0)
    return _tree(oracle_mod, 3, cells, sigma), np.array(sigma)


def test_early_stop_removes_hidden_voxels(oracle_mod):
    tree, sigma = _wall_scene(oracle_mod)
    rng = np.random.default_rng(4)
    n = 3000
    o = np.column_stack([np.full(n, -3.0), rng.uniform(-0.99, 0.99, n), rng.uniform(-0.99, 0.99, n)])
    d = np.column_stack([np.ones(n), rng.uniform(-0.1, 0.1, n), rng.uniform(-0.1, 0.1, n)])
    wall, back = sigma > 1.0, sigma == 1.0
    for mode in (0, 1):
        w = tree.leaf_weights(o, d, gamma=1e-4, mode=mode)
        assert np.all(w[wall] > 0.99)
        assert np.all(w[back] == 0.0)  # the walk stopped inside the wall
    # without the stop the back layer is reached: alpha counts it fully,
    # its contribution is below exp(-1e4 * 0.25)
    w0 = tree.leaf_weights(o, d, gamma=0.0, mode=0)
    assert np.all(w0[back] > 0.1)
    w1 = tree.leaf_weights(o, d, gamma=0.0, mode=1)
    assert np.all(w1[back] < 1e-300)


def test_order_of_rays_does_not_matter(oracle_mod):
    sc = scenes.scene_small()
    tree = oracle_mod.OracleTree(sc["depth"], sc["sh_degree"], sc["center"], sc["half"], sc["cells"],
                                 sc["sigma"], sc["sh"])
    o, d = scenes.random_rays(600, 33)
    p = np.random.default_rng(0).permutation(len(o))
    for mode in (0, 1):
        a = tree.leaf_weights(o, d, gamma=1e-4, mode=mode)
        b = tree.leaf_weights(o[p], d[p], gamma=1e-4, mode=mode)
        assert np.array_equal(a, b)
        # two halves accumulated into one array give the same maxima
        c = tree.leaf_weights(o[:300], d[:300], gamma=1e-4, mode=mode)
        tree.leaf_weights(o[300:], d[300:], gamma=1e-4, mode=mode, weight=c)
        assert np.array_equal(a, c)
