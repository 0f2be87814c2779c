"""The traversal index (po_tree_index_host, the host half of
po_tree_build_index) against the plain octree: for every finest cell of
random trees, the leaf and level the index names (nodes above level D - 3,
then one 8x8x8 brick) equal those of the descent through the caller's child
array (Sec. 4.2, "Rendering": the walk steps through the leaves that hold
the cells it crosses).  Host only."""
import ctypes

import numpy as np
import pytest

from paper_2103_14024_amd import _lib as L
from paper_2103_14024_amd import scenes
from paper_2103_14024_amd.tree import build_host, make_desc


def _slot(c, D, L):
    sft = D - 1 - L
    return (((c[0] >> sft) & 1) << 2) | (((c[1] >> sft) & 1) << 1) | ((c[2] >> sft) & 1)


def _plain(child, D, c):
    """(leaf or -1, level) of the cell's leaf by descent from the root."""
    node = 0
    for lv in range(D):
        e = int(child[node, _slot(c, D, lv)])
        if e > 0:
            node = e
            continue
        return (-e - 1 if e < 0 else -1), lv + 1
    raise AssertionError("descent below depth D")


def _indexed(index, n_top, D, c):
    M = D - 3
    node = 0
    for lv in range(M):
        e = int(index[node * 8 + _slot(c, D, lv)])
        if lv + 1 < M and 0 < e < n_top:
            node = e
            continue
        if lv + 1 == M and e >= n_top:
            b = e - n_top
            pos = _slot(c, D, M) * 64 + _slot(c, D, M + 1) * 8 + _slot(c, D, M + 2)
            v = int(index[n_top * 8 + b * 512 + pos])
            return (v >> 2) - 1, D - (v & 3)
        assert e <= 0, (lv, e)
        return (-e - 1 if e < 0 else -1), lv + 1
    raise AssertionError("no entry")


def _index(desc, child, n_leaves):
    nt, nb = ctypes.c_int64(), ctypes.c_int64()
    ch = np.ascontiguousarray(child, np.int32)
    L.call("po_tree_index_host", ctypes.byref(desc), ch.shape[0], ch.ctypes.data, n_leaves, ctypes.byref(nt),
           ctypes.byref(nb), None)
    out = np.full(nt.value * 8 + nb.value * 512, -7, np.int32)
    L.call("po_tree_index_host", ctypes.byref(desc), ch.shape[0], ch.ctypes.data, n_leaves, ctypes.byref(nt),
           ctypes.byref(nb), out.ctypes.data)
    return out, nt.value, nb.value


@pytest.mark.parametrize("depth,seed", [(4, 0), (5, 1), (6, 2), (6, 5)])
def test_index_names_the_leaf_of_every_cell(depth, seed):
    cells = scenes.random_tree_cells(depth, seed)
    child, _ = build_host(depth, 1, cells)
    desc = make_desc(depth, 1)
    index, nt, nb = _index(desc, child, len(cells))
    assert nb > 0 and nt >= 1 and not np.any(index == -7)
    n = 1 << depth
    for i in range(n):
        for j in range(n):
            for k in range(n):
                c = (i, j, k)
                assert _indexed(index, nt, depth, c) == _plain(child, depth, c), c


def test_index_on_sampled_cells_of_a_blob_band():
    s = scenes.scene_blobs(depth=7, sh_degree=1)
    child, _ = build_host(7, 1, s["cells"])
    desc = make_desc(7, 1)
    index, nt, nb = _index(desc, child, len(s["cells"]))
    # every data leaf appears in the index exactly as often as it has finest cells
    D, M = 7, 4
    rng = np.random.default_rng(0)
    for c in rng.integers(0, 1 << D, (20000, 3)):
        c = tuple(int(v) for v in c)
        assert _indexed(index, nt, D, c) == _plain(child, D, c), c
    # the cells of the band itself (all data, finest level)
    for cell in s["cells"][rng.choice(len(s["cells"]), 5000, replace=False)]:
        c = tuple(int(v) for v in cell[1:])
        leaf, lv = _indexed(index, nt, D, c)
        assert lv == D and leaf >= 0
    # counts: 2^(3(D - level)) entries per leaf of a level below M
    bricks = index[nt * 8:].reshape(nb, 512)
    leaves = (bricks >> 2) - 1
    data = leaves[leaves >= 0]
    assert len(np.unique(data)) == len(data)   # every finest leaf once
    assert M == D - 3


def test_index_refuses_shallow_and_malformed_trees():
    cells = scenes.random_tree_cells(5, 3)
    child, _ = build_host(5, 1, cells)
    nt, nb = ctypes.c_int64(), ctypes.c_int64()
    lib = L.lib()
    ch = np.ascontiguousarray(child, np.int32)
    d3 = make_desc(3, 1)
    assert lib.po_tree_index_host(ctypes.byref(d3), ch.shape[0], ch.ctypes.data, len(cells), ctypes.byref(nt),
                                  ctypes.byref(nb), None) == L.PO_ERR_INVALID
    bad = ch.copy()
    bad[0, 0] = ch.shape[0] + 3
    d5 = make_desc(5, 1)
    assert lib.po_tree_index_host(ctypes.byref(d5), bad.shape[0], bad.ctypes.data, len(cells), ctypes.byref(nt),
                                  ctypes.byref(nb), None) == L.PO_ERR_TREE
