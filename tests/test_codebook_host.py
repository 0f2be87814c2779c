"""The library's codebook builder (po_codebook_build, host C++, App. B.2)
against the oracle's median cut: the two are written independently from the
same exact definition, so box numbers and float16 colours must agree bit for
bit.  Also the argument checks of the entry point."""
import ctypes

import numpy as np
import pytest

from paper_2103_14024_amd import _lib as L
from paper_2103_14024_amd import scenes
from paper_2103_14024_amd.tree import codebook_build


def _check(oracle_mod, sh, M):
    cb, idx, boxes = codebook_build(sh, M)
    n, _, K = sh.shape
    o_idx, books = oracle_mod.codebook(sh, M)
    for k in range(K):
        nb = len(books[k])
        assert boxes[k] == nb
        np.testing.assert_array_equal(idx[:, k].astype(np.int64), o_idx[:, k])
        np.testing.assert_array_equal(cb[k, :nb, :3], books[k].view(np.uint16))
        assert np.all(cb[k, nb:] == 0) and np.all(cb[k, :, 3] == 0)
    assert np.all(idx[:, K:] == 0)
    return cb, idx, boxes


@pytest.mark.parametrize("M", [1, 7, 64, 1000])
def test_builder_matches_oracle(oracle_mod, M):
    rng = np.random.default_rng(M)
    sh = rng.normal(0, 0.5, (3000, 3, 9)).astype(np.float32)
    sh[::7] = sh[3]          # repeated leaves: medians inside runs of equal values
    sh[5::11, 1, :] = 0.25   # ties on one axis
    _check(oracle_mod, sh, M)


def test_scene_leaves_and_full_size_codebook(oracle_mod):
    sc = scenes.scene_small(sh_degree=3)
    sh = np.asarray(sc["sh"], np.float32)
    cb, idx, boxes = _check(oracle_mod, sh, 65536)
    # more colours than leaves: every leaf keeps its own colour up to float16 rounding
    dec = np.stack([cb[k][idx[:, k], :3] for k in range(16)], axis=2).view(np.float16).astype(np.float32)
    np.testing.assert_array_equal(dec, sh.astype(np.float16).astype(np.float32))


def test_builder_argument_errors():
    lib = L.lib()
    sh = np.zeros((10, 3, 9), np.float32)
    cb = np.zeros((9, 16, 4), np.uint16)
    idx = np.zeros((10, 12), np.uint16)

    def run(n=10, K=9, coef_stride=27, M=16, index_stride=12, coef=sh):
        return lib.po_codebook_build(n, K, coef.ctypes.data, coef_stride, M, cb.ctypes.data, idx.ctypes.data,
                                     index_stride, None)

    assert run() == L.PO_OK
    assert run(M=0) == L.PO_ERR_INVALID
    assert run(M=65537) == L.PO_ERR_INVALID
    assert run(K=0) == L.PO_ERR_INVALID and run(K=36) == L.PO_ERR_INVALID
    assert run(coef_stride=26) == L.PO_ERR_INVALID
    assert run(index_stride=8) == L.PO_ERR_INVALID
    assert run(n=-1) == L.PO_ERR_INVALID
    bad = sh.copy()
    bad[4, 2, 3] = np.nan
    assert run(coef=bad) == L.PO_ERR_INVALID and b"finite" in lib.po_last_error()
    assert lib.po_codebook_build(0, 9, None, 27, 16, cb.ctypes.data, None, 12, None) == L.PO_OK
