"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every entry point include/plenoctree.h declares, the octree builder
produces the tree its cell list defines, the validator rejects malformed
trees, and invalid arguments are refused before any GPU work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2103_14024_amd import _lib as L
from paper_2103_14024_amd import scenes
from paper_2103_14024_amd.tree import build_host, make_desc, validate_host

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "plenoctree.h")).read()
    declared = set(re.findall(r"^\s*(?:po_status|const char\*)\s+(po_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 17
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert getattr(lib, name) is not None
    assert L.version().startswith("plenoctree-mi355x")


def test_release_queues_without_any(lib):
    # nothing was rendered in pieces: nothing to free, no device touched
    L.call("po_release_queues")


def test_status_strings(lib):
    for s in range(6):
        assert L.status_str(s)
    assert L.status_str(0) == "ok"


def _walk(child, depth, lv, i, j, k):
    """Entry reached by descending from the root towards cell (lv, i, j, k)."""
    node = 0
    for L_ in range(lv):
        s = lv - 1 - L_
        oct_ = ((i >> s) & 1) << 2 | ((j >> s) & 1) << 1 | ((k >> s) & 1)
        e = int(child[node, oct_])
        if L_ == lv - 1:
            return e
        assert e > 0, "path to a leaf crosses a non-internal entry"
        node = e
    raise AssertionError


@pytest.mark.parametrize("seed,depth", [(0, 3), (1, 5), (2, 6)])
def test_builder_matches_cell_list(lib, seed, depth):
    cells = scenes.random_tree_cells(depth, seed)
    child, perm = build_host(depth, 2, cells)
    n = len(cells)
    assert sorted(perm.tolist()) == list(range(n))
    # every leaf j is reached at its own cell, and only there
    for j in range(n):
        lv, i, jj, k = cells[perm[j]]
        assert _walk(child, depth, lv, i, jj, k) == -j - 1
    assert (child < 0).sum() == n
    # internal nodes: exactly the distinct ancestors of the cells
    anc = {(0, 0, 0, 0)}
    for lv, i, j, k in cells:
        for a in range(1, lv):
            s = lv - a
            anc.add((a, i >> s, j >> s, k >> s))
    assert child.shape[0] == len(anc)
    # nodes numbered level by level: a child node id is larger than its parent's
    for v in range(child.shape[0]):
        for e in child[v]:
            if e > 0:
                assert e > v
    validate_host(depth, 2, child, n)


def test_builder_leaves_in_morton_order(lib):
    cells = scenes.spheres_cells(5, 3, 0)
    rng = np.random.default_rng(0)
    shuffled = cells[rng.permutation(len(cells))]
    child, perm = build_host(5, 2, shuffled)
    ijk = shuffled[perm][:, 1:].astype(np.int64)

    def morton(x, y, z):
        key = 0
        for b in range(5):
            key |= ((x >> b) & 1) << (3 * b + 2) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b)
        return key

    keys = [morton(*r) for r in ijk]
    assert keys == sorted(keys)


def test_builder_empty_and_full(lib):
    child, perm = build_host(3, 0, np.zeros((0, 4), np.int32))
    assert child.shape == (1, 8) and np.all(child == 0) and len(perm) == 0
    cells = np.array([[1, i >> 2 & 1, i >> 1 & 1, i & 1] for i in range(8)], np.int32)
    child, perm = build_host(1, 0, cells)
    assert child.shape == (1, 8) and sorted((-child[0] - 1).tolist()) == list(range(8))


@pytest.mark.parametrize("cells,msg", [
    ([[0, 0, 0, 0]], "level"),
    ([[4, 0, 0, 0]], "level"),
    ([[2, 4, 0, 0]], "coordinates"),
    ([[2, 0, -1, 0]], "coordinates"),
    ([[2, 1, 1, 1], [2, 1, 1, 1]], "overlap"),
    ([[1, 0, 0, 0], [3, 1, 2, 3]], "overlap"),
])
def test_builder_rejects_bad_cells(lib, cells, msg):
    with pytest.raises(L.PlenOctreeError) as ei:
        build_host(3, 1, np.asarray(cells, np.int32))
    assert ei.value.status == L.PO_ERR_TREE and msg in str(ei.value)


def _good_tree():
    cells = scenes.random_tree_cells(4, 3)
    child, perm = build_host(4, 1, cells)
    return cells, child


def test_validator_rejects_malformed(lib):
    cells, child = _good_tree()
    n = len(cells)
    validate_host(4, 1, child, n)
    internal = np.argwhere(child > 0)

    def bad(mutate, msg, depth=4, sigma=None):
        c = child.copy()
        mutate(c)
        with pytest.raises(L.PlenOctreeError) as ei:
            validate_host(depth, 1, c, n, sigma=sigma)
        assert ei.value.status == L.PO_ERR_TREE and msg in str(ei.value), str(ei.value)

    r, s = internal[-1]
    bad(lambda c: c.__setitem__((r, s), child.shape[0] + 5), "outside")           # out-of-range child
    bad(lambda c: c.__setitem__((r, s), -n - 3), "outside")                        # out-of-range leaf
    r2, s2 = internal[0]
    bad(lambda c: c.__setitem__((child[r2, s2], 0), child[r2, s2]), "more than once")   # cycle
    leaf_slot = np.argwhere(child < 0)[0]
    other = np.argwhere(child == 0)[0]
    bad(lambda c: c.__setitem__(tuple(other), child[tuple(leaf_slot)]), "more than once")  # shared leaf
    bad(lambda c: c.__setitem__((r, s), 0), "unreachable")                          # orphaned subtree
    bad(lambda c: None, "depth", depth=2)                                            # level > D
    sig = np.ones(n, np.float32)
    sig[n // 2] = np.nan
    bad(lambda c: None, "non-finite", sigma=sig)


def test_bind_and_argument_errors(lib):
    """bind only records pointers, so fake non-NULL addresses exercise it; every
    invalid render argument must be refused before a launch."""
    desc = make_desc(5, 2)
    h = ctypes.c_void_p()
    fake = 0x10000
    L.call("po_tree_bind", ctypes.byref(desc), 10, fake, 20, fake, fake, ctypes.byref(h))
    assert h.value
    opts = L.po_render_opts()
    opts.bg[0] = opts.bg[1] = opts.bg[2] = 1.0
    opts.stop_T = 1e-4
    st = lib.po_render_rays(h, -1, fake, fake, ctypes.byref(opts), fake, None, None)
    assert st == L.PO_ERR_INVALID
    assert lib.po_render_rays(h, 0, None, None, ctypes.byref(opts), None, None, None) == L.PO_OK  # n == 0: no-op
    assert lib.po_render_rays(h, 5, None, fake, ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    assert lib.po_render_rays(None, 5, fake, fake, ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    assert lib.po_render_rays(h, 5, fake, fake, None, fake, None, None) == L.PO_ERR_INVALID
    opts.flags = L.PO_OUT_AUX
    assert lib.po_render_rays(h, 5, fake, fake, ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    opts.flags = 0x80
    assert lib.po_render_rays(h, 5, fake, fake, ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    opts.flags = 0
    opts.stop_T = float("nan")
    assert lib.po_render_rays(h, 5, fake, fake, ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    opts.stop_T = 1e-4
    opts.max_steps = -1
    assert lib.po_render_rays(h, 5, fake, fake, ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    opts.max_steps = 0
    opts.clip[2] = float("nan")  # slicing plane must be finite
    assert lib.po_render_rays(h, 5, fake, fake, ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    opts.clip[2] = 0.0
    # viewer options have no gradient
    for field, val in (("sh_off", 2), ("clip", 1.0)):
        if field == "sh_off":
            opts.sh_off = val
        else:
            opts.clip[3] = val
        st = lib.po_render_rays_backward(h, 5, fake, fake, ctypes.byref(opts), fake, fake, fake, fake, None)
        assert st == L.PO_ERR_UNSUPPORTED and b"slicing" in lib.po_last_error()
        opts.sh_off, opts.clip[3] = 0, 0.0
    cam = L.po_camera()
    cam.width, cam.height, cam.fx, cam.fy = 0, 10, 1.0, 1.0
    assert lib.po_render_camera(h, ctypes.byref(cam), ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    cam.width, cam.fx = 10, 0.0
    assert lib.po_render_camera(h, ctypes.byref(cam), ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    cam.fx = 1.0
    cam.c2w[3] = float("inf")
    assert lib.po_render_camera(h, ctypes.byref(cam), ctypes.byref(opts), fake, None, None) == L.PO_ERR_INVALID
    cam.c2w[3] = 0.0
    assert lib.po_render_camera(h, ctypes.byref(cam), ctypes.byref(opts), None, None, None) == L.PO_ERR_INVALID
    n_t = ctypes.c_int32()
    L.call("po_camera_tiles", ctypes.byref(cam), ctypes.byref(n_t))
    assert n_t.value == 1
    # backward on a float16 tree is unsupported
    d16 = make_desc(5, 2, dtype=L.PO_F16, sh_stride=28)
    h16 = ctypes.c_void_p()
    L.call("po_tree_bind", ctypes.byref(d16), 10, fake, 20, fake, fake, ctypes.byref(h16))
    st = lib.po_render_rays_backward(h16, 5, fake, fake, ctypes.byref(opts), fake, fake, fake, fake, None)
    assert st == L.PO_ERR_UNSUPPORTED
    # batches: count and tile ranges
    jobs = (L.po_job * 1)()
    jobs[0].tree = h.value
    jobs[0].cam = cam
    jobs[0].opts = opts
    jobs[0].d_rgb = fake
    jobs[0].tile_begin, jobs[0].tile_end = 0, 2
    assert lib.po_render_batch(1, jobs, None) == L.PO_ERR_INVALID
    assert lib.po_render_batch(17, jobs, None) == L.PO_ERR_INVALID
    assert lib.po_render_batch(0, None, None) == L.PO_OK
    lib.po_tree_destroy(h16)
    lib.po_tree_destroy(h)


@pytest.mark.parametrize("field,value", [("depth", 0), ("depth", 16), ("sh_degree", 5), ("sh_degree", -1),
                                         ("half_size", 0.0), ("dtype", 7), ("sh_stride", 5)])
def test_bad_descriptions(lib, field, value):
    desc = make_desc(5, 2)
    setattr(desc, field, value)
    h = ctypes.c_void_p()
    st = lib.po_tree_bind(ctypes.byref(desc), 10, 0x1000, 20, 0x1000, 0x1000, ctypes.byref(h))
    assert st == L.PO_ERR_INVALID and L.lib().po_last_error()


def test_fp16_stride_must_be_dword_multiple(lib):
    desc = make_desc(5, 2, dtype=L.PO_F16, sh_stride=27)
    h = ctypes.c_void_p()
    assert lib.po_tree_bind(ctypes.byref(desc), 10, 0x1000, 20, 0x1000, 0x1000, ctypes.byref(h)) == L.PO_ERR_INVALID
    desc.sh_stride = 0  # 3K = 27 halves: not a multiple of 4 bytes
    assert lib.po_tree_bind(ctypes.byref(desc), 10, 0x1000, 20, 0x1000, 0x1000, ctypes.byref(h)) == L.PO_ERR_INVALID


@pytest.mark.parametrize("seed,depth", [(0, 4), (3, 6)])
def test_leaf_cells_recover_the_builder_input(lib, seed, depth):
    cells = scenes.random_tree_cells(depth, seed)
    child, perm = build_host(depth, 2, cells)
    desc = make_desc(depth, 2)
    n = len(cells)
    out = np.empty((n, 4), np.int32)
    ch = np.ascontiguousarray(child)
    L.call("po_tree_leaf_cells", ctypes.byref(desc), ch.shape[0], ch.ctypes.data, n, out.ctypes.data)
    # leaf j of the tree is the caller's cell perm[j]
    np.testing.assert_array_equal(out, np.asarray(cells, np.int32)[perm])
    # a leaf index no entry references is reported as (-1, -1, -1, -1)
    out2 = np.empty((n + 1, 4), np.int32)
    L.call("po_tree_leaf_cells", ctypes.byref(desc), ch.shape[0], ch.ctypes.data, n + 1, out2.ctypes.data)
    assert np.all(out2[n] == -1) and np.array_equal(out2[:n], out)
    # a malformed array is refused
    bad = ch.copy()
    bad[0, 0] = ch.shape[0] + 5
    st = lib.po_tree_leaf_cells(ctypes.byref(desc), bad.shape[0], bad.ctypes.data, n, out.ctypes.data)
    assert st == L.PO_ERR_TREE


def test_codebook_bind_and_render_errors(lib):
    fake = 0x10000
    d16 = make_desc(5, 2, dtype=L.PO_F16)
    h = ctypes.c_void_p()
    # codebook trees need float16 densities, an even index stride >= K and 1..65536 aligned entries
    d32 = make_desc(5, 2)
    assert lib.po_tree_bind_codebook(ctypes.byref(d32), 10, fake, 20, fake, fake, fake, 256, ctypes.byref(h)) == L.PO_ERR_INVALID
    assert lib.po_tree_bind_codebook(ctypes.byref(d16), 10, fake, 20, fake, fake, fake, 0, ctypes.byref(h)) == L.PO_ERR_INVALID
    assert lib.po_tree_bind_codebook(ctypes.byref(d16), 10, fake, 20, fake, fake, fake, 65537, ctypes.byref(h)) == L.PO_ERR_INVALID
    assert lib.po_tree_bind_codebook(ctypes.byref(d16), 10, fake, 20, fake, fake, fake + 4, 16, ctypes.byref(h)) == L.PO_ERR_INVALID
    assert lib.po_tree_bind_codebook(ctypes.byref(d16), 10, fake, 20, fake, fake, None, 16, ctypes.byref(h)) == L.PO_ERR_INVALID
    odd = make_desc(5, 2, dtype=L.PO_F16, sh_stride=11)
    assert lib.po_tree_bind_codebook(ctypes.byref(odd), 10, fake, 20, fake, fake, fake, 16, ctypes.byref(h)) == L.PO_ERR_INVALID
    short = make_desc(5, 2, dtype=L.PO_F16, sh_stride=8)
    assert lib.po_tree_bind_codebook(ctypes.byref(short), 10, fake, 20, fake, fake, fake, 16, ctypes.byref(h)) == L.PO_ERR_INVALID
    L.call("po_tree_bind_codebook", ctypes.byref(d16), 10, fake, 20, fake, fake, fake, 16, ctypes.byref(h))
    opts = L.po_render_opts()
    opts.stop_T = 1e-4
    # no viewer outputs and no gradients for codebook trees
    opts.flags = L.PO_OUT_AUX
    assert lib.po_render_rays(h, 5, fake, fake, ctypes.byref(opts), fake, fake, None) == L.PO_ERR_UNSUPPORTED
    opts.flags = 0
    opts.sh_off = 1
    cam = L.po_camera()
    cam.width, cam.height, cam.fx, cam.fy = 8, 8, 1.0, 1.0
    assert lib.po_render_camera(h, ctypes.byref(cam), ctypes.byref(opts), fake, None, None) == L.PO_ERR_UNSUPPORTED
    opts.sh_off = 0
    st = lib.po_render_rays_backward(h, 5, fake, fake, ctypes.byref(opts), fake, fake, fake, fake, None)
    assert st == L.PO_ERR_UNSUPPORTED
    lib.po_tree_destroy(h)
