"""Visibility filter of the conversion (Sec. 4.2, "Filtering"): alpha renders
of the training views raise every leaf's weight to the largest ray weight it
receives; leaves below a threshold are dropped and the octree is rebuilt from
the remaining cells.  Thin wrappers over po_leaf_weights and
po_tree_leaf_cells; the rebuild goes through the host builder."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from .render import _out, _stream_ptr, make_opts
from .tree import Tree

MODES = {"alpha": L.PO_WEIGHT_ALPHA, "contrib": L.PO_WEIGHT_CONTRIB}


def leaf_weights(tree: Tree, cams, stop_T=1e-4, mode="alpha", weight=None, alpha_out=None, stream=None):
    """Largest ray weight per leaf (float32 (n_leaves,) device tensor, tree
    leaf order) over the pixel rays of `cams`.  mode "alpha": the segment's
    1 - exp(-sigma delta); "contrib": T (1 - exp(-sigma delta)).  `weight`,
    if given, is raised in place.  `alpha_out`, if given, is a list of
    (H, W) float32 tensors, one per camera, that receive 1 - T."""
    import torch

    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    w = weight if weight is not None else torch.zeros(tree.n_leaves, dtype=torch.float32, device=tree.sigma.device)
    _out(w, (tree.n_leaves,), "weight")
    opts = make_opts(stop_T=stop_T)
    for i, cam in enumerate(cams):
        a = None
        if alpha_out is not None:
            a = _out(alpha_out[i], (cam.height, cam.width), "alpha_out[%d]" % i)
        c = cam.to_c()
        L.call("po_leaf_weights", tree.handle, ctypes.byref(c), ctypes.byref(opts), MODES[mode],
               w.data_ptr() if tree.n_leaves else None, a.data_ptr() if a is not None else None,
               _stream_ptr(stream))
    return w


def leaf_cells(tree: Tree) -> np.ndarray:
    """(n_leaves, 4) int32 (level, i, j, k) of every leaf, in tree leaf order."""
    child = np.ascontiguousarray(tree.child.cpu().numpy())
    cells = np.empty((tree.n_leaves, 4), np.int32)
    L.call("po_tree_leaf_cells", ctypes.byref(tree.desc), int(child.shape[0]), child.ctypes.data, tree.n_leaves,
           cells.ctypes.data if tree.n_leaves else None)
    return cells


def prune(tree: Tree, weight, tau: float):
    """New tree holding the leaves of `tree` whose weight is >= tau (Sec.
    4.2: the remaining voxels become the leaves, everything else empty).
    Returns (tree, kept) with kept the old leaf indices, in the caller order
    of the new tree's cells (its perm maps them to its leaf order)."""
    w = weight.float().cpu().numpy() if hasattr(weight, "cpu") else np.asarray(weight, np.float32)
    if w.shape != (tree.n_leaves,):
        raise ValueError("weight must hold one value per leaf")
    cells = leaf_cells(tree)
    kept = np.flatnonzero((w >= tau) & (cells[:, 0] >= 0))
    sig = tree.sigma.float().cpu().numpy()[kept]
    sh = tree.sh[:, :3 * tree.K].float().cpu().numpy()[kept]
    dtype = "f16" if tree.dtype == L.PO_F16 else "f32"
    lobes = tree.lobes.cpu().numpy() if tree.lobes is not None else None
    new = Tree.from_cells(tree.depth, tree.sh_degree, cells[kept], sig, sh, tree.center, tree.half, dtype=dtype,
                          device=tree.sigma.device, stride=tree.stride, lobes=lobes)
    return new, kept
