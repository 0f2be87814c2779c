"""ctypes binding of libplenoctree.so (include/plenoctree.h), names unchanged.

Argument marshalling only: every step of rendering and differentiation runs
in the HIP library.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libplenoctree.so")

PO_OK, PO_ERR_INVALID, PO_ERR_TREE, PO_ERR_OOM, PO_ERR_DEVICE, PO_ERR_UNSUPPORTED = range(6)
PO_F32, PO_F16 = 0, 1
PO_OUT_AUX = 1
PO_ONE_PASS = 2
PO_WEIGHT_ALPHA, PO_WEIGHT_CONTRIB = 0, 1
PO_MAX_DEPTH = 15
PO_MAX_SH_DEGREE = 4
PO_BATCH_MAX_JOBS = 16
PO_TILE = 16


class po_tree_desc(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("sh_degree", ctypes.c_int32), ("center", ctypes.c_float * 3),
                ("half_size", ctypes.c_float), ("dtype", ctypes.c_int32), ("sh_stride", ctypes.c_int32)]


class po_render_opts(ctypes.Structure):
    _fields_ = [("bg", ctypes.c_float * 3), ("stop_T", ctypes.c_float), ("max_steps", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("sh_off", ctypes.c_uint32), ("clip", ctypes.c_float * 4)]


class po_camera(ctypes.Structure):
    _fields_ = [("c2w", ctypes.c_float * 12), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class po_job(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_void_p), ("cam", po_camera), ("opts", po_render_opts),
                ("d_rgb", ctypes.c_void_p), ("d_aux", ctypes.c_void_p), ("tile_begin", ctypes.c_int32),
                ("tile_end", ctypes.c_int32)]


class PlenOctreeError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn}: {status_str(status)} ({status}): {msg}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32

# name -> argtypes; every function returns po_status (int)
_SIGS = {
    "po_builder_create": [ctypes.POINTER(po_tree_desc), _I64, _P, ctypes.POINTER(_P)],
    "po_builder_sizes": [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
    "po_builder_emit": [_P, _P, _P],
    "po_builder_destroy": [_P],
    "po_tree_validate": [ctypes.POINTER(po_tree_desc), _I64, _P, _I64, _P],
    "po_tree_bind": [ctypes.POINTER(po_tree_desc), _I64, _P, _I64, _P, _P, ctypes.POINTER(_P)],
    "po_tree_bind_sg": [ctypes.POINTER(po_tree_desc), _I64, _P, _I64, _P, _P, _P, ctypes.POINTER(_P)],
    "po_tree_bind_codebook": [ctypes.POINTER(po_tree_desc), _I64, _P, _I64, _P, _P, _P, _I32, ctypes.POINTER(_P)],
    "po_codebook_build": [_I64, _I32, _P, _I64, _I32, _P, _P, _I64, _P],
    "po_tree_destroy": [_P],
    "po_tree_build_index": [_P, _P],
    "po_tree_index_host": [ctypes.POINTER(po_tree_desc), _I64, _P, _I64, _P, _P, _P],
    "po_render_rays": [_P, _I64, _P, _P, ctypes.POINTER(po_render_opts), _P, _P, _P],
    "po_render_camera": [_P, ctypes.POINTER(po_camera), ctypes.POINTER(po_render_opts), _P, _P, _P],
    "po_render_camera_noalloc": [_P, ctypes.POINTER(po_camera), ctypes.POINTER(po_render_opts), _P, _P, _P],
    "po_render_rays_backward": [_P, _I64, _P, _P, ctypes.POINTER(po_render_opts), _P, _P, _P, _P, _P],
    "po_render_rays_keep": [_P, _I64, _P, _P, ctypes.POINTER(po_render_opts), _P, _P, _P],
    "po_render_rays_backward_kept": [_P, _I64, _P, _P, ctypes.POINTER(po_render_opts), _P, _P, _P, _P, _P, _P],
    "po_render_batch": [_I32, ctypes.POINTER(po_job), _P],
    "po_camera_tiles": [ctypes.POINTER(po_camera), ctypes.POINTER(_I32)],
    "po_camera_rays": [ctypes.POINTER(po_camera), _P, _P, _P],
    "po_mse_grad": [_I64, _P, _P, ctypes.c_float, _P, _P, _P],
    "po_sgd_step": [_I64, _P, _P, ctypes.c_float, _I32, _P],
    "po_gather_rays": [_I64, _P, _I64, _P, _P, _P, _P, _P, _P, _P],
    "po_draw_batch": [_I64, ctypes.c_uint64, ctypes.c_uint64, _I64, _P, _P, _P, _P, _P, _P, _P, _P],
    "po_leaf_weights": [_P, ctypes.POINTER(po_camera), ctypes.POINTER(po_render_opts), _I32, _P, _P, _P],
    "po_tree_leaf_cells": [ctypes.POINTER(po_tree_desc), _I64, _P, _I64, _P],
    "po_device_errors": [ctypes.POINTER(_I64)],
    "po_device_errors_reset": [],
    "po_release_queues": [],
    "po_reserve_queues": [_P],
    "po_traversal_stats": [_P, ctypes.POINTER(po_camera), ctypes.POINTER(po_render_opts), _P, _P],
    "po_traversal_stats_rays": [_P, _I64, _P, _P, ctypes.POINTER(po_render_opts), _P, _P],
}
EXPORTS = list(_SIGS) + ["po_status_str", "po_last_error", "po_version"]


def lib():
    """The loaded library; raises if libplenoctree.so has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()' or python paper_2103_14024_amd/_build.py)")
    L = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    for name in ("po_status_str",):
        getattr(L, name).restype = ctypes.c_char_p
        getattr(L, name).argtypes = [ctypes.c_int]
    for name in ("po_last_error", "po_version"):
        getattr(L, name).restype = ctypes.c_char_p
        getattr(L, name).argtypes = []
    _lib = L
    return L


def status_str(s: int) -> str:
    return lib().po_status_str(s).decode()


def check(status: int, fn: str) -> None:
    if status != PO_OK:
        raise PlenOctreeError(status, fn, lib().po_last_error().decode())


def call(name: str, *args) -> None:
    """Calls po_<name> and raises PlenOctreeError on a non-OK status."""
    check(getattr(lib(), name)(*args), name)


def version() -> str:
    return lib().po_version().decode()
