"""Rendering and gradient calls (thin wrappers over the C ABI) and the
torch.autograd.Function used for direct octree optimisation (Sec. 4.3)."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib as L


def _torch():
    import torch

    return torch


# columns of the aux output: final transmittance (1 - alpha), data samples,
# traversal steps, expected termination distance (depth map)
AUX_T, AUX_SAMPLES, AUX_STEPS, AUX_DEPTH = 0, 1, 2, 3
AUX_WIDTH = 4


def make_opts(bg=(1.0, 1.0, 1.0), stop_T=1e-4, max_steps=0, aux=False, sh_off=0, clip=None,
              one_pass=False) -> L.po_render_opts:
    """Render options.  sh_off: bit k leaves out SH basis function k; clip:
    slicing plane (nx, ny, nz, w), only n.x + w >= 0 is rendered; one_pass:
    every ray walked to its end by one lane, never in pieces."""
    o = L.po_render_opts()
    for k in range(3):
        o.bg[k] = float(bg[k])
    o.stop_T = float(stop_T)
    o.max_steps = int(max_steps)
    o.flags = (L.PO_OUT_AUX if aux else 0) | (L.PO_ONE_PASS if one_pass else 0)
    o.sh_off = int(sh_off) & 0xFFFFFFFF
    if clip is not None:
        c = [float(v) for v in clip]
        if len(c) != 4:
            raise ValueError("clip must hold 4 values (nx, ny, nz, w)")
        for k in range(4):
            o.clip[k] = c[k]
    return o


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _out(t, shape, name):
    """A caller-supplied output must be a contiguous float32 device tensor of the given shape."""
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float32 and tuple(t.shape) == tuple(shape) and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor of shape {tuple(shape)}")
    return t


def _rays3(t, name):
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.shape[1] == 3 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 (n, 3) device tensor")


@dataclass
class Camera:
    """Pinhole camera: c2w row-major 3x4 (right, up, backward, position)."""
    c2w: np.ndarray
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def to_c(self) -> L.po_camera:
        c = L.po_camera()
        m = np.asarray(self.c2w, np.float32).reshape(12)
        for i in range(12):
            c.c2w[i] = float(m[i])
        c.width, c.height = int(self.width), int(self.height)
        c.fx, c.fy, c.cx, c.cy = float(self.fx), float(self.fy), float(self.cx), float(self.cy)
        return c

    @property
    def n_tiles(self) -> int:
        return ((self.width + L.PO_TILE - 1) // L.PO_TILE) * ((self.height + L.PO_TILE - 1) // L.PO_TILE)


def render_rays(tree, origins, dirs, bg=(1.0, 1.0, 1.0), stop_T=1e-4, aux=False, max_steps=0, out=None,
                aux_out=None, stream=None, sh_off=0, clip=None, one_pass=False):
    """Colours (n, 3) of rays (origins, dirs: float32 (n, 3) device tensors);
    with aux also the (n, 4) columns AUX_T, AUX_SAMPLES, AUX_STEPS, AUX_DEPTH."""
    torch = _torch()
    _rays3(origins, "origins")
    _rays3(dirs, "dirs")
    n = origins.shape[0]
    if dirs.shape[0] != n:
        raise ValueError("origins and dirs differ in length")
    rgb = _out(out, (n, 3), "out") if out is not None else torch.empty((n, 3), dtype=torch.float32,
                                                                       device=origins.device)
    a = None
    if aux:
        a = _out(aux_out, (n, AUX_WIDTH), "aux_out") if aux_out is not None else torch.empty(
            (n, AUX_WIDTH), dtype=torch.float32, device=origins.device)
    opts = make_opts(bg, stop_T, max_steps, aux, sh_off, clip, one_pass)
    L.call("po_render_rays", tree.handle, n, origins.data_ptr(), dirs.data_ptr(), ctypes.byref(opts),
           rgb.data_ptr(), a.data_ptr() if a is not None else None, _stream_ptr(stream))
    return (rgb, a) if aux else rgb


def render_camera(tree, cam: Camera, bg=(1.0, 1.0, 1.0), stop_T=1e-4, aux=False, max_steps=0, out=None,
                  aux_out=None, stream=None, device="cuda", sh_off=0, clip=None, one_pass=False):
    """Image (H, W, 3) of a camera; with aux also (H, W, 4) aux columns."""
    torch = _torch()
    shape = (cam.height, cam.width, 3)
    img = _out(out, shape, "out") if out is not None else torch.empty(shape, dtype=torch.float32, device=device)
    a = None
    if aux:
        ashape = (cam.height, cam.width, AUX_WIDTH)
        a = _out(aux_out, ashape, "aux_out") if aux_out is not None else torch.empty(
            ashape, dtype=torch.float32, device=device)
    opts = make_opts(bg, stop_T, max_steps, aux, sh_off, clip, one_pass)
    c = cam.to_c()
    L.call("po_render_camera", tree.handle, ctypes.byref(c), ctypes.byref(opts), img.data_ptr(),
           a.data_ptr() if a is not None else None, _stream_ptr(stream))
    return (img, a) if aux else img


def render_camera_noalloc(tree, cam: Camera, out, aux_out=None, bg=(1.0, 1.0, 1.0), stop_T=1e-4, max_steps=0,
                          stream=None, sh_off=0, clip=None, one_pass=False):
    """render_camera through po_render_camera_noalloc, for callers that cannot
    allocate device memory: the library allocates nothing (its work queue is
    a fixed per-device array), and the caller passes the image `out`
    (H, W, 3) and, for the aux columns, `aux_out` (H, W, 4).  Calls on one
    GPU share that queue and must not overlap.  Images of more than 2^22
    pixels are rejected."""
    shape = (cam.height, cam.width, 3)
    img = _out(out, shape, "out")
    a = None
    if aux_out is not None:
        a = _out(aux_out, (cam.height, cam.width, AUX_WIDTH), "aux_out")
    opts = make_opts(bg, stop_T, max_steps, a is not None, sh_off, clip, one_pass)
    c = cam.to_c()
    L.call("po_render_camera_noalloc", tree.handle, ctypes.byref(c), ctypes.byref(opts), img.data_ptr(),
           a.data_ptr() if a is not None else None, _stream_ptr(stream))
    return (img, a) if a is not None else img


def camera_rays(cam: Camera, stream=None, device="cuda"):
    """(origins, unit dirs) of a camera's pixel-centre rays, (H*W, 3) float32 each."""
    torch = _torch()
    n = cam.width * cam.height
    o = torch.empty((n, 3), dtype=torch.float32, device=device)
    d = torch.empty((n, 3), dtype=torch.float32, device=device)
    c = cam.to_c()
    L.call("po_camera_rays", ctypes.byref(c), o.data_ptr(), d.data_ptr(), _stream_ptr(stream))
    return o, d


def render_rays_backward(tree, origins, dirs, rgb_fwd, grad_rgb, bg=(1.0, 1.0, 1.0), stop_T=1e-4, max_steps=0,
                         grad_sigma=None, grad_sh=None, stream=None, one_pass=False):
    """Accumulates dL/dsigma (n_leaves,) and dL/dsh (n_leaves, stride); returns both."""
    torch = _torch()
    _rays3(origins, "origins")
    _rays3(dirs, "dirs")
    _rays3(rgb_fwd, "rgb_fwd")
    _rays3(grad_rgb, "grad_rgb")
    n = origins.shape[0]
    for t, name in ((dirs, "dirs"), (rgb_fwd, "rgb_fwd"), (grad_rgb, "grad_rgb")):
        if t.shape[0] != n:
            raise ValueError(f"{name} has {t.shape[0]} rows, origins {n}")
    # the kernels add into grad_sigma[leaf] and grad_sh[leaf * stride + e]
    shape_sh = (tree.n_leaves, tree.stride)
    if grad_sigma is None:
        grad_sigma = torch.zeros((tree.n_leaves,), dtype=torch.float32, device=origins.device)
    else:
        _out(grad_sigma, (tree.n_leaves,), "grad_sigma")
    if grad_sh is None:
        grad_sh = torch.zeros(shape_sh, dtype=torch.float32, device=origins.device)
    else:
        _out(grad_sh, shape_sh, "grad_sh")
    opts = make_opts(bg, stop_T, max_steps, one_pass=one_pass)
    L.call("po_render_rays_backward", tree.handle, n, origins.data_ptr(), dirs.data_ptr(),
           ctypes.byref(opts), rgb_fwd.data_ptr(), grad_rgb.data_ptr(), grad_sigma.data_ptr(), grad_sh.data_ptr(),
           _stream_ptr(stream))
    return grad_sigma, grad_sh


def _slots(t, n):
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.int32 and tuple(t.shape) == (n,) and t.is_contiguous()):
        raise ValueError(f"ray_slot must be a contiguous int32 device tensor of shape ({n},)")
    return t


def render_rays_keep(tree, origins, dirs, ray_slot, bg=(1.0, 1.0, 1.0), stop_T=1e-4, max_steps=0, out=None,
                     stream=None, one_pass=False):
    """render_rays (float32 tree, no aux or viewer options) that keeps its
    pieces in the stream's work queue for render_rays_backward_kept;
    ray_slot: (n,) int32 device tensor the library overwrites."""
    torch = _torch()
    _rays3(origins, "origins")
    _rays3(dirs, "dirs")
    n = origins.shape[0]
    if dirs.shape[0] != n:
        raise ValueError("origins and dirs differ in length")
    _slots(ray_slot, n)
    rgb = _out(out, (n, 3), "out") if out is not None else torch.empty((n, 3), dtype=torch.float32,
                                                                       device=origins.device)
    opts = make_opts(bg, stop_T, max_steps, one_pass=one_pass)
    L.call("po_render_rays_keep", tree.handle, n, origins.data_ptr(), dirs.data_ptr(), ctypes.byref(opts),
           rgb.data_ptr(), ray_slot.data_ptr(), _stream_ptr(stream))
    return rgb


def render_rays_backward_kept(tree, origins, dirs, rgb_fwd, grad_rgb, ray_slot, grad_sigma, grad_sh,
                              bg=(1.0, 1.0, 1.0), stop_T=1e-4, max_steps=0, stream=None, one_pass=False):
    """render_rays_backward of the rays of the last render_rays_keep on the
    same stream (same tree, tensors and options), reusing its pieces;
    accumulates into grad_sigma (n_leaves,) and grad_sh (n_leaves, stride)."""
    _rays3(origins, "origins")
    _rays3(dirs, "dirs")
    _rays3(rgb_fwd, "rgb_fwd")
    _rays3(grad_rgb, "grad_rgb")
    n = origins.shape[0]
    for t, name in ((dirs, "dirs"), (rgb_fwd, "rgb_fwd"), (grad_rgb, "grad_rgb")):
        if t.shape[0] != n:
            raise ValueError(f"{name} has {t.shape[0]} rows, origins {n}")
    _slots(ray_slot, n)
    _out(grad_sigma, (tree.n_leaves,), "grad_sigma")
    _out(grad_sh, (tree.n_leaves, tree.stride), "grad_sh")
    opts = make_opts(bg, stop_T, max_steps, one_pass=one_pass)
    L.call("po_render_rays_backward_kept", tree.handle, n, origins.data_ptr(), dirs.data_ptr(), ctypes.byref(opts),
           rgb_fwd.data_ptr(), grad_rgb.data_ptr(), grad_sigma.data_ptr(), grad_sh.data_ptr(), ray_slot.data_ptr(),
           _stream_ptr(stream))
    return grad_sigma, grad_sh


class RenderRaysFn:
    """torch.autograd.Function over (sigma, sh) of a float32 tree.

    Forward renders the rays (the first pass of App. B.3's Remark, storing the
    full colour C); backward replays the walk and accumulates the leaf
    gradients with atomics (the second pass).  The forward keeps its pieces
    (render_rays_keep), and the backward differentiates over them when they
    are still valid (no other split work on the stream in between, first
    backward of this forward), else it walks the rays again
    (render_rays_backward): both give the gradient of the same colours."""

    _fn = None

    @classmethod
    def get(cls):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, sigma, sh, tree, origins, dirs, bg, stop_T):
                    if sigma.data_ptr() != tree.sigma.data_ptr() or sh.data_ptr() != tree.sh.data_ptr():
                        raise ValueError("sigma/sh must be the tensors the tree is bound to")
                    if tree.dtype == L.PO_F32:
                        slot = torch.empty(origins.shape[0], dtype=torch.int32, device=origins.device)
                        rgb = render_rays_keep(tree, origins, dirs, slot, bg=bg, stop_T=stop_T)
                    else:
                        # float16 and codebook trees render; their backward is refused
                        slot = None
                        rgb = render_rays(tree, origins, dirs, bg=bg, stop_T=stop_T)
                    ctx.tree, ctx.bg, ctx.stop_T, ctx.kept = tree, bg, stop_T, slot is not None
                    ctx.save_for_backward(origins, dirs, rgb, slot)
                    return rgb

                @staticmethod
                def backward(ctx, grad_rgb):
                    origins, dirs, rgb, slot = ctx.saved_tensors
                    g = grad_rgb.contiguous()
                    tr = ctx.tree
                    gs = torch.zeros((tr.n_leaves,), dtype=torch.float32, device=origins.device)
                    gh = torch.zeros((tr.n_leaves, tr.stride), dtype=torch.float32, device=origins.device)
                    kept = ctx.kept
                    if kept:
                        try:
                            render_rays_backward_kept(tr, origins, dirs, rgb, g, slot, gs, gh, bg=ctx.bg,
                                                      stop_T=ctx.stop_T)
                        except L.PlenOctreeError as e:
                            if e.status != L.PO_ERR_INVALID:
                                raise
                            kept = False  # the kept pieces are gone: walk the rays again
                    if not kept:
                        render_rays_backward(tr, origins, dirs, rgb, g, bg=ctx.bg, stop_T=ctx.stop_T,
                                             grad_sigma=gs, grad_sh=gh)
                    return gs, gh, None, None, None, None, None

            cls._fn = _F
        return cls._fn


def render_rays_differentiable(tree, origins, dirs, bg=(1.0, 1.0, 1.0), stop_T=1e-4):
    """Differentiable render of a float32 tree: gradients flow to tree.sigma
    and tree.sh (set requires_grad on them first)."""
    return RenderRaysFn.get().apply(tree.sigma, tree.sh, tree, origins, dirs, tuple(bg), float(stop_T))


@dataclass
class Job:
    tree: object
    cam: Camera
    out: object            # (H, W, 3) float32 device tensor
    tile_begin: int = 0
    tile_end: int = -1     # -1: to the last tile
    bg: tuple = (1.0, 1.0, 1.0)
    stop_T: float = 1e-4
    aux_out: object = None  # (H, W, 4) float32 device tensor or None
    sh_off: int = 0
    clip: object = None
    one_pass: bool = False  # never in pieces (jobs of >= 256 tiles otherwise are)


def render_batch(jobs, stream=None) -> None:
    """Renders up to 16 camera jobs (any trees, any sizes, tile sub-ranges);
    jobs of 256 tiles or more are rendered in pieces unless one_pass is set."""
    arr = (L.po_job * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        _out(j.out, (j.cam.height, j.cam.width, 3), "Job.out")
        if j.aux_out is not None:
            _out(j.aux_out, (j.cam.height, j.cam.width, AUX_WIDTH), "Job.aux_out")
        arr[i].tree = j.tree.handle.value
        arr[i].cam = j.cam.to_c()
        arr[i].opts = make_opts(j.bg, j.stop_T, 0, j.aux_out is not None, j.sh_off, j.clip, j.one_pass)
        arr[i].d_rgb = j.out.data_ptr()
        arr[i].d_aux = j.aux_out.data_ptr() if j.aux_out is not None else None
        arr[i].tile_begin = int(j.tile_begin)
        arr[i].tile_end = int(j.cam.n_tiles if j.tile_end < 0 else j.tile_end)
    L.call("po_render_batch", len(jobs), arr, _stream_ptr(stream))


def traversal_stats(tree, cam=None, origins=None, dirs=None, stop_T=1e-4, max_steps=0, stream=None) -> dict:
    """Unit counts of the one-pass walk of a camera's pixel rays, or of the
    rays (origins, dirs), waiting for the stream: rays, data samples, cells
    visited and child entries read."""
    v = (ctypes.c_int64 * 4)()
    opts = make_opts((1.0, 1.0, 1.0), stop_T, max_steps)
    if cam is not None:
        c = cam.to_c()
        L.call("po_traversal_stats", tree.handle, ctypes.byref(c), ctypes.byref(opts),
               ctypes.cast(v, ctypes.c_void_p), _stream_ptr(stream))
    else:
        _rays3(origins, "origins")
        _rays3(dirs, "dirs")
        if dirs.shape[0] != origins.shape[0]:
            raise ValueError("origins and dirs differ in length")
        L.call("po_traversal_stats_rays", tree.handle, origins.shape[0], origins.data_ptr(), dirs.data_ptr(),
               ctypes.byref(opts), ctypes.cast(v, ctypes.c_void_p), _stream_ptr(stream))
    return {"rays": int(v[0]), "samples": int(v[1]), "cells": int(v[2]), "node_loads": int(v[3])}


def device_errors() -> int:
    v = ctypes.c_int64()
    L.call("po_device_errors", ctypes.byref(v))
    return int(v.value)


def reset_device_errors() -> None:
    L.call("po_device_errors_reset")


def reserve_queues(stream=None) -> None:
    """Allocates the split-render work queue of `stream` now (torch's current
    stream by default), so that no later render on it allocates."""
    L.call("po_reserve_queues", _stream_ptr(stream))


def release_queues() -> None:
    """Frees the split-render work queues (waits for the devices first)."""
    L.call("po_release_queues")
