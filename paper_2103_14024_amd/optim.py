"""Direct optimisation of a PlenOctree's leaf values (Sec. 4.3; App. B.5).

The tree structure is fixed; the raw densities and SH coefficients of a
float32 tree are fitted to target pixel colours with the NeRF loss (Sec. 3,
eqn:nerfloss; here the mean over the batch and the colour channels) and plain
SGD.  One step: forward render of a random ray batch that keeps its pieces
(the first pass of the App. B.3 scheme), loss gradient, backward replay with
atomics over the same pieces (second pass), SGD updates that also clear the
gradients -- library calls only, the batch drawn on the device from a
counter-based generator (po_draw_batch).  torch holds the buffers.
"""
from __future__ import annotations

import ctypes

from . import _lib as L
from .render import _stream_ptr, make_opts


class Trainer:
    """SGD on tree.sigma and tree.sh (float32 tree) against a ray dataset.

    origins, dirs, target: (N, 3) float32 device tensors (all training
    pixels); each step draws `batch` of them uniformly with replacement, step
    k taking elements [k batch, (k + 1) batch) of the SplitMix64 sequence of
    `seed`."""

    def __init__(self, tree, origins, dirs, target, lr_sigma, lr_sh, batch=65536, bg=(1.0, 1.0, 1.0), stop_T=1e-4,
                 seed=0):
        import torch

        if tree.dtype != L.PO_F32:
            raise ValueError("optimisation needs a float32 tree")
        self.tree, self.o, self.d, self.t = tree, origins, dirs, target
        self.lr_sigma, self.lr_sh, self.batch = float(lr_sigma), float(lr_sh), int(batch)
        self.bg, self.stop_T = tuple(bg), float(stop_T)
        dev = origins.device
        if not 0 <= int(seed) < 2 ** 64:
            raise ValueError("seed must fit in 64 bits")
        self.seed = int(seed)
        f = dict(dtype=torch.float32, device=dev)
        self.bo = torch.empty((batch, 3), **f)
        self.bd = torch.empty((batch, 3), **f)
        self.bt = torch.empty((batch, 3), **f)
        self.rgb = torch.empty((batch, 3), **f)
        self.grad_rgb = torch.empty((batch, 3), **f)
        self.sq = torch.zeros(1, **f)
        self.slot = torch.empty(batch, dtype=torch.int32, device=dev)
        self.g_sigma = torch.zeros_like(tree.sigma)
        self.g_sh = torch.zeros_like(tree.sh)
        self.opts = make_opts(bg, stop_T)
        self.steps = 0

    def step(self, stream=None):
        """One SGD step on `stream` (None: torch's current stream); returns the
        batch loss as a 1-element device tensor (mean squared error over rays
        and channels), valid once the stream has completed.  The batch gather
        and the loss scaling run on the same stream as the library calls."""
        import torch

        ts = stream if stream is not None else torch.cuda.current_stream(self.o.device)
        s = _stream_ptr(ts)
        n = self.batch
        tr = self.tree
        with torch.cuda.stream(ts):
            # the batch, and the loss accumulator cleared
            L.call("po_draw_batch", n, ctypes.c_uint64(self.seed), ctypes.c_uint64(self.steps * n), self.o.shape[0],
                   self.o.data_ptr(), self.d.data_ptr(), self.t.data_ptr(), self.bo.data_ptr(), self.bd.data_ptr(),
                   self.bt.data_ptr(), self.sq.data_ptr(), s)
            # the render keeps its pieces for the backward (App. B.3's two passes)
            L.call("po_render_rays_keep", tr.handle, n, self.bo.data_ptr(), self.bd.data_ptr(),
                   ctypes.byref(self.opts), self.rgb.data_ptr(), self.slot.data_ptr(), s)
            L.call("po_mse_grad", n, self.rgb.data_ptr(), self.bt.data_ptr(), ctypes.c_float(1.0 / (3 * n)),
                   self.grad_rgb.data_ptr(), self.sq.data_ptr(), s)
            L.call("po_render_rays_backward_kept", tr.handle, n, self.bo.data_ptr(), self.bd.data_ptr(),
                   ctypes.byref(self.opts), self.rgb.data_ptr(), self.grad_rgb.data_ptr(), self.g_sigma.data_ptr(),
                   self.g_sh.data_ptr(), self.slot.data_ptr(), s)
            L.call("po_sgd_step", tr.sigma.numel(), tr.sigma.data_ptr(), self.g_sigma.data_ptr(),
                   ctypes.c_float(self.lr_sigma), 1, s)
            L.call("po_sgd_step", tr.sh.numel(), tr.sh.data_ptr(), self.g_sh.data_ptr(),
                   ctypes.c_float(self.lr_sh), 1, s)
            loss = self.sq / (3 * n)
        self.steps += 1
        return loss

    def save(self, path) -> None:
        """Checkpoints the fit: the tree's values, the step count and the
        batch seed (written with Tree.save)."""
        import numpy as np

        self.tree.save(path, step=self.steps, seed=np.uint64(self.seed))

    def load(self, path) -> None:
        """Resumes from a file written by save: the leaf values are copied into
        this trainer's tree in place (its structure must match the file's), and
        the step count and the batch seed are restored."""
        import numpy as np
        import torch

        from .tree import read_checkpoint

        f, meta = read_checkpoint(path)
        tr = self.tree
        if (f["depth"] != tr.depth or f["sh_degree"] != tr.sh_degree or f["sigma"].dtype != np.float32
                or tuple(f["sh"].shape) != tuple(tr.sh.shape)
                or not np.array_equal(f["child"], tr.child.cpu().numpy())):
            raise ValueError("checkpoint tree does not match the trainer's tree")
        if "step" not in meta or "seed" not in meta:
            raise ValueError("checkpoint lacks the trainer state")
        tr.sigma.copy_(torch.from_numpy(f["sigma"]))
        tr.sh.copy_(torch.from_numpy(f["sh"]))
        self.steps = int(meta["step"])
        self.seed = int(np.asarray(meta["seed"]).astype(np.uint64))


def training_set(gt_tree, cams, bg=(1.0, 1.0, 1.0), stop_T=1e-4, device="cuda"):
    """Rays of all pixels of `cams` and their colours rendered from gt_tree:
    (origins, dirs, target), each (sum H*W, 3) float32 on `device`."""
    import torch

    from .render import camera_rays, render_rays

    os_, ds_, ts_ = [], [], []
    for cam in cams:
        o, d = camera_rays(cam, device=device)
        os_.append(o)
        ds_.append(d)
        ts_.append(render_rays(gt_tree, o, d, bg=bg, stop_T=stop_T))
    return torch.cat(os_), torch.cat(ds_), torch.cat(ts_)


def dataset_mse(tree, origins, dirs, target, bg=(1.0, 1.0, 1.0), stop_T=1e-4, chunk=1 << 20) -> float:
    """Mean squared error of the tree's renders over a whole ray set."""
    from .render import render_rays

    tot = 0.0
    for a in range(0, origins.shape[0], chunk):
        rgb = render_rays(tree, origins[a:a + chunk], dirs[a:a + chunk], bg=bg, stop_T=stop_T)
        tot += float(((rgb - target[a:a + chunk]) ** 2).sum())
    return tot / (3 * origins.shape[0])


def psnr(mse: float) -> float:
    import math

    return -10.0 * math.log10(max(mse, 1e-30))
