"""PlenOctree construction (host, C ABI builder) and device residency."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L


def n_coef(sh_degree: int) -> int:
    return (sh_degree + 1) ** 2


def default_stride(sh_degree: int) -> int:
    """SH record stride in elements: 3K rounded up to a multiple of 4, so
    float32 records are 16-byte and float16 records 8-byte multiples."""
    return (3 * n_coef(sh_degree) + 3) // 4 * 4


def codebook_stride(sh_degree: int) -> int:
    """Index record stride of codebook trees: K rounded up to a multiple of 4."""
    return (n_coef(sh_degree) + 3) // 4 * 4


def codebook_build(sh, M: int = 65536, index_stride=None):
    """Median-cut codebooks of leaf coefficients sh (n, 3, K) (po_codebook_build).

    Returns (codebook (K, M, 4) uint16 float16 bits, index (n, stride) uint16,
    boxes (K,) int32 colours used per basis function)."""
    sh = np.ascontiguousarray(np.asarray(sh, np.float32))
    n, three, K = sh.shape
    if three != 3:
        raise ValueError("sh must be (n, 3, K)")
    stride = (K + 3) // 4 * 4 if index_stride is None else int(index_stride)
    cb = np.zeros((K, int(M), 4), np.uint16)
    idx = np.zeros((n, stride), np.uint16)
    boxes = np.zeros(K, np.int32)
    L.call("po_codebook_build", n, K, sh.ctypes.data if n else None, 3 * K, int(M), cb.ctypes.data,
           idx.ctypes.data if n else None, stride, boxes.ctypes.data)
    return cb, idx, boxes


def make_desc(depth, sh_degree, center=(0.0, 0.0, 0.0), half=1.0, dtype=L.PO_F32, sh_stride=0) -> L.po_tree_desc:
    d = L.po_tree_desc()
    d.depth = int(depth)
    d.sh_degree = int(sh_degree)
    for k in range(3):
        d.center[k] = float(center[k])
    d.half_size = float(half)
    d.dtype = int(dtype)
    d.sh_stride = int(sh_stride)
    return d


def _dtype_code(dtype) -> int:
    if dtype in ("f32", "float32", L.PO_F32):
        return L.PO_F32
    if dtype in ("f16", "float16", L.PO_F16):
        return L.PO_F16
    raise ValueError(f"unknown leaf dtype {dtype!r}")


def build_host(depth, sh_degree, cells, center=(0.0, 0.0, 0.0), half=1.0):
    """Runs the library's octree builder on a (n, 4) int32 cell list.

    Returns (child (n_nodes, 8) int32, perm (n,) int64): leaf j of the tree is
    cell perm[j] of the input."""
    cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 4))
    desc = make_desc(depth, sh_degree, center, half)
    b = ctypes.c_void_p()
    L.call("po_builder_create", ctypes.byref(desc), cells.shape[0], cells.ctypes.data, ctypes.byref(b))
    try:
        nn, nl = ctypes.c_int64(), ctypes.c_int64()
        L.call("po_builder_sizes", b, ctypes.byref(nn), ctypes.byref(nl))
        child = np.empty((nn.value, 8), np.int32)
        perm = np.empty(nl.value, np.int64)
        L.call("po_builder_emit", b, child.ctypes.data, perm.ctypes.data if nl.value else None)
    finally:
        L.lib().po_builder_destroy(b)
    return child, perm


def validate_host(depth, sh_degree, child, n_leaves, sigma=None, dtype=L.PO_F32, center=(0, 0, 0), half=1.0) -> None:
    """Checks a host child array (and optional densities); raises PlenOctreeError."""
    child = np.ascontiguousarray(np.asarray(child, np.int32).reshape(-1, 8))
    desc = make_desc(depth, sh_degree, center, half, dtype)
    sp = None
    if sigma is not None:
        sigma = np.ascontiguousarray(np.asarray(sigma, np.float16 if dtype == L.PO_F16 else np.float32))
        sp = sigma.ctypes.data
    L.call("po_tree_validate", ctypes.byref(desc), child.shape[0], child.ctypes.data, int(n_leaves), sp)


class Tree:
    """A PlenOctree resident in HBM: the child array, the raw densities and
    the SH records (float32 or float16) as torch tensors, bound to a library
    handle.  The handle borrows the tensors; this object keeps them alive."""

    def __init__(self, depth, sh_degree, child, sigma, sh, center=(0.0, 0.0, 0.0), half=1.0, perm=None,
                 lobes=None, codebook=None, index=True):
        import torch

        self.depth, self.sh_degree = int(depth), int(sh_degree)
        self.K = n_coef(sh_degree)
        self.center, self.half = tuple(float(c) for c in center), float(half)
        if sigma.dtype == torch.float32:
            self.dtype = L.PO_F32
        elif sigma.dtype == torch.float16:
            self.dtype = L.PO_F16
        else:
            raise TypeError("sigma must be float32 or float16")
        if codebook is not None:
            # codebook tree: sh holds the 16-bit positions (int16 storage), codebook (K, M, 4) float16
            if sigma.dtype != torch.float16 or sh.dtype != torch.int16:
                raise TypeError("codebook trees take float16 sigma and int16 (16-bit position) records")
        elif sh.dtype != sigma.dtype:
            raise TypeError("sigma and sh must share a dtype")
        if child.dtype != torch.int32 or child.dim() != 2 or child.shape[1] != 8:
            raise TypeError("child must be an int32 (n_nodes, 8) tensor")
        for t in (child, sigma, sh):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("tree arrays must be contiguous device tensors")
        self.n_leaves = int(sigma.shape[0])
        rec_min = self.K if codebook is not None else 3 * self.K
        if sh.dim() != 2 or sh.shape[0] != self.n_leaves or sh.shape[1] < rec_min:
            raise ValueError(f"sh must be (n_leaves, stride >= {rec_min})")
        self.stride = int(sh.shape[1])
        self.child, self.sigma, self.sh = child, sigma, sh
        self.perm = perm
        self.lobes = lobes
        self.codebook = codebook
        self.desc = make_desc(depth, sh_degree, center, half, self.dtype, self.stride)
        h = ctypes.c_void_p()
        leaf_ptrs = (sigma.data_ptr() if self.n_leaves else None, sh.data_ptr() if self.n_leaves else None)
        if codebook is not None:
            if not (codebook.is_cuda and codebook.dtype == torch.float16 and codebook.dim() == 3
                    and codebook.shape[0] == self.K and codebook.shape[2] == 4 and codebook.is_contiguous()):
                raise ValueError(f"codebook must be a contiguous float16 ({self.K}, M, 4) device tensor")
            L.call("po_tree_bind_codebook", ctypes.byref(self.desc), int(child.shape[0]), child.data_ptr(),
                   self.n_leaves, *leaf_ptrs, codebook.data_ptr(), int(codebook.shape[1]), ctypes.byref(h))
        elif lobes is None:
            L.call("po_tree_bind", ctypes.byref(self.desc), int(child.shape[0]), child.data_ptr(), self.n_leaves,
                   *leaf_ptrs, ctypes.byref(h))
        else:
            # spherical-Gaussian colour basis: (K, 4) float32 device lobes (axis, bandwidth)
            if not (lobes.is_cuda and lobes.dtype == torch.float32 and tuple(lobes.shape) == (self.K, 4)
                    and lobes.is_contiguous()):
                raise ValueError(f"lobes must be a contiguous float32 ({self.K}, 4) device tensor")
            L.call("po_tree_bind_sg", ctypes.byref(self.desc), int(child.shape[0]), child.data_ptr(),
                   self.n_leaves, *leaf_ptrs, lobes.data_ptr(), ctypes.byref(h))
        self._h = h
        # the traversal index (8x8x8 bricks below level depth - 3; trees of
        # depth < 4 have none): renders walk it instead of `child`
        self.indexed = bool(index) and self.depth >= 4
        if self.indexed:
            L.call("po_tree_build_index", h, ctypes.c_void_p(torch.cuda.current_stream(child.device).cuda_stream))

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def n_nodes(self) -> int:
        return int(self.child.shape[0])

    def nbytes(self) -> int:
        arrays = [self.child, self.sigma, self.sh] + [t for t in (self.lobes, self.codebook) if t is not None]
        return sum(int(t.numel() * t.element_size()) for t in arrays)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and L._lib is not None:
            L._lib.po_tree_destroy(h)
            self._h = None

    @classmethod
    def from_cells(cls, depth, sh_degree, cells, sigma, sh, center=(0.0, 0.0, 0.0), half=1.0, dtype="f32",
                   device="cuda", stride=None, lobes=None, index=True):
        """Builds the tree on the host from leaf cells (level, i, j, k) with
        values in the caller's order, reorders the values into leaf order and
        uploads everything to `device`.  lobes: None (SH colour basis) or
        (K, 4) spherical-Gaussian lobes (axis, bandwidth)."""
        import torch

        code = _dtype_code(dtype)
        cells = np.asarray(cells, np.int32).reshape(-1, 4)
        n = cells.shape[0]
        K = n_coef(sh_degree)
        child, perm = build_host(depth, sh_degree, cells, center, half)
        stride = default_stride(sh_degree) if stride is None else int(stride)
        sig = np.asarray(sigma, np.float32).reshape(n)[perm]
        rec = np.zeros((n, stride), np.float32)
        rec[:, :3 * K] = np.asarray(sh, np.float32).reshape(n, 3 * K)[perm]
        if code == L.PO_F16:
            if np.abs(sig).max(initial=0) > 65504 or np.abs(rec).max(initial=0) > 65504:
                raise ValueError("leaf values exceed the float16 range")
            sig = sig.astype(np.float16)
            rec = rec.astype(np.float16)
        dev = torch.device(device)
        t_child = torch.from_numpy(child).to(dev)
        t_sig = torch.from_numpy(np.ascontiguousarray(sig)).to(dev)
        t_sh = torch.from_numpy(rec).to(dev)
        t_lobes = None
        if lobes is not None:
            t_lobes = torch.from_numpy(np.ascontiguousarray(np.asarray(lobes, np.float32).reshape(K, 4))).to(dev)
        return cls(depth, sh_degree, t_child, t_sig, t_sh, center, half, perm=perm, lobes=t_lobes, index=index)

    @classmethod
    def from_scene(cls, scene: dict, dtype="f32", device="cuda", stride=None, index=True):
        return cls.from_cells(scene["depth"], scene["sh_degree"], scene["cells"], scene["sigma"], scene["sh"],
                              scene["center"], scene["half"], dtype=dtype, device=device, stride=stride,
                              lobes=scene.get("lobes"), index=index)

    @classmethod
    def from_cells_codebook(cls, depth, sh_degree, cells, sigma, sh, M=65536, center=(0.0, 0.0, 0.0), half=1.0,
                            device="cuda", index_stride=None, index=True):
        """Codebook tree (App. B.2): the coefficients are median-cut per basis
        function in the caller's cell order (po_codebook_build), the densities
        kept as float16; records hold 16-bit codebook positions."""
        import torch

        cells = np.asarray(cells, np.int32).reshape(-1, 4)
        n = cells.shape[0]
        K = n_coef(sh_degree)
        child, perm = build_host(depth, sh_degree, cells, center, half)
        sig = np.asarray(sigma, np.float32).reshape(n)
        if np.abs(sig).max(initial=0) > 65504:
            raise ValueError("densities exceed the float16 range")
        cb, idx, _ = codebook_build(np.asarray(sh, np.float32).reshape(n, 3, K), M, index_stride)
        dev = torch.device(device)
        t_child = torch.from_numpy(child).to(dev)
        t_sig = torch.from_numpy(np.ascontiguousarray(sig[perm].astype(np.float16))).to(dev)
        t_idx = torch.from_numpy(np.ascontiguousarray(idx[perm]).view(np.int16)).to(dev)
        t_cb = torch.from_numpy(cb.view(np.float16)).to(dev)
        return cls(depth, sh_degree, t_child, t_sig, t_idx, center, half, perm=perm, codebook=t_cb, index=index)

    def leaf_values(self):
        """(sigma (n,), sh (n, 3, K)) as float32 NumPy arrays in the caller's cell
        order (codebook trees: the decoded coefficients)."""
        sig = self.sigma.float().cpu().numpy()
        if self.codebook is not None:
            pos = self.sh[:, :self.K].cpu().numpy().view(np.uint16).astype(np.int64)
            cb = self.codebook.float().cpu().numpy()
            sh = np.stack([cb[k][pos[:, k], :3] for k in range(self.K)], axis=2)
        else:
            sh = self.sh[:, :3 * self.K].float().cpu().numpy().reshape(-1, 3, self.K)
        if self.perm is None:
            return sig, sh
        inv = np.empty_like(self.perm)
        inv[self.perm] = np.arange(len(self.perm))
        return sig[inv], sh[inv]
