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


def validate_host(depth, sh_degree, child, n_leaves, sigma=None, dtype=L.PO_F32, center=(0, 0, 0), half=1.0,
                  sh_stride=0) -> None:
    """Checks a host child array (and optional densities); raises PlenOctreeError."""
    child = np.ascontiguousarray(np.asarray(child, np.int32).reshape(-1, 8))
    desc = make_desc(depth, sh_degree, center, half, dtype, sh_stride)
    sp = None
    if sigma is not None:
        sigma = np.ascontiguousarray(np.asarray(sigma, np.float16 if dtype == L.PO_F16 else np.float32))
        sp = sigma.ctypes.data
    L.call("po_tree_validate", ctypes.byref(desc), child.shape[0], child.ctypes.data, int(n_leaves), sp)


CHECKPOINT_VERSION = 1
_CKPT_LEAF_DTYPES = {"sigma": (np.float32, np.float16), "sh": (np.float32, np.float16, np.int16)}


def write_checkpoint(path, fields: dict, meta: dict | None = None) -> None:
    """Writes a tree as an uncompressed .npz of plain arrays (nothing pickled).

    fields: depth, sh_degree, center (3,), half, child (n_nodes, 8) int32,
    sigma (n,) float32/float16, sh (n, stride) float32/float16 (int16 codebook
    positions), and optionally perm (n,) int64, lobes (K, 4) float32,
    codebook (K, M, 4) float16.  meta: extra numeric scalars or arrays (a step
    count, a seed, a generator state), stored under "meta_<name>"."""
    arrays = {"version": np.int32(CHECKPOINT_VERSION),
              "depth": np.int32(fields["depth"]), "sh_degree": np.int32(fields["sh_degree"]),
              "center": np.asarray(fields["center"], np.float64).reshape(3), "half": np.float64(fields["half"]),
              "child": np.ascontiguousarray(fields["child"])}
    for k in ("sigma", "sh", "perm", "lobes", "codebook"):
        if fields.get(k) is not None:
            arrays[k] = np.ascontiguousarray(fields[k])
    for k, v in (meta or {}).items():
        a = np.asarray(v)
        if a.dtype.kind not in "biuf":
            raise TypeError(f"checkpoint meta {k!r} must be numeric")
        arrays["meta_" + k] = a
    with open(path, "wb") as f:
        np.savez(f, **arrays)


def read_checkpoint(path):
    """Reads a file written by write_checkpoint with NumPy's non-pickling
    loader and checks its structure (shapes, dtypes and the child array, with
    the library's validator) before anything reaches a device.

    Returns (fields, meta) as host arrays; raises ValueError or
    PlenOctreeError on a malformed file."""
    with np.load(path, allow_pickle=False) as z:
        a = {k: z[k] for k in z.files}
    for k in ("version", "depth", "sh_degree", "center", "half", "child", "sigma", "sh"):
        if k not in a:
            raise ValueError(f"checkpoint lacks {k!r}")
    if int(a["version"]) != CHECKPOINT_VERSION:
        raise ValueError(f"checkpoint version {int(a['version'])}, expected {CHECKPOINT_VERSION}")
    depth, deg = int(a["depth"]), int(a["sh_degree"])
    child, sigma, sh = a["child"], a["sigma"], a["sh"]
    for k, ok in _CKPT_LEAF_DTYPES.items():
        if a[k].dtype not in [np.dtype(t) for t in ok]:
            raise ValueError(f"checkpoint {k} has dtype {a[k].dtype}")
    if child.dtype != np.int32 or child.ndim != 2 or child.shape[1] != 8:
        raise ValueError("checkpoint child must be (n_nodes, 8) int32")
    n, K = sigma.shape[0], n_coef(deg)
    codebook = a.get("codebook")
    if sigma.ndim != 1 or sh.ndim != 2 or sh.shape[0] != n or sh.shape[1] < (K if codebook is not None else 3 * K):
        raise ValueError("checkpoint sigma/sh shapes do not match the leaf count and SH degree")
    if codebook is None and sh.dtype != sigma.dtype:
        raise ValueError("checkpoint sigma and sh must share a dtype")
    if "perm" in a and (a["perm"].dtype != np.int64 or a["perm"].shape != (n,)):
        raise ValueError("checkpoint perm must be (n_leaves,) int64")
    if "lobes" in a and (a["lobes"].dtype != np.float32 or a["lobes"].shape != (K, 4)):
        raise ValueError(f"checkpoint lobes must be ({K}, 4) float32")
    if codebook is not None and (codebook.dtype != np.float16 or codebook.ndim != 3 or codebook.shape[0] != K
                                 or codebook.shape[2] != 4 or sh.dtype != np.int16 or sigma.dtype != np.float16):
        raise ValueError("checkpoint codebook trees take float16 sigma, int16 records and a (K, M, 4) float16 codebook")
    center, half = tuple(float(c) for c in a["center"]), float(a["half"])
    if codebook is None:
        validate_host(depth, deg, child, n, sigma, L.PO_F16 if sigma.dtype == np.float16 else L.PO_F32, center, half,
                      sh.shape[1])
    else:
        # records of 16-bit codebook positions: the structure is checked alone
        validate_host(depth, deg, child, n, None, L.PO_F32, center, half)
        if not np.isfinite(sigma).all():
            raise ValueError("checkpoint densities must be finite")
    fields = {"depth": depth, "sh_degree": deg, "center": center, "half": half, "child": child, "sigma": sigma, "sh": sh,
              "perm": a.get("perm"), "lobes": a.get("lobes"), "codebook": codebook}
    meta = {k[5:]: v for k, v in a.items() if k.startswith("meta_")}
    return fields, meta


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

    def save(self, path, **meta) -> None:
        """Writes the tree (structure, leaf values, leaf order, basis lobes or
        codebook) to an .npz file; meta: extra numeric values to store."""
        t = lambda x: None if x is None else x.detach().cpu().numpy()  # noqa: E731
        write_checkpoint(path, {"depth": self.depth, "sh_degree": self.sh_degree, "center": self.center,
                                "half": self.half, "child": t(self.child), "sigma": t(self.sigma), "sh": t(self.sh),
                                "perm": self.perm, "lobes": t(self.lobes), "codebook": t(self.codebook)}, meta)

    @classmethod
    def load(cls, path, device="cuda", index=True):
        """Reads a file written by save (checked on the host first) and binds
        it on `device`.  Returns (tree, meta)."""
        import torch

        f, meta = read_checkpoint(path)
        dev = torch.device(device)
        up = lambda x: None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
        tree = cls(f["depth"], f["sh_degree"], up(f["child"]), up(f["sigma"]), up(f["sh"]), f["center"], f["half"],
                   perm=f["perm"], lobes=up(f["lobes"]), codebook=up(f["codebook"]), index=index)
        return tree, meta

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
