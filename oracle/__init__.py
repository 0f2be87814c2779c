"""FP64 CPU oracle for PlenOctree rendering -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product library never does, and this package imports
nothing from it: both sides receive the same seeded inputs from the scene
generators and nothing else.

The arithmetic lives in ``oracle.c`` (plain C, double precision, optional
OpenMP over rays).  This module only compiles it with gcc and marshals NumPy
arrays through ctypes.  See ``oracle.c`` for the passages of the paper each
function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.environ.get("PO_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compiles oracle.c into liboracle.so with gcc (-O2, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=False)
    L = ctypes.CDLL(_SO)
    L.orc_tree_new.restype = ctypes.c_void_p
    L.orc_tree_new.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int64,
                               _i32p, _dp, _dp, ctypes.c_char_p, ctypes.c_int]
    L.orc_tree_free.argtypes = [ctypes.c_void_p]
    L.orc_tree_n_nodes.restype = ctypes.c_int64
    L.orc_tree_n_nodes.argtypes = [ctypes.c_void_p]
    L.orc_sh_basis.argtypes = [ctypes.c_int, _dp, _dp]
    L.orc_sg_basis.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    L.orc_tree_set_sg.restype = ctypes.c_int
    L.orc_tree_set_sg.argtypes = [ctypes.c_void_p, _dp]
    L.orc_ray_segments.restype = ctypes.c_int64
    L.orc_ray_segments.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int64, _dp, _dp, _i64p]
    L.orc_render_rays.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double,
                                  _dp, _dp, _i64p, _dp]
    L.orc_render_rays_view.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double,
                                       ctypes.c_uint32, _dp, _dp, _dp, _i64p, _dp]
    L.orc_leaf_weights.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp]
    L.orc_half_bits.restype = ctypes.c_uint16
    L.orc_half_bits.argtypes = [ctypes.c_double]
    L.orc_median_cut.restype = ctypes.c_int64
    L.orc_median_cut.argtypes = [ctypes.c_int64, _dp, ctypes.c_int64, _i64p, ctypes.POINTER(ctypes.c_uint16)]
    L.orc_camera_rays.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, _dp, _dp]
    L.orc_render_camera.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp,
                                    ctypes.c_double, _dp, _dp, _i64p]
    L.orc_grad.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double, _dp,
                           _dp, _dp]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib = L
    return L


def _d(a):
    """Contiguous float64 copy (exact promotion from float32 / float16)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))


def sh_basis(lmax: int, dirs) -> np.ndarray:
    """Real SH values, (n, (lmax+1)^2), at the (normalised) directions dirs (n, 3)."""
    L = _load()
    d = _d(dirs).reshape(-1, 3)
    K = (lmax + 1) ** 2
    out = np.zeros((d.shape[0], K), np.float64)
    for i in range(d.shape[0]):
        L.orc_sh_basis(lmax, _p(d[i]), _p(out[i]))
    return out


def sg_basis(lobes, dirs) -> np.ndarray:
    """Spherical-Gaussian values (n, K) at directions (n, 3) for lobes (K, 4) = (axis, bandwidth)."""
    L = _load()
    lb = _d(lobes).reshape(-1, 4)
    dirs = _d(dirs).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], lb.shape[0]), np.float64)
    for i in range(dirs.shape[0]):
        L.orc_sg_basis(lb.shape[0], _p(lb), _p(dirs[i]), _p(out[i]))
    return out


def half_bits(x: float) -> int:
    """IEEE binary16 bits of x (round to nearest even)."""
    return int(_load().orc_half_bits(float(x)))


def median_cut(points, M: int):
    """Median cut of points (n, 3) into at most M boxes: returns (idx (n,)
    int64 box of each point, codebook (nb, 3) float16, nb)."""
    L = _load()
    pts = _d(points).reshape(-1, 3)
    n = pts.shape[0]
    idx = np.zeros(n, np.int64)
    cb = np.zeros((max(M, 1), 3), np.uint16)
    nb = L.orc_median_cut(n, _p(pts), int(M), _p(idx, _i64p), cb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)))
    if nb < 0:
        raise MemoryError("oracle median cut")
    return idx, cb[:nb].view(np.float16), int(nb)


def codebook(sh, M: int):
    """Codebook compression of leaf coefficients sh (n, 3, K): for each basis
    function k the RGB triples (sh[:, :, k]) are median-cut into at most M
    colours.  Returns (idx (n, K) int64, codebooks: list of K (nb_k, 3)
    float16 arrays)."""
    sh = np.asarray(sh)
    n, _, K = sh.shape
    idx = np.zeros((n, K), np.int64)
    books = []
    for k in range(K):
        i_k, cb_k, _ = median_cut(sh[:, :, k], M)
        idx[:, k] = i_k
        books.append(cb_k)
    return idx, books


def codebook_decode(idx, books):
    """Leaf coefficients (n, 3, K) float64 of a codebook tree."""
    n, K = idx.shape
    out = np.zeros((n, 3, K), np.float64)
    for k in range(K):
        out[:, :, k] = books[k].astype(np.float64)[idx[:, k]]
    return out


def camera_rays(c2w, W, H, fx, fy, cx, cy):
    """Pixel-centre pinhole rays (origins, directions), each (H*W, 3) float64."""
    L = _load()
    c = _d(c2w).reshape(12)
    o = np.zeros((W * H, 3), np.float64)
    d = np.zeros((W * H, 3), np.float64)
    L.orc_camera_rays(_p(c), int(W), int(H), float(fx), float(fy), float(cx), float(cy), _p(o), _p(d))
    return o, d


class OracleTree:
    """The oracle's own octree, built from a list of leaf cells.

    cells: (n, 4) int (level, i, j, k); sigma: (n,) raw densities;
    sh: (n, 3, K) coefficients, K = (lmax+1)^2, channel-major.
    lobes: None for the SH basis, or (K, 4) spherical-Gaussian lobes (axis,
    bandwidth) that replace it.  Values are promoted exactly to float64.
    """

    def __init__(self, depth, lmax, center, half, cells, sigma, sh, lobes=None):
        L = _load()
        self.depth, self.lmax = int(depth), int(lmax)
        self.K = (self.lmax + 1) ** 2
        cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 4))
        n = cells.shape[0]
        sig = _d(sigma).reshape(n)
        shv = _d(sh).reshape(n, 3, self.K)
        ctr = _d(center).reshape(3)
        err = ctypes.create_string_buffer(256)
        h = L.orc_tree_new(self.depth, self.lmax, _p(ctr), float(half), n, _p(cells, _i32p),
                           _p(sig), _p(shv), err, 256)
        if not h:
            raise ValueError("oracle tree: " + err.value.decode())
        self._h = ctypes.c_void_p(h)
        self.n_leaves = n
        if lobes is not None:
            lb = _d(lobes).reshape(self.K, 4)
            if L.orc_tree_set_sg(self._h, _p(lb)) != 0:
                raise ValueError("oracle tree: SG lobe axes must be non-zero")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_tree_free(h)
            self._h = None

    @property
    def n_nodes(self) -> int:
        return _load().orc_tree_n_nodes(self._h)

    def render_rays(self, o, d, bg=(1.0, 1.0, 1.0), gamma=0.0):
        """Returns (rgb (n,3), T (n,), n_samples (n,), max clamped sigma met (n,))."""
        L = _load()
        o = _d(o).reshape(-1, 3)
        d = _d(d).reshape(-1, 3)
        n = o.shape[0]
        rgb = np.zeros((n, 3), np.float64)
        T = np.zeros(n, np.float64)
        ns = np.zeros(n, np.int64)
        sm = np.zeros(n, np.float64)
        L.orc_render_rays(self._h, n, _p(o), _p(d), _p(_d(bg)), float(gamma), _p(rgb), _p(T),
                          _p(ns, _i64p), _p(sm))
        return rgb, T, ns, sm

    def render_view(self, o, d, bg=(1.0, 1.0, 1.0), gamma=0.0, sh_off=0, clip=None):
        """Viewer render: returns (rgb (n,3), T (n,), n_samples (n,), depth (n,)).

        sh_off: bit k drops basis function k; clip: (nx, ny, nz, w), keep n.x + w >= 0."""
        L = _load()
        o = _d(o).reshape(-1, 3)
        d = _d(d).reshape(-1, 3)
        n = o.shape[0]
        rgb = np.zeros((n, 3), np.float64)
        T = np.zeros(n, np.float64)
        ns = np.zeros(n, np.int64)
        dep = np.zeros(n, np.float64)
        cp = None if clip is None else _p(_d(clip).reshape(4))
        L.orc_render_rays_view(self._h, n, _p(o), _p(d), _p(_d(bg)), float(gamma), int(sh_off) & 0xffffffff,
                               cp, _p(rgb), _p(T), _p(ns, _i64p), _p(dep))
        return rgb, T, ns, dep

    def render_camera(self, c2w, W, H, fx, fy, cx, cy, bg=(1.0, 1.0, 1.0), gamma=0.0):
        """Returns (rgb (H,W,3), T (H,W), n_samples (H,W))."""
        L = _load()
        rgb = np.zeros((H, W, 3), np.float64)
        T = np.zeros((H, W), np.float64)
        ns = np.zeros((H, W), np.int64)
        L.orc_render_camera(self._h, _p(_d(c2w).reshape(12)), int(W), int(H), float(fx), float(fy),
                            float(cx), float(cy), _p(_d(bg)), float(gamma), _p(rgb), _p(T),
                            _p(ns, _i64p))
        return rgb, T, ns

    def grad(self, o, d, g, bg=(1.0, 1.0, 1.0), gamma=0.0):
        """dL/dsigma_raw (n_leaves,) and dL/dsh (n_leaves, 3, K) for upstream g = dL/dC (n, 3)."""
        L = _load()
        o = _d(o).reshape(-1, 3)
        d = _d(d).reshape(-1, 3)
        g = _d(g).reshape(-1, 3)
        gs = np.zeros(self.n_leaves, np.float64)
        gsh = np.zeros((self.n_leaves, 3, self.K), np.float64)
        L.orc_grad(self._h, o.shape[0], _p(o), _p(d), _p(_d(bg)), float(gamma), _p(g), _p(gs), _p(gsh))
        return gs, gsh

    def leaf_weights(self, o, d, gamma=0.0, mode=0, weight=None):
        """Largest ray weight per leaf (n_leaves,) over the rays (o, d): mode 0
        1 - exp(-sigma delta), mode 1 T (1 - exp(-sigma delta)); weight, if
        given, is raised in place (float64) and returned."""
        L = _load()
        o = _d(o).reshape(-1, 3)
        d = _d(d).reshape(-1, 3)
        w = np.zeros(self.n_leaves, np.float64) if weight is None else weight
        assert w.dtype == np.float64 and w.shape == (self.n_leaves,) and w.flags.c_contiguous
        L.orc_leaf_weights(self._h, o.shape[0], _p(o), _p(d), float(gamma), int(mode), _p(w))
        return w

    def segments(self, o, d, cap=1 << 16):
        """Segments of one ray: (a (m,), b (m,), leaf (m,)); leaf -1 is empty space."""
        L = _load()
        a = np.zeros(cap, np.float64)
        b = np.zeros(cap, np.float64)
        lf = np.zeros(cap, np.int64)
        m = L.orc_ray_segments(self._h, _p(_d(o).reshape(3)), _p(_d(d).reshape(3)), cap, _p(a), _p(b),
                               _p(lf, _i64p))
        m = min(m, cap)
        return a[:m], b[:m], lf[:m]
