"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *draws inputs*: leaf cells of a sparse octree, raw leaf
values, camera poses and intrinsics, and free rays.  It holds none of the
rendering arithmetic (no traversal, SH, sigmoid or compositing), so the GPU
path and the CPU oracle can both consume what it produces without sharing code.

Shapes follow the paper's evaluation setup: 800x800 views from cameras on the
upper hemisphere looking at a central object (Sec. 5.1, "Datasets"), a 512^3
finest grid and degree-3 SH (Sec. 5.2), leaves holding a density plus per-
channel SH coefficients (Sec. 4.2).  The paper's datasets are not available;
these scenes stand in for them.

Cells are (level, i, j, k) int32 rows: a cube of edge 2*half / 2^level whose
integer coordinates at that level are (i, j, k), inside the box
[center - half, center + half]^3.
"""
from __future__ import annotations

import math

import numpy as np

BOX_CENTER = (0.0, 0.0, 0.0)
BOX_HALF = 1.0


# --------------------------------------------------------------------------
# leaf values
# --------------------------------------------------------------------------

def n_coef(sh_degree: int) -> int:
    return (sh_degree + 1) ** 2


def leaf_values(n: int, sh_degree: int, seed: int, mu: float = 2.0, s: float = 1.0,
                sh_std: float = 0.5):
    """Raw densities ~ lognormal(mu, s) and SH coefficients ~ N(0, sh_std^2).

    Returns sigma (n,) float32 and sh (n, 3, K) float32 (channel-major).
    """
    rng = np.random.default_rng(seed)
    sigma = rng.lognormal(mean=mu, sigma=s, size=n).astype(np.float32)
    sh = (rng.standard_normal((n, 3, n_coef(sh_degree)), dtype=np.float32) * np.float32(sh_std))
    return sigma, sh


def sg_lobes(K: int, seed: int, lam_range=(2.0, 12.0)) -> np.ndarray:
    """K spherical-Gaussian lobes (K, 4) float32: unit axes drawn uniformly
    on the sphere, bandwidths uniform in lam_range."""
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((K, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    lam = rng.uniform(lam_range[0], lam_range[1], (K, 1))
    return np.concatenate([p, lam], 1).astype(np.float32)


def perturb(sigma, sh, std: float, seed: int):
    """Adds N(0, std^2) noise to a copy of sigma and sh (float32)."""
    rng = np.random.default_rng(seed)
    s2 = (np.asarray(sigma, np.float32) + rng.standard_normal(np.shape(sigma), dtype=np.float32) * np.float32(std))
    h2 = (np.asarray(sh, np.float32) + rng.standard_normal(np.shape(sh), dtype=np.float32) * np.float32(std))
    return s2.astype(np.float32), h2.astype(np.float32)


# --------------------------------------------------------------------------
# geometry: which finest-level voxels are leaves
# --------------------------------------------------------------------------

def _centers_1d(depth: int, half: float = BOX_HALF, c: float = 0.0):
    n = 1 << depth
    h = 2.0 * half / n
    return (c - half) + (np.arange(n, dtype=np.float64) + 0.5) * h, h


def spheres_cells(depth: int = 5, n_spheres: int = 3, seed: int = 0,
                  r_range=(0.2, 0.4), c_range: float = 0.6) -> np.ndarray:
    """Voxels at the finest level whose centre is within one voxel edge of the
    surface of a union of seeded spheres: |min_i(|x - mu_i| - r_i)| <= h."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-c_range, c_range, size=(n_spheres, 3))
    r = rng.uniform(r_range[0], r_range[1], size=n_spheres)
    xs, h = _centers_1d(depth)
    X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
    P = np.stack([X, Y, Z], -1)
    sdf = np.full(X.shape, np.inf)
    for i in range(n_spheres):
        sdf = np.minimum(sdf, np.linalg.norm(P - mu[i], axis=-1) - r[i])
    ii, jj, kk = np.nonzero(np.abs(sdf) <= h)
    return _cells(depth, ii, jj, kk)


# Frozen parameters of the depth-9 "sum of 20 Gaussian blobs" surface band.
BLOB_PARAMS = dict(n_blobs=20, c_range=0.62, s_range=(0.13, 0.24), a_range=(0.7, 1.3), iso=0.3)
# Half-width of the surface band in finest-voxel edges.  Twenty separate blobs
# inside the box cannot carry ~3M one-voxel band leaves at 512^3 (that needs a
# surface area near the box's own); a band of two voxel edges each side does.
BLOB_BAND = 2.0


def blob_field_params(seed: int, n_blobs=20, c_range=0.62, s_range=(0.13, 0.24),
                      a_range=(0.7, 1.3), iso=0.3):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-c_range, c_range, size=(n_blobs, 3))
    s = rng.uniform(s_range[0], s_range[1], size=n_blobs)
    a = rng.uniform(a_range[0], a_range[1], size=n_blobs)
    return mu, s, a, iso


def _blob_factors(coords, mu, s, a):
    """1-D factors of the separable blobs on a coordinate axis: value factors
    g[b, axis, i] (the amplitude folded into the x factor) and derivative
    multipliers q[b, axis, i] = -(x_i - mu_b)/s_b^2.  float64."""
    nb = len(a)
    g = np.empty((nb, 3, len(coords)))
    q = np.empty_like(g)
    for ax in range(3):
        diff = coords[None, :] - mu[:, ax][:, None]
        g[:, ax] = np.exp(-diff ** 2 / (2 * s[:, None] ** 2))
        q[:, ax] = -diff / s[:, None] ** 2
    g[:, 0] *= a[:, None]
    return g, q


def _field_blocks(gx, gy, gz, qx, qy, qz):
    """Field and gradient on blocks.  Inputs (nblk, nb, m) per axis; returns
    f, fx, fy, fz of shape (nblk, m_z, m_y * m_x)."""
    yx = gy[:, :, :, None] * gx[:, :, None, :]
    nblk, nb, my, mx = yx.shape
    yx = yx.reshape(nblk, nb, my * mx)
    yxq = (gy[:, :, :, None] * (gx * qx)[:, :, None, :]).reshape(nblk, nb, my * mx)
    yqx = ((gy * qy)[:, :, :, None] * gx[:, :, None, :]).reshape(nblk, nb, my * mx)
    gzt = np.transpose(gz, (0, 2, 1))
    f = gzt @ yx
    fx = gzt @ yxq
    fy = gzt @ yqx
    fz = np.transpose(gz * qz, (0, 2, 1)) @ yx
    return f, fx, fy, fz


def blobs_cells(depth: int = 9, seed: int = 0, band: float = BLOB_BAND, block_log2: int = 3,
                **kw) -> np.ndarray:
    """Voxels of the finest level lying in the band |f(x_c) - iso| / |grad f(x_c)| <= band * h
    around the iso-surface of f(x) = sum_i a_i exp(-|x - mu_i|^2 / (2 s_i^2)).

    Evaluated coarse to fine: the field is first evaluated at the centres of
    blocks of (2^block_log2)^3 voxels, blocks whose centre lies within a wide
    margin of the surface (band + 2 block diagonals, in the same distance
    estimate) are kept, and only their voxels are then evaluated exactly.
    The Gaussians are separable, so each block is a sum over blobs of outer
    products of 1-D factors (float64).
    """
    p = dict(BLOB_PARAMS)
    p.update(kw)
    mu, s, a, iso = blob_field_params(seed, **p)
    n = 1 << depth
    B = 1 << min(block_log2, depth)
    nbk = n // B
    xs, h = _centers_1d(depth)
    xc, hc = _centers_1d(depth - min(block_log2, depth))
    # coarse pass over block centres
    g, q = _blob_factors(xc, mu, s, a)
    cand = []
    for z0 in range(0, nbk, 16):
        z1 = min(nbk, z0 + 16)
        gx = g[None, :, 0, :]
        gy = g[None, :, 1, :]
        gz = g[None, :, 2, z0:z1]
        f, fx, fy, fz = _field_blocks(gx, gy, gz, q[None, :, 0, :], q[None, :, 1, :], q[None, :, 2, z0:z1])
        gn = np.sqrt(fx * fx + fy * fy + fz * fz)[0]
        ok = np.abs(f[0] - iso) <= (band * h + 2.0 * math.sqrt(3.0) * hc) * gn
        kz, yxi = np.nonzero(ok)
        cand.append(np.stack([yxi % nbk, yxi // nbk, kz + z0], -1))
    cand = np.concatenate(cand, 0) if cand else np.zeros((0, 3), np.int64)
    # fine pass over candidate blocks
    g, q = _blob_factors(xs, mu, s, a)
    off = np.arange(B)
    out = []
    for c0 in range(0, len(cand), 4096):
        cb = cand[c0:c0 + 4096]
        ix = cb[:, 0:1] * B + off[None]
        iy = cb[:, 1:2] * B + off[None]
        iz = cb[:, 2:3] * B + off[None]
        gx = np.transpose(g[:, 0, :][:, ix], (1, 0, 2))
        gy = np.transpose(g[:, 1, :][:, iy], (1, 0, 2))
        gz = np.transpose(g[:, 2, :][:, iz], (1, 0, 2))
        qx = np.transpose(q[:, 0, :][:, ix], (1, 0, 2))
        qy = np.transpose(q[:, 1, :][:, iy], (1, 0, 2))
        qz = np.transpose(q[:, 2, :][:, iz], (1, 0, 2))
        f, fx, fy, fz = _field_blocks(gx, gy, gz, qx, qy, qz)
        gn = np.sqrt(fx * fx + fy * fy + fz * fz)
        ok = np.abs(f - iso) <= (band * h) * gn
        bi, kz, yxi = np.nonzero(ok)
        out.append(np.stack([cb[bi, 0] * B + yxi % B, cb[bi, 1] * B + yxi // B, cb[bi, 2] * B + kz], -1))
    ijk = np.concatenate(out, 0) if out else np.zeros((0, 3), np.int64)
    return _cells(depth, ijk[:, 0], ijk[:, 1], ijk[:, 2])


def _cells(depth, i, j, k) -> np.ndarray:
    n = len(i)
    c = np.empty((n, 4), np.int32)
    c[:, 0] = depth
    c[:, 1] = i
    c[:, 2] = j
    c[:, 3] = k
    return c


def subdivide(cells: np.ndarray, sigma, sh, which) -> tuple:
    """Replaces each cell listed in `which` by its 8 children carrying the
    same values (a test input whose render must not change)."""
    which = np.asarray(which)
    keep = np.ones(len(cells), bool)
    keep[which] = False
    kids, ks, kh = [], [], []
    for w in which:
        lv, i, j, k = cells[w]
        for c in range(8):
            kids.append((lv + 1, 2 * i + (c >> 2 & 1), 2 * j + (c >> 1 & 1), 2 * k + (c & 1)))
            ks.append(sigma[w])
            kh.append(sh[w])
    nc = np.concatenate([cells[keep], np.asarray(kids, np.int32).reshape(-1, 4)], 0)
    ns = np.concatenate([np.asarray(sigma)[keep], np.asarray(ks, np.asarray(sigma).dtype)], 0)
    nh = np.concatenate([np.asarray(sh)[keep], np.asarray(kh, np.asarray(sh).dtype).reshape(-1, *np.shape(sh)[1:])], 0)
    return nc.astype(np.int32), ns, nh


def random_tree_cells(max_depth: int, seed: int, p_split: float = 0.6, p_leaf: float = 0.6) -> np.ndarray:
    """A random sparse tree with leaves at mixed levels (1..max_depth)."""
    rng = np.random.default_rng(seed)
    out = []

    def rec(level, i, j, k):
        for c in range(8):
            ci, cj, ck = 2 * i + (c >> 2 & 1), 2 * j + (c >> 1 & 1), 2 * k + (c & 1)
            if level + 1 < max_depth and rng.random() < p_split:
                rec(level + 1, ci, cj, ck)
            elif rng.random() < p_leaf:
                out.append((level + 1, ci, cj, ck))

    rec(0, 0, 0, 0)
    return np.asarray(out, np.int32).reshape(-1, 4)


# --------------------------------------------------------------------------
# cameras and rays
# --------------------------------------------------------------------------

def intrinsics(W: int, H: int, fov_x_deg: float = 40.0):
    """Pinhole focal lengths and principal point: fx = fy = (W/2) / tan(fov_x/2)."""
    f = 0.5 * W / math.tan(math.radians(fov_x_deg) * 0.5)
    return f, f, 0.5 * W, 0.5 * H


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Row-major 3x4 camera-to-world matrix of a camera at `eye` looking at
    `target` (columns: right, up, backward, position; the camera looks down -z)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    u = np.asarray(up, np.float64)
    if np.linalg.norm(np.cross(f, u)) < 1e-6:
        u = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, u)
    r /= np.linalg.norm(r)
    cu = np.cross(r, f)
    m = np.zeros((3, 4), np.float64)
    m[:, 0], m[:, 1], m[:, 2], m[:, 3] = r, cu, -f, eye
    return m.astype(np.float32)


def hemisphere_poses(n: int, radius: float = 4.0, seed: int = 2) -> np.ndarray:
    """n poses with eyes area-uniform on the upper hemisphere (z ~ U(0,1),
    phi ~ U(0, 2 pi)) of the given radius, looking at the origin.  (n, 3, 4) float32."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.0, 1.0, n)
    phi = rng.uniform(0.0, 2 * math.pi, n)
    rr = np.sqrt(np.maximum(0.0, 1 - z * z))
    eyes = radius * np.stack([rr * np.cos(phi), rr * np.sin(phi), z], -1)
    return np.stack([look_at(e) for e in eyes], 0)


def random_rays(n: int, seed: int, radius: float = 3.0, spread: float = 1.2):
    """Free rays: origins on a sphere of the given radius, aimed at points drawn
    uniformly in [-spread, spread]^3 (so some rays miss the box).
    Directions are not normalised.  float32 (n, 3) each."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    o = radius * v / np.linalg.norm(v, axis=1, keepdims=True)
    tgt = rng.uniform(-spread, spread, (n, 3))
    d = tgt - o
    d *= rng.uniform(0.5, 2.0, (n, 1))
    return o.astype(np.float32), d.astype(np.float32)


def inside_rays(n: int, seed: int, half: float = 0.9):
    """Rays that start inside the box, random unit-ish directions."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-half, half, (n, 3))
    d = rng.standard_normal((n, 3))
    return o.astype(np.float32), d.astype(np.float32)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def scene_small(seed: int = 0, data_seed: int = 1, depth: int = 5, sh_degree: int = 2):
    """Plain render, FP32 parity case: depth 5 (32^3), 3 spheres, SH degree 2."""
    cells = spheres_cells(depth, 3, seed)
    sigma, sh = leaf_values(len(cells), sh_degree, data_seed)
    return dict(depth=depth, sh_degree=sh_degree, center=BOX_CENTER, half=BOX_HALF,
                cells=cells, sigma=sigma, sh=sh)


def scene_blobs(depth: int = 9, sh_degree: int = 3, seed: int = 0, data_seed: int = 1):
    """Surface band of a sum of 20 seeded Gaussian blobs; ~3M leaves at depth 9."""
    cells = blobs_cells(depth, seed)
    sigma, sh = leaf_values(len(cells), sh_degree, data_seed)
    return dict(depth=depth, sh_degree=sh_degree, center=BOX_CENTER, half=BOX_HALF,
                cells=cells, sigma=sigma, sh=sh)


def scene_train(depth: int = 8, sh_degree: int = 2, seed: int = 1, data_seed: int = 3):
    """Ground-truth tree of the differentiation workload: the blob band at
    depth 8 (~0.64M leaves) with its own seeds, SH degree 2."""
    return scene_blobs(depth, sh_degree, seed, data_seed)


# (depth, SH degree, geometry seed) of the four resident scenes of the serving workload
SERVE_SCENES = [(8, 2, 11), (9, 3, 0), (9, 2, 12), (10, 3, 13)]


def serve_scenes(data_seed: int = 21):
    """The four resident scenes of the serving workload (0.6M to 9.5M leaves)."""
    return [scene_blobs(d, l, s, data_seed + i) for i, (d, l, s) in enumerate(SERVE_SCENES)]


def small_pose(seed: int = 2, radius: float = 4.0) -> np.ndarray:
    """One camera on the upper hemisphere of the radius-4 sphere."""
    return hemisphere_poses(1, radius, seed)[0]
