"""Brute-force dense-grid renderer used to pin the oracle's traversal.

It knows nothing about octrees: the leaf cells are painted into a dense grid
at the finest level, every crossing of the ray with every grid plane is
listed and sorted, and each interval between consecutive crossings takes the
value of the voxel containing its midpoint.  The piecewise-constant
compositing of Sec. 3 (eqn:quad) with the background term of App. B.3 is then
applied to those intervals.  Colours use scipy's complex spherical harmonics
(Condon-Shortley phase included) and the real combination of App. B.1.
Tiny inputs only (depth <= 5).
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def real_sh_scipy(lmax: int, d) -> np.ndarray:
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    theta = np.arccos(np.clip(d[2], -1.0, 1.0))
    phi = np.arctan2(d[1], d[0])
    out = np.zeros((lmax + 1) ** 2)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m < 0:
                v = np.sqrt(2.0) * (-1) ** m * y.imag
            elif m == 0:
                v = y.real
            else:
                v = np.sqrt(2.0) * (-1) ** m * y.real
            out[l * l + l + m] = v
    return out


def densify(depth, cells) -> np.ndarray:
    n = 1 << depth
    grid = -np.ones((n, n, n), np.int64)
    for idx, (lv, i, j, k) in enumerate(np.asarray(cells)):
        s = 1 << (depth - lv)
        grid[i * s:(i + 1) * s, j * s:(j + 1) * s, k * s:(k + 1) * s] = idx
    return grid


def render_ray(grid, center, half, lmax, sigma, sh, o, d, bg):
    n = grid.shape[0]
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    lo = np.asarray(center, np.float64) - half
    h = 2.0 * half / n
    # box interval
    t0, t1 = 0.0, np.inf
    for k in range(3):
        if d[k] == 0.0:
            if not (lo[k] <= o[k] < lo[k] + 2 * half):
                return np.asarray(bg, np.float64).copy(), 1.0
            continue
        a = (lo[k] - o[k]) / d[k]
        b = (lo[k] + 2 * half - o[k]) / d[k]
        t0 = max(t0, min(a, b))
        t1 = min(t1, max(a, b))
    if not t1 > t0:
        return np.asarray(bg, np.float64).copy(), 1.0
    ts = [t0, t1]
    for k in range(3):
        if d[k] == 0.0:
            continue
        planes = lo[k] + h * np.arange(n + 1)
        tk = (planes - o[k]) / d[k]
        ts.extend(tk[(tk > t0) & (tk < t1)].tolist())
    ts = np.unique(np.asarray(ts))
    Y = real_sh_scipy(lmax, d)
    C = np.zeros(3)
    T = 1.0
    for ta, tb in zip(ts[:-1], ts[1:]):
        if not tb > ta:
            continue
        mid = o + 0.5 * (ta + tb) * d
        idx = np.floor((mid - lo) / h).astype(np.int64)
        idx = np.clip(idx, 0, n - 1)
        leaf = grid[idx[0], idx[1], idx[2]]
        if leaf < 0:
            continue
        sig = max(float(sigma[leaf]), 0.0)
        tau = sig * (tb - ta)
        c = 1.0 / (1.0 + np.exp(-(np.asarray(sh[leaf], np.float64) @ Y)))
        C += T * (-np.expm1(-tau)) * c
        T *= np.exp(-tau)
    return C + T * np.asarray(bg, np.float64), T


def render_rays(depth, center, half, lmax, cells, sigma, sh, o, d, bg=(1.0, 1.0, 1.0)):
    grid = densify(depth, cells)
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    rgb = np.zeros((len(o), 3))
    T = np.zeros(len(o))
    for r in range(len(o)):
        rgb[r], T[r] = render_ray(grid, center, half, lmax, sigma, sh, o[r], d[r], bg)
    return rgb, T
