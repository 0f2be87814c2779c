"""Comparison of GPU leaf gradients with the FP64 oracle gradient (App. B.3),
with the threshold-straddle reading of the early stop.

Early stopping (Sec. 4.2, "Rendering") ends a ray after the first data
sample that leaves T below stop_T.  Where that T lands within a relative
STRADDLE of stop_T, float32 and float64 may stop one sample apart, and both
results are correct renders.  Such rays are the ones whose oracle sample count
differs between stop_T (1 - STRADDLE) and stop_T (1 + STRADDLE); for them
either branch is accepted, every other ray must match the single oracle
result.  Gradients are summed over rays with float atomics in no fixed order,
so the bar is relative: per entry the distance to the nearest admissible
oracle value is at most GRAD_TOL * max |oracle|, and the cosine similarity is
at least GRAD_COS.
"""
from __future__ import annotations

import sys

import numpy as np

STRADDLE = 1e-5
GRAD_TOL = 1e-4
GRAD_COS = 0.99999


def grad_envelope(ot, o, d, g, bg, gamma):
    """Per-entry oracle bounds ((lo, hi) of dsigma, (lo, hi) of dsh, in the
    caller's cell order) of the summed gradient of rays (o, d) with upstream
    g = dL/dC, and the number of straddling rays."""
    o, d, g = (np.asarray(x, np.float64) for x in (o, d, g))
    if gamma <= 0.0:
        gs, gsh = ot.grad(o, d, g, bg=bg, gamma=0.0)
        return (gs, gs), (gsh, gsh), 0
    g_lo, g_hi = gamma * (1.0 - STRADDLE), gamma * (1.0 + STRADDLE)
    ns_lo = ot.render_rays(o, d, bg=bg, gamma=g_lo)[2]   # stops later: more samples
    ns_hi = ot.render_rays(o, d, bg=bg, gamma=g_hi)[2]
    strad = np.nonzero(ns_lo != ns_hi)[0]
    # two branches only: no two consecutive transmittances inside the band
    assert np.all(ns_lo[strad] - ns_hi[strad] == 1)
    keep = np.ones(len(o), bool)
    keep[strad] = False
    gs, gsh = ot.grad(o[keep], d[keep], g[keep], bg=bg, gamma=gamma)
    ls, hs, lh, hh = gs.copy(), gs.copy(), gsh.copy(), gsh.copy()
    for r in strad:
        a_s, a_h = ot.grad(o[r:r + 1], d[r:r + 1], g[r:r + 1], bg=bg, gamma=g_lo)
        b_s, b_h = ot.grad(o[r:r + 1], d[r:r + 1], g[r:r + 1], bg=bg, gamma=g_hi)
        ls += np.minimum(a_s, b_s)
        hs += np.maximum(a_s, b_s)
        lh += np.minimum(a_h, b_h)
        hh += np.maximum(a_h, b_h)
    return (ls, hs), (lh, hh), len(strad)


def check(got, lo, hi, what, slack=0.0):
    """got against the oracle bounds [lo, hi]; slack (scalar or per entry) is
    an extra absolute allowance, e.g. the float32 rounding of a parameter
    update."""
    got = np.asarray(got, np.float64)
    ref = np.clip(got, lo - slack, hi + slack)
    scale = max(np.abs(lo).max(), np.abs(hi).max())
    err = np.abs(got - ref).max() / scale
    cos = float((got * ref).sum() / (np.linalg.norm(got) * np.linalg.norm(ref)))
    print(f"[gpu] {what}: max |gpu - oracle| {err:.2e} of max|g| ({scale:.3e}), cosine {cos:.8f}",
          file=sys.stderr, flush=True)
    assert err <= GRAD_TOL, what
    assert cos >= GRAD_COS, what


def to_cells(tree, gs, gsh):
    """Leaf-order gradients of a tree -> caller cell order, (n,) and (n, 3, K)."""
    perm = tree.perm
    K = tree.K
    a = np.zeros(len(perm), np.float64)
    b = np.zeros((len(perm), 3 * K), np.float64)
    a[perm] = np.asarray(gs, np.float64)
    b[perm] = np.asarray(gsh, np.float64)[:, :3 * K]
    return a, b.reshape(-1, 3, K)
