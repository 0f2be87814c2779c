"""Pins for the gradient comparison used by the GPU tests (tests/gradcheck.py):
the threshold-straddle envelope accepts exactly the two oracle branches of a
ray whose transmittance lands on stop_T, and rejects a wrong stop rule or a
perturbed entry.  CPU only: every 'GPU result' here is an oracle gradient."""
import numpy as np
import pytest

import gradcheck
from paper_2103_14024_amd import scenes


def _setup(oracle_mod):
    s = scenes.scene_small()
    ot = oracle_mod.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"], s["sigma"], s["sh"])
    o, d = scenes.random_rays(400, 5, spread=1.0)
    o, d = o.astype(np.float64), d.astype(np.float64)
    g = np.random.default_rng(3).standard_normal((len(o), 3))
    return ot, o, d, g


def test_envelope_is_exact_without_early_stop(oracle_mod):
    ot, o, d, g = _setup(oracle_mod)
    (ls, hs), (lh, hh), n = gradcheck.grad_envelope(ot, o, d, g, (1.0, 1.0, 1.0), 0.0)
    assert n == 0 and np.array_equal(ls, hs) and np.array_equal(lh, hh)
    gradcheck.check(ls, ls, hs, "exact")


def test_straddling_ray_accepts_both_branches_only(oracle_mod):
    ot, o, d, g = _setup(oracle_mod)
    bg = (0.9, 0.4, 0.1)
    # T after the first sample of every ray (stop_T = 1 stops there), and the
    # number of samples without early stop
    _, T1, _, _ = ot.render_rays(o, d, bg=bg, gamma=1.0)
    _, _, ns, _ = ot.render_rays(o, d, bg=bg, gamma=0.0)
    r0 = int(np.nonzero((ns >= 3) & (T1 > 0.2) & (T1 < 0.9))[0][0])
    gamma = float(T1[r0])     # ray r0 lands exactly on stop_T after its first sample
    (ls, hs), (lh, hh), n = gradcheck.grad_envelope(ot, o, d, g, bg, gamma)
    assert n >= 1
    eps = gradcheck.STRADDLE
    a_s, a_h = ot.grad(o, d, g, bg=bg, gamma=gamma * (1.0 + eps))   # r0 stops after its first sample
    b_s, b_h = ot.grad(o, d, g, bg=bg, gamma=gamma * (1.0 - eps))   # r0 goes on
    scale = max(np.abs(ls).max(), np.abs(hs).max())
    assert np.abs(a_s - b_s).max() > 1e-2 * scale     # the branches differ well beyond the bar
    for x_s, x_h in ((a_s, a_h), (b_s, b_h)):
        gradcheck.check(x_s, ls, hs, "branch dsigma")
        gradcheck.check(x_h, lh, hh, "branch dsh")
    # no early stop at all: rejected
    c_s, c_h = ot.grad(o, d, g, bg=bg, gamma=0.0)
    with pytest.raises(AssertionError):
        gradcheck.check(c_s, ls, hs, "no stop dsigma")
    # one entry off by three times the bar: rejected
    bad = a_s.copy()
    k = int(np.argmax(np.abs(a_s)))
    bad[k] += 3 * gradcheck.GRAD_TOL * scale * np.sign(a_s[k])
    with pytest.raises(AssertionError):
        gradcheck.check(bad, ls, hs, "perturbed dsigma")
    # within the bar: accepted
    ok = a_s.copy()
    ok[k] += 0.5 * gradcheck.GRAD_TOL * scale
    gradcheck.check(ok, ls, hs, "within the bar")


def test_slack_is_an_absolute_allowance(oracle_mod):
    ot, o, d, g = _setup(oracle_mod)
    gs, _ = ot.grad(o, d, g, gamma=0.0)
    scale = np.abs(gs).max()
    bad = gs + 5 * gradcheck.GRAD_TOL * scale
    with pytest.raises(AssertionError):
        gradcheck.check(bad, gs, gs, "shifted")
    gradcheck.check(bad, gs, gs, "shifted with slack", slack=np.full_like(gs, 5 * gradcheck.GRAD_TOL * scale))
