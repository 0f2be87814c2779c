"""Pins for the oracle's real spherical harmonics (App. B.1).

The oracle builds the real basis from the complex definition with a general
associated-Legendre recurrence.  These tests pin it against things that do not
share that route: quadrature orthonormality, scipy's complex SH, textbook
closed-form polynomials and the values at the pole.
"""
import math

import numpy as np
import pytest

from dense_bruteforce import real_sh_scipy


def _grid(n_theta=10, n_phi=20):
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).reshape(-1)
    return dirs, wts


@pytest.mark.parametrize("lmax", [2, 3, 4])
def test_orthonormal_by_quadrature(oracle_mod, lmax):
    # Gauss-Legendre in cos(theta) x uniform phi integrates the degree-2*lmax
    # products exactly, so the Gram matrix must be the identity.
    dirs, w = _grid()
    Y = oracle_mod.sh_basis(lmax, dirs)
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


def test_against_scipy_complex_sh(oracle_mod):
    rng = np.random.default_rng(5)
    dirs = rng.standard_normal((200, 3))
    Y = oracle_mod.sh_basis(4, dirs)
    for i in range(len(dirs)):
        assert np.abs(Y[i] - real_sh_scipy(4, dirs[i])).max() < 1e-13


def _closed_form(d):
    x, y, z = d / np.linalg.norm(d)
    pi = math.pi
    return np.array([
        0.5 / math.sqrt(pi),
        math.sqrt(3 / (4 * pi)) * y, math.sqrt(3 / (4 * pi)) * z, math.sqrt(3 / (4 * pi)) * x,
        0.5 * math.sqrt(15 / pi) * x * y,
        0.5 * math.sqrt(15 / pi) * y * z,
        0.25 * math.sqrt(5 / pi) * (3 * z * z - 1),
        0.5 * math.sqrt(15 / pi) * x * z,
        0.25 * math.sqrt(15 / pi) * (x * x - y * y),
        0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y),
        0.5 * math.sqrt(105 / pi) * x * y * z,
        0.25 * math.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1),
        0.25 * math.sqrt(7 / pi) * (5 * z ** 3 - 3 * z),
        0.25 * math.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1),
        0.25 * math.sqrt(105 / pi) * z * (x * x - y * y),
        0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),
    ])


def test_closed_form_polynomials(oracle_mod):
    # Textbook real SH polynomials up to degree 3 in the Condon-Shortley
    # convention whose sign cancels the (-1)^m of the real combination.
    rng = np.random.default_rng(7)
    dirs = rng.standard_normal((100, 3))
    Y = oracle_mod.sh_basis(3, dirs)
    for i in range(len(dirs)):
        assert np.abs(Y[i] - _closed_form(dirs[i])).max() < 1e-13


def test_pole_values(oracle_mod):
    Y = oracle_mod.sh_basis(4, [[0.0, 0.0, 1.0]])[0]
    for l in range(5):
        for m in range(-l, l + 1):
            want = math.sqrt((2 * l + 1) / (4 * math.pi)) if m == 0 else 0.0
            assert abs(Y[l * l + l + m] - want) < 1e-14


def test_degree_one_is_scaled_direction(oracle_mod):
    d = np.array([0.3, -0.5, 0.812403840463596])
    Y = oracle_mod.sh_basis(1, [d])[0]
    c = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[1:4], c * np.array([d[1], d[2], d[0]]) / np.linalg.norm(d), atol=1e-15)
    # basis does not depend on the length of the direction
    assert np.allclose(oracle_mod.sh_basis(3, [7.5 * d]), oracle_mod.sh_basis(3, [d]), atol=1e-15)
