"""Pins for the oracle's solid-harmonic basis (Sec. 3.1, eqs. (1.1)-(1.9))."""
import math

import numpy as np
import pytest
from scipy.special import lpmv, eval_legendre

from oracle.basis import basis, index


def _points(n, seed, scale=0.9):
    g = np.random.default_rng(seed)
    v = g.normal(size=(n, 3))
    v *= (scale * g.random(n) ** (1 / 3) / np.linalg.norm(v, axis=1))[:, None]
    return v


def _from_legendre(x, y, z, p):
    """Assemble R^_n^m from eq. (1.1)-(1.2) with the renormalized alpha of
    Sec. 3.1, alpha = (-1)^n sqrt(4 pi/(2n+1)), and Y_n^m = N_n^m P_n^|m| e^{i m phi},
    N_n^m = (-1)^m sqrt((2n+1)/(4pi) (n-|m|)!/(n+|m|)!): real part for m >= 0,
    imaginary part for m < 0 (eq. (1.4)).  P_n^m carries the Condon-Shortley
    phase of eq. (1.3), as scipy's lpmv does."""
    r = np.sqrt(x * x + y * y + z * z)
    mu = np.where(r > 0, z / np.where(r > 0, r, 1), 1.0)
    ph = np.arctan2(y, x)
    out = np.zeros((p * p, x.size))
    for n in range(p):
        for m in range(-n, n + 1):
            am = abs(m)
            c = (-1) ** (n + m) * math.sqrt(math.factorial(n - am) / math.factorial(n + am))
            v = c * r ** n * lpmv(am, n, mu) * np.exp(1j * m * ph)
            out[index(n, m)] = v.real if m >= 0 else v.imag
    return out


def test_low_order_closed_forms():
    x, y, z = _points(50, 1).T
    R = basis(x, y, z, 3)
    s2 = math.sqrt(2.0)
    np.testing.assert_allclose(R[index(0, 0)], 1.0)
    np.testing.assert_allclose(R[index(1, 0)], -z, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(R[index(1, 1)], -x / s2, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(R[index(1, -1)], y / s2, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(R[index(2, 0)], (2 * z * z - x * x - y * y) / 2, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("p", [6, 14])
def test_matches_associated_legendre_assembly(p):
    x, y, z = _points(300, p).T
    R = basis(x, y, z, p)
    ref = _from_legendre(x, y, z, p)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.max(np.abs(R - ref) / scale) < 1e-12


def test_index_stacking():
    seen = sorted(index(n, m) for n in range(7) for m in range(-n, n + 1))
    assert seen == list(range(49))
    assert index(0, 0) == 0 and index(1, -1) == 1 and index(1, 1) == 3   # t = (n+1)^2 - (n-m) minus one


def test_addition_identity():
    """sum_m (R^_n^m)^2 = r^{2n} (1 + P_n(cos theta)^2)/2 (Legendre addition theorem)."""
    x, y, z = _points(200, 7).T
    p = 12
    R = basis(x, y, z, p)
    r = np.sqrt(x * x + y * y + z * z)
    for n in range(p):
        s = sum(R[index(n, m)] ** 2 for m in range(-n, n + 1))
        ref = r ** (2 * n) * (1 + eval_legendre(n, z / r) ** 2) / 2
        np.testing.assert_allclose(s, ref, rtol=1e-12, atol=1e-300)


def test_gradient_matches_central_differences():
    x, y, z = _points(40, 3).T
    p = 10
    _, G = basis(x, y, z, p, grad=True)
    h = 1e-6
    for k in range(3):
        dp = [x, y, z]
        dm = [x, y, z]
        dp = [a + (h if i == k else 0) for i, a in enumerate(dp)]
        dm = [a - (h if i == k else 0) for i, a in enumerate(dm)]
        fd = (basis(*dp, p) - basis(*dm, p)) / (2 * h)
        scale = np.abs(fd).max() + 1e-30
        assert np.max(np.abs(G[k] - fd)) / scale < 1e-8


def test_harmonic():
    """Every R^_n^m solves Laplace's equation: div grad R^ = 0 (checked by central
    differences of the exact gradient)."""
    x, y, z = _points(40, 4).T
    p = 10
    h = 1e-5
    lap = 0
    for k in range(3):
        dp = [a + (h if i == k else 0) for i, a in enumerate((x, y, z))]
        dm = [a - (h if i == k else 0) for i, a in enumerate((x, y, z))]
        lap = lap + (basis(*dp, p, grad=True)[1][k] - basis(*dm, p, grad=True)[1][k]) / (2 * h)
    R = basis(x, y, z, p)
    assert np.max(np.abs(lap)) < 1e-7 * max(1.0, np.abs(R).max())


def test_gradient_lowers_degree():
    """grad R^_n^m is a homogeneous polynomial of degree n-1 (eq. (1.9) expands the
    far-field gradient over the same basis): doubling the point scales it by 2^(n-1)."""
    x, y, z = _points(20, 5).T
    p = 9
    _, G1 = basis(x, y, z, p, grad=True)
    _, G2 = basis(2 * x, 2 * y, 2 * z, p, grad=True)
    for n in range(1, p):
        for m in range(-n, n + 1):
            t = index(n, m)
            np.testing.assert_allclose(G2[:, t], 2.0 ** (n - 1) * G1[:, t], rtol=1e-12, atol=1e-14)
