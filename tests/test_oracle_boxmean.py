"""Pins for the box averages (App. B: R_t^(0); App. C: Phi0)."""
import numpy as np
import pytest

from oracle.basis import basis, index
from oracle.boxmean import basis_box_means, box_potential_mean
from oracle.geometry import circumradius


def _prism_potential(x, box):
    """Textbook closed form of int_box dV/|y - x| for a rectangular prism
    (MacMillan's potential of a homogeneous parallelepiped), written with the
    corner function F(a,b,c) = ab ln(c+r) + bc ln(a+r) + ca ln(b+r)
    - a^2/2 atan(bc/(ar)) - b^2/2 atan(ca/(br)) - c^2/2 atan(ab/(cr)) summed with
    alternating signs over the eight corners.  Independent of App. C's face/edge
    reduction.  Valid for points off the planes of the faces."""
    d = np.asarray(box, float)
    tot = np.zeros(x.shape[0])
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                a = sx * d[0] / 2 - x[:, 0]
                b = sy * d[1] / 2 - x[:, 1]
                c = sz * d[2] / 2 - x[:, 2]
                r = np.sqrt(a * a + b * b + c * c)
                F = (a * b * np.log(c + r) + b * c * np.log(a + r) + c * a * np.log(b + r)
                     - a * a / 2 * np.arctan(b * c / (a * r)) - b * b / 2 * np.arctan(c * a / (b * r))
                     - c * c / 2 * np.arctan(a * b / (c * r)))
                tot += sx * sy * sz * F
    return tot


def _quad_exterior(x, box, n=24):
    d = np.asarray(box, float)
    g, w = np.polynomial.legendre.leggauss(n)
    X, Y, Z = np.meshgrid(g * d[0] / 2, g * d[1] / 2, g * d[2] / 2, indexing="ij")
    Wt = (w[:, None, None] * w[None, :, None] * w[None, None, :]) / 8.0
    out = []
    for p in x:
        r = np.sqrt((X - p[0]) ** 2 + (Y - p[1]) ** 2 + (Z - p[2]) ** 2)
        out.append(np.sum(Wt / r))
    return np.array(out)


BOXES = [(1.0, 1.0, 1.0), (1.0, 1.0, 2.5), (1.7, 1.2, 1.4)]


@pytest.mark.parametrize("box", BOXES)
def test_phi0_matches_prism_formula(box):
    g = np.random.default_rng(2)
    d = np.asarray(box)
    x = (g.random((400, 3)) - 0.5) * d * 3.2        # inside and outside the box
    V = np.prod(d)
    np.testing.assert_allclose(box_potential_mean(x, box), _prism_potential(x, box) / V, rtol=2e-12, atol=1e-14)


@pytest.mark.parametrize("box", BOXES)
def test_phi0_matches_quadrature_outside(box):
    d = np.asarray(box)
    g = np.random.default_rng(3)
    v = g.normal(size=(20, 3))
    x = v / np.linalg.norm(v, axis=1)[:, None] * (circumradius(box) * (1.3 + g.random(20)))[:, None]
    np.testing.assert_allclose(box_potential_mean(x, box), _quad_exterior(x, box), rtol=1e-11)


@pytest.mark.parametrize("box", BOXES)
def test_phi0_poisson(box):
    """Laplacian of Phi0 is -4 pi / V0 inside the box and 0 outside."""
    d = np.asarray(box)
    V = np.prod(d)
    g = np.random.default_rng(4)
    inside = (g.random((10, 3)) - 0.5) * d * 0.8
    outside = (g.random((10, 3)) - 0.5) * d * 0.6 + d * np.array([1.2, 0, 0])
    h = 1e-3
    for pts, ref in ((inside, -4 * np.pi / V), (outside, 0.0)):
        lap = -6 * box_potential_mean(pts, box)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            lap += box_potential_mean(pts + e, box) + box_potential_mean(pts - e, box)
        lap /= h * h
        np.testing.assert_allclose(lap, ref, atol=2e-4 * 4 * np.pi / V)


def test_phi0_far_field():
    """Phi0 = 1/|x| + (1/24) sum_k d_k^2 (3 x_k^2 - |x|^2)/|x|^5 + O(|x|^-5)."""
    box = np.array([1.0, 1.3, 2.0])
    g = np.random.default_rng(5)
    v = g.normal(size=(10, 3))
    x = v / np.linalg.norm(v, axis=1)[:, None] * 60.0
    r = np.linalg.norm(x, axis=1)
    ref = 1 / r + sum(box[k] ** 2 * (3 * x[:, k] ** 2 - r ** 2) for k in range(3)) / (24 * r ** 5)
    np.testing.assert_allclose(box_potential_mean(x, box), ref, rtol=2e-8)  # next term ~ (d/|x|)^4 relative


def test_phi0_continuous_across_faces_and_on_edges():
    box = (1.0, 1.2, 0.8)
    y = np.array([[0.5, 0.1, 0.2], [0.5, 0.6, 0.4], [0.5, 0.6, -0.1], [-0.5, -0.6, 0.0]])
    for e in (1e-9, -1e-9):
        a = box_potential_mean(y + np.array([e, 0, 0]), box)
        b = box_potential_mean(y, box)
        assert np.all(np.isfinite(b))
        np.testing.assert_allclose(a, b, rtol=1e-7)


@pytest.mark.parametrize("box", BOXES)
def test_basis_box_means(box):
    d = np.asarray(box)
    p = 9
    R0 = circumradius(box)
    m = basis_box_means(box, p, R0)
    # odd degrees vanish by the box's symmetry
    for n in range(1, p, 2):
        for mm in range(-n, n + 1):
            assert abs(m[index(n, mm)]) < 1e-15
    # R^_2^0 = (2z^2 - x^2 - y^2)/2 and <x_k^2> = d_k^2/12
    ref = (2 * d[2] ** 2 - d[0] ** 2 - d[1] ** 2) / 24 / R0 ** 2
    assert abs(m[index(2, 0)] - ref) < 1e-15
    assert m[index(0, 0)] == pytest.approx(1.0, abs=1e-15)
    # exactness: more nodes change nothing
    g, w = np.polynomial.legendre.leggauss(12)
    X, Y, Z = np.meshgrid(g * d[0] / 2, g * d[1] / 2, g * d[2] / 2, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel() / 8
    ref = basis(X.ravel() / R0, Y.ravel() / R0, Z.ravel() / R0, p) @ W
    np.testing.assert_allclose(m, ref, atol=1e-14)
