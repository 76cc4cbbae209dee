"""Pins of the oracle's two-dimensional method (oracle/twod.py).

The paper states that the method applies to 2-D problems (Sec. 1) without
details.  What fixes the results here is not the oracle's own formulas but the
mathematics of the plane: closed forms and harmonicity of the basis, quadrature
and the Laplacian of the uniform-rectangle potential, the Jacobi theta-function
closed form of the doubly periodic log potential, brute-force sums over growing
squares of images (extrapolated), the independence of the Ewald split from its
parameter, periodicity and translation invariance.
"""
import math

import numpy as np
import pytest

from oracle import _native
from oracle.twod import (EwaldLog2D, Plan2D, _rect_primitive, basis2d, basis_box_means2d, near_set2d,
                         rect_mean_potential, shell_sum2d, theta_sum)

BOX = np.array([1.0, 1.3])


def _cell(n=30, seed=1, box=BOX):
    g = np.random.default_rng(seed)
    x = (g.random((n, 2)) - 0.5) * box
    q = g.standard_normal(n)
    q -= q.mean()
    return x, q


def _worst(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _worst_upto_const(a, b):
    d = a - b
    return float(np.abs(d - d.mean()).max() / np.abs(b).max())


def test_basis_closed_forms_harmonicity_and_gradient():
    g = np.random.default_rng(2)
    x, y = g.uniform(-0.8, 0.8, 20), g.uniform(-0.8, 0.8, 20)
    R, G = basis2d(x, y, 9, grad=True)
    assert np.allclose(R[0], 1.0)
    assert np.allclose(R[1], x) and np.allclose(R[2], y)
    assert np.allclose(R[3], x * x - y * y) and np.allclose(R[4], 2 * x * y)
    assert np.allclose(R[5], x ** 3 - 3 * x * y * y) and np.allclose(R[6], 3 * x * x * y - y ** 3)
    h = 1e-3
    lap = (-basis2d(x + 2 * h, y, 9) + 16 * basis2d(x + h, y, 9) - 30 * R + 16 * basis2d(x - h, y, 9)
           - basis2d(x - 2 * h, y, 9) - basis2d(x, y + 2 * h, 9) + 16 * basis2d(x, y + h, 9) - 30 * R
           + 16 * basis2d(x, y - h, 9) - basis2d(x, y - 2 * h, 9)) / (12 * h * h)
    assert np.abs(lap).max() < 1e-7
    h = 1e-6
    gx = (basis2d(x + h, y, 9) - basis2d(x - h, y, 9)) / (2 * h)
    gy = (basis2d(x, y + h, 9) - basis2d(x, y - h, 9)) / (2 * h)
    assert np.abs(gx - G[0]).max() < 1e-8 and np.abs(gy - G[1]).max() < 1e-8


def test_rectangle_primitive_and_mean_potential():
    """d^2F/dudv = log(u^2 + v^2); Phi0 against 64 x 64 Gauss-Legendre quadrature
    outside the box, its Laplacian -2 pi / V inside and 0 outside, and the
    monopole far away."""
    g = np.random.default_rng(3)
    for u, v in g.uniform(-2, 2, (6, 2)):
        h = 1e-4
        fd = (_rect_primitive(u + h, v + h) - _rect_primitive(u - h, v + h) - _rect_primitive(u + h, v - h)
              + _rect_primitive(u - h, v - h)) / (4 * h * h)
        assert abs(fd - math.log(u * u + v * v)) < 1e-6
    gl, wl = np.polynomial.legendre.leggauss(64)
    X, Y = np.meshgrid(0.5 * BOX[0] * gl, 0.5 * BOX[1] * gl, indexing="ij")
    W = np.outer(wl, wl) / 4.0
    pts = np.array([[0.9, 0.1], [-0.2, 1.0], [1.1, -1.2], [-0.85, -0.3], [3.0, 2.0]])
    quad = np.array([np.sum(W * -0.5 * np.log((X - a) ** 2 + (Y - b) ** 2)) for a, b in pts])
    assert np.abs(rect_mean_potential(pts, BOX) - quad).max() < 1e-13
    h = 1e-3
    for pt, want in (([0.1, -0.2], -2 * math.pi / (BOX[0] * BOX[1])), ([0.9, 0.8], 0.0)):
        pt = np.array(pt)
        lap = 0.0
        for e in (np.array([h, 0.0]), np.array([0.0, h])):
            f = [rect_mean_potential(pt + s * e, BOX)[0] for s in (-2, -1, 0, 1, 2)]
            lap += (-f[0] + 16 * f[1] - 30 * f[2] + 16 * f[3] - f[4]) / (12 * h * h)
        assert abs(lap - want) < 1e-6
    far = np.array([[40.0, 30.0]])
    assert abs(rect_mean_potential(far, BOX)[0] + math.log(50.0)) < 1e-4


def test_box_means_of_the_basis():
    R0 = 0.5 * math.hypot(*BOX)
    m = basis_box_means2d(BOX, 9, R0)
    assert m[0] == pytest.approx(1.0, abs=1e-15)
    assert abs(m[3] - (BOX[0] ** 2 - BOX[1] ** 2) / 12 / R0 ** 2) < 1e-15
    odd = [1, 2, 5, 6, 9, 10, 13, 14]              # Re/Im w^n with n odd, and Im w^2
    assert np.abs(m[odd]).max() < 1e-15 and abs(m[4]) < 1e-15
    assert np.allclose(basis_box_means2d(BOX, 9, R0), basis_box_means2d(BOX, 15, R0)[:17], atol=1e-15)


def test_ewald_does_not_depend_on_alpha():
    x, q = _cell()
    a = EwaldLog2D(BOX, alpha=2.0).solve(x, q)
    for alpha in (3.0, 5.0):
        b = EwaldLog2D(BOX, alpha=alpha).solve(x, q)
        assert _worst(b[0], a[0]) < 1e-13 and _worst(b[1], a[1]) < 1e-13


@pytest.mark.parametrize("box", [(1.0, 1.3), (1.0, 1.0), (2.0, 0.7), (0.6, 1.5)])
def test_ewald_equals_the_theta_function_closed_form(box):
    box = np.array(box)
    x, q = _cell(25, seed=4, box=box)
    g = np.random.default_rng(5)
    y = np.concatenate([(g.random((15, 2)) - 0.5) * box, x[:3]])
    e = EwaldLog2D(box).solve(x, q, targets=y)
    t = theta_sum(x, q, box, targets=y)
    assert _worst_upto_const(t[0], e[0]) < 1e-13
    assert _worst(t[1], e[1]) < 1e-13


def test_ewald_equals_brute_force_squares_for_a_cell_without_dipole():
    """Squares of images |i|, |j| <= K = 32 .. 256, three Richardson steps; the
    square order shifts the potential by a constant (the cell's second moment),
    so potentials are compared up to a constant, fields exactly."""
    g = np.random.default_rng(6)
    xh = (g.random((10, 2)) - 0.5) * BOX * 0.9
    qh = g.standard_normal(10)
    qh -= qh.mean()
    x, q = np.concatenate([xh, -xh]), np.concatenate([qh, qh])
    assert np.abs(q @ x).max() < 1e-14
    e = EwaldLog2D(BOX).solve(x, q)
    b = shell_sum2d(x, q, BOX)
    assert _worst_upto_const(b[0], e[0]) < 1e-9 and _worst(b[1], e[1]) < 1e-9


def test_near_set_is_complete():
    x, q = _cell(200, seed=7)
    R_b = 1.5 * 0.5 * math.hypot(*BOX)
    xs, qs, base, img = near_set2d(x, q, BOX, R_b)
    for i in range(-4, 5):
        for j in range(-4, 5):
            p = np.array([i * BOX[0], j * BOX[1]])
            inside = set(np.nonzero(((x + p) ** 2).sum(1) <= R_b ** 2 * (1 - 1e-9))[0])
            sel = np.all(np.isclose(xs - x[base], p[None, :], rtol=0, atol=1e-12), axis=1)
            assert inside <= set(base[sel])
    assert len(set(zip(base, img))) == len(base)


def test_fit_has_only_the_constant_null_space():
    for box in ((1.0, 1.3), (2.0, 0.7), (1.0, 1.0)):
        for p in (8, 20, 40):
            pl = Plan2D(box, p, lam=1.5)
            assert pl.L == 4 * p and pl.rank == pl.P - 1 and pl.cond < 10


def test_method_matches_ewald_and_converges_geometrically():
    x, q = _cell(40, seed=8)
    e = EwaldLog2D(BOX).solve(x, q)
    errs = []
    for p in (12, 20, 30, 40):
        ph, f = Plan2D(BOX, p, lam=1.5).solve(x, q)
        errs.append(max(_worst(ph, e[0]), _worst(f, e[1])))
    assert errs[-1] < 2e-10
    assert all(a > 20 * b for a, b in zip(errs[:-1], errs[1:]))


@pytest.mark.parametrize("box", [(1.0, 1.0), (2.0, 0.7), (0.6, 1.5)])
def test_method_in_other_cells_and_with_a_strong_dipole(box):
    """p = 50: elongated cells converge more slowly (3e-9 at p = 40 for 2 x 0.7)."""
    box = np.array(box)
    x, q = _cell(30, seed=9, box=box)
    e = EwaldLog2D(box).solve(x, q)
    ph, f = Plan2D(box, 50, lam=1.5).solve(x, q)
    assert _worst(ph, e[0]) < 1e-10 and _worst(f, e[1]) < 1e-10
    # positive charges at +x, negative at -x
    g = np.random.default_rng(10)
    n = 20
    xd = (g.random((n, 2)) - 0.5) * box
    xd[: n // 2, 0] = 0.3 * box[0] + 0.15 * box[0] * g.random(n // 2)
    xd[n // 2:, 0] = -0.45 * box[0] + 0.15 * box[0] * g.random(n // 2)
    qd = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    e = EwaldLog2D(box).solve(xd, qd)
    ph, f = Plan2D(box, 50, lam=1.5).solve(xd, qd)
    assert _worst(ph, e[0]) < 1e-10 and _worst(f, e[1]) < 1e-10


def test_targets_on_particles_and_periodicity_and_translation():
    x, q = _cell(60, seed=11)
    pl = Plan2D(BOX, 50, lam=1.5)
    g = np.random.default_rng(12)
    y = np.concatenate([(g.random((30, 2)) - 0.5) * BOX, x[:10]])
    e = EwaldLog2D(BOX).solve(x, q, targets=y)
    ph, f = pl.solve(x, q, targets=y)
    assert _worst(ph, e[0]) < 1e-10 and _worst(f, e[1]) < 1e-10
    for k in range(2):
        a = y[:30].copy()
        a[:, k] = -0.5 * BOX[k]
        b = a.copy()
        b[:, k] = 0.5 * BOX[k]
        pa, fa = pl.solve(x, q, targets=a)
        pb, fb = pl.solve(x, q, targets=b)
        assert _worst(pb, pa) < 1e-10 and _worst(fb, fa) < 1e-10
    phi, f = pl.solve(x, q)
    s = np.array([0.37, -0.21])
    xs = (x + s + 0.5 * BOX) % BOX - 0.5 * BOX
    phi2, f2 = pl.solve(xs, q)
    assert _worst(phi2, phi) < 1e-10 and _worst(f2, f) < 5e-10


def test_direct_log_sum_against_numpy():
    g = np.random.default_rng(13)
    t, s, q = g.random((7, 2)), g.random((9, 2)), g.standard_normal(9)
    t[0] = s[0]
    ph, gr = _native.direct_log2d(t, s, q)
    d = t[:, None, :] - s[None, :, :]
    r2 = (d * d).sum(-1)
    live = r2 > 0
    want = np.where(live, -0.5 * np.log(np.where(live, r2, 1.0)), 0.0) @ q
    wg = -(np.where(live, 1.0 / np.where(live, r2, 1.0), 0.0)[:, :, None] * d * q[None, :, None]).sum(1)
    assert np.abs(ph - want).max() < 1e-14 and np.abs(gr - wg).max() < 1e-13


def _energy2d(pl, x, q):
    phi, _ = pl.solve(x, q)
    return 0.5 * float(q @ phi)


def test_plane_adjoint_matches_finite_differences():
    """The exact gradient of the plane method's energy against central
    differences (h = 1e-5) in positions and in neutral pairs of charges."""
    from oracle.twod import energy_gradients2d
    pl = Plan2D(BOX, 20, lam=1.5)
    x, q = _cell(40, seed=61)
    E, dEdx, dEdq = energy_gradients2d(pl, x, q)
    assert abs(E - _energy2d(pl, x, q)) < 1e-14 * abs(E)
    assert abs(dEdq.sum()) < 1e-12 * np.abs(dEdq).sum()
    P = np.array([[i * BOX[0], j * BOX[1]] for i in range(-3, 4) for j in range(-3, 4)])
    d = np.abs(np.linalg.norm(x[:, None, :] + P[None, :, :], axis=2) - pl.R_b).min(axis=1)
    h = 1e-5
    for i in np.nonzero(d > 1e-3)[0][:5]:
        for k in range(2):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (_energy2d(pl, xp, q) - _energy2d(pl, xm, q)) / (2 * h)
            assert abs(dEdx[i, k] - fd) < 1e-7 * max(1.0, abs(fd))
    for i, j in ((0, 1), (5, 33), (12, 39)):
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qp[j] -= h
        qm[i] -= h
        qm[j] += h
        fd = (_energy2d(pl, x, qp) - _energy2d(pl, x, qm)) / (2 * h)
        assert abs((dEdq[i] - dEdq[j]) - fd) < 1e-8 * max(1.0, abs(fd))
