"""Pins of the oracle's two-axis periodization (oracle/slab.py) and of its
independent reference, the slab Ewald sum (oracle/ewald2d.py).

The paper only states that the periodic extension may be done along one or two
coordinates (Sec. 1, closing paragraph).  What fixes the result here is not the
oracle's own formulas but: brute-force lattice sums over growing square shells
of in-plane images (extrapolated), the splitting parameter's irrelevance in the
Ewald sum, Gauss's law for the slab, the decay of the exact potential's in-plane
Fourier modes away from the charges, periodicity in x and y, and translation
invariance.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.ewald2d import Ewald2D
from oracle.slab import SlabPlan, decay_modes, plane_points, slab_near_set

BOX = np.array([1.0, 1.2, 0.8])


def _cell(n=6, seed=3, box=BOX):
    g = np.random.default_rng(seed)
    x = (g.random((n, 3)) - 0.5) * box
    q = g.standard_normal(n)
    q -= q.mean()
    return x, q


def _worst(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_ewald2d_does_not_depend_on_the_splitting_parameter():
    x, q = _cell(12, seed=1)
    ref = Ewald2D(BOX, alpha=3.0).solve(x, q)
    for a in (4.5, 7.0):
        phi, f = Ewald2D(BOX, alpha=a).solve(x, q)
        assert _worst(phi, ref[0]) < 1e-13 and _worst(f, ref[1]) < 1e-13


def _shell_sum(x, q, K, box=BOX):
    """Direct sum over the images |i1|, |i2| <= K (a square shell, symmetric under
    p -> -p), the self pair skipped: potential and field at the particles."""
    i1, i2 = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    P = np.stack([i1.ravel() * box[0], i2.ravel() * box[1], np.zeros(i1.size)], 1)
    phi = np.zeros(len(x))
    grad = np.zeros((len(x), 3))
    for j in range(len(x)):
        D = x[:, None, :] - (x[j][None, None, :] + P[None, :, :])
        r = np.sqrt((D * D).sum(2))
        ok = r > 0
        rs = np.where(ok, r, 1.0)
        phi += q[j] * np.where(ok, 1 / rs, 0).sum(1)
        grad += q[j] * (np.where(ok, -1 / rs ** 3, 0)[:, :, None] * D).sum(1)
    return phi, -grad


def test_ewald2d_equals_the_brute_force_lattice_sum():
    """Square shells K = 32, 64, 128, 256; the truncation error of a symmetric shell
    expands in powers of 1/K, removed by three Richardson steps.  Potentials are
    compared as differences (the lattice sum's constant is not the Ewald one)."""
    x, q = _cell()
    pe, fe = Ewald2D(BOX).solve(x, q)
    Ks = (32, 64, 128, 256)
    for k in (0, 1):
        lv = [_shell_sum(x, q, K)[k] for K in Ks]
        for order in (1, 2, 3):   # eliminate the 1/K, 1/K^2, 1/K^3 terms in turn
            f2 = 2.0 ** order
            lv = [(f2 * b - a) / (f2 - 1) for a, b in zip(lv[:-1], lv[1:])]
        if k == 0:
            ph = lv[0]
            assert _worst(ph - ph[0], pe - pe[0]) < 2e-8
        else:
            assert _worst(lv[0], fe) < 2e-8


def test_ewald2d_satisfies_gauss_law_for_the_slab():
    """The planar mean of E_z is -4 pi Q_above(z0) / A at any height z0 (and 0
    above and below the neutral slab): the trapezoid rule over the periodic cell
    converges fast for the smooth field at planes between the charges (64 x 64
    points here; a wrong plane-average mode would be off by O(1))."""
    x, q = _cell(8, seed=5)
    e = Ewald2D(BOX)
    m = 64
    g = (np.arange(m) + 0.5) / m - 0.5
    X, Y = np.meshgrid(g * BOX[0], g * BOX[1], indexing="ij")
    A = BOX[0] * BOX[1]
    zs = np.sort(x[:, 2])
    gap = int(np.argmax(np.diff(zs)))          # the plane between charges farthest from both
    for z0 in (0.5 * (zs[gap] + zs[gap + 1]), 0.55 * BOX[2], -0.55 * BOX[2]):
        pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z0)], 1)
        _, f = e.solve(x, q, targets=pts)
        q_above = q[x[:, 2] > z0].sum()
        assert abs(f[:, 2].mean() + 4 * math.pi * q_above / A) < 1e-6 * max(1.0, abs(4 * math.pi * q_above / A))


def test_exact_potential_satisfies_the_decay_rows():
    """The premise of the decay rows: on the planes z = +-z_d the exact slab
    potential (Ewald) has <(d/dz + s|k|) phi, trig(k.rho)> = 0 for every mode."""
    x, q = _cell(10, seed=7)
    pl = SlabPlan(BOX, 12, lam=1.6)
    e = Ewald2D(BOX, zspan=2 * pl.zd)
    for s, pts, proj in pl.planes:
        phi, f = e.solve(x, q, targets=pts)
        scale = np.abs(f[:, 2]).max()
        for kk, wv in proj:
            assert abs((-f[:, 2] + s * kk * phi) @ wv) < 1e-9 * scale


def test_modes_and_plane_quadrature():
    modes = decay_modes(3, BOX)
    assert len(modes) == 4 * 7 - 3                       # (nk+1)(2nk+1) - nk, one per +-k pair
    assert np.allclose(modes[0], 0.0)
    keys = {(round(a, 12), round(b, 12)) for a, b in modes}
    assert not any((round(-a, 12), round(-b, 12)) in keys for a, b in modes if (a, b) != (0.0, 0.0))
    pts, w = plane_points(BOX, 0.3, 9)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(w @ pts[:, 0] ** 2 - BOX[0] ** 2 / 12) < 1e-15     # mean of x^2 over the rectangle
    assert abs(w @ (pts[:, 0] ** 4 * pts[:, 1] ** 2) - BOX[0] ** 4 / 80 * BOX[1] ** 2 / 12) < 1e-15


def test_near_set_uses_in_plane_images_only():
    x, q = W.uniform_box(400, BOX, charges="gauss", seed=9)
    xs, qs, base, img = slab_near_set(x, q, BOX, 1.5)
    shift = xs - x[base]
    assert np.all(shift[:, 2] == 0.0)
    # complete: every in-plane image within the ball of the widest range is kept
    for i in range(-3, 4):
        for j in range(-3, 4):
            p = np.array([i * BOX[0], j * BOX[1], 0.0])
            inside = np.nonzero(((x + p) ** 2).sum(1) <= 1.5 ** 2 * (1 - 1e-9))[0]
            sel = np.all(np.isclose(shift, p[None, :], rtol=0, atol=1e-12), axis=1)
            assert set(inside) <= set(base[sel])


def test_periodicity_alone_leaves_the_slab_fit_ill_posed():
    """The periodicity rows alone: their matrix loses rank and its condition number
    explodes with p (x/y-periodic harmonic functions e^{+-|k|z} e^{ik.rho} are
    well approximated by polynomials in the ball); with the decay rows the fit has
    full rank and a moderate condition number."""
    for p, bound in ((12, 1e3), (16, 1e4)):
        pl = SlabPlan(BOX, p, lam=1.6)
        s = np.linalg.svd(pl.A_per, compute_uv=False)
        assert s[-1] / s[0] < 1e-6
        assert pl.rank == p * p - 1 and pl.cond < bound


def test_slab_matches_ewald_and_converges_with_p():
    x, q = W.uniform_box(300, BOX, charges="gauss", seed=5)
    pe, fe = Ewald2D(BOX).solve(x, q)
    errs = []
    for p in (12, 16, 20):
        phi, f = SlabPlan(BOX, p, lam=1.6).solve(x, q)
        d = phi - pe
        errs.append((np.linalg.norm(f - fe) / np.linalg.norm(fe),
                     np.linalg.norm(d - d.mean()) / np.linalg.norm(pe - pe.mean())))
    assert errs[-1][0] < 1e-6 and errs[-1][1] < 2e-6
    assert errs[0][0] > 20 * errs[-1][0] and errs[0][1] > 20 * errs[-1][1]


@pytest.mark.parametrize("box", [(1.0, 1.0, 0.3), (1.0, 1.0, 2.0), (2.0, 1.0, 0.7)])
def test_slab_matches_ewald_for_thin_thick_and_elongated_cells(box):
    box = np.asarray(box)
    x, q = W.uniform_box(200, box, charges="gauss", seed=15)
    pe, fe = Ewald2D(box).solve(x, q)
    phi, f = SlabPlan(box, 20, lam=1.6).solve(x, q)
    d = phi - pe
    assert np.linalg.norm(f - fe) / np.linalg.norm(fe) < 2e-6
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(pe - pe.mean()) < 3e-6


def test_strongly_dipolar_cell_along_the_free_axis():
    """Positive charges near the top, negative near the bottom: the uniform field
    the dipole layer sets up inside the cell (Gauss's law, the k = 0 decay rows)
    is reproduced."""
    g = np.random.default_rng(21)
    n = 100
    x = (g.random((n, 3)) - 0.5) * BOX
    x[: n // 2, 2] = 0.3 + 0.05 * g.random(n // 2)
    x[n // 2:, 2] = -0.35 + 0.05 * g.random(n // 2)
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    pe, fe = Ewald2D(BOX).solve(x, q)
    phi, f = SlabPlan(BOX, 20, lam=1.6).solve(x, q)
    assert np.linalg.norm(f - fe) / np.linalg.norm(fe) < 1e-6
    assert abs(f[:, 2].mean() - fe[:, 2].mean()) < 1e-6 * np.abs(fe[:, 2]).mean()


def test_periodic_in_x_and_y_and_translation_invariant_in_plane():
    x, q = W.uniform_box(250, BOX, charges="gauss", seed=31)
    pl = SlabPlan(BOX, 20, lam=1.6)
    g = np.random.default_rng(32)
    y = (g.random((40, 3)) - 0.5) * BOX
    for k in (0, 1):
        a = y.copy()
        a[:, k] = -0.5 * BOX[k]
        b = a.copy()
        b[:, k] = 0.5 * BOX[k]
        pa, fa = pl.solve(x, q, targets=a)
        pb, fb = pl.solve(x, q, targets=b)
        assert _worst(pb, pa) < 2e-6 and _worst(fb, fa) < 2e-6
    phi, f = pl.solve(x, q)
    s = np.array([0.37, -0.21, 0.0])
    xs = (x + s + 0.5 * BOX) % BOX - 0.5 * BOX
    xs[:, 2] = x[:, 2]
    phi2, f2 = pl.solve(xs, q)
    d = phi2 - phi
    assert np.linalg.norm(f2 - f) / np.linalg.norm(f) < 2e-6
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(phi - phi.mean()) < 3e-6


def test_slab_adjoint_matches_finite_differences():
    """The exact energy gradient with the decay rows' adjoint sources (a charge and
    a dipole at each plane point, oracle/adjoint.py) against central differences
    (h = 1e-5) in positions and in neutral pairs of charges."""
    from oracle.adjoint import energy_gradients_decay
    box = np.array([1.0, 1.2, 0.8])
    pl = SlabPlan(box, 8, lam=1.6)
    x, q = W.uniform_box(30, box, charges="gauss", seed=5)

    def energy(xx, qq):
        phi, _ = pl.solve(xx, qq)
        return 0.5 * float(qq @ phi)

    E, dEdx, dEdq = energy_gradients_decay(pl, x, q)
    assert abs(E - energy(x, q)) < 1e-14 * abs(E)
    h = 1e-5
    for i in (0, 3, 7):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (energy(xp, q) - energy(xm, q)) / (2 * h)
            assert abs(dEdx[i, k] - fd) < 2e-8 * max(1.0, abs(fd))
    for i, j in ((0, 1), (4, 22)):
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qp[j] -= h
        qm[i] -= h
        qm[j] += h
        fd = (energy(x, qp) - energy(x, qm)) / (2 * h)
        assert abs((dEdq[i] - dEdq[j]) - fd) < 1e-8 * max(1.0, abs(fd))
