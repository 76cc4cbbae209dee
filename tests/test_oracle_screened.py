"""Pins of the oracle for the screened Coulomb kernel exp(-kappa r)/r
(oracle/screened.py): the direct sums against the mathematics of the kernel,
the Ewald-type split against its own splitting parameter and against
brute-force lattice sums, and the method against the split.

The paper gives no worked example for this kernel (Sec. 1 and the Conclusion
say the method applies to other kernels, details to be worked out), so what
fixes the results is: the modified Helmholtz equation, the Coulomb limit
kappa -> 0, the exponential convergence of the lattice sum, periodicity and
translation invariance.
"""
import numpy as np
import pytest

import workloads as W
from oracle import _native
from oracle.screened import EwaldScreened, ScreenedPlan, kernel_matrix, lattice_sum

BOX = np.array([1.0, 1.2, 0.8])


def _cell(n=12, seed=1, box=BOX, neutral=False):
    g = np.random.default_rng(seed)
    x = (g.random((n, 3)) - 0.5) * box
    q = g.standard_normal(n)
    if neutral:
        q -= q.mean()
    return x, q


def _worst(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_direct_sum_solves_the_modified_helmholtz_equation():
    """Away from the charges, Laplace(phi) = kappa^2 phi (central differences,
    h = 1e-3, fourth-order stencil)."""
    x, q = _cell(6, seed=2)
    kappa = 3.0
    g = np.random.default_rng(3)
    y = (g.random((20, 3)) - 0.5) * 4.0 + 3.0       # well away from the charges
    h = 1e-3
    phi = _native.direct_screened(y, x, q, kappa, grad=False)
    lap = np.zeros(len(y))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        f = [_native.direct_screened(y + s * e, x, q, kappa, grad=False) for s in (-2, -1, 1, 2)]
        lap += (-f[0] + 16 * f[1] - 30 * phi + 16 * f[2] - f[3]) / (12 * h * h)
    assert np.abs(lap - kappa ** 2 * phi).max() < 1e-6 * np.abs(kappa ** 2 * phi).max()


def test_direct_sum_gradient_and_coulomb_limit():
    x, q = _cell(8, seed=4)
    y = (np.random.default_rng(5).random((15, 3)) - 0.5) * 3.0
    phi, grad = _native.direct_screened(y, x, q, 1.7)
    h = 1e-5
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (_native.direct_screened(y + e, x, q, 1.7, grad=False)
              - _native.direct_screened(y - e, x, q, 1.7, grad=False)) / (2 * h)
        assert np.abs(fd - grad[:, k]).max() < 1e-7 * np.abs(grad).max()
    # kappa -> 0: the Coulomb sum (the 1/r direct sum is pinned on its own)
    pc, gc = _native.direct(y, x, q)
    ps, gs = _native.direct_screened(y, x, q, 1e-9)
    assert _worst(ps, pc) < 1e-7 and _worst(gs, gc) < 1e-7
    # near a charge phi ~ q/r
    yy = x[:1] + np.array([[1e-7, 0.0, 0.0]])
    assert abs(_native.direct_screened(yy, x[:1], q[:1], 1.7, grad=False)[0] * 1e-7 / q[0] - 1.0) < 1e-6


def test_kernel_at_coincident_points_is_zero():
    x, q = _cell(5, seed=6)
    phi, grad = _native.direct_screened(x[:1], x[:1], q[:1], 2.0)
    assert phi[0] == 0.0 and np.all(grad == 0.0)


@pytest.mark.parametrize("kappa", [0.5, 2.0, 6.0])
def test_ewald_split_does_not_depend_on_alpha(kappa):
    x, q = _cell()
    a = EwaldScreened(BOX, kappa, alpha=3.0).solve(x, q)
    for alpha in (4.5, 7.0):
        b = EwaldScreened(BOX, kappa, alpha=alpha).solve(x, q)
        assert _worst(b[0], a[0]) < 1e-13 and _worst(b[1], a[1]) < 1e-13


@pytest.mark.parametrize("kappa", [2.0, 6.0])
def test_ewald_split_equals_the_brute_force_lattice_sum(kappa):
    """The lattice sum converges absolutely; summed over every image whose
    terms exceed 1e-17, it is exact to rounding.  Net charge is not zero here."""
    x, q = _cell(10, seed=7)
    assert abs(q.sum()) > 0.5
    e = EwaldScreened(BOX, kappa).solve(x, q)
    b = lattice_sum(x, q, BOX, kappa)
    assert _worst(b[0], e[0]) < 1e-13 and _worst(b[1], e[1]) < 1e-13
    g = np.random.default_rng(8)
    y = (g.random((7, 3)) - 0.5) * BOX
    e = EwaldScreened(BOX, kappa).solve(x, q, targets=y)
    b = lattice_sum(x, q, BOX, kappa, targets=y)
    assert _worst(b[0], e[0]) < 1e-13 and _worst(b[1], e[1]) < 1e-13


def test_fit_has_no_null_space():
    """Full column rank: no constant or other periodic solution to remove."""
    R0 = 0.5 * np.linalg.norm(BOX)
    cen = W.thomson_points(256, 1.5 * R0)
    for kappa in (0.5, 2.0, 6.0):
        pl = ScreenedPlan(BOX, kappa, cen, 16, lam=1.5)
        assert pl.rank == pl.M == 256
        assert np.allclose(pl.A, kernel_matrix(pl.yc, cen, kappa) - kernel_matrix(pl.yt, cen, kappa), rtol=0, atol=0)


@pytest.mark.parametrize("kappa,bound", [(2.0, 4e-6), (6.0, 3e-6)])
def test_method_matches_the_ewald_split_and_converges(kappa, bound):
    """Method accuracy against the independent split, non-neutral charges;
    the error falls when the centres and check points grow."""
    x, q = W.uniform_box(300, BOX, charges="gauss", seed=5)
    q = q + 0.1                                      # a net charge is allowed
    ref = EwaldScreened(BOX, kappa).solve(x, q)
    R0 = 0.5 * np.linalg.norm(BOX)
    errs = []
    for M, p in ((256, 16), (400, 20)):
        pl = ScreenedPlan(BOX, kappa, W.thomson_points(M, 1.5 * R0), p, lam=1.5)
        ph, f = pl.solve(x, q)
        errs.append(max(np.linalg.norm(ph - ref[0]) / np.linalg.norm(ref[0]),
                        np.linalg.norm(f - ref[1]) / np.linalg.norm(ref[1])))
    assert errs[1] < bound and errs[0] > 3 * errs[1]


def test_method_is_periodic_and_translation_invariant():
    kappa = 3.0
    x, q = W.uniform_box(250, BOX, charges="gauss", seed=31)
    R0 = 0.5 * np.linalg.norm(BOX)
    pl = ScreenedPlan(BOX, kappa, W.thomson_points(400, 1.5 * R0), 20, lam=1.5)
    g = np.random.default_rng(32)
    y = (g.random((40, 3)) - 0.5) * BOX
    for k in range(3):
        a = y.copy()
        a[:, k] = -0.5 * BOX[k]
        b = a.copy()
        b[:, k] = 0.5 * BOX[k]
        pa, fa = pl.solve(x, q, targets=a)
        pb, fb = pl.solve(x, q, targets=b)
        assert _worst(pb, pa) < 2e-5 and _worst(fb, fa) < 2e-5
    phi, f = pl.solve(x, q)
    s = np.array([0.37, -0.21, 0.13])
    xs = (x + s + 0.5 * BOX) % BOX - 0.5 * BOX
    phi2, f2 = pl.solve(xs, q)
    assert np.linalg.norm(phi2 - phi) / np.linalg.norm(phi) < 1e-5
    assert np.linalg.norm(f2 - f) / np.linalg.norm(f) < 1e-5


def _screened_energy(pl, x, q):
    phi, _ = pl.solve(x, q)
    return 0.5 * float(q @ phi)


def test_screened_adjoint_matches_finite_differences():
    """The exact gradient of the screened method's energy against central
    differences (h = 1e-5) in positions and in single charges (any net charge)."""
    from oracle.screened import energy_gradients_screened
    R0 = 0.5 * np.linalg.norm(BOX)
    pl = ScreenedPlan(BOX, 2.0, W.thomson_points(64, 1.5 * R0), 8, lam=1.5)
    x, q = _cell(30, seed=51)
    E, dEdx, dEdq = energy_gradients_screened(pl, x, q)
    assert abs(E - _screened_energy(pl, x, q)) < 1e-14 * abs(E)
    P = np.array([[i, j, k] for i in (-2, -1, 0, 1, 2) for j in (-2, -1, 0, 1, 2) for k in (-2, -1, 0, 1, 2)]) * BOX
    d = np.abs(np.linalg.norm(x[:, None, :] + P[None, :, :], axis=2) - pl.R_b).min(axis=1)
    h = 1e-5
    for i in np.nonzero(d > 1e-3)[0][:4]:
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (_screened_energy(pl, xp, q) - _screened_energy(pl, xm, q)) / (2 * h)
            assert abs(dEdx[i, k] - fd) < 1e-7 * max(1.0, abs(fd))
    for i in (0, 7, 19):
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qm[i] -= h
        fd = (_screened_energy(pl, x, qp) - _screened_energy(pl, x, qm)) / (2 * h)
        assert abs(dEdq[i] - fd) < 1e-8 * max(1.0, abs(fd))
