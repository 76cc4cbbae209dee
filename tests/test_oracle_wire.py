"""Pins of the oracle's one-axis periodization (oracle/wire.py).

The paper only states that the periodic extension may be done along one or two
coordinates (Sec. 1, closing paragraph).  What fixes the result here is not the
oracle's own formulas but: brute-force sums over growing symmetric rows of
images (extrapolated), which are themselves checked against the Fourier
representation of a periodic row of charges (a series of K_0 Bessel functions,
from Poisson summation along x), the decay of the exact potential's Fourier
modes away from the axis, the exact null space of the periodicity rows,
periodicity in x and translation invariance along x.
"""
import math

import numpy as np
from scipy.special import k0, k1, kv, kvp

import workloads as W
from oracle.wire import WirePlan, decay_beta, line_sum, wire_near_set

BOX = np.array([1.0, 1.2, 0.8])


def _cell(n=40, seed=3, box=BOX):
    g = np.random.default_rng(seed)
    x = (g.random((n, 3)) - 0.5) * box
    q = g.standard_normal(n)
    q -= q.mean()
    return x, q


def _fourier_row(x, q, d, y, nmax=400):
    """sum_j q_j sum_i 1/|y - x_j - i d e_x| for neutral charges, up to a constant:
    sum_j q_j [-(2/d) log rho_j + (4/d) sum_n K_0(2 pi n rho_j/d) cos(2 pi n (y_x - x_jx)/d)],
    rho_j the distance of y from the row through x_j; and the field."""
    phi = np.zeros(len(y))
    f = np.zeros((len(y), 3))
    for j in range(len(x)):
        dx = y[:, 0] - x[j, 0]
        dy, dz = y[:, 1] - x[j, 1], y[:, 2] - x[j, 2]
        rho = np.hypot(dy, dz)
        phi += q[j] * (-2.0 / d) * np.log(rho)
        frho = q[j] * (2.0 / d) / rho                      # -d/drho of the log term
        fx = np.zeros(len(y))
        for n in range(1, nmax + 1):
            k = 2.0 * math.pi * n / d
            phi += q[j] * (4.0 / d) * k0(k * rho) * np.cos(k * dx)
            frho += q[j] * (4.0 / d) * k * k1(k * rho) * np.cos(k * dx)
            fx += q[j] * (4.0 / d) * k * k0(k * rho) * np.sin(k * dx)
        f[:, 0] += fx
        f[:, 1] += frho * dy / rho
        f[:, 2] += frho * dz / rho
    return phi, f


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _worst(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_brute_force_row_sum_equals_the_fourier_series():
    """Targets kept at least 0.1 from every charge's row so the K_0 series
    converges (terms below 1e-30 at n = 400)."""
    x, q = _cell(8, seed=11)
    g = np.random.default_rng(12)
    y = (g.random((30, 3)) - 0.5) * BOX
    rho = np.min([np.hypot(y[:, 1] - x[j, 1], y[:, 2] - x[j, 2]) for j in range(len(x))], axis=0)
    y = y[rho > 0.1]
    pb, fb = line_sum(x, q, BOX, targets=y)
    pf, ff = _fourier_row(x, q, BOX[0], y)
    assert _worst(pb - pb.mean(), pf - pf.mean()) < 1e-8
    assert _worst(fb, ff) < 1e-8


def test_decay_ratio_against_the_bessel_derivative_and_its_asymptote():
    """k K_m'(k rho)/K_m(k rho) against scipy's K_m and K_m' where they are finite,
    and against the large-argument expansion -1 - 1/(2z) - (4m^2 - 1)/(8z^2) where
    K_m underflows; k = 0 gives -m/rho."""
    for z in (0.01, 0.3, 2.0, 20.0, 100.0):
        for m in (0, 1, 5, 39):
            assert abs(decay_beta(z, m, 1.0) / (z * kvp(m, z) / kv(m, z)) - 1.0) < 1e-14
    for m in (0, 1, 2):
        z = 2000.0
        assert abs(decay_beta(z, m, 1.0) / z - (-1.0 - 0.5 / z - (4 * m * m - 1) / (8 * z * z))) < 1e-9
    assert decay_beta(0.0, 3, 0.5) == -6.0


def test_exact_potential_satisfies_the_decay_rows():
    x, q = _cell(12, seed=7)
    pl = WirePlan(BOX, 12, lam=1.6)
    ph, f = line_sum(x, q, BOX, targets=pl.pts)
    drho = -(f[:, 1] * np.cos(pl.theta) + f[:, 2] * np.sin(pl.theta))
    scale = np.abs(f).max()
    for beta, wv in pl.modes:
        assert abs((drho - beta * ph) @ wv) < 1e-8 * scale


def test_periodicity_rows_alone_have_an_exact_null_space():
    """rho^m cos/sin(m theta), m = 1..p-1, are harmonic, x-independent polynomials:
    2(p-1) exact null vectors of the periodicity rows; with the decay rows the fit
    has full rank and a small condition number."""
    for p in (8, 12):
        pl = WirePlan(BOX, p, lam=1.6)
        s = np.linalg.svd(pl.A_per, compute_uv=False)
        assert np.sum(s > 1e-10 * s[0]) <= p * p - 1 - 2 * (p - 1)
        assert pl.rank == p * p - 1 and pl.cond < 100


def test_near_set_uses_images_along_x_only():
    x, q = W.uniform_box(300, BOX, charges="gauss", seed=9)
    xs, qs, base, img = wire_near_set(x, q, BOX, 1.5)
    shift = xs - x[base]
    assert np.all(shift[:, 1:] == 0.0)
    for i in range(-3, 4):
        p = np.array([i * BOX[0], 0.0, 0.0])
        inside = np.nonzero(((x + p) ** 2).sum(1) <= 1.5 ** 2 * (1 - 1e-9))[0]
        sel = np.all(np.isclose(shift, p[None, :], rtol=0, atol=1e-12), axis=1)
        assert set(inside) <= set(base[sel])


def test_method_matches_the_row_sum_and_converges_with_p():
    x, q = _cell()
    pe, fe = line_sum(x, q, BOX)
    errs = []
    for p in (12, 16, 20):
        phi, f = WirePlan(BOX, p, lam=1.6).solve(x, q)
        d = phi - pe
        errs.append((_rel(f, fe), np.linalg.norm(d - d.mean()) / np.linalg.norm(pe - pe.mean())))
    assert errs[-1][0] < 1e-6 and errs[-1][1] < 2e-6
    assert errs[0][0] > 20 * errs[-1][0] and errs[0][1] > 20 * errs[-1][1]


def test_charges_next_to_the_cylinder():
    """Charges a hair inside the box's long edges sit h from the decay cylinder:
    the quadrature still resolves their near potential."""
    x, q = _cell()
    x[0] = [0.1, 0.5999, 0.3999]
    x[1] = [-0.3, -0.5999, 0.3999]
    x[2] = [0.45, 0.5999, -0.3999]
    q -= q.mean()
    pe, fe = line_sum(x, q, BOX)
    phi, f = WirePlan(BOX, 20, lam=1.6).solve(x, q)
    d = phi - pe
    assert _rel(f, fe) < 2e-6 and np.linalg.norm(d - d.mean()) / np.linalg.norm(pe - pe.mean()) < 3e-6


def test_thin_and_long_cells_and_a_transverse_dipole():
    """p = 16 (errors 2e-6 .. 6e-6 here) to keep the CPU suite short."""
    for box in ((1.0, 0.5, 0.5), (0.5, 1.0, 0.8), (2.0, 1.0, 0.7)):
        box = np.asarray(box)
        x, q = _cell(30, seed=21, box=box)
        pe, fe = line_sum(x, q, box)
        phi, f = WirePlan(box, 16, lam=1.6).solve(x, q)
        d = phi - pe
        assert _rel(f, fe) < 1e-5, box
        assert np.linalg.norm(d - d.mean()) / np.linalg.norm(pe - pe.mean()) < 1.5e-5, box
    # positive charges at +y, negative at -y: a dipole moment per length across the wire
    g = np.random.default_rng(22)
    n = 40
    x = (g.random((n, 3)) - 0.5) * BOX
    x[: n // 2, 1] = 0.4 + 0.1 * g.random(n // 2)
    x[n // 2:, 1] = -0.5 + 0.1 * g.random(n // 2)
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    pe, fe = line_sum(x, q, BOX)
    phi, f = WirePlan(BOX, 16, lam=1.6).solve(x, q)
    assert _rel(f, fe) < 5e-6


def test_periodic_in_x_and_translation_invariant_along_x():
    x, q = W.uniform_box(200, BOX, charges="gauss", seed=31)
    pl = WirePlan(BOX, 16, lam=1.6)
    g = np.random.default_rng(32)
    y = (g.random((40, 3)) - 0.5) * BOX
    a = y.copy()
    a[:, 0] = -0.5 * BOX[0]
    b = a.copy()
    b[:, 0] = 0.5 * BOX[0]
    pa, fa = pl.solve(x, q, targets=a)
    pb, fb = pl.solve(x, q, targets=b)
    assert _worst(pb, pa) < 5e-6 and _worst(fb, fa) < 5e-6
    phi, f = pl.solve(x, q)
    xs = x.copy()
    xs[:, 0] = (x[:, 0] + 0.37 + 0.5 * BOX[0]) % BOX[0] - 0.5 * BOX[0]
    phi2, f2 = pl.solve(xs, q)
    d = phi2 - phi
    assert _rel(f2, f) < 6e-6
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(phi - phi.mean()) < 2.5e-5


def test_wire_adjoint_matches_finite_differences():
    """The exact energy gradient with the decay rows' adjoint sources (a charge and
    a radial dipole at each cylinder point, oracle/adjoint.py) against central
    differences (h = 1e-5) in positions and in neutral pairs of charges."""
    from oracle.adjoint import energy_gradients_decay
    pl = WirePlan(BOX, 8, lam=1.6)
    x, q = W.uniform_box(30, BOX, charges="gauss", seed=5)

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
