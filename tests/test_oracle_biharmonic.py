"""Pins of the oracle's biharmonic-kernel method (oracle/biharmonic.py), K(r) = r:
the corner primitive of the box mean against its defining derivative and
quadrature, the Almansi basis against the expansion it must reproduce, the
Ewald-type reference against the Laplacian relation to the Coulomb sum and its
own split independence, and the method against that reference."""
import numpy as np
import pytest

from oracle.biharmonic import (BiharmonicPlan, EwaldBih, basis_bh, box_distance_mean, corner_primitive,
                               n_basis)
from oracle.boxmean import box_potential_mean
from oracle.ewald import Ewald


BOX = np.array([1.0, 1.1, 0.9])


def _cell(n, seed, box=BOX):
    g = np.random.default_rng(seed)
    x = (g.random((n, 3)) - 0.5) * box
    q = g.standard_normal(n)
    return x, q - q.mean()


def test_corner_primitive_third_derivative_is_r():
    """d^3 F/(dx dy dz) = r at points of every sign pattern, by a central
    difference in each variable (error O(h^2))."""
    g = np.random.default_rng(1)
    h = 1e-3
    for _ in range(40):
        p = g.uniform(-2, 2, size=3)
        p[np.abs(p) < 0.05] = 0.3
        acc = 0.0
        for a in (-1, 1):
            for b in (-1, 1):
                for c in (-1, 1):
                    acc += a * b * c * corner_primitive(p[0] + a * h, p[1] + b * h, p[2] + c * h)
        assert abs(acc / (8 * h ** 3) - np.linalg.norm(p)) < 2e-5 * np.linalg.norm(p)


def _mean_by_quadrature(xs, box, n):
    """(1/V) int |y - x| dV: tensor Gauss-Legendre, the box split at x when x is
    inside (so each piece has the cusp at a corner)."""
    out = []
    for x in xs:
        cuts = []
        for k in range(3):
            lo, hi = -box[k] / 2, box[k] / 2
            cuts.append([lo, x[k], hi] if lo < x[k] < hi else [lo, hi])
        tot = 0.0
        t, w = np.polynomial.legendre.leggauss(n)
        for i in range(len(cuts[0]) - 1):
            for j in range(len(cuts[1]) - 1):
                for k in range(len(cuts[2]) - 1):
                    lo = np.array([cuts[0][i], cuts[1][j], cuts[2][k]])
                    hi = np.array([cuts[0][i + 1], cuts[1][j + 1], cuts[2][k + 1]])
                    mid, half = (lo + hi) / 2, (hi - lo) / 2
                    P = np.stack(np.meshgrid(*(mid[a] + half[a] * t for a in range(3)), indexing="ij"), -1).reshape(-1, 3)
                    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel() * np.prod(half)
                    tot += (np.linalg.norm(P - x, axis=1) * W).sum()
        out.append(tot / np.prod(box))
    return np.array(out)


def test_box_distance_mean_against_quadrature():
    far = np.array([[2.5, 0.3, -1.7], [0.2, 3.1, 0.4], [-4.0, 2.0, 1.0], [0.0, 0.0, 1.6]])
    np.testing.assert_allclose(box_distance_mean(far, BOX), _mean_by_quadrature(far, BOX, 24), rtol=1e-13)
    inside = np.array([[0.1, 0.2, -0.3], [0.45, -0.5, 0.4], [0.0, 0.0, 0.0], [0.5, 0.55, 0.45]])
    np.testing.assert_allclose(box_distance_mean(inside, BOX), _mean_by_quadrature(inside, BOX, 40), rtol=1e-9)


def test_box_distance_mean_laplacian_is_twice_the_box_potential():
    """Delta |y - x| = 2/|y - x|, so Delta Psi0 = 2 Phi0 (App. C's box-mean
    potential, pinned on its own), here by second differences."""
    g = np.random.default_rng(2)
    xs = np.concatenate([(g.random((6, 3)) - 0.5) * BOX, g.uniform(-2, 2, size=(4, 3))])
    h = 2e-3
    lap = -6 * box_distance_mean(xs, BOX)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        lap += box_distance_mean(xs + e, BOX) + box_distance_mean(xs - e, BOX)
    np.testing.assert_allclose(lap / h ** 2, 2 * box_potential_mean(xs, BOX), rtol=2e-6)


def test_basis_reproduces_the_far_expansion_of_r():
    """|x - y| for a source y outside S_b is biharmonic inside: the Almansi basis
    fits it to rounding at p = 24, and the harmonics alone cannot."""
    R0 = 0.5 * np.linalg.norm(BOX)
    g = np.random.default_rng(3)
    pts = g.standard_normal((3000, 3))
    pts *= (R0 * g.random(3000) ** (1 / 3) / np.linalg.norm(pts, axis=1))[:, None]
    y = np.array([2.1, -1.3, 1.7]) * R0 / np.linalg.norm([2.1, -1.3, 1.7]) * 2.5
    target = np.linalg.norm(pts - y, axis=1)
    B = basis_bh(pts, 24, R0)
    c, *_ = np.linalg.lstsq(B.T, target, rcond=None)
    assert np.abs(B.T @ c - target).max() < 1e-10 * target.max()
    H = B[:24 * 24]
    c, *_ = np.linalg.lstsq(H.T, target, rcond=None)
    assert np.abs(H.T @ c - target).max() > 1e-3 * target.max()
    assert B.shape[0] == n_basis(24) == 24 * 24 + 22 * 22


def test_basis_gradient_against_differences():
    R0 = 0.5 * np.linalg.norm(BOX)
    g = np.random.default_rng(4)
    y = (g.random((5, 3)) - 0.5) * BOX
    _, dB = basis_bh(y, 10, R0, grad=True)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (basis_bh(y + e, 10, R0) - basis_bh(y - e, 10, R0)) / (2 * h)
        np.testing.assert_allclose(dB[k], fd, atol=1e-7 * np.abs(fd).max())


@pytest.fixture(scope="module")
def ewald_case():
    x, q = _cell(40, 5)
    return x, q, EwaldBih(BOX).solve(x, q)


def test_ewald_split_independence(ewald_case):
    x, q, ref = ewald_case
    phi, field = EwaldBih(BOX, alpha=3.3).solve(x, q)
    assert np.abs(phi - ref[0]).max() < 1e-13 * np.abs(ref[0]).max()
    assert np.abs(field - ref[1]).max() < 1e-13 * np.abs(ref[1]).max()


def test_ewald_laplacian_is_twice_the_coulomb_sum(ewald_case):
    """Delta r = 2/r, and both periodic sums have zero mean, so Delta phi_r equals
    2 phi_Coulomb exactly (the Coulomb Ewald sum is pinned on its own); checked
    away from the particles by second differences."""
    x, q = _cell(8, 6)
    g = np.random.default_rng(6)
    y = (g.random((400, 3)) - 0.5) * BOX
    sh = np.stack(np.meshgrid(*([np.arange(-1, 2)] * 3), indexing="ij"), -1).reshape(-1, 3) * BOX
    dmin = np.linalg.norm(y[:, None, None, :] - x[None, :, None, :] - sh[None, None, :, :], axis=3).min(axis=(1, 2))
    y = y[dmin > 0.15][:6]
    E = EwaldBih(BOX)
    h = 5e-3
    lap = -3 * 30 * E.solve(x, q, targets=y)[0]   # fourth-order second differences
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        f = [E.solve(x, q, targets=y + j * e)[0] for j in (-2, -1, 1, 2)]
        lap += -f[0] + 16 * f[1] + 16 * f[2] - f[3]
    pc = Ewald(BOX).solve(x, q, targets=y)[0]
    np.testing.assert_allclose(lap / (12 * h ** 2), 2 * pc, rtol=0, atol=1e-6 * np.abs(pc).max())


def test_ewald_field_is_minus_the_gradient_and_periodic(ewald_case):
    x, q, _ = ewald_case
    E = EwaldBih(BOX)
    g = np.random.default_rng(7)
    y = (g.random((4, 3)) - 0.5) * BOX
    phi, field = E.solve(x, q, targets=y)
    h = 1e-5
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (E.solve(x, q, targets=y + e)[0] - E.solve(x, q, targets=y - e)[0]) / (2 * h)
        np.testing.assert_allclose(-fd, field[:, k], atol=1e-8 * np.abs(field).max())
        ys = y + BOX[k] * np.eye(3)[k]
        p2, f2 = E.solve(x, q, targets=ys)
        assert np.abs(p2 - phi).max() < 1e-13 * np.abs(phi).max()
        assert np.abs(f2 - field).max() < 1e-12 * np.abs(field).max()


def test_method_matches_the_ewald_reference(ewald_case):
    """Value and gradient periodicity rows, p = 30, lambda = 2.5: the method's
    truncation error is below 1e-12 of the result."""
    x, q, ref = ewald_case
    pl = BiharmonicPlan(BOX, 30, lam=2.5)
    assert pl.A.shape == (4 * pl.L, pl.P - 1) and pl.rank == pl.P - 1
    phi, field = pl.solve(x, q)
    assert np.abs(phi - ref[0]).max() < 1e-12 * np.abs(ref[0]).max()
    assert np.abs(field - ref[1]).max() < 1e-12 * np.abs(field).max()


def test_method_converges_geometrically_in_p(ewald_case):
    x, q, ref = ewald_case
    errs = []
    for p in (12, 18, 24):
        phi, _ = BiharmonicPlan(BOX, p, lam=1.6).solve(x, q)
        errs.append(np.abs(phi - ref[0]).max() / np.abs(ref[0]).max())
    assert errs[0] > 10 * errs[1] > 100 * errs[2] and errs[2] < 1e-6


def test_value_rows_alone_do_not_fix_the_fit():
    """The reading's reason for the gradient rows: with the value rows only, A
    has a numerical null space beyond the dropped constant."""
    pl = BiharmonicPlan(BOX, 12, lam=1.5)
    Av = pl.A[: pl.L]
    s = np.linalg.svd(Av, compute_uv=False)
    assert (s > 1e-13 * s[0]).sum() < pl.P - 1
    assert pl.rank == pl.P - 1


def test_targets_translation_and_coincident_points():
    """Shifting every particle and target by one vector leaves phi and the field
    unchanged; a target on a particle gets the particle's own value (r is
    continuous and K(0) = 0)."""
    x, q = _cell(30, 8)
    pl = BiharmonicPlan(BOX, 30, lam=2.5)
    phi, field = pl.solve(x, q)
    s = np.array([0.07, -0.11, 0.05])
    xs = (x + s + BOX / 2) % BOX - BOX / 2
    phi2, field2 = pl.solve(xs, q)
    assert np.abs(phi2 - phi).max() < 1e-11 * np.abs(phi).max()
    assert np.abs(field2 - field).max() < 1e-11 * np.abs(field).max()
    y = np.concatenate([x[:5], [[0.2, -0.3, 0.1]]])
    pt, ft = pl.solve(x, q, targets=y)
    np.testing.assert_allclose(pt[:5], phi[:5], rtol=0, atol=1e-13 * np.abs(phi).max())
    np.testing.assert_allclose(ft[:5], field[:5], rtol=0, atol=1e-13 * np.abs(field).max())


def _energy(plan, x, q):
    return 0.5 * float(q @ plan.solve(x, q)[0])


def test_exact_energy_gradient_matches_differences():
    """The oracle's exact adjoint for K = r (charges and dipoles at the check
    points and partners) against central differences of its own energy, in
    positions (particles whose images stay clear of the near-ball sphere) and in
    neutral pairs of charges."""
    from oracle.biharmonic import energy_gradients_bih
    from oracle.geometry import lattice_vectors
    x, q = _cell(30, 9)
    pl = BiharmonicPlan(BOX, 12, lam=1.6)
    E, dx, dq = energy_gradients_bih(pl, x, q)
    assert abs(E - _energy(pl, x, q)) < 1e-14 * abs(E)
    P = lattice_vectors(pl.box, pl.R_b)
    clear = np.abs(np.linalg.norm(x[:, None, :] + P[None, :, :], axis=2) - pl.R_b).min(axis=1) > 1e-3
    h = 1e-5
    for i in np.nonzero(clear)[0][:4]:
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (_energy(pl, xp, q) - _energy(pl, xm, q)) / (2 * h)
            assert abs(dx[i, k] - fd) < 1e-7 * max(1.0, abs(fd))
    assert abs(dq.sum()) < 1e-12 * np.abs(dq).sum()
    for i, j in [(0, 1), (5, 20), (11, 29)]:
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qp[j] -= h
        qm[i] -= h
        qm[j] += h
        fd = (_energy(pl, x, qp) - _energy(pl, x, qm)) / (2 * h)
        assert abs((dq[i] - dq[j]) - fd) < 1e-8 * max(1.0, abs(fd))
