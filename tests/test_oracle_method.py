"""Pins for the oracle's implementation of the method (Sec. 2.3, Sec. 3) against
the Madelung constant, Table 1, Ewald, periodicity and translation invariance."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle.ewald import Ewald, MADELUNG_NACL
from oracle.method import Plan

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _eps_M(p, R_b=1.5):
    c = W.nacl_cell()
    phi, _ = Plan(c["box"], p, R_b=R_b).solve(c["x"], c["q"])
    return np.max(np.abs(phi * 0.5 / (-c["q"] * MADELUNG_NACL) - 1))


@pytest.mark.parametrize("p", [8, 12, 16])
def test_table1_gauss_grid_order_of_magnitude(p):
    """Table 1, Gauss column (lambda = sqrt 3): same order of magnitude (the
    paper's azimuth placement and partner rule are not stated)."""
    ref = GOLD["table1_gauss"]["eps_M"][str(p)]
    e = _eps_M(p)
    assert ref / 10 < e < ref * 10


def test_madelung_high_accuracy():
    """Sec. 4.1: p = 35, R_b = 1.5 gives eps_M ~ 6e-14."""
    assert _eps_M(35) < 5 * GOLD["nacl_small_test"]["eps_M"]["35"]


def test_error_decays_like_lambda_power():
    """Fig. 3 text / eq. (errb1): eps ~ C (R0/R_b)^p; the slope of log eps_M over p
    is close to -ln lambda (lambda = sqrt 3)."""
    ps = np.array([8, 12, 16, 20, 24])
    e = np.array([_eps_M(p) for p in ps])
    slope = np.polyfit(ps, np.log(e), 1)[0]
    assert -1.6 * np.log(np.sqrt(3)) < slope < -0.6 * np.log(np.sqrt(3))


@pytest.mark.parametrize("box,p,tol", [((1.0, 1.0, 1.0), 12, 3e-5), ((1.0, 1.0, 1.0), 24, 5e-9),
                                       ((1.0, 1.3, 2.1), 16, 3e-6), ((2.0, 1.0, 1.0), 20, 3e-7)])
def test_method_matches_ewald(box, p, tol):
    x, q = W.uniform_box(150, box, charges="gauss", seed=p)
    R0 = 0.5 * np.linalg.norm(box)
    phi, E = Plan(box, p, lam=np.sqrt(3)).solve(x, q)
    phe, Ee = Ewald(box).solve(x, q)
    assert _rel(phi, phe) < tol
    assert _rel(E, Ee) < tol


def test_method_matches_ewald_with_dipole_at_generic_targets():
    """Charges with a large dipole moment: the periodicity fit reproduces the
    conducting-boundary Ewald field with no extra side condition."""
    box = (1.0, 1.0, 1.0)
    g = np.random.default_rng(8)
    x = (g.random((40, 3)) - 0.5) * 0.9
    q = np.where(x[:, 0] > 0, 1.0, -1.0)
    q -= q.mean()
    y = (g.random((30, 3)) - 0.5)
    phi, E = Plan(box, 20, R_b=1.5).solve(x, q, targets=y)
    phe, Ee = Ewald(box).solve(x, q, targets=y)
    assert _rel(phi, phe) < 1e-7 and _rel(E, Ee) < 1e-7


def test_periodicity_on_faces():
    """phi(y + d_k e_k) = phi(y) (eq. (7)) at points on the faces."""
    box = np.array([1.0, 1.2, 0.9])
    x, q = W.uniform_box(100, box, charges="gauss", seed=2)
    g = np.random.default_rng(1)
    ys, ys2 = [], []
    for k in range(3):
        y = (g.random((10, 3)) - 0.5) * box
        y[:, k] = -box[k] / 2
        ys.append(y)
        y2 = y.copy()
        y2[:, k] += box[k]
        ys2.append(y2)
    pl = Plan(box, 24, lam=np.sqrt(3))
    a = pl.solve(x, q, targets=np.concatenate(ys))
    b = pl.solve(x, q, targets=np.concatenate(ys2))
    # truncation error at p = 24, lambda = sqrt 3 is ~1e-8 (it matches the error against Ewald)
    assert _rel(a[0], b[0]) < 1e-7 and _rel(a[1], b[1]) < 1e-7


def test_translation_invariance():
    """Shifting every particle by s (wrapped) changes the near/far split entirely
    but not the periodic solution."""
    box = np.array([1.0, 1.0, 1.3])
    x, q = W.uniform_box(120, box, charges="gauss", seed=3)
    pl = Plan(box, 24, lam=np.sqrt(3))
    a = pl.solve(x, q)
    xs = W.wrap(x + np.array([0.31, -0.17, 0.52]), box)
    b = pl.solve(xs, q)
    assert _rel(a[0], b[0]) < 1e-7 and _rel(a[1], b[1]) < 1e-7


def test_least_squares_normal_equations():
    x, q = W.uniform_box(200, (1, 1, 1), seed=6)
    pl = Plan((1, 1, 1), 12, R_b=1.5)
    parts = pl.solve(x, q, return_parts=True)
    r = pl.A @ parts["C"][1:] - parts["f"]
    assert np.abs(pl.A.T @ r).max() < 1e-10 * np.abs(pl.A.T @ parts["f"]).max()
    C2 = np.linalg.lstsq(pl.A, parts["f"], rcond=None)[0]
    np.testing.assert_allclose(parts["C"][1:], C2, rtol=1e-11, atol=1e-12 * np.abs(C2).max())
    assert pl.rank == pl.P - 1


def test_zero_mean_constant_only_shifts():
    x, q = W.uniform_box(100, (1, 1, 1), charges="gauss", seed=7)
    pl = Plan((1, 1, 1), 12, R_b=1.5)
    a = pl.solve(x, q, with_mean=True)
    b = pl.solve(x, q, with_mean=False)
    dd = a[0] - b[0]
    assert np.ptp(dd) < 1e-12 * np.abs(a[0]).max()
    np.testing.assert_array_equal(a[1], b[1])


def test_target_on_particle_uses_K0_zero():
    x, q = W.uniform_box(50, (1, 1, 1), charges="gauss", seed=8)
    pl = Plan((1, 1, 1), 12, R_b=1.5)
    a = pl.solve(x, q)
    b = pl.solve(x, q, targets=x[:7])
    np.testing.assert_allclose(b[0], a[0][:7], rtol=1e-14)
    np.testing.assert_allclose(b[1], a[1][:7], rtol=1e-14)


def test_rocksalt_lattice_madelung():
    """An 8^3-site rock-salt lattice (the small-cell analogue of the 32^3 lattice
    workload): every site's potential times the spacing is -q M (eq. (st1))."""
    r = W.rocksalt(8)
    # the truncation error grows with N (eq. (errb4.1)): 4e-6 at p = 16, 1.5e-7 at p = 20
    phi, E = Plan(r["box"], 20, R_b=1.5).solve(r["x"], r["q"])
    assert np.max(np.abs(phi * r["spacing"] / (-r["q"] * MADELUNG_NACL) - 1)) < 5e-7
    assert np.abs(E).max() * r["spacing"] ** 2 < 2e-6


def test_random_check_points_table1_order_of_magnitude():
    """Table 1, random columns (lambda = sqrt 3): the largest error over a few
    random sets is of the order of the paper's maximum over 100 sets."""
    GOLD_R = GOLD["table1_random"]["eps_M"]
    c = W.nacl_cell()
    for p, col, f in [(12, 1, 3), (16, 1, 3), (12, 2, 5)]:
        errs = []
        for seed in range(3):
            yc = W.random_sphere(f * p * p, np.sqrt(3) / 2, seed)
            phi, _ = Plan(c["box"], p, R_b=1.5, check_points=yc).solve(c["x"], c["q"])
            errs.append(np.max(np.abs(phi * 0.5 / (-c["q"] * MADELUNG_NACL) - 1)))
        ref = GOLD_R[str(p)][col]
        assert ref / 10 < max(errs) < ref * 10


@pytest.mark.parametrize("p", [8, 12, 16])
def test_table1_thomson_400_order_of_magnitude(p):
    """Table 1, T(400) column (lambda = sqrt 3): 400 Thomson check points give eps_M
    of the paper's order (the set's orientation and the partner rule are not
    stated; the paper's points come from a database, ours from a minimizer)."""
    ref = GOLD["table1_thomson"]["eps_M"]["400"][str(p)]
    c = W.nacl_cell()
    yc = W.thomson_points(400, np.sqrt(3) / 2)
    phi, _ = Plan(c["box"], p, R_b=1.5, check_points=yc).solve(c["x"], c["q"])
    e = np.max(np.abs(phi * 0.5 / (-c["q"] * MADELUNG_NACL) - 1))
    assert ref / 10 < e < ref * 10


def test_rbf_basis_madelung_and_ewald():
    """Sec. 4.1, RBF basis (eq. (5)) with 256 Thomson sources on the sphere S_b and
    the Gauss check points of p = 16: eps_M of the order of the paper's 1.32e-7;
    random charges match Ewald to the method's accuracy."""
    ref = GOLD["rbf_basis"]
    c = W.nacl_cell()
    cen = W.thomson_points(ref["M"], 1.5)
    pl = Plan(c["box"], ref["p"], R_b=1.5, basis="rbf", centres=cen)
    phi, E = pl.solve(c["x"], c["q"])
    e = np.max(np.abs(phi * 0.5 / (-c["q"] * MADELUNG_NACL) - 1))
    assert ref["eps_M"] / 10 < e < ref["eps_M"] * 10
    assert pl.rank == ref["M"]
    box = (1.0, 1.2, 0.9)
    x, q = W.uniform_box(120, box, charges="gauss", seed=31)
    R0 = 0.5 * np.linalg.norm(box)
    pl = Plan(box, 16, lam=np.sqrt(3), basis="rbf", centres=W.fibonacci_sphere(256, np.sqrt(3) * R0))
    a = pl.solve(x, q)
    b = Ewald(box).solve(x, q)
    assert _rel(a[0], b[0]) < 3e-5 and _rel(a[1], b[1]) < 3e-5


def test_rbf_box_means_are_phi0_at_centres():
    """For the RBF basis the box integral of R_t is Phi0 at the centre (App. C,
    as Sec. 3.4 notes): check one against direct quadrature."""
    box = (1.0, 1.0, 1.0)
    cen = W.fibonacci_sphere(8, 1.5)
    pl = Plan(box, 6, R_b=1.5, basis="rbf", centres=cen)
    g, w = np.polynomial.legendre.leggauss(20)
    X, Y, Z = np.meshgrid(g / 2, g / 2, g / 2, indexing="ij")
    Wt = (w[:, None, None] * w[None, :, None] * w[None, None, :]) / 8
    for t in range(3):
        r = np.sqrt((X - cen[t, 0]) ** 2 + (Y - cen[t, 1]) ** 2 + (Z - cen[t, 2]) ** 2)
        assert abs(pl.R0mean[1 + t] - np.sum(Wt / r)) < 1e-12


def _table2_pmin(lam):
    return {r[0]: r[1] for r in GOLD["table2"]["rows"]}[lam]


@pytest.mark.parametrize("lam, p_low", [(1.3, 30), (1.5, 20), (1.7, 16)])
def test_table2_p_min_meets_the_tolerance(lam, p_low):
    """Sec. 4.2, Table 2: N = 27,000 charges +-1 on a grid in the unit cube, Gauss
    check points, tolerance eps_2 = 5e-7 (eq. (st2)).  At the paper's p_min the
    method meets the tolerance against the independent Ewald sum (stored by
    tests/golden/make_reference.py from the oracle), and at a lower p it does not."""
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "ref_table2.npz"))
    x, q = W.grid_charges(30, 2)
    sub = ref["subset"]

    def eps2(p):
        phi, _ = Plan((1.0, 1.0, 1.0), p, lam=lam).solve(x, q, targets=x[sub])
        return _rel(phi, ref["phi_ewald"])

    assert eps2(_table2_pmin(lam)) < 5e-7
    assert eps2(p_low) > 5e-7


def test_table4_spherical_and_rbf_bases():
    """Sec. 4.2, Table 4 (lambda = 1.5, p = 16, N = 27,000 grid charges): eps_2 of
    the spherical basis and of 256 Thomson RBF centres on S_b, against the
    independent Ewald sum, within a factor 2 of the paper's 1.3e-5 and 2.6e-5,
    with the RBF basis the less accurate of the two, as the paper finds."""
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "ref_table2.npz"))
    gold = GOLD["table4"]["eps_2"]["27000"]
    x, q = W.grid_charges(30, 2)
    sub = ref["subset"]
    sph, _ = Plan((1.0, 1.0, 1.0), 16, lam=1.5).solve(x, q, targets=x[sub])
    cen = W.thomson_points(256, 1.5 * np.sqrt(3) / 2)
    rbf, _ = Plan((1.0, 1.0, 1.0), 16, lam=1.5, basis="rbf", centres=cen).solve(x, q, targets=x[sub])
    e_sph, e_rbf = _rel(sph, ref["phi_ewald"]), _rel(rbf, ref["phi_ewald"])
    assert gold["spherical"] / 2 < e_sph < gold["spherical"] * 2
    assert gold["rbf"] / 2 < e_rbf < gold["rbf"] * 2
    assert e_rbf > e_sph


def test_table3_p_min_meets_the_tolerance():
    """Sec. 4.2, Table 3 (216,000 grid charges, tolerance eps_2 = 5e-7): at the
    paper's p_min (lambda = 1.3 / 1.5 / 1.7 -> 34 / 25 / 19) the method meets the
    tolerance against the Ewald sum (both stored by make_reference.py from the
    oracle; recomputing them takes minutes)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "ref_table3.npz")
    ref = np.load(path)
    rows = {r[0]: r[1] for r in GOLD["table3"]["rows"]}
    for lam in (1.3, 1.5, 1.7):
        phi = ref["phi_method_%g_%d" % (lam, rows[lam])]
        assert _rel(phi, ref["phi_ewald"]) < 5e-7


def test_aspect_ratio_does_not_degrade_accuracy():
    """Sec. 4.2 (Table 5 discussion): at fixed lambda = 1.3 and p = 34 the box
    aspect ratio hardly changes the accuracy.  A 5:1:1 box meets the same
    tolerance against the Ewald sum as the cube, and its fitting matrix stays well
    conditioned with the basis evaluated at y/R0."""
    errs = []
    for k, box in enumerate([(1.0, 1.0, 1.0), (5.0, 1.0, 1.0)]):
        x, q = W.uniform_box(600, box, charges="gauss", seed=90 + k)
        pl = Plan(box, 34, lam=1.3)
        phi, _ = pl.solve(x, q)
        ref, _ = Ewald(box).solve(x, q)
        errs.append(_rel(phi, ref))
        assert pl.rank == 34 * 34 - 1 and pl.cond < 100
    assert max(errs) < 5e-7 and errs[1] < 10 * errs[0]
