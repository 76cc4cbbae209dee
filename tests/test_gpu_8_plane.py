"""The method in the plane (Sec. 1: it applies to 2-D problems), kernel -log r,
periodic along x and y: the HIP path against the oracle's 2-D method
(oracle/twod.py), which its own pins tie to an independent 2-D Ewald split, the
Jacobi theta-function closed form and brute-force squares of images.

Bars (tests/gpu_common.py): FP64 <= 1e-12, FP32 pairs with FP64 accumulation
<= 1e-6, on the relative L2 error and on the worst element; near-set sizes exact.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import TOL, dev, err, golden, load_ps, rel
from oracle.twod import EwaldLog2D, Plan2D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOX = (1.0, 1.3)


@pytest.fixture(scope="module")
def ps():
    return load_ps()


def _cell(n, seed, box=BOX):
    g = np.random.default_rng(seed)
    x = (g.random((n, 2)) - 0.5) * np.array(box)
    q = g.standard_normal(n)
    return x, q - q.mean()


def _plane(ps, box, p, x, q, prec, lam=1.5, targets=None, **kw):
    pl = ps.Plan(box, p, lam=lam, precision=prec, n_max=len(q), m_max=0 if targets is None else len(targets),
                 dim=2, **kw)
    phi, field = pl.eval(dev(x.T), dev(q), targets=None if targets is None else dev(targets.T))
    pl.status()
    return pl, phi.cpu().numpy(), field.cpu().numpy().T


def test_plane_tables_match_oracle(ps):
    """Check points on the circumcircle (z = 0), partners along x or y, the
    pseudo-inverse, the box means of the harmonic polynomials."""
    for box, p in ((BOX, 16), ((2.0, 0.7), 40), ((1.0, 1.0), 12), ((0.6, 1.5), 100)):
        op = Plan2D(box, p, lam=1.5)
        pl = ps.Plan(box, p, lam=1.5, n_max=10, dim=2)
        inf = pl.info()
        assert inf["dim"] == 2 and inf["P"] == 2 * p - 1 and inf["L"] == op.L == 4 * p
        assert inf["rank"] == op.rank and abs(inf["cond"] / op.cond - 1) < 1e-9 and inf["n_rows"] == op.L
        yc, yt, pinv, bm = (t.numpy() for t in pl.tables())
        np.testing.assert_allclose(yc[:, :2], op.yc, atol=4e-15 * op.R0)
        np.testing.assert_allclose(yt[:, :2], op.yt, atol=4e-15 * op.R0)
        assert np.all(yc[:, 2] == 0.0) and np.all(yt[:, 2] == 0.0)
        assert err(pinv, op.Apinv) < 1e-12
        np.testing.assert_allclose(bm, op.R0mean, atol=1e-14)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plane_matches_oracle(ps, prec):
    x, q = _cell(3000, 201)
    ref = Plan2D(BOX, 32, lam=1.5).solve(x, q, return_parts=True)
    pl, phi, field = _plane(ps, BOX, 32, x, q, prec)
    e1, e2 = err(phi, ref["phi"]), err(field, ref["field"])
    print(prec, "plane err phi %.3e field %.3e" % (e1, e2))
    assert pl.info()["n_near_last"] == ref["n_near"]
    assert e1 <= TOL[prec] and e2 <= TOL[prec]
    assert rel(pl.coefficients().numpy(), ref["C"]) < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("box", [(1.0, 1.0), (2.0, 0.7), (0.6, 1.5)])
def test_plane_other_cells(ps, box):
    x, q = _cell(1500, 202, box)
    ref = Plan2D(box, 40, lam=1.6).solve(x, q)
    _, phi, field = _plane(ps, box, 40, x, q, "fp64", lam=1.6)
    assert err(phi, ref[0]) <= TOL["fp64"] and err(field, ref[1]) <= TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plane_separate_targets_on_particles_and_three_row_positions(ps, prec):
    """Targets anywhere in the box, some exactly on particles (K(0) = 0); positions
    given with a z row, which the plane does not read."""
    x, q = _cell(1200, 203)
    g = np.random.default_rng(204)
    y = (g.random((300, 2)) - 0.5) * np.array(BOX)
    y[:30] = x[:30]
    ref = Plan2D(BOX, 24, lam=1.5).solve(x, q, targets=y)
    _, phi, field = _plane(ps, BOX, 24, x, q, prec, targets=y)
    assert err(phi, ref[0]) <= TOL[prec] and err(field, ref[1]) <= TOL[prec]
    x3 = np.concatenate([x, g.random((len(q), 1))], axis=1)     # an arbitrary z row
    pl = ps.Plan(BOX, 24, lam=1.5, precision=prec, n_max=len(q), dim=2)
    phi3, field3 = pl.eval(dev(x3.T), dev(q))
    pl.status()
    phi2, field2 = pl.eval(dev(x.T), dev(q))
    pl.status()
    assert torch.equal(phi3, phi2) and torch.equal(field3, field2) and field2.shape == (2, len(q))


def test_plane_against_the_ewald_split(ps):
    """Method accuracy: FP32 at p = 40 against the independent 2-D Ewald split."""
    x, q = _cell(400, 205)
    pe, fe = EwaldLog2D(BOX).solve(x, q)
    _, phi, field = _plane(ps, BOX, 40, x, q, "fp32")
    assert err(phi, pe) < 1e-6 and err(field, fe) < 1e-6


def test_plane_batch(ps):
    """One graph launch over three rectangles of different shapes and sizes (FP64)."""
    boxes = [np.array(BOX), np.array([1.1, 1.0]), np.array([2.0, 0.7])]
    ns = [900, 700, 500]
    data = [_cell(n, 210 + k, b) for k, (n, b) in enumerate(zip(ns, boxes))]
    bp = ps.BatchedPlan([dict(box=b, n_max=n) for b, n in zip(boxes, ns)], p=30, lam=1.5, precision="fp64", dim=2)
    off = np.concatenate([[0], np.cumsum(ns)])
    phi, field = bp.eval(dev(np.concatenate([d[0] for d in data]).T), dev(np.concatenate([d[1] for d in data])), off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    for k in range(3):
        ref = Plan2D(boxes[k], 30, lam=1.5).solve(data[k][0], data[k][1])
        sl = slice(off[k], off[k + 1])
        assert err(phi[sl], ref[0]) <= TOL["fp64"] and err(field[sl], ref[1]) <= TOL["fp64"], k


def test_plane_plan_file_gradient_and_refusals(ps, tmp_path):
    """A reloaded plane plan gives bitwise the same sums; the physical gradient
    works (-q field, phi projected); non-neutral charges are refused."""
    from paper_1310_4374_amd import PeriodicSumError
    x, q = _cell(800, 206)
    pl = ps.Plan(BOX, 20, lam=1.5, precision="fp32", n_max=800, dim=2)
    X, Q = dev(x.T), dev(q)
    phi0, field0 = pl.eval(X, Q)
    pl.status()
    path = tmp_path / "plane.plan"
    pl.save(path)
    pl2 = ps.Plan.load(path)
    assert pl2.info()["dim"] == 2 and pl2.dim == 2
    phi1, field1 = pl2.eval(X, Q)
    pl2.status()
    assert torch.equal(phi0, phi1) and torch.equal(field0, field1)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=False)
    f = field0.cpu().numpy()
    assert gx.shape == (2, 800)
    assert np.allclose(gx.cpu().numpy(), -q[None, :] * f, rtol=0, atol=1e-12 * np.abs(f).max())
    ph = phi0.cpu().numpy()
    assert np.allclose(gq.cpu().numpy(), ph - ph.mean(), rtol=0, atol=1e-12 * np.abs(ph).max())
    assert abs(float(e.item()) - 0.5 * float(q @ ph)) < 1e-10 * abs(float(e.item()))
    pl.eval(X, dev(q + 0.1))
    with pytest.raises(PeriodicSumError, match="NOT_NEUTRAL"):
        pl.status()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plane_exact_adjoint_matches_oracle(ps, prec):
    """The exact gradient of the plane method's energy (the plane's moments,
    check-point charges, psi over the near images) against the oracle's, itself
    pinned to finite differences; dE/dq projected onto sum dq = 0."""
    from oracle.twod import energy_gradients2d
    x, q = _cell(1000, 207)
    E, dx, dq = energy_gradients2d(Plan2D(BOX, 24, lam=1.5), x, q)
    pl = ps.Plan(BOX, 24, lam=1.5, precision=prec, n_max=len(q), dim=2)
    X, Q = dev(x.T), dev(q)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=True)
    pl.status()
    assert abs(float(e.item()) / E - 1) <= TOL[prec]
    assert gx.shape == (2, len(q))
    assert err(gx.cpu().numpy().T, dx) <= TOL[prec] and err(gq.cpu().numpy(), dq) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_plane_full_size_workload(ps, prec):
    """The benchmark's plane workload (N = 100,000 in the unit square, p = 32,
    lambda = 1.5, the default launch shape it times): 2,000 sampled particles
    against the oracle's stored values (tests/golden/ref_plane.npz), near-set size exact."""
    c = W.config_plane()
    ref = golden("ref_plane.npz")
    pl, phi, field = _plane(ps, c["box"], c["p"], c["x"], c["q"], prec, lam=c["lam"])
    sub = ref["subset"]
    assert pl.info()["n_near_last"] == int(ref["n_near"])
    assert err(phi[sub], ref["phi"]) <= TOL[prec] and err(field[sub], ref["field"]) <= TOL[prec]
