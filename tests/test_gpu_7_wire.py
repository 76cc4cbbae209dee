"""Periodization along x only (a wire, y and z free; Sec. 1, closing paragraph):
the HIP path against the oracle's wire method (oracle/wire.py), which its own
pins tie to brute-force row sums and to their K_0 Fourier series.

Bars (tests/gpu_common.py): FP64 <= 1e-12, FP32 pairs with FP64 accumulation
<= 1e-6, on the relative L2 error and on the worst element; near-set sizes exact.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import TOL, dev, err, load_ps, rel
from oracle.wire import WirePlan, line_sum

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOX = (1.0, 1.2, 0.8)


@pytest.fixture(scope="module")
def ps():
    return load_ps()


def _wire(ps, box, p, x, q, prec, lam=1.6, targets=None, **kw):
    pl = ps.Plan(box, p, lam=lam, precision=prec, n_max=len(q), m_max=0 if targets is None else len(targets),
                 periodic="x", **kw)
    phi, field = pl.eval(dev(x.T), dev(q), targets=None if targets is None else dev(targets.T))
    pl.status()
    return pl, phi.cpu().numpy(), field.cpu().numpy().T


def test_wire_tables_match_oracle(ps):
    """Check points kept (|y_1| > d1/2), partners along x, the pseudo-inverse of
    the fit with its cylinder decay rows (Bessel-function ratios), box means."""
    for box, p in ((BOX, 12), ((1.0, 0.5, 0.5), 10), ((2.0, 1.0, 0.7), 9), ((0.3, 1.0, 0.9), 10)):
        op = WirePlan(np.array(box), p, lam=1.6)
        pl = ps.Plan(box, p, lam=1.6, n_max=10, periodic="x")
        inf = pl.info()
        assert inf["periodic"] == 1 and inf["L"] == op.L and inf["n_rows"] == op.A.shape[0]
        assert inf["rank"] == op.rank and abs(inf["cond"] / op.cond - 1) < 1e-9
        yc, yt, pinv, bm = (t.numpy() for t in pl.tables())
        np.testing.assert_allclose(yc, op.yc, atol=4e-15 * op.R0)
        np.testing.assert_allclose(yt, op.yt, atol=4e-15 * op.R0)
        assert err(pinv, op.Apinv) < 1e-11
        np.testing.assert_allclose(bm, op.R0mean, atol=1e-14)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wire_matches_oracle(ps, prec):
    x, q = W.uniform_box(2000, np.array(BOX), charges="gauss", seed=171)
    ref = WirePlan(np.array(BOX), 16, lam=1.6).solve(x, q, return_parts=True)
    pl, phi, field = _wire(ps, BOX, 16, x, q, prec)
    e1, e2 = err(phi, ref["phi"]), err(field, ref["field"])
    print(prec, "wire err phi %.3e field %.3e" % (e1, e2))
    assert pl.info()["n_near_last"] == ref["n_near"]
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


@pytest.mark.parametrize("box", [(1.0, 0.5, 0.5), (0.3, 1.0, 0.9), (2.0, 1.0, 0.7)])
def test_wire_thin_short_and_long_cells(ps, box):
    x, q = W.uniform_box(1500, np.array(box), charges="gauss", seed=172)
    ref = WirePlan(np.array(box), 12, lam=1.6).solve(x, q)
    _, phi, field = _wire(ps, box, 12, x, q, "fp64")
    assert err(phi, ref[0]) <= TOL["fp64"] and err(field, ref[1]) <= TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wire_separate_targets(ps, prec):
    """Separate targets anywhere in the box, some exactly on particles (K(0) = 0)."""
    x, q = W.uniform_box(1200, np.array(BOX), charges="gauss", seed=173)
    g = np.random.default_rng(174)
    y = (g.random((300, 3)) - 0.5) * np.array(BOX)
    y[:30] = x[:30]
    ref = WirePlan(np.array(BOX), 14, lam=1.6).solve(x, q, targets=y)
    _, phi, field = _wire(ps, BOX, 14, x, q, prec, targets=y)
    assert err(phi, ref[0]) <= TOL[prec] and err(field, ref[1]) <= TOL[prec]


def test_wire_against_the_row_sum(ps):
    """Method accuracy at p = 20: the library's FP32 wire solve against the
    Richardson-extrapolated brute-force row sum (fields; potentials up to the
    constant, which the row sum does not fix)."""
    x, q = W.uniform_box(150, np.array(BOX), charges="gauss", seed=175)
    pe, fe = line_sum(x, q, np.array(BOX))
    _, phi, field = _wire(ps, BOX, 20, x, q, "fp32")
    d = phi - pe
    assert rel(field, fe) < 2e-6
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(pe - pe.mean()) < 4e-6


def test_batch_of_wire_slab_and_three_axis_systems(ps):
    """One graph launch over a wire, a slab and a triply periodic box: each
    system matches its own oracle (FP64)."""
    from oracle.method import Plan as OPlan
    from oracle.slab import SlabPlan
    boxes = [np.array(BOX), np.array([1.1, 1.0, 1.3]), np.array([1.0, 1.5, 0.6])]
    per = ["x", "xy", "xyz"]
    ns = [900, 700, 500]
    data = [W.uniform_box(n, b, charges="gauss", seed=180 + k) for k, (n, b) in enumerate(zip(ns, boxes))]
    bp = ps.BatchedPlan([dict(box=b, n_max=n, periodic=s) for b, n, s in zip(boxes, ns, per)], p=12, lam=1.6,
                        precision="fp64")
    off = np.concatenate([[0], np.cumsum(ns)])
    phi, field = bp.eval(dev(np.concatenate([d[0] for d in data]).T), dev(np.concatenate([d[1] for d in data])), off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    oracles = {"x": WirePlan, "xy": SlabPlan, "xyz": OPlan}
    for k in range(3):
        ref = oracles[per[k]](boxes[k], 12, lam=1.6).solve(data[k][0], data[k][1])
        sl = slice(off[k], off[k + 1])
        assert err(phi[sl], ref[0]) <= TOL["fp64"] and err(field[sl], ref[1]) <= TOL["fp64"], k


def test_wire_plan_file_and_adjoint_modes(ps, tmp_path):
    """A reloaded wire plan gives bitwise the same sums; the physical gradient
    mode works."""
    x, q = W.uniform_box(800, np.array(BOX), charges="gauss", seed=176)
    pl = ps.Plan(BOX, 10, lam=1.6, precision="fp32", n_max=800, periodic="x")
    X, Q = dev(x.T), dev(q)
    phi0, field0 = pl.eval(X, Q)
    pl.status()
    path = tmp_path / "wire.plan"
    pl.save(path)
    pl2 = ps.Plan.load(path)
    assert pl2.info()["periodic"] == 1
    phi1, field1 = pl2.eval(X, Q)
    pl2.status()
    assert torch.equal(phi0, phi1) and torch.equal(field0, field1)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=False)
    f = field0.cpu().numpy()
    assert np.allclose(gx.cpu().numpy(), -q[None, :] * f, rtol=0, atol=1e-12 * np.abs(f).max())
    del e


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_wire_full_size_workload(ps, prec):
    """The benchmark's wire workload (N = 100,000, p = 16, lambda = 1.5, the
    default launch shape it times): 2,000 sampled particles against the oracle's
    stored values (tests/golden/ref_wire.npz), near-set size exact."""
    from gpu_common import golden
    c = W.config_partial("x")
    ref = golden("ref_wire.npz")
    pl, phi, field = _wire(ps, c["box"], c["p"], c["x"], c["q"], prec, lam=c["lam"])
    sub = ref["subset"]
    assert pl.info()["n_near_last"] == int(ref["n_near"])
    assert err(phi[sub], ref["phi"]) <= TOL[prec] and err(field[sub], ref["field"]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wire_exact_adjoint_matches_oracle(ps, prec):
    """The exact energy gradient with the decay rows: a charge and a dipole at each
    decay point join psi (k_adj_decay_src, k_adj_decay), against the oracle's
    gradient (oracle/adjoint.py, pinned to finite differences)."""
    from oracle.adjoint import energy_gradients_decay
    x, q = W.uniform_box(700, np.array(BOX), charges="gauss", seed=77)
    E, dx, dq = energy_gradients_decay(WirePlan(np.array(BOX), 12, lam=1.6), x, q)
    pl = ps.Plan(BOX, 12, lam=1.6, precision=prec, n_max=len(q), periodic="x")
    X, Q = dev(x.T), dev(q)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=True)
    pl.status()
    assert abs(float(e.item()) / E - 1) <= TOL[prec]
    assert err(gx.cpu().numpy().T, dx) <= TOL[prec] and err(gq.cpu().numpy(), dq) <= TOL[prec]
