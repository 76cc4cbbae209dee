"""Periodization along x and y only (a slab, z free; Sec. 1, closing paragraph):
the HIP path against the oracle's slab method (oracle/slab.py), which its own
pins tie to an independent slab Ewald sum and to brute-force lattice sums.

Bars (tests/gpu_common.py): FP64 <= 1e-12, FP32 pairs with FP64 accumulation
<= 1e-6, on the relative L2 error and on the worst element; near-set sizes exact.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import TOL, dev, err, load_ps, rel
from oracle.ewald2d import Ewald2D
from oracle.slab import SlabPlan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOX = (1.0, 1.2, 0.8)


@pytest.fixture(scope="module")
def ps():
    return load_ps()


def _slab(ps, box, p, x, q, prec, lam=1.6, **kw):
    pl = ps.Plan(box, p, lam=lam, precision=prec, n_max=len(q), periodic="xy", **kw)
    phi, field = pl.eval(dev(x.T), dev(q))
    pl.status()
    return pl, phi.cpu().numpy(), field.cpu().numpy().T


def test_slab_tables_match_oracle(ps):
    """Check points kept (those an in-plane shift moves into S0), partners along x
    or y only, the pseudo-inverse of the fit with its decay rows, box means."""
    for box, p in ((BOX, 12), ((1.0, 1.0, 0.3), 10), ((2.0, 1.0, 0.7), 9)):
        op = SlabPlan(box, p, lam=1.6)
        pl = ps.Plan(box, p, lam=1.6, n_max=10, periodic="xy")
        inf = pl.info()
        assert inf["periodic"] == 3 and inf["L"] == op.L and inf["n_rows"] == op.A.shape[0]
        assert inf["rank"] == op.rank and abs(inf["cond"] / op.cond - 1) < 1e-9
        yc, yt, pinv, bm = (t.numpy() for t in pl.tables())
        np.testing.assert_allclose(yc, op.yc, atol=4e-15 * op.R0)
        np.testing.assert_allclose(yt, op.yt, atol=4e-15 * op.R0)
        assert err(pinv, op.Apinv) < 1e-11
        np.testing.assert_allclose(bm, op.R0mean, atol=1e-14)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_slab_matches_oracle(ps, prec):
    x, q = W.uniform_box(2000, np.array(BOX), charges="gauss", seed=71)
    ref = SlabPlan(BOX, 16, lam=1.6).solve(x, q, return_parts=True)
    pl, phi, field = _slab(ps, BOX, 16, x, q, prec)
    e1, e2 = err(phi, ref["phi"]), err(field, ref["field"])
    print(prec, "slab err phi %.3e field %.3e" % (e1, e2))
    assert pl.info()["n_near_last"] == ref["n_near"]
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


@pytest.mark.parametrize("box", [(1.0, 1.0, 0.3), (1.0, 1.0, 2.0), (2.0, 1.0, 0.7)])
def test_slab_thin_thick_and_elongated_cells(ps, box):
    x, q = W.uniform_box(1500, np.array(box), charges="gauss", seed=72)
    ref = SlabPlan(box, 12, lam=1.6).solve(x, q)
    _, phi, field = _slab(ps, box, 12, x, q, "fp64")
    assert err(phi, ref[0]) <= TOL["fp64"] and err(field, ref[1]) <= TOL["fp64"]


def test_slab_against_the_slab_ewald_sum(ps):
    """Method accuracy at p = 20: the library's FP32 slab solve against the
    independent slab Ewald sum (fields; potentials up to the constant, which
    the two sides fix by different conventions)."""
    x, q = W.uniform_box(300, np.array(BOX), charges="gauss", seed=73)
    pe, fe = Ewald2D(BOX).solve(x, q)
    _, phi, field = _slab(ps, BOX, 20, x, q, "fp32")
    d = phi - pe
    assert rel(field, fe) < 2e-6
    assert np.linalg.norm(d - d.mean()) / np.linalg.norm(pe - pe.mean()) < 4e-6


def test_batch_of_slab_and_three_axis_systems(ps):
    """One graph launch over a slab box and two triply periodic boxes: each system
    matches its own oracle (FP64)."""
    boxes = [np.array(BOX), np.array([1.1, 1.0, 1.3]), np.array([1.0, 1.5, 0.6])]
    per = ["xy", "xyz", "xy"]
    ns = [900, 700, 500]
    data = [W.uniform_box(n, b, charges="gauss", seed=80 + k) for k, (n, b) in enumerate(zip(ns, boxes))]
    bp = ps.BatchedPlan([dict(box=b, n_max=n, periodic=s) for b, n, s in zip(boxes, ns, per)], p=12, lam=1.6,
                        precision="fp64")
    off = np.concatenate([[0], np.cumsum(ns)])
    phi, field = bp.eval(dev(np.concatenate([d[0] for d in data]).T), dev(np.concatenate([d[1] for d in data])), off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    from oracle.method import Plan as OPlan
    for k in range(3):
        op = SlabPlan(boxes[k], 12, lam=1.6) if per[k] == "xy" else OPlan(boxes[k], 12, lam=1.6)
        ref = op.solve(data[k][0], data[k][1])
        sl = slice(off[k], off[k + 1])
        assert err(phi[sl], ref[0]) <= TOL["fp64"] and err(field[sl], ref[1]) <= TOL["fp64"], k


def test_slab_plan_file_and_adjoint_modes(ps, tmp_path):
    """A reloaded slab plan gives bitwise the same sums; the physical gradient
    mode works."""
    x, q = W.uniform_box(800, np.array(BOX), charges="gauss", seed=74)
    pl = ps.Plan(BOX, 10, lam=1.6, precision="fp32", n_max=800, periodic="xy")
    X, Q = dev(x.T), dev(q)
    phi0, field0 = pl.eval(X, Q)
    pl.status()
    path = tmp_path / "slab.plan"
    pl.save(path)
    pl2 = ps.Plan.load(path)
    assert pl2.info()["periodic"] == 3
    phi1, field1 = pl2.eval(X, Q)
    pl2.status()
    assert torch.equal(phi0, phi1) and torch.equal(field0, field1)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=False)
    assert np.allclose(gx.cpu().numpy(), -q[None, :] * field0.cpu().numpy(), rtol=0, atol=1e-12 * np.abs(field0.cpu().numpy()).max())
    del e


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_slab_full_size_workload(ps, prec):
    """The benchmark's slab workload (N = 100,000, p = 16, lambda = 1.5, the
    default launch shape it times): 2,000 sampled particles against the oracle's
    stored values (tests/golden/ref_slab.npz), near-set size exact."""
    from gpu_common import golden
    c = W.config_partial("xy")
    ref = golden("ref_slab.npz")
    pl, phi, field = _slab(ps, c["box"], c["p"], c["x"], c["q"], prec, lam=c["lam"])
    sub = ref["subset"]
    assert pl.info()["n_near_last"] == int(ref["n_near"])
    assert err(phi[sub], ref["phi"]) <= TOL[prec] and err(field[sub], ref["field"]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_slab_exact_adjoint_matches_oracle(ps, prec):
    """The exact energy gradient with the decay rows: a charge and a dipole at each
    decay point join psi (k_adj_decay_src, k_adj_decay), against the oracle's
    gradient (oracle/adjoint.py, pinned to finite differences)."""
    from oracle.adjoint import energy_gradients_decay
    x, q = W.uniform_box(700, np.array(BOX), charges="gauss", seed=77)
    E, dx, dq = energy_gradients_decay(SlabPlan(np.array(BOX), 12, lam=1.6), x, q)
    pl = ps.Plan(BOX, 12, lam=1.6, precision=prec, n_max=len(q), periodic="xy")
    X, Q = dev(x.T), dev(q)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=True)
    pl.status()
    assert abs(float(e.item()) / E - 1) <= TOL[prec]
    assert err(gx.cpu().numpy().T, dx) <= TOL[prec] and err(gq.cpu().numpy(), dq) <= TOL[prec]
