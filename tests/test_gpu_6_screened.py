"""The screened Coulomb kernel exp(-kappa r)/r (one of the paper's "other
kernels", Sec. 1) with the kernel-at-centres basis of eq. (5): the HIP path
against the oracle's screened method (oracle/screened.py), whose own pins tie
it to an Ewald-type split and brute-force lattice sums.

Bars (tests/gpu_common.py): FP64 <= 1e-12, FP32 pairs with FP64 accumulation
<= 1e-6, on the relative L2 error and on the worst element; near-set sizes exact.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import TOL, dev, err, load_ps, rel
from oracle.screened import EwaldScreened, ScreenedPlan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOX = np.array([1.0, 1.2, 0.8])
R0 = 0.5 * float(np.linalg.norm(BOX))


@pytest.fixture(scope="module")
def ps():
    return load_ps()


def _centres(M=256, lam=1.5, r0=R0):
    return W.thomson_points(M, lam * r0)


def _solve(ps, box, p, x, q, prec, kappa, cen, lam=1.5, targets=None):
    pl = ps.Plan(box, p, lam=lam, precision=prec, n_max=len(q), m_max=0 if targets is None else len(targets),
                 centres=cen, kernel="screened", kappa=kappa)
    phi, field = pl.eval(dev(x.T), dev(q), targets=None if targets is None else dev(targets.T))
    pl.status()
    return pl, phi.cpu().numpy(), field.cpu().numpy().T


def test_screened_tables_match_oracle(ps):
    cen = _centres()
    for kappa in (0.7, 3.0):
        op = ScreenedPlan(BOX, kappa, cen, 16, lam=1.5)
        pl = ps.Plan(BOX, 16, lam=1.5, n_max=10, centres=cen, kernel="screened", kappa=kappa)
        inf = pl.info()
        assert inf["kernel"] == 1 and inf["kappa"] == kappa
        assert inf["P"] == 257 and inf["rank"] == op.rank == 256 and abs(inf["cond"] / op.cond - 1) < 1e-8
        yc, yt, pinv, bm = (t.numpy() for t in pl.tables())
        np.testing.assert_allclose(yc, op.yc, atol=4e-15 * R0)
        np.testing.assert_allclose(yt, op.yt, atol=4e-15 * R0)
        # two FP64 pseudo-inverses of a matrix with cond ~ 1e4: entries agree to ~cond x 1e-16
        assert rel(pinv, op.Apinv) < 1e-11
        assert np.all(bm == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kappa", [0.7, 3.0, 9.0])
def test_screened_matches_oracle(ps, prec, kappa):
    """Gaussian charges with a net charge (allowed for this kernel)."""
    x, q = W.uniform_box(2000, BOX, charges="gauss", seed=91)
    q = q + 0.05
    cen = _centres()
    ref = ScreenedPlan(BOX, kappa, cen, 16, lam=1.5).solve(x, q, return_parts=True)
    pl, phi, field = _solve(ps, BOX, 16, x, q, prec, kappa, cen)
    e1, e2 = err(phi, ref["phi"]), err(field, ref["field"])
    print(prec, kappa, "screened err phi %.3e field %.3e" % (e1, e2))
    assert pl.info()["n_near_last"] == ref["n_near"]
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_screened_separate_targets_and_coincident_points(ps, prec):
    """Separate targets, some placed exactly on particles (K(0) = 0 there)."""
    x, q = W.uniform_box(1200, BOX, charges="gauss", seed=92)
    g = np.random.default_rng(93)
    y = (g.random((300, 3)) - 0.5) * BOX
    y[:40] = x[:40]
    cen = _centres()
    ref = ScreenedPlan(BOX, 2.0, cen, 16, lam=1.5).solve(x, q, targets=y)
    _, phi, field = _solve(ps, BOX, 16, x, q, prec, 2.0, cen, targets=y)
    assert err(phi, ref[0]) <= TOL[prec] and err(field, ref[1]) <= TOL[prec]


def test_screened_method_accuracy_against_the_split(ps):
    """Method accuracy of the FP32 library at M = 400 centres, p = 20: the
    independent split to 3e-6 (the oracle's own method error at these
    parameters is 1.2e-6 / 2.0e-6, tests/test_oracle_screened.py)."""
    x, q = W.uniform_box(300, BOX, charges="gauss", seed=5)
    q = q + 0.1
    ref = EwaldScreened(BOX, 2.0).solve(x, q)
    _, phi, field = _solve(ps, BOX, 20, x, q, "fp32", 2.0, _centres(400))
    assert rel(phi, ref[0]) < 3e-6 and rel(field, ref[1]) < 3e-6


def test_screened_batch_matches_oracle_per_system(ps):
    """One graph launch over three boxes of different shapes and sizes (FP32)."""
    boxes = [BOX, np.array([1.1, 1.0, 1.3]), np.array([1.0, 1.5, 0.6])]
    ns = [900, 700, 500]
    data = [W.uniform_box(n, b, charges="gauss", seed=95 + k) for k, (n, b) in enumerate(zip(ns, boxes))]
    cens = [_centres(256, 1.5, 0.5 * float(np.linalg.norm(b))) for b in boxes]
    bp = ps.BatchedPlan([dict(box=b, n_max=n, centres=c) for b, n, c in zip(boxes, ns, cens)], p=16, lam=1.5,
                        precision="fp32", kernel="screened", kappa=2.5)
    off = np.concatenate([[0], np.cumsum(ns)])
    phi, field = bp.eval(dev(np.concatenate([d[0] for d in data]).T), dev(np.concatenate([d[1] for d in data])), off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    for k in range(3):
        ref = ScreenedPlan(boxes[k], 2.5, cens[k], 16, lam=1.5).solve(data[k][0], data[k][1])
        sl = slice(off[k], off[k + 1])
        assert err(phi[sl], ref[0]) <= TOL["fp32"] and err(field[sl], ref[1]) <= TOL["fp32"], k


def test_screened_plan_file_and_gradients(ps, tmp_path):
    """A reloaded plan gives bitwise the same sums; the physical gradient is
    -q field and phi (no projection: any charges)."""
    x, q = W.uniform_box(800, BOX, charges="gauss", seed=97)
    q = q + 0.2
    cen = _centres()
    pl = ps.Plan(BOX, 16, lam=1.5, precision="fp32", n_max=800, centres=cen, kernel="screened", kappa=2.0)
    X, Q = dev(x.T), dev(q)
    phi0, field0 = pl.eval(X, Q)
    pl.status()
    path = tmp_path / "screened.plan"
    pl.save(path)
    pl2 = ps.Plan.load(path)
    assert pl2.info()["kernel"] == 1 and pl2.info()["kappa"] == 2.0
    phi1, field1 = pl2.eval(X, Q)
    pl2.status()
    assert torch.equal(phi0, phi1) and torch.equal(field0, field1)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=False)
    f = field0.cpu().numpy()
    assert np.allclose(gx.cpu().numpy(), -q[None, :] * f, rtol=0, atol=1e-12 * np.abs(f).max())
    assert np.allclose(gq.cpu().numpy(), phi0.cpu().numpy(), rtol=0, atol=1e-12 * np.abs(phi0.cpu().numpy()).max())
    assert abs(float(e.item()) - 0.5 * float(q @ phi0.cpu().numpy())) < 1e-10 * abs(float(e.item()))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_screened_exact_adjoint_matches_oracle(ps, prec):
    """The exact gradient of the screened method's energy (moments at the centres,
    check-point charges w = (A^+)^T u, psi over the near images) against the
    oracle's, itself pinned to finite differences; no projection of dE/dq."""
    from oracle.screened import energy_gradients_screened
    x, q = W.uniform_box(900, BOX, charges="gauss", seed=98)
    q = q + 0.1
    cen = _centres()
    E, dx, dq = energy_gradients_screened(ScreenedPlan(BOX, 2.0, cen, 16, lam=1.5), x, q)
    pl = ps.Plan(BOX, 16, lam=1.5, precision=prec, n_max=len(q), centres=cen, kernel="screened", kappa=2.0)
    X, Q = dev(x.T), dev(q)
    e = pl.energy(X, Q)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(X, Q, one, exact=True)
    pl.status()
    assert abs(float(e.item()) / E - 1) <= TOL[prec]
    assert err(gx.cpu().numpy().T, dx) <= TOL[prec] and err(gq.cpu().numpy(), dq) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_screened_full_size_workload(ps, prec):
    """The benchmark's screened workload (N = 100,000, kappa = 2, 256 centres,
    p = 16, the default launch shape it times): 2,000 sampled particles against
    the oracle's stored values (tests/golden/ref_screened.npz), near-set size exact."""
    from gpu_common import golden
    c = W.config_screened()
    ref = golden("ref_screened.npz")
    pl, phi, field = _solve(ps, c["box"], c["p"], c["x"], c["q"], prec, c["kappa"], c["centres"], lam=c["lam"])
    sub = ref["subset"]
    assert pl.info()["n_near_last"] == int(ref["n_near"])
    assert err(phi[sub], ref["phi"]) <= TOL[prec] and err(field[sub], ref["field"]) <= TOL[prec]
