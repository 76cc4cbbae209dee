"""Edge cases of the variants (slab, wire, the plane, the screened kernel):
ragged particle counts across launch shapes, one plan across counts, zero
charges, and nearly coincident pairs in the plane, each against its oracle
(oracle/slab.py, oracle/wire.py, oracle/twod.py, oracle/screened.py).

Bars (tests/gpu_common.py): FP64 <= 1e-12, FP32 <= 1e-6, on the relative L2
error and on the worst element.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import TOL, dev, err, load_ps
from oracle.screened import ScreenedPlan
from oracle.slab import SlabPlan
from oracle.twod import Plan2D
from oracle.wire import WirePlan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOX3 = (1.0, 1.1, 0.9)
BOX2 = (1.0, 1.3)


@pytest.fixture(scope="module")
def ps():
    return load_ps()


def _cell(n, seed, box):
    g = np.random.default_rng(seed)
    x = (g.random((n, len(box))) - 0.5) * np.array(box)
    q = g.standard_normal(n)
    return x, q - q.mean()


def _variant(ps, kind, n, prec, bt=0, split=0, seed=0):
    """(oracle plan, library plan, positions, charges) of one variant case."""
    if kind == "plane":
        x, q = _cell(n, seed, BOX2)
        if n == 2:
            x, q = np.array([[0.3, 0.1], [-0.05, 0.02]]), np.array([1.0, -1.0])
        return (Plan2D(BOX2, 24, lam=1.5),
                ps.Plan(BOX2, 24, lam=1.5, precision=prec, n_max=n, dim=2, tile_targets=bt, n_split=split), x, q)
    x, q = _cell(n, seed, BOX3)
    if n == 2:
        x, q = np.array([[0.1, 0.2, -0.3], [-0.25, 0.05, 0.4]]), np.array([1.0, -1.0])
    if kind == "slab":
        return (SlabPlan(BOX3, 10, lam=1.6),
                ps.Plan(BOX3, 10, lam=1.6, precision=prec, n_max=n, periodic="xy", tile_targets=bt, n_split=split),
                x, q)
    if kind == "wire":
        return (WirePlan(np.array(BOX3), 10, lam=1.6),
                ps.Plan(BOX3, 10, lam=1.6, precision=prec, n_max=n, periodic="x", tile_targets=bt, n_split=split),
                x, q)
    cen = W.thomson_points(128, 1.5 * 0.5 * float(np.linalg.norm(BOX3)))
    q = q + 0.3                                        # a net charge: the screened kernel takes any charges
    return (ScreenedPlan(BOX3, 2.0, cen, 10, lam=1.6),
            ps.Plan(BOX3, 10, lam=1.6, precision=prec, n_max=n, centres=cen, kernel="screened", kappa=2.0,
                    tile_targets=bt, n_split=split), x, q)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["slab", "wire", "plane", "screened"])
@pytest.mark.parametrize("n,bt,split", [(2, 0, 0), (63, 64, 0), (257, 128, 3), (1025, 256, 1)])
def test_ragged_sizes_and_launch_shapes(ps, kind, prec, n, bt, split):
    op, pl, x, q = _variant(ps, kind, n, prec, bt, split, seed=300 + n)
    ref = op.solve(x, q)
    phi, field = pl.eval(dev(x.T), dev(q))
    pl.status()
    assert err(phi.cpu().numpy(), ref[0]) <= TOL[prec]
    assert err(field.cpu().numpy().T, ref[1]) <= TOL[prec]


@pytest.mark.parametrize("kind", ["slab", "wire", "plane"])
def test_one_plan_across_counts_and_zero_charges(ps, kind):
    """One FP32 plan serves 1,500, 400 and 1,500 particles in turn (the work
    tables are rebuilt per count), then all-zero charges, which give exactly
    zero potential and field."""
    op, pl, _, _ = _variant(ps, kind, 1500, "fp32", seed=1)
    for n, seed in ((1500, 401), (400, 402), (1500, 401)):
        x, q = _cell(n, seed, BOX2 if kind == "plane" else BOX3)
        ref = op.solve(x, q)
        phi, field = pl.eval(dev(x.T), dev(q))
        pl.status()
        assert err(phi.cpu().numpy(), ref[0]) <= TOL["fp32"], n
        assert err(field.cpu().numpy().T, ref[1]) <= TOL["fp32"], n
    phi, field = pl.eval(dev(x.T), dev(np.zeros(len(x))))
    pl.status()
    assert not torch.any(phi != 0) and not torch.any(field != 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plane_nearly_coincident_pairs(ps, prec):
    """Pairs of charges 1e-4 .. 1e-7 apart in the plane: -log r reaches 16 and the
    pairs' mutual field dominates the field norm; the FP32 path's two-float
    relative coordinates keep both within the FP32 bar."""
    g = np.random.default_rng(24)
    x, q = _cell(1500, 24, BOX2)
    pairs = []
    for sep in np.logspace(-4, -7, 40):
        c = g.uniform(-0.45, 0.45, size=2) * np.array(BOX2)
        u = g.standard_normal(2)
        u /= np.linalg.norm(u)
        pairs += [c, c + sep * u]
    xp = np.array(pairs)
    m = g.uniform(0.5, 1.5, size=len(xp) // 2)
    X = np.concatenate([x, xp])
    Q = np.concatenate([q, np.stack([m, -m], axis=1).ravel()])
    Q -= Q.mean()
    ref = Plan2D(BOX2, 24, lam=1.5).solve(X, Q)
    pl = ps.Plan(BOX2, 24, lam=1.5, precision=prec, n_max=len(Q), dim=2)
    phi, field = pl.eval(dev(X.T), dev(Q))
    pl.status()
    assert err(phi.cpu().numpy(), ref[0]) <= TOL[prec]
    assert err(field.cpu().numpy().T, ref[1]) <= TOL[prec]


def test_plane_fp32_error_follows_the_cancellation(ps):
    """A +-1 pair in the 1 x 1.3 cell whose separation lies near a symmetry point of
    the lattice: the periodic field at the particles is over 50 times smaller than
    the sum of the magnitudes of the near entries' contributions.  FP32 rounds
    each contribution to about 1e-7 of itself, so relative to this field the FP32
    error is that cancellation factor kappa times larger: the bar here is
    1e-7 x kappa for the FP32 field, the usual bars otherwise."""
    x, q = np.array([[0.1, 0.2], [-0.3, -0.45]]), np.array([1.0, -1.0])
    op = Plan2D(BOX2, 24, lam=1.5)
    ref = op.solve(x, q)
    xs, qs, _, _ = op.near(x, q)
    mag = []
    for i in range(2):
        d = x[i] - xs
        r2 = (d * d).sum(1)
        live = r2 > 0
        mag.append(np.sum(np.abs(qs[live]) / np.sqrt(r2[live])))
    kappa = max(mag) / np.abs(ref[1]).max()
    assert kappa > 50
    for prec, bar in (("fp64", TOL["fp64"]), ("fp32", 1e-7 * kappa)):
        pl = ps.Plan(BOX2, 24, lam=1.5, precision=prec, n_max=2, dim=2)
        phi, field = pl.eval(dev(x.T), dev(q))
        pl.status()
        e = err(field.cpu().numpy().T, ref[1])
        print(prec, "cancellation %.1f, field error %.3e" % (kappa, e))
        assert e <= bar and err(phi.cpu().numpy(), ref[0]) <= TOL[prec]
