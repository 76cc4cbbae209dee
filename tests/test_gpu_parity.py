"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: FP64 path rel-L2 <= 1e-12 for the potential and the field; FP32 path
(FP32 pair arithmetic, FP64 accumulation) rel-L2 <= 1e-6.  Integer work (the
near-set size) must match exactly.  Sizes span several tiles and ragged tails.
"""
import numpy as np
import pytest

import workloads as W
from oracle.adjoint import energy_gradients, physics_gradients
from oracle.method import Plan as OPlan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_4374_amd as m
    m.lib()
    return m


def _run(ps, box, p, x, q, prec, R_b=None, lam=None, targets=None, **kw):
    pl = ps.Plan(box, p, R_b=R_b, lam=lam, precision=prec, n_max=len(q),
                 m_max=0 if targets is None else len(targets), **kw)
    phi, field = pl.eval(_dev(x.T), _dev(q), targets=None if targets is None else _dev(targets.T))
    pl.status()
    return pl, phi.cpu().numpy(), field.cpu().numpy().T


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_cube_config(ps, prec):
    """Cube 1^3, N=1000 uniform, q=+-1, p=12, R_b=1.5 (the small workload)."""
    c = W.config1()
    op = OPlan(c["box"], c["p"], R_b=c["R_b"])
    ref = op.solve(c["x"], c["q"], return_parts=True)
    pl, phi, field = _run(ps, c["box"], c["p"], c["x"], c["q"], prec, R_b=c["R_b"])
    print(prec, "rel-L2 phi %.3e field %.3e" % (_rel(phi, ref["phi"]), _rel(field, ref["field"])))
    assert _rel(phi, ref["phi"]) <= TOL[prec]
    assert _rel(field, ref["field"]) <= TOL[prec]
    info = pl.info()
    assert info["n_near_last"] == ref["n_near"]
    assert info["L"] == 2 * c["p"] ** 2 - c["p"] and info["rank"] == c["p"] ** 2 - 1
    assert info["mean_corners"] == 0  # 16 waves of 64 particles: the per-entry box mean
    # FP64: the coefficients to rounding; FP32: the check-point sums are FP32 pair
    # sums (FP64 accumulation), which moves C by ~1e-6 relative
    C = pl.coefficients().numpy()
    ctol = 1e-12 if prec == "fp64" else 2e-5
    assert _rel(C[1:], ref["C"][1:]) < ctol
    assert abs(C[0] - ref["C"][0]) < ctol * max(1.0, abs(ref["C"][0]))


def test_plan_tables_match_oracle(ps):
    for box, p, kw in [((1, 1, 1), 12, dict(R_b=1.5)), ((1, 1, 2.5), 20, dict(lam=1.5)), ((1.3, 1.9, 1.1), 9, dict(lam=1.7))]:
        pl = ps.Plan(box, p, n_max=10, **kw)
        op = OPlan(box, p, R_b=kw.get("R_b"), lam=kw.get("lam"))
        yc, yt, pinv, bm = (t.numpy() for t in pl.tables())
        np.testing.assert_allclose(yc, op.yc, atol=1e-15 * op.R0 * 4)
        np.testing.assert_allclose(yt, op.yt, atol=1e-15 * op.R0 * 4)
        assert _rel(pinv, op.Apinv) < 1e-12
        np.testing.assert_allclose(bm, op.R0mean, atol=1e-14)
        inf = pl.info()
        assert inf["rank"] == op.rank and abs(inf["cond"] / op.cond - 1) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("box,lam,p,n", [((1.0, 1.3, 2.1), 1.73, 10, 700), ((2.0, 1.0, 1.0), 1.5, 12, 1500)])
def test_non_cubic_boxes(ps, prec, box, lam, p, n):
    x, q = W.uniform_box(n, box, charges="gauss", seed=n)
    ref = OPlan(box, p, lam=lam).solve(x, q)
    _, phi, field = _run(ps, box, p, x, q, prec, lam=lam)
    assert _rel(phi, ref[0]) <= TOL[prec]
    assert _rel(field, ref[1]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,bt,split", [(2, 0, 0), (63, 64, 0), (257, 128, 3), (1025, 256, 1), (3001, 64, 0)])
def test_ragged_sizes_and_launch_shapes(ps, prec, n, bt, split):
    box = (1.0, 1.0, 1.0)
    if n == 2:
        x = np.array([[0.1, 0.2, -0.3], [-0.25, 0.05, 0.4]])
        q = np.array([1.0, -1.0])
    else:
        x, q = W.uniform_box(n, box, charges="gauss", seed=n)
    ref = OPlan(box, 8, R_b=1.5).solve(x, q)
    _, phi, field = _run(ps, box, 8, x, q, prec, R_b=1.5, tile_targets=bt, n_split=split)
    assert _rel(phi, ref[0]) <= TOL[prec]
    assert _rel(field, ref[1]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_plan_across_particle_counts(ps, prec):
    """One plan (n_max = 3,000) serves evals of 3,000, 500 and 2,000 particles in
    turn and then 3,000 again: the per-shape work tables are rebuilt for each
    count, and every result meets the bar.  Some particles sit exactly on the
    lower faces x_k = -d_k/2, which belong to the box (Sec. 1)."""
    box = (1.0, 1.1, 0.9)
    pl = ps.Plan(box, 10, lam=1.6, precision=prec, n_max=3000)
    for n, seed in ((3000, 31), (500, 32), (2000, 33), (3000, 31)):
        x, q = W.uniform_box(n, box, charges="gauss", seed=seed)
        for k in range(3):
            x[5 * k:5 * k + 5, k] = -0.5 * box[k]
        ref = OPlan(box, 10, lam=1.6).solve(x, q)
        phi, field = pl.eval(_dev(x.T), _dev(q))
        pl.status()
        assert _rel(phi.cpu().numpy(), ref[0]) <= TOL[prec], n
        assert _rel(field.cpu().numpy().T, ref[1]) <= TOL[prec], n


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_separate_targets_and_coincident_points(ps, prec):
    """M evaluation points in the box (Sec. 1); targets placed exactly on
    particles take K(0) = 0 for that pair."""
    box = (1.0, 1.2, 0.9)
    x, q = W.uniform_box(500, box, charges="gauss", seed=3)
    g = np.random.default_rng(4)
    y = (g.random((300, 3)) - 0.5) * np.asarray(box)
    y[:20] = x[100:120]
    ref = OPlan(box, 10, lam=1.7).solve(x, q, targets=y)
    _, phi, field = _run(ps, box, 10, x, q, prec, lam=1.7, targets=y)
    assert _rel(phi, ref[0]) <= TOL[prec]
    assert _rel(field, ref[1]) <= TOL[prec]


def test_mean_none_shifts_by_constant(ps):
    c = W.config1()
    _, a, fa = _run(ps, c["box"], 10, c["x"], c["q"], "fp64", R_b=1.5)
    pl = ps.Plan(c["box"], 10, R_b=1.5, n_max=1000, mean="none")
    b, fb = pl.eval(_dev(c["x"].T), _dev(c["q"]))
    d = a - b.cpu().numpy()
    assert np.ptp(d) < 1e-12 * np.abs(a).max()
    np.testing.assert_array_equal(fa, fb.cpu().numpy().T)
    assert pl.coefficients().numpy()[0] == 0.0


def test_rocksalt_madelung(ps):
    """Unjittered rock-salt lattice (32^3 sites, spacing 1/32, p = 16, R_b = 1.5):
    the potential at the sites equals the oracle's (which, like the method,
    carries the truncation error at these parameters), all sites are
    equivalent up to that error, and phi * spacing approaches -q M (eq. (st1))."""
    from oracle.ewald import MADELUNG_NACL
    r = W.rocksalt(32)
    ref = _golden("ref_cfg5.npz")
    _, phi, field = _run(ps, r["box"], 16, r["x"], r["q"], "fp64", R_b=1.5)
    np.testing.assert_allclose(phi[:2], ref["lattice_phi"], rtol=1e-12)
    err = np.abs(phi * r["spacing"] / (-r["q"] * MADELUNG_NACL) - 1)
    print("Madelung max rel err %.3e (oracle %.3e)" % (err.max(), np.abs(ref["lattice_phi"] * r["spacing"] / (-ref["lattice_q"] * MADELUNG_NACL) - 1).max()))
    assert err.max() < 2e-4
    # the sites are physically equivalent; the method's truncation error varies
    # with the position in the box, so their spread is at that error's level
    assert np.ptp(phi * r["spacing"] * r["q"]) < 4e-4 * MADELUNG_NACL


def test_status_reports_data_errors(ps):
    from paper_1310_4374_amd import PeriodicSumError
    c = W.config1()
    pl = ps.Plan(c["box"], 8, R_b=1.5, n_max=1000)
    q = c["q"].copy()
    q[0] += 0.5
    pl.eval(_dev(c["x"].T), _dev(q))
    with pytest.raises(PeriodicSumError, match="NOT_NEUTRAL"):
        pl.status()
    x = c["x"].copy()
    x[5, 1] = 0.5  # upper face is outside the half-open box
    pl.eval(_dev(x.T), _dev(c["q"]))
    with pytest.raises(PeriodicSumError, match="OUT_OF_BOX"):
        pl.status()
    # a NaN coordinate or charge is reported the same way (every index the
    # kernels form comes from counts, and the cell key clamps NaN to cell 0)
    x = c["x"].copy()
    x[11, 2] = np.nan
    pl.eval(_dev(x.T), _dev(c["q"]))
    with pytest.raises(PeriodicSumError, match="OUT_OF_BOX"):
        pl.status()
    q = c["q"].copy()
    q[3] = np.nan
    pl.eval(_dev(c["x"].T), _dev(q))
    with pytest.raises(PeriodicSumError, match="OUT_OF_BOX"):
        pl.status()
    pl.eval(_dev(c["x"].T), _dev(c["q"]))
    pl.status()
    with pytest.raises(PeriodicSumError, match="INVALID"):
        pl.eval(_dev(np.zeros((3, 2000))), _dev(np.zeros(2000)))
    # a near list that 32-bit entry indices cannot address is refused before allocation
    with pytest.raises(PeriodicSumError, match="UNSUPPORTED"):
        ps.Plan(c["box"], 4, R_b=1.5, n_max=2 ** 30)


def test_synchronous_validation(ps, monkeypatch):
    """With PS_VALIDATE set when a plan is made, eval itself reports the data
    errors (single and batched plans); without it, eval only enqueues and the
    error waits for status()."""
    from paper_1310_4374_amd import PeriodicSumError
    c = W.config1()
    x, q = _dev(c["x"].T), _dev(c["q"])
    q_bad = q.clone()
    q_bad[0] += 0.5
    monkeypatch.setenv("PS_VALIDATE", "1")
    pl = ps.Plan(c["box"], 8, R_b=1.5, n_max=1000)
    bp = ps.BatchedPlan([dict(box=c["box"], n_max=600), dict(box=c["box"], n_max=400)], p=8, R_b=1.5, precision="fp64")
    pl.eval(x, q)
    with pytest.raises(PeriodicSumError, match="NOT_NEUTRAL"):
        pl.eval(x, q_bad)
    pl.eval(x, q)
    x_out = x.clone()
    x_out[0, 7] = 0.5
    with pytest.raises(PeriodicSumError, match="OUT_OF_BOX"):
        pl.energy(x_out, q)
    # two neutral halves of the +-1 charges; then one of them made non-neutral
    order = np.argsort(c["q"], kind="stable")
    idx = np.concatenate([order[:300], order[-300:], order[300:500], order[-500:-300]])
    xb, qb = x[:, torch.tensor(idx, device="cuda:0")].contiguous(), q[torch.tensor(idx, device="cuda:0")].contiguous()
    bp.eval(xb, qb, [0, 600, 1000])
    qb[600] = 0.0
    with pytest.raises(PeriodicSumError, match="NOT_NEUTRAL"):
        bp.eval(xb, qb, [0, 600, 1000])
    monkeypatch.setenv("PS_VALIDATE", "0")
    pl2 = ps.Plan(c["box"], 8, R_b=1.5, n_max=1000)
    pl2.eval(x, q_bad)
    with pytest.raises(PeriodicSumError, match="NOT_NEUTRAL"):
        pl2.status()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_charges_give_zero(ps, prec):
    """Degenerate input: all charges zero (neutral).  Every stage sums zeros, so
    the potential and the field are exactly zero, in a single plan and in a
    batch next to an ordinary box (which still matches the oracle)."""
    x, _ = W.uniform_box(777, (1.0, 1.2, 0.9), charges="gauss", seed=71)
    z = np.zeros(777)
    pl = ps.Plan((1.0, 1.2, 0.9), 10, lam=1.6, precision=prec, n_max=777)
    phi, field = pl.eval(_dev(x.T), _dev(z))
    pl.status()
    assert not torch.any(phi != 0) and not torch.any(field != 0)
    x2, q2 = W.uniform_box(500, (1.1, 1.0, 1.3), charges="gauss", seed=72)
    bp = ps.BatchedPlan([dict(box=(1.0, 1.2, 0.9), n_max=777), dict(box=(1.1, 1.0, 1.3), n_max=500)], p=10, lam=1.6,
                        precision=prec)
    phi, field = bp.eval(_dev(np.concatenate([x, x2]).T), _dev(np.concatenate([z, q2])), [0, 777, 1277])
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    assert not np.any(phi[:777]) and not np.any(field[:777])
    ref = OPlan((1.1, 1.0, 1.3), 10, lam=1.6).solve(x2, q2)
    assert _rel(phi[777:], ref[0]) <= TOL[prec] and _rel(field[777:], ref[1]) <= TOL[prec]


def test_bitwise_reproducible(ps):
    c = W.config1()
    for prec in ("fp64", "fp32"):
        pl = ps.Plan(c["box"], 12, R_b=1.5, n_max=1000, precision=prec)
        a = pl.eval(_dev(c["x"].T), _dev(c["q"]))
        b = pl.eval(_dev(c["x"].T), _dev(c["q"]))
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_independent_plans_on_two_streams(ps):
    """Two plans (one single box, one batch) evaluated concurrently on two
    default-priority streams, several rounds without synchronizing in between:
    plans share no device state, so every result equals the plan's own
    sequential eval bit for bit."""
    xa, qa = W.uniform_box(3000, (1.0, 1.1, 1.2), charges="gauss", seed=81)
    xb = [W.uniform_box(n, b, charges="gauss", seed=82 + k)
          for k, (n, b) in enumerate(zip((900, 1400), ((1.3, 1.0, 1.0), (1.0, 1.5, 1.2))))]
    pa = ps.Plan((1.0, 1.1, 1.2), 10, lam=1.6, precision="fp32", n_max=3000)
    pb = ps.BatchedPlan([dict(box=(1.3, 1.0, 1.0), n_max=900), dict(box=(1.0, 1.5, 1.2), n_max=1400)], p=10, lam=1.6,
                        precision="fp64")
    XA, QA = _dev(xa.T), _dev(qa)
    XB, QB = _dev(np.concatenate([d[0] for d in xb]).T), _dev(np.concatenate([d[1] for d in xb]))
    off = [0, 900, 2300]
    ref_a = [t.clone() for t in pa.eval(XA, QA)]
    ref_b = [t.clone() for t in pb.eval(XB, QB, off)]
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    sa.wait_stream(torch.cuda.current_stream())
    sb.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):
        with torch.cuda.stream(sa):
            oa = pa.eval(XA, QA)
        with torch.cuda.stream(sb):
            ob = pb.eval(XB, QB, off)
        outs.append((oa, ob))
    torch.cuda.synchronize()
    pa.status()
    pb.status()
    for oa, ob in outs:
        assert torch.equal(oa[0], ref_a[0]) and torch.equal(oa[1], ref_a[1])
        assert torch.equal(ob[0], ref_b[0]) and torch.equal(ob[1], ref_b[1])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_energy_and_exact_adjoint(ps, prec, tol):
    box = (1.0, 1.1, 0.9)
    x, q = W.uniform_box(800, box, charges="gauss", seed=12)
    op = OPlan(box, 10, lam=1.7)
    E, dx, dq, _ = energy_gradients(op, x, q)
    pl = ps.Plan(box, 10, lam=1.7, n_max=800, precision=prec)
    xt, qt = _dev(x.T), _dev(q)
    e = pl.energy(xt, qt)
    g = torch.full((1,), 2.0, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(xt, qt, g, exact=True)
    assert abs(float(e.cpu()[0]) - E) <= tol * abs(E)
    assert _rel(gx.cpu().numpy().T, 2 * dx) <= tol
    assert _rel(gq.cpu().numpy(), 2 * dq) <= tol
    px, pq = physics_gradients(op, x, q)
    hx, hq = pl.energy_vjp(xt, qt, g, exact=False)
    assert _rel(hx.cpu().numpy().T, 2 * px) <= tol
    assert _rel(hq.cpu().numpy(), 2 * pq) <= tol


def test_autograd_matches_finite_differences(ps):
    """The autograd.Function's backward (exact adjoint, FP64) against central
    differences h = 1e-5 of the library's own energy."""
    box = (1.0, 1.0, 1.0)
    x, q = W.uniform_box(400, box, charges="gauss", seed=21)
    pl = ps.Plan(box, 10, R_b=1.5, n_max=400)
    xt = _dev(x.T).requires_grad_(True)
    qt = _dev(q).requires_grad_(True)
    E = ps.PeriodicEnergy.apply(xt, qt, pl, True)
    E.backward()
    gx, gq = xt.grad.cpu().numpy(), qt.grad.cpu().numpy()
    h = 1e-5

    def energy(xx, qq):
        return float(pl.energy(_dev(xx.T), _dev(qq)).cpu()[0])

    from oracle.geometry import lattice_vectors
    P = lattice_vectors(box, 1.5)
    dist = np.abs(np.linalg.norm(x[:, None, :] + P[None], axis=2) - 1.5).min(1)
    for i in np.nonzero(dist > 1e-3)[0][:4]:
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (energy(xp, q) - energy(xm, q)) / (2 * h)
            assert abs(gx[k, i] - fd) < 1e-6 * max(1.0, abs(fd))
    for i, j in [(0, 1), (7, 300)]:
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qp[j] -= h
        qm[i] -= h
        qm[j] += h
        fd = (energy(x, qp) - energy(x, qm)) / (2 * h)
        assert abs((gq[i] - gq[j]) - fd) < 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_matches_oracle_and_single(ps, prec):
    g = np.random.default_rng(5)
    systems, xs, qs = [], [], []
    for k in range(7):
        box = g.uniform(1.0, 2.0, size=3)
        n = int(g.integers(50, 1500))
        x, q = W.uniform_box(n, box, charges="gauss", seed=100 + k)
        systems.append(dict(box=box, n_max=n))
        xs.append(x)
        qs.append(q)
    lam = float(np.sqrt(3))
    bp = ps.BatchedPlan(systems, p=10, lam=lam, precision=prec)
    off = np.concatenate([[0], np.cumsum([len(q) for q in qs])])
    X = np.concatenate(xs)
    Q = np.concatenate(qs)
    phi, field = bp.eval(_dev(X.T), _dev(Q), off)
    phi2, field2 = bp.eval(_dev(X.T), _dev(Q), off)   # second launch of the same graph
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    assert np.array_equal(phi, phi2.cpu().numpy())
    for k in range(7):
        sl = slice(off[k], off[k + 1])
        ref = OPlan(systems[k]["box"], 10, lam=lam).solve(xs[k], qs[k])
        assert _rel(phi[sl], ref[0]) <= TOL[prec]
        assert _rel(field[sl], ref[1]) <= TOL[prec]


def test_batched_plan_across_particle_counts(ps):
    """One batched plan evaluated with changing per-system particle counts
    (each within its n_max), then with the first counts again: the work tables
    and the captured graph are rebuilt for each shape, and every system matches
    the oracle (FP32 pairs, bar 1e-6)."""
    boxes = [(1.0, 1.0, 1.0), (1.5, 1.2, 1.0), (1.1, 1.9, 1.4)]
    n_max = [1200, 900, 1500]
    bp = ps.BatchedPlan([dict(box=b, n_max=m) for b, m in zip(boxes, n_max)], p=10, lam=1.7, precision="fp32")
    for counts in ((1200, 900, 1500), (300, 900, 40), (1200, 900, 1500)):
        xs, qs = [], []
        for k, n in enumerate(counts):
            x, q = W.uniform_box(n, boxes[k], charges="gauss", seed=200 + 10 * k + n % 7)
            xs.append(x)
            qs.append(q)
        off = np.concatenate([[0], np.cumsum(counts)])
        phi, field = bp.eval(_dev(np.concatenate(xs).T), _dev(np.concatenate(qs)), off)
        bp.status()
        phi, field = phi.cpu().numpy(), field.cpu().numpy().T
        for k in range(3):
            sl = slice(off[k], off[k + 1])
            ref = OPlan(boxes[k], 10, lam=1.7).solve(xs[k], qs[k])
            assert _rel(phi[sl], ref[0]) <= TOL["fp32"], (counts, k)
            assert _rel(field[sl], ref[1]) <= TOL["fp32"], (counts, k)


def test_batched_graph_replays_with_eager_work_between(ps):
    """The batched path replays one captured graph while the caller's buffers
    stay put; new particle data written into those buffers between replays,
    with unrelated eager work and synchronizations in between, must give that
    data's sums on every replay (each replay checked against the oracle)."""
    g = np.random.default_rng(17)
    boxes = [g.uniform(1.0, 2.0, size=3) for _ in range(3)]
    ns = [700, 260, 1100]
    systems = [dict(box=b, n_max=n) for b, n in zip(boxes, ns)]
    off = np.concatenate([[0], np.cumsum(ns)])
    lam = float(np.sqrt(3))
    bp = ps.BatchedPlan(systems, p=10, lam=lam, precision="fp64")
    X = torch.empty(3, off[-1], dtype=torch.float64, device="cuda:0")
    Q = torch.empty(off[-1], dtype=torch.float64, device="cuda:0")
    phi = torch.empty(off[-1], dtype=torch.float64, device="cuda:0")
    field = torch.empty(3, off[-1], dtype=torch.float64, device="cuda:0")
    single = ps.Plan(boxes[0], 10, lam=lam, precision="fp64", n_max=ns[0])
    first = None
    for rep in range(4):
        data = [W.uniform_box(n, b, charges="gauss", seed=300 + 10 * rep + k) for k, (n, b) in enumerate(zip(ns, boxes))]
        X.copy_(_dev(np.concatenate([d[0] for d in data]).T))
        Q.copy_(_dev(np.concatenate([d[1] for d in data])))
        bp.eval(X, Q, off, out=(phi, field))
        torch.cuda.synchronize()
        # eager work between replays: a single-box solve and a torch reduction
        sp, _ = single.eval(_dev(data[0][0].T), _dev(data[0][1]))
        junk = torch.randn(1 << 20, device="cuda:0").sum()
        torch.cuda.synchronize()
        bp.status()
        ph, fl = phi.cpu().numpy(), field.cpu().numpy().T
        assert np.isfinite(float(junk))
        assert _rel(ph[off[0]:off[1]], sp.cpu().numpy()) <= 1e-13
        for k in range(3):
            sl = slice(off[k], off[k + 1])
            ref = OPlan(boxes[k], 10, lam=lam).solve(data[k][0], data[k][1])
            assert _rel(ph[sl], ref[0]) <= TOL["fp64"], (rep, k)
            assert _rel(fl[sl], ref[1]) <= TOL["fp64"], (rep, k)
        if first is None:
            first = (data, ph.copy())
    # replaying the first data again reproduces the first replay bit for bit
    data, ph0 = first
    X.copy_(_dev(np.concatenate([d[0] for d in data]).T))
    Q.copy_(_dev(np.concatenate([d[1] for d in data])))
    bp.eval(X, Q, off, out=(phi, field))
    assert np.array_equal(phi.cpu().numpy(), ph0)


def test_batched_entry_on_a_single_plan_with_profiling_and_new_buffers(ps):
    """A one-box plan driven through the batched entry point while stage
    profiling is on: the graph holds no event records (stage times stay those
    of the last eager eval), and a replay into other output buffers (the graph
    is captured again for them) gives the eager eval's results bit for bit."""
    import ctypes
    n = 1500
    x, q = W.uniform_box(n, (1.0, 1.2, 0.9), charges="gauss", seed=41)
    pl = ps.Plan((1.0, 1.2, 0.9), 10, lam=1.7, precision="fp32", n_max=n)
    pl.set_profiling(True)
    xt, qt = _dev(x.T), _dev(q)
    phi_e, field_e = pl.eval(xt, qt)
    st = pl.stage_times()
    off = (ctypes.c_int64 * 2)(0, n)
    L = ps._lib.lib()
    for rep in range(3):
        phi = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        field = torch.full((3, n), float("nan"), dtype=torch.float64, device="cuda:0")
        ps._lib.check(L.periodic_sum_eval_batched(
            pl.handle, off, *(ctypes.c_void_p(t.data_ptr()) for t in (xt[0], xt[1], xt[2], qt, phi, field[0], field[1], field[2])),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        pl.status()
        assert torch.equal(phi, phi_e) and torch.equal(field, field_e), rep
    assert pl.stage_times() == st
    pl.set_profiling(False)


# --------------------------------------------------------------------------
# full-size workloads: sampled particles against stored oracle values
# (tests/golden/make_reference.py, oracle only)
# --------------------------------------------------------------------------
def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    if not os.path.exists(path):
        pytest.skip("reference %s not generated" % name)
    return np.load(path)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_uniform_cube(ps, prec):
    """N = 100,000 uniform in the unit cube, q ~ N(0,1) minus mean, p = 16,
    in the launch configuration the benchmark times; 2,000 sampled particles."""
    c = W.config2()
    ref = _golden("ref_cfg2.npz")
    pl, phi, field = _run(ps, c["box"], c["p"], c["x"], c["q"], prec, R_b=c["R_b"])
    sub = ref["subset"]
    assert pl.info()["n_near_last"] == int(ref["n_near"])
    assert pl.info()["mean_corners"] == 1  # the box mean by corner points
    e1, e2 = _rel(phi[sub], ref["phi"]), _rel(field[sub], ref["field"])
    print(prec, "cfg2 rel-L2 phi %.3e field %.3e" % (e1, e2))
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


def test_full_size_clustered_anisotropic(ps):
    """N = 1,000,000 in 64 Gaussian blobs, box 1x1x2.5, p = 20, lambda = 1.5,
    FP32 pairs with FP64 accumulation; 2,000 sampled particles."""
    c = W.config3()
    ref = _golden("ref_cfg3.npz")
    pl, phi, field = _run(ps, c["box"], c["p"], c["x"], c["q"], "fp32", lam=c["lam"])
    sub = ref["subset"]
    assert pl.info()["n_near_last"] == int(ref["n_near"])
    e1, e2 = _rel(phi[sub], ref["phi"]), _rel(field[sub], ref["field"])
    print("cfg3 rel-L2 phi %.3e field %.3e" % (e1, e2))
    assert e1 <= 1e-6 and e2 <= 1e-6


def test_full_size_batch(ps):
    """512 boxes, d_k ~ U[1,2], N ~ log-uniform[200, 20000], p = 12, lambda = sqrt 3,
    FP32 pairs, one graph launch; sampled particles of six systems."""
    c = W.config4()
    ref = _golden("ref_cfg4.npz")
    systems = [dict(box=s["box"], n_max=len(s["q"])) for s in c["systems"]]
    bp = ps.BatchedPlan(systems, p=c["p"], lam=c["lam"], precision="fp32")
    off = np.concatenate([[0], np.cumsum([len(s["q"]) for s in c["systems"]])])
    X = np.concatenate([s["x"] for s in c["systems"]])
    Q = np.concatenate([s["q"] for s in c["systems"]])
    phi, field = bp.eval(_dev(X.T), _dev(Q), off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    for k in ref["systems"]:
        sub = ref["sub_%d" % k] + off[k]
        assert _rel(phi[sub], ref["phi_%d" % k]) <= 1e-6
        assert _rel(field[sub], ref["field_%d" % k]) <= 1e-6


def test_full_size_rocksalt_energy_gradient(ps):
    """Jittered 32^3 rock-salt lattice, p = 16: sampled potentials and fields
    against the oracle; the physical gradient is -q field; the exact adjoint
    agrees with central differences on sampled coordinates."""
    c = W.config5()
    ref = _golden("ref_cfg5.npz")
    n = len(c["q"])
    pl = ps.Plan(c["box"], c["p"], R_b=c["R_b"], n_max=n)
    xt, qt = _dev(c["x"].T), _dev(c["q"])
    phi, field = pl.eval(xt, qt)
    sub = ref["subset"]
    assert _rel(phi.cpu().numpy()[sub], ref["phi"]) <= 1e-12
    assert _rel(field.cpu().numpy().T[sub], ref["field"]) <= 1e-12
    e = pl.energy(xt, qt)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(xt, qt, one, exact=True)
    px, _ = pl.energy_vjp(xt, qt, one, exact=False)
    gx = gx.cpu().numpy()
    assert _rel(px.cpu().numpy()[:, sub].T, -c["q"][sub, None] * ref["field"]) <= 1e-12
    # exact adjoint vs physical gradient: method truncation level
    assert _rel(gx, px.cpu().numpy()) < 1e-3
    h = 1e-5

    def energy(xx):
        return float(pl.energy(_dev(xx.T), qt).cpu()[0])

    x = c["x"]
    for i in sub[:3]:
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (energy(xp) - energy(xm)) / (2 * h)
            assert abs(gx[k, i] - fd) < 1e-5 * max(1.0, abs(fd)), (i, k, gx[k, i], fd)
    del e


def test_autotuned_batch_still_matches_oracle(ps):
    """The autotuner only changes the launch shape: results stay at the bar."""
    g = np.random.default_rng(9)
    systems, xs, qs = [], [], []
    for k in range(5):
        box = g.uniform(1.0, 2.0, size=3)
        n = int(g.integers(100, 2500))
        x, q = W.uniform_box(n, box, charges="gauss", seed=200 + k)
        systems.append(dict(box=box, n_max=n))
        xs.append(x)
        qs.append(q)
    lam = float(np.sqrt(3))
    bp = ps.BatchedPlan(systems, p=9, lam=lam, precision="fp32")
    off = np.concatenate([[0], np.cumsum([len(q) for q in qs])])
    X, Q = _dev(np.concatenate(xs).T), _dev(np.concatenate(qs))
    ms = bp.autotune(X, Q, off)
    assert ms > 0 and bp.info()["tile_targets"] in (64, 128, 256)
    phi, field = bp.eval(X, Q, off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    nb = bp.near_counts()
    for k in range(5):
        sl = slice(off[k], off[k + 1])
        op = OPlan(systems[k]["box"], 9, lam=lam)
        parts = op.solve(xs[k], qs[k], return_parts=True)
        assert nb[k] == parts["n_near"]
        assert _rel(phi[sl], parts["phi"]) <= 1e-6
        assert _rel(field[sl], parts["field"]) <= 1e-6


# --------------------------------------------------------------------------
# RBF basis (eq. (5)) and caller-given check points
# --------------------------------------------------------------------------
# The RBF fitting matrix is far less well conditioned (cond(A) ~ 1e6 for 256
# centres at p = 16) than the renormalized spherical basis (~10).  Two correct
# FP64 pseudo-inverses may then differ by up to ~cond(A) x 1e-16 in the
# coefficients; the potentials at the particles agree much better (measured
# 1.3e-13), and the FP64 bar for this variant is set at 1e-11.
TOL_RBF = {"fp64": 1e-11, "fp32": 1e-6}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rbf_basis_matches_oracle(ps, prec):
    c = W.config1()
    cen = W.fibonacci_sphere(256, 1.5)
    op = OPlan(c["box"], 16, R_b=1.5, basis="rbf", centres=cen)
    ref = op.solve(c["x"], c["q"], return_parts=True)
    pl = ps.Plan(c["box"], 16, R_b=1.5, precision=prec, n_max=1000, centres=cen)
    phi, field = pl.eval(_dev(c["x"].T), _dev(c["q"]))
    pl.status()
    e1, e2 = _rel(phi.cpu().numpy(), ref["phi"]), _rel(field.cpu().numpy().T, ref["field"])
    print(prec, "rbf rel-L2 phi %.3e field %.3e cond %.3e" % (e1, e2, op.cond))
    assert e1 <= TOL_RBF[prec] and e2 <= TOL_RBF[prec]
    inf = pl.info()
    assert inf["P"] == 257 and inf["rank"] == op.rank
    _, _, pinv, bm = (t.numpy() for t in pl.tables())
    np.testing.assert_allclose(bm, op.R0mean, rtol=1e-13)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_random_check_points_match_oracle(ps, prec):
    box = (1.0, 1.2, 0.9)
    R0 = 0.5 * np.linalg.norm(box)
    yc = W.random_sphere(3 * 12 * 12, R0, seed=7)
    x, q = W.uniform_box(900, box, charges="gauss", seed=77)
    ref = OPlan(box, 12, lam=1.6, check_points=yc).solve(x, q)
    pl = ps.Plan(box, 12, lam=1.6, precision=prec, n_max=900, check_points=yc)
    phi, field = pl.eval(_dev(x.T), _dev(q))
    pl.status()
    assert pl.info()["L"] == 432
    assert _rel(phi.cpu().numpy(), ref[0]) <= TOL[prec]
    assert _rel(field.cpu().numpy().T, ref[1]) <= TOL[prec]


def test_rbf_energy_adjoint_matches_oracle(ps):
    box = (1.0, 1.0, 1.0)
    x, q = W.uniform_box(500, box, charges="gauss", seed=5)
    cen = W.fibonacci_sphere(120, 1.5)
    op = OPlan(box, 10, R_b=1.5, basis="rbf", centres=cen)
    E, dx, dq, _ = energy_gradients(op, x, q)
    pl = ps.Plan(box, 10, R_b=1.5, n_max=500, centres=cen)
    xt, qt = _dev(x.T), _dev(q)
    e = pl.energy(xt, qt)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(xt, qt, one, exact=True)
    assert abs(float(e.cpu()[0]) - E) <= 1e-9 * abs(E)
    assert _rel(gx.cpu().numpy().T, dx) <= 1e-9
    assert _rel(gq.cpu().numpy(), dq) <= 1e-9


def test_batched_mixed_bases(ps):
    """One batch holding a spherical-basis box and an RBF-basis box."""
    g = np.random.default_rng(3)
    boxes = [np.array([1.0, 1.3, 1.1]), np.array([1.2, 1.0, 1.0])]
    xs, qs = [], []
    for k, b in enumerate(boxes):
        x, q = W.uniform_box(700 + 300 * k, b, charges="gauss", seed=300 + k)
        xs.append(x)
        qs.append(q)
    lam = 1.7
    R0 = [0.5 * np.linalg.norm(b) for b in boxes]
    cen = W.fibonacci_sphere(200, lam * R0[1])
    systems = [dict(box=boxes[0], n_max=len(qs[0])), dict(box=boxes[1], n_max=len(qs[1]), centres=cen)]
    bp = ps.BatchedPlan(systems, p=12, lam=lam, precision="fp64")
    off = np.concatenate([[0], np.cumsum([len(q) for q in qs])])
    phi, field = bp.eval(_dev(np.concatenate(xs).T), _dev(np.concatenate(qs)), off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    r0 = OPlan(boxes[0], 12, lam=lam).solve(xs[0], qs[0])
    r1 = OPlan(boxes[1], 12, lam=lam, basis="rbf", centres=cen).solve(xs[1], qs[1])
    assert _rel(phi[off[0]:off[1]], r0[0]) <= 1e-12 and _rel(field[off[0]:off[1]], r0[1]) <= 1e-12
    assert _rel(phi[off[1]:off[2]], r1[0]) <= 1e-9 and _rel(field[off[1]:off[2]], r1[1]) <= 1e-9


def test_batched_box_mean_by_corners_and_by_entries(ps):
    """The box mean C1 takes two routes: by corner points for boxes whose image
    range fits the per-wave column masks (at most 64 (x, y) image columns and
    31 z images) when the launch has at least 2,048 workgroups of 64
    particles x corner-column slices, else by near entries.  Here 40 boxes
    with sides U[1, 2] (unequal image ranges per axis) of 4,000 particles
    (2,520 chunks, at least 2 slices each) take the corner route and the
    1 x 1 x 10 box at lambda = 1.3 (15 x 15 image columns) the per-entry one;
    sampled systems of both match the oracle (FP64, bar 1e-12)."""
    g = np.random.default_rng(901)
    boxes = [g.uniform(1.0, 2.0, size=3) for _ in range(40)] + [np.array([1.0, 1.0, 10.0])]
    ns = [4000] * 40 + [400]
    data = [W.uniform_box(n, b, charges="gauss", seed=900 + k) for k, (b, n) in enumerate(zip(boxes, ns))]
    bp = ps.BatchedPlan([dict(box=b, n_max=n) for b, n in zip(boxes, ns)], p=8, lam=1.3, precision="fp64")
    off = np.concatenate([[0], np.cumsum(ns)])
    phi, field = bp.eval(_dev(np.concatenate([d[0] for d in data]).T), _dev(np.concatenate([d[1] for d in data])), off)
    bp.status()
    assert bp.info()["mean_corners"] == 40
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    for k in (0, 17, 39, 40):
        ref = OPlan(boxes[k], 8, lam=1.3).solve(data[k][0], data[k][1])
        sl = slice(off[k], off[k + 1])
        assert _rel(phi[sl], ref[0]) <= 1e-12 and _rel(field[sl], ref[1]) <= 1e-12, k


# --------------------------------------------------------------------------
# plan files: the set phase saved and reloaded
# --------------------------------------------------------------------------
def test_plan_save_load_round_trip(ps, tmp_path):
    """A reloaded plan has the same tables, shape and info, and gives bitwise the
    same sums as the plan it was saved from; a corrupted file is refused."""
    box = (1.0, 1.2, 0.9)
    x, q = W.uniform_box(3000, box, charges="gauss", seed=41)
    pl = ps.Plan(box, 12, lam=float(np.sqrt(3)), precision="fp32", n_max=3000, tile_targets=128)
    phi0, field0 = pl.eval(_dev(x.T), _dev(q))
    pl.status()
    path = tmp_path / "cube.plan"
    pl.save(path)
    pl2 = ps.Plan.load(path)
    i1, i2 = pl.info(), pl2.info()
    for k in ("p", "P", "L", "n_images", "rank", "R0", "R_b", "cond", "tile_targets", "nsys"):
        assert i1[k] == i2[k], k
    for a, b in zip(pl.tables(), pl2.tables()):
        assert torch.equal(a, b)
    phi1, field1 = pl2.eval(_dev(x.T), _dev(q))
    pl2.status()
    assert torch.equal(phi0, phi1) and torch.equal(field0, field1)
    data = bytearray(path.read_bytes())
    data[len(data) // 2] ^= 0x10
    bad = tmp_path / "bad.plan"
    bad.write_bytes(bytes(data))
    with pytest.raises(ps.PeriodicSumError) as err:
        ps.Plan.load(bad)
    assert err.value.status == ps._lib.PS_E_IO


def test_batched_plan_save_load_mixed_bases(ps, tmp_path):
    """A batch of a spherical box, an RBF box and a box with caller-given check
    points, saved after autotuning and reloaded, reproduces its sums bitwise."""
    boxes = [np.array([1.0, 1.3, 1.1]), np.array([1.2, 1.0, 1.0]), np.array([1.1, 1.1, 0.9])]
    ns = [700, 1000, 500]
    data = [W.uniform_box(n, b, charges="gauss", seed=500 + k) for k, (n, b) in enumerate(zip(ns, boxes))]
    lam = 1.7
    R0 = [0.5 * np.linalg.norm(b) for b in boxes]
    systems = [dict(box=boxes[0], n_max=ns[0]),
               dict(box=boxes[1], n_max=ns[1], centres=W.fibonacci_sphere(200, lam * R0[1])),
               dict(box=boxes[2], n_max=ns[2], check_points=W.random_sphere(400, R0[2], seed=9))]
    bp = ps.BatchedPlan(systems, p=12, lam=lam, precision="fp32")
    off = np.concatenate([[0], np.cumsum(ns)])
    X = _dev(np.concatenate([d[0] for d in data]).T)
    Q = _dev(np.concatenate([d[1] for d in data]))
    bp.autotune(X, Q, off)
    phi0, field0 = bp.eval(X, Q, off)
    bp.status()
    path = tmp_path / "batch.plan"
    bp.save(path)
    bp2 = ps.BatchedPlan.load(path)
    assert bp2.nsys == 3 and bp2.info()["tile_targets"] == bp.info()["tile_targets"]
    phi1, field1 = bp2.eval(X, Q, off)
    bp2.status()
    assert torch.equal(phi0, phi1) and torch.equal(field0, field1)
    ref = OPlan(boxes[0], 12, lam=lam).solve(data[0][0], data[0][1])
    assert _rel(phi1.cpu().numpy()[off[0]:off[1]], ref[0]) <= TOL["fp32"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_thomson_check_points_and_centres_match_oracle(ps, prec):
    """400 Thomson check points (Table 1's T(400)) with the spherical basis, and
    with 256 Thomson RBF centres on S_b (Sec. 4.1): the library matches the oracle
    given the same point sets."""
    box = (1.0, 1.1, 0.95)
    lam = 1.7
    R0 = 0.5 * np.linalg.norm(box)
    yc = W.thomson_points(400, R0)
    cen = W.thomson_points(256, lam * R0)
    x, q = W.uniform_box(800, box, charges="gauss", seed=88)
    for kw, tol in ((dict(check_points=yc), TOL[prec]), (dict(check_points=yc, centres=cen), TOL_RBF[prec])):
        okw = dict(kw)
        if "centres" in okw:
            okw["basis"] = "rbf"
        ref = OPlan(box, 14, lam=lam, **okw).solve(x, q)
        pl = ps.Plan(box, 14, lam=lam, precision=prec, n_max=800, **kw)
        phi, field = pl.eval(_dev(x.T), _dev(q))
        pl.status()
        assert _rel(phi.cpu().numpy(), ref[0]) <= tol
        assert _rel(field.cpu().numpy().T, ref[1]) <= tol


@pytest.mark.parametrize("lam, p", [(1.3, 34), (1.5, 24), (1.7, 19)])
def test_table2_accuracy_at_the_papers_p_min(ps, lam, p):
    """Sec. 4.2, Table 2 (27,000 grid charges, FP64, tolerance eps_2 = 5e-7): at the
    paper's p_min the library's potential is within the tolerance of the Ewald sum
    at 2,000 sampled charges, and matches the oracle's method there."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ref_table2.npz")
    if not os.path.exists(path):
        pytest.skip("reference ref_table2.npz not generated")
    ref = np.load(path)
    x, q = W.grid_charges(30, 2)
    sub = ref["subset"]
    pl = ps.Plan((1.0, 1.0, 1.0), p, lam=lam, precision="fp64", n_max=len(q))
    phi, _ = pl.eval(_dev(x.T), _dev(q))
    pl.status()
    ph = phi.cpu().numpy()[sub]
    assert _rel(ph, ref["phi_ewald"]) < 5e-7
    assert _rel(ph, ref["phi_method_%g_%d" % (lam, p)]) <= TOL["fp64"]


def test_parameter_selection_in_the_table2_setting(ps):
    """Sec. 3.3, eqs. (o1)-(o2), in the setting of Table 2 (27,000 grid charges,
    FP64, tolerance 5e-7 on phi): for each lambda the selector's p meets the
    tolerance against the oracle's independent Ewald sum at the 2,000 stored
    sample charges, and p - 1 does not (to within 20%: the selector measures all
    charges against a high-p solve, not a sample against Ewald).  The chosen
    candidate is the fastest of those that meet the tolerance."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ref_table2.npz")
    if not os.path.exists(path):
        pytest.skip("reference ref_table2.npz not generated")
    ref = np.load(path)
    x, q = W.grid_charges(30, 2)
    sub = ref["subset"]
    tol = 5e-7
    xt, qt = _dev(x.T), _dev(q)
    best, rows = ps.select_parameters((1.0, 1.0, 1.0), xt, qt, tol, lambdas=(1.3, 1.5, 1.7), precision="fp64",
                                      p_ref=36)
    for r in rows:
        print("lambda %.2f p %d solves %d B_P %.2e err %.2e ms %.2f set %.2fs" % (
            r["lambda"], r["p"], r["n_solves"], r["B_P"], r["err"], r["ms"], r["set_s"]))
    assert best is not None
    assert best["ms"] == min(r["ms"] for r in rows if r["p"] > 0 and r["err_prec"] <= tol)

    def eps2(lam, p):
        pl = ps.Plan((1.0, 1.0, 1.0), p, lam=lam, precision="fp64", n_max=len(q))
        phi, _ = pl.eval(xt, qt)
        pl.status()
        return _rel(phi.cpu().numpy()[sub], ref["phi_ewald"])

    for r in rows:
        assert r["p"] > 0 and r["err"] <= tol and r["err_prec"] <= tol
        assert eps2(r["lambda"], r["p"]) < 1.2 * tol
        assert eps2(r["lambda"], r["p"] - 1) > tol / 1.2


def test_parameter_selection_fp32_is_minimal(ps):
    """The selector in FP32 at a looser tolerance (1e-5, 3,000 uniform charges):
    the fastest candidate's FP32 solve meets the tolerance, and for every
    candidate an FP64 solve at p - 1 misses it against the same high-p
    reference, so the search stops at the smallest passing p."""
    box = (1.0, 1.2, 0.9)
    x, q = W.uniform_box(3000, box, charges="gauss", seed=21)
    xt, qt = _dev(x.T), _dev(q)
    tol = 1e-5
    best, rows = ps.select_parameters(box, xt, qt, tol, lambdas=(1.2, 1.5), precision="fp32", p_ref=30)
    assert best is not None and best["err_prec"] <= tol
    refp = ps.Plan(box, 30, lam=1.5, precision="fp64", n_max=len(q))
    phi_ref = refp.eval(xt, qt)[0].cpu().numpy()
    for r in rows:
        assert r["p"] > 2 and r["err"] <= tol
        pl = ps.Plan(box, r["p"] - 1, lam=r["lambda"], precision="fp64", n_max=len(q))
        phi = pl.eval(xt, qt)[0].cpu().numpy()
        assert _rel(phi, phi_ref) > tol


def test_largest_truncation_number_energy_and_adjoint(ps):
    """p = 40, the largest truncation number the library accepts (P = 1600 basis
    terms, L = 3160 check points): energy and exact adjoint match the oracle."""
    box = (1.0, 1.1, 0.9)
    x, q = W.uniform_box(300, box, charges="gauss", seed=12)
    op = OPlan(box, 40, lam=1.3)
    E, dx, dq, _ = energy_gradients(op, x, q)
    pl = ps.Plan(box, 40, lam=1.3, n_max=300, precision="fp64")
    inf = pl.info()
    assert inf["P"] == 1600 and inf["L"] == 3160 and inf["rank"] == op.rank
    xt, qt = _dev(x.T), _dev(q)
    e = pl.energy(xt, qt)
    g = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(xt, qt, g, exact=True)
    pl.status()
    assert abs(float(e.cpu()[0]) - E) <= 1e-12 * abs(E)
    assert _rel(gx.cpu().numpy().T, dx) <= 1e-11
    assert _rel(gq.cpu().numpy(), dq) <= 1e-11


# --------------------------------------------------------------------------
# elongated and flat boxes of Table 5 (hundreds of lattice images)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_elongated_box_matches_oracle(ps, prec):
    """Table 5's 10 x 1 x 1 box at lambda = 1.3 (A_gf = 53.9; 3 x 15 x 15 lattice
    images before pruning): the library matches the oracle."""
    box = (10.0, 1.0, 1.0)
    x, q = W.uniform_box(2000, box, charges="gauss", seed=51)
    ref = OPlan(box, 16, lam=1.3).solve(x, q)
    pl = ps.Plan(box, 16, lam=1.3, precision=prec, n_max=2000)
    phi, field = pl.eval(_dev(x.T), _dev(q))
    pl.status()
    assert _rel(phi.cpu().numpy(), ref[0]) <= TOL[prec]
    assert _rel(field.cpu().numpy().T, ref[1]) <= TOL[prec]


def test_table5_near_set_sizes(ps):
    """Table 5 (N = 1e5 uniform, lambda = 1.3): the device's near-set size for each
    box is within 6 standard deviations of A_gf lambda^3 N (eq. (o2.1)), as the
    paper's counts are."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))["table5"]
    for k, (box, nb_paper) in enumerate(zip(gold["boxes"], gold["N_b"])):
        d = np.asarray(box, float)
        agf = np.pi / 6 * np.sum(d * d) ** 1.5 / np.prod(d)
        mean = agf * gold["lambda"] ** 3 * gold["N"]
        x, q = W.uniform_box(gold["N"], d, charges="gauss", seed=60 + k)
        pl = ps.Plan(d, 8, lam=gold["lambda"], precision="fp32", n_max=gold["N"])
        pl.eval(_dev(x.T), _dev(q))
        pl.status()
        nb = pl.near_counts()[0]
        assert abs(nb - mean) < 6 * np.sqrt(mean), (box, nb, mean)
        assert abs(nb_paper - mean) < 6 * np.sqrt(mean)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nearly_coincident_pairs(ps, prec):
    """Pairs of charges 1e-4 .. 1e-7 apart, whose mutual field dominates the field
    norm: the FP32 path's two-float relative coordinates keep the separation
    exact enough that both potential and field meet the FP32 bar."""
    g = np.random.default_rng(23)
    box = (1.0, 1.0, 1.0)
    x, q = W.uniform_box(1500, box, charges="gauss", seed=23)
    pairs = []
    for k, sep in enumerate(np.logspace(-4, -7, 40)):
        c = g.uniform(-0.45, 0.45, size=3)
        u = g.standard_normal(3)
        u /= np.linalg.norm(u)
        pairs += [c, c + sep * u]
    xp = np.array(pairs)
    m = g.uniform(0.5, 1.5, size=len(xp) // 2)
    qp = np.stack([m, -m], axis=1).ravel()        # each close pair is a dipole
    X = np.concatenate([x, xp])
    Q = np.concatenate([q, qp])
    Q -= Q.mean()
    ref = OPlan(box, 12, R_b=1.5).solve(X, Q)
    pl = ps.Plan(box, 12, R_b=1.5, precision=prec, n_max=len(Q))
    phi, field = pl.eval(_dev(X.T), _dev(Q))
    pl.status()
    assert _rel(phi.cpu().numpy(), ref[0]) <= TOL[prec]
    assert _rel(field.cpu().numpy().T, ref[1]) <= TOL[prec]


def test_binding_refuses_mismatched_tensors(ps):
    """float32 or short charge arrays and offsets that do not cover the packed
    arrays are refused before the library runs; the plan still works after."""
    c = W.config1()
    pl = ps.Plan(c["box"], 8, R_b=1.5, n_max=1000)
    x = _dev(c["x"].T)
    with pytest.raises(ValueError):
        pl.eval(x, _dev(c["q"]).float())
    with pytest.raises(ValueError):
        pl.eval(x, _dev(c["q"][:999]))
    with pytest.raises(ValueError):
        pl.eval(x, _dev(c["q"]), out=(torch.empty(1000, device="cuda:0", dtype=torch.float64),
                                      torch.empty(1000, 3, device="cuda:0", dtype=torch.float64)))
    bp = ps.BatchedPlan([dict(box=c["box"], n_max=600), dict(box=c["box"], n_max=600)], p=8, lam=1.8)
    with pytest.raises(ValueError):
        bp.eval(x, _dev(c["q"]), [0, 500, 900])
    phi, _ = pl.eval(x, _dev(c["q"]))
    pl.status()
    assert np.isfinite(phi.cpu().numpy()).all()


def test_eval_captured_in_a_user_graph(ps):
    """After a warm-up call with the same shapes, periodic_sum_eval only enqueues
    kernels, so a caller can capture it into a graph: replays with new particle
    data in the same buffers (eager work and synchronizations in between) match
    eager evaluations of that data bitwise."""
    box = (1.0, 1.2, 0.9)
    n = 1200
    pl = ps.Plan(box, 10, lam=1.7, precision="fp32", n_max=n)
    X = torch.empty(3, n, dtype=torch.float64, device="cuda:0")
    Q = torch.empty(n, dtype=torch.float64, device="cuda:0")
    phi = torch.empty(n, dtype=torch.float64, device="cuda:0")
    field = torch.empty(3, n, dtype=torch.float64, device="cuda:0")

    def load(seed):
        x, q = W.uniform_box(n, box, charges="gauss", seed=seed)
        X.copy_(_dev(x.T))
        Q.copy_(_dev(q))

    load(700)
    pl.eval(X, Q, out=(phi, field))          # warm-up: builds the plan's tables
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pl.eval(X, Q, out=(phi, field))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        load(710 + rep)
        g.replay()
        torch.cuda.synchronize()
        got_phi, got_field = phi.clone(), field.clone()
        junk = torch.randn(1 << 18, device="cuda:0").sum()
        eager_phi, eager_field = pl.eval(X, Q)
        torch.cuda.synchronize()
        pl.status()
        assert torch.isfinite(junk)
        assert torch.equal(got_phi, eager_phi) and torch.equal(got_field, eager_field), rep


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_table4_bases_against_ewald(ps, prec):
    """Sec. 4.2, Table 4 (lambda = 1.5, p = 16, 27,000 grid charges): the library's
    eps_2 against the Ewald sum for the spherical basis and for 256 Thomson RBF
    centres is within a factor 2 of the paper's, and the potential matches the
    oracle's method at the sampled charges."""
    import json
    import os
    here = os.path.dirname(__file__)
    path = os.path.join(here, "golden", "ref_table2.npz")
    if not os.path.exists(path):
        pytest.skip("reference ref_table2.npz not generated")
    ref = np.load(path)
    gold = json.load(open(os.path.join(here, "golden", "paper_tables.json")))["table4"]["eps_2"]["27000"]
    x, q = W.grid_charges(30, 2)
    sub = ref["subset"]
    cen = W.thomson_points(256, 1.5 * np.sqrt(3) / 2)
    for name, kw, tol in (("spherical", {}, TOL[prec]), ("rbf", dict(centres=cen), TOL_RBF[prec])):
        pl = ps.Plan((1.0, 1.0, 1.0), 16, lam=1.5, precision=prec, n_max=len(q), **kw)
        phi, _ = pl.eval(_dev(x.T), _dev(q))
        pl.status()
        ph = phi.cpu().numpy()[sub]
        e2 = _rel(ph, ref["phi_ewald"])
        assert gold[name] / 2 < e2 < gold[name] * 2, (name, e2)
        assert _rel(ph, ref["phi_table4_" + name]) <= tol


@pytest.mark.parametrize("lam, p", [(1.3, 34), (1.5, 25), (1.7, 19)])
def test_table3_accuracy_at_the_papers_p_min(ps, lam, p):
    """Sec. 4.2, Table 3 (216,000 grid charges, FP64, tolerance eps_2 = 5e-7): at the
    paper's p_min the library meets the tolerance against the Ewald sum at 2,000
    sampled charges and matches the oracle's method there."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ref_table3.npz")
    if not os.path.exists(path):
        pytest.skip("reference ref_table3.npz not generated")
    ref = np.load(path)
    x, q = W.grid_charges(60, 3)
    sub = ref["subset"]
    pl = ps.Plan((1.0, 1.0, 1.0), p, lam=lam, precision="fp64", n_max=len(q))
    phi, _ = pl.eval(_dev(x.T), _dev(q))
    pl.status()
    ph = phi.cpu().numpy()[sub]
    assert _rel(ph, ref["phi_ewald"]) < 5e-7
    assert _rel(ph, ref["phi_method_%g_%d" % (lam, p)]) <= TOL["fp64"]


def test_stage_profiling(ps):
    """set_profiling / stage_times: refused before a profiled eval; afterwards eight
    non-negative stage durations whose sum matches the eval's own event timing,
    with the particle pair sums the largest stage at this size."""
    from paper_1310_4374_amd import PeriodicSumError
    x, q = W.uniform_box(20000, (1.0, 1.0, 1.0), charges="gauss", seed=99)
    pl = ps.Plan((1.0, 1.0, 1.0), 12, R_b=1.5, precision="fp32", n_max=20000)
    xt, qt = _dev(x.T), _dev(q)
    pl.eval(xt, qt)
    with pytest.raises(PeriodicSumError, match="INVALID"):
        pl.stage_times()
    pl.set_profiling(True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    pl.eval(xt, qt)
    b.record()
    st = pl.stage_times()
    pl.status()
    total = a.elapsed_time(b)
    assert list(st) == list(ps._lib.STAGES)
    assert all(v >= 0.0 for v in st.values())
    assert max(st, key=st.get) == "pairs"
    assert abs(sum(st.values()) - total) < 0.2 * total + 0.05
    pl.set_profiling(False)
