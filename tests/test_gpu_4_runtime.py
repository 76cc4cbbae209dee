"""Runtime behaviour of the library on the GPU: data errors, synchronous
validation, bitwise reproducibility, concurrent plans on two streams, graph
capture and replay, stage profiling, plan files and the binding's argument
checks.  Results are still checked against the oracle or bit for bit against
eager evaluations.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import GOLDEN, TOL, dev, err, golden, load_ps, rel, run, worst  # noqa: F401
from oracle.adjoint import energy_gradients, physics_gradients  # noqa: F401
from oracle.method import Plan as OPlan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    return load_ps()


def test_status_reports_data_errors(ps):
    from paper_1310_4374_amd import PeriodicSumError
    c = W.config1()
    pl = ps.Plan(c["box"], 8, R_b=1.5, n_max=1000)
    q = c["q"].copy()
    q[0] += 0.5
    pl.eval(dev(c["x"].T), dev(q))
    with pytest.raises(PeriodicSumError, match="NOT_NEUTRAL"):
        pl.status()
    x = c["x"].copy()
    x[5, 1] = 0.5  # upper face is outside the half-open box
    pl.eval(dev(x.T), dev(c["q"]))
    with pytest.raises(PeriodicSumError, match="OUT_OF_BOX"):
        pl.status()
    # a NaN coordinate or charge is reported the same way (every index the
    # kernels form comes from counts, and the cell key clamps NaN to cell 0)
    x = c["x"].copy()
    x[11, 2] = np.nan
    pl.eval(dev(x.T), dev(c["q"]))
    with pytest.raises(PeriodicSumError, match="OUT_OF_BOX"):
        pl.status()
    q = c["q"].copy()
    q[3] = np.nan
    pl.eval(dev(c["x"].T), dev(q))
    with pytest.raises(PeriodicSumError, match="OUT_OF_BOX"):
        pl.status()
    pl.eval(dev(c["x"].T), dev(c["q"]))
    pl.status()
    with pytest.raises(PeriodicSumError, match="INVALID"):
        pl.eval(dev(np.zeros((3, 2000))), dev(np.zeros(2000)))
    # a near list that 32-bit entry indices cannot address is refused before allocation
    with pytest.raises(PeriodicSumError, match="UNSUPPORTED"):
        ps.Plan(c["box"], 4, R_b=1.5, n_max=2 ** 30)


def test_synchronous_validation(ps, monkeypatch):
    """With PS_VALIDATE set when a plan is made, eval itself reports the data
    errors (single and batched plans); without it, eval only enqueues and the
    error waits for status()."""
    from paper_1310_4374_amd import PeriodicSumError
    c = W.config1()
    x, q = dev(c["x"].T), dev(c["q"])
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


def test_bitwise_reproducible(ps):
    c = W.config1()
    for prec in ("fp64", "fp32"):
        pl = ps.Plan(c["box"], 12, R_b=1.5, n_max=1000, precision=prec)
        a = pl.eval(dev(c["x"].T), dev(c["q"]))
        b = pl.eval(dev(c["x"].T), dev(c["q"]))
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
    XA, QA = dev(xa.T), dev(qa)
    XB, QB = dev(np.concatenate([d[0] for d in xb]).T), dev(np.concatenate([d[1] for d in xb]))
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
        X.copy_(dev(np.concatenate([d[0] for d in data]).T))
        Q.copy_(dev(np.concatenate([d[1] for d in data])))
        bp.eval(X, Q, off, out=(phi, field))
        torch.cuda.synchronize()
        # eager work between replays: a single-box solve and a torch reduction
        sp, _ = single.eval(dev(data[0][0].T), dev(data[0][1]))
        junk = torch.randn(1 << 20, device="cuda:0").sum()
        torch.cuda.synchronize()
        bp.status()
        ph, fl = phi.cpu().numpy(), field.cpu().numpy().T
        assert np.isfinite(float(junk))
        assert err(ph[off[0]:off[1]], sp.cpu().numpy()) <= 1e-13
        for k in range(3):
            sl = slice(off[k], off[k + 1])
            ref = OPlan(boxes[k], 10, lam=lam).solve(data[k][0], data[k][1])
            assert err(ph[sl], ref[0]) <= TOL["fp64"], (rep, k)
            assert err(fl[sl], ref[1]) <= TOL["fp64"], (rep, k)
        if first is None:
            first = (data, ph.copy())
    # replaying the first data again reproduces the first replay bit for bit
    data, ph0 = first
    X.copy_(dev(np.concatenate([d[0] for d in data]).T))
    Q.copy_(dev(np.concatenate([d[1] for d in data])))
    bp.eval(X, Q, off, out=(phi, field))
    assert np.array_equal(phi.cpu().numpy(), ph0)


def test_batched_entry_on_a_single_plan_with_profiling_and_new_buffers(ps):
    """A one-box plan driven through the batched entry point while stage
    profiling is on: the graph holds no event records (the plan's count of
    profiled evals does not move over the graph launches, and the stage times
    stay those of the last eager eval, read once and kept), and a replay into
    other output buffers (the graph is captured again for them) gives the eager
    eval's results bit for bit."""
    import ctypes
    n = 1500
    x, q = W.uniform_box(n, (1.0, 1.2, 0.9), charges="gauss", seed=41)
    pl = ps.Plan((1.0, 1.2, 0.9), 10, lam=1.7, precision="fp32", n_max=n)
    pl.set_profiling(True)
    xt, qt = dev(x.T), dev(q)
    phi_e, field_e = pl.eval(xt, qt)
    st = pl.stage_times()
    recorded = pl.info()["profiled_evals"]
    assert recorded == 1
    epoch = pl.forward_epoch()
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
    assert pl.info()["profiled_evals"] == recorded       # no event recorded inside the graph
    assert pl.forward_epoch() == epoch + 3               # but every launch is a forward pass
    assert pl.stage_times() == st                        # the cached durations of the eager eval
    pl.eval(xt, qt)                                      # a new profiled eager eval records again
    assert pl.info()["profiled_evals"] == recorded + 1
    assert all(v >= 0.0 for v in pl.stage_times().values())
    pl.set_profiling(False)


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
        X.copy_(dev(x.T))
        Q.copy_(dev(q))

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


def test_stage_profiling(ps):
    """set_profiling / stage_times: refused before a profiled eval; afterwards eight
    non-negative stage durations whose sum matches the eval's own event timing,
    with the particle pair sums the largest stage at this size."""
    from paper_1310_4374_amd import PeriodicSumError
    x, q = W.uniform_box(20000, (1.0, 1.0, 1.0), charges="gauss", seed=99)
    pl = ps.Plan((1.0, 1.0, 1.0), 12, R_b=1.5, precision="fp32", n_max=20000)
    xt, qt = dev(x.T), dev(q)
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
    assert pl.stage_times() == st          # no profiled eval since: the same means again
    # a window of 20 profiled evals (more than the 16 kept unread) read once:
    # the means add up to the loop's time per eval
    a.record()
    for _ in range(20):
        pl.eval(xt, qt)
    b.record()
    st20 = pl.stage_times()
    total = a.elapsed_time(b) / 20
    assert max(st20, key=st20.get) == "pairs"
    assert abs(sum(st20.values()) - total) < 0.2 * total + 0.05
    pl.set_profiling(False)


def test_plan_save_load_round_trip(ps, tmp_path):
    """A reloaded plan has the same tables, shape and info, and gives bitwise the
    same sums as the plan it was saved from; a corrupted file is refused."""
    box = (1.0, 1.2, 0.9)
    x, q = W.uniform_box(3000, box, charges="gauss", seed=41)
    pl = ps.Plan(box, 12, lam=float(np.sqrt(3)), precision="fp32", n_max=3000, tile_targets=128)
    phi0, field0 = pl.eval(dev(x.T), dev(q))
    pl.status()
    path = tmp_path / "cube.plan"
    pl.save(path)
    pl2 = ps.Plan.load(path)
    i1, i2 = pl.info(), pl2.info()
    for k in ("p", "P", "L", "n_images", "rank", "R0", "R_b", "cond", "tile_targets", "nsys"):
        assert i1[k] == i2[k], k
    for a, b in zip(pl.tables(), pl2.tables()):
        assert torch.equal(a, b)
    phi1, field1 = pl2.eval(dev(x.T), dev(q))
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
    X = dev(np.concatenate([d[0] for d in data]).T)
    Q = dev(np.concatenate([d[1] for d in data]))
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
    assert err(phi1.cpu().numpy()[off[0]:off[1]], ref[0]) <= TOL["fp32"]


def test_binding_refuses_mismatched_tensors(ps):
    """float32 or short charge arrays and offsets that do not cover the packed
    arrays are refused before the library runs; the plan still works after."""
    c = W.config1()
    pl = ps.Plan(c["box"], 8, R_b=1.5, n_max=1000)
    x = dev(c["x"].T)
    with pytest.raises(ValueError):
        pl.eval(x, dev(c["q"]).float())
    with pytest.raises(ValueError):
        pl.eval(x, dev(c["q"][:999]))
    with pytest.raises(ValueError):
        pl.eval(x, dev(c["q"]), out=(torch.empty(1000, device="cuda:0", dtype=torch.float64),
                                      torch.empty(1000, 3, device="cuda:0", dtype=torch.float64)))
    bp = ps.BatchedPlan([dict(box=c["box"], n_max=600), dict(box=c["box"], n_max=600)], p=8, lam=1.8)
    with pytest.raises(ValueError):
        bp.eval(x, dev(c["q"]), [0, 500, 900])
    phi, _ = pl.eval(x, dev(c["q"]))
    pl.status()
    assert np.isfinite(phi.cpu().numpy()).all()
