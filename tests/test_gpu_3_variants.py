"""Check-point and basis variants (caller-given and Thomson check points, the
RBF basis of eq. (5)), the accuracy settings of Tables 2-4, and parameter
selection (Sec. 3.3): the HIP path against the FP64 CPU oracle and the
oracle's independent Ewald sum.
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


# The RBF fitting matrix is far less well conditioned (cond(A) ~ 1e6 for 256
# centres at p = 16) than the renormalized spherical basis (~10), yet the
# potentials and fields of two correct FP64 pseudo-inverses agree to ~1e-13
# (measured on the GPU): the FP64 bar is the same 1e-12 as for every other form.
TOL_RBF = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rbf_basis_matches_oracle(ps, prec):
    c = W.config1()
    cen = W.fibonacci_sphere(256, 1.5)
    op = OPlan(c["box"], 16, R_b=1.5, basis="rbf", centres=cen)
    ref = op.solve(c["x"], c["q"], return_parts=True)
    pl = ps.Plan(c["box"], 16, R_b=1.5, precision=prec, n_max=1000, centres=cen)
    phi, field = pl.eval(dev(c["x"].T), dev(c["q"]))
    pl.status()
    e1, e2 = err(phi.cpu().numpy(), ref["phi"]), err(field.cpu().numpy().T, ref["field"])
    print(prec, "rbf err phi %.3e field %.3e cond %.3e" % (e1, e2, op.cond))
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
    phi, field = pl.eval(dev(x.T), dev(q))
    pl.status()
    assert pl.info()["L"] == 432
    assert err(phi.cpu().numpy(), ref[0]) <= TOL[prec]
    assert err(field.cpu().numpy().T, ref[1]) <= TOL[prec]


def test_rbf_energy_adjoint_matches_oracle(ps):
    box = (1.0, 1.0, 1.0)
    x, q = W.uniform_box(500, box, charges="gauss", seed=5)
    cen = W.fibonacci_sphere(120, 1.5)
    op = OPlan(box, 10, R_b=1.5, basis="rbf", centres=cen)
    E, dx, dq, _ = energy_gradients(op, x, q)
    pl = ps.Plan(box, 10, R_b=1.5, n_max=500, centres=cen)
    xt, qt = dev(x.T), dev(q)
    e = pl.energy(xt, qt)
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, gq = pl.energy_vjp(xt, qt, one, exact=True)
    print("rbf adjoint: E %.3e dx %.3e dq %.3e" % (abs(float(e.cpu()[0]) - E) / abs(E), err(gx.cpu().numpy().T, dx),
                                                   err(gq.cpu().numpy(), dq)))
    assert abs(float(e.cpu()[0]) - E) <= 1e-12 * abs(E)
    assert err(gx.cpu().numpy().T, dx) <= 1e-12
    assert err(gq.cpu().numpy(), dq) <= 1e-12


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
    phi, field = bp.eval(dev(np.concatenate(xs).T), dev(np.concatenate(qs)), off)
    bp.status()
    phi, field = phi.cpu().numpy(), field.cpu().numpy().T
    r0 = OPlan(boxes[0], 12, lam=lam).solve(xs[0], qs[0])
    r1 = OPlan(boxes[1], 12, lam=lam, basis="rbf", centres=cen).solve(xs[1], qs[1])
    assert err(phi[off[0]:off[1]], r0[0]) <= 1e-12 and err(field[off[0]:off[1]], r0[1]) <= 1e-12
    print("mixed bases, RBF box: phi %.3e field %.3e" % (err(phi[off[1]:off[2]], r1[0]), err(field[off[1]:off[2]], r1[1])))
    assert err(phi[off[1]:off[2]], r1[0]) <= 1e-12 and err(field[off[1]:off[2]], r1[1]) <= 1e-12


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
        phi, field = pl.eval(dev(x.T), dev(q))
        pl.status()
        assert err(phi.cpu().numpy(), ref[0]) <= tol
        assert err(field.cpu().numpy().T, ref[1]) <= tol


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
    phi, _ = pl.eval(dev(x.T), dev(q))
    pl.status()
    ph = phi.cpu().numpy()[sub]
    assert rel(ph, ref["phi_ewald"]) < 5e-7
    assert err(ph, ref["phi_method_%g_%d" % (lam, p)]) <= TOL["fp64"]


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
    phi, _ = pl.eval(dev(x.T), dev(q))
    pl.status()
    ph = phi.cpu().numpy()[sub]
    assert rel(ph, ref["phi_ewald"]) < 5e-7
    assert err(ph, ref["phi_method_%g_%d" % (lam, p)]) <= TOL["fp64"]


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
        phi, _ = pl.eval(dev(x.T), dev(q))
        pl.status()
        ph = phi.cpu().numpy()[sub]
        e2 = rel(ph, ref["phi_ewald"])
        assert gold[name] / 2 < e2 < gold[name] * 2, (name, e2)
        assert err(ph, ref["phi_table4_" + name]) <= tol


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
    xt, qt = dev(x.T), dev(q)
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
        return rel(phi.cpu().numpy()[sub], ref["phi_ewald"])

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
    xt, qt = dev(x.T), dev(q)
    tol = 1e-5
    best, rows = ps.select_parameters(box, xt, qt, tol, lambdas=(1.2, 1.5), precision="fp32", p_ref=30)
    assert best is not None and best["err_prec"] <= tol
    refp = ps.Plan(box, 30, lam=1.5, precision="fp64", n_max=len(q))
    phi_ref = refp.eval(xt, qt)[0].cpu().numpy()
    for r in rows:
        assert r["p"] > 2 and r["err"] <= tol
        pl = ps.Plan(box, r["p"] - 1, lam=r["lambda"], precision="fp64", n_max=len(q))
        phi = pl.eval(xt, qt)[0].cpu().numpy()
        assert rel(phi, phi_ref) > tol
