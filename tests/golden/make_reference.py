"""Write the oracle's reference values for the full-size workloads, and the
independent Ewald potential for the parameter-choice tests of Table 2.

Calls only the FP64 CPU oracle (oracle/) on the seeded inputs of workloads/;
nothing here comes from the HIP library.  The outputs let GPU tests and the
benchmark compare sampled particles at full size without re-running the slow
oracle on the GPU machine.  Usage: python tests/golden/make_reference.py cfg2 [cfg2_hard cfg3 cfg3_hard cfg4 cfg5 table2 table3 screened slab wire plane biharmonic]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.ewald import Ewald  # noqa: E402
from oracle.geometry import lattice_vectors  # noqa: E402
from oracle.method import Plan  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def _save(name, **arrs):
    path = os.path.join(OUT, name)
    np.savez_compressed(path, **arrs)
    print("wrote", path, flush=True)


def cfg2():
    c = W.config2()
    pl = Plan(c["box"], c["p"], R_b=c["R_b"])
    sub = c["subset"]
    parts = pl.solve(c["x"], c["q"], targets=c["x"][sub], return_parts=True)
    _save("ref_cfg2.npz", subset=sub, phi=parts["phi"], field=parts["field"], C=parts["C"], n_near=parts["n_near"])


def hard_targets(x, box, R_b, band=1e-3, nclose=200):
    """Indices of the particles where a defect would hide from a norm over a
    random sample: those with a lattice image within `band` of the near-ball
    sphere |x + p| = R_b (in or out of the near set by a hair), those within
    `band` of a box face, and the `nclose` particles with the closest periodic
    neighbours (the pairs that dominate the field norm)."""
    from scipy.spatial import cKDTree
    d = np.asarray(box, dtype=np.float64)
    sphere = np.zeros(len(x), dtype=bool)
    for p in lattice_vectors(box, R_b):
        sphere |= np.abs(np.linalg.norm(x + p, axis=1) - R_b) < band
    face = np.any(np.abs(x) > 0.5 * d - band, axis=1)
    tree = cKDTree(np.mod(x + 0.5 * d, d), boxsize=d)
    dist, _ = tree.query(np.mod(x + 0.5 * d, d), k=2)
    close = np.argsort(dist[:, 1], kind="stable")[:nclose]
    pick = {"sphere": np.nonzero(sphere)[0], "face": np.nonzero(face)[0], "close": np.sort(close)}
    return pick


def _hard(name, c, plan, extra, band=1e-3, nclose=200, cap=None, seed=0):
    """Reference values at the hard targets (capped per kind by a seeded
    choice) plus `extra` seeded random particles."""
    R_b = plan.R_b
    kinds = hard_targets(c["x"], c["box"], R_b, band, nclose)
    g = np.random.Generator(np.random.PCG64(seed))
    out = {}
    allidx = []
    for k, idx in kinds.items():
        if cap is not None and len(idx) > cap:
            idx = np.sort(g.choice(idx, size=cap, replace=False))
        out["idx_" + k] = idx
        allidx.append(idx)
    rand = np.sort(g.choice(len(c["q"]), size=extra, replace=False)) if extra else np.zeros(0, dtype=np.int64)
    out["idx_random"] = rand
    allidx.append(rand)
    sub = np.unique(np.concatenate(allidx))
    phi, field = plan.solve(c["x"], c["q"], targets=c["x"][sub])
    out.update(subset=sub, phi=phi, field=field)
    print(name, {k: len(v) for k, v in out.items() if k.startswith("idx_")}, "targets", len(sub), flush=True)
    _save(name, **out)


def cfg2_hard():
    """Uniform cube, N = 1e5: 20,000 random particles and the hard targets."""
    c = W.config2()
    _hard("ref_cfg2_hard.npz", c, Plan(c["box"], c["p"], R_b=c["R_b"]), extra=20000, seed=2202)


def cfg3_hard():
    """Clustered box 1 x 1 x 2.5, N = 1e6: the hard targets (at most 300 of each kind)."""
    c = W.config3()
    _hard("ref_cfg3_hard.npz", c, Plan(c["box"], c["p"], lam=c["lam"]), extra=0, cap=300, seed=3303)


def cfg3():
    c = W.config3()
    pl = Plan(c["box"], c["p"], lam=c["lam"])
    sub = c["subset"]
    parts = pl.solve(c["x"], c["q"], targets=c["x"][sub], return_parts=True)
    _save("ref_cfg3.npz", subset=sub, phi=parts["phi"], field=parts["field"], C=parts["C"], n_near=parts["n_near"])


def cfg4(nsample=300):
    c = W.config4()
    n = np.array([len(s["q"]) for s in c["systems"]])
    order = np.argsort(n)
    pick = np.unique(np.concatenate([order[:2], order[len(n) // 2 - 1: len(n) // 2 + 1], order[-2:]]))
    out = {"systems": pick}
    for k in pick:
        s = c["systems"][k]
        g = np.random.Generator(np.random.PCG64(1000 + int(k)))
        sub = np.sort(g.choice(len(s["q"]), size=min(nsample, len(s["q"])), replace=False))
        pl = Plan(s["box"], c["p"], lam=c["lam"])
        phi, field = pl.solve(s["x"], s["q"], targets=s["x"][sub])
        out["sub_%d" % k] = sub
        out["phi_%d" % k] = phi
        out["field_%d" % k] = field
    _save("ref_cfg4.npz", **out)


def cfg5(nsample=200):
    c = W.config5()
    g = np.random.Generator(np.random.PCG64(555))
    sub = np.sort(g.choice(len(c["q"]), size=nsample, replace=False))
    pl = Plan(c["box"], c["p"], R_b=c["R_b"])
    phi, field = pl.solve(c["x"], c["q"], targets=c["x"][sub])
    # unjittered lattice: every site is equivalent, so two sites (one per sign) suffice
    r = W.rocksalt(32)
    lphi, lfield = pl.solve(r["x"], r["q"], targets=r["x"][:2])
    _save("ref_cfg5.npz", subset=sub, phi=phi, field=field, lattice_phi=lphi, lattice_q=r["q"][:2])


def table2():
    """Sec. 4.2, Tables 2 and 4: 27,000 charges +-1 on a 30^3 grid in the unit cube.
    The classical Ewald sum (O2) at 2,000 seeded sample charges, the reference for
    the relative L2 error eps_2 of eq. (st2), and the method (O1) there for the
    parameters of the GPU tests."""
    x, q = W.grid_charges(30, 2)
    sub = np.sort(W.rng(7).choice(len(q), 2000, replace=False))
    phi, _ = Ewald((1.0, 1.0, 1.0)).solve(x, q, targets=x[sub])
    out = dict(subset=sub, phi_ewald=phi)
    for lam, p in TABLE2_CASES:   # the method (O1) at Table 2's p_min, for GPU parity
        out["phi_method_%g_%d" % (lam, p)], _ = Plan((1.0, 1.0, 1.0), p, lam=lam).solve(x, q, targets=x[sub])
    # Table 4: lambda = 1.5, p = 16, spherical basis and 256 Thomson RBF centres on S_b
    out["phi_table4_spherical"], _ = Plan((1.0, 1.0, 1.0), 16, lam=1.5).solve(x, q, targets=x[sub])
    cen = W.thomson_points(256, 1.5 * np.sqrt(3) / 2)
    out["phi_table4_rbf"], _ = Plan((1.0, 1.0, 1.0), 16, lam=1.5, basis="rbf", centres=cen).solve(x, q, targets=x[sub])
    _save("ref_table2.npz", **out)


TABLE2_CASES = ((1.3, 34), (1.5, 24), (1.7, 19))


def table3():
    """Sec. 4.2, Table 3: 216,000 charges +-1 on a 60^3 grid in the unit cube; the
    Ewald sum (O2) and the method (O1) at Table 3's p_min, at 2,000 sampled charges."""
    x, q = W.grid_charges(60, 3)
    sub = np.sort(W.rng(8).choice(len(q), 2000, replace=False))
    phi, _ = Ewald((1.0, 1.0, 1.0)).solve(x, q, targets=x[sub])
    out = dict(subset=sub, phi_ewald=phi)
    for lam, p in TABLE3_CASES:
        out["phi_method_%g_%d" % (lam, p)], _ = Plan((1.0, 1.0, 1.0), p, lam=lam).solve(x, q, targets=x[sub])
        print("table3 lam %g p %d eps_2 %.3e" % (lam, p, np.linalg.norm(out["phi_method_%g_%d" % (lam, p)] - phi)
                                                    / np.linalg.norm(phi)), flush=True)
    _save("ref_table3.npz", **out)


TABLE3_CASES = ((1.3, 34), (1.5, 25), (1.7, 19))


def screened():
    """The screened-kernel workload (workloads.config_screened) at its sampled particles."""
    from oracle.screened import ScreenedPlan
    c = W.config_screened()
    pl = ScreenedPlan(c["box"], c["kappa"], c["centres"], c["p"], lam=c["lam"])
    sub = c["subset"]
    parts = pl.solve(c["x"], c["q"], targets=c["x"][sub], return_parts=True)
    _save("ref_screened.npz", subset=sub, phi=parts["phi"], field=parts["field"], C=parts["C"],
          n_near=parts["n_near"])


def _partial(periodic, name):
    from oracle.slab import SlabPlan
    from oracle.wire import WirePlan
    c = W.config_partial(periodic)
    pl = (SlabPlan if periodic == "xy" else WirePlan)(c["box"], c["p"], lam=c["lam"])
    sub = c["subset"]
    parts = pl.solve(c["x"], c["q"], targets=c["x"][sub], return_parts=True)
    _save(name, subset=sub, phi=parts["phi"], field=parts["field"], C=parts["C"], n_near=parts["n_near"])


def slab():
    """The slab workload (workloads.config_partial("xy")) at its sampled particles."""
    _partial("xy", "ref_slab.npz")


def wire():
    """The wire workload (workloads.config_partial("x")) at its sampled particles."""
    _partial("x", "ref_wire.npz")


def plane():
    """The plane workload (workloads.config_plane) at its sampled particles."""
    from oracle.twod import Plan2D
    c = W.config_plane()
    pl = Plan2D(c["box"], c["p"], lam=c["lam"])
    sub = c["subset"]
    parts = pl.solve(c["x"], c["q"], targets=c["x"][sub], return_parts=True)
    _save("ref_plane.npz", subset=sub, phi=parts["phi"], field=parts["field"], C=parts["C"], n_near=parts["n_near"])


def biharmonic():
    """The biharmonic workload (workloads.config_biharmonic) at its sampled particles."""
    from oracle.biharmonic import BiharmonicPlan
    c = W.config_biharmonic()
    pl = BiharmonicPlan(c["box"], c["p"], lam=c["lam"])
    sub = c["subset"]
    parts = pl.solve(c["x"], c["q"], targets=c["x"][sub], return_parts=True)
    _save("ref_biharmonic.npz", subset=sub, phi=parts["phi"], field=parts["field"], C=parts["C"],
          n_near=parts["n_near"])


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cfg2"]:
        t = time.time()
        globals()[name]()
        print(name, "%.1fs" % (time.time() - t), flush=True)
