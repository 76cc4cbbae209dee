"""Pins for the oracle's exact energy gradients (derived from eqs. (3), (8), (10),
(pfx3)-(pfx4)) against central finite differences of the oracle energy."""
import numpy as np
import pytest

import workloads as W
from oracle.adjoint import energy_gradients, physics_gradients
from oracle.method import Plan, energy


def _safe_particles(plan, x, n, margin=1e-3):
    """Particles whose images all stay clear of the sphere |x + p| = R_b, so a
    step of 1e-5 does not change the near set."""
    from oracle.geometry import lattice_vectors
    P = lattice_vectors(plan.box, plan.R_b)
    d = np.abs(np.linalg.norm(x[:, None, :] + P[None, :, :], axis=2) - plan.R_b).min(axis=1)
    return np.nonzero(d > margin)[0][:n]


@pytest.mark.parametrize("box,p", [((1.0, 1.0, 1.0), 12), ((1.1, 0.9, 1.4), 10)])
def test_position_gradient_matches_central_differences(box, p):
    x, q = W.uniform_box(40, box, charges="gauss", seed=p)
    pl = Plan(box, p, lam=np.sqrt(3))
    _, dEdx, _, _ = energy_gradients(pl, x, q)
    h = 1e-5
    for i in _safe_particles(pl, x, 4):
        for k in range(3):
            xp = x.copy()
            xp[i, k] += h
            xm = x.copy()
            xm[i, k] -= h
            fd = (energy(pl, xp, q) - energy(pl, xm, q)) / (2 * h)
            assert abs(dEdx[i, k] - fd) < 1e-7 * max(1.0, abs(fd))


def test_charge_gradient_matches_neutral_differences():
    box = (1.0, 1.0, 1.0)
    x, q = W.uniform_box(40, box, charges="gauss", seed=4)
    pl = Plan(box, 12, R_b=1.5)
    _, _, dEdq, _ = energy_gradients(pl, x, q)
    assert abs(dEdq.sum()) < 1e-12 * np.abs(dEdq).sum()
    h = 1e-5
    for i, j in [(0, 1), (2, 30), (11, 39)]:
        qp = q.copy()
        qp[i] += h
        qp[j] -= h
        qm = q.copy()
        qm[i] -= h
        qm[j] += h
        fd = (energy(pl, x, qp) - energy(pl, x, qm)) / (2 * h)
        assert abs((dEdq[i] - dEdq[j]) - fd) < 1e-8 * max(1.0, abs(fd))


def test_exact_and_physical_gradients_agree_to_method_error():
    box = (1.0, 1.0, 1.0)
    x, q = W.uniform_box(60, box, charges="gauss", seed=5)
    pl = Plan(box, 16, R_b=1.5)
    _, dx, dq, _ = energy_gradients(pl, x, q)
    px, pq = physics_gradients(pl, x, q)
    assert np.linalg.norm(dx - px) / np.linalg.norm(dx) < 1e-5
    assert np.linalg.norm(dq - pq) / np.linalg.norm(dq) < 1e-5


def test_rbf_adjoint_matches_finite_differences():
    import workloads
    box = (1.0, 1.0, 1.0)
    x, q = W.uniform_box(30, box, charges="gauss", seed=41)
    pl = Plan(box, 10, R_b=1.5, basis="rbf", centres=workloads.fibonacci_sphere(100, 1.5))
    _, dEdx, dEdq, _ = energy_gradients(pl, x, q)
    h = 1e-5
    for i in _safe_particles(pl, x, 3):
        for k in range(3):
            xp = x.copy()
            xp[i, k] += h
            xm = x.copy()
            xm[i, k] -= h
            fd = (energy(pl, xp, q) - energy(pl, xm, q)) / (2 * h)
            assert abs(dEdx[i, k] - fd) < 1e-6 * max(1.0, abs(fd))
    qp, qm = q.copy(), q.copy()
    qp[0] += h
    qp[1] -= h
    qm[0] -= h
    qm[1] += h
    fd = (energy(pl, x, qp) - energy(pl, x, qm)) / (2 * h)
    assert abs((dEdq[0] - dEdq[1]) - fd) < 1e-7 * max(1.0, abs(fd))
