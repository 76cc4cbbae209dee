"""Gradient of the periodic energy E = (1/2) sum_i q_i phi(x_i) computed by the
method, with respect to the positions x_i and the charges q_i.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The paper has no adjoint; this is the exact derivative of the discrete method
(eqs. (3), (8), (10), (pfx3)-(pfx4)), derived as follows.  Write
E = E_nn + E_ff + E_c with
  E_nn = (1/2) sum_i q_i phi_near(x_i),
  E_ff = (1/2) u^T C,   u_t = sum_k q_k R_t(x_k),   C = A^+ f,
  E_c  = (1/2) C1 sum_i q_i  (zero for neutral charges).
With w = (A^+)^T u, E_ff = (1/2) w^T f and f_l = phi_near(y~_l) - phi_near(y_l)
depends on the near entries z = x_i + p only.  Collecting every place where a
particle enters -- as a target, and as each of its near images -- gives

  dE/dx_i = (1/2) q_i grad phi(x_i) + (1/2) q_i sum_{p: (i,p) near} grad psi(x_i + p)
  dE/dq_i = (1/2) phi(x_i)          + (1/2)     sum_{p: (i,p) near} psi(x_i + p)

where psi(z) = sum_k q_k K(z - x_k) + sum_l w_l [K(z - y~_l) - K(z - y_l)] is
the potential of the base particles plus check-point charges +w_l at the
partners and -w_l at the check points, with K(0) = 0.  C1 drops out of dE/dx
because the charges are neutral; dE/dq is only defined on the neutral set, so it
is returned projected onto sum dq = 0 (its mean removed).  Changes of the near
set when a particle crosses the sphere |x + p| = R_b are jumps, not slopes, and
are not part of the derivative.
"""
import numpy as np

from . import _native


def energy_gradients(plan, x, q):
    """Return (E, dE/dx (N,3), dE/dq (N,), parts) for the oracle plan."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    parts = plan.solve(x, q, return_parts=True)
    phi = parts["phi"]
    grad = -parts["field"]
    E = 0.5 * float(np.sum(q * phi))
    u = plan.moments(x, q)                                          # (P-1,)
    w = plan.Apinv.T @ u                                            # (L,)
    xs, qs, base, _ = plan.near(x, q)
    src = np.concatenate([x, plan.yt, plan.yc])
    srq = np.concatenate([q, w, -w])
    psi, gpsi = _native.direct(xs, src, srq, grad=True)
    dpsi = np.zeros(x.shape[0])
    gsum = np.zeros_like(x)
    np.add.at(dpsi, base, psi)
    np.add.at(gsum, base, gpsi)
    dEdx = 0.5 * q[:, None] * (grad + gsum)
    dEdq = 0.5 * (phi + dpsi)
    dEdq = dEdq - dEdq.mean()
    return E, dEdx, dEdq, parts


def physics_gradients(plan, x, q):
    """The physical approximation dE/dx_i = -q_i field_i, dE/dq_i = phi_i
    (projected onto sum dq = 0)."""
    phi, field = plan.solve(x, q)
    g = phi - phi.mean()
    return -q[:, None] * field, g


def energy_gradients_decay(plan, x, q):
    """The same gradient for a plan whose fit has decay rows (a slab or a wire:
    oracle/slab.py, oracle/wire.py).  With w = (A^+)^T u split into the L
    periodicity weights and the decay-row weights w_r, the decay rows add to
    E_ff = (1/2) w^T f the term (1/2) sum_r w_r f_r, and each f_r is a weighted
    sum over the decay points y_i of E_n(y_i) + c_r phi_near(y_i) (E_n the field
    along the point's normal n_i; c_r = -s|k| on a slab's plane s, beta on the
    wire's cylinder).  Collected per point, a_i = sum_r w_r W_ri and
    b_i = sum_r w_r c_r W_ri, that term is (1/2) sum_j q_j psi_dec(z_j) over the
    near entries z_j with
        psi_dec(z) = sum_i b_i / |z - y_i| + a_i n_i . (y_i - z) / |y_i - z|^3,
    a charge b_i and a dipole -a_i n_i at each decay point; psi_dec joins psi in
    the formulas above.  Returns (E, dE/dx (N,3), dE/dq (N,))."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    parts = plan.solve(x, q, return_parts=True)
    phi = parts["phi"]
    E = 0.5 * float(np.sum(q * phi))
    from .basis import basis as basis_fn
    u = basis_fn(*(x.T / plan.R0), plan.p)[1:] @ q
    w = plan.Apinv.T @ u                                             # (L + n_dec,)
    xs, _, base, _ = plan.near(x, q)
    src = np.concatenate([x, plan.yt, plan.yc])
    srq = np.concatenate([q, w[: plan.L], -w[: plan.L]])
    psi, gpsi = _native.direct(xs, src, srq, grad=True)
    pts, nrm, a, b = plan.decay_sources(w[plan.L:])
    for c0 in range(0, len(xs), 256):
        d = xs[c0:c0 + 256, None, :] - pts[None, :, :]              # z - y_i
        r2 = (d * d).sum(-1)
        ri = 1.0 / np.sqrt(r2)
        ri3 = ri ** 3
        nd = (d * nrm[None, :, :]).sum(-1)                          # n_i . (z - y_i)
        psi[c0:c0 + 256] += (b[None, :] * ri - a[None, :] * nd * ri3).sum(1)
        # grad_z of b/r is -b d/r^3; of -a n.d/r^3 it is -a (n/r^3 - 3 (n.d) d/r^5)
        g = -(b[None, :] * ri3)[:, :, None] * d
        g -= a[None, :, None] * (nrm[None, :, :] * ri3[:, :, None] - 3.0 * (nd * ri3 / r2)[:, :, None] * d)
        gpsi[c0:c0 + 256] += g.sum(1)
    dpsi = np.zeros(x.shape[0])
    gsum = np.zeros_like(x)
    np.add.at(dpsi, base, psi)
    np.add.at(gsum, base, gpsi)
    dEdx = 0.5 * q[:, None] * (-parts["field"] + gsum)
    dEdq = 0.5 * (phi + dpsi)
    return E, dEdx, dEdq - dEdq.mean()
