"""The method for the screened Coulomb kernel K(r) = exp(-kappa r)/r, and an
independent Ewald-type reference for its periodic sum.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The paper presents the periodization for any kernel that has a fast summation
algorithm, whose periodic sum makes sense and that can be expanded over a local
basis (Sec. 1; Sec. 2), and works the details out for the Laplace kernel
(Sec. 3).  This module is the reading used here for the screened Coulomb
(Yukawa) kernel, the Green's function of the modified Helmholtz operator
Delta - kappa^2 (up to 4 pi), step for step as in algorithm "set"/"get"
(Sec. 2.3):

  * the lattice sum converges absolutely (the kernel decays exponentially), so
    the charges need not be neutral and the summation order does not matter;
  * basis: the kernel itself at M given centres outside the ball S_b (eq. (5),
    "equivalent sources"), R_t(y) = K(y - c_t), t = 1..M.  The operator
    Delta - kappa^2 has no nonzero bounded periodic solution (its Fourier symbol
    -(|k|^2 + kappa^2) never vanishes), so the periodicity rows have no null
    space: every coefficient comes from the fit, with no constant term and no
    zero-mean condition (contrast the Laplace kernel, Sec. 3);
  * steps 1-3 (near set, check points, partners), 5 (SVD pseudo-inverse with
    the same rcond) and 7-8 as for 1/r; K(0) = 0 for coincident points.

Reference: the kernel is the integral
    K(r) = (2/sqrt(pi)) int_0^inf exp(-r^2 t^2 - kappa^2/(4 t^2)) dt;
splitting it at t = alpha gives a real-space part (t > alpha, in closed form
with erfc, summed over images within a cut-off) and a smooth part whose
lattice sum is, by Poisson summation, the Fourier series
    (4 pi / V) sum_k exp(-(k^2 + kappa^2)/(4 alpha^2)) / (k^2 + kappa^2) e^{i k.r}
over every reciprocal vector, k = 0 included.  The smooth part at r = 0,
    (2 alpha/sqrt(pi)) exp(-kappa^2/(4 alpha^2)) - kappa erfc(kappa/(2 alpha)),
is removed for coincident points.  The result does not depend on alpha.
"""
import math

import numpy as np

from . import _native
from .checkpoints import gauss_sphere, partners
from .geometry import circumradius, near_set


def kernel_matrix(y, centres, kappa):
    """K(y_i - c_t) for points y and centres c: (len(y), len(c))."""
    d = np.asarray(y, dtype=np.float64)[:, None, :] - np.asarray(centres, dtype=np.float64)[None, :, :]
    r = np.sqrt((d * d).sum(2))
    return np.exp(-kappa * r) / r


class ScreenedPlan:
    """Algorithm "set" for K = exp(-kappa r)/r with the kernel-at-centres basis."""

    def __init__(self, box, kappa, centres, p, R_b=None, lam=None, rcond=1e-13, check_points=None):
        self.box = np.asarray(box, dtype=np.float64)
        self.kappa = float(kappa)
        self.p = int(p)
        self.R0 = circumradius(self.box)                                    # step 1
        self.R_b = float(R_b) if R_b is not None else float(lam) * self.R0
        if check_points is None:
            check_points = gauss_sphere(self.p, self.R0)                    # step 2
        self.yc = np.asarray(check_points, dtype=np.float64)
        self.L = self.yc.shape[0]
        self.yt, self.shift_axis = partners(self.yc, self.box)              # step 3
        self.centres = np.asarray(centres, dtype=np.float64)
        self.M = self.centres.shape[0]
        self.A = kernel_matrix(self.yc, self.centres, self.kappa) - kernel_matrix(self.yt, self.centres, self.kappa)
        U, s, Vt = np.linalg.svd(self.A, full_matrices=False)               # step 5
        keep = s > rcond * s[0]
        self.rank = int(keep.sum())
        self.cond = s[0] / s[keep][-1]
        self.Apinv = (Vt[keep].T / s[keep][None, :]) @ U[:, keep].T        # M x L

    def near(self, x, q):
        return near_set(x, q, self.box, self.R_b)

    def solve(self, x, q, targets=None, return_parts=False):
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y0 = x if targets is None else np.asarray(targets, dtype=np.float64)
        xs, qs, _, _ = self.near(x, q)                                      # steps 1-2
        ph = _native.direct_screened(np.concatenate([self.yc, self.yt]), xs, qs, self.kappa, grad=False)
        f = ph[self.L:] - ph[: self.L]                                      # steps 3-4
        C = self.Apinv @ f                                                  # step 5
        phin, gn = _native.direct_screened(y0, xs, qs, self.kappa)         # step 3 at y0
        phif, gf = _native.direct_screened(y0, self.centres, C, self.kappa)  # step 7
        phi = phin + phif                                                   # step 8
        field = -(gn + gf)
        if return_parts:
            return dict(phi=phi, field=field, C=C, f=f, n_near=xs.shape[0])
        return phi, field


def energy_gradients_screened(plan, x, q):
    """E = (1/2) sum_i q_i phi(x_i) for the screened method and its exact gradient,
    derived as for the Coulomb method (oracle/adjoint.py) with the moments
    u_t = sum_k q_k K(c_t - x_k) at the centres, w = (A^+)^T u, and
    psi(z) = sum_k q_k K(z - x_k) + sum_l w_l [K(z - y~_l) - K(z - y_l)]:
      dE/dx_i = (1/2) q_i grad phi(x_i) + (1/2) q_i sum_{p: (i,p) near} grad psi(x_i + p),
      dE/dq_i = (1/2) phi(x_i)          + (1/2)     sum_{p: (i,p) near} psi(x_i + p).
    There is no constant and the charges need not be neutral, so dE/dq is not
    projected.  Returns (E, dE/dx (N,3), dE/dq (N,))."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    phi, field = plan.solve(x, q)
    E = 0.5 * float(np.sum(q * phi))
    u = _native.direct_screened(plan.centres, x, q, plan.kappa, grad=False)
    w = plan.Apinv.T @ u
    xs, _, base, _ = plan.near(x, q)
    src = np.concatenate([x, plan.yt, plan.yc])
    srq = np.concatenate([q, w, -w])
    psi, gpsi = _native.direct_screened(xs, src, srq, plan.kappa)
    dpsi = np.zeros(x.shape[0])
    gsum = np.zeros_like(x)
    np.add.at(dpsi, base, psi)
    np.add.at(gsum, base, gpsi)
    return E, 0.5 * q[:, None] * (-field + gsum), 0.5 * (phi + dpsi)


class EwaldScreened:
    """Periodic sum of exp(-kappa r)/r by the split described above."""

    def __init__(self, box, kappa, alpha=None, tol=1e-16):
        self.box = np.asarray(box, dtype=np.float64)
        self.kappa = float(kappa)
        self.alpha = float(alpha) if alpha is not None else 5.0 / float(self.box.min())
        a = math.sqrt(-math.log(tol))
        b = self.kappa / (2.0 * self.alpha)
        self.rcut = (a + b) / self.alpha
        self.kmax = 2.0 * self.alpha * a
        self.V = float(np.prod(self.box))
        nmax = np.ceil(self.kmax * self.box / (2 * np.pi)).astype(int)
        g = [np.arange(-n, n + 1) for n in nmax]
        N1, N2, N3 = np.meshgrid(*g, indexing="ij")
        n = np.stack([N1.ravel(), N2.ravel(), N3.ravel()], axis=1)
        k = 2 * np.pi * n / self.box[None, :]
        k2 = (k * k).sum(1)
        sel = k2 <= self.kmax ** 2
        self.k = k[sel]
        k2 = k2[sel] + self.kappa ** 2
        self.w = (4 * np.pi / self.V) * np.exp(-k2 / (4 * self.alpha ** 2)) / k2
        m = np.ceil(self.rcut / self.box + 1.0).astype(int)
        gi = [np.arange(-v, v + 1) for v in m]
        I1, I2, I3 = np.meshgrid(*gi, indexing="ij")
        self.shifts = np.stack([I1.ravel(), I2.ravel(), I3.ravel()], axis=1) * self.box[None, :]
        self.self_term = (2 * self.alpha / math.sqrt(math.pi)) * math.exp(-b * b) - self.kappa * math.erfc(b)

    def solve(self, x, q, targets=None):
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y = x if targets is None else np.asarray(targets, dtype=np.float64)
        phi1, g1 = _native.ewald_screened_real(y, x, q, self.shifts, self.kappa, self.alpha, self.rcut)
        self_q = np.zeros(y.shape[0])
        if targets is None:
            self_q = q.copy()
        else:
            for j in range(x.shape[0]):
                same = np.all(y == x[j][None, :], axis=1)
                self_q[same] += q[j]
        ph = self.k @ x.T
        sre = np.cos(ph) @ q
        sim = np.sin(ph) @ q
        phi2, g2 = _native.ewald_recip(y, self.k, self.w, sre, sim)
        return phi1 + phi2 - self.self_term * self_q, -(g1 + g2)


def lattice_sum(x, q, box, kappa, targets=None, tol=1e-17):
    """Brute force: the sum over every image whose box comes within R of the
    cell, R chosen so that exp(-kappa R)/R < tol (terms beyond it are smaller)."""
    box = np.asarray(box, dtype=np.float64)
    R = 1.0
    while math.exp(-kappa * R) / R > tol:
        R *= 1.1
    m = np.ceil(R / box + 1.0).astype(int)
    gi = [np.arange(-v, v + 1) for v in m]
    I1, I2, I3 = np.meshgrid(*gi, indexing="ij")
    shifts = np.stack([I1.ravel(), I2.ravel(), I3.ravel()], axis=1) * box[None, :]
    keep = np.sqrt((np.maximum(np.abs(shifts) - box[None, :], 0.0) ** 2).sum(1)) <= R
    y = np.asarray(x, dtype=np.float64) if targets is None else np.asarray(targets, dtype=np.float64)
    phi, g = _native.direct_screened(y, x, q, kappa, shifts=shifts[keep])
    return phi, -g
