"""The periodized-sum method for K = 1/r, step by step in FP64 (paper Sec. 2.3
algorithms "set" and "get", specialised to the Laplace kernel in Sec. 3).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

Conventions shared with the product path (both sides implement them on their
own; nothing is shared except the input arrays, such as user check points or
RBF centres):
  * basis R_t(y) = R^_t(y / R0) -- the renormalized solid harmonics of
    eq. (1.7)-(1.8) evaluated at the point scaled by the circumradius, which is
    the same expansion with C_t absorbing R0^n; t = 1 (the constant) is dropped
    from the fit (Sec. 3, null space) and C1 comes from the zero-mean condition
    (eq. (pfx2)-(pfx4) with phi_mean = 0, the Ewald convention of App. D);
  * the least-squares solution is C = A^+ f with the SVD pseudo-inverse that
    keeps singular values above rcond * sigma_max (the paper recommends a
    rank-revealing factorization and gives no tolerance);
  * outputs are the potential phi and the field -grad phi at the targets.
"""
import numpy as np

from . import _native
from .basis import basis as basis_fn
from .boxmean import basis_box_means, box_potential_mean
from .checkpoints import gauss_sphere, partners
from .geometry import circumradius, near_set


class Plan:
    """Algorithm "set" (steps 1-6).

    basis="spherical": the renormalized solid harmonics (Sec. 3.1); p is the
    truncation number and the constant term is fixed by C1.
    basis="rbf": the kernel placed at M given centres outside the box
    (eq. (5), "equivalent sources"), R_t(y) = K(y - x_t); coefficient t = 1 is
    again the constant C1 and C_2.. C_{M+1} multiply the M kernels.  `p` then
    only sets the default Gauss check-point grid."""

    def __init__(self, box, p, R_b=None, lam=None, rcond=1e-13, check_points=None, basis="spherical", centres=None):
        self.box = np.asarray(box, dtype=np.float64)
        self.p = int(p)
        self.kind = basis
        self.R0 = circumradius(self.box)                                    # step 1
        self.R_b = float(R_b) if R_b is not None else float(lam) * self.R0
        self.lam = self.R_b / self.R0
        if check_points is None:
            check_points = gauss_sphere(self.p, self.R0)                    # step 2
        self.yc = np.asarray(check_points, dtype=np.float64)
        self.L = self.yc.shape[0]
        self.yt, self.shift_axis = partners(self.yc, self.box)              # step 3
        if basis == "rbf":
            self.centres = np.asarray(centres, dtype=np.float64)
            self.P = self.centres.shape[0] + 1
            self.A = (_kernel_matrix(self.yc, self.centres) - _kernel_matrix(self.yt, self.centres))  # L x M
        else:
            self.P = self.p * self.p
            Ry = basis_fn(*(self.yc.T / self.R0), self.p)[1:]               # step 4, t = 2..P
            Ryt = basis_fn(*(self.yt.T / self.R0), self.p)[1:]
            self.A = (Ry - Ryt).T                                           # L x (P-1)
        U, s, Vt = np.linalg.svd(self.A, full_matrices=False)               # step 5
        keep = s > rcond * s[0]
        self.sigma = s
        self.rank = int(keep.sum())
        self.cond = s[0] / s[keep][-1]
        self.Apinv = (Vt[keep].T / s[keep][None, :]) @ U[:, keep].T        # (P-1) x L
        if basis == "rbf":
            # box means of K(y - x_t) are the box-mean potentials Phi0(x_t) (App. C)
            self.R0mean = np.concatenate([[1.0], box_potential_mean(self.centres, self.box)])
        else:
            self.R0mean = basis_box_means(self.box, self.p, self.R0)        # step 6 (App. B)

    def far_field(self, C, y0):
        """phi_far and grad phi_far at the points y0 (step 7)."""
        if self.kind == "rbf":
            phif, gf = _native.direct(y0, self.centres, C[1:], grad=True)
            return phif, gf
        Rv, Rg = basis_fn(*(y0.T / self.R0), self.p, grad=True)
        phif = C[1:] @ Rv[1:]
        gf = np.stack([C[1:] @ Rg[k, 1:] for k in range(3)], axis=1) / self.R0
        return phif, gf

    def moments(self, x, q):
        """u_t = sum_k q_k R_t(x_k), t = 2..P (used by the energy gradient)."""
        if self.kind == "rbf":
            return _native.direct(self.centres, x, q, grad=False)
        return basis_fn(*(x.T / self.R0), self.p)[1:] @ q

    # ----- algorithm "get" -----
    def near(self, x, q):
        return near_set(x, q, self.box, self.R_b)                           # steps 1-2

    def solve(self, x, q, targets=None, with_mean=True, return_parts=False):
        """Steps 3-8 at the targets (default: the particles, Y0 = X0).
        Returns (phi, field) with field = -grad phi."""
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y0 = x if targets is None else np.asarray(targets, dtype=np.float64)
        xs, qs, _, _ = self.near(x, q)
        # step 3: near sums at the check points and their partners, and at Y0
        phc = _native.direct(np.concatenate([self.yc, self.yt]), xs, qs, grad=False)
        f = phc[self.L:] - phc[: self.L]                                    # step 4
        C = np.zeros(self.P)
        C[1:] = self.Apinv @ f                                              # step 5
        if with_mean:                                                       # step 6
            S = float(np.sum(qs * box_potential_mean(xs, self.box)))
            C[0] = 0.0 - S - float(C[1:] @ self.R0mean[1:])
        phin, gn = _native.direct(y0, xs, qs, grad=True)
        phif, gf = self.far_field(C, y0)                                    # step 7
        phi = phin + phif + C[0]                                            # step 8
        grad = gn + gf
        if return_parts:
            return dict(phi=phi, field=-grad, phi_near=phin, phi_far=phif, C=C, f=f,
                        grad_near=gn, grad_far=gf, n_near=xs.shape[0])
        return phi, -grad

    def check_sums(self, x, q):
        """phi_near at Y_c1 (first L) then Y_c2 (last L)."""
        xs, qs, _, _ = self.near(x, q)
        return _native.direct(np.concatenate([self.yc, self.yt]), xs, qs, grad=False)


def _kernel_matrix(y, centres):
    """K(y_l - x_t) = 1/|y_l - x_t| for every check point and centre."""
    d = y[:, None, :] - centres[None, :, :]
    return 1.0 / np.sqrt((d * d).sum(axis=2))


def solve(x, q, box, p, R_b=None, lam=None, targets=None, rcond=1e-13, with_mean=True):
    return Plan(box, p, R_b=R_b, lam=lam, rcond=rcond).solve(x, q, targets=targets, with_mean=with_mean)


def energy(plan, x, q):
    """E = (1/2) sum_i q_i phi(x_i)."""
    phi, _ = plan.solve(x, q)
    return 0.5 * float(np.sum(q * phi))
