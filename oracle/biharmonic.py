"""The method for the biharmonic kernel K(r) = r, and an independent Ewald-type
reference for its periodic sum.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The paper works the method out for the Laplace kernel and remarks (Sec. 3,
null space of A) that other equations, the biharmonic one among them, share
its rank deficiency: the constant is a periodic solution of the homogeneous
equation, so the fit determines every coefficient but the constant one.  This
module is the reading used here for K(r) = r, the free-space Green's function
of the biharmonic operator (Delta^2 r = -8 pi delta), step for step as in
algorithm "set"/"get" (Sec. 2.3):

  * the periodic sum exists for neutral charges: the periodic problem
    Delta^2 phi = -8 pi sum q delta has a solution only when the source has zero
    mean; it is then unique up to a constant, fixed here (as for 1/r,
    eq. (pfx3)) by a zero box mean;
  * basis: the potential of the far images is biharmonic inside S_b, so by
    Almansi's representation it is h1 + |y|^2 h2 with h1, h2 harmonic.  The
    basis is the renormalized solid harmonics of degrees 0..p-1 (eqs.
    (1.6)-(1.8)) at y/R0 followed by |y/R0|^2 times those of degrees 0..p-3,
    P = p^2 + (p-2)^2 terms, all polynomials of degree <= p-1.  The constant
    (t = 1) is dropped from the fit (null space) and C1 comes from the zero
    box mean;
  * steps 1-3 (near set, Gauss check points, partners), 5 (SVD pseudo-inverse
    with the same rcond) and 7-8 as for 1/r; K(0) = 0 (which r gives anyway);
  * step 4, the fit: periodicity of the values at the check pairs (eq. (8))
    does not fix a biharmonic function -- a fourth-order operator needs more
    than values on the sphere (for instance (|u|^2 - 1) h with h harmonic
    vanishes on it), and measured, the value rows alone leave A rank deficient
    and the result off by 1e-2 at every p.  So each check pair also asks for the
    same gradient: with u = y/R0, rows L + k L + l are
    d/du_k B_t(u_l) - d/du_k B_t(u~_l) with right-hand side
    d/du_k phi_near(u~_l) - d/du_k phi_near(u_l), k = x, y, z (4L rows in all);
  * step 6: the box mean of a near entry's r is Psi0(x) = (1/V0) int |y - x| dV,
    evaluated in closed form from a corner primitive (box_distance_mean); the
    box means of the polynomial basis by tensor Gauss-Legendre, exact.

Reference (EwaldBih): r = S(r) - 1/(2 alpha^2 r) + m(r), m = r smoothed by the
normalized Gaussian exp(-alpha^2 r^2), whose Fourier transform is
-8 pi exp(-k^2/(4 alpha^2))/k^4; S (oracle/pairs.c) decays like a Gaussian and is
summed over images in real space, the 1/r part is the Coulomb Ewald sum
(oracle/ewald.py) times -1/(2 alpha^2), and m's lattice sum is its Fourier
series without k = 0.  Coincident points take S(0) = -2/(alpha sqrt(pi)) (the
limit of S - 1/(2 alpha^2 r)); m(0) is in the Fourier series.  Each part has
zero mean for neutral charges, so the sum has, and the result does not depend
on alpha.  Independent of the expansion: Delta phi = 2 phi_Coulomb, since
Delta r = 2/r and both periodic functions have zero mean.
"""
import math

import numpy as np

from . import _native
from .basis import basis as sh_basis
from .checkpoints import gauss_sphere, partners
from .ewald import Ewald
from .geometry import circumradius, near_set


def n_basis(p):
    """P = p^2 + (p-2)^2: harmonics of degree <= p-1 and |y|^2 times degree <= p-3."""
    return p * p + (p - 2) * (p - 2)


def basis_bh(y, p, R0, grad=False):
    """The biharmonic basis at points y (n, 3): values (P, n); with grad=True also
    d/dy, (3, P, n)."""
    s = np.asarray(y, dtype=np.float64).T / R0
    q2 = (p - 2) * (p - 2)
    if not grad:
        H = sh_basis(s[0], s[1], s[2], p)
        return np.concatenate([H, (s * s).sum(0)[None, :] * H[:q2]])
    H, dH = sh_basis(s[0], s[1], s[2], p, grad=True)
    s2 = (s * s).sum(0)
    val = np.concatenate([H, s2[None, :] * H[:q2]])
    g = np.empty((3,) + val.shape)
    for k in range(3):
        g[k] = np.concatenate([dH[k], s2[None, :] * dH[k][:q2] + 2.0 * s[k][None, :] * H[:q2]]) / R0
    return val, g


def basis_box_means_bh(box, p, R0):
    """(1/V0) int_{Omega0} B_t dV: tensor Gauss-Legendre with floor((p-1)/2) + 1
    nodes per axis, exact for the polynomials of degree <= p-1 (as App. B)."""
    d = np.asarray(box, dtype=np.float64)
    nq = (p - 1) // 2 + 1
    xg, wg = np.polynomial.legendre.leggauss(nq)
    X, Y, Z = np.meshgrid(xg, xg, xg, indexing="ij")
    W = (wg[:, None, None] * wg[None, :, None] * wg[None, None, :]).reshape(-1)
    pts = np.stack([0.5 * d[0] * X.reshape(-1), 0.5 * d[1] * Y.reshape(-1), 0.5 * d[2] * Z.reshape(-1)], axis=1)
    return (basis_bh(pts, p, R0) * W[None, :]).sum(axis=1) / 8.0


def _ln_sum(a, b, c):
    """log(c + sqrt(a^2 + b^2 + c^2)), with the sum formed as (a^2 + b^2)/(r - c)
    for c < 0; 0 where the argument vanishes (its coefficient vanishes there)."""
    r = np.sqrt(a * a + b * b + c * c)
    den = np.where(r - c == 0.0, 1.0, r - c)
    s = np.where(c >= 0.0, c + r, (a * a + b * b) / den)
    return np.where(s > 0.0, np.log(np.where(s > 0.0, s, 1.0)), 0.0)


def _atan_term(a, b, c):
    """a^4 atan(b c / (a r)), 0 at a = 0."""
    r = np.sqrt(a * a + b * b + c * c)
    den = np.where(a * r == 0.0, 1.0, a * r)
    return np.where(a == 0.0, 0.0, a ** 4 * np.arctan(b * c / den))


def corner_primitive(x, y, z):
    """F with d^3 F / (dx dy dz) = sqrt(x^2 + y^2 + z^2):
    F = xyz r/4 + (1/6) [xy (x^2 + y^2) ln(z + r) + yz (y^2 + z^2) ln(x + r)
        + zx (z^2 + x^2) ln(y + r)] - (1/12) [x^4 atan(yz/(xr)) + y^4 atan(zx/(yr))
        + z^4 atan(xy/(zr))].
    (From int r dV = (1/4) closed integral of r (x . n) dS, each face integral of
    sqrt(a^2 + u^2 + v^2) in closed form.)"""
    r = np.sqrt(x * x + y * y + z * z)
    t = x * y * z * r / 4.0
    t = t + (x * y * (x * x + y * y) * _ln_sum(x, y, z) + y * z * (y * y + z * z) * _ln_sum(y, z, x)
             + z * x * (z * z + x * x) * _ln_sum(z, x, y)) / 6.0
    t = t - (_atan_term(x, y, z) + _atan_term(y, z, x) + _atan_term(z, x, y)) / 12.0
    return t


def box_distance_mean(xs, box):
    """Psi0(x) = (1/V0) int_{Omega0} |y - x| dV(y): the triple difference of the
    corner primitive over the corners of Omega0 - x."""
    xs = np.atleast_2d(np.asarray(xs, dtype=np.float64))
    d = np.asarray(box, dtype=np.float64)
    tot = np.zeros(xs.shape[0])
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                sgn = (-1.0) ** (a + b + c + 1)  # + at the upper corner (1, 1, 1)
                X = (a - 0.5) * d[0] - xs[:, 0]
                Y = (b - 0.5) * d[1] - xs[:, 1]
                Z = (c - 0.5) * d[2] - xs[:, 2]
                tot += sgn * corner_primitive(X, Y, Z)
    return tot / float(np.prod(d))


class BiharmonicPlan:
    """Algorithm "set" for K = r with the Almansi basis (see the module notes)."""

    def __init__(self, box, p, R_b=None, lam=None, rcond=1e-13, check_points=None):
        self.box = np.asarray(box, dtype=np.float64)
        self.p = int(p)
        self.R0 = circumradius(self.box)                                    # step 1
        self.R_b = float(R_b) if R_b is not None else float(lam) * self.R0
        if check_points is None:
            check_points = gauss_sphere(self.p, self.R0)                    # step 2
        self.yc = np.asarray(check_points, dtype=np.float64)
        self.L = self.yc.shape[0]
        self.yt, self.shift_axis = partners(self.yc, self.box)              # step 3
        self.P = n_basis(self.p)
        Bc, dBc = basis_bh(self.yc, self.p, self.R0, grad=True)
        Bt, dBt = basis_bh(self.yt, self.p, self.R0, grad=True)
        rows = [(Bc - Bt)[1:].T] + [self.R0 * (dBc[k] - dBt[k])[1:].T for k in range(3)]
        self.A = np.concatenate(rows)                                       # 4L x (P-1)
        U, s, Vt = np.linalg.svd(self.A, full_matrices=False)               # step 5
        keep = s > rcond * s[0]
        self.sigma = s
        self.rank = int(keep.sum())
        self.cond = s[0] / s[keep][-1]
        self.Apinv = (Vt[keep].T / s[keep][None, :]) @ U[:, keep].T        # (P-1) x 4L
        self.R0mean = basis_box_means_bh(self.box, self.p, self.R0)        # step 6

    def near(self, x, q):
        return near_set(x, q, self.box, self.R_b)

    def far_field(self, C, y0):
        B, dB = basis_bh(y0, self.p, self.R0, grad=True)
        return C[1:] @ B[1:], np.stack([C[1:] @ dB[k, 1:] for k in range(3)], axis=1)

    def solve(self, x, q, targets=None, with_mean=True, return_parts=False):
        """Steps 3-8 at the targets (default: the particles).  Returns (phi, field)
        with field = -grad phi."""
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y0 = x if targets is None else np.asarray(targets, dtype=np.float64)
        xs, qs, _, _ = self.near(x, q)
        phc, gc = _native.direct_dist(np.concatenate([self.yc, self.yt]), xs, qs)           # step 3
        L = self.L
        f = np.concatenate([phc[L:] - phc[:L]] + [self.R0 * (gc[L:, k] - gc[:L, k]) for k in range(3)])  # step 4
        C = np.zeros(self.P)
        C[1:] = self.Apinv @ f                                              # step 5
        if with_mean:                                                       # step 6
            S = float(np.sum(qs * box_distance_mean(xs, self.box)))
            C[0] = 0.0 - S - float(C[1:] @ self.R0mean[1:])
        phin, gn = _native.direct_dist(y0, xs, qs)
        phif, gf = self.far_field(C, y0)                                    # step 7
        phi = phin + phif + C[0]                                            # step 8
        grad = gn + gf
        if return_parts:
            return dict(phi=phi, field=-grad, C=C, f=f, n_near=xs.shape[0])
        return phi, -grad


def energy_gradients_bih(plan, x, q):
    """Gradient of E = (1/2) sum_i q_i phi(x_i) computed by the method for K = r,
    with respect to positions and charges: the derivation of oracle/adjoint.py
    (eqs. (3), (8), (10)) with this fit's rows.  With u_t = sum_k q_k B_t(x_k)
    (t >= 2) and w = (A^+)^T u split into the value weights w_l and the gradient
    weights w_kl (rows L + k L + l), E_ff = (1/2) w^T f is (1/2) sum_j q_j psi(z_j)
    over the near entries z_j with
        psi(z) = sum_l w_l [K(y~_l - z) - K(y_l - z)]
               + sum_l D_l . [grad K(y~_l - z) - grad K(y_l - z)],
    D_l = R0 (w_xl, w_yl, w_zl), grad K(y - z) = (y - z)/|y - z| taken in y: a
    charge and a dipole at each check point and partner.  psi joins the base
    particles' potential in the formulas of oracle/adjoint.py; C1 drops out
    because the charges are neutral, and dE/dq is projected onto sum dq = 0.
    Returns (E, dE/dx (N,3), dE/dq (N,))."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    parts = plan.solve(x, q, return_parts=True)
    phi = parts["phi"]
    E = 0.5 * float(np.sum(q * phi))
    u = basis_bh(x, plan.p, plan.R0)[1:] @ q                           # (P-1,)
    w = plan.Apinv.T @ u                                                # (4L,)
    L = plan.L
    D = plan.R0 * w[L:].reshape(3, L).T                                 # (L, 3)
    xs, _, base, _ = plan.near(x, q)
    src = np.concatenate([x, plan.yt, plan.yc])
    srq = np.concatenate([q, w[:L], -w[:L]])
    psi, gpsi = _native.direct_dist(xs, src, srq)
    for pts, sgn in ((plan.yt, 1.0), (plan.yc, -1.0)):
        for c0 in range(0, len(xs), 256):
            d = pts[None, :, :] - xs[c0:c0 + 256, None, :]              # y - z
            r = np.sqrt((d * d).sum(-1))
            dd = (d * D[None, :, :]).sum(-1)                            # D . (y - z)
            psi[c0:c0 + 256] += sgn * (dd / r).sum(1)
            # grad_z of D.(y - z)/|y - z| is -D/r + (D.(y - z)) (y - z)/r^3
            g = -D[None, :, :] / r[:, :, None] + (dd / r ** 3)[:, :, None] * d
            gpsi[c0:c0 + 256] += sgn * g.sum(1)
    dpsi = np.zeros(x.shape[0])
    gsum = np.zeros_like(x)
    np.add.at(dpsi, base, psi)
    np.add.at(gsum, base, gpsi)
    dEdx = 0.5 * q[:, None] * (-parts["field"] + gsum)
    dEdq = 0.5 * (phi + dpsi)
    return E, dEdx, dEdq - dEdq.mean()


class EwaldBih:
    """Ewald-type reference for the periodic sum of K = r (see the module notes)."""

    def __init__(self, box, alpha=None, tol=1e-16):
        self.box = np.asarray(box, dtype=np.float64)
        dmin = float(self.box.min())
        self.alpha = float(alpha) if alpha is not None else 5.0 / dmin
        a = math.sqrt(-math.log(tol))
        self.rcut = a / self.alpha
        kmax = 2.0 * self.alpha * a
        self.V = float(np.prod(self.box))
        nmax = np.ceil(kmax * self.box / (2 * np.pi)).astype(int)
        g = [np.arange(-n, n + 1) for n in nmax]
        N1, N2, N3 = np.meshgrid(*g, indexing="ij")
        n = np.stack([N1.ravel(), N2.ravel(), N3.ravel()], axis=1)
        n = n[np.any(n != 0, axis=1)]
        k = 2 * np.pi * n / self.box[None, :]
        k2 = (k * k).sum(1)
        sel = k2 <= kmax ** 2
        self.k = k[sel]
        k2 = k2[sel]
        self.w = (-8 * np.pi / self.V) * np.exp(-k2 / (4 * self.alpha ** 2)) / (k2 * k2)
        m = np.ceil(self.rcut / self.box + 1.0).astype(int)
        gi = [np.arange(-v, v + 1) for v in m]
        I1, I2, I3 = np.meshgrid(*gi, indexing="ij")
        self.shifts = np.stack([I1.ravel(), I2.ravel(), I3.ravel()], axis=1) * self.box[None, :]
        self.coulomb = Ewald(self.box)

    def solve(self, x, q, targets=None):
        """phi and field = -grad phi at the targets (default: the particles)."""
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y = x if targets is None else np.asarray(targets, dtype=np.float64)
        phi1, g1 = _native.ewald_bih_real(y, x, q, self.shifts, self.alpha, self.rcut)
        self_q = q.copy() if targets is None else np.array([q[np.all(x == t[None, :], axis=1)].sum() for t in y])
        phi1 = phi1 - 2.0 / (self.alpha * math.sqrt(math.pi)) * self_q
        ph = self.k @ x.T
        phi2, g2 = _native.ewald_recip(y, self.k, self.w, np.cos(ph) @ q, np.sin(ph) @ q)
        pc, ec = self.coulomb.solve(x, q, targets=targets)
        h = 1.0 / (2.0 * self.alpha ** 2)
        return phi1 + phi2 - h * pc, -(g1 + g2) - h * ec
