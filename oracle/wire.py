"""The method with the periodic extension along one coordinate only: x periodic,
y and z free (a wire).  The paper states that the periodization may be done
along one or two coordinates (Sec. 1, closing paragraph) and gives no further
details; this module is the reading used here, step for step as in algorithm
"set"/"get" (Sec. 2.3) and the Laplace specialisation (Sec. 3).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

Problem: phi(y) = sum over p = (i d1, 0, 0) of sum_j q_j K(y - x_j - p), the
images summed in inversion-symmetric order, neutral charges, vacuum around the
wire (the field vanishes far from the x axis).

Why periodicity alone is not enough.  Every function harmonic and periodic in
x near the axis is a combination of
  rho^m e^{i m theta}                          (k = 0: harmonic polynomials in y, z),
  I_m(|k| rho) e^{i m theta} e^{i k x},  k = 2 pi n / d1 != 0,
(rho, theta the polar coordinates in the y-z plane), and rho^m e^{i m theta} for
m <= p - 1 lies exactly in the degree-(p-1) polynomial space: the periodicity
rows have an exact null space besides the constant, and the I_m modes make
them ill-conditioned.  What selects the wire's far field is its behaviour
away from the axis: outside a cylinder holding every charge the potential is
harmonic, periodic in x and bounded (neutral charges), so each of its Fourier
modes in (x, theta) is the decaying solution, K_m(|k| rho) for k != 0,
rho^-m for k = 0 and m >= 1, a constant for k = m = 0.

Reading (every step is the 3-D method's unless stated):
  * near set (steps 1-2): the ball |x_j + p| <= R_b over the images along x;
  * check points (step 2): the Gauss spherical grid's points that a shift by one
    period along x moves into S0 (|y_1| > d1 / 2); partner (step 3) shifted
    along x towards the centre;
  * decay rows on the cylinder rho = rho_d, rho_d = sqrt((d2/2)^2 + (d3/2)^2) + h,
    h = R0/10, over one period in x: for k = 2 pi n / d1, n = 0..n_k,
    n_k = ceil(p/4) + 1, and m = 0..p-1, for each cosine/sine in x (the cosine
    only for n = 0) and in theta (the cosine only for m = 0), one row
        < d phi/d rho - beta_{k,m} phi, trig(k x) trig(m theta) >_cylinder = 0,
    beta = |k| K_m'(|k| rho_d) / K_m(|k| rho_d) for k != 0, -m / rho_d for k = 0
    (0 for m = 0: no net line charge).  <g>_cylinder is the mean over
    x in [-d1/2, d1/2] by m_x Gauss-Legendre points and theta by m_t equispaced
    points, m_x = max(2p + 8, ceil(4 d1 / h)), m_t = max(4p, ceil(8 pi rho_d / h)).
    With phi = phi_near + sum_t C_t R_t the row reads
        sum_t C_t <(dR_t/drho - beta R_t) trig> = -<(dphi_near/drho - beta phi_near) trig>,
    the right side from the near sums (potential and gradient) at the cylinder
    points.  The cylinder stays h from every source and inside the ball;
  * the fit (step 5): periodicity and decay rows together, the same SVD
    pseudo-inverse; C1 (step 6) from the zero box mean, a convention; far field
    and outputs (steps 7-8) as in 3-D.
"""
import math

import numpy as np
from scipy.special import kve

from . import _native
from .basis import basis as basis_fn
from .boxmean import basis_box_means, box_potential_mean
from .checkpoints import gauss_sphere
from .geometry import circumradius


def wire_near_set(x, q, box, R_b):
    """Steps 1-2 over the images along x, with the 3-D tie rule.
    Returns (xs, qs, base index, image number)."""
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(box, dtype=np.float64)
    K = int(math.floor(R_b / d[0] + 0.5))
    shifts = [0] + [i for i in range(-K, K + 1) if i != 0]
    thr = R_b * R_b * (1.0 + 1e-12)
    out_x, out_q, out_i, out_m = [], [], [], []
    for m, i in enumerate(shifts):
        X = x[:, 0] + i * d[0]
        Y = x[:, 1]
        Z = x[:, 2]
        keep = (X * X + Y * Y) + Z * Z <= thr
        idx = np.nonzero(keep)[0]
        out_x.append(np.stack([X[idx], Y[idx], Z[idx]], axis=1))
        out_q.append(q[idx])
        out_i.append(idx)
        out_m.append(np.full(idx.size, m))
    return (np.concatenate(out_x), np.concatenate(out_q), np.concatenate(out_i), np.concatenate(out_m))


def decay_beta(k, m, rho):
    """d/drho log of the decaying radial factor of mode (k, m) at rho:
    k K_m'(k rho) / K_m(k rho), with K_m' = -(K_{m-1} + K_{m+1}) / 2 and the
    exponentially scaled K (the scale cancels), so that thin periods (k rho in
    the hundreds, where K itself underflows) stay finite."""
    if k == 0.0:
        return -m / rho
    z = k * rho
    return -k * (kve(abs(m - 1), z) + kve(m + 1, z)) / (2.0 * kve(m, z))


class WirePlan:
    """Algorithm "set" for the wire (x periodic, y and z free)."""

    def __init__(self, box, p, R_b=None, lam=None, rcond=1e-13):
        self.box = np.asarray(box, dtype=np.float64)
        d = self.box
        self.p = int(p)
        self.P = self.p * self.p
        self.R0 = circumradius(d)                                            # step 1
        self.R_b = float(R_b) if R_b is not None else float(lam) * self.R0
        y = gauss_sphere(self.p, self.R0)                                   # step 2
        y = y[np.abs(y[:, 0]) > 0.5 * d[0]]
        yt = y.copy()                                                       # step 3
        yt[:, 0] = y[:, 0] - np.sign(y[:, 0]) * d[0]
        self.yc, self.yt, self.L = y, yt, y.shape[0]
        Ry = basis_fn(*(self.yc.T / self.R0), self.p)[1:]                    # step 4, t = 2..P
        Ryt = basis_fn(*(self.yt.T / self.R0), self.p)[1:]
        self.A_per = (Ry - Ryt).T
        # decay rows on the cylinder
        self.h = self.R0 / 10.0
        self.rho = math.hypot(0.5 * d[1], 0.5 * d[2]) + self.h
        self.nk = math.ceil(self.p / 4) + 1
        self.mx = max(2 * self.p + 8, math.ceil(4.0 * d[0] / self.h))
        self.mt = max(4 * self.p, math.ceil(8.0 * math.pi * self.rho / self.h))
        g, w = np.polynomial.legendre.leggauss(self.mx)
        th = 2.0 * math.pi * np.arange(self.mt) / self.mt
        X, TH = np.meshgrid(0.5 * d[0] * g, th, indexing="ij")
        self.theta = TH.ravel()
        self.pts = np.stack([X.ravel(), self.rho * np.cos(self.theta), self.rho * np.sin(self.theta)], axis=1)
        self.wts = (w[:, None] / 2.0 * np.full(self.mt, 1.0 / self.mt)[None, :]).ravel()
        R, Rg = basis_fn(*(self.pts.T / self.R0), self.p, grad=True)
        dR = (Rg[1] * np.cos(self.theta) + Rg[2] * np.sin(self.theta)) / self.R0
        self.modes = []                    # (beta, weights per point) per row
        rows = []
        for n in range(self.nk + 1):
            k = 2.0 * math.pi * n / d[0]
            for m in range(self.p):
                beta = decay_beta(k, m, self.rho) if (n, m) != (0, 0) else 0.0
                for fx in ((np.cos,) if n == 0 else (np.cos, np.sin)):
                    for ft in ((np.cos,) if m == 0 else (np.cos, np.sin)):
                        wv = self.wts * fx(k * self.pts[:, 0]) * ft(m * self.theta)
                        self.modes.append((beta, wv))
                        rows.append((dR[1:] - beta * R[1:]) @ wv)
        self.A_dec = np.array(rows)
        self.A = np.vstack([self.A_per, self.A_dec])
        U, sv, Vt = np.linalg.svd(self.A, full_matrices=False)               # step 5
        keep = sv > rcond * sv[0]
        self.rank = int(keep.sum())
        self.cond = sv[0] / sv[keep][-1]
        self.Apinv = (Vt[keep].T / sv[keep][None, :]) @ U[:, keep].T
        self.R0mean = basis_box_means(d, self.p, self.R0)                   # step 6 (App. B)

    def near(self, x, q):
        return wire_near_set(x, q, self.box, self.R_b)

    def decay_sources(self, w_dec):
        """The decay rows' adjoint sources for row weights w_dec (oracle/adjoint.py):
        the cylinder points, their outward normal (0, cos theta, sin theta) (the
        rows take E_rho), a_i = sum_r w_r W_ri and b_i = sum_r w_r beta_r W_ri."""
        a = np.zeros(len(self.pts))
        b = np.zeros(len(self.pts))
        for wr, (beta, wv) in zip(w_dec, self.modes):
            a += wr * wv
            b += wr * beta * wv
        nrm = np.stack([np.zeros_like(self.theta), np.cos(self.theta), np.sin(self.theta)], axis=1)
        return self.pts, nrm, a, b

    def rhs(self, xs, qs):
        """The periodicity rows, then -<(dphi_near/drho - beta phi_near) trig> per decay row."""
        phc = _native.direct(np.concatenate([self.yc, self.yt]), xs, qs, grad=False)
        ph, gr = _native.direct(self.pts, xs, qs, grad=True)
        drho = gr[:, 1] * np.cos(self.theta) + gr[:, 2] * np.sin(self.theta)
        dec = np.array([-((drho - beta * ph) @ wv) for beta, wv in self.modes])
        return np.concatenate([phc[self.L:] - phc[: self.L], dec])

    def solve(self, x, q, targets=None, with_mean=True, return_parts=False):
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y0 = x if targets is None else np.asarray(targets, dtype=np.float64)
        xs, qs, _, _ = self.near(x, q)
        f = self.rhs(xs, qs)                                                 # steps 3-4
        C = np.zeros(self.P)
        C[1:] = self.Apinv @ f                                               # step 5
        if with_mean:                                                        # step 6
            S = float(np.sum(qs * box_potential_mean(xs, self.box)))
            C[0] = 0.0 - S - float(C[1:] @ self.R0mean[1:])
        phin, gn = _native.direct(y0, xs, qs, grad=True)
        Rv, Rg = basis_fn(*(y0.T / self.R0), self.p, grad=True)               # step 7
        phif = C[1:] @ Rv[1:]
        gf = np.stack([C[1:] @ Rg[k, 1:] for k in range(3)], axis=1) / self.R0
        phi = phin + phif + C[0]                                             # step 8
        field = -(gn + gf)
        if return_parts:
            return dict(phi=phi, field=field, C=C, f=f, n_near=xs.shape[0])
        return phi, field


def line_sum(x, q, box, targets=None, Ks=(128, 256, 512, 1024)):
    """Brute force: sums over the images |i| <= K along x, the self pair skipped,
    for each K, then three Richardson steps (the truncation error of the
    symmetric sum expands in powers of 1/K).  Potential and field."""
    x = np.asarray(x, dtype=np.float64)
    y = x if targets is None else np.asarray(targets, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    vals = []
    for K in Ks:
        sh = np.zeros((2 * K + 1, 3))
        sh[:, 0] = np.arange(-K, K + 1) * box[0]
        phi, g = _native.direct_images(y, x, q, sh)
        vals.append((phi, -g))
    for order in (1, 2, 3):
        f2 = 2.0 ** order
        vals = [tuple((f2 * b - a) / (f2 - 1) for a, b in zip(u, v)) for u, v in zip(vals[:-1], vals[1:])]
    return vals[0]
