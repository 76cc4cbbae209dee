"""The method in two dimensions: charges in a d1 x d2 rectangle, periodic along
both axes, kernel K(r) = -log r (the Green's function of the 2-D Laplacian up
to 2 pi).  The paper states that the method applies to 2-D problems (Sec. 1)
and presents it in 3-D; this module is the reading used here, step for step as
in algorithms "set"/"get" (Sec. 2.3) with the Laplace specialisation of Sec. 3
carried to the plane.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

Problem: phi(y) = sum over p = (i d1, j d2) of sum_j q_j K(y - x_j - p), neutral
charges (sum q = 0), K(0) = 0 for the self pair; the lattice sum converges only
conditionally, and the method (like the Ewald split below) returns the periodic
solution, which is unique up to a constant.

Reading:
  * circumradius R0 = |(d1, d2)|/2, near radius R_b = lambda R0 (step 1); the
    near set is every image x_j + p with |x_j + p| <= R_b (steps 1-2, the 3-D tie
    rule);
  * basis: the harmonic polynomials of the plane, at w = (x + i y)/R0:
    R_1 = 1, R_{2n} = Re w^n, R_{2n+1} = Im w^n, n = 1..p-1 (P = 2p - 1 functions;
    the 2-D counterpart of the solid harmonics of Sec. 3.1).  Gradients by
    Cauchy-Riemann from d/dw w^n = n w^(n-1);
  * check points (step 2): L = 4p points equispaced on the circumcircle,
    theta_l = 2 pi l / L (the trapezoidal rule, exact on the circle for
    trigonometric polynomials below degree L, plays the part of the Gauss grid);
    partners (step 3) by the 3-D rule over the two axes;
  * fit (steps 4-5): A_lt = R_t(y_l) - R_t(y~_l), t = 2..P, SVD pseudo-inverse.
    A periodic harmonic function on the torus is a constant, so the constant is
    the only null vector and C1 is fixed by the zero box mean (step 6) with
    <R_t> by tensor Gauss-Legendre and Phi0(x) = <K(y - x)>_box in closed form
    (the potential of a uniform rectangle, below);
  * far field and outputs (steps 7-8) as in 3-D: phi = phi_near + sum_t C_t R_t + C1,
    field = -grad phi.
"""
import math

import numpy as np
from scipy.special import exp1

from . import _native

EULER_GAMMA = 0.57721566490153286061


def circumradius2d(box):
    return 0.5 * math.hypot(float(box[0]), float(box[1]))


def basis2d(x, y, p, grad=False):
    """R_t at the scaled point (x, y) (already divided by R0), t = 1..P, P = 2p - 1,
    as rows of an array (P, ...); with grad also (2, P, ...) d/dx and d/dy of R_t
    in the scaled variables."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = x + 1j * y
    P = 2 * p - 1
    R = np.zeros((P,) + w.shape)
    R[0] = 1.0
    G = np.zeros((2, P) + w.shape) if grad else None
    wm1 = np.ones_like(w)                   # w^(n-1)
    for n in range(1, p):
        if grad:
            d = n * wm1                      # d/dw w^n
            G[0, 2 * n - 1], G[1, 2 * n - 1] = d.real, -d.imag   # Re w^n
            G[0, 2 * n], G[1, 2 * n] = d.imag, d.real            # Im w^n
        wm1 = wm1 * w
        R[2 * n - 1], R[2 * n] = wm1.real, wm1.imag
    return (R, G) if grad else R


def circle_points(p, R0):
    L = 4 * p
    th = 2.0 * math.pi * np.arange(L) / L
    return R0 * np.stack([np.cos(th), np.sin(th)], axis=1)


def partners2d(y, box):
    """Step 3 over the two axes: shift the coordinate k maximising
    d_k (2|y_k| - d_k) by one period towards the centre (ties: the smaller k)."""
    d = np.asarray(box, dtype=np.float64)
    g = d[None, :] * (2.0 * np.abs(y) - d[None, :])
    k = np.argmax(g, axis=1)                 # first maximum on ties
    yt = y.copy()
    idx = np.arange(len(y))
    yt[idx, k] = y[idx, k] - np.sign(y[idx, k]) * d[k]
    return yt


def near_set2d(x, q, box, R_b):
    """Steps 1-2: every image x_j + (i d1, j d2) with |x_j + p| <= R_b (tie rule
    of the 3-D method).  Returns (xs, qs, base index, image number); image 0 is
    the box itself."""
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(box, dtype=np.float64)
    K = [int(math.floor(R_b / d[k] + 0.5)) for k in range(2)]
    shifts = [(0, 0)] + [(i, j) for i in range(-K[0], K[0] + 1) for j in range(-K[1], K[1] + 1) if (i, j) != (0, 0)]
    thr = R_b * R_b * (1.0 + 1e-12)
    out_x, out_q, out_i, out_m = [], [], [], []
    for m, (i, j) in enumerate(shifts):
        X = x[:, 0] + i * d[0]
        Y = x[:, 1] + j * d[1]
        idx = np.nonzero(X * X + Y * Y <= thr)[0]
        out_x.append(np.stack([X[idx], Y[idx]], axis=1))
        out_q.append(q[idx])
        out_i.append(idx)
        out_m.append(np.full(idx.size, m))
    return (np.concatenate(out_x), np.concatenate(out_q), np.concatenate(out_i), np.concatenate(out_m))


def _rect_primitive(u, v):
    """F with d^2 F / du dv = log(u^2 + v^2):
    F = u v (log(u^2 + v^2) - 3) + u^2 atan(v/u) + v^2 atan(u/v), each term taken
    as its limit 0 where its prefactor vanishes."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    r2 = u * u + v * v
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(r2 > 0.0, u * v * (np.log(np.where(r2 > 0.0, r2, 1.0)) - 3.0), 0.0)
        t2 = np.where(u != 0.0, u * u * np.arctan(v / np.where(u != 0.0, u, 1.0)), 0.0)
        t3 = np.where(v != 0.0, v * v * np.arctan(u / np.where(v != 0.0, v, 1.0)), 0.0)
    return t1 + t2 + t3


def rect_mean_potential(x, box):
    """Phi0(x) = (1/V) int_box -log|y - x| dy (step 6): the potential of a uniform
    rectangle, -(1/(2V)) times the corner sum of F."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = np.asarray(box, dtype=np.float64)
    a1, b1 = -0.5 * d[0] - x[:, 0], 0.5 * d[0] - x[:, 0]
    a2, b2 = -0.5 * d[1] - x[:, 1], 0.5 * d[1] - x[:, 1]
    s = _rect_primitive(b1, b2) - _rect_primitive(a1, b2) - _rect_primitive(b1, a2) + _rect_primitive(a1, a2)
    return -s / (2.0 * d[0] * d[1])


def basis_box_means2d(box, p, R0):
    """<R_t> over the box by tensor Gauss-Legendre, N_q = floor((p-1)/2) + 1 nodes
    per axis (exact for the degree p - 1 polynomials)."""
    nq = (p - 1) // 2 + 1
    g, w = np.polynomial.legendre.leggauss(nq)
    X, Y = np.meshgrid(0.5 * box[0] * g, 0.5 * box[1] * g, indexing="ij")
    W = np.outer(w, w) / 4.0
    R = basis2d(X / R0, Y / R0, p)
    return np.tensordot(R, W, axes=([1, 2], [0, 1]))


class Plan2D:
    """Algorithm "set" in the plane."""

    def __init__(self, box, p, R_b=None, lam=None, rcond=1e-13):
        self.box = np.asarray(box, dtype=np.float64)[:2]
        d = self.box
        self.p = int(p)
        self.P = 2 * self.p - 1
        self.R0 = circumradius2d(d)                                          # step 1
        self.R_b = float(R_b) if R_b is not None else float(lam) * self.R0
        self.yc = circle_points(self.p, self.R0)                            # step 2
        self.yt = partners2d(self.yc, d)                                    # step 3
        self.L = len(self.yc)
        Ry = basis2d(self.yc[:, 0] / self.R0, self.yc[:, 1] / self.R0, self.p)[1:]   # step 4
        Ryt = basis2d(self.yt[:, 0] / self.R0, self.yt[:, 1] / self.R0, self.p)[1:]
        self.A = (Ry - Ryt).T
        U, sv, Vt = np.linalg.svd(self.A, full_matrices=False)                # step 5
        keep = sv > rcond * sv[0]
        self.rank = int(keep.sum())
        self.cond = sv[0] / sv[keep][-1]
        self.Apinv = (Vt[keep].T / sv[keep][None, :]) @ U[:, keep].T
        self.R0mean = basis_box_means2d(d, self.p, self.R0)                 # step 6

    def near(self, x, q):
        return near_set2d(x, q, self.box, self.R_b)

    def solve(self, x, q, targets=None, with_mean=True, return_parts=False):
        x = np.asarray(x, dtype=np.float64)[:, :2]
        q = np.asarray(q, dtype=np.float64)
        y0 = x if targets is None else np.asarray(targets, dtype=np.float64)[:, :2]
        xs, qs, _, _ = self.near(x, q)
        phc = _native.direct_log2d(np.concatenate([self.yc, self.yt]), xs, qs, grad=False)   # step 3
        f = phc[self.L:] - phc[: self.L]                                    # step 4
        C = np.zeros(self.P)
        C[1:] = self.Apinv @ f                                               # step 5
        if with_mean:                                                        # step 6
            S = float(np.sum(qs * rect_mean_potential(xs, self.box)))
            C[0] = 0.0 - S - float(C[1:] @ self.R0mean[1:])
        phin, gn = _native.direct_log2d(y0, xs, qs)
        Rv, Rg = basis2d(y0[:, 0] / self.R0, y0[:, 1] / self.R0, self.p, grad=True)   # step 7
        phif = C[1:] @ Rv[1:]
        gf = np.stack([C[1:] @ Rg[k, 1:] for k in range(2)], axis=1) / self.R0
        phi = phin + phif + C[0]                                             # step 8
        field = -(gn + gf)
        if return_parts:
            return dict(phi=phi, field=field, C=C, f=f, n_near=xs.shape[0])
        return phi, field


def energy_gradients2d(plan, x, q):
    """E = (1/2) sum_i q_i phi(x_i) for the plane's method and its exact gradient,
    derived as in 3-D (oracle/adjoint.py): moments u_t = sum_k q_k R_t(x_k / R0),
    t = 2..P, w = (A^+)^T u, psi(z) = sum_k q_k K(z - x_k) + sum_l w_l [K(z - y~_l)
    - K(z - y_l)] with K = -log r;
      dE/dx_i = (1/2) q_i grad phi(x_i) + (1/2) q_i sum_{p: (i,p) near} grad psi(x_i + p),
      dE/dq_i = (1/2) phi(x_i)          + (1/2)     sum_{p: (i,p) near} psi(x_i + p),
    C1 dropping out for neutral charges and dE/dq projected onto sum dq = 0.
    Returns (E, dE/dx (N,2), dE/dq (N,))."""
    x = np.asarray(x, dtype=np.float64)[:, :2]
    q = np.asarray(q, dtype=np.float64)
    phi, field = plan.solve(x, q)
    E = 0.5 * float(np.sum(q * phi))
    u = basis2d(x[:, 0] / plan.R0, x[:, 1] / plan.R0, plan.p)[1:] @ q
    w = plan.Apinv.T @ u
    xs, _, base, _ = plan.near(x, q)
    src = np.concatenate([x, plan.yt, plan.yc])
    srq = np.concatenate([q, w, -w])
    psi, gpsi = _native.direct_log2d(xs, src, srq)
    dpsi = np.zeros(x.shape[0])
    gsum = np.zeros_like(x)
    np.add.at(dpsi, base, psi)
    np.add.at(gsum, base, gpsi)
    dq = 0.5 * (phi + dpsi)
    return E, 0.5 * q[:, None] * (-field + gsum), dq - dq.mean()


class EwaldLog2D:
    """Independent Ewald split of the 2-D periodic log sum (conducting boundary,
    zero cell mean).  From -log r = (1/2) int_0^inf (exp(-r^2 t) - exp(-t)) dt / t,
    split at t = alpha^2:
      real space  (1/2) E1(alpha^2 r^2) over the images,
      reciprocal  (2 pi / A) sum_{k != 0} exp(-k^2/(4 alpha^2)) / k^2 cos(k.(y - x_j)),
    the k = 0 terms cancelling for neutral charges; the self pair contributes the
    finite part of (1/2) E1(alpha^2 r^2) + log r at r = 0, -gamma/2 - log alpha."""

    def __init__(self, box, alpha=None, tol=1e-17):
        self.box = np.asarray(box, dtype=np.float64)[:2]
        self.A = float(self.box[0] * self.box[1])
        self.alpha = float(alpha) if alpha is not None else 2.5 / math.sqrt(self.A)
        s = -math.log(tol)
        self.rcut = math.sqrt(s) / self.alpha
        self.kcut = 2.0 * self.alpha * math.sqrt(s)

    def solve(self, x, q, targets=None):
        x = np.asarray(x, dtype=np.float64)[:, :2]
        q = np.asarray(q, dtype=np.float64)
        y = x if targets is None else np.asarray(targets, dtype=np.float64)[:, :2]
        d, a = self.box, self.alpha
        phi = np.zeros(len(y))
        fld = np.zeros((len(y), 2))
        K = [int(math.ceil(self.rcut / d[k])) + 1 for k in range(2)]
        for i in range(-K[0], K[0] + 1):
            for j in range(-K[1], K[1] + 1):
                sh = np.array([i * d[0], j * d[1]])
                for c0 in range(0, len(y), 256):
                    yy = y[c0:c0 + 256]
                    r = yy[:, None, :] - x[None, :, :] - sh[None, None, :]
                    r2 = (r * r).sum(-1)
                    live = (r2 > 0.0) & (r2 < self.rcut ** 2)
                    s2 = np.where(live, r2, 1.0)
                    phi[c0:c0 + 256] += (np.where(live, 0.5 * exp1(a * a * s2), 0.0) * q[None, :]).sum(1)
                    g = np.where(live, np.exp(-a * a * s2) / s2, 0.0) * q[None, :]
                    fld[c0:c0 + 256] += (g[:, :, None] * r).sum(1)
                    if i == 0 and j == 0:
                        phi[c0:c0 + 256] += ((r2 == 0.0) * q[None, :]).sum(1) * (-0.5 * EULER_GAMMA - math.log(a))
        n1 = int(math.ceil(self.kcut * d[0] / (2 * math.pi)))
        n2 = int(math.ceil(self.kcut * d[1] / (2 * math.pi)))
        for i in range(-n1, n1 + 1):
            for j in range(-n2, n2 + 1):
                if i == 0 and j == 0:
                    continue
                k = np.array([2 * math.pi * i / d[0], 2 * math.pi * j / d[1]])
                k2 = float(k @ k)
                if k2 > self.kcut ** 2:
                    continue
                wk = 2.0 * math.pi / self.A * math.exp(-k2 / (4 * a * a)) / k2
                S = np.sum(q * np.exp(-1j * (x @ k)))
                e = np.exp(1j * (y @ k)) * S
                phi += wk * e.real
                fld += wk * e.imag[:, None] * k[None, :]
        return phi, fld


def theta_sum(x, q, box, targets=None, nterms=40):
    """Closed form of the doubly periodic log potential of neutral charges:
    G(z) = -log|theta_1(pi z / d1 | tau)| + pi y^2 / (d1 d2), tau = i d2/d1, is the
    periodic Green's function with a neutralising background (Jacobi's theta
    function, nome exp(-pi d2/d1)); sum_j q_j G(y - x_j) is the periodic solution
    up to a constant.  Differences y - x_j are wrapped into the principal cell
    (G is doubly periodic).  At a coincident point the pair contributes the
    regular part of G, lim (G(z) + log|z|) = -log(pi theta_1'(0) / d1).
    Returns (phi, field)."""
    x = np.asarray(x, dtype=np.float64)[:, :2]
    y = x if targets is None else np.asarray(targets, dtype=np.float64)[:, :2]
    d = np.asarray(box, dtype=np.float64)[:2]
    A = d[0] * d[1]
    nome = math.exp(-math.pi * d[1] / d[0])
    n = np.arange(nterms)
    cn = 2.0 * (-1.0) ** n * nome ** ((n + 0.5) ** 2)
    reg = -math.log(math.pi * float((cn * (2 * n + 1)).sum()) / d[0])
    phi = np.zeros(len(y))
    fld = np.zeros((len(y), 2))
    for j in range(len(x)):
        r = y - x[j]
        r = r - d * np.floor(r / d + 0.5)
        skip = np.all(r == 0.0, axis=1)
        v = math.pi * (r[:, 0] + 1j * r[:, 1]) / d[0]
        arg = (2 * n[None, :] + 1) * v[:, None]
        th = (cn[None, :] * np.sin(arg)).sum(1)
        dth = (cn[None, :] * (2 * n[None, :] + 1) * np.cos(arg)).sum(1)
        th = np.where(skip, 1.0, th)
        g = (math.pi / d[0]) * dth / th                # d/dz log theta_1(pi z / d1)
        phi += q[j] * np.where(skip, reg, -np.log(np.abs(th)) + math.pi * r[:, 1] ** 2 / A)
        # -grad of -Re log theta_1 is (Re g, -Im g); the background term adds (0, -2 pi y / A)
        fld[:, 0] += np.where(skip, 0.0, q[j] * g.real)
        fld[:, 1] += np.where(skip, 0.0, q[j] * (-g.imag - 2.0 * math.pi * r[:, 1] / A))
    return phi, fld


def shell_sum2d(x, q, box, targets=None, Ks=(32, 64, 128, 256), steps=3):
    """Brute force: sums over the squares of images |i|, |j| <= K (the self pair
    skipped) for each K, then Richardson steps assuming a truncation error in
    powers of 1/K.  For cells without a dipole moment."""
    x = np.asarray(x, dtype=np.float64)[:, :2]
    y = x if targets is None else np.asarray(targets, dtype=np.float64)[:, :2]
    d = np.asarray(box, dtype=np.float64)[:2]
    vals = []
    for K in Ks:
        ii, jj = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
        sh = np.stack([ii.ravel() * d[0], jj.ravel() * d[1]], axis=1)
        phi, g = _native.direct_log2d(y, x, q, shifts=sh)
        vals.append((phi, -g))
    for order in range(1, steps + 1):
        f2 = 2.0 ** order
        vals = [tuple((f2 * b - a) / (f2 - 1) for a, b in zip(u, v)) for u, v in zip(vals[:-1], vals[1:])]
    return vals[0]
