"""The method with the periodic extension along two coordinates only: x and y
periodic, z free (a slab).  The paper states that the periodization may be done
along one or two coordinates (Sec. 1, closing paragraph) and gives no further
details; this module is the reading used here, step for step as in algorithm
"set"/"get" (Sec. 2.3) and the Laplace specialisation (Sec. 3).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

Problem: phi(y) = sum over p = (i1 d1, i2 d2, 0) of sum_j q_j K(y - x_j - p), the
lattice summed in inversion-symmetric order, neutral charges, vacuum on both
sides in z (the field vanishes far from the slab).

Why periodicity alone is not enough here.  In 3-D the far field is fixed, up to
the constant, by periodicity along all three axes (Sec. 3: a triply periodic
harmonic function is constant).  With two periodic axes every
  e^{+|k| z} e^{i k.rho},  e^{-|k| z} e^{i k.rho},  k = 2 pi (n1/d1, n2/d2),
and also 1 and z, is harmonic and periodic in x and y.  Degree-(p-1)
polynomials approximate the low-|k| ones in the ball ever better as p grows, so
a fit to x/y periodicity alone is ill-posed: its condition number grows without
bound with p.  What selects the slab's far field among them is its behaviour
away from the charges: above the box the total potential is harmonic, periodic
and bounded, so each in-plane Fourier mode decays, phi_k(z) ~ e^{-|k| z}; below
it phi_k(z) ~ e^{+|k| z}; for k = 0 this is Gauss's law with no charge beyond
the plane (the planar mean of dphi/dz vanishes).

Reading (every step is the 3-D method's unless stated):
  * near set (steps 1-2): the ball |x_j + p| <= R_b over the in-plane images only;
  * check points (step 2): the Gauss spherical grid on S0, keeping the points
    that a shift by one period along x or y moves into S0 (|y_k| > d_k / 2 for
    k = 1 or 2); the partner (step 3) is the 3-D rule restricted to k in {1, 2};
    the dropped points, around the z poles, have no partner inside S0;
  * decay rows: on the planes z = +-z_d, z_d = d3/2 + h, h = R0/10, for every
    in-plane reciprocal vector k = 2 pi (n1/d1, n2/d2) with |n1|, |n2| <= n_k,
    n_k = ceil(p/4) + 1, taken once per +-k pair (n1 > 0, or n1 = 0 and n2 >= 0),
    and for its cosine and sine (the cosine only for k = 0), one row
        < (d/dz + s |k|) phi, trig(k.rho) >_plane = 0,   s = +1 on top, -1 below,
    where <g>_plane is the mean over the cell's cross-section rectangle at that
    height, by m x m Gauss-Legendre points, m = max(2p + 8, ceil(4 max(d1, d2) / h)).
    With phi = phi_near + sum_t C_t R_t the row reads
        sum_t C_t <(dR_t/dz + s|k| R_t) trig> = -<(dphi_near/dz + s|k| phi_near) trig>,
    the right side from the near sums (potential and gradient) at the plane
    points, like the check-point sums.  The planes lie a distance h beyond every
    source, so the quadrature sees a smooth integrand, and inside the ball where
    the expansion converges;
  * the fit (step 5): the periodicity rows and the decay rows together, the
    same SVD pseudo-inverse; the constant C1 (step 6) from the zero box mean, a
    convention as in 3-D; far field and outputs (steps 7-8) as in 3-D.
"""
import math

import numpy as np

from . import _native
from .basis import basis as basis_fn
from .boxmean import basis_box_means, box_potential_mean
from .checkpoints import gauss_sphere
from .geometry import circumradius


def slab_lattice_vectors(box, R_b):
    """In-plane lattice vectors p = (i1 d1, i2 d2, 0) whose box can reach the ball
    |x| <= R_b, p = 0 first."""
    d = np.asarray(box, dtype=np.float64)
    k = np.floor(R_b / d[:2] + 0.5).astype(int)
    vs = [(0, 0)]
    for i in range(-k[0], k[0] + 1):
        for j in range(-k[1], k[1] + 1):
            if (i, j) != (0, 0):
                vs.append((i, j))
    ii = np.array(vs, dtype=np.float64)
    return np.stack([ii[:, 0] * d[0], ii[:, 1] * d[1], np.zeros(len(ii))], axis=1)


def slab_near_set(x, q, box, R_b):
    """Steps 1-2 over the in-plane images, with the 3-D tie rule: kept when
    ((X*X + Y*Y) + Z*Z) <= R_b^2 (1 + 1e-12), no fused multiply-add.
    Returns (xs, qs, base index, image number)."""
    x = np.asarray(x, dtype=np.float64)
    P = slab_lattice_vectors(box, R_b)
    thr = R_b * R_b * (1.0 + 1e-12)
    out_x, out_q, out_i, out_m = [], [], [], []
    for m, p in enumerate(P):
        X = x[:, 0] + p[0]
        Y = x[:, 1] + p[1]
        Z = x[:, 2] + p[2]
        keep = (X * X + Y * Y) + Z * Z <= thr
        idx = np.nonzero(keep)[0]
        out_x.append(np.stack([X[idx], Y[idx], Z[idx]], axis=1))
        out_q.append(q[idx])
        out_i.append(idx)
        out_m.append(np.full(idx.size, m))
    return (np.concatenate(out_x), np.concatenate(out_q), np.concatenate(out_i), np.concatenate(out_m))


def slab_partners(y, box):
    """Keep the check points with an in-plane partner inside S0 and return
    (kept points, partners, shifted axis): the axis k in {0, 1} maximizing
    d_k (2|y_k| - d_k) > 0 (ties to the smaller k), shifted towards the centre."""
    y = np.asarray(y, dtype=np.float64)
    d = np.asarray(box, dtype=np.float64)
    gain = d[None, :2] * (2.0 * np.abs(y[:, :2]) - d[None, :2])
    k = np.argmax(gain, axis=1)
    rows = np.arange(y.shape[0])
    keep = gain[rows, k] > 0.0
    y, k = y[keep], k[keep]
    rows = np.arange(y.shape[0])
    yt = y.copy()
    yt[rows, k] = y[rows, k] - np.sign(y[rows, k]) * d[k]
    return y, yt, k


def decay_modes(nk, box):
    """In-plane reciprocal vectors k = 2 pi (n1/d1, n2/d2), |n1|, |n2| <= nk, one of
    each +-k pair (n1 > 0, or n1 = 0 and n2 >= 0), in (n1, n2) row-major order."""
    d = np.asarray(box, dtype=np.float64)
    out = []
    for n1 in range(0, nk + 1):
        for n2 in range(-nk, nk + 1):
            if n1 == 0 and n2 < 0:
                continue
            out.append((2 * math.pi * n1 / d[0], 2 * math.pi * n2 / d[1]))
    return np.array(out)


def plane_points(box, z, m):
    """m x m Gauss-Legendre points on the cross-section rectangle at height z, and
    weights summing to 1 (the mean over the rectangle)."""
    d = np.asarray(box, dtype=np.float64)
    g, w = np.polynomial.legendre.leggauss(m)
    X, Y = np.meshgrid(0.5 * d[0] * g, 0.5 * d[1] * g, indexing="ij")
    W = (w[:, None] * w[None, :]).ravel() / 4.0
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1), W


class SlabPlan:
    """Algorithm "set" for the slab (x, y periodic, z free)."""

    def __init__(self, box, p, R_b=None, lam=None, rcond=1e-13, check_points=None):
        self.box = np.asarray(box, dtype=np.float64)
        d = self.box
        self.p = int(p)
        self.R0 = circumradius(d)                                            # step 1
        self.R_b = float(R_b) if R_b is not None else float(lam) * self.R0
        if check_points is None:
            check_points = gauss_sphere(self.p, self.R0)                     # step 2
        self.yc, self.yt, self.shift_axis = slab_partners(check_points, d)   # step 3
        self.L = self.yc.shape[0]
        self.P = self.p * self.p
        Ry = basis_fn(*(self.yc.T / self.R0), self.p)[1:]                    # step 4, t = 2..P
        Ryt = basis_fn(*(self.yt.T / self.R0), self.p)[1:]
        self.A_per = (Ry - Ryt).T                                            # L x (P-1)
        # decay rows on the planes z = +-z_d
        self.h = self.R0 / 10.0
        self.zd = 0.5 * d[2] + self.h
        self.nk = math.ceil(self.p / 4) + 1
        self.m = max(2 * self.p + 8, math.ceil(4.0 * max(d[0], d[1]) / self.h))
        self.modes = decay_modes(self.nk, d)
        self.planes = []                  # (sign, points, [(|k|, weights per point)] per row)
        rows = []
        for s in (1.0, -1.0):
            pts, W = plane_points(d, s * self.zd, self.m)
            R, Rg = basis_fn(*(pts.T / self.R0), self.p, grad=True)
            dz = Rg[2] / self.R0
            proj = []
            for k in self.modes:
                kk = float(np.hypot(k[0], k[1]))
                ph = pts[:, :2] @ k
                for trig in (np.cos,) if kk == 0.0 else (np.cos, np.sin):
                    wv = W * trig(ph)
                    proj.append((kk, wv))
                    rows.append((dz[1:] + s * kk * R[1:]) @ wv)
            self.planes.append((s, pts, proj))
        self.A_dec = np.array(rows)                                          # n_dec x (P-1)
        self.A = np.vstack([self.A_per, self.A_dec])
        U, sv, Vt = np.linalg.svd(self.A, full_matrices=False)               # step 5
        keep = sv > rcond * sv[0]
        self.rank = int(keep.sum())
        self.cond = sv[0] / sv[keep][-1]
        self.Apinv = (Vt[keep].T / sv[keep][None, :]) @ U[:, keep].T         # (P-1) x (L + n_dec)
        self.R0mean = basis_box_means(d, self.p, self.R0)                   # step 6 (App. B)

    def near(self, x, q):
        return slab_near_set(x, q, self.box, self.R_b)

    def decay_sources(self, w_dec):
        """The decay rows' adjoint sources for row weights w_dec (oracle/adjoint.py):
        the plane points, their normal +z (the rows take E_z), a_i = sum_r w_r W_ri
        and b_i = sum_r w_r (-s|k|) W_ri."""
        pts, nrm, a, b = [], [], [], []
        r = 0
        for s, p_, proj in self.planes:
            av = np.zeros(len(p_))
            bv = np.zeros(len(p_))
            for kk, wv in proj:
                av += w_dec[r] * wv
                bv += w_dec[r] * (-s * kk) * wv
                r += 1
            pts.append(p_)
            nrm.append(np.tile([0.0, 0.0, 1.0], (len(p_), 1)))
            a.append(av)
            b.append(bv)
        return np.concatenate(pts), np.concatenate(nrm), np.concatenate(a), np.concatenate(b)

    def far_field(self, C, y0):
        Rv, Rg = basis_fn(*(y0.T / self.R0), self.p, grad=True)
        phif = C[1:] @ Rv[1:]
        gf = np.stack([C[1:] @ Rg[k, 1:] for k in range(3)], axis=1) / self.R0
        return phif, gf

    def rhs(self, xs, qs):
        """f: the periodicity rows phi_near(y~_l) - phi_near(y_l), then the decay
        rows -<(dphi_near/dz + s|k| phi_near) trig(k.rho)>_plane."""
        phc = _native.direct(np.concatenate([self.yc, self.yt]), xs, qs, grad=False)
        f = [phc[self.L:] - phc[: self.L]]
        for s, pts, proj in self.planes:
            ph, gr = _native.direct(pts, xs, qs, grad=True)
            f.append(np.array([-((gr[:, 2] + s * kk * ph) @ wv) for kk, wv in proj]))
        return np.concatenate(f)

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
        phif, gf = self.far_field(C, y0)                                     # step 7
        phi = phin + phif + C[0]                                             # step 8
        grad = gn + gf
        if return_parts:
            return dict(phi=phi, field=-grad, C=C, f=f, n_near=xs.shape[0], phi_near=phin, phi_far=phif)
        return phi, -grad
