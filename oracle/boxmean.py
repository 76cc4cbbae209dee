"""Box averages needed for the zero-mean constant C1 (paper Sec. 3.4, eqs.
(pfx2)-(pfx4); App. B and App. C).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).
"""
import numpy as np

from .basis import basis


def basis_box_means(box, p, scale):
    """R_t^(0) = (1/V0) int_{Omega0} R_t(y) dV for the basis evaluated at y/scale
    (App. B, eqs. (A1)-(A2)): tensor Gauss-Legendre with N_q = floor((p-1)/2) + 1
    nodes per axis, exact for the polynomials of degree <= p-1."""
    d = np.asarray(box, dtype=np.float64)
    nq = (p - 1) // 2 + 1
    xg, wg = np.polynomial.legendre.leggauss(nq)
    X, Y, Z = np.meshgrid(xg, xg, xg, indexing="ij")
    W = (wg[:, None, None] * wg[None, :, None] * wg[None, None, :]).reshape(-1)
    pts = np.stack([0.5 * d[0] * X.reshape(-1), 0.5 * d[1] * Y.reshape(-1), 0.5 * d[2] * Z.reshape(-1)]) / scale
    Rv = basis(pts[0], pts[1], pts[2], p)
    return (Rv * W[None, :]).sum(axis=1) / 8.0


def _H(x, y, z):
    """Primitive of eq. (B8)-(B9): H(x,y,z) = -z int f(r;|y|) dx with
    f = (rho - |y|)/r^2, r^2 = x^2 + z^2, rho = sqrt(r^2 + y^2):
    H = |y| (atan(x/z) - atan(|y| x/(z rho))) - z ln(rho + x), and H = 0 at z = 0.
    rho + x is formed as (y^2 + z^2)/(rho - x) when x < 0 to avoid cancellation."""
    ay = np.abs(y)
    rho = np.sqrt(x * x + y * y + z * z)
    zs = np.where(z == 0.0, 1.0, z)
    s = np.where(x >= 0.0, rho + x, (y * y + z * z) / np.where(rho - x == 0.0, 1.0, rho - x))
    s = np.where(s > 0.0, s, 1.0)
    h = ay * (np.arctan(x / zs) - np.arctan(ay * x / (zs * np.where(rho == 0.0, 1.0, rho)))) - z * np.log(s)
    return np.where(z == 0.0, 0.0, h)


def box_faces(box):
    """The six faces of Omega0 = [-d/2, d/2]^3: (outward normal n_k, centre y_k0,
    and the four edges as (outward in-plane normal n', midpoint, length))."""
    d = np.asarray(box, dtype=np.float64)
    faces = []
    for a in range(3):
        for sgn in (-1.0, 1.0):
            n = np.zeros(3)
            n[a] = sgn
            c = np.zeros(3)
            c[a] = sgn * d[a] / 2
            edges = []
            for b in range(3):
                if b == a:
                    continue
                o = 3 - a - b  # the axis the edge runs along
                for sb in (-1.0, 1.0):
                    nn = np.zeros(3)
                    nn[b] = sb
                    mid = c.copy()
                    mid[b] = sb * d[b] / 2
                    edges.append((nn, mid, d[o]))
            faces.append((n, c, edges))
    return faces


def box_potential_mean(xs, box):
    """Phi0(x) = (1/V0) int_{Omega0} dV(y)/|y - x|  (eq. (pfx4)), evaluated as in
    App. C: divergence theorem to the six faces (eq. (B1)-(B2)),
    Phi0 = -(1/(2 V0)) sum_k (n_k . x_k) L_k(x_k) with x_k = x - y_k0;
    each face integral L_k by the in-plane divergence theorem to its four edges
    (eq. (B3)-(B5)); each edge integral by the primitive H (eq. (B6)-(B9)).

    Reading of the loosely specified edge frame: for an edge with outward
    in-plane normal n', the frame is i'_y = n_k (face normal), i'_z = n'
    and i'_x = i'_y x i'_z (so that i'_z = i'_x x i'_y as the paper requires),
    starting at the edge end y_kj0 = midpoint - (l/2) i'_x."""
    xs = np.atleast_2d(np.asarray(xs, dtype=np.float64))
    d = np.asarray(box, dtype=np.float64)
    V0 = d[0] * d[1] * d[2]
    total = np.zeros(xs.shape[0])
    for n, c, edges in box_faces(d):
        xk = xs - c[None, :]
        hk = xk @ n
        Lk = np.zeros(xs.shape[0])
        for nn, mid, length in edges:
            ex = np.cross(n, nn)
            y0 = mid - 0.5 * length * ex
            rel = xs - y0[None, :]
            xkj = rel @ ex
            ykj = rel @ n
            zkj = rel @ nn
            Lk += _H(length - xkj, np.abs(ykj), zkj) - _H(-xkj, np.abs(ykj), zkj)
        total += hk * Lk
    return -total / (2.0 * V0)
