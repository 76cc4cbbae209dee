"""Geometry of the periodization (paper Sec. 2.1 and 2.3).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).
"""
import numpy as np


def circumradius(box):
    """R0 = (1/2) sqrt(d1^2 + d2^2 + d3^2)   (algorithm "set", step 1)."""
    d = np.asarray(box, dtype=np.float64)
    return 0.5 * np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])


def geometric_factor(box):
    """A_gf of eq. (o2.1): N_b = A_gf lambda^3 N on average."""
    d1, d2, d3 = np.asarray(box, dtype=np.float64)
    return np.pi / 6.0 * (d1 * d1 + d2 * d2 + d3 * d3) ** 1.5 / (d1 * d2 * d3)


def image_range(box, R_b):
    """Largest |i_k| of a lattice vector p = (i1 d1, i2 d2, i3 d3) whose box can
    reach the ball |x| <= R_b: the image box i spans i_k d_k +- d_k/2."""
    d = np.asarray(box, dtype=np.float64)
    return np.floor(R_b / d + 0.5).astype(int)


def lattice_vectors(box, R_b):
    """All lattice vectors p (eq. (2)) in the image range, p = (0,0,0) first."""
    d = np.asarray(box, dtype=np.float64)
    k = image_range(box, R_b)
    vs = [(0, 0, 0)]
    for i in range(-k[0], k[0] + 1):
        for j in range(-k[1], k[1] + 1):
            for l in range(-k[2], k[2] + 1):
                if (i, j, l) != (0, 0, 0):
                    vs.append((i, j, l))
    ii = np.array(vs, dtype=np.float64)
    return ii * d  # p = (i1 d1, i2 d2, i3 d3)


def near_set(x, q, box, R_b):
    """Algorithm "get", steps 1-2: extend the box periodically to cover the ball
    S_b and keep the sources with |x_j + p| <= R_b.

    Reading: ties on the sphere |x + p| = R_b (lattices) are kept when
    |x+p|^2 <= R_b^2 (1 + 1e-12), with the squared norm formed as
    ((X*X + Y*Y) + Z*Z) from X = x + p_x etc., without fused multiply-add.

    Returns (xs (N_b,3), qs (N_b,), base index (N_b,), image number (N_b,));
    image 0 is p = 0 and holds every particle in its original order.
    """
    x = np.asarray(x, dtype=np.float64)
    P = lattice_vectors(box, R_b)
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
