"""Check points and their periodic partners (paper Sec. 2.2 and algorithm "set",
steps 2-3).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).
"""
import numpy as np


def gauss_sphere(p, R0):
    """Gauss spherical grid on the sphere of radius R0 (Sec. 2.2, distribution ii):
    polar nodes at the zeros of the Legendre polynomial P_p(cos theta), azimuths
    equispaced.  The paper gives only the count L = 2p^2 - p (Fig. 2 caption);
    reading: 2p - 1 azimuths phi_b = 2 pi b / (2p - 1), b = 0..2p-2, starting at 0.
    Returns (L, 3), ordered polar-node-major."""
    mu, _ = np.polynomial.legendre.leggauss(p)
    nphi = 2 * p - 1
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1.0 - mu * mu)
    pts = np.empty((p, nphi, 3))
    pts[:, :, 0] = R0 * st[:, None] * np.cos(phi)[None, :]
    pts[:, :, 1] = R0 * st[:, None] * np.sin(phi)[None, :]
    pts[:, :, 2] = R0 * mu[:, None]
    return pts.reshape(-1, 3)


def partners(y, box):
    """Partner points y~_l (algorithm "set", step 3): one Cartesian coordinate of
    y_l is shifted by the box period so that the new point lies in S0.

    Reading (the paper leaves k and the direction open): pick the coordinate
    k* that maximizes d_k (2|y_k| - d_k) -- the shift that moves the point
    deepest into S0, since |y~|^2 = |y|^2 - d_k (2|y_k| - d_k) -- with ties
    going to the smallest k, and shift towards the centre:
    y~_k* = y_k* - sign(y_k*) d_k*."""
    y = np.asarray(y, dtype=np.float64)
    d = np.asarray(box, dtype=np.float64)
    gain = d[None, :] * (2.0 * np.abs(y) - d[None, :])
    k = np.argmax(gain, axis=1)  # first maximum -> smallest k on ties
    yt = y.copy()
    rows = np.arange(y.shape[0])
    yt[rows, k] = y[rows, k] - np.sign(y[rows, k]) * d[k]
    return yt, k
