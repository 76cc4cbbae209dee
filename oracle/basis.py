"""Renormalized real regular solid harmonics (paper Sec. 3.1).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The basis functions R^_n^m, n = 0..p-1, m = -n..n, are produced exactly the way
the paper prescribes: the Cartesian recurrence of eq. (1.6) for R~_n^m, then the
renormalization of eq. (1.7), R^_n^m = sqrt((n-|m|)! (n+|m|)!) R~_n^m, stacked
with the linear index of eq. (1.8), t = (n+1)^2 - (n-m) (1-based).

Reading: in eq. (1.7) the factorials (n-m)!(n+m)! are symmetric in m, so
|m| and m give the same value.  In the diagonal step of eq. (1.6) the term
R~_0^{-0} is the imaginary part of R_0^0 and therefore zero; the paper states the
|m| = 1 values separately for that reason.

The gradient is obtained by forward-mode differentiation of the same recurrence:
each quantity is carried as (value, d/dx, d/dy, d/dz) and every product uses the
product rule.  This is exact (no finite differences) and needs no separate
coefficient relations, which the paper defers to another reference.
"""
import math
import numpy as np


def index(n, m):
    """0-based position of (n, m) in the stacked vector of eq. (1.8)."""
    return n * n + n + m


def _dual(v, k):
    d = np.zeros((4,) + np.shape(v))
    d[0] = v
    d[1 + k] = 1.0
    return d


def _mul(a, b):
    out = np.empty_like(a)
    out[0] = a[0] * b[0]
    out[1:] = a[0] * b[1:] + b[0] * a[1:]
    return out


def basis(x, y, z, p, grad=False):
    """Return R^_t at the points, shape (p*p, npts); with grad=True also the
    gradient, shape (3, p*p, npts).  Degrees n = 0..p-1 (truncation number p)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    X, Y, Z = _dual(x, 0), _dual(y, 1), _dual(z, 2)
    r2 = _mul(X, X) + _mul(Y, Y) + _mul(Z, Z)
    R = {}  # (n, m) -> dual array of R~_n^m (eq. (1.6), before renormalization)
    one = np.zeros_like(X)
    one[0] = 1.0
    R[(0, 0)] = one
    if p > 1:
        R[(1, 1)] = -0.5 * X
        R[(1, -1)] = 0.5 * Y
    for m in range(2, p):
        a, b = R[(m - 1, m - 1)], R[(m - 1, -(m - 1))]
        R[(m, m)] = -(_mul(X, a) + _mul(Y, b)) / (2.0 * m)
        R[(m, -m)] = (_mul(Y, a) - _mul(X, b)) / (2.0 * m)
    for m in range(-(p - 1), p):
        am = abs(m)
        if am + 1 < p:
            R[(am + 1, m)] = -_mul(Z, R[(am, m)])
        for n in range(am + 2, p):
            R[(n, m)] = -((2 * n - 1) * _mul(Z, R[(n - 1, m)]) + _mul(r2, R[(n - 2, m)])) / ((n - am) * (n + am))
    P = p * p
    out = np.empty((4, P, x.size))
    for n in range(p):
        for m in range(-n, n + 1):
            s = math.sqrt(float(math.factorial(n - abs(m)) * math.factorial(n + abs(m))))  # eq. (1.7)
            out[:, index(n, m), :] = s * R[(n, m)]
    if grad:
        return out[0], out[1:]
    return out[0]
