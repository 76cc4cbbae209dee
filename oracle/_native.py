"""ctypes loader for the oracle's C direct sums (oracle/pairs.c).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_pairs.so")
_lib = None


def build(force=False):
    """Compile pairs.c with gcc (FP64, OpenMP, no fast-math, no FMA contraction)."""
    src = os.path.join(_HERE, "pairs.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        L = ctypes.c_long
        _lib.orc_direct.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, dp, dp, dp, dp]
        _lib.orc_direct_images.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, L, dp, dp, dp, dp, dp, dp, dp]
        _lib.orc_ewald_real.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, L, dp, dp, dp,
                                        ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        _lib.orc_ewald_recip.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        D = ctypes.c_double
        _lib.orc_direct_screened.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, L, dp, dp, dp, D, dp, dp, dp, dp]
        _lib.orc_ewald_screened_real.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, L, dp, dp, dp, D, D, D,
                                                 dp, dp, dp, dp]
        _lib.orc_direct_log2d.argtypes = [L, dp, dp, L, dp, dp, dp, L, dp, dp, dp, dp, dp]
        _lib.orc_direct_dist.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, L, dp, dp, dp, dp, dp, dp, dp]
        _lib.orc_ewald_bih_real.argtypes = [L, dp, dp, dp, L, dp, dp, dp, dp, L, dp, dp, dp, D, D,
                                            dp, dp, dp, dp]
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cols(a):
    a = np.asarray(a, dtype=np.float64)
    return [np.ascontiguousarray(a[:, k]) for k in range(3)]


def direct(targets, sources, q, grad=True):
    """phi(y) = sum_j q_j K(y - x_j) and grad phi at each target (K(0) = 0)."""
    tx, ty, tz = _cols(targets)
    sx, sy, sz = _cols(sources)
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)] if grad else None
    null = ctypes.POINTER(ctypes.c_double)()
    lib().orc_direct(n, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz), _p(sq), _p(phi),
                     *(tuple(_p(a) for a in g) if grad else (null, null, null)))
    return (phi, np.stack(g, axis=1)) if grad else phi


def direct_images(targets, sources, q, shifts):
    tx, ty, tz = _cols(targets)
    sx, sy, sz = _cols(sources)
    px, py, pz = _cols(shifts)
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)]
    lib().orc_direct_images(n, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz), _p(sq),
                            px.size, _p(px), _p(py), _p(pz), _p(phi), *(_p(a) for a in g))
    return phi, np.stack(g, axis=1)


def ewald_real(targets, sources, q, shifts, xi, rcut):
    tx, ty, tz = _cols(targets)
    sx, sy, sz = _cols(sources)
    px, py, pz = _cols(shifts)
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)]
    lib().orc_ewald_real(n, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz), _p(sq),
                         px.size, _p(px), _p(py), _p(pz), float(xi), float(rcut), _p(phi), *(_p(a) for a in g))
    return phi, np.stack(g, axis=1)


def ewald_recip(targets, kvec, w, sre, sim):
    tx, ty, tz = _cols(targets)
    kx, ky, kz = _cols(kvec)
    w = np.ascontiguousarray(w, dtype=np.float64)
    sre = np.ascontiguousarray(sre, dtype=np.float64)
    sim = np.ascontiguousarray(sim, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)]
    lib().orc_ewald_recip(n, _p(tx), _p(ty), _p(tz), kx.size, _p(kx), _p(ky), _p(kz), _p(w), _p(sre), _p(sim),
                          _p(phi), *(_p(a) for a in g))
    return phi, np.stack(g, axis=1)


def direct_screened(targets, sources, q, kappa, shifts=None, grad=True):
    """phi(y) = sum_p sum_j q_j exp(-kappa r)/r, r = |y - x_j - p| (K(0) = 0), over
    the given shifts (default: none, the free-space sum), and grad phi."""
    tx, ty, tz = _cols(targets)
    sx, sy, sz = _cols(sources)
    px, py, pz = _cols(np.zeros((1, 3)) if shifts is None else shifts)
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)] if grad else None
    null = ctypes.POINTER(ctypes.c_double)()
    lib().orc_direct_screened(n, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz), _p(sq),
                              px.size, _p(px), _p(py), _p(pz), float(kappa), _p(phi),
                              *(tuple(_p(a) for a in g) if grad else (null, null, null)))
    return (phi, np.stack(g, axis=1)) if grad else phi


def ewald_screened_real(targets, sources, q, shifts, kappa, alpha, rcut):
    tx, ty, tz = _cols(targets)
    sx, sy, sz = _cols(sources)
    px, py, pz = _cols(shifts)
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)]
    lib().orc_ewald_screened_real(n, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz), _p(sq),
                                  px.size, _p(px), _p(py), _p(pz), float(kappa), float(alpha), float(rcut),
                                  _p(phi), *(_p(a) for a in g))
    return phi, np.stack(g, axis=1)


def direct_log2d(targets, sources, q, shifts=None, grad=True):
    """Two dimensions: phi(y) = sum_p sum_j q_j (-log |y - x_j - p|) (K(0) = 0) over
    the given 2-D shifts (default: none, the free-space sum), and grad phi.
    targets, sources: (n, 2)."""
    t = np.asarray(targets, dtype=np.float64)
    s = np.asarray(sources, dtype=np.float64)
    sh = np.zeros((1, 2)) if shifts is None else np.asarray(shifts, dtype=np.float64)
    tx, ty = (np.ascontiguousarray(t[:, k]) for k in range(2))
    sx, sy = (np.ascontiguousarray(s[:, k]) for k in range(2))
    px, py = (np.ascontiguousarray(sh[:, k]) for k in range(2))
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(2)] if grad else None
    null = ctypes.POINTER(ctypes.c_double)()
    lib().orc_direct_log2d(n, _p(tx), _p(ty), sx.size, _p(sx), _p(sy), _p(sq), px.size, _p(px), _p(py), _p(phi),
                           *(tuple(_p(a) for a in g) if grad else (null, null)))
    return (phi, np.stack(g, axis=1)) if grad else phi


def direct_dist(targets, sources, q, shifts=None, grad=True):
    """The biharmonic kernel: phi(y) = sum_p sum_j q_j |y - x_j - p| (K(0) = 0) over
    the given shifts (default: none, the free-space sum), and grad phi."""
    tx, ty, tz = _cols(targets)
    sx, sy, sz = _cols(sources)
    px, py, pz = _cols(np.zeros((1, 3)) if shifts is None else shifts)
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)] if grad else None
    null = ctypes.POINTER(ctypes.c_double)()
    lib().orc_direct_dist(n, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz), _p(sq),
                          px.size, _p(px), _p(py), _p(pz), _p(phi),
                          *(tuple(_p(a) for a in g) if grad else (null, null, null)))
    return (phi, np.stack(g, axis=1)) if grad else phi


def ewald_bih_real(targets, sources, q, shifts, alpha, rcut):
    tx, ty, tz = _cols(targets)
    sx, sy, sz = _cols(sources)
    px, py, pz = _cols(shifts)
    sq = np.ascontiguousarray(q, dtype=np.float64)
    n = tx.size
    phi = np.zeros(n)
    g = [np.zeros(n) for _ in range(3)]
    lib().orc_ewald_bih_real(n, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz), _p(sq),
                             px.size, _p(px), _p(py), _p(pz), float(alpha), float(rcut),
                             _p(phi), *(_p(a) for a in g))
    return phi, np.stack(g, axis=1)
