"""Ewald summation for charges periodic in x and y only (a slab, vacuum on both
sides in z): an independent FP64 reference for the two-axis periodization.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The kernel is split as in App. D, K = erfc(a r)/r + erf(a r)/r.  The short-range
part is summed over in-plane images within a cut-off.  The smooth part is written
as a Fourier series over the in-plane reciprocal lattice k = 2 pi (n1/d1, n2/d2),
each mode an exact function of the height difference z:
  k != 0:  (pi / (A k)) [e^{k z} erfc(k/(2a) + a z) + e^{-k z} erfc(k/(2a) - a z)] cos(k . rho),
  k  = 0:  -(2 pi / A) [z erf(a z) + exp(-a^2 z^2) / (a sqrt(pi))],
the plane average of a Gaussian-smeared charge (the second derivative in z of
the k = 0 mode is -4 pi times the smeared density, and its slope is odd in z).
With neutral charges the constants dropped from the k = 0 mode cancel.  The
self term -2a/sqrt(pi) q_i is removed at particle targets.  Far from the slab the
field vanishes and the planar mean of phi tends to constants on either side.
"""
import math

import numpy as np
from scipy.special import erf, erfc


class Ewald2D:
    def __init__(self, box, alpha=None, tol=1e-16, zspan=None):
        self.box = np.asarray(box, dtype=np.float64)
        d = self.box
        self.area = d[0] * d[1]
        self.a = float(alpha) if alpha is not None else 4.0 / min(d[0], d[1])
        s = math.sqrt(-math.log(tol))                 # erfc(s) ~ e^{-s^2}
        self.rcut = s / self.a
        zs = float(zspan) if zspan is not None else float(d[2])
        # the growing branch e^{k|z|} erfc(k/(2a) - a|z|) needs k/(2a) - a|z| beyond s
        self.kmax = 2.0 * self.a * (s + self.a * zs)
        nmax = np.ceil(self.kmax * d[:2] / (2 * np.pi)).astype(int)
        n1, n2 = np.meshgrid(np.arange(-nmax[0], nmax[0] + 1), np.arange(-nmax[1], nmax[1] + 1), indexing="ij")
        n = np.stack([n1.ravel(), n2.ravel()], axis=1)
        n = n[np.any(n != 0, axis=1)]
        k = 2 * np.pi * n / d[None, :2]
        kk = np.sqrt((k * k).sum(1))
        sel = kk <= self.kmax
        self.k, self.kk = k[sel], kk[sel]
        m = np.ceil(self.rcut / d[:2] + 1.0).astype(int)
        i1, i2 = np.meshgrid(np.arange(-m[0], m[0] + 1), np.arange(-m[1], m[1] + 1), indexing="ij")
        self.shifts = np.stack([i1.ravel() * d[0], i2.ravel() * d[1], np.zeros(i1.size)], axis=1)

    def _mode(self, z):
        """(F, dF/dz) of every k != 0 mode at height differences z: arrays (nk, ...)."""
        a, k = self.a, self.kk.reshape((-1,) + (1,) * np.ndim(z))
        u1 = k / (2 * a) + a * z
        u2 = k / (2 * a) - a * z
        e1 = np.exp(k * z) * erfc(u1)
        e2 = np.exp(-k * z) * erfc(u2)
        F = (math.pi / (self.area * k)) * (e1 + e2)
        # d/dz: the two erfc-derivative terms are equal and opposite, since
        # kz - u1^2 = -kz - u2^2 = -k^2/(4a^2) - a^2 z^2
        dF = (math.pi / self.area) * (e1 - e2)
        return F, dF

    def solve(self, x, q, targets=None):
        """phi and field = -grad phi at the targets (default: the particles, whose
        own charge is excluded)."""
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y = x if targets is None else np.asarray(targets, dtype=np.float64)
        a = self.a
        phi = np.zeros(y.shape[0])
        grad = np.zeros((y.shape[0], 3))
        # short range: erfc(a r)/r over in-plane images
        for p in self.shifts:
            D = y[:, None, :] - (x[None, :, :] + p[None, None, :])
            r = np.sqrt((D * D).sum(2))
            ok = r > 0.0
            rs = np.where(ok, r, 1.0)
            v = np.where(ok & (r < self.rcut), erfc(a * rs) / rs, 0.0)
            dv = np.where(ok & (r < self.rcut),
                          -(erfc(a * rs) / rs + 2 * a / math.sqrt(math.pi) * np.exp(-a * a * rs * rs)) / (rs * rs), 0.0)
            phi += v @ q
            grad += np.einsum("ij,ijk->ik", dv * q[None, :], D)
        # smooth part, k != 0: sum_j q_j F_k(z_ij) cos(k . rho_ij)
        Z = y[:, None, 2] - x[None, :, 2]
        F, dF = self._mode(Z)                              # (nk, Ny, Nx)
        ph_y = self.k @ y[:, :2].T                         # (nk, Ny)
        ph_x = self.k @ x[:, :2].T                         # (nk, Nx)
        C = np.cos(ph_y)[:, :, None] * np.cos(ph_x)[:, None, :] + np.sin(ph_y)[:, :, None] * np.sin(ph_x)[:, None, :]
        S = np.sin(ph_y)[:, :, None] * np.cos(ph_x)[:, None, :] - np.cos(ph_y)[:, :, None] * np.sin(ph_x)[:, None, :]
        phi += np.einsum("kij,kij,j->i", F, C, q)
        grad[:, 0] += np.einsum("k,kij,kij,j->i", -self.k[:, 0], F, S, q)
        grad[:, 1] += np.einsum("k,kij,kij,j->i", -self.k[:, 1], F, S, q)
        grad[:, 2] += np.einsum("kij,kij,j->i", dF, C, q)
        # smooth part, k = 0: the plane average of the smeared charges
        phi += -(2 * math.pi / self.area) * ((Z * erf(a * Z) + np.exp(-a * a * Z * Z) / (a * math.sqrt(math.pi))) @ q)
        grad[:, 2] += -(2 * math.pi / self.area) * (erf(a * Z) @ q)
        if targets is None:
            phi -= 2 * a / math.sqrt(math.pi) * q
        return phi, -grad
