"""Classical Ewald summation (paper App. D, eqs. (e1)-(e6)) as an independent
FP64 reference for periodic potentials and fields.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The split K = K1 + K2 with K1 = erfc(xi r)/r (K1(0) = -2 xi/sqrt(pi)) and
K2 = erf(xi r)/r follows eq. (e1).  The real-space part sums K1 over images
within a cut-off (eq. (e3)).  The smooth part K2 is written as its exact Fourier
series with the k = 0 mode removed -- the explicit sum that the paper's gridded
Gaussian spreading + FFT approximates (eqs. (e4)-(e5)).  With the zero mode
removed and net charge zero the cell mean of phi is zero (eq. (e6)), the
convention the method's constant C1 reproduces.  No surface (dipole) term is
added (conducting boundary).
"""
import math

import numpy as np

from . import _native


class Ewald:
    def __init__(self, box, xi=None, tol=1e-16):
        self.box = np.asarray(box, dtype=np.float64)
        dmin = float(self.box.min())
        self.xi = float(xi) if xi is not None else 5.0 / dmin
        a = math.sqrt(-math.log(tol))           # erfc(a) ~ e^{-a^2}: a ~ 6
        self.rcut = a / self.xi
        self.kmax = 2.0 * self.xi * a
        self.V = float(np.prod(self.box))
        nmax = np.ceil(self.kmax * self.box / (2 * np.pi)).astype(int)
        g = [np.arange(-n, n + 1) for n in nmax]
        N1, N2, N3 = np.meshgrid(*g, indexing="ij")
        n = np.stack([N1.ravel(), N2.ravel(), N3.ravel()], axis=1)
        n = n[np.any(n != 0, axis=1)]
        k = 2 * np.pi * n / self.box[None, :]
        k2 = (k * k).sum(1)
        sel = k2 <= self.kmax ** 2
        self.k = k[sel]
        k2 = k2[sel]
        self.w = (4 * np.pi / self.V) * np.exp(-k2 / (4 * self.xi ** 2)) / k2
        # images whose box can come within rcut of the unit cell
        m = np.ceil(self.rcut / self.box + 1.0).astype(int)
        gi = [np.arange(-v, v + 1) for v in m]
        I1, I2, I3 = np.meshgrid(*gi, indexing="ij")
        self.shifts = np.stack([I1.ravel(), I2.ravel(), I3.ravel()], axis=1) * self.box[None, :]

    def solve(self, x, q, targets=None):
        """phi and field = -grad phi at the targets (default: the particles)."""
        x = np.asarray(x, dtype=np.float64)
        q = np.asarray(q, dtype=np.float64)
        y = x if targets is None else np.asarray(targets, dtype=np.float64)
        # real space: sum over images of K1, skipping coincident points
        phi1, g1 = _native.ewald_real(y, x, q, self.shifts, self.xi, self.rcut)
        # coincident points (the self pair, or a target placed on a source) take K1(0)
        self_q = np.zeros(y.shape[0])
        if targets is None:
            self_q = q.copy()
        else:
            for j in range(x.shape[0]):
                same = np.all(y == x[j][None, :], axis=1)
                self_q[same] += q[j]
        phi1 = phi1 - 2.0 * self.xi / math.sqrt(math.pi) * self_q
        # smooth part: Fourier series of K2 without the k = 0 mode
        ph = self.k @ x.T                                       # (nk, N)
        sre = np.cos(ph) @ q
        sim = np.sin(ph) @ q
        phi2, g2 = _native.ewald_recip(y, self.k, self.w, sre, sim)
        return phi1 + phi2, -(g1 + g2)


MADELUNG_NACL = 1.74756459463318219063621203554  # paper eq. (st1), magnitude
