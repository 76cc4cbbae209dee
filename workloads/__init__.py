"""Seeded synthetic inputs for the periodic Coulomb sum.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic, so both the FP64 oracle and the HIP path can consume the
same inputs without sharing any code of the method.

Every generator uses numpy's PCG64 with seed ``20131015 + k`` (k = the
workload number below) unless a seed is passed.  Positions are wrapped into the
half-open box [-d/2, d/2) per axis; charges are exactly neutral in the sense the
method needs (sum below 1e-12 of the sum of magnitudes).

Workloads (the paper's test systems are synthetic: a rock-salt cell in the
small-size tests, random charges in a unit cube in the large-scale tests, and
boxes of several aspect ratios):

1. cube 1x1x1, N=1000 uniform, q=+-1 (500 each, shuffled)
2. cube 1x1x1, N=100,000 uniform, q ~ N(0,1) minus its mean, with a seeded
   2,000-particle subset for sampled comparisons
3. box 1x1x2.5, N=1,000,000 in 64 Gaussian blobs (sigma = 0.03 d_k per axis,
   wrapped), q=+-1 balanced
4. 512 independent boxes, d_k ~ U[1,2], N ~ log-uniform[200, 20000], uniform
   positions, q ~ N(0,1) minus the mean
5. rock-salt lattice of 32^3 sites (spacing 1/32 in a unit cube), q=(-1)^(i+j+k),
   positions jittered by N(0, 0.002^2) per coordinate
"""
import functools

import numpy as np

BASE_SEED = 20131015


def rng(k, seed=None):
    return np.random.Generator(np.random.PCG64(BASE_SEED + k if seed is None else seed))


def wrap(x, d):
    """Map coordinates into [-d/2, d/2) per axis (x: (N,3), d: (3,))."""
    d = np.asarray(d, dtype=np.float64)
    x = x - d * np.floor(x / d + 0.5)
    # guard the half-open upper edge against rounding
    x = np.where(x >= d / 2, x - d, x)
    x = np.where(x < -d / 2, x + d, x)
    return np.ascontiguousarray(x)


def _neutral_pm1(g, n):
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    g.shuffle(q)
    return q


def _neutral_gauss(g, n):
    q = g.standard_normal(n)
    return q - q.mean()


def uniform_box(n, box, charges="pm1", seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    d = np.asarray(box, dtype=np.float64)
    x = wrap((g.random((n, 3)) - 0.5) * d, d)
    q = _neutral_pm1(g, n) if charges == "pm1" else _neutral_gauss(g, n)
    return x, q


def config1():
    g = rng(1)
    d = np.array([1.0, 1.0, 1.0])
    x = wrap((g.random((1000, 3)) - 0.5) * d, d)
    return dict(box=d, x=x, q=_neutral_pm1(g, 1000), p=12, R_b=1.5)


def config2(n=100_000, nsub=2000):
    g = rng(2)
    d = np.array([1.0, 1.0, 1.0])
    x = wrap((g.random((n, 3)) - 0.5) * d, d)
    q = _neutral_gauss(g, n)
    sub = np.sort(g.choice(n, size=min(nsub, n), replace=False))
    return dict(box=d, x=x, q=q, p=16, R_b=1.5, subset=sub)


def config3(n=1_000_000, nblob=64, nsub=2000):
    g = rng(3)
    d = np.array([1.0, 1.0, 2.5])
    centres = (g.random((nblob, 3)) - 0.5) * d
    per = n // nblob
    counts = np.full(nblob, per)
    counts[: n - per * nblob] += 1
    lab = np.repeat(np.arange(nblob), counts)
    x = centres[lab] + g.standard_normal((n, 3)) * (0.03 * d)
    x = wrap(x, d)
    q = _neutral_pm1(g, n)
    sub = np.sort(g.choice(n, size=min(nsub, n), replace=False))
    return dict(box=d, x=x, q=q, p=20, lam=1.5, subset=sub)


def config_screened(n=100_000, nsub=2000):
    """Screened-kernel workload (exp(-kappa r)/r, kappa = 2): N uniform in the unit
    cube, Gaussian charges plus 0.05 (a net charge, which this kernel allows),
    the kernel at M = 256 Thomson centres on the sphere of radius 1.5 R0,
    R0 = |d|/2, as the basis (eq. (5)); p = 16 sets the Gauss check grid."""
    g = rng(6)
    d = np.array([1.0, 1.0, 1.0])
    x = wrap((g.random((n, 3)) - 0.5) * d, d)
    q = g.standard_normal(n) + 0.05
    sub = np.sort(g.choice(n, size=min(nsub, n), replace=False))
    centres = thomson_points(256, 1.5 * 0.5 * float(np.linalg.norm(d)))
    return dict(box=d, x=x, q=q, p=16, lam=1.5, kappa=2.0, centres=centres, subset=sub)


def config_partial(periodic, n=100_000, nsub=2000):
    """The uniform-cube workload with fewer periodic axes: "xy" (a slab, z free)
    or "x" (a wire, y and z free).  N uniform in the unit cube, Gaussian charges
    minus their mean, p = 16, lambda = 1.5."""
    g = rng({"xy": 7, "x": 8}[periodic])
    d = np.array([1.0, 1.0, 1.0])
    x = wrap((g.random((n, 3)) - 0.5) * d, d)
    q = _neutral_gauss(g, n)
    sub = np.sort(g.choice(n, size=min(nsub, n), replace=False))
    return dict(box=d, x=x, q=q, p=16, lam=1.5, periodic=periodic, subset=sub)


def config_plane(n=100_000, nsub=2000):
    """The method in the plane (kernel -log r): N uniform in the unit square,
    Gaussian charges minus their mean, p = 32, lambda = 1.5.  Positions (N, 2)."""
    g = rng(9)
    d = np.array([1.0, 1.0])
    x = wrap((g.random((n, 2)) - 0.5) * d, d)
    q = _neutral_gauss(g, n)
    sub = np.sort(g.choice(n, size=min(nsub, n), replace=False))
    return dict(box=d, x=x, q=q, p=32, lam=1.5, subset=sub)


def config_biharmonic(n=100_000, nsub=2000):
    """The biharmonic kernel r: N uniform in the unit cube, Gaussian charges
    minus their mean, p = 24 (P = 24^2 + 22^2 = 1060), lambda = 1.5."""
    g = rng(10)
    d = np.array([1.0, 1.0, 1.0])
    x = wrap((g.random((n, 3)) - 0.5) * d, d)
    q = _neutral_gauss(g, n)
    sub = np.sort(g.choice(n, size=min(nsub, n), replace=False))
    return dict(box=d, x=x, q=q, p=24, lam=1.5, subset=sub)


def config4(nsys=512, nmin=200, nmax=20000):
    g = rng(4)
    systems = []
    for _ in range(nsys):
        d = g.uniform(1.0, 2.0, size=3)
        n = int(round(np.exp(g.uniform(np.log(nmin), np.log(nmax)))))
        x = wrap((g.random((n, 3)) - 0.5) * d, d)
        q = _neutral_gauss(g, n)
        systems.append(dict(box=d, x=x, q=q))
    return dict(systems=systems, p=12, lam=float(np.sqrt(3.0)))


def rocksalt(m=32, jitter=0.0, seed=None):
    """m^3 sites -1/2 + (i+1/2)/m of a unit cube, q = (-1)^(i+j+k)."""
    g = rng(5, seed)
    i = np.arange(m)
    I, J, K = np.meshgrid(i, i, i, indexing="ij")
    s = (np.stack([I, J, K], axis=-1).reshape(-1, 3) + 0.5) / m - 0.5
    q = np.where(((I + J + K).reshape(-1) % 2) == 0, 1.0, -1.0)
    d = np.array([1.0, 1.0, 1.0])
    if jitter > 0:
        s = s + g.normal(0.0, jitter, size=s.shape)
    return dict(box=d, x=wrap(s, d), q=q, spacing=1.0 / m)


def config5(jitter=0.002):
    r = rocksalt(32, jitter=jitter)
    r.update(p=16, R_b=1.5)
    return r


def nacl_cell(d=1.0):
    """Eight charges at (+-d/4, +-d/4, +-d/4) with q = s1*s2*s3: one rock-salt
    cell of period d, nearest-neighbour distance d/2."""
    s = np.array([[a, b, c] for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)], dtype=np.float64)
    x = s * (d / 4.0)
    q = s[:, 0] * s[:, 1] * s[:, 2]
    return dict(box=np.array([d, d, d]), x=x, q=q)


def fibonacci_sphere(m, radius):
    """m nearly uniform points on a sphere (spherical Fibonacci lattice):
    z_t = 1 - (2t + 1)/m, azimuth t * pi (3 - sqrt 5).  Deterministic and cheap;
    also the starting point of thomson_points."""
    t = np.arange(m, dtype=np.float64)
    z = 1.0 - (2.0 * t + 1.0) / m
    ph = t * np.pi * (3.0 - np.sqrt(5.0))
    r = np.sqrt(1.0 - z * z)
    return np.ascontiguousarray(radius * np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1))


def grid_charges(m, seed):
    """m^3 charges at the cell centres of a regular m x m x m grid in the unit cube
    [-1/2, 1/2)^3, with random signs, m^3/2 of each (m even): the accuracy and
    parameter-choice tests of Sec. 4.2 (Tables 2 and 3, Figs. 4-6)."""
    g = (np.arange(m, dtype=np.float64) + 0.5) / m - 0.5
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    n = m ** 3
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    rng(seed).shuffle(q)
    return np.ascontiguousarray(x), q


def thomson_energy(x):
    """Coulomb energy sum_{i<j} 1/|x_i - x_j| of a point set."""
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    iu = np.triu_indices(len(x), 1)
    return float(np.sum(1.0 / d[iu]))


def _thomson_energy_grad(v):
    """Energy of the points v/|v| (flattened) and its gradient with respect to v."""
    y = v.reshape(-1, 3)
    n = np.linalg.norm(y, axis=1)
    x = y / n[:, None]
    dv = x[:, None, :] - x[None, :, :]
    r2 = (dv ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    inv = 1.0 / np.sqrt(r2)
    e = 0.5 * float(inv.sum())
    gx = -(dv * (inv ** 3)[..., None]).sum(1)           # dE/dx_i
    g = (gx - (gx * x).sum(1)[:, None] * x) / n[:, None]  # through the normalization
    return e, g.ravel()


@functools.lru_cache(maxsize=16)
def _thomson_unit(m, gtol):
    from scipy.optimize import minimize
    x0 = fibonacci_sphere(m, 1.0)
    if m < 2:
        return x0
    res = minimize(_thomson_energy_grad, x0.ravel(), jac=True, method="L-BFGS-B",
                   options={"maxiter": 20000, "gtol": gtol, "ftol": 0.0, "maxcor": 30})
    x = res.x.reshape(-1, 3)
    return np.ascontiguousarray(x / np.linalg.norm(x, axis=1)[:, None])


def thomson_points(m, radius, gtol=1e-10):
    """m points on a sphere at a local minimum of their mutual Coulomb energy (the
    Thomson problem), for check points and RBF centres.  Deterministic: L-BFGS on
    the energy of the normalized points, started from the Fibonacci lattice.
    Stands in for a database of Thomson points."""
    return np.ascontiguousarray(radius * _thomson_unit(int(m), float(gtol)))


def random_sphere(m, radius, seed):
    """m points uniform on a sphere (seeded), for random check-point sets."""
    g = np.random.Generator(np.random.PCG64(seed))
    v = g.standard_normal((m, 3))
    return np.ascontiguousarray(radius * v / np.linalg.norm(v, axis=1)[:, None])
