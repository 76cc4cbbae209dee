"""Pins for the oracle's classical Ewald sum (App. D) against the Madelung
constant (eq. (st1)), its splitting-parameter independence and brute-force
image sums over expanding cubes."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import _native
from oracle.ewald import Ewald, MADELUNG_NACL

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def test_madelung_constant_paper_value():
    assert abs(GOLD["madelung_nacl"]["value"] + MADELUNG_NACL) < 1e-17


def test_ewald_madelung():
    c = W.nacl_cell()
    phi, E = Ewald(c["box"]).solve(c["x"], c["q"])
    # phi at a site times the nearest-neighbour distance (d/2) is -q * M
    np.testing.assert_allclose(phi * 0.5, -c["q"] * MADELUNG_NACL, rtol=1e-14)
    assert np.abs(E).max() < 1e-12


def test_ewald_madelung_lattice16():
    """The 32^3-site rock-salt lattice (nearest-neighbour 1/32)."""
    r = W.rocksalt(8)
    phi, _ = Ewald(r["box"], xi=12.0).solve(r["x"], r["q"])
    np.testing.assert_allclose(phi * r["spacing"], -r["q"] * MADELUNG_NACL, rtol=1e-13)


@pytest.mark.parametrize("box", [(1.0, 1.0, 1.0), (1.0, 1.3, 2.1)])
def test_ewald_independent_of_splitting(box):
    x, q = W.uniform_box(60, box, charges="gauss", seed=9)
    a = Ewald(box, xi=4.0 / min(box)).solve(x, q)
    b = Ewald(box, xi=7.0 / min(box)).solve(x, q)
    for u, v in zip(a, b):
        assert np.linalg.norm(u - v) / np.linalg.norm(v) < 1e-13


def _zero_dipole_cell(seed, box):
    g = np.random.default_rng(seed)
    d = np.asarray(box, float)
    while True:
        x = (g.random((8, 3)) - 0.5) * d * 0.7
        q = np.array([1.0, -1, 1, -1, 1, -1, 1, -1])
        D = (q[:, None] * x).sum(0)
        x[0] -= D                         # q_0 = +1: removes the dipole
        if np.all(np.abs(x) < d / 2):
            return x, q


def test_ewald_matches_cube_shell_brute_force():
    """Direct image sums over expanding cubes |i|_inf <= K of a neutral cell with
    zero dipole converge to the conducting-boundary (Ewald) field, and to its
    potential up to one constant; Richardson extrapolation in K (error ~ K^-2)."""
    box = (1.0, 1.0, 1.0)
    x, q = _zero_dipole_cell(1, box)
    res = []
    for K in (24, 48):
        r = np.arange(-K, K + 1)
        I, J, L = np.meshgrid(r, r, r, indexing="ij")
        shifts = np.stack([I.ravel(), J.ravel(), L.ravel()], 1).astype(float)
        phi, g = _native.direct_images(x, x, q, shifts)
        res.append((phi, -g))
    phi_bf = (4 * res[1][0] - res[0][0]) / 3
    E_bf = (4 * res[1][1] - res[0][1]) / 3
    phi_e, E_e = Ewald(box).solve(x, q)
    dphi = (phi_bf - phi_bf.mean()) - (phi_e - phi_e.mean())
    assert np.abs(dphi).max() < 1e-6 * np.abs(phi_e).max()
    assert np.abs(E_bf - E_e).max() < 1e-6 * np.abs(E_e).max()


def test_ewald_net_force_zero():
    x, q = W.uniform_box(80, (1.2, 1.0, 0.9), charges="gauss", seed=4)
    _, E = Ewald((1.2, 1.0, 0.9)).solve(x, q)
    F = q[:, None] * E
    assert np.abs(F.sum(0)).max() < 1e-11 * np.abs(F).sum()
