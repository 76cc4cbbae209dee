"""Pins for the oracle's geometry: check-point counts, partners, near-set sizes
(Sec. 2.2-2.3, eq. (o2.1), Tables 2, 3 and 5)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle.checkpoints import gauss_sphere, partners
from oracle.geometry import circumradius, geometric_factor, lattice_vectors, near_set

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("table", ["table2", "table3"])
def test_evaluation_point_counts_match_tables(table):
    """N + 2L with L = 2p^2 - p Gauss-grid check points (Fig. 2 caption, Sec. 4.2)
    reproduces the N+2L column of Tables 2 and 3 exactly."""
    t = GOLD[table]
    for lam, p, nb, n2l in t["rows"]:
        L = gauss_sphere(p, 1.0).shape[0]
        assert L == 2 * p * p - p
        assert t["N"] + 2 * L == n2l


def test_check_points_on_sphere_and_partners_inside():
    for box in [(1, 1, 1), (1, 1, 2.5), (2, 1, 1), (1.3, 1.9, 1.1)]:
        R0 = circumradius(box)
        for p in (8, 12, 20):
            y = gauss_sphere(p, R0)
            np.testing.assert_allclose(np.linalg.norm(y, axis=1), R0, rtol=1e-14)
            yt, k = partners(y, box)
            d = np.asarray(box, float)
            # partner differs by exactly one box period along one axis
            diff = y - yt
            nz = np.abs(diff) > 0
            assert np.all(nz.sum(axis=1) == 1)
            np.testing.assert_allclose(np.abs(diff[np.arange(len(k)), k]), d[k], rtol=1e-15)
            # the partner lies strictly inside S0 (algorithm "set", step 3)
            assert np.all(np.linalg.norm(yt, axis=1) < R0 * (1 - 1e-6))


def test_geometric_factor_matches_table5():
    t = GOLD["table5"]
    for box, agf in zip(t["boxes"], t["A_gf"]):
        assert abs(geometric_factor(box) - agf) < 0.006 * agf


def test_table_near_counts_consistent_with_ball():
    """Expected N_b = A_gf lambda^3 N (eq. (o2.1)); the tables' random-source counts
    must sit within a few standard deviations (sqrt N_b) of it."""
    for key in ("table2", "table3"):
        t = GOLD[key]
        for lam, p, nb, _ in t["rows"]:
            mean = geometric_factor((1, 1, 1)) * lam ** 3 * t["N"]
            assert abs(nb - mean) < 6 * np.sqrt(mean)
    t = GOLD["table5"]
    for box, nb in zip(t["boxes"], t["N_b"]):
        mean = geometric_factor(box) * t["lambda"] ** 3 * t["N"]
        assert abs(nb - mean) < 6 * np.sqrt(mean)


@pytest.mark.parametrize("box,lam", [((1, 1, 1), 1.3), ((2, 1, 1), 1.3), ((1, 1, 2.5), 1.5)])
def test_oracle_near_set_size(box, lam):
    n = 20000
    x, q = W.uniform_box(n, box, seed=11)
    Rb = lam * circumradius(box)
    xs, qs, base, img = near_set(x, q, box, Rb)
    mean = geometric_factor(box) * lam ** 3 * n
    assert abs(xs.shape[0] - mean) < 6 * np.sqrt(mean)
    assert np.all(np.linalg.norm(xs, axis=1) <= Rb * (1 + 1e-12))
    # image 0 holds every particle unchanged and first
    assert np.array_equal(base[:n], np.arange(n)) and np.all(img[:n] == 0)
    np.testing.assert_array_equal(xs[:n], x)


def test_near_set_is_complete():
    """Every lattice image inside the ball is found: brute force over a wider
    lattice finds no extra points."""
    box = (1.0, 1.4, 0.8)
    x, q = W.uniform_box(300, box, seed=5)
    Rb = 1.6 * circumradius(box)
    xs, _, _, _ = near_set(x, q, box, Rb)
    d = np.asarray(box)
    cnt = 0
    for i in range(-5, 6):
        for j in range(-5, 6):
            for k in range(-5, 6):
                y = x + np.array([i, j, k]) * d
                cnt += int(np.sum(np.linalg.norm(y, axis=1) <= Rb))
    assert cnt == xs.shape[0]


def test_lattice_starts_at_zero():
    P = lattice_vectors((1, 1, 1), 1.5)
    assert np.all(P[0] == 0) and P.shape[0] == 125
