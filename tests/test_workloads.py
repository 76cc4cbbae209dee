"""Pins for the shared input generators: the Thomson-point minimizer against the
closed-form minimal configurations of the Thomson problem for 2, 4, 6 and 12
points (antipodal pair, tetrahedron, octahedron, icosahedron)."""
import numpy as np
import pytest

import workloads as W


def _icosahedron():
    g = (1 + 5 ** 0.5) / 2
    v = []
    for a in (-1, 1):
        for b in (-1, 1):
            v += [[0, a, b * g], [a, b * g, 0], [b * g, 0, a]]
    v = np.array(v, float)
    return v / np.linalg.norm(v, axis=1)[:, None]


@pytest.mark.parametrize("m, energy", [
    (2, 0.5),
    (4, 6 / np.sqrt(8 / 3)),                       # six edges of length sqrt(8/3)
    (6, 12 / np.sqrt(2) + 3 / 2),                  # twelve edges sqrt 2, three diameters
    (12, None),
])
def test_thomson_points_reach_the_known_minima(m, energy):
    if energy is None:
        energy = W.thomson_energy(_icosahedron())
    x = W.thomson_points(m, 2.0) / 2.0
    assert np.allclose(np.linalg.norm(x, axis=1), 1.0, atol=1e-14)
    assert abs(W.thomson_energy(x) - energy) < 1e-9 * energy


def test_thomson_points_are_stationary_and_below_the_start():
    x = W.thomson_points(256, 1.0)
    _, g = W._thomson_energy_grad(x.ravel())
    assert np.abs(g).max() < 1e-4
    assert W.thomson_energy(x) < W.thomson_energy(W.fibonacci_sphere(256, 1.0)) - 5.0
