"""Pins for the FP64 Ewald correction (periodic gravity of the box's total mass, Sec. 4.1 / 4.3).

Checked against what the mathematics fixes, not against the formula itself: the simple-cubic
lattice constant, independence from the splitting parameter alpha (a wrong sign, factor or dropped
term in either the real-space or the wave-vector sum breaks it), force = -grad(potential), the
cubic symmetry points, and the harmonic pull of the neutralising background near the centre.
"""
import numpy as np
import pytest

import oracle as O

L, G, M = 1.0, 1.0, 1.0
C = np.array([0.3, 0.45, 0.6])
NREP, HMAX2 = 3, 64  # converged to ~1e-13 for alpha L in [2, 3]


def ew(x, alpha, potential=False):
    return O.ewald(np.atleast_2d(x), L, G, M, C, alpha, NREP, HMAX2, potential=potential)


@pytest.mark.parametrize("alpha", [2.0, 2.5, 3.0])
def test_simple_cubic_lattice_constant(alpha):
    # the potential of the periodic images plus background at the mass itself: 2.837297479 G M / L
    _, p = ew(C, alpha, potential=True)
    assert abs(p[0] * L / (G * M) - 2.837297479) < 1e-9


def test_independent_of_the_splitting_parameter():
    x = np.random.default_rng(3).uniform(0, L, size=(40, 3))
    a2, p2 = ew(x, 2.0, potential=True)
    for alpha in (2.5, 3.2):
        a, p = ew(x, alpha, potential=True)
        assert np.abs(a - a2).max() <= 1e-10 * np.abs(a2).max()
        assert np.abs(p - p2).max() <= 1e-10 * np.abs(p2).max()


def test_force_is_minus_gradient_of_potential():
    x = np.random.default_rng(4).uniform(0, L, size=(10, 3))
    a = ew(x, 2.0)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        _, pp = ew(x + e, 2.0, potential=True)
        _, pm = ew(x - e, 2.0, potential=True)
        g = (pp - pm) / (2 * h)
        assert np.abs(a[:, d] + g).max() <= 1e-7 * np.abs(a).max()


def test_zero_at_symmetry_points_and_odd_about_the_mass():
    half = L / 2
    # the full periodic force (correction plus the central copy's direct pull) vanishes where the
    # lattice is symmetric: body, face and edge centres between the images
    r = np.array([[half, half, half], [half, 0, 0], [0, half, 0], [0, 0, half], [half, half, 0]])
    x = C + r
    rw = (x - C) - L * np.rint((x - C) / L)  # the copy the correction takes as central (a tie: either)
    direct = -G * M * rw / np.linalg.norm(rw, axis=1)[:, None] ** 3
    assert np.abs(ew(x, 2.0) + direct).max() <= 1e-12
    assert np.abs(ew(C, 2.0)).max() <= 1e-12
    r = np.random.default_rng(5).uniform(-half, half, size=(20, 3))
    assert np.abs(ew(C + r, 2.0) + ew(C - r, 2.0)).max() <= 1e-12


def test_background_pull_near_the_mass():
    # the images cancel to first order by cubic symmetry; the uniform background of density -M/L^3
    # pushes outwards: a = 4 pi G M r / (3 L^3) + O(r^3)
    r = 1e-3 * np.array([[1.0, 0.0, 0.0], [0.3, -0.7, 0.2], [0.0, 0.0, -1.0]])
    a = ew(C + r, 2.0)
    want = 4 * np.pi * G * M / (3 * L**3) * r
    assert np.abs(a - want).max() <= 1e-5 * np.abs(want).max()
