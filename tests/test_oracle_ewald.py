"""Pins for the FP64 Ewald correction (periodic gravity of the box's total mass, Sec. 4.1 / 4.3).

Checked against what the mathematics fixes, not against the formula itself: the simple-cubic
lattice constant, independence from the splitting parameter alpha (a wrong sign, factor or dropped
term in either the real-space or the wave-vector sum breaks it), force = -grad(potential), the
cubic symmetry points, and the harmonic pull of the neutralising background near the centre.

The box's second-moment terms are pinned by the exact sum they approximate: the corrections of a
small cluster's particles, each taken as a monopole at its own position, differ from the expansion
about the cluster's centre of mass by O(size^3) with the second moment and by O(size^2) without
it (a wrong sign, factor, trace term or component order leaves an O(size^2) error).  An isotropic
second moment adds no force (the kernel's Laplacian is the background's constant 4 pi / L^3) and
shifts the potential by -2 pi G s / L^3; alpha independence and force = -grad(potential) hold with
a second moment as without.
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


def moment6(m, y, c):
    d = y - c
    S = np.einsum("j,ja,jb->ab", m, d, d)
    return np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]])


def test_second_moment_matches_the_images_of_a_small_cluster():
    rng = np.random.default_rng(11)
    m = rng.uniform(0.5, 1.5, size=7)
    u = rng.normal(size=(7, 3)) * np.array([1.0, 0.6, 1.4])  # anisotropic, so S has every component
    x = C + rng.uniform(-0.35, 0.35, size=(24, 3))
    err = {"mono": [], "quad": []}
    for size in (0.02, 0.01, 0.005):
        y = C + size * u
        c = (m[:, None] * y).sum(0) / m.sum()
        exact_a, exact_p = np.zeros((len(x), 3)), np.zeros(len(x))
        for j in range(len(m)):
            a, p = O.ewald(x, L, G, m[j], y[j], 2.0, NREP, HMAX2, potential=True)
            exact_a += a
            exact_p += p
        ma, mp = O.ewald(x, L, G, m.sum(), c, 2.0, NREP, HMAX2, potential=True)
        qa, qp = O.ewald(x, L, G, m.sum(), c, 2.0, NREP, HMAX2, potential=True, S=moment6(m, y, c))
        err["mono"].append((np.abs(ma - exact_a).max(), np.abs(mp - exact_p).max()))
        err["quad"].append((np.abs(qa - exact_a).max(), np.abs(qp - exact_p).max()))
    for k in range(2):  # acceleration, potential
        mono = [e[k] for e in err["mono"]]
        quad = [e[k] for e in err["quad"]]
        for i in range(2):
            assert 3.6 < mono[i] / mono[i + 1] < 4.4, mono
            assert 7.2 < quad[i] / quad[i + 1] < 8.8, quad
        assert quad[-1] < 0.05 * mono[-1]


def test_isotropic_second_moment_adds_no_force():
    x = np.random.default_rng(12).uniform(0, L, size=(30, 3))
    s = 0.013
    a0, p0 = ew(x, 2.0, potential=True)
    a1, p1 = O.ewald(x, L, G, M, C, 2.0, NREP, HMAX2, potential=True, S=[s, s, s, 0, 0, 0])
    assert np.abs(a1 - a0).max() <= 1e-11 * np.abs(a0).max()
    assert np.abs((p1 - p0) - (-2 * np.pi * G * s / L**3)).max() <= 1e-11


S_ANISO = np.array([0.021, 0.008, 0.013, 0.004, -0.006, 0.0025])


def test_second_moment_independent_of_the_splitting_parameter():
    x = np.random.default_rng(13).uniform(0, L, size=(40, 3))
    a2, p2 = O.ewald(x, L, G, M, C, 2.0, NREP, HMAX2, potential=True, S=S_ANISO)
    m2 = O.ewald(x, L, G, M, C, 2.0, NREP, HMAX2)
    assert np.abs(a2 - m2).max() > 1e-3 * np.abs(m2).max()  # the terms are not negligible here
    for alpha in (2.5, 3.2):
        a, p = O.ewald(x, L, G, M, C, alpha, NREP, HMAX2, potential=True, S=S_ANISO)
        assert np.abs(a - a2).max() <= 1e-10 * np.abs(a2).max()
        assert np.abs(p - p2).max() <= 1e-10 * np.abs(p2).max()


def test_second_moment_force_is_minus_gradient_of_potential():
    x = np.random.default_rng(14).uniform(0, L, size=(10, 3))
    a = O.ewald(x, L, G, M, C, 2.0, NREP, HMAX2, S=S_ANISO)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        _, pp = O.ewald(x + e, L, G, M, C, 2.0, NREP, HMAX2, potential=True, S=S_ANISO)
        _, pm = O.ewald(x - e, L, G, M, C, 2.0, NREP, HMAX2, potential=True, S=S_ANISO)
        assert np.abs(a[:, d] + (pp - pm) / (2 * h)).max() <= 1e-7 * np.abs(a).max()


def test_second_moment_near_the_centre_and_across_the_series_switch():
    # the central copy's kernels take their series below alpha s = 1 and the recursion above: both
    # must give the same smooth function, finite at the centre, where the force vanishes by symmetry
    alpha = 2.0
    e = np.array([0.48, -0.6, 0.64])  # a unit direction
    s = np.array([0.0, 1e-6, 0.5 / alpha - 1e-8, 0.5 / alpha + 1e-8, 1.0 / alpha - 1e-8, 1.0 / alpha + 1e-8])
    a, p = O.ewald(C + s[:, None] * e, L, G, M, C, alpha, NREP, HMAX2, potential=True, S=S_ANISO)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(p))
    assert np.abs(a[0]).max() <= 1e-12
    assert abs(p[0] - p[1]) <= 1e-9
    assert np.abs(a[4] - a[5]).max() <= 1e-7 and abs(p[4] - p[5]) <= 1e-7
    assert np.abs(a[2] - a[3]).max() <= 1e-7 and abs(p[2] - p[3]) <= 1e-7
