"""Pins for the FP64 Lennard-Jones checker: closed forms, brute force with minimum image, conservation."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _two_atoms(r, types=(0, 0), L=20.0, rcut=2.5, prm=None):
    prm = prm or dict(eps_t=[1.0, 0.5], sig_t=[1.0, 0.88], mass_t=[1.0, 2.0])
    xyz = np.array([[5.0, 6.0, 7.0], [5.0 + r, 6.0, 7.0]])
    return W.build_lj(xyz, np.array(types), [L, L, L], rcut, **prm)


def _pair_force_x(w):
    acc = O.lj_brute(w)
    m = w.mass_t[w.rec[:, 3].astype(int)]
    i = int(np.argmin(w.rec[:, 0]))  # atom on the left
    return acc[i, 0] * m[i]


@pytest.mark.parametrize("types", [(0, 0), (1, 1), (0, 1)])
def test_zero_force_at_potential_minimum(types):
    e_t, s_t = np.array([1.0, 0.5]), np.array([1.0, 0.88])
    s = 0.5 * (s_t[types[0]] + s_t[types[1]])
    rmin = 2 ** (1 / 6) * s
    # positions are FP32: test the sign change across r_min and the magnitude near it
    f_in = _pair_force_x(_two_atoms(rmin * 0.999, types))
    f_out = _pair_force_x(_two_atoms(rmin * 1.001, types))
    assert f_in < 0 < f_out  # left atom pushed left inside r_min, pulled right outside
    f_at = _pair_force_x(_two_atoms(rmin, types))
    assert abs(f_at) < 1e-4 * 24 * math.sqrt(e_t[types[0]] * e_t[types[1]]) / s


def test_force_at_sigma_closed_form():
    # |F(sigma)| = 24 eps / sigma, repulsive
    e32 = np.float32([1.0, 0.5]).astype(np.float64)  # parameters are FP32 inputs, promoted
    s32 = np.float32([1.0, 0.88]).astype(np.float64)
    for types in [(0, 0), (1, 1), (0, 1)]:
        eps = math.sqrt(e32[types[0]] * e32[types[1]])
        sig = 0.5 * (s32[types[0]] + s32[types[1]])
        w = _two_atoms(sig, types)
        r = float(w.rec[1, 0]) - float(w.rec[0, 0])  # actual FP32 separation
        want = 24 * eps * (2 * (sig / r) ** 12 - (sig / r) ** 6) / r
        np.testing.assert_allclose(-_pair_force_x(w), want, rtol=1e-12)
        np.testing.assert_allclose(want, 24 * eps / sig, rtol=2e-5)


def test_potential_minimum_depth():
    w = _two_atoms(2 ** (1 / 6), (0, 0))
    _, pot = O.lj_brute(w, potential=True)
    np.testing.assert_allclose(pot.sum(), -1.0, rtol=1e-10)


def test_cutoff_is_strict():
    assert _pair_force_x(_two_atoms(2.6)) == 0.0
    assert _pair_force_x(_two_atoms(2.4)) != 0.0


def test_cell_tasks_equal_minimum_image_brute_force():
    w = W.lj_small()
    a_t, pot_t, n_in = O.lj_tasks(w, potential=True)
    a_b, pot_b = O.lj_brute(w, potential=True)
    np.testing.assert_allclose(a_t, a_b, rtol=1e-11, atol=1e-11 * np.abs(a_b).max())
    np.testing.assert_allclose(pot_t.sum(), pot_b.sum(), rtol=1e-12)
    assert n_in > 0


def test_cell_tasks_periodic_box_crossing():
    # an FCC box whose atoms sit near every face: forces equal the minimum-image brute force
    xyz, _, L = W.fcc_modulated(5, 5, 5, 0.8442, 400, seed=9)
    w = W.build_lj(xyz, W.two_types(400, 3), L, 2.5, **W.LJ_TWO_TYPES)
    a_t = O.lj_tasks(w)
    a_b = O.lj_brute(w)
    np.testing.assert_allclose(a_t, a_b, rtol=1e-11, atol=1e-11 * np.abs(a_b).max())


def test_newton_third_law_lj():
    w = W.lj_small()
    acc = O.lj_tasks(w)
    m = w.mass_t[w.rec[:, 3].astype(int)].astype(np.float64)
    net = np.sum(m[:, None] * acc, axis=0)
    assert np.linalg.norm(net) <= 1e-12 * np.sum(m * np.linalg.norm(acc, axis=1))


def test_lj_energy_conservation_velocity_verlet():
    # single type, shifted potential; velocity Verlet with cells rebuilt every step
    xyz, L = W.simple_cubic(8, 0.8442, seed=31)
    n = xyz.shape[0]
    rng = np.random.default_rng(31)
    v = rng.normal(size=(n, 3)) * 0.5
    v -= v.mean(0)
    prm = dict(eps_t=[1.0], sig_t=[1.0], mass_t=[1.0])
    rc = 2.5
    u_rc = 4 * (rc**-12 - rc**-6)
    dt, steps = 0.002, 150

    def force(x):
        w = W.build_lj(x, np.zeros(n, np.int32), L, rc, **prm)
        a, pot, nin = O.lj_tasks(w, potential=True)
        out = np.empty_like(a)
        out[w.perm] = a
        return out, pot.sum() - nin * u_rc

    x = W.wrap_box(xyz, L).astype(np.float64)
    a, U = force(x)
    E0 = 0.5 * np.sum(v * v) + U
    for _ in range(steps):
        v = v + 0.5 * dt * a
        x = np.mod(x + dt * v, L)
        a, U = force(x)
        v = v + 0.5 * dt * a
    E1 = 0.5 * np.sum(v * v) + U
    # truncated (not shifted) force: a small drift from pairs crossing r_c; a wrong force explodes
    assert abs(E1 - E0) <= 2e-3 * abs(E0), (E0, E1)


def test_lj_force_is_minus_energy_gradient():
    # F_i = -dU/dx_i by central differences of the total potential energy (decisions frozen)
    w = W.lj_small()
    pos = w.rec[:, :3].astype(np.float64)
    m = w.mass_t[w.rec[:, 3].astype(int)].astype(np.float64)
    F = O.lj_tasks(w) * m[:, None]
    rng = np.random.default_rng(32)
    h = 1e-6
    for i in rng.choice(w.n, size=15, replace=False):
        for q in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, q] += h
            p2[i, q] -= h
            g = (O.lj_energy_at(w, p1) - O.lj_energy_at(w, p2)) / (2 * h)
            assert abs(F[i, q] + g) <= 1e-6 * max(1.0, abs(F[i]).max()), (i, q, F[i, q], g)
