"""Pins for the FP64 gravity checker: closed forms, brute force, invariants.

Each pin ties the checker to something other than itself: a closed-form
force, an all-pairs sum, a conservation law or a convergence order.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def test_two_body_closed_form():
    # two bodies at distance r along a random axis: |a| = G m r / (r^2 + eps^2)^{3/2}, pointing at the source
    rng = np.random.default_rng(1)
    for _ in range(20):
        r = 10 ** rng.uniform(-3, 1)
        eps = 10 ** rng.uniform(-3, 0)
        G = rng.uniform(0.5, 2.0)
        m = rng.uniform(0.1, 3.0, size=2)
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        pos = np.stack([np.zeros(3), r * e])  # separation exactly r * e
        acc = O.grav_brute(pos, m, G, eps)
        want0 = G * m[1] * r / (r * r + eps * eps) ** 1.5 * e
        want1 = -G * m[0] * r / (r * r + eps * eps) ** 1.5 * e
        assert np.linalg.norm(acc[0] - want0) <= 1e-13 * np.linalg.norm(want0)
        assert np.linalg.norm(acc[1] - want1) <= 1e-13 * np.linalg.norm(want1)


def test_single_particle_monopole_equals_pair_term():
    rng = np.random.default_rng(2)
    xs = rng.normal(size=3)
    m = 0.37
    mom = np.concatenate([xs, [m], np.zeros(6)])
    pts = rng.normal(size=(50, 3)) * 3
    a_node = O.node_acc_points(pts, mom, order=2, G=1.3, eps=0.02)
    for p, a in zip(pts, a_node):
        a_pair = O.grav_brute(np.stack([p, xs]), np.array([1.0, m]), 1.3, 0.02)[0]
        np.testing.assert_allclose(a, a_pair, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("G,m,s", [(1.0, 1.0, 0.5), (2.5, 0.3, 0.1)])
def test_quadrupole_axial_closed_form(G, m, s):
    # eps = 0; masses m at +-s z-hat.  Exact second-order expansions of the potential:
    #  on the z axis:  Phi = -2Gm/z - 2Gm s^2/z^3      => a_z = -2Gm/z^2 - 6Gm s^2/z^4
    #  on the x axis:  Phi = -2Gm/x + Gm s^2/x^3       => a_x = -2Gm/x^2 + 3Gm s^2/x^4
    mom = np.array([0, 0, 0, 2 * m, 0, 0, 2 * m * s * s, 0, 0, 0], float)
    for z in [3.0, 7.0, 20.0]:
        a = O.node_acc_points(np.array([[0, 0, z]]), mom, order=2, G=G, eps=0.0)[0]
        np.testing.assert_allclose(a[2], -2 * G * m / z**2 - 6 * G * m * s * s / z**4, rtol=1e-14)
        assert abs(a[0]) < 1e-300 and abs(a[1]) < 1e-300
        a = O.node_acc_points(np.array([[z, 0, 0]]), mom, order=2, G=G, eps=0.0)[0]
        np.testing.assert_allclose(a[0], -2 * G * m / z**2 + 3 * G * m * s * s / z**4, rtol=1e-14)
    # monopole alone drops the s^2 terms
    a = O.node_acc_points(np.array([[0, 0, 5.0]]), mom, order=1, G=G, eps=0.0)[0]
    np.testing.assert_allclose(a[2], -2 * G * m / 25.0, rtol=1e-14)


def test_multipole_convergence_order():
    # a random cluster of size ~1 viewed from distance d: node error vs the direct sum falls as
    # d^-2 relative (monopole) and d^-3 relative (quadrupole); a wrong quadrupole term stalls at d^-2
    rng = np.random.default_rng(3)
    xk = rng.normal(size=(40, 3)) * 0.3
    mk = rng.uniform(0.5, 1.5, size=40)
    rng_node = np.array([[0, 40]], np.int32)
    mom = O.node_moments(rng_node, xk, mk)[0]
    dirs = rng.normal(size=(16, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    ds = np.array([8.0, 16.0, 32.0, 64.0])
    for order, slope_want in [(1, -2.0), (2, -3.0)]:
        errs = []
        for d in ds:
            pts = mom[:3] + d * dirs
            a_node = O.node_acc_points(pts, mom, order=order, G=1.0, eps=0.01)
            e = []
            for p, an in zip(pts, a_node):
                a_dir = O.grav_brute(np.vstack([p, xk]), np.concatenate([[1.0], mk]), 1.0, 0.01)[0]
                e.append(np.linalg.norm(an - a_dir) / np.linalg.norm(a_dir))
            errs.append(np.median(e))
        slope = np.polyfit(np.log(ds), np.log(errs), 1)[0]
        assert abs(slope - slope_want) < 0.25, (order, slope, errs)


def test_theta_zero_lists_equal_brute_force():
    w = W.build_grav(W.uniform_cube(1500, 11), bucket=16, theta=0.0)
    assert w.n_count.sum() == 0
    rec = w.rec.astype(np.float64)
    a_lists = O.grav_workload(w, order=2)
    a_brute = O.grav_brute(rec[:, :3], rec[:, 3], 1.0, 0.01)
    np.testing.assert_allclose(a_lists, a_brute, rtol=1e-12, atol=1e-12 * np.abs(a_brute).max())


def test_newton_third_law_direct_sum():
    rec = W.plummer(2000, 12).astype(np.float64)
    acc = O.grav_brute(rec[:, :3], rec[:, 3], 1.0, 0.01)
    net = np.sum(rec[:, 3:4] * acc, axis=0)
    scale = np.sum(rec[:, 3] * np.linalg.norm(acc, axis=1))
    assert np.linalg.norm(net) <= 1e-13 * scale


def test_tree_lists_approximate_brute_force():
    # theta = 0.7 lists with quadrupoles stay close to the exact sum (BH error scale ~1e-3)
    w = W.build_grav(W.plummer(3000, 13), bucket=16, theta=0.7)
    rec = w.rec.astype(np.float64)
    a_q = O.grav_workload(w, order=2)
    a_m = O.grav_workload(w, order=1)
    a_b = O.grav_brute(rec[:, :3], rec[:, 3], 1.0, 0.01)
    eq = np.linalg.norm(a_q - a_b, axis=1) / np.linalg.norm(a_b, axis=1)
    em = np.linalg.norm(a_m - a_b, axis=1) / np.linalg.norm(a_b, axis=1)
    assert np.median(eq) < 2e-3 and np.median(eq) < np.median(em)


def test_node_table_matches_fp64_moments():
    w = W.nbody_plummer(n=20000, seed=14)
    rec = w.rec.astype(np.float64)
    mom = O.node_moments(w.node_range, rec[:, :3], rec[:, 3])
    nodes = w.nodes.astype(np.float64)
    np.testing.assert_allclose(nodes[:, 3], mom[:, 3], rtol=1e-6)
    side = w.node_side
    assert np.all(np.abs(nodes[:, :3] - mom[:, :3]).max(axis=1) <= 1e-6 * np.maximum(side, np.abs(mom[:, :3]).max(axis=1)))
    Sabs = np.abs(mom[:, 4:7]).sum(axis=1)
    assert np.all(np.abs(nodes[:, 4:10] - mom[:, 4:10]).max(axis=1) <= 1e-6 * Sabs + 1e-30)
    np.testing.assert_allclose(nodes[:, 10], mom[:, 4] + mom[:, 5] + mom[:, 6], rtol=1e-6, atol=1e-30)


def test_energy_conservation_and_reversibility_leapfrog():
    # KDK leapfrog with the checker's direct-sum forces conserves E = K + W to O(dt^2) and is
    # time reversible; a sign or factor error in the force breaks both
    n = 256
    rec = W.plummer(n, 15).astype(np.float64)
    x = rec[:, :3].copy()
    m = rec[:, 3].copy()
    rng = np.random.default_rng(15)
    v = rng.normal(size=(n, 3)) * math.sqrt(1.0 / 6.0)
    v -= np.sum(m[:, None] * v, axis=0) / m.sum()
    eps, dt, steps = 0.05, 2.0**-9, 200

    def energy(x, v):
        _, pot = O.grav_brute(x, m, 1.0, eps, potential=True)
        return 0.5 * np.sum(m[:, None] * v * v) + 0.5 * np.sum(m * pot)

    def run(x, v, k):
        a = O.grav_brute(x, m, 1.0, eps)
        for _ in range(k):
            v = v + 0.5 * dt * a
            x = x + dt * v
            a = O.grav_brute(x, m, 1.0, eps)
            v = v + 0.5 * dt * a
        return x, v

    E0 = energy(x, v)
    x1, v1 = run(x, v, steps)
    E1 = energy(x1, v1)
    assert abs(E1 - E0) <= 1e-5 * abs(E0)
    x2, v2 = run(x1, -v1, steps)
    assert np.abs(x2 - x).max() <= 1e-9


# ---------------------------------------------------------------- potential of the list terms

def _one_target(x, mom, order, G, eps):
    """(acc, pot) at point x of one node term through the list sum."""
    t = dict(i_begin=np.array([0]), i_count=np.array([1]), n_first=np.array([0]), n_count=np.array([1]),
             j_first=np.array([0]), j_nr=np.array([0]), node_idx=np.array([0]), ranges=np.zeros((0, 2), np.int32))
    acc, pot = O.grav_lists(t, np.array([x], float), np.array([1.0]), np.array([mom], float), order, G, eps,
                            potential=True)
    return acc[0], pot[0]


def test_two_body_potential_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(10):
        r, eps, G = 10 ** rng.uniform(-2, 1), 10 ** rng.uniform(-3, 0), rng.uniform(0.5, 2.0)
        m = rng.uniform(0.1, 3.0, size=2)
        pos = np.array([[0.0, 0.0, 0.0], [0.0, r, 0.0]])
        _, pot = O.grav_brute(pos, m, G, eps, potential=True)
        want = -G / math.sqrt(r * r + eps * eps)
        np.testing.assert_allclose(pot, want * m[::-1], rtol=1e-14)
        # the list sum with each body's direct range covering both ids (the self term is skipped)
        t = dict(i_begin=np.array([0, 1]), i_count=np.array([1, 1]), n_first=np.array([0, 0]),
                 n_count=np.array([0, 0]), j_first=np.array([0, 1]), j_nr=np.array([1, 1]),
                 node_idx=np.zeros(0, np.int32), ranges=np.array([[0, 2], [0, 2]]))
        _, lp = O.grav_lists(t, pos, m, np.zeros((1, 10)), 1, G, eps, potential=True)
        np.testing.assert_allclose(lp, want * m[::-1], rtol=1e-14)


@pytest.mark.parametrize("G,m,s", [(1.0, 1.0, 0.5), (2.5, 0.3, 0.1)])
def test_quadrupole_potential_axial_closed_form(G, m, s):
    # eps = 0, masses m at +-s z-hat: on the z axis Phi = -2Gm/z - 2Gm s^2/z^3, on the x axis
    # Phi = -2Gm/x + Gm s^2/x^3 (exact to second order); the monopole keeps -2Gm/r only
    mom = np.array([0, 0, 0, 2 * m, 0, 0, 2 * m * s * s, 0, 0, 0], float)
    for z in [3.0, 7.0, 20.0]:
        _, p = _one_target([0, 0, z], mom, 2, G, 0.0)
        np.testing.assert_allclose(p, -2 * G * m / z - 2 * G * m * s * s / z**3, rtol=1e-14)
        _, p = _one_target([z, 0, 0], mom, 2, G, 0.0)
        np.testing.assert_allclose(p, -2 * G * m / z + G * m * s * s / z**3, rtol=1e-14)
        _, p = _one_target([z, 0, 0], mom, 1, G, 0.0)
        np.testing.assert_allclose(p, -2 * G * m / z, rtol=1e-14)


def test_list_potential_at_theta_zero_equals_brute_force():
    w = W.build_grav(W.plummer(1500, 91), bucket=16, theta=0.0)
    assert w.node_idx.size == 0
    rec = w.rec.astype(np.float64)
    _, pot = O.grav_lists(O.workload_tasks(w), rec[:, :3], rec[:, 3], O.moments_from_nodes32(w.nodes), 2,
                          potential=True)
    _, want = O.grav_brute(rec[:, :3], rec[:, 3], potential=True)
    np.testing.assert_allclose(pot, want, rtol=1e-13)


@pytest.mark.parametrize("order", [1, 2])
def test_list_force_is_minus_gradient_of_list_potential(order):
    # lists and node moments frozen: a_i = -grad_i phi_i by central differences (a sign or factor
    # slip in either the quadrupole potential or its force would fail this)
    w = W.build_grav(W.plummer(4096, 92), bucket=16, theta=0.7)
    rec = w.rec.astype(np.float64)
    pos, mass, mom = rec[:, :3].copy(), rec[:, 3], O.moments_from_nodes32(w.nodes)
    tasks = O.workload_tasks(w)
    acc = O.grav_lists(tasks, pos, mass, mom, order)
    rng = np.random.default_rng(5)
    h = 1e-5
    for i in rng.choice(w.n, 12, replace=False):
        g = np.zeros(3)
        for d in range(3):
            pp = pos.copy(); pp[i, d] += h
            pm = pos.copy(); pm[i, d] -= h
            g[d] = (O.grav_lists(tasks, pp, mass, mom, order, potential=True)[1][i] -
                    O.grav_lists(tasks, pm, mass, mom, order, potential=True)[1][i]) / (2 * h)
        np.testing.assert_allclose(-g, acc[i], rtol=2e-6, atol=1e-8 * np.linalg.norm(acc[i]))
