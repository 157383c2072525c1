"""Pins for the checker's vector-Jacobian products: central finite differences in FP64."""
import numpy as np

import oracle as O
import workloads as W

H = 1e-6


def _grav_loss(w, g, pos, mass):
    mom = O.node_moments(w.node_range, pos, mass)
    a = O.grav_lists(O.workload_tasks(w), pos, mass, mom, order=1, G=1.0, eps=0.01)
    return float(np.sum(g * a))


def test_grav_vjp_matches_finite_differences():
    w = W.build_grav(W.plummer(512, 51), bucket=16, theta=0.7)
    assert w.n_count.sum() > 0  # nodes are exercised
    rng = np.random.default_rng(52)
    g = rng.normal(size=(w.n, 3))
    rec = w.rec.astype(np.float64)
    pos, mass = rec[:, :3].copy(), rec[:, 3].copy()
    mom = O.node_moments(w.node_range, pos, mass)
    gpos, gmass = O.vjp_grav_mono(w, g, pos=pos, mass=mass, mom=mom)
    for i in rng.choice(w.n, size=12, replace=False):
        for q in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, q] += H
            p2[i, q] -= H
            fd = (_grav_loss(w, g, p1, mass) - _grav_loss(w, g, p2, mass)) / (2 * H)
            assert abs(fd - gpos[i, q]) <= 1e-7 * max(1.0, abs(gpos).max()), (i, q, fd, gpos[i, q])
        m1, m2 = mass.copy(), mass.copy()
        m1[i] += H * mass[i]
        m2[i] -= H * mass[i]
        fd = (_grav_loss(w, g, pos, m1) - _grav_loss(w, g, pos, m2)) / (2 * H * mass[i])
        assert abs(fd - gmass[i]) <= 1e-6 * max(1.0, abs(gmass).max()), (i, fd, gmass[i])


def test_grav_vjp_directional_derivative():
    # <gpos, v> equals the directional derivative of L along v (all coordinates at once)
    w = W.build_grav(W.uniform_cube(400, 53), bucket=8, theta=0.6)
    rng = np.random.default_rng(54)
    g = rng.normal(size=(w.n, 3))
    v = rng.normal(size=(w.n, 3))
    rec = w.rec.astype(np.float64)
    pos, mass = rec[:, :3].copy(), rec[:, 3].copy()
    gpos, _ = O.vjp_grav_mono(w, g, pos=pos, mass=mass, mom=O.node_moments(w.node_range, pos, mass))
    h = 1e-7
    fd = (_grav_loss(w, g, pos + h * v, mass) - _grav_loss(w, g, pos - h * v, mass)) / (2 * h)
    np.testing.assert_allclose(np.sum(gpos * v), fd, rtol=1e-6)


def _lj_loss(w, g, pos, mass, e, s):
    return float(np.sum(g * O.lj_at(w, pos, mass, e, s)))


def test_lj_vjp_matches_finite_differences():
    w = W.lj_small()
    rng = np.random.default_rng(55)
    g = rng.normal(size=(w.n, 3))
    pos = w.rec[:, :3].astype(np.float64)
    mass = w.mass_t[w.rec[:, 3].astype(int)].astype(np.float64) * rng.uniform(0.8, 1.2, size=w.n)
    e, s = w.eps_t.astype(np.float64), w.sig_t.astype(np.float64)
    gpos, gmass, ge, gs = O.vjp_lj(w, g, pos=pos, mass=mass, eps_t=e, sig_t=s)
    scale = np.abs(gpos).max()
    for i in rng.choice(w.n, size=10, replace=False):
        for q in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, q] += H
            p2[i, q] -= H
            fd = (_lj_loss(w, g, p1, mass, e, s) - _lj_loss(w, g, p2, mass, e, s)) / (2 * H)
            assert abs(fd - gpos[i, q]) <= 1e-7 * scale, (i, q, fd, gpos[i, q])
        m1, m2 = mass.copy(), mass.copy()
        m1[i] += H
        m2[i] -= H
        fd = (_lj_loss(w, g, pos, m1, e, s) - _lj_loss(w, g, pos, m2, e, s)) / (2 * H)
        assert abs(fd - gmass[i]) <= 1e-7 * max(1.0, np.abs(gmass).max())
    for t in range(2):
        e1, e2 = e.copy(), e.copy()
        e1[t] += H
        e2[t] -= H
        fd = (_lj_loss(w, g, pos, mass, e1, s) - _lj_loss(w, g, pos, mass, e2, s)) / (2 * H)
        np.testing.assert_allclose(ge[t], fd, rtol=1e-7, atol=1e-9 * abs(ge).max())
        s1, s2 = s.copy(), s.copy()
        s1[t] += H
        s2[t] -= H
        fd = (_lj_loss(w, g, pos, mass, e, s1) - _lj_loss(w, g, pos, mass, e, s2)) / (2 * H)
        np.testing.assert_allclose(gs[t], fd, rtol=1e-7, atol=1e-9 * abs(gs).max())


def _grav_loss_q(w, g, pos, mass):
    mom = O.node_moments(w.node_range, pos, mass)
    a = O.grav_lists(O.workload_tasks(w), pos, mass, mom, order=2, G=1.0, eps=0.01)
    return float(np.sum(g * a))


def test_quadrupole_vjp_matches_finite_differences():
    # node moments (c, M, S) re-derived from the perturbed members: the node chain through S is tested
    w = W.build_grav(W.plummer(512, 56), bucket=16, theta=0.7)
    assert w.n_count.sum() > 0
    rng = np.random.default_rng(57)
    g = rng.normal(size=(w.n, 3))
    rec = w.rec.astype(np.float64)
    pos, mass = rec[:, :3].copy(), rec[:, 3].copy()
    gpos, gmass = O.vjp_grav(w, g, order=2, pos=pos, mass=mass, mom=O.node_moments(w.node_range, pos, mass))
    for i in rng.choice(w.n, size=12, replace=False):
        for q in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, q] += H
            p2[i, q] -= H
            fd = (_grav_loss_q(w, g, p1, mass) - _grav_loss_q(w, g, p2, mass)) / (2 * H)
            assert abs(fd - gpos[i, q]) <= 1e-7 * max(1.0, abs(gpos).max()), (i, q, fd, gpos[i, q])
        m1, m2 = mass.copy(), mass.copy()
        m1[i] += H * mass[i]
        m2[i] -= H * mass[i]
        fd = (_grav_loss_q(w, g, pos, m1) - _grav_loss_q(w, g, pos, m2)) / (2 * H * mass[i])
        assert abs(fd - gmass[i]) <= 1e-6 * max(1.0, abs(gmass).max()), (i, fd, gmass[i])


def test_quadrupole_vjp_directional_derivative_and_monopole_case():
    w = W.build_grav(W.uniform_cube(400, 58), bucket=8, theta=0.6)
    rng = np.random.default_rng(59)
    g = rng.normal(size=(w.n, 3))
    v = rng.normal(size=(w.n, 3))
    rec = w.rec.astype(np.float64)
    pos, mass = rec[:, :3].copy(), rec[:, 3].copy()
    mom = O.node_moments(w.node_range, pos, mass)
    gpos, _ = O.vjp_grav(w, g, order=2, pos=pos, mass=mass, mom=mom)
    h = 1e-7
    fd = (_grav_loss_q(w, g, pos + h * v, mass) - _grav_loss_q(w, g, pos - h * v, mass)) / (2 * h)
    np.testing.assert_allclose(np.sum(gpos * v), fd, rtol=1e-6)
    # order 1 is the monopole routine
    a1 = O.vjp_grav(w, g, order=1, pos=pos, mass=mass, mom=mom)
    b1 = O.vjp_grav_mono(w, g, pos=pos, mass=mass, mom=mom)
    assert np.array_equal(a1[0], b1[0]) and np.array_equal(a1[1], b1[1])
