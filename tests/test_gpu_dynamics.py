"""GPU forces inside a time integration: energy drift of a KDK leapfrog against the oracle's.

Gravity: theta = 0 makes every bucket's list all leaves as direct ranges, so the tree built once at
t = 0 stays exact while particles move; each step uploads the positions and runs the combined pass
with in-place reads (REORG_NONE).  Lennard-Jones: the cells and their pair tasks are rebuilt from
the positions at every step (one new batch per step), as a cell-list MD code does.  The bar: the
GPU-force run's relative energy drift stays within twice the FP64 oracle run's plus 1e-6 (the
oracle's drift is the integrator's own error, and for LJ also that of pairs crossing the cutoff of
the truncated force).
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from gpu_helpers import GravRig, grav_tasks, whole

pytestmark = pytest.mark.gpu


def test_leapfrog_energy_drift_with_gpu_forces():
    """Plummer 4,096 (masses 1/N), G = 1, eps = 0.01, dt = 2^-10, 512 steps.  The drift is the largest
    |E(t) - E(0)| / |E(0)| over checkpoints every 32 steps."""
    import torch
    print("[gpu] leapfrog energy drift, Plummer 4096, theta 0", flush=True)
    n, eps, dt, steps = 4096, 0.01, 2.0**-10, 512
    w = W.build_grav(W.plummer(n, 15), bucket=16, theta=0.0)
    m = w.rec[:, 3].astype(np.float64)
    x0 = w.rec[:, :3].astype(np.float64)
    rng = np.random.default_rng(15)
    v0 = rng.normal(size=(n, 3)) * math.sqrt(1.0 / 6.0)
    v0 -= np.sum(m[:, None] * v0, axis=0) / m.sum()

    def energy(x, v):
        _, pot = O.grav_brute(x, m, 1.0, eps, potential=True)
        return 0.5 * np.sum(m[:, None] * v * v) + 0.5 * np.sum(m * pot)

    ctx = gc.Context(0)
    rig = GravRig(ctx, w)
    b = rig.batch(whole(w))
    prm = gc.grav_params(order=1, G=1.0, eps=eps)
    b.reorganize(rig.pool, gc.REORG_NONE)

    def gpu_acc(x):
        rec = np.empty((n, 4), np.float32)
        rec[:, :3] = x
        rec[:, 3] = w.rec[:, 3]
        rig.src.copy_(torch.from_numpy(rec))
        b.launch(prm, rig.nodes, rig.acc)
        torch.cuda.synchronize()
        return rig.acc.cpu().numpy()[:, :3].astype(np.float64)

    def run(force, E0):
        x, v = x0.copy(), v0.copy()
        a = force(x)
        worst = 0.0
        for s in range(steps):
            v = v + 0.5 * dt * a
            x = x + dt * v
            a = force(x)
            v = v + 0.5 * dt * a
            if (s + 1) % 32 == 0:
                worst = max(worst, abs(energy(x, v) - E0))
        return x, worst / abs(E0)

    E0 = energy(x0, v0)
    xo, drift_o = run(lambda x: O.grav_brute(x, m, 1.0, eps), E0)
    xg, drift_g = run(gpu_acc, E0)
    print(f"[gpu] energy drift oracle {drift_o:.3e} gpu {drift_g:.3e}", flush=True)
    assert drift_g <= 2.0 * drift_o + 1e-6
    # the trajectories stay together (FP32 forces: differences grow from ~1e-7 per step)
    assert np.abs(xg - xo).max() <= 1e-4
    b.destroy()
    rig.close()
    ctx.close()


def test_lj_leapfrog_energy_drift_with_gpu_forces():
    """FCC 4,000 atoms at density 0.8442, T = 1, one type (eps = sigma = m = 1), r_c = 2.5,
    dt = 0.005, 1,000 steps; energy with the potential shifted to zero at r_c.  The drift is the
    largest |E(t) - E(0)| / |E(0)| over the run (the end value alone wanders with the chaotic
    trajectory; the largest excursion is set by the integrator and the cutoff crossings)."""
    import torch
    print("[gpu] LJ leapfrog energy drift, FCC 4000, cells rebuilt per step", flush=True)
    xyz, v0, L = W.fcc_modulated(10, 10, 10, 0.8442, 4000, seed=33, temperature=1.0)
    n = xyz.shape[0]
    prm_t = dict(eps_t=[1.0], sig_t=[1.0], mass_t=[1.0])
    rc, dt, steps = 2.5, 0.005, 1000
    u_rc = 4.0 * (rc**-12 - rc**-6)
    types = np.zeros(n, np.int32)
    Lf = W.build_lj(xyz, types, L, rc, **prm_t).L  # box lengths as the workload holds them

    def oracle_force(x):
        w = W.build_lj(x, types, Lf, rc, **prm_t)
        a, pot, nin = O.lj_tasks(w, potential=True)
        out = np.empty_like(a)
        out[w.perm] = a
        return out, pot.sum() - nin * u_rc

    ctx = gc.Context(0)
    src = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    acc = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    eps = torch.ones(1, dtype=torch.float32, device="cuda")
    sig = torch.ones(1, dtype=torch.float32, device="cuda")
    mass = torch.ones(1, dtype=torch.float32, device="cuda")
    pool = gc.Pool(ctx, n, n)
    pool.set_source(src)
    prm = gc.lj_params(eps, sig, mass, rc)

    def gpu_force(x):
        w = W.build_lj(x, types, Lf, rc, **prm_t)
        src.copy_(torch.from_numpy(np.ascontiguousarray(w.rec)))
        ranges = np.stack([w.j_begin, w.j_count], axis=1).astype(np.int32)
        t = gc.tasks_from_csr(w.i_begin, w.i_count, np.arange(w.n_tasks, dtype=np.int32),
                              np.ones(w.n_tasks, np.int32), flags=np.where(w.self_flag != 0, gc.TASK_SELF, 0),
                              shift=w.shift)
        b = gc.Batch(ctx, gc.KIND_LJ, n)
        b.submit(t, ranges)
        b.commit()
        b.reorganize(pool, gc.REORG_NONE)
        b.launch(prm, None, acc)
        torch.cuda.synchronize()
        a = acc.cpu().numpy()[:, :3].astype(np.float64)
        b.destroy()
        out = np.empty_like(a)
        out[w.perm] = a
        _, pot, nin = O.lj_tasks(w, potential=True)  # energy bookkeeping only; the run moves on GPU forces
        return out, pot.sum() - nin * u_rc

    def run(force, tag):
        x = W.wrap_box(xyz, Lf).astype(np.float64)
        v = v0.copy()
        a, U = force(x)
        E0 = 0.5 * np.sum(v * v) + U
        worst, x100 = 0.0, None
        for s in range(steps):
            v = v + 0.5 * dt * a
            x = np.mod(x + dt * v, Lf)
            a, U = force(x)
            v = v + 0.5 * dt * a
            worst = max(worst, abs(0.5 * np.sum(v * v) + U - E0))
            if s + 1 == 100:
                x100 = x.copy()
            if (s + 1) % 250 == 0:
                print(f"[gpu] {tag} step {s + 1}", flush=True)
        return E0, worst / abs(E0), x100

    E0o, drift_o, xo = run(oracle_force, "oracle")
    E0g, drift_g, xg = run(gpu_force, "gpu")
    print(f"[gpu] LJ energy drift oracle {drift_o:.3e} gpu {drift_g:.3e}", flush=True)
    assert abs(E0g - E0o) <= 1e-12 * abs(E0o)  # same start, same energy bookkeeping
    assert drift_g <= 2.0 * drift_o + 1e-6
    # after 100 steps the two runs still agree (they part later: the dynamics are chaotic)
    d = np.abs(((xg - xo + Lf / 2) % Lf) - Lf / 2).max()
    assert d <= 1e-3, d
    pool.destroy()
    ctx.close()
