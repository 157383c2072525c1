"""GPU forces inside a time integration: energy drift of a KDK leapfrog against the oracle's.

theta = 0 makes every bucket's list all leaves as direct ranges, so the tree built once at t = 0
stays exact while particles move; each step uploads the positions and runs the combined pass with
in-place reads (REORG_NONE).  The bar: the GPU-force run's relative energy drift stays within twice
the FP64 oracle run's plus 1e-6 (the oracle's drift is the integrator's own O(dt^2) error).
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
    import torch
    print("[gpu] leapfrog energy drift, Plummer 1024, theta 0", flush=True)
    n, eps, dt, steps = 1024, 0.05, 2.0**-9, 200
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

    def run(force):
        x, v = x0.copy(), v0.copy()
        a = force(x)
        for _ in range(steps):
            v = v + 0.5 * dt * a
            x = x + dt * v
            a = force(x)
            v = v + 0.5 * dt * a
        return x, v

    E0 = energy(x0, v0)
    xo, vo = run(lambda x: O.grav_brute(x, m, 1.0, eps))
    xg, vg = run(gpu_acc)
    drift_o = abs(energy(xo, vo) - E0) / abs(E0)
    drift_g = abs(energy(xg, vg) - E0) / abs(E0)
    print(f"[gpu] energy drift oracle {drift_o:.3e} gpu {drift_g:.3e}", flush=True)
    assert drift_g <= 2.0 * drift_o + 1e-6
    # the trajectories stay together (FP32 forces: differences grow from ~1e-7 per step)
    assert np.abs(xg - xo).max() <= 1e-3
    b.destroy()
    rig.close()
    ctx.close()
