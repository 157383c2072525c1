"""GPU parity of the combined Ewald kernel against the FP64 oracle (Sec. 4.1 periodic gravity).

Bar: per-task relative L2 <= 1e-5 of the correction.  The box's mass, centre of mass and second
moment are passed to both sides as the same FP32 values.
"""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from gpu_helpers import GravRig, rel_l2_per_task, whole

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


def box_moments(w):
    m = w.rec[:, 3].astype(np.float64)
    M = np.float32(m.sum())
    com = (w.rec[:, :3].astype(np.float64) * m[:, None]).sum(0) / m.sum()
    return float(M), com.astype(np.float32)


# an anisotropic second moment (xx yy zz xy xz yz) of a box of mass ~1, as a clustered box has; the
# uniform box's own is nearly isotropic and adds almost no force
S_ANISO = np.array([0.021, 0.008, 0.013, 0.004, -0.006, 0.0025], dtype=np.float32)


@pytest.mark.parametrize("mode", [gc.REORG_NONE, gc.REORG_PACK])
@pytest.mark.parametrize("alpha,nrep,hmax2", [(0.0, 1, 10), (2.6, 2, 20), (3.0, 0, 4), (2.0, 4, 64)])
@pytest.mark.parametrize("second_moment", [False, True])
def test_ewald_matches_oracle(ctx, mode, alpha, nrep, hmax2, second_moment):
    print(f"[gpu] ewald uniform-4096 mode {mode} alpha {alpha} nrep {nrep} hmax2 {hmax2} S {second_moment}",
          flush=True)
    w = W.nbody_tiny()
    M, com = box_moments(w)
    S = S_ANISO if second_moment else None
    rig = GravRig(ctx, w)
    b = rig.batch(whole(w))
    b.reorganize(rig.pool, mode)
    rig.acc.zero_()
    b.ewald(gc.ewald_params(1.0, M, com, alpha=alpha, nrep=nrep, hmax2=hmax2, S=S), rig.acc)
    rig.torch.cuda.synchronize()
    acc = rig.acc.cpu().numpy()
    ref = O.ewald(w.rec[:, :3], 1.0, 1.0, M, com.astype(np.float64), alpha if alpha > 0 else 2.0, nrep, hmax2,
                  S=None if S is None else S.astype(np.float64))
    if second_moment:  # the terms must matter at this bar, or the test shows nothing
        mono = O.ewald(w.rec[:, :3], 1.0, 1.0, M, com.astype(np.float64), alpha if alpha > 0 else 2.0, nrep, hmax2)
        assert rel_l2_per_task(mono, ref, whole(w)).min() > 100 * TOL
    err = rel_l2_per_task(acc, ref, whole(w))
    assert err.max() <= TOL, err.max()
    b.destroy()
    rig.close()


@pytest.mark.parametrize("second_moment", [False, True])
def test_ewald_adds_and_handles_a_target_at_the_centre(ctx, second_moment):
    # acc += correction; a target sitting exactly at com takes the series branch (zero correction)
    w = W.nbody_tiny()
    M, _ = box_moments(w)
    com = w.rec[7, :3].copy()  # any point may be the expansion centre
    S = S_ANISO if second_moment else None
    rig = GravRig(ctx, w)
    b = rig.batch(whole(w))
    b.reorganize(rig.pool, gc.REORG_PACK)
    rig.acc.fill_(1.0)
    b.ewald(gc.ewald_params(1.0, M, com, S=S), rig.acc)
    rig.torch.cuda.synchronize()
    acc = rig.acc.cpu().numpy()
    ref = O.ewald(w.rec[:, :3], 1.0, 1.0, M, com.astype(np.float64), 2.0, 1, 10,
                  S=None if S is None else S.astype(np.float64))
    assert np.all(np.isfinite(acc))
    assert np.abs(acc[7, :3] - 1.0).max() <= 1e-6
    assert np.all(acc[:, 3] == 1.0)
    err = rel_l2_per_task(acc[:, :3] - 1.0, ref, whole(w))
    assert err.max() <= 1e-4, err.max()  # the +1 offset costs ~1e-7 absolute per component
    b.destroy()
    rig.close()


def test_ewald_rejects_bad_parameters(ctx):
    w = W.nbody_tiny()
    rig = GravRig(ctx, w)
    b = rig.batch(whole(w))
    b.reorganize(rig.pool, gc.REORG_NONE)
    for kw in (dict(L=0.0), dict(nrep=5), dict(hmax2=65), dict(alpha=-1.0), dict(S=[0, 0, float("nan"), 0, 0, 0]),
               dict(S=[float("inf"), 0, 0, 0, 0, 0])):
        args = dict(L=1.0, M=1.0, com=(0.5, 0.5, 0.5))
        args.update(kw)
        with pytest.raises(gc.GcError) as e:
            b.ewald(gc.ewald_params(**args), rig.acc)
        assert e.value.status == 1
    b.destroy()
    rig.close()


@pytest.mark.parametrize("mode", [gc.REORG_NONE, gc.REORG_PACK])
def test_ewald_full_size_uniform_262144_sampled(ctx, mode):
    # the workload the bench times (262,144 uniform targets, buckets of 32, nrep 1, |h|^2 <= 10, the box's
    # own second moment), checked on 4,096 sampled targets against the oracle
    print(f"[gpu] ewald uniform-262144 mode {mode} sampled", flush=True)
    w = W.build_grav(W.uniform_cube(262144, 1005), bucket=32, theta=0.7)
    m = w.rec[:, 3].astype(np.float64)
    com = ((w.rec[:, :3].astype(np.float64) * m[:, None]).sum(0) / m.sum()).astype(np.float32)
    d = w.rec[:, :3].astype(np.float64) - com.astype(np.float64)
    S2 = np.einsum("j,ja,jb->ab", m, d, d)
    S = np.array([S2[0, 0], S2[1, 1], S2[2, 2], S2[0, 1], S2[0, 2], S2[1, 2]], dtype=np.float32)
    M = float(np.float32(m.sum()))
    rig = GravRig(ctx, w)
    b = rig.batch(whole(w))
    b.reorganize(rig.pool, mode)
    rig.acc.zero_()
    b.ewald(gc.ewald_params(1.0, M, com, nrep=1, hmax2=10, S=S), rig.acc)
    rig.torch.cuda.synchronize()
    acc = rig.acc.cpu().numpy()[:, :3].astype(np.float64)
    ids = np.random.default_rng(77).choice(w.n, size=4096, replace=False)
    ref = O.ewald(w.rec[ids, :3], 1.0, 1.0, M, com.astype(np.float64), 2.0, 1, 10, S=S.astype(np.float64))
    err = np.linalg.norm(acc[ids] - ref) / np.linalg.norm(ref)
    assert err <= TOL, err
    assert np.abs(acc[ids] - ref).max() <= TOL * np.abs(ref).max()
    b.destroy()
    rig.close()
