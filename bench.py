"""Benchmark of the combined irregular-task force path on one MI355X.

Workload (the irregular N-body configuration with reuse): 262,144 particles from
a Plummer sphere (scale radius 1, cut at 10), FP32 records, octree buckets of
32, Barnes-Hut theta = 0.7 with monopole + quadrupole nodes, Plummer softening
0.01.  The 27k bucket tasks arrive in 32 rounds of Poisson(2048) consecutive
buckets (tree order, wrapping: about 2.4 passes over the buckets).  Half of all particles are resident at uniformly random pool slots
(the base residency); each round finds about half of its particle union
resident and the reorganisation stages the rest from the particle array in
HBM; the next round first evicts what this one staged, so the base holds.

One step = every round of one full force evaluation: eviction of the previous
round's staging + reorganisation (chare-table lookup, slot assignment,
staging, packing gather) + the combined force kernel, all captured in one HIP
graph (the batched form), replayed once per step.

Prints one JSON line on stdout; diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G-interactions/s combined force kernel (%FP32 peak); reorganize GB/s; bwd/fwd"
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector (packed); plain FMA issue gives half: 78.6
PEAK_FP32_NONPACKED_TFLOPS = 78.6
N_SIMD, CLOCK_GHZ = 256 * 4, 2.4   # MI355X: 256 CUs x 4 SIMDs at 2.4 GHz
LJ_VALU_PER_EVAL = 20.5            # Lennard-Jones gather loop: 41 VALU instructions per two pair evaluations
PEAK_HBM_GBPS = 8000.0
# launch shapes (tile, targets per lane) of the whole-step form that the bench may time; the GPU tests
# check every one of them against the per-round launches and the oracle
STEP_SHAPES = ((256, 1), (256, 2), (320, 1), (320, 2), (384, 1), (384, 2))
# launch shapes (tile, targets per lane, waves per task) of the rounds form's combined pass that the bench may
# time; the GPU tests check every one of them against the per-round launches and the oracle
TPL_TEXT = {0: "one target per lane", 1: "one target per lane", 2: "two targets per lane",
            3: "one or two targets per lane, whichever fills more lanes for the task"}
ROUNDS_SHAPES = ((256, 1, 2), (256, 2, 2), (256, 3, 2), (256, 3, 1), (256, 2, 4), (512, 2, 2))


def flop_counts() -> dict:
    """Algorithmic flop per interaction, read from the library's header (one place for the counts)."""
    import re
    txt = open(os.path.join(ROOT, "paper_2008_05712_amd", "csrc", "gc_internal.h")).read()
    return {k: int(v) for k, v in re.findall(r"constexpr int (kFlops\w+) = (\d+);", txt)}


_FLOPS = flop_counts()
FLOPS_PAIR, FLOPS_QUAD, FLOPS_LJ = _FLOPS["kFlopsPair"], _FLOPS["kFlopsQuad"], _FLOPS["kFlopsLJ"]
# algorithmic bytes of one reorganisation: per union entry the id, its slot_of entry, its slot out,
# the record read and the packed write; per missing record the pool write, the slot_of and occupancy
# updates and the missing list (id and slot); per pool slot the occupancy read of the free-slot scan
REORG_BYTES_PER_UNION = 4 + 4 + 4 + 16 + 16
REORG_BYTES_PER_MISSING = 16 + 4 + 4 + 4 + 4
REORG_BYTES_PER_SLOT = 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profiled_traffic(profile: str, shape: dict):
    """HBM bytes per launch of the profiled kernel from a committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (profiles/<profile>.json: one entry per profiled launch shape), or None when any of its
    source files differs from the profiled one or no entry has this launch shape."""
    import hashlib
    side = os.path.join(ROOT, "profiles", profile + ".json")
    try:
        meta = json.load(open(side))
        for rel, digest in meta["sources"].items():
            if hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest() != digest:
                return None
        for ent in meta["entries"]:
            if ent["shape"] == shape:
                return int(ent["traffic_bytes_per_launch"])
    except (OSError, ValueError, KeyError, AttributeError, TypeError):
        return None
    return None


def time_kernel(fn, stream, reps: int = 10) -> float:
    """Average ms of fn() (device work on `stream`) over reps launches, HIP events on that stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def leg_instances(gc, W, torch, ctx, args):
    """64 independent Plummer instances (sizes log-uniform in 2,048..262,144) in one id space.  Against
    each other: the plain per-instance form (one combined launch per instance, in order on one stream,
    default shape), a HIP graph of per-instance launches (tuned shape; launches overlap on the graph's
    side streams), and every task of all instances in one batch: one launch with the autotuner's
    shape (its aggregation count tuned too), captured in a graph.  Then the whole batch's
    reorganisation (PACK) with half of all ids resident at random slots: the aggregated reorganise."""
    t0 = time.time()
    w = W.nbody_instances(k=64, seed=4000)
    inst = w.meta["instance_of_task"]
    log(f"[bench] instances: N={w.n} tasks={w.n_tasks} build {time.time() - t0:.1f}s")
    n_direct, n_node = w.split_interactions()
    inter = n_direct + n_node
    flops = n_direct * FLOPS_PAIR + n_node * FLOPS_QUAD
    dev = torch.device("cuda")
    src = torch.from_numpy(w.rec).to(dev)
    nodes = torch.from_numpy(w.nodes).to(dev)
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, 1)
    pool.set_source(src)
    stream = torch.cuda.current_stream()
    res = {"workload": f"nbody-plummer-x64 (N={w.n}, {w.n_tasks} tasks, {inter} interactions)"}

    def batch_of(sel, mode=gc.REORG_NONE, p=pool):
        bt = W.task_subset(w, sel)
        b = gc.Batch(ctx, gc.KIND_GRAV, w.n)
        b.submit(gc.tasks_from_csr(bt["i_begin"], bt["i_count"], bt["j_first"], bt["j_nr"], bt["n_first"],
                                   bt["n_count"]), bt["ranges"], bt["node_idx"])
        b.commit()
        b.reorganize(p, mode)
        return b

    # one batch over every instance; the autotuner picks the shape, then the aggregation count
    allb = batch_of(np.arange(w.n_tasks))
    best, times, _ = allb.autotune(gc.grav_params(order=2), nodes, acc, reps=2)
    shape = dict(tile=best.tile, waves_per_block=best.waves_per_block, schedule=best.schedule,
                 targets_per_lane=best.targets_per_lane)
    one = gc.grav_params(order=2, aggregation=0, **shape)
    res["autotuned"] = dict(shape, aggregation=best.aggregation, one_launch_ms=round(float(times[36]), 4),
                            aggregation_ms=[round(float(x), 4) for x in times[36:]])
    # the plain per-instance form
    per = [batch_of(np.nonzero(inst == k)[0]) for k in range(64)]
    prm0 = gc.grav_params(order=2)

    def run_plain():
        for b in per:
            b.launch(prm0, nodes, acc)
    plain = time_kernel(run_plain, stream, reps=3)
    # a graph of per-instance launches with the tuned shape
    side = torch.cuda.Stream()
    g = gc.Graph(ctx, per, [pool] * 64, [gc.REORG_NONE] * 64, gc.grav_params(order=2, **shape), nodes, acc,
                 stream=side)
    torch.cuda.synchronize()
    per_graph = time_kernel(lambda: g.launch(stream=stream), stream, reps=5)
    g.destroy()
    for b in per:
        b.destroy()
    # the whole batch in one launch, captured
    g1 = gc.Graph(ctx, [allb], [pool], [gc.REORG_NONE], one, nodes, acc, stream=side)
    torch.cuda.synchronize()
    one_ms = time_kernel(lambda: g1.launch(stream=stream), stream, reps=5)
    g1.destroy()
    forms = {"plain_per_instance_ms": round(plain, 4), "per_instance_graph_ms": round(per_graph, 4),
             "one_launch_graph_ms": round(one_ms, 4)}
    best_form = min(forms, key=forms.get)
    res.update({"forms": forms, "best_form": best_form,
                "one_launch_vs_plain_per_instance": round(plain / one_ms, 3),
                "one_launch_vs_per_instance_graph": round(per_graph / one_ms, 3),
                "one_launch_ginteractions_per_s": round(inter / (one_ms * 1e-3) / 1e9, 3)})
    bt = flops / (one_ms * 1e-3) / 1e12
    res["roofline"] = {"bound": "alu", "achieved": round(bt, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(bt / PEAK_FP32_TFLOPS, 4), "flops_per_launch": int(flops),
                       "avg_launch_ms": round(one_ms, 5),
                       "kernel": f"k_grav<2> over all {w.n_tasks} tasks (tile {best.tile}, {best.waves_per_block} "
                                 f"waves, schedule {best.schedule}, {best.targets_per_lane} targets per lane)",
                       "frac_of_nonpacked_peak": round(bt / PEAK_FP32_NONPACKED_TFLOPS, 4)}
    allb.destroy()
    pool.destroy()
    # the aggregated reorganisation: PACK of the whole batch's union, half of all ids resident at random
    # slots of a pool of capacity N (each call stages the other half, after evicting the last call's)
    pool2 = gc.Pool(ctx, w.n, w.n)
    pool2.set_source(src)
    bids, bslots = W.residency(np.arange(w.n, dtype=np.int32), w.n, 0.5, seed=4999)
    pool2.place(torch.from_numpy(bids).to(dev), torch.from_numpy(bslots).to(dev))
    rb = batch_of(np.arange(w.n_tasks), gc.REORG_PACK, pool2)
    torch.cuda.synchronize()
    nu, nm = int(rb.maps()["U"].size), int(rb.maps()["missing"].size)
    ms = 0.0
    for _ in range(5):
        pool2.evict_staged(rb)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rb.reorganize(pool2, gc.REORG_PACK, check_capacity=False)
        e1.record(stream)
        e1.synchronize()
        ms += e0.elapsed_time(e1) / 5
    rb.status()
    alg = nu * (16 + 16 + 4 + 4) + nm * 16
    gbps = alg / (ms * 1e-3) / 1e9
    res["aggregated_reorganize"] = {"union": nu, "missing": nm, "ms": round(ms, 4), "algorithmic_bytes": int(alg),
                                    "gbps": round(gbps, 1), "frac_hbm": round(gbps / PEAK_HBM_GBPS, 4)}
    rb.destroy()
    pool2.destroy()
    return res


def lj_kept_evaluations(w) -> int:
    """Pair evaluations of the gather form after its candidate pruning, counted on the host with the
    kernel's rule: per target cell, the sources (the other cell of each of its tasks, in the cell's
    frame: x_j + shift on the i side, x_i - shift on the j side) within r_c of the bounding box of the
    cell's atoms (squared distance at most 1.001 r_c^2), times the cell's atom count; a self task
    evaluates all its atoms.  Padding slots of the tiles are not counted."""
    pos = w.rec[:, :3].astype(np.float64)
    ic = w.i_count.astype(np.int64)
    jc = w.j_count.astype(np.int64)
    selfm = w.self_flag != 0
    # each cell's bounding box, from its self task's range
    cb, cn = w.i_begin[selfm].astype(np.int64), ic[selfm]
    starts = np.zeros(w.n, np.int64) - 1
    starts[cb] = np.arange(cb.size)
    cell_of = np.maximum.accumulate(starts)  # cells are contiguous id ranges in id order
    lo = np.full((cb.size, 3), np.inf)
    hi = np.full((cb.size, 3), -np.inf)
    np.minimum.at(lo, cell_of, pos)
    np.maximum.at(hi, cell_of, pos)
    rc2 = float(w.rcut) ** 2 * 1.001
    total = int(np.sum(ic[selfm] * ic[selfm]))
    cross = np.nonzero(~selfm)[0]
    sh = w.shift.astype(np.float64)
    for side in (0, 1):  # 0: the i cell is the target, sources from j; 1: the reverse
        tb = (w.i_begin if side == 0 else w.j_begin)[cross].astype(np.int64)
        tn = (ic if side == 0 else jc)[cross]
        sb = (w.j_begin if side == 0 else w.i_begin)[cross].astype(np.int64)
        sn = (jc if side == 0 else ic)[cross]
        sgn = 1.0 if side == 0 else -1.0
        for c0 in range(0, cross.size, 200000):
            sl = slice(c0, c0 + 200000)
            n = sn[sl]
            task = np.repeat(np.arange(n.size), n)
            first = np.repeat(np.cumsum(n) - n, n)
            atom = np.repeat(sb[sl], n) + (np.arange(task.size) - first)
            p = pos[atom] + sgn * sh[cross[sl]][task]
            cell = cell_of[tb[sl]][task]
            d = np.maximum(np.maximum(lo[cell] - p, p - hi[cell]), 0.0)
            kept = np.bincount(task, weights=((d * d).sum(1) <= rc2).astype(np.float64), minlength=n.size)
            total += int(np.sum(kept.astype(np.int64) * tn[sl]))
    return total


def leg_lj(gc, W, torch, ctx):
    """1,048,576 LJ atoms (FCC, half-box thinned), one combined cell-pair launch per step."""
    t0 = time.time()
    w = W.lj_fcc()
    log(f"[bench] lj: N={w.n} tasks={w.n_tasks} build {time.time() - t0:.1f}s")
    dev = torch.device("cuda")
    src = torch.from_numpy(w.rec).to(dev)
    eps, sig, mass = (torch.from_numpy(x).to(dev) for x in (w.eps_t, w.sig_t, w.mass_t))
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, 1)
    pool.set_source(src)
    ranges = np.stack([w.j_begin, w.j_count], axis=1).astype(np.int32)
    t = gc.tasks_from_csr(w.i_begin, w.i_count, np.arange(w.n_tasks, dtype=np.int32), np.ones(w.n_tasks, np.int32),
                          flags=np.where(w.self_flag != 0, gc.TASK_SELF, 0), shift=w.shift)
    b = gc.Batch(ctx, gc.KIND_LJ, w.n)
    b.submit(t, ranges)
    b.commit()
    b.reorganize(pool, gc.REORG_NONE)
    stream = torch.cuda.current_stream()
    out = {"workload": f"lj-fcc-{w.n} (rc 2.5, {w.n_tasks} cell-pair tasks)"}
    for sched in (0, 1):
        prm = gc.lj_params(eps, sig, mass, w.rcut, schedule=sched)
        ms = time_kernel(lambda: b.launch(prm, None, acc), stream)
        out[f"ms_sched{sched}"] = round(ms, 4)
    ms = min(out["ms_sched0"], out["ms_sched1"])
    # in-cutoff pair count from one oracle-free pass: candidates from the task sizes; pairs estimated
    # from the density (reported exactly by the parity tests' oracle runs)
    cand = w.candidates()
    out.update({"candidates": cand, "candidates_per_s_G": round(cand / (ms * 1e-3) / 1e9, 3), "ms": ms})
    # the gather form evaluates a pair of two different cells from both sides and a cell's self task
    # over all its atoms (the atom itself gives a zero separation), less what its pruning leaves out:
    # pair evaluations per launch, and the VALU issue they take at LJ_VALU_PER_EVAL wavefront-lane
    # slots each (the one-type loop) as a fraction of the chip's issue rate, 4 cycles per wavefront
    # instruction per SIMD
    ic = w.i_count.astype(np.int64)
    jc = w.j_count.astype(np.int64)
    unpruned = int(np.sum(np.where(w.self_flag != 0, ic * ic, 2 * ic * jc)))
    evals = lj_kept_evaluations(w)
    issue_ms = evals * LJ_VALU_PER_EVAL / 64 * 4 / (N_SIMD * CLOCK_GHZ * 1e9) * 1e3
    out.update({"pair_evaluations": evals, "pair_evaluations_unpruned": unpruned,
                "valu_issue_ms": round(issue_ms, 4), "valu_issue_frac": round(issue_ms / ms, 4)})
    # the algorithmic work: pairs inside the cutoff (counted on the device with the pass's FP32
    # decision), FLOPS_LJ flop each with both atoms updated
    pairs = b.lj_count_pairs(w.rcut)
    lj_tflops = pairs * FLOPS_LJ / (ms * 1e-3) / 1e12
    out.update({"in_cutoff_pairs": pairs, "pairs_per_s_G": round(pairs / (ms * 1e-3) / 1e9, 3),
                "evaluations_per_in_cutoff_pair": round(evals / pairs, 3),
                "candidates_per_in_cutoff_pair": round(cand / pairs, 3),
                "algorithmic_tflops": round(lj_tflops, 3), "algorithmic_frac": round(lj_tflops / PEAK_FP32_TFLOPS, 4)})
    b.destroy()
    pool.destroy()
    return out


def leg_ewald(gc, W, torch, ctx):
    """Ewald correction (periodic gravity) of 262,144 particles uniform in the unit box, buckets of 32:
    one combined launch over every target, 27 real-space images and the 73 wave-vector pairs with
    |h|^2 <= 10 at alpha = 2 / L; the box expanded to its second moment about the centre of mass
    (`ms`), and the monopole alone (`ms_monopole`)."""
    t0 = time.time()
    w = W.build_grav(W.uniform_cube(262144, 1005), bucket=32, theta=0.7)
    log(f"[bench] ewald: N={w.n} tasks={w.n_tasks} build {time.time() - t0:.1f}s")
    dev = torch.device("cuda")
    src = torch.from_numpy(w.rec).to(dev)
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, 1)
    pool.set_source(src)
    b = gc.Batch(ctx, gc.KIND_GRAV, w.n)
    b.submit(gc.tasks_from_csr(w.i_begin, w.i_count, w.j_first, w.j_nr, w.n_first, w.n_count), w.ranges, w.node_idx)
    b.commit()
    b.reorganize(pool, gc.REORG_NONE)
    m = w.rec[:, 3].astype(np.float64)
    com = (w.rec[:, :3].astype(np.float64) * m[:, None]).sum(0) / m.sum()
    d = w.rec[:, :3].astype(np.float64) - com
    S2 = np.einsum("j,ja,jb->ab", m, d, d)
    S = [S2[0, 0], S2[1, 1], S2[2, 2], S2[0, 1], S2[0, 2], S2[1, 2]]
    stream = torch.cuda.current_stream()
    prm0 = gc.ewald_params(1.0, float(m.sum()), com, nrep=1, hmax2=10)
    ms0 = time_kernel(lambda: b.ewald(prm0, acc), stream)
    prm = gc.ewald_params(1.0, float(m.sum()), com, nrep=1, hmax2=10, S=S)
    ms = time_kernel(lambda: b.ewald(prm, acc), stream)
    b.destroy()
    pool.destroy()
    return {"workload": f"uniform-{w.n} periodic unit box ({w.n_tasks} bucket tasks), nrep 1, |h|^2 <= 10, "
                        "box monopole and second moment",
            "ms": round(ms, 4), "targets_per_s_G": round(w.n / (ms * 1e-3) / 1e9, 3), "ms_monopole": round(ms0, 4)}


def leg_walk(gc, W, torch, ctx, w):
    """Device Barnes-Hut list walk of every bucket of the step's workload (gc_tree_walk: count pass,
    scan, fill; outputs already sized), wall time of the call, which waits for its own results."""
    dev = torch.device("cuda")
    args = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in
            (w.node_range.astype(np.int32), w.node_mom64[:, :3], w.node_side, w.rec, w.meta["leaf"].astype(np.int32))]
    nf, nidx, rf, rng = gc.tree_walk(ctx, *args, w.theta)  # sizes the outputs
    nb = int(args[4].numel())
    totals = (ctypes.c_int64 * 2)()
    call = lambda: ctx.check(gc.lib().gc_tree_walk(
        ctx.h, int(args[0].shape[0]), args[0].data_ptr(), args[1].data_ptr(), args[2].data_ptr(), args[3].data_ptr(),
        int(args[3].shape[0]), nb, args[4].data_ptr(), float(w.theta), nf.data_ptr(), rf.data_ptr(), nidx.data_ptr(),
        int(nidx.numel()), rng.data_ptr(), int(rng.shape[0]), totals, torch.cuda.current_stream().cuda_stream),
        "gc_tree_walk")
    for _ in range(3):
        call()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    ms = (time.perf_counter() - t0) / reps * 1e3
    return {"workload": f"nbody-plummer-{w.n}: {nb} buckets, theta {w.theta}", "ms": round(ms, 4),
            "node_entries": int(totals[0]), "direct_ranges": int(totals[1]),
            "buckets_per_s_M": round(nb / (ms * 1e-3) / 1e6, 3)}


def leg_adjoint(gc, W, torch, ctx):
    """Backward / forward time: gravity on the 4,096-particle uniform set (monopole) and on the
    262,144-particle Plummer set (quadrupole), and the two-type LJ adjoint at 1,048,576 atoms."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    res = {}
    w = W.nbody_tiny()
    src = torch.from_numpy(w.rec).to(dev)
    nodes = torch.from_numpy(w.nodes).to(dev)
    nr = torch.from_numpy(np.ascontiguousarray(w.node_range)).to(dev)
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, 1)
    pool.set_source(src)
    b = gc.Batch(ctx, gc.KIND_GRAV, w.n)
    b.submit(gc.tasks_from_csr(w.i_begin, w.i_count, w.j_first, w.j_nr, w.n_first, w.n_count), w.ranges, w.node_idx)
    b.commit()
    b.reorganize(pool, gc.REORG_NONE)
    prm = gc.grav_params(order=1)
    cot = torch.randn((w.n, 4), device=dev)
    gpos = torch.zeros((w.n, 4), device=dev)
    gmass = torch.zeros(w.n, device=dev)
    fwd = time_kernel(lambda: b.launch(prm, nodes, acc), stream)
    bwd = time_kernel(lambda: b.backward(prm, nodes, nr, w.nodes.shape[0], cot, gpos, gmass), stream)
    res["gravity_uniform_4096"] = {"fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4), "bwd_fwd": round(bwd / fwd, 3)}
    b.destroy()
    pool.destroy()
    # the quadrupole adjoint over all 27,026 tasks of the Plummer 262,144 workload (one launch each way)
    w = W.nbody_plummer()
    src = torch.from_numpy(w.rec).to(dev)
    nodes = torch.from_numpy(w.nodes).to(dev)
    nr = torch.from_numpy(np.ascontiguousarray(w.node_range)).to(dev)
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, 1)
    pool.set_source(src)
    b = gc.Batch(ctx, gc.KIND_GRAV, w.n)
    b.submit(gc.tasks_from_csr(w.i_begin, w.i_count, w.j_first, w.j_nr, w.n_first, w.n_count), w.ranges, w.node_idx)
    b.commit()
    b.reorganize(pool, gc.REORG_NONE)
    prm = gc.grav_params(order=2)
    cot = torch.randn((w.n, 4), device=dev)
    gpos = torch.zeros((w.n, 4), device=dev)
    gmass = torch.zeros(w.n, device=dev)
    fwd = time_kernel(lambda: b.launch(prm, nodes, acc), stream)
    bwd = time_kernel(lambda: b.backward(prm, nodes, nr, w.nodes.shape[0], cot, gpos, gmass), stream, reps=3)
    res["gravity_quadrupole_plummer_262144"] = {"fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4),
                                                "bwd_fwd": round(bwd / fwd, 3)}
    b.destroy()
    pool.destroy()
    w = W.lj_fcc(two_type=True)
    src = torch.from_numpy(w.rec).to(dev)
    eps, sig, mass = (torch.from_numpy(x).to(dev) for x in (w.eps_t, w.sig_t, w.mass_t))
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, 1)
    pool.set_source(src)
    ranges = np.stack([w.j_begin, w.j_count], axis=1).astype(np.int32)
    t = gc.tasks_from_csr(w.i_begin, w.i_count, np.arange(w.n_tasks, dtype=np.int32), np.ones(w.n_tasks, np.int32),
                          flags=np.where(w.self_flag != 0, gc.TASK_SELF, 0), shift=w.shift)
    b = gc.Batch(ctx, gc.KIND_LJ, w.n)
    b.submit(t, ranges)
    b.commit()
    b.reorganize(pool, gc.REORG_NONE)
    prm = gc.lj_params(eps, sig, mass, w.rcut)
    cot = torch.randn((w.n, 4), device=dev)
    gpos = torch.zeros((w.n, 4), device=dev)
    gmass = torch.zeros(w.n, device=dev)
    gpar = torch.zeros(2 * w.eps_t.size, device=dev)
    fwd = time_kernel(lambda: b.launch(prm, None, acc), stream)
    bwd = time_kernel(lambda: b.backward(prm, None, None, 0, cot, gpos, gmass, gpar), stream)
    res["lj_two_type_1048576"] = {"fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4), "bwd_fwd": round(bwd / fwd, 3)}
    res["bwd_fwd"] = res["lj_two_type_1048576"]["bwd_fwd"]
    b.destroy()
    pool.destroy()
    return res


def leg_reorg_stress(gc, torch, ctx, log2_pool: int = 26, log2_union: int = 24, reps: int = 5):
    """The reorganisation at HBM scale: a pool and id space of 2^26 records (1 GiB each for the pool and
    the source), a request whose union is 2^24 ids (2^18 runs of 64 consecutive ids at uniformly random
    run positions), half of it resident at uniformly random slots; each call stages the other half and
    packs all 2^24 records (PACK), after the previous call's staging is evicted."""
    n = 1 << log2_pool
    nu = 1 << log2_union
    run = 64
    rng = np.random.default_rng(6000)
    starts = np.sort(rng.choice(n // run, size=nu // run, replace=False)).astype(np.int64) * run
    ic = np.full(starts.size, run, np.int32)
    z = np.zeros(starts.size, np.int32)
    t = gc.tasks_from_csr(starts.astype(np.int32), ic, z, z)
    union = (starts[:, None] + np.arange(run)[None, :]).reshape(-1)
    res_ids = np.sort(rng.choice(union, size=nu // 2, replace=False)).astype(np.int32)
    res_slots = rng.choice(n, size=nu // 2, replace=False).astype(np.int32)
    dev = torch.device("cuda")
    src = torch.rand((n, 4), device=dev)
    pool = gc.Pool(ctx, n, n)
    pool.set_source(src)
    pool.place(torch.from_numpy(res_ids).to(dev), torch.from_numpy(res_slots).to(dev))
    b = gc.Batch(ctx, gc.KIND_GRAV, n)
    b.submit(t, np.zeros((0, 2), np.int32))
    b.commit()
    stream = torch.cuda.current_stream()
    b.reorganize(pool, gc.REORG_PACK, check_capacity=True)
    torch.cuda.synchronize()
    missing = int(b.maps()["missing"].size)
    ms = 0.0
    for _ in range(reps):
        pool.evict_staged(b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.reorganize(pool, gc.REORG_PACK, check_capacity=False)
        e1.record(stream)
        e1.synchronize()
        ms += e0.elapsed_time(e1) / reps
    b.status()
    # algorithmic bytes: per union entry the record read and the packed write (16 + 16), its id (4) and
    # its chare-table entry (4); per missing record the staged write into its slot (16).  The
    # occupancy scan, the chare-table and occupancy updates and the missing lists are implementation
    # traffic, reported beside it
    alg = nu * (16 + 16 + 4 + 4) + missing * 16
    impl = nu * 4 + missing * (4 + 4 + 8) + n * 4
    b.destroy()
    pool.destroy()
    del src
    # a plain copy of known size (256 MiB read + 256 MiB written) in the same run: the reference that
    # scales a profiler's FETCH_SIZE / WRITE_SIZE counters to bytes
    cx = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    cy = torch.empty_like(cx)
    cy.copy_(cx)
    torch.cuda.synchronize()
    del cx, cy
    gbps = alg / (ms * 1e-3) / 1e9
    return {"workload": f"pool 2^{log2_pool} records, union 2^{log2_union} ids (runs of {run}), half resident "
                        f"at random slots, PACK", "kernel": "k_reorg", "ms": round(ms, 4), "union": nu,
            "missing": missing, "algorithmic_bytes": int(alg), "implementation_bytes": int(impl),
            "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                         "frac": round(gbps / PEAK_HBM_GBPS, 4)},
            "gbps_incl_implementation_bytes": round((alg + impl) / (ms * 1e-3) / 1e9, 1)}


def leg_staging(gc, W, torch, ctx, w, rounds, prm, nodes, steps: int = 10):
    """The irregular workload with its records in ordinary host memory: every round the host finds the
    missing records in its mirror of the chare table, packs them into pinned memory and copies them in
    on a side stream (the copy of one round overlaps the pass of the round before); the same with the
    copies on the compute stream (no overlap); and redundant transfers (every record of each round's
    union copied each round).  Wall time per step, PCIe bytes per step."""
    dev = torch.device("cuda")
    host = np.ascontiguousarray(w.rec, dtype=np.float32)
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, w.n)
    pool.set_host_source(host)
    bids, bslots = W.residency(np.arange(w.n, dtype=np.int32), w.n, 0.5, seed=5000)
    pool.reset()
    pool.place(torch.from_numpy(bids).to(dev), torch.from_numpy(bslots).to(dev))
    batches = []
    for r in rounds:
        bt = W.task_subset(w, r)
        b = gc.Batch(ctx, gc.KIND_GRAV, w.n)
        b.submit(gc.tasks_from_csr(bt["i_begin"], bt["i_count"], bt["j_first"], bt["j_nr"], bt["n_first"],
                                   bt["n_count"]), bt["ranges"], bt["node_idx"])
        b.commit()
        batches.append(b)
    side = torch.cuda.Stream()

    host = {"evict": 0.0, "reorganize": 0.0, "launch": 0.0}

    def one(mode, use_side, clock=False):
        for k, b in enumerate(batches):
            t0 = time.perf_counter()
            pool.evict_staged(batches[k - 1])
            t1 = time.perf_counter()
            b.reorganize(pool, mode, check_capacity=False, side=side if use_side else None)
            t2 = time.perf_counter()
            b.launch(prm, nodes, acc)
            if clock:
                host["evict"] += t1 - t0
                host["reorganize"] += t2 - t1
                host["launch"] += time.perf_counter() - t2

    out = {"workload": f"nbody-plummer-{w.n}, {len(rounds)} rounds, source records in pageable host memory"}
    for name, mode, use_side in (("pack_side_stream", gc.REORG_PACK, True), ("pack_one_stream", gc.REORG_PACK, False),
                                 ("redundant_side_stream", gc.REORG_REDUNDANT, True)):
        for _ in range(2):
            one(mode, use_side)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            one(mode, use_side, clock=name == "pack_side_stream")
        torch.cuda.synchronize()
        out[f"{name}_ms"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
    out["host_ms_per_step_pack_side_stream"] = {k: round(v * 1e3 / steps, 4) for k, v in host.items()}
    sizes = []
    for b in batches:
        m = b.maps()
        sizes.append((int(m["U"].size), int(m["missing"].size)))
    pool.evict_staged(batches[-1])
    # the last reorganisation of each batch above was REDUNDANT; one PACK pass for the missing counts
    one(gc.REORG_PACK, True)
    torch.cuda.synchronize()
    miss = [int(b.maps()["missing"].size) for b in batches]
    pool.evict_staged(batches[-1])
    unions = [u for u, _ in sizes]
    out.update({"pcie_bytes_per_step_pack": 16 * sum(miss), "pcie_bytes_per_step_redundant": 16 * sum(unions),
                "transfer_reduction": round(1 - sum(miss) / sum(unions), 4),
                "overlap_gain": round(out["pack_one_stream_ms"] / out["pack_side_stream_ms"], 3)})
    for b in batches:
        b.status()
        b.destroy()
    pool.destroy()
    return out


def leg_rebuild(gc, W, torch, ctx, w, rounds, prm, steps: int = 5):
    """A step whose lists are rebuilt: the device list walk of every bucket, each round's tasks made
    from the walk's output and committed on the device (union and positions by mark and scan), then
    the rounds' reorganisations (PACK, half of all ids resident at random slots, each round evicting
    the staging of the one before) and combined passes.  Against it: the same step with the walk's
    lists copied to the host and each round submitted and committed there."""
    dev = torch.device("cuda")
    src = torch.from_numpy(w.rec).to(dev)
    nodes = torch.from_numpy(w.nodes).to(dev)
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    pool = gc.Pool(ctx, w.n, w.n)
    pool.set_source(src)
    bids, bslots = W.residency(np.arange(w.n, dtype=np.int32), w.n, 0.5, seed=5000)
    pool.reset()
    pool.place(torch.from_numpy(bids).to(dev), torch.from_numpy(bslots).to(dev))
    targs = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in
             (w.node_range.astype(np.int32), w.node_mom64[:, :3], w.node_side, w.rec, w.meta["leaf"].astype(np.int32))]
    bounds_h = np.array([int(r[0]) for r in rounds] + [w.n_tasks], np.int64)
    bounds = torch.from_numpy(bounds_h).to(dev)
    n_nodes = int(w.nodes.shape[0])
    batches = [gc.Batch(ctx, gc.KIND_GRAV, w.n) for _ in rounds]
    phase = {"walk": 0.0, "commit": 0.0, "pass": 0.0}
    # the walk's outputs, sized once (the tree does not change between steps)
    nf, nidx, rf, rng = gc.tree_walk(ctx, *targs, w.theta)
    nb = int(targs[4].numel())
    totals = (ctypes.c_int64 * 2)()

    def walk():
        ctx.check(gc.lib().gc_tree_walk(
            ctx.h, int(targs[0].shape[0]), targs[0].data_ptr(), targs[1].data_ptr(), targs[2].data_ptr(),
            targs[3].data_ptr(), int(targs[3].shape[0]), nb, targs[4].data_ptr(), float(w.theta), nf.data_ptr(),
            rf.data_ptr(), nidx.data_ptr(), int(nidx.numel()), rng.data_ptr(), int(rng.shape[0]), totals,
            torch.cuda.current_stream().cuda_stream), "gc_tree_walk")

    def passes():
        for k, b in enumerate(batches):
            if k:
                pool.evict_staged(batches[k - 1])
            b.reorganize(pool, gc.REORG_PACK, check_capacity=False)
            b.launch(prm, nodes, acc)
        pool.evict_staged(batches[-1])

    def step_device(timed=False):
        t0 = time.perf_counter()
        walk()
        bh = torch.stack([nf[bounds], rf[bounds]]).cpu().numpy()
        t1 = time.perf_counter()
        for k, b in enumerate(batches):
            b0, b1 = int(bounds_h[k]), int(bounds_h[k + 1])
            tasks = gc.walk_tasks(ctx, b0, b1, targs[4], targs[0], nf, rf)
            b.reset()
            b.submit_device(tasks, rng[bh[1, k]:bh[1, k + 1]], nidx[bh[0, k]:bh[0, k + 1]], n_nodes)
            b.commit()
        t2 = time.perf_counter()
        passes()
        torch.cuda.synchronize()
        if timed:
            phase["walk"] += t1 - t0
            phase["commit"] += t2 - t1
            phase["pass"] += time.perf_counter() - t2

    def step_host():
        walk()
        nfh, rfh, nih, rgh = nf.cpu().numpy(), rf.cpu().numpy(), nidx.cpu().numpy(), rng.cpu().numpy()
        leaf = w.meta["leaf"]
        for k, b in enumerate(batches):
            b0, b1 = int(bounds_h[k]), int(bounds_h[k + 1])
            lv = leaf[b0:b1]
            t = gc.tasks_from_csr(w.node_range[lv, 0], w.node_range[lv, 1], rfh[b0:b1] - rfh[b0],
                                  np.diff(rfh[b0:b1 + 1]), nfh[b0:b1] - nfh[b0], np.diff(nfh[b0:b1 + 1]))
            b.reset()
            b.submit(t, rgh[rfh[b0]:rfh[b1]], nih[nfh[b0]:nfh[b1]])
            b.commit()
        passes()
        torch.cuda.synchronize()

    out = {"workload": f"nbody-plummer-{w.n}: {w.n_tasks} buckets in {len(rounds)} rounds, walk theta {w.theta}"}
    for name, fn in (("device", step_device), ("host", step_host)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(True) if name == "device" else fn()
        out[f"step_with_rebuild_{name}_commit_ms"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
    out["device_phases_ms"] = {k: round(v * 1e3 / steps, 4) for k, v in phase.items()}
    for b in batches:
        b.status()
        b.destroy()
    pool.destroy()
    return out


def cpu_baseline(W, w, rounds, args):
    """The FP64 oracle on a bounded sample of the same rounds (host cores)."""
    import oracle as O
    ns = min(args.cpu_sample_rounds, len(rounds))
    sample = np.concatenate(rounds[:ns])
    bt = W.task_subset(w, sample)
    ic = bt["i_count"].astype(np.int64)
    cs = np.concatenate([[0], np.cumsum(bt["ranges"][:, 1].astype(np.int64))])
    nint = int(np.sum(ic * (cs[bt["j_first"] + bt["j_nr"]] - cs[bt["j_first"]] - 1 + bt["n_count"])))
    # the sample is evaluated repeatedly for about args.cpu_seconds (at least once, at most 200 times)
    reps, dt = 0, 0.0
    while reps == 0 or (dt < args.cpu_seconds and reps < 200):
        tc = time.perf_counter()
        O.grav_workload(w, order=2, tasks=bt)
        dt += time.perf_counter() - tc
        reps += 1
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": nint * reps / dt / 1e9, "unit": "G-interactions/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": f"first {ns} of {len(rounds)} rounds ({len(sample)} bucket tasks, {nint} interactions), "
                      f"FP64, evaluated {reps} times in {dt:.1f} s",
            "one_thread_uniform_4096": cpu_one_thread_small()}


# run in a child process so that its OpenMP runtime starts with one thread; it touches no GPU
_ONE_THREAD = """
import json, time, numpy as np, oracle as O, workloads as W
w = W.nbody_tiny()
ic = w.i_count.astype(np.int64)
nint = int(np.sum(ic * (w.direct_counts().astype(np.int64) - 1 + w.n_count)))
reps, dt = 0, 0.0
while reps == 0 or (dt < 2.0 and reps < 200):
    tc = time.perf_counter()
    O.grav_workload(w, order=1)
    dt += time.perf_counter() - tc
    reps += 1
print(json.dumps({"value": nint * reps / dt / 1e9, "reps": reps, "seconds": dt, "interactions": nint}))
"""


def cpu_one_thread_small():
    """The oracle on one thread over every task of nbody-uniform-4096 (monopole)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD], env=env, capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-300:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": round(d["value"], 4), "unit": "G-interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"every task of nbody-uniform-4096 ({d['interactions']} interactions, monopole), FP64, "
                      f"evaluated {d['reps']} times in {d['seconds']:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="pack", choices=["pack", "indirect", "sorted", "redundant"])
    ap.add_argument("--form", default="step", choices=["step", "rounds", "eager"],
                    help="step: one whole-step persistent launch (graph); rounds: a graph of per-round launches; "
                         "eager: per-round launches from the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rounds", type=int, default=1000, help="rounds of the step timed on the CPU")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="about how long the CPU baseline repeats its sample")
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--rounds", type=int, default=32, help="Poisson(2048) rounds per step (wrapping the tree order)")
    ap.add_argument("--quick", action="store_true",
                    help="skip the mode comparison, the single-launch measurement and the batched, LJ and adjoint legs")
    ap.add_argument("--tile", type=int, default=0, help="fixed force-kernel shape instead of the autotuner's")
    ap.add_argument("--waves", type=int, default=4)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--targets-per-lane", type=int, default=0, help="with --tile: 1, 2 or 3 (per task) targets per lane")
    ap.add_argument("--step-tile", type=int, default=0, help="fixed tile of the whole-step launch instead of timing 256, 320 and 384")
    ap.add_argument("--step-tpl", type=int, default=0, help="fixed targets per lane of the step forms instead of timing the tested ones")
    ap.add_argument("--step-waves", type=int, default=0, help="fixed waves per task of the step forms instead of timing the tested ones")
    ap.add_argument("--step-schedule", default="", choices=["", "step", "rounds"],
                    help="only the whole-step launch or only the rounds form (default: the faster)")
    ap.add_argument("--leg", default="", choices=["", "reorg-stress", "staging", "rebuild", "lj", "instances",
                                                  "combined", "ewald", "adjoint", "walk"],
                    help="run one measurement leg alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): there is no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2008_05712_amd as gc
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    modes = dict(pack=gc.REORG_PACK, indirect=gc.REORG_INDIRECT, sorted=gc.REORG_SORTED,
                 redundant=gc.REORG_REDUNDANT, none=gc.REORG_NONE)
    mode = modes[args.mode]

    if args.leg in ("reorg-stress", "lj", "instances", "ewald", "adjoint"):
        ctx = gc.Context(0)
        fn = {"reorg-stress": lambda: leg_reorg_stress(gc, torch, ctx), "lj": lambda: leg_lj(gc, W, torch, ctx),
              "instances": lambda: leg_instances(gc, W, torch, ctx, args),
              "ewald": lambda: leg_ewald(gc, W, torch, ctx), "adjoint": lambda: leg_adjoint(gc, W, torch, ctx)}[args.leg]
        print(json.dumps({"leg": args.leg, **fn()}), flush=True)
        ctx.close()
        return
    t0 = time.time()
    w = W.nbody_plummer(n=args.n, seed=1002)
    # the step: args.rounds Poisson(2048) rounds of consecutive buckets, wrapping around the tree order
    # (32: about 2.4 passes over the buckets); the host-source and list-rebuild legs take one pass
    rounds = W.poisson_rounds(w.n_tasks, 2048, seed=1002, n_rounds=args.rounds)
    rounds_pass = W.poisson_rounds(w.n_tasks, 2048, seed=1002)
    log(f"[bench] workload N={w.n} tasks={w.n_tasks} rounds={len(rounds)} build {time.time() - t0:.1f}s")
    # interactions of the step (a task in several rounds counts once per round) and of one pass
    ic_all = w.i_count.astype(np.int64)
    dir_t = ic_all * (w.direct_counts().astype(np.int64) - 1)
    node_t = ic_all * w.n_count.astype(np.int64)
    step_tasks = np.concatenate(rounds)
    n_direct, n_node = int(dir_t[step_tasks].sum()), int(node_t[step_tasks].sum())
    interactions = n_direct + n_node
    flops_step = n_direct * FLOPS_PAIR + n_node * FLOPS_QUAD
    interactions_all = int(dir_t.sum() + node_t.sum())
    flops_all = int(dir_t.sum()) * FLOPS_PAIR + int(node_t.sum()) * FLOPS_QUAD

    ctx = gc.Context(0)
    dev = torch.device("cuda")
    src = torch.from_numpy(w.rec).to(dev)
    nodes = torch.from_numpy(w.nodes).to(dev)
    if args.leg == "combined":
        # every task of the step in one launch, no reorganisation: the autotuner's shapes
        allb = gc.Batch(ctx, gc.KIND_GRAV, w.n)
        allb.submit(gc.tasks_from_csr(w.i_begin, w.i_count, w.j_first, w.j_nr, w.n_first, w.n_count), w.ranges,
                    w.node_idx)
        allb.commit()
        pl = gc.Pool(ctx, w.n, 1)
        pl.set_source(src)
        allb.reorganize(pl, gc.REORG_NONE)
        acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
        b2, t2, _ = allb.autotune(gc.grav_params(order=2), nodes, acc, reps=5)
        names = [f"t{t}_w{wv}_s{sc}_p{tp}" for t in (128, 256, 512) for wv in (2, 4, 8) for sc in (0, 1) for tp in (1, 2)]
        print(json.dumps({"leg": "combined", "best": dict(tile=b2.tile, waves=b2.waves_per_block, schedule=b2.schedule,
                                                          tpl=b2.targets_per_lane, aggregation=b2.aggregation),
                          "ms": {n: round(float(x), 4) for n, x in zip(names, t2)},
                          "aggregation_ms": [round(float(x), 4) for x in t2[36:]]}), flush=True)
        return
    if args.leg == "walk":
        print(json.dumps({"leg": "walk", **leg_walk(gc, W, torch, ctx, w)}), flush=True)
        ctx.close()
        return
    if args.leg in ("staging", "rebuild"):
        p2 = gc.grav_params(order=2, G=1.0, eps=0.01, tile=320, targets_per_lane=2)
        out = leg_staging(gc, W, torch, ctx, w, rounds_pass, p2, nodes) if args.leg == "staging" else \
            leg_rebuild(gc, W, torch, ctx, w, rounds_pass, p2)
        print(json.dumps({"leg": args.leg, **out}), flush=True)
        ctx.close()
        return
    acc = torch.zeros((w.n, 4), dtype=torch.float32, device=dev)
    cap = w.n
    pool = gc.Pool(ctx, w.n, cap)
    pool.set_source(src)
    # base residency: half of all particles at uniformly random slots; every round evicts what the
    # round before it staged, so each round finds about half of its union resident
    bids, bslots = W.residency(np.arange(w.n, dtype=np.int32), cap, 0.5, seed=5000)
    bids, bslots = torch.from_numpy(bids).to(dev), torch.from_numpy(bslots).to(dev)

    def base_state():
        pool.reset()
        pool.place(bids, bslots)

    batches, unions, round_flops = [], [], []
    for r in rounds:
        bt = W.task_subset(w, r)
        b = gc.Batch(ctx, gc.KIND_GRAV, w.n)
        b.submit(gc.tasks_from_csr(bt["i_begin"], bt["i_count"], bt["j_first"], bt["j_nr"], bt["n_first"],
                                   bt["n_count"]), bt["ranges"], bt["node_idx"])
        b.commit()
        batches.append(b)
        unions.append(int(W.batch_union(bt).size))
        ic = bt["i_count"].astype(np.int64)
        cs = np.concatenate([[0], np.cumsum(bt["ranges"][:, 1].astype(np.int64))])
        dcount = cs[bt["j_first"] + bt["j_nr"]] - cs[bt["j_first"]]
        round_flops.append(int(np.sum(ic * (dcount - 1))) * FLOPS_PAIR + int(np.sum(ic * bt["n_count"])) * FLOPS_QUAD)
    stream = torch.cuda.current_stream()
    R = len(batches)

    # ---- force-kernel shape: the autotuner's choice on the largest round (tile x waves x schedule x
    # targets per lane)
    tuned = None
    if args.tile:
        prm = gc.grav_params(order=2, G=1.0, eps=0.01, schedule=args.schedule, tile=args.tile,
                             waves_per_block=args.waves, targets_per_lane=args.targets_per_lane)
    else:
        big = int(np.argmax([len(r) for r in rounds]))
        base_state()
        batches[big].reorganize(pool, mode, check_capacity=False)
        best, times, _ = batches[big].autotune(gc.grav_params(order=2, G=1.0, eps=0.01), nodes, acc, reps=3)
        prm = gc.grav_params(order=2, G=1.0, eps=0.01, schedule=best.schedule, tile=best.tile,
                             waves_per_block=best.waves_per_block, targets_per_lane=best.targets_per_lane,
                             aggregation=best.aggregation)
        # candidate 16 is the default shape: tile 256, 4 waves, one block per task, one target per lane
        tuned = dict(tile=best.tile, waves_per_block=best.waves_per_block, schedule=best.schedule,
                     targets_per_lane=best.targets_per_lane, aggregation=best.aggregation,
                     ms=round(float(np.nanmin(times)), 5), default_shape_ms=round(float(times[16]), 5),
                     aggregation_ms=[round(float(x), 5) for x in times[36:]])
        log(f"[bench] autotuned: {tuned}")

    def one_pass(m, timed=None):
        """Every round once, eagerly: evict the previous round's staging, reorganise, launch.  With
        `timed`, HIP events on the launch stream bracket each reorganisation and each combined pass;
        the host enqueues the whole pass before reading them, so the device runs the rounds back to
        back and the intervals are device time, not host submission time."""
        ev = []
        for k, b in enumerate(batches):
            pool.evict_staged(batches[k - 1])
            if timed is not None:
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record(stream)
            b.reorganize(pool, m, check_capacity=False)
            if timed is not None:
                e[1].record(stream)
            b.launch(prm, nodes, acc)
            if timed is not None:
                e[2].record(stream)
                ev.append(e)
        if timed is not None:
            ev[-1][2].synchronize()
            for k, e in enumerate(ev):
                timed[0][k] += e[0].elapsed_time(e[1])
                timed[1][k] += e[1].elapsed_time(e[2])

    # a first pass from the base state: per-round missing counts (for the algorithmic bytes)
    base_state()
    one_pass(mode)
    torch.cuda.synchronize()
    missing = [int(b.maps()["missing"].size) if mode != gc.REORG_REDUNDANT else 0 for b in batches]
    pool.evict_staged(batches[-1])

    def capture(form, p):
        side = torch.cuda.Stream()
        g = gc.Graph(ctx, batches, [pool] * R, [mode] * R, p, nodes, acc, stream=side, fixture=gc.FIXTURE_EVICT_STAGED)
        torch.cuda.synchronize()
        return g

    # ---- the batched forms: a graph of per-round launches, and one whole-step persistent launch whose
    # tile and targets per lane are picked by timing the captured step (4 waves per task)
    forms = {}
    round_graph = capture("rounds", prm)
    forms["round_graph_ms"] = round(time_kernel(lambda: round_graph.launch(stream=stream), stream, reps=10), 4)
    sprm, step_graph, step_shapes, best_ms = None, None, {}, None
    if mode == gc.REORG_PACK:
        # the whole-step launch (4 waves per task) and the rounds form (one persistent launch for every
        # round's reorganisation, then one combined pass over all rounds' tasks), in their tested shapes
        cands = [(gc.SCHED_STEP, tl, tp, 4) for tl, tp in STEP_SHAPES] + \
                [(gc.SCHED_ROUNDS, tl, tp, wv) for tl, tp, wv in ROUNDS_SHAPES]
        cands = [c for c in cands if (not args.step_tile or c[1] == args.step_tile) and
                 (not args.step_tpl or c[2] == args.step_tpl) and (not args.step_waves or c[3] == args.step_waves) and
                 (not args.step_schedule or c[0] == {"step": gc.SCHED_STEP, "rounds": gc.SCHED_ROUNDS}[args.step_schedule])]
        if not cands:
            log(f"[bench] --step-tile {args.step_tile} --step-tpl {args.step_tpl} --step-waves {args.step_waves} "
                f"--step-schedule {args.step_schedule}: "
                f"not a tested shape {STEP_SHAPES} / {ROUNDS_SHAPES}")
            sys.exit(2)
        # every candidate captured, then timed in three interleaved passes (the best of the three per
        # shape), so that a drift of the clock during the sweep does not pick the shape
        graphs = []
        for sc, tl, tp, wv in cands:
            p = gc.grav_params(order=2, G=1.0, eps=0.01, schedule=sc, tile=tl, targets_per_lane=tp, waves_per_block=wv)
            name = "step" if sc == gc.SCHED_STEP else f"rounds_w{wv}"
            graphs.append((f"{name}_tile{tl}_tpl{tp}", p, capture("step", p)))
        for _ in range(3):
            for name, p, g in graphs:
                ms = round(time_kernel(lambda: g.launch(stream=stream), stream, reps=10), 4)
                step_shapes[name] = min(ms, step_shapes.get(name, ms))
        for name, p, g in graphs:
            if best_ms is None or step_shapes[name] < best_ms:
                sprm, step_graph, best_ms = p, g, step_shapes[name]
        for name, p, g in graphs:
            if g is not step_graph:
                g.destroy()
        forms["step_graph_ms_by_shape"] = step_shapes
    log(f"[bench] forms: {forms}")
    form = args.form if (args.form != "step" or step_graph is not None) else "rounds"
    graph = {"step": step_graph, "rounds": round_graph, "eager": None}[form]

    def step():
        if graph is None:
            one_pass(mode)
        else:
            graph.launch(stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # HIP events on the launch stream bracket every step inside the timed region: the device time of
    # each step's launch (for the whole-step form, the eviction kernel and the k_step launch)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t1 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        step()
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ms_step = (t2 - t1) * 1e3 / args.steps
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    avg_launch_ms = float(np.mean(launch_ms))
    value = interactions / (ms_step * 1e-3) / 1e9
    log(f"[bench] step {ms_step:.4f} ms  {value:.1f} G-interactions/s ({form}); launch {avg_launch_ms:.4f} ms "
        f"(min {min(launch_ms):.4f}, max {max(launch_ms):.4f})")
    # the device-side error words of every batch the timed launches used: a bounded wait that gave up
    # would have left unspecified accelerations in the timed region
    try:
        if graph is not None:
            graph.status(stream=stream)
        for b in batches:
            b.status(stream=stream)
    except gc.GcError as e:
        log(f"[bench] FAILED: {e}")
        sys.exit(3)
    # the eager form's step time, for comparison
    torch.cuda.synchronize()
    te = time.perf_counter()
    for _ in range(3):
        one_pass(mode)
    torch.cuda.synchronize()
    forms["eager_ms"] = round((time.perf_counter() - te) * 1e3 / 3, 4)
    pool.evict_staged(batches[-1])
    # the plain per-batch form with indirect access: per-round launches from the host, address lists
    one_pass(gc.REORG_INDIRECT)  # sizes the list buffers (not timed)
    pool.evict_staged(batches[-1])
    torch.cuda.synchronize()
    te = time.perf_counter()
    for _ in range(3):
        one_pass(gc.REORG_INDIRECT)
    torch.cuda.synchronize()
    forms["eager_indirect_ms"] = round((time.perf_counter() - te) * 1e3 / 3, 4)
    pool.evict_staged(batches[-1])
    forms["timed_vs_eager_indirect"] = round(forms["eager_indirect_ms"] / ms_step, 3)
    if graph is not None and form == "step":
        step_kernel_ms = avg_launch_ms
    # the same whole-step launch with the source records in pinned host memory: the staging of the
    # missing records reads them across PCIe (the boundary's host-buffer path; never the bench value)
    if not args.quick and sprm is not None:
        hsrc = torch.from_numpy(np.ascontiguousarray(w.rec)).pin_memory()
        pool.set_source(hsrc)
        hg = capture("step", sprm)
        hms = time_kernel(lambda: hg.launch(stream=stream), stream, reps=10)
        hg.destroy()
        pool.set_source(src)
        forms["step_graph_pinned_host_source_ms"] = round(hms, 4)
        forms["pinned_host_source_ginteractions_per_s"] = round(interactions / (hms * 1e-3) / 1e9, 3)
        del hsrc

    # ---- per-phase device times with HIP events on the launch stream (eager, same work)
    def phases(m, reps):
        t = (np.zeros(R), np.zeros(R))
        for _ in range(reps):
            one_pass(m, timed=t)
        pool.evict_staged(batches[-1])
        torch.cuda.synchronize()
        return t[0] / reps, t[1] / reps

    r_ms, k_ms = phases(mode, 5)
    kern_ms = float(k_ms.sum())
    achieved_tflops = sum(round_flops) / (kern_ms * 1e-3) / 1e12
    reorg_ms = float(r_ms.sum())
    round_bytes = [u * REORG_BYTES_PER_UNION + m * REORG_BYTES_PER_MISSING + cap * REORG_BYTES_PER_SLOT
                   for u, m in zip(unions, missing)]
    reorg_gbps = sum(round_bytes) / (reorg_ms * 1e-3) / 1e9
    log(f"[bench] kernel sum {kern_ms:.4f} ms  reorganize sum {reorg_ms:.4f} ms")

    # ---- the reorganisation modes side by side (the indirect-access kernel is the plain per-batch form)
    mode_cmp = None
    if not args.quick:
        mode_cmp = {}
        for name in ("pack", "indirect", "sorted", "redundant", "none"):
            try:
                one_pass(modes[name])  # sizes the mode's buffers (not timed)
            except gc.GcError as e:
                mode_cmp[name] = {"error": str(e)}
                continue
            pool.evict_staged(batches[-1])
            rm, km = phases(modes[name], 3)
            mode_cmp[name] = {"reorganize_ms": round(float(rm.sum()), 4), "kernel_ms": round(float(km.sum()), 4),
                              "kernel_ginteractions_per_s": round(interactions / (float(km.sum()) * 1e-3) / 1e9, 2),
                              "reorganize_plus_kernel_ms": round(float(rm.sum() + km.sum()), 4)}
        log(f"[bench] modes: {mode_cmp}")

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same rounds
    cpu = None if args.no_cpu_baseline else cpu_baseline(W, w, rounds, args)

    # ---- calibration copy of known size (read 256 MiB + write 256 MiB): HBM rate on this machine, and the
    # reference kernel that scales the FETCH_SIZE / WRITE_SIZE counters of a profiled run
    cx = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    cy = torch.empty_like(cx)
    copy_ms = time_kernel(lambda: cy.copy_(cx), stream, reps=5)
    copy_gbps = 2 * cx.numel() * 4 / (copy_ms * 1e-3) / 1e9
    del cx, cy

    # ---- one launch over all 27k tasks (the fully combined request): kernel efficiency at occupancy
    combined_all = None
    if not args.quick:
        allb = gc.Batch(ctx, gc.KIND_GRAV, w.n)
        allb.submit(gc.tasks_from_csr(w.i_begin, w.i_count, w.j_first, w.j_nr, w.n_first, w.n_count), w.ranges,
                    w.node_idx)
        allb.commit()
        allb.reorganize(pool, gc.REORG_NONE)
        ball, tall, _ = allb.autotune(gc.grav_params(order=2, G=1.0, eps=0.01), nodes, acc, reps=3)
        pall = gc.grav_params(order=2, G=1.0, eps=0.01, schedule=ball.schedule, tile=ball.tile,
                              waves_per_block=ball.waves_per_block, targets_per_lane=ball.targets_per_lane)
        ms_all = time_kernel(lambda: allb.launch(pall, nodes, acc), stream)
        combined_all = {"ms": round(ms_all, 4), "tflops": round(flops_all / (ms_all * 1e-3) / 1e12, 3),
                        "ginteractions_per_s": round(interactions_all / (ms_all * 1e-3) / 1e9, 3),
                        "shape": dict(tile=ball.tile, waves_per_block=ball.waves_per_block, schedule=ball.schedule,
                                      targets_per_lane=ball.targets_per_lane),
                        "shape_ms": {f"t{t}_w{wv}_s{sc}_p{tp}": round(float(tall[i]), 4) for i, (t, wv, sc, tp) in
                                     enumerate((t, wv, sc, tp) for t in (128, 256, 512) for wv in (2, 4, 8)
                                               for sc in (0, 1) for tp in (1, 2))}}
        allb.destroy()
    occ_blocks, n_cu = ctx.occupancy(prm)
    step_occ = ctx.occupancy(sprm)[0] if sprm is not None else None

    extra = {}
    if not args.quick:
        extra["batched_instances"] = leg_instances(gc, W, torch, ctx, args)
        extra["lj"] = leg_lj(gc, W, torch, ctx)
        extra["ewald"] = leg_ewald(gc, W, torch, ctx)
        extra["adjoint"] = leg_adjoint(gc, W, torch, ctx)
        extra["tree_walk"] = leg_walk(gc, W, torch, ctx, w)
        extra["rebuild"] = leg_rebuild(gc, W, torch, ctx, w, rounds_pass, prm)
        extra["staging"] = leg_staging(gc, W, torch, ctx, w, rounds_pass, prm, nodes)
        extra["reorg_stress"] = leg_reorg_stress(gc, torch, ctx)

    form_text = {"step": "one whole-step persistent launch (HIP graph) per step",
                 "rounds": "one HIP graph of per-round launches per step", "eager": "per-round launches"}[form]
    if form == "step" and sprm is not None and sprm.schedule == gc.SCHED_ROUNDS:
        form_text = ("one HIP graph per step: every round's reorganisation in one persistent launch, then one "
                     "combined pass over all rounds' tasks")
    tpl = max(1, prm.targets_per_lane)
    per_round = {"kernel": f"k_grav<2, false, {'true' if prm.schedule else 'false'}, {'true' if tpl == 2 else 'false'}> "
                           f"(tile {prm.tile}, {prm.waves_per_block} waves per task, {tpl} targets per lane)",
                 "kernel_ms_per_step": round(kern_ms, 4), "avg_launch_ms": round(kern_ms / R, 5),
                 "tflops": round(achieved_tflops, 3), "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4),
                 "traffic": None}  # counters are taken for the timed form's kernels only
    if form == "step":
        # the dominant (and only) kernel of a step: algorithmic flop of the whole step over its duration
        step_tflops = flops_step / (step_kernel_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(step_tflops, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(step_tflops / PEAK_FP32_TFLOPS, 4),
                    # counters are taken for the rounds form, the one timed on this workload
                    "traffic": None if sprm.schedule == gc.SCHED_STEP else
                    profiled_traffic("k_grav_rounds_quad_plummer262144_traffic",
                                     {"tile": sprm.tile, "targets_per_lane": sprm.targets_per_lane,
                                      "waves_per_block": sprm.waves_per_block}),
                    "kernel": (f"k_step<2, {'true' if sprm.targets_per_lane == 2 else 'false'}> (every round's "
                               f"reorganisation, with the eviction of what it staged, and combined quadrupole pass; "
                               f"tile {sprm.tile}, 4 waves per task, {sprm.targets_per_lane} targets per lane)")
                    if sprm.schedule == gc.SCHED_STEP else
                    (f"k_step<2, 1, false> (every round's reorganisation and eviction; no force code) + "
                     f"k_grav_rounds<2, {sprm.targets_per_lane}> (one combined quadrupole pass over every round's "
                     f"tasks; tile {sprm.tile}, {sprm.waves_per_block} wave{'s' if sprm.waves_per_block > 1 else ''} per task, "
                     f"{TPL_TEXT[sprm.targets_per_lane]}), "
                     f"timed together: the step's whole device time"),
                    "flops_per_launch": flops_step, "avg_launch_ms": round(step_kernel_ms, 5),
                    "frac_of_nonpacked_peak": round(step_tflops / PEAK_FP32_NONPACKED_TFLOPS, 4)}
    else:
        roofline = {"bound": "alu", "achieved": per_round["tflops"], "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "frac": per_round["frac"], "traffic": per_round["traffic"], "kernel": per_round["kernel"],
                    "flops_per_step": flops_step, "kernel_ms_per_step": per_round["kernel_ms_per_step"],
                    "avg_launch_ms": per_round["avg_launch_ms"],
                    "frac_of_nonpacked_peak": round(achieved_tflops / PEAK_FP32_NONPACKED_TFLOPS, 4)}
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"nbody-plummer-{w.n}: bucket 32, theta 0.7, monopole+quadrupole, eps 0.01, "
                               f"{R} Poisson(2048) rounds of consecutive buckets (wrapping the tree order), "
                               f"half of all particles resident at random slots "
                               f"(each round evicts the previous round's staging), the missing records staged "
                               f"from a copy of every record in HBM (host-source rates: forms and staging), "
                               f"{args.mode} reorganisation, {form_text}",
                   "n": w.n, "tasks": w.n_tasks, "rounds": R, "interactions_per_step": interactions,
                   "mode": args.mode, "form": form},
        "roofline": roofline,
        "per_round_force_kernel": per_round,
        "forms": forms,
        "cpu_baseline": cpu,
        "reorganize": {"gbps": round(reorg_gbps, 2), "frac_hbm": round(reorg_gbps / PEAK_HBM_GBPS, 4),
                       "ms_per_step": round(reorg_ms, 4), "avg_launch_ms": round(reorg_ms / R, 5),
                       "algorithmic_bytes_per_step": int(sum(round_bytes)),
                       "union_per_round": unions, "missing_per_round": missing,
                       "note": "one launch per round over ~35k union entries: latency-bound, cache-resident"},
        "kernel_only_ginteractions_per_s": round(interactions / (kern_ms * 1e-3) / 1e9, 3),
        "autotune_largest_round": tuned,
        "modes": mode_cmp,
        "combined_all_tasks_one_launch": combined_all,
        "occupancy": {"blocks_per_cu": occ_blocks, "cus": n_cu, "waves_per_block": prm.waves_per_block,
                      "step_kernel_blocks_per_cu": step_occ},
        "hbm_copy_gbps": round(copy_gbps, 1),
        "bwd_fwd": extra.get("adjoint", {}).get("bwd_fwd"),
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    for g in (round_graph, step_graph):
        if g is not None:
            g.destroy()
    for b in batches:
        b.destroy()
    pool.destroy()
    ctx.close()


if __name__ == "__main__":
    main()
