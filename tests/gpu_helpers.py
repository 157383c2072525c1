"""Marshalling between seeded workloads and the device library for the GPU tests."""
from __future__ import annotations

import numpy as np

import paper_2008_05712_amd as gc
import workloads as W


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def grav_tasks(b: dict) -> np.ndarray:
    return gc.tasks_from_csr(b["i_begin"], b["i_count"], b["j_first"], b["j_nr"], b["n_first"], b["n_count"])


def whole(w) -> dict:
    return dict(i_begin=w.i_begin, i_count=w.i_count, n_first=w.n_first, n_count=w.n_count, j_first=w.j_first,
                j_nr=w.j_nr, node_idx=w.node_idx, ranges=w.ranges)


class GravRig:
    """Device copies of one gravity workload: source records, node table, output."""

    def __init__(self, ctx: gc.Context, w, capacity: int | None = None):
        torch = torch_cuda()
        self.torch = torch
        self.ctx, self.w = ctx, w
        self.src = torch.from_numpy(np.ascontiguousarray(w.rec)).cuda()
        self.nodes = torch.from_numpy(np.ascontiguousarray(w.nodes)).cuda()
        self.acc = torch.zeros((w.n, 4), dtype=torch.float32, device="cuda")
        self.pool = gc.Pool(ctx, w.n, capacity or w.n)
        self.pool.set_source(self.src)

    def batch(self, tasks: dict) -> gc.Batch:
        b = gc.Batch(self.ctx, gc.KIND_GRAV, self.w.n)
        b.submit(grav_tasks(tasks), tasks["ranges"], tasks["node_idx"])
        b.commit()
        return b

    def place(self, ids: np.ndarray, slots: np.ndarray):
        torch = self.torch
        self.pool.place(torch.from_numpy(ids.astype(np.int32)).cuda(), torch.from_numpy(slots.astype(np.int32)).cuda())

    def run(self, b: gc.Batch, mode: int, order: int, fill: float = np.nan, **prm) -> np.ndarray:
        self.acc.fill_(fill)
        b.reorganize(self.pool, mode)
        b.launch(gc.grav_params(order=order, **prm), self.nodes, self.acc)
        self.torch.cuda.synchronize()
        return self.acc.cpu().numpy()

    def close(self):
        self.pool.destroy()


def rel_l2_per_task(acc_gpu, acc_ref, tasks: dict) -> np.ndarray:
    import oracle as O
    return O.per_task_rel_l2(acc_gpu[:, :3].astype(np.float64), acc_ref, tasks["i_begin"], tasks["i_count"])


__all__ = ["GravRig", "grav_tasks", "whole", "rel_l2_per_task", "torch_cuda", "W"]
