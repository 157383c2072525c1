"""torch.autograd.Function wrappers over the combined pass (forward: gc_launch_combined,
backward: gc_backward).  Argument marshalling only; both directions run in the HIP library."""
from __future__ import annotations

import torch

from . import Batch, Context, Pool, ForceParams, FORCE_LJ, REORG_NONE


class CombinedGravity(torch.autograd.Function):
    """acc = combined monopole gravity of `rec` (float32 [n, 4]: x, y, z, m) over `batch`'s lists.

    The batch is reorganised in place mode NONE against `pool` whose source is `rec` itself.
    Backward returns dL/drec with (dL/dx, dL/dy, dL/dz, dL/dm) per particle."""

    @staticmethod
    def forward(ctx_, rec, nodes, node_range, batch: Batch, pool: Pool, prm: ForceParams):
        pool.set_source(rec)
        batch.reorganize(pool, REORG_NONE)
        acc = torch.empty_like(rec)
        batch.launch(prm, nodes, acc)
        ctx_.save_for_backward(nodes, node_range)
        ctx_.batch, ctx_.prm, ctx_.n = batch, prm, rec.shape[0]
        return acc

    @staticmethod
    def backward(ctx_, gacc):
        nodes, node_range = ctx_.saved_tensors
        cot = gacc.contiguous()
        gpos = torch.zeros((ctx_.n, 4), dtype=torch.float32, device=cot.device)
        gmass = torch.zeros(ctx_.n, dtype=torch.float32, device=cot.device)
        ctx_.batch.backward(ctx_.prm, nodes, node_range, node_range.shape[0], cot, gpos, gmass)
        grec = gpos.clone()
        grec[:, 3] = gmass
        return grec, None, None, None, None, None


class CombinedLJ(torch.autograd.Function):
    """acc = combined Lennard-Jones accelerations of `rec` (float32 [n, 4]: x, y, z, type).

    Differentiable inputs: positions (columns 0-2 of rec), per-type eps_t and sig_t.  The
    per-atom mass gradient (mass as if each atom had its own) is exposed as `ctx.gmass` of the
    last backward through `CombinedLJ.last_gmass`."""

    last_gmass = None

    @staticmethod
    def forward(ctx_, rec, eps_t, sig_t, mass_t, r_cut: float, batch: Batch, pool: Pool):
        pool.set_source(rec)
        batch.reorganize(pool, REORG_NONE)
        prm = ForceParams()
        prm.kind = FORCE_LJ
        prm.n_types = int(eps_t.numel())
        prm.eps_t, prm.sig_t, prm.mass_t = eps_t.data_ptr(), sig_t.data_ptr(), mass_t.data_ptr()
        prm.r_cut = r_cut
        acc = torch.empty_like(rec)
        batch.launch(prm, None, acc)
        ctx_.save_for_backward(eps_t, sig_t, mass_t)
        ctx_.batch, ctx_.prm, ctx_.n = batch, prm, rec.shape[0]
        return acc

    @staticmethod
    def backward(ctx_, gacc):
        eps_t, sig_t, mass_t = ctx_.saved_tensors
        cot = gacc.contiguous()
        gpos = torch.zeros((ctx_.n, 4), dtype=torch.float32, device=cot.device)
        gmass = torch.zeros(ctx_.n, dtype=torch.float32, device=cot.device)
        gparam = torch.zeros(2 * eps_t.numel(), dtype=torch.float32, device=cot.device)
        ctx_.batch.backward(ctx_.prm, None, None, 0, cot, gpos, gmass, gparam)
        CombinedLJ.last_gmass = gmass
        grec = gpos.clone()
        grec[:, 3] = 0.0
        nt = eps_t.numel()
        return grec, gparam[:nt].clone(), gparam[nt:].clone(), None, None, None, None


__all__ = ["CombinedGravity", "CombinedLJ", "Context"]
