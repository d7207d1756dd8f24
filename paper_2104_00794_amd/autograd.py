"""Differentiation through the probed modelling operator.

``ProbedModeling.apply(m, grid, geom, probe)`` returns the traces d = F(m; q)
(Eq. 2).  Its backward is the hand-written adjoint with the probed imaging
condition (Eq. 4, Algorithm 1): the forward pass keeps only the probed
wavefield ubar (S x r x N values) instead of the N x n_t history, so probing
acts as a recompute-free checkpoint.  With identity probes (r = n_t) the
backward is the exact adjoint-state gradient (Eq. 3).

The gradient is with respect to the squared slowness on the physical grid,
for perturbations that vanish on its outermost nodes (the model is extended
into the absorbing layer by edge replication, and the gradient is that of the
extended model restricted to the physical grid).
"""
from __future__ import annotations

import torch

from . import tpx


class ProbedModeling(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, grid: tpx.Grid, geom: tpx.Geometry, probe: tpx.Probe):
        m = m.detach().contiguous()
        d, state = tpx.forward_probed(grid, geom, probe, m)
        ctx.save_for_backward(m, state)
        ctx.grid, ctx.geom, ctx.probe = grid, geom, probe
        return d

    @staticmethod
    def backward(ctx, grad_d):
        m, state = ctx.saved_tensors
        g = tpx.backward_probed(ctx.grid, ctx.geom, ctx.probe, m, grad_d.contiguous().to(torch.float32), state)
        return g, None, None, None


def modeling(m, grid: tpx.Grid, geom: tpx.Geometry, probe: tpx.Probe):
    """d = F(m; q) with the probed adjoint as its backward."""
    return ProbedModeling.apply(m, grid, geom, probe)


def exact_probe(grid: tpx.Grid) -> tpx.Probe:
    """Identity probes: the backward is then the exact gradient (memory N x n_t)."""
    return tpx.Probe(kind="identity", r=grid.nt)


def misfit(d, d_obs):
    """0.5 ||d - d_obs||^2 (Eq. 2)."""
    r = d - d_obs
    return 0.5 * torch.sum(r * r)
