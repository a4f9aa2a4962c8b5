"""torch.autograd wrapper of the FWIME predicted-data map.

d_pred(m, p~) = f(m) + B~(m) p~  (the modeled data of eq. fwime.obj).  The
forward pass runs fwime_forward_tape, which keeps sqrt(nt)-spaced checkpoints
of the background and scattered wavefields on the device; the backward pass
runs the hand-written adjoint-state backward (fwime_backward_tape) with the
incoming gradient as adjoint source and returns
  dL/dm  = (B^* + T^*) dL/dd   (Born and tomographic parts of
                                eqs. fwime.gradient.born and .tomo),
  dL/dp~ = B~^* dL/dd.
Any scalar loss built in torch on top of d_pred (e.g. the misfit and the DSO
penalty of eq. fwime.obj) then differentiates through the HIP path.
"""
from __future__ import annotations

import torch

from ._abi import Context, Geometry, Grid


class FwimeOp(torch.autograd.Function):
    @staticmethod
    def forward(fctx, vel, ptilde, ctx: Context, grid: Grid, geom: Geometry):
        nh = int(ptilde.shape[0])
        vel = vel.detach().contiguous()
        ptilde = ptilde.detach().contiguous()
        data = torch.empty((geom.nshots, geom.nrec, grid.nt), device=vel.device, dtype=torch.float32)
        tape = ctx.fwime_forward_tape(grid, vel, geom, nh, ptilde, data)
        fctx.tape = tape
        fctx.ctx = ctx
        return data

    @staticmethod
    def backward(fctx, grad_data):
        tape = fctx.tape
        if tape is None:
            raise RuntimeError("FwimeOp backward called twice (the tape serves one backward)")
        g = tape.grid
        gv = torch.empty((g.nx, g.nz), device=grad_data.device, dtype=torch.float32)
        gp = torch.empty((tape.nh, g.nx, g.nz), device=grad_data.device, dtype=torch.float32)
        try:
            fctx.ctx.fwime_backward_tape(tape, grad_data.contiguous().float(), gv, gp)
        finally:
            tape.free()
            fctx.tape = None
        return gv, gp, None, None, None


def predicted_data(vel, ptilde, ctx: Context, grid: Grid, geom: Geometry):
    """d_pred = f(m) + B~(m) p~, differentiable in vel and ptilde."""
    return FwimeOp.apply(vel, ptilde, ctx, grid, geom)
