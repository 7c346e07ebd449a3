"""torch.autograd bridge for K unrolled fixed-step PDHG iterations.

PDHGUnroll.apply(solver, K, c, rhs, l, u, x0, y0) -> (x_K, y_K)

Forward: installs (c, rhs, l, u) in the handle (pdhg_set_data), starts every
instance at (x0, y0) (pdhg_set_state), and runs K recorded fixed-step
iterations (pdhg_iterate with record = 1: checkpoints every
opts.unroll_checkpoint steps).  Backward: pdhg_backward replays each
checkpoint segment with the clip masks and runs the reverse steps on the GPU.
A handle keeps one tape: backward raises PDHGError (PDHG_ERR_STATE) when a
later forward call or set_data on the same handle has replaced it.

All tensors are FP64 and concatenated over the solver's batch (the y parts in
the caller's row order).  tau, sigma and the Ruiz factors are constants of
the handle.  (x0, y0) should be feasible (l <= x0 <= u, y0 >= 0 on ">=" rows):
the handle starts from their projection.
"""
from __future__ import annotations

import numpy as np
import torch

from . import PDHG_ERR_STATE, SOL_CURRENT, PDHGError


def _np(t):
    return None if t is None else t.detach().to("cpu", torch.float64).contiguous().numpy()


class PDHGUnroll(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, K: int, c, rhs, l, u, x0, y0):
        solver.set_data(_np(c), _np(rhs), _np(l), _np(u))
        xs, ys = _np(x0), _np(y0)
        xo = yo = 0
        for i, (n, m) in enumerate(solver.sizes):
            solver.set_state(xs[xo:xo + n], ys[yo:yo + m], inst=i)
            xo += n
            yo += m
        solver.iterate(int(K), record=True)
        ctx.generation = solver.info()["record_generation"]
        xk, yk = [], []
        for i in range(solver.batch):
            x, y = solver.solution(inst=i, which=SOL_CURRENT)
            xk.append(x)
            yk.append(y)
        ctx.solver = solver
        dev = c.device
        return (torch.from_numpy(np.concatenate(xk)).to(dev), torch.from_numpy(np.concatenate(yk)).to(dev))

    @staticmethod
    def backward(ctx, gx, gy):
        s = ctx.solver
        if s.info()["record_generation"] != ctx.generation:
            # another forward (or new data) replaced this call's tape in the handle
            raise PDHGError(PDHG_ERR_STATE, "the handle's recorded steps are no longer those of this "
                            "forward call (a later forward or set_data replaced them)")
        nt = sum(n for n, _ in s.sizes)
        mt = sum(m for _, m in s.sizes)
        gxn = np.zeros(nt) if gx is None else _np(gx)
        gyn = np.zeros(mt) if gy is None else _np(gy)
        g = s.backward(gxn, gyn)
        dev = gx.device if gx is not None else gy.device
        t = {k: torch.from_numpy(v).to(dev) for k, v in g.items()}
        return None, None, t["c"], t["rhs"], t["l"], t["u"], t["x0"], t["y0"]
