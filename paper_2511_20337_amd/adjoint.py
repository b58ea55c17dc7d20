"""Differentiation through N steps: a torch.autograd.Function over the C ABI.

Forward runs N steps of ``mhd_step`` with a given (frozen) time-step sequence
and keeps a checkpoint of the state every ``every`` steps. Backward replays
each segment forward from its checkpoint (storing that segment's states) and
applies ``mhd_adjoint_step`` in reverse. Memory: N/every checkpoints plus one
segment of ``every`` states; ``every = 1`` keeps every state of the forward
pass, so the backward replays nothing. Torch only holds buffers and orders the calls;
all arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

import torch

from . import mhd


class MHDSteps(torch.autograd.Function):
    """U_N = Phi_{dt_{N-1}} o ... o Phi_{dt_0} (U_0).

    Inputs: U0 (float64 CUDA tensor, state layout), dts (float64 CPU tensor of
    N time steps), a ``mhd.Context`` created with ``with_adjoint=True``, and
    the checkpoint interval. Gradients flow to U0 and dts."""

    @staticmethod
    def forward(fctx, U0, dts, solver, every):
        every = max(1, int(every))
        dt_list = [float(x) for x in dts.detach().cpu().tolist()]
        U = U0.detach().clone()
        checkpoints = {}
        for s, dt in enumerate(dt_list):
            if s % every == 0:
                checkpoints[s] = U.clone()
            solver.step(U, dt)
        fctx.solver = solver
        fctx.dt_list = dt_list
        fctx.every = every
        fctx.checkpoints = checkpoints
        fctx.dts_shape = dts.shape
        return U

    @staticmethod
    def backward(fctx, gU):
        solver = fctx.solver
        dts = fctx.dt_list
        n = len(dts)
        bar = gU.detach().contiguous().clone()
        # dt-bar (its partial sums re-read the stage's records) only when the
        # time steps require a gradient
        want_dt = fctx.needs_input_grad[1]
        dtbar_dev = torch.zeros(n, dtype=torch.float64, device=bar.device)
        tmp = torch.empty_like(bar)
        for start in reversed(sorted(fctx.checkpoints)):
            stop = min(start + fctx.every, n)
            # replay the segment, keeping the state at the start of each step
            # (the adjoint step only reads its state, so the checkpoint itself
            # serves as the first)
            states = [fctx.checkpoints[start]]
            for s in range(start, stop - 1):
                U = states[-1].clone()
                solver.step(U, dts[s])
                states.append(U)
            for s in range(stop - 1, start - 1, -1):
                solver.adjoint_step(states[s - start], dts[s], bar, out=tmp,
                                    dtbar_out=dtbar_dev[s:s + 1] if want_dt else None)
                bar, tmp = tmp, bar
        dtbar = dtbar_dev.cpu().reshape(fctx.dts_shape) if want_dt else None
        return bar, dtbar, None, None


def run_with_grad(solver, U0, dts, every=8):
    """Differentiable N-step run (see MHDSteps)."""
    if not isinstance(dts, torch.Tensor):
        dts = torch.tensor(list(dts), dtype=torch.float64)
    return MHDSteps.apply(U0, dts, solver, every)


def record_dts(solver, U0, nsteps):
    """Unperturbed forward run that records the CFL time steps (copy of U0)."""
    U = U0.detach().clone()
    dts = []
    for _ in range(nsteps):
        dt = solver.dt(U)
        dts.append(dt)
        solver.step(U, dt)
    return torch.tensor(dts, dtype=torch.float64), U
