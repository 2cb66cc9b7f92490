"""Differentiable rollout of the CHNS step: torch.autograd.Function over
``Grid.step`` (forward) and ``Grid.adjoint_step`` (reverse), with
checkpointing.

The forward pass advances ``nsteps`` steps and keeps the state (phi, u, p)
only every ``checkpoint_every`` steps.  The backward pass walks the segments
in reverse: it re-runs the forward steps of a segment from its checkpoint,
keeping the segment's states and recording each step's forward fields
(``Grid.step_record``), then applies the reverse step to them in reverse
order (``Grid.adjoint_step_recorded``), so no step is computed a third time.
Forward and recomputation run the same kernels on the same inputs, so the
gradient does not depend on ``checkpoint_every`` (bit for bit).

Differentiable inputs: the initial phi field, the initial velocity, and the
surface tension sigma and mobility M, which enter the properties as
We = 1/sigma and Pe = 1/(M sigma) (so k_M = M sigma / Cn).  Every arithmetic
step runs in the library's HIP kernels; this module only sequences calls and
copies device tensors.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Sequence, Tuple

from . import CHNS_OPT_TIME_GUESS, Grid, _torch


def props_for(props, sigma: float, mobility: float):
    """Properties with We = 1/sigma and Pe = 1/(M sigma), the rest kept."""
    return props.copy(We=1.0 / sigma, Pe=1.0 / (mobility * sigma))


def _snapshot(st: Dict) -> Dict:
    return {"phi": st["phi"].clone(), "u": [x.clone() for x in st["u"]], "p": st["p"].clone(),
            "mu": st["mu"]}


def _restore(grid: Grid, snap: Dict) -> Dict:
    torch = _torch()
    return {"phi": snap["phi"].clone(), "u": [x.clone() for x in snap["u"]], "p": snap["p"].clone(),
            "mu": torch.zeros_like(snap["phi"])}


def _run(grid: Grid, props, sigma: float, mobility: float, phi0, u0: Sequence, nsteps: int, every: int):
    torch = _torch()
    grid.set_properties(props_for(props, sigma, mobility))
    # the reverse sweep recomputes segments from checkpoints with step
    # records, which start the pressure solve from the stored p: the forward
    # steps do the same, so that the recomputation repeats them bit for bit
    grid.set_option(CHNS_OPT_TIME_GUESS, 0)
    st = {"phi": phi0.detach().clone().contiguous(), "u": [x.detach().clone().contiguous() for x in u0],
          "p": torch.zeros_like(phi0), "mu": torch.zeros_like(phi0)}
    checkpoints: List[Dict] = []
    for n in range(nsteps):
        if n % every == 0:
            checkpoints.append(_snapshot(st))
        grid.step(st, 1, stats=False)
    return st, checkpoints


class CHNSRollout:
    """Namespace for the autograd.Function (built lazily so that importing
    the package does not import torch)."""

    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is not None:
            return cls._fn
        torch = _torch()

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, grid, props, nsteps, every, params, phi0, *u0):
                sigma, mobility = (float(v) for v in params.detach().cpu().tolist())
                st, checkpoints = _run(grid, props, sigma, mobility, phi0, u0, nsteps, every)
                ctx.grid, ctx.props, ctx.nsteps, ctx.every = grid, props, nsteps, every
                ctx.sigma, ctx.mobility = sigma, mobility
                ctx.checkpoints = checkpoints
                ctx.params_meta = (params.dtype, params.device)
                return (st["phi"], *st["u"])

            @staticmethod
            def backward(ctx, gphi, *gu):
                grid: Grid = ctx.grid
                grid.set_properties(props_for(ctx.props, ctx.sigma, ctx.mobility))
                grid.attach_adjoint()
                ref = ctx.checkpoints[0]["phi"]
                lam = {"phi": (gphi if gphi is not None else torch.zeros_like(ref)).detach().clone().contiguous(),
                       "u": [(g if g is not None else torch.zeros_like(ref)).detach().clone().contiguous()
                             for g in gu]}
                grad = (ctypes.c_double * 2)(0.0, 0.0)
                nseg = len(ctx.checkpoints)
                recs = [grid.new_record() for _ in range(min(ctx.every, ctx.nsteps))]
                for seg in reversed(range(nseg)):
                    start = seg * ctx.every
                    end = min(start + ctx.every, ctx.nsteps)
                    st = _restore(grid, ctx.checkpoints[seg])
                    states = []
                    for i in range(end - start):
                        states.append({"phi": st["phi"].clone(), "u": [x.clone() for x in st["u"]]})
                        grid.step_record(st, recs[i])
                    for i in reversed(range(end - start)):
                        grid.adjoint_step_recorded(states[i], recs[i], lam, lam, grad)
                dtype, device = ctx.params_meta
                gparams = torch.tensor([grad[0], grad[1]], dtype=dtype, device=device)
                return (None, None, None, None, gparams, lam["phi"], *lam["u"])

        cls._fn = _F
        return _F


def rollout(grid: Grid, props, phi0, u0: Sequence, sigma, mobility, nsteps: int,
            checkpoint_every: int = 20) -> Tuple:
    """Differentiable ``nsteps``-step rollout.  phi0, u0[a]: float64 device
    tensors of the grid's cell / face shape; sigma, mobility: float64 scalar
    tensors (may require grad).  Returns (phi^N, u_0^N, ..., u_{d-1}^N)."""
    torch = _torch()
    if checkpoint_every < 1:
        raise ValueError("checkpoint_every must be >= 1")
    params = torch.stack([torch.as_tensor(sigma, dtype=torch.float64),
                          torch.as_tensor(mobility, dtype=torch.float64)])
    return CHNSRollout.function().apply(grid, props, int(nsteps), int(checkpoint_every), params, phi0, *u0)
