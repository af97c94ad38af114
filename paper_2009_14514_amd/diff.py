"""Differentiable WCSPH substeps on the GPU behind torch.autograd.

The forward substeps and their hand-written adjoint run in librts.so
(rts_diff_forward / rts_diff_backward); this module moves torch tensors in
and out as planes and exposes the run as an autograd function of the
initial velocities (and positions), the Tait stiffness B and the viscosity
alpha.
"""
from __future__ import annotations

import numpy as np

from . import _rts
from .sim import Simulation


def _torch():
    import torch
    return torch


def _planes(t):
    """(n, 3) float32 tensor -> contiguous planes x[n], y[n], z[n]."""
    return t.detach().to(_torch().float32).t().contiguous()


def _unplanes(t, n):
    return t.view(3, n).t().contiguous()


class DiffRollout:
    """n_sub substeps of the differentiable WCSPH step on one scene's walls
    and grid, with checkpoints every ckpt_every substeps."""

    def __init__(self, scene, n_sub=16, ckpt_every=4, list_cap=448, dt=None):
        torch = _torch()
        self.sim = Simulation(scene)          # context, walls and grid; its state is scratch
        self.n = scene.n
        self.n_sub, self.ckpt_every, self.list_cap = n_sub, ckpt_every, list_cap
        self.dt = float(dt if dt is not None else scene.params.get("diff_dt", 1e-4))
        self.B0 = float(self.sim.info["B"])
        self.alpha0 = float(scene.params["visc_alpha"])
        desc = self.desc(self.B0, self.alpha0)
        nbytes = _rts.diff_tape_bytes(self.sim.ctx, desc, self.n)
        self.tape = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.sim.device)
        addr = self.tape.data_ptr()
        self.tape_ptr = addr + (-addr) % 256
        self.tape_bytes = nbytes
        self._last = None
        self.generation = 0       # forward runs so far: the tape holds the last one only

    def desc(self, B, alpha):
        return _rts.diff_desc(self.n_sub, self.ckpt_every, self.list_cap, self.dt, B, alpha)

    def forward(self, x0, v0, B, alpha):
        """x0, v0: (n, 3) CUDA tensors; returns x(T), v(T) as (n, 3) float32."""
        torch = _torch()
        n = self.n
        px, pv = _planes(x0), _planes(v0)
        xT = torch.empty(3 * n, dtype=torch.float32, device=self.sim.device)
        vT = torch.empty_like(xT)
        d = self.desc(B, alpha)
        _rts.diff_forward(self.sim.ctx, d, n, px.data_ptr(), pv.data_ptr(), xT.data_ptr(),
                          vT.data_ptr(), self.tape_ptr, self.tape_bytes)
        self.sim.sync(raise_on_error=True)
        self._last = (float(B), float(alpha))
        self.generation += 1
        return _unplanes(xT, n), _unplanes(vT, n)

    def backward(self, xT_bar, vT_bar=None):
        """Adjoint of the last forward run: (dL/dx0, dL/dv0, dL/dB, dL/dalpha)."""
        torch = _torch()
        if self._last is None:
            raise RuntimeError("backward needs a forward run first")
        n = self.n
        gx = torch.empty(3 * n, dtype=torch.float32, device=self.sim.device)
        gv = torch.empty_like(gx)
        pxb = _planes(xT_bar)
        pvb = _planes(vT_bar) if vT_bar is not None else None
        d = self.desc(*self._last)
        gB, ga = _rts.diff_backward(self.sim.ctx, d, n, pxb.data_ptr(),
                                    pvb.data_ptr() if pvb is not None else 0, gx.data_ptr(),
                                    gv.data_ptr(), self.tape_ptr, self.tape_bytes)
        return _unplanes(gx, n), _unplanes(gv, n), gB, ga

    def close(self):
        self.sim.close()


def rollout_function():
    """torch.autograd.Function: (x0, v0, B, alpha, rollout) -> x(T)."""
    torch = _torch()

    class WCSPHRollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x0, v0, B, alpha, model):
            xT, _ = model.forward(x0, v0, float(B), float(alpha))
            ctx.model = model
            ctx.generation = model.generation
            ctx.dtypes = (B.dtype, alpha.dtype, B.device)
            return xT

        @staticmethod
        def backward(ctx, g):
            # the rollout keeps one tape: a later forward run on the same
            # rollout has overwritten the checkpoints this backward needs
            if ctx.model.generation != ctx.generation:
                raise RuntimeError("the rollout ran forward again after this call; its tape "
                                   "no longer holds this call's checkpoints (use one "
                                   "DiffRollout per pending backward)")
            gx, gv, gB, ga = ctx.model.backward(g)
            bdt, adt, dev = ctx.dtypes
            return (gx, gv, torch.tensor(gB, dtype=bdt, device=dev),
                    torch.tensor(ga, dtype=adt, device=dev), None)

    return WCSPHRollout
