"""Differentiable runs of the D2Q9 ternary LB step through torch.autograd.

``TernaryLB.apply(h_bottom, kappa, runner)`` advances ``runner.nsteps`` time
steps from the runner's fixed initial state with wetting parameters
``h_bottom`` ([3][nx], the wall below y = 0) and bulk coefficients ``kappa``
([3]) and returns the concentrations C ([3][ny][nx]) of the final state.  Its
backward pass is the hand-written reverse step of libtlb driven through the
checkpoints the forward pass stored every ``runner.every`` (~sqrt(nsteps))
steps; nothing is differentiated by torch itself.

The initial state is fixed when the runner is made (equilibrium populations
of C0 under the wetting parameters given then); the gradients are those of
the run from that state, so they do not include the dependence of the
initial populations on h_bottom or kappa.

A runner holds one checkpoint store and one set of parameters, so only the
most recent ``TernaryLB.apply`` on a runner can be differentiated: a backward
pass of an earlier call raises ``RuntimeError`` instead of returning the
gradients of the later one.

The library works on a stream of the runner's own.  Every call orders it
after torch's current stream on entry and orders torch's current stream
after it on exit, so tensors handed over in either direction are safe to use
without further synchronisation.
"""
from __future__ import annotations

import math

import torch

from . import tlb


class Runner:
    """A tlb_sim with a fixed initial state, a step count and a checkpoint store.

    ``h`` ([2][3][nx], walls only) gives the wetting parameters of both walls for
    the initial state; the top wall keeps them for the whole run, the bottom
    wall takes ``h_bottom`` of each forward call.
    """

    def __init__(self, params, C0, nsteps, every=None, h=None):
        self.stream = torch.cuda.Stream()
        self.sim = tlb.Sim(params, stream=self.stream.cuda_stream)
        self.params = params
        self.nsteps = int(nsteps)
        self.every = int(every) if every else max(1, int(math.ceil(math.sqrt(self.nsteps))))
        self.dtype = torch.float32 if params.prec == tlb.TLB_F32 else torch.float64
        self.nx, self.ny = params.nx, params.ny
        if params.walls_y and h is not None:
            self.sim.set_wetting_both(h)
        self.sim.init_equilibrium(C0)
        with torch.cuda.stream(self.stream):
            self.state0 = torch.empty(self.sim.state_bytes(), dtype=torch.uint8, device="cuda")
            slots = tlb.tlb_checkpoint_slots(self.nsteps, self.every)
            self.ckpt = torch.empty(slots * self.sim.state_bytes(), dtype=torch.uint8, device="cuda")
        tlb.check(tlb.tlb_save_state_dev(self.sim.handle, self.state0.data_ptr()), "tlb_save_state_dev")
        self.sim.synchronize()
        # forward calls made so far; the checkpoints and parameters are those of the last one
        self.generation = 0

    def _enter(self, *tensors):
        """Order the runner's stream after torch's current one; keep ``tensors`` alive for it."""
        self.stream.wait_stream(torch.cuda.current_stream())
        for t in tensors:
            t.record_stream(self.stream)

    def _leave(self):
        torch.cuda.current_stream().wait_stream(self.stream)

    def set_parameters(self, h_bottom, kappa):
        self.sim.set_kappa([float(k) for k in kappa.detach().cpu().tolist()])
        if self.params.walls_y:
            hb = h_bottom.detach().to(device="cuda", dtype=self.dtype).contiguous()
            self._enter(hb)
            tlb.check(tlb.tlb_set_wetting_dev(self.sim.handle, 0, hb.data_ptr()), "tlb_set_wetting_dev")
            self._leave()

    def forward(self):
        self.generation += 1
        C = torch.empty((3, self.ny, self.nx), dtype=self.dtype, device="cuda")
        self._enter(C)
        tlb.check(tlb.tlb_load_state_dev(self.sim.handle, self.state0.data_ptr(), 0), "tlb_load_state_dev")
        tlb.check(tlb.tlb_forward_checkpointed(self.sim.handle, self.nsteps, self.every, self.ckpt.data_ptr()),
                  "tlb_forward_checkpointed")
        for m in range(3):
            tlb.check(tlb.tlb_get_field_dev(self.sim.handle, m, C[m].data_ptr()), "tlb_get_field_dev")
        self._leave()
        return C

    def backward(self, dLdC):
        g = dLdC.detach().to(device="cuda", dtype=self.dtype).contiguous()
        dh = torch.zeros((2, 3, self.nx), dtype=torch.float64, device="cuda")
        dk = torch.zeros(3, dtype=torch.float64, device="cuda")
        self._enter(g, dh, dk)
        tlb.check(tlb.tlb_adjoint_backward(self.sim.handle, self.nsteps, self.every, self.ckpt.data_ptr(),
                                           g.data_ptr(), dh.data_ptr(), dk.data_ptr()), "tlb_adjoint_backward")
        self._leave()
        return dh, dk


class TernaryLB(torch.autograd.Function):
    """C_final = TernaryLB.apply(h_bottom, kappa, runner)."""

    @staticmethod
    def forward(ctx, h_bottom, kappa, runner):
        runner.set_parameters(h_bottom, kappa)
        ctx.runner = runner
        out = runner.forward()
        ctx.generation = runner.generation
        ctx.h_meta = (h_bottom.dtype, h_bottom.device)
        ctx.k_meta = (kappa.dtype, kappa.device)
        return out

    @staticmethod
    def backward(ctx, dLdC):
        if ctx.generation != ctx.runner.generation:
            raise RuntimeError("TernaryLB: the runner's checkpoints belong to a later forward call "
                               f"({ctx.runner.generation}, this call was {ctx.generation}); only the most "
                               "recent call on a runner can be differentiated")
        dh, dk = ctx.runner.backward(dLdC)
        return (dh[0].to(dtype=ctx.h_meta[0], device=ctx.h_meta[1]),
                dk.to(dtype=ctx.k_meta[0], device=ctx.k_meta[1]), None)
