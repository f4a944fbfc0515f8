"""Differentiable modelling: least-squares misfit of recorded traces and its exact gradient.

For each shot the forward run keeps only checkpoints, the level pairs (u^n, u^{n-1}) at
n = 0, C, 2C, ... (pinned buffers, no copies), and the residual traces r = d - d_obs with
J = 1/2 sum r^2 accumulated in FP64.  The backward pass walks the segments from the last one:
it recomputes the segment's levels from its checkpoint, then runs the transposed recursion
(Tarantola 1984)

    mu^m = 2 g mu^{m+1} + L(kappa g mu^{m+1}) - g^2 mu^{m+2} + R^T r^{m-1},   m = N .. 1,

with mu^{N+1} = mu^{N+2} = 0, and accumulates dJ/dkappa += g mu^m L u^{m-1} (rtm_adjoint_step,
rtm_inject, rtm_gradient_accumulate).  The chain rule through kappa = (v dt / h)^2 gives dJ/dv
(rtm_velocity_gradient).  Injection weights are held at the values of the model they were built
from (the gradient treats them as constants).

By default the recursion runs in scaled form, on the state w = kappa g mu: multiplying the step above
by kappa g turns it into w^m = g (2 w^{m+1} - g w^{m+2} + kappa L w^{m+1}) + kappa g R^T r^{m-1}, the
forward update itself (rtm_step_whole, then rtm_inject with the receiver weights kappa_r g_r from
rtm_scaled_adjoint_factors), so an adjoint step costs one forward step.  The gradient is then
G = sum w^m L u^{m-1} (rtm_gradient_accumulate_scaled) and dJ/dv = 2 G / v
(rtm_velocity_gradient_scaled).  adjoint="direct" runs the mu recursion with rtm_adjoint_step.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _abi
from .grid import Grid
from .propagator import Propagator, Sources

MISFIT_CHUNKS = 1024      # chunks of the residual's FP64 sum (one workgroup each, fixed order)


class Shot:
    """One shot: source cells and weights, receiver cells, observed traces (device, (nsteps, nrec))."""

    def __init__(self, src_ijk, src_w, rec_ijk, observed: torch.Tensor | None = None):
        self.src_ijk = np.asarray(src_ijk, dtype=np.int64).reshape(-1, 3)
        self.src_w = np.asarray(src_w, dtype=np.float32).reshape(-1)
        self.rec_ijk = np.asarray(rec_ijk, dtype=np.int64).reshape(-1, 3)
        self.observed = observed


class MisfitProblem:
    """J(v) = 1/2 sum over shots, steps and receivers of (d - d_obs)^2 on one grid."""

    def __init__(self, grid: Grid, nsteps: int, wavelet, shots: list[Shot], checkpoint_every: int = 50,
                 schedule: str = "fused", adjoint: str = "scaled"):
        """schedule: the propagator schedule of the forward and recomputation runs (all give the
        same bits; the one-launch schedule is the fastest on one GPU).  adjoint: "scaled" (the
        recursion on w = kappa g mu, run by the forward kernel) or "direct" (rtm_adjoint_step on mu);
        the two agree to FP32 rounding."""
        if adjoint not in ("scaled", "direct"):
            raise ValueError(adjoint)
        self.adjoint = adjoint
        self.g = grid
        self.schedule = schedule
        self.nsteps = int(nsteps)
        self.wavelet = np.asarray(wavelet, dtype=np.float32)[:nsteps]
        self.shots = shots
        self.C = int(checkpoint_every)
        self._work = None

    # ------------------------------------------------------------------------------------------
    def kappa(self, v: torch.Tensor) -> torch.Tensor:
        return self.g.kappa_from_velocity(v)

    def _sources(self, shot: Shot, amp=None):
        amp = np.repeat(self.wavelet[:, None], len(shot.src_w), axis=1) if amp is None else amp
        return Sources(self.g, shot.src_ijk, shot.src_w, amp)

    def model(self, kappa: torch.Tensor, shot: Shot, amp=None) -> torch.Tensor:
        """Traces of one shot (device (nsteps, nrec)); amp overrides the source series."""
        prop = Propagator(self.g, kappa, sources=self._sources(shot, amp), receivers=shot.rec_ijk,
                          schedule=self.schedule)
        tr = prop.new_traces(self.nsteps)
        prop.run(self.nsteps, tr)
        return tr

    def _residual(self, tr: torch.Tensor, shot: Shot, resid: torch.Tensor, misfit: torch.Tensor):
        """resid = traces - observed, misfit += 1/2 |resid|^2 summed in FP64 over MISFIT_CHUNKS chunks
        of the samples in a fixed order (the same bits on every call)."""
        if getattr(self, "_partials", None) is None:
            self._partials = torch.empty(MISFIT_CHUNKS, dtype=torch.float64, device=self.g.device)
        _abi.rtm_misfit_residual_chunks(tr, shot.observed, resid, tr.numel(), self._partials, MISFIT_CHUNKS, misfit,
                                        torch.cuda.current_stream())

    def forward(self, kappa: torch.Tensor, shot: Shot, misfit: torch.Tensor):
        """Forward run with checkpoints; returns (checkpoints {n: (u^n, u^{n-1})}, residual traces)."""
        g = self.g
        prop = Propagator(g, kappa, sources=self._sources(shot), receivers=shot.rec_ijk, schedule=self.schedule)
        tr = prop.new_traces(self.nsteps)
        ckpt = {}
        for n in range(self.nsteps):
            if n % self.C == 0:
                ckpt[n] = (prop.pin_current(), prop.pin_previous())
            prop.step(tr)
        prop.sync()
        resid = torch.empty_like(tr)
        self._residual(tr, shot, resid, misfit)
        return ckpt, resid

    def backward(self, kappa: torch.Tensor, shot: Shot, ckpt, resid: torch.Tensor, grad_kappa: torch.Tensor,
                 y_src: torch.Tensor | None = None):
        """Adjoint pass of one shot; adds its gradient term to grad_kappa (dJ/dkappa, or in the scaled
        form G = kappa dJ/dkappa).  With y_src (device (nsteps, nsrc)), also records the source-side
        adjoint state mu^{n+1}[s] into it."""
        g, N, C = self.g, self.nsteps, self.C
        st = torch.cuda.current_stream()
        scaled = self.adjoint == "scaled"
        if self._work is None and not scaled:
            self._work = g.field()
        work = self._work
        nrec, nsrc = len(shot.rec_ijk), len(shot.src_ijk)
        rec_idx = torch.from_numpy(g.index(shot.rec_ijk)).to(g.device)
        src_idx = torch.from_numpy(g.index(shot.src_ijk)).to(g.device)
        if scaled:
            # receiver weights kappa_r g_r, and 1 / (kappa_s g_s) to turn w back into mu at the sources
            rec_w = torch.empty(nrec, dtype=torch.float32, device=g.device)
            src_scale = torch.empty(nsrc, dtype=torch.float32, device=g.device)
            _abi.rtm_scaled_adjoint_factors(g.c, kappa, rec_idx, nrec, rec_w, None, st)
            _abi.rtm_scaled_adjoint_factors(g.c, kappa, src_idx, nsrc, None, src_scale, st)
        else:
            rec_w = torch.ones(nrec, dtype=torch.float32, device=g.device)
        mu_a, mu_b = g.field(), g.field()           # mu^{m+1}, mu^{m+2} (or w); zero ghost rings
        prop = Propagator(g, kappa, sources=self._sources(shot), schedule=self.schedule)
        nseg = (N + C - 1) // C
        for seg in range(nseg - 1, -1, -1):
            n0, n1 = seg * C, min(N, seg * C + C)
            u0, um = ckpt[n0]
            # recompute u^{n0} .. u^{n1-1}
            prop.set_levels(u0, um, n0)
            levels = {n0: u0}
            prop.pinned.add(u0.data_ptr())
            for n in range(n0, n1 - 1):
                prop.step()
                levels[n + 1] = prop.pin_current()
            prop.sync()
            for m in range(n1, n0, -1):
                # mu^m (or w^m) from the two later levels, in place over the older one
                if scaled:
                    _abi.rtm_step_whole(g.c, mu_b, mu_a, mu_b, kappa, st)
                else:
                    _abi.rtm_adjoint_step(g.c, mu_b, mu_a, mu_b, kappa, work, st)
                _abi.rtm_inject(g.c, mu_b, rec_idx, rec_w, resid.data_ptr() + 4 * (m - 1) * nrec, nrec, st)
                if scaled:
                    _abi.rtm_gradient_accumulate_scaled(g.c, grad_kappa, levels[m - 1], mu_b, st)
                else:
                    _abi.rtm_gradient_accumulate(g.c, grad_kappa, levels[m - 1], mu_b, st)
                if y_src is not None:
                    out = y_src.data_ptr() + 4 * (m - 1) * nsrc
                    if scaled:
                        _abi.rtm_record_weighted(g.c, mu_b, src_idx, src_scale, out, nsrc, st)
                    else:
                        _abi.rtm_record(g.c, mu_b, src_idx, out, nsrc, st)
                mu_a, mu_b = mu_b, mu_a
            for t in levels.values():
                prop.unpin(t)
            del ckpt[n0]

    # ------------------------------------------------------------------------------------------
    def misfit_and_gradient(self, v: torch.Tensor):
        """(J as a float, dJ/dv as a compact (nz, ny, nx) device tensor)."""
        g = self.g
        v = v.to(device=g.device, dtype=torch.float32).contiguous()
        kappa = self.kappa(v)
        misfit = torch.zeros(1, dtype=torch.float64, device=g.device)
        grad_k = g.field()
        for shot in self.shots:
            ckpt, resid = self.forward(kappa, shot, misfit)
            self.backward(kappa, shot, ckpt, resid, grad_k)
        gv = torch.empty(g.shape, dtype=torch.float32, device=g.device)
        if self.adjoint == "scaled":
            _abi.rtm_velocity_gradient_scaled(g.c, gv, grad_k, v, torch.cuda.current_stream())
        else:
            _abi.rtm_velocity_gradient(g.c, gv, grad_k, v, g.dt / g.h, torch.cuda.current_stream())
        return float(misfit.item()), gv

    def misfit(self, v: torch.Tensor) -> float:
        g = self.g
        kappa = self.kappa(v.to(device=g.device, dtype=torch.float32).contiguous())
        misfit = torch.zeros(1, dtype=torch.float64, device=g.device)
        for shot in self.shots:
            tr = self.model(kappa, shot)
            resid = torch.empty_like(tr)
            self._residual(tr, shot, resid, misfit)
        return float(misfit.item())


class VelocityMisfit(torch.autograd.Function):
    """J = MisfitProblem misfit of a velocity model; backward gives dJ/dv by the adjoint state."""

    @staticmethod
    def forward(ctx, v: torch.Tensor, problem: MisfitProblem):
        J, gv = problem.misfit_and_gradient(v.detach())
        ctx.save_for_backward(gv)
        return torch.tensor(J, dtype=torch.float64, device=v.device)

    @staticmethod
    def backward(ctx, gJ):
        (gv,) = ctx.saved_tensors
        return (gJ.to(gv.dtype) * gv), None


def velocity_misfit(v: torch.Tensor, problem: MisfitProblem) -> torch.Tensor:
    return VelocityMisfit.apply(v, problem)
