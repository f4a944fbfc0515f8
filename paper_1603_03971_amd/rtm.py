"""One-shot reverse time migration on the device.

Forward: model the source wavefield u and keep u^k at the imaging levels k in
T = {k in 1..N : k % s == 0}.  A kept level is simply a pinned time-level buffer, so keeping it costs
no copy (the time levels rotate by pointer).  Backward: propagate the receiver wavefield r with the
same update in reverse time, injecting the time-reversed residual traces at the receivers
(r^{m+1} = update(r^m, r^{m-1}) + sum_r w_r d^{N-1-m}_r); r^{m+1} is the receiver wavefield at
forward level k = N - m.  Image: the zero-lag cross-correlation I = sum_{k in T} u^k r^{N+1-k}
(Claerbout 1971), accumulated in FP32 by rtm_image_accumulate.

The helpers default to the propagator's one-launch schedule (one GPU, nothing to overlap); every
schedule gives the same bits.

Source and receiver weights are the point-source weights (v dt)^2 / h^3 at their cells.  The
residual d_true - d_bg is injected as two injections (+w d_true, -w d_bg), so no trace arithmetic
happens outside the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _abi
from .grid import Grid
from .propagator import Propagator, Sources


def _cells_velocity(v, ijk):
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    return np.asarray(v)[ijk[:, 2], ijk[:, 1], ijk[:, 0]]


def model_shot(grid: Grid, kappa: torch.Tensor, v_at_src, src_ijk, wavelet, rec_ijk, nsteps: int,
               schedule: str = "fused") -> torch.Tensor:
    """Forward modelling of one shot: traces (nsteps, nrec) on the device."""
    w = grid.injection_weights(v_at_src)
    amp = np.repeat(np.asarray(wavelet, dtype=np.float32)[:nsteps, None], len(w), axis=1)
    prop = Propagator(grid, kappa, sources=Sources(grid, src_ijk, w, amp), receivers=rec_ijk, schedule=schedule)
    traces = prop.new_traces(nsteps)
    prop.run(nsteps, traces)
    return traces


class ShotImager:
    """Forward pass with kept snapshots and backward pass with imaging, for one shot."""

    def __init__(self, grid: Grid, kappa_bg: torch.Tensor, v_bg, src_ijk, wavelet, rec_ijk, nsteps: int,
                 image_every: int = 4, schedule: str = "fused", snapshots=None, corrector=None):
        self.g = grid
        self.kappa = kappa_bg
        self.v_bg = v_bg
        self.src_ijk = np.asarray(src_ijk, dtype=np.int64).reshape(-1, 3)
        self.rec_ijk = np.asarray(rec_ijk, dtype=np.int64).reshape(-1, 3)
        self.wavelet = np.asarray(wavelet, dtype=np.float32)
        self.nsteps = int(nsteps)
        self.s = int(image_every)
        self.schedule = schedule
        self.snapshots = snapshots            # None = FP32 pinned levels, else a snapshot codec
        # optional on_level hook that edits the state (e.g. a learned dispersion correction), run
        # before imaging; one hook for both passes or a (forward, backward) pair
        self.corrector = corrector if isinstance(corrector, (tuple, list)) else (corrector, corrector)

    def forward(self):
        """Source wavefield; returns {k: snapshot} for k in T."""
        g = self.g
        w = g.injection_weights(_cells_velocity(self.v_bg, self.src_ijk))
        amp = np.repeat(self.wavelet[:self.nsteps, None], len(w), axis=1)
        prop = Propagator(g, self.kappa, sources=Sources(g, self.src_ijk, w, amp), schedule=self.schedule)
        snaps = {}

        def keep(k, p):
            if self.corrector[0] is not None:
                self.corrector[0](k, p)
            if k % self.s == 0:
                if self.snapshots is None:
                    snaps[k] = p.pin_current()
                else:
                    snaps[k] = self.snapshots.encode(p.u_cur, p.level_stream)

        prop.run(self.nsteps, on_level=keep)
        return snaps

    def backward(self, snaps, data_true: torch.Tensor, data_bg: torch.Tensor | None = None,
                 image_fn=None) -> torch.Tensor:
        """Receiver wavefield and image.  data_*: device traces (nsteps, nrec) at the receivers.
        image_fn(snapshot, receiver level, stream), if given, replaces the imaging of each pair
        (e.g. to form the image on another grid); the returned field is then left zero."""
        g = self.g
        N = self.nsteps
        wr = g.injection_weights(_cells_velocity(self.v_bg, self.rec_ijk))
        srcs = [Sources(g, self.rec_ijk, wr, data_true, reverse_time=True)]
        if data_bg is not None:
            srcs.append(Sources(g, self.rec_ijk, -wr, data_bg, reverse_time=True))
        prop = Propagator(g, self.kappa, sources=srcs, schedule=self.schedule)
        image = g.field()

        def correlate(level, p):
            if self.corrector[1] is not None:
                self.corrector[1](level, p)
            k = N + 1 - level                 # forward level this receiver level pairs with
            if k in snaps:
                if image_fn is not None:
                    image_fn(snaps[k], p.u_cur, p.level_stream)
                elif self.snapshots is None:
                    _abi.rtm_image_accumulate(g.c, image, snaps[k], p.u_cur, 1.0, p.level_stream)
                else:
                    self.snapshots.image_accumulate(image, snaps[k], p.u_cur, 1.0, p.level_stream)

        prop.run(N, on_level=correlate)
        return image


def migrate_shot(grid: Grid, kappa_bg, v_bg, src_ijk, wavelet, rec_ijk, data_true, data_bg, nsteps: int,
                 image_every: int = 4, schedule: str = "fused", snapshots=None, corrector=None) -> torch.Tensor:
    """Zero-lag RTM image (padded device field) of one shot from its recorded traces."""
    imager = ShotImager(grid, kappa_bg, v_bg, src_ijk, wavelet, rec_ijk, nsteps, image_every, schedule, snapshots,
                        corrector)
    snaps = imager.forward()
    return imager.backward(snaps, data_true, data_bg)


def rtm_shot(grid: Grid, v_true, v_bg, src_ijk, rec_ijk, nsteps: int, fpeak: float = 15.0, image_every: int = 4,
             schedule: str = "fused", snapshots=None):
    """Synthetic one-shot RTM: model d_true and d_bg, migrate the reflection data with the background.
    Returns (image field, d_true, d_bg)."""
    kap_true = grid.kappa_from_velocity(v_true)
    kap_bg = grid.kappa_from_velocity(v_bg)
    wav = grid.ricker(nsteps, fpeak)
    vs = _cells_velocity(v_bg, src_ijk)
    d_true = model_shot(grid, kap_true, vs, src_ijk, wav, rec_ijk, nsteps, schedule)
    d_bg = model_shot(grid, kap_bg, vs, src_ijk, wav, rec_ijk, nsteps, schedule)
    del kap_true
    image = migrate_shot(grid, kap_bg, v_bg, src_ijk, wav, rec_ijk, d_true, d_bg, nsteps, image_every, schedule,
                         snapshots)
    return image, d_true, d_bg
