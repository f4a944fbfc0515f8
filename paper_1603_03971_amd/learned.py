"""Learned dispersion corrector for a coarse grid.

A fine grid (spacing h, radius-4 stencil, step dt) is shadowed by a coarse grid with spacing 2h, the
radius-2 stencil and step 2dt: eight times fewer cells and half the steps, so a coarse step is about
16x cheaper per unit of simulated time, at the price of numerical dispersion (mostly temporal at
twice the step).  Every K coarse steps a three-layer 3-D CNN maps the normalised coarse state
(u^n / s and (u^n - u^{n-1}) / s, each also times a velocity channel) to corrections of the same two
quantities that move the coarse state towards the fine solution restricted to the coarse grid
(s = max |u^n|).  The network runs in
the library's BF16 MFMA kernels with FP32 accumulation and is trained on the device with Adam on
fine/coarse window pairs from seeded random velocity models; its gradients are checked against
an FP64 reference in the tests.

Coarse level n corresponds to fine level 2n.  The coarse sponge is half as wide in cells with
alpha scaled by 2 sqrt(2), so that one coarse step damps like two fine steps at the same distance.
"""
from __future__ import annotations

import math
import time
from dataclasses import asdict, dataclass, replace

import numpy as np
import torch

from . import _abi, synth
from .grid import Grid
from .propagator import Propagator, Sources, tune_grid

C = 16                          # channels of every layer
TAPS = 27
WEIGHTS = TAPS * C * C          # BF16 weights of one layer, [tap][out][in]
LAYER = WEIGHTS + C             # parameters of one layer (weights, then FP32 bias)
NPARAM = 3 * LAYER
IN_CHANNELS = 4                 # a = u^n / s, d = (u^n - u^{n-1}) / s, m a, m d with m = (v - V_REF) / V_SCALE
OUT_CHANNELS = 2                # corrections of a and d
V_REF, V_SCALE = 2250.0, 750.0
RESTRICT = _abi.RTM_RESTRICT_FULL   # fine -> coarse references by full weighting


def _cur():
    return torch.cuda.current_stream()


# -------------------------------------------------------------------------------------------------
# Coarse grid
# -------------------------------------------------------------------------------------------------
def coarse_grid(fine: Grid, radius: int = 2) -> Grid:
    """The coarse companion of `fine`: half the cells per axis, spacing 2h, step 2dt, radius 2 (or 4).
    Its Courant number v (2dt) / (2h) equals the fine one, which is below the radius-4 limit and
    hence below the larger radius-2 limit, so the coarse grid is stable whenever the fine one is."""
    if fine.nx % 2 or fine.ny % 2 or fine.nz % 2:
        raise ValueError("fine grid dimensions must be even")
    if fine.radius != 4:
        raise ValueError("the fine grid uses the radius-4 stencil")
    if radius not in (2, 4):
        raise ValueError("coarse radius 2 or 4")
    g = Grid(fine.nx // 2, fine.ny // 2, fine.nz // 2, 2.0 * fine.h, 2.0 * fine.dt, radius=radius,
             sponge_width=max(fine.sponge_width // 2, 1), sponge_alpha=fine.sponge_alpha * 2.0 * math.sqrt(2.0),
             device=fine.device)
    return g


def plain_grid(fine: Grid, spacing: int, radius: int, step: int) -> Grid:
    """A plain (uncorrected) solver for the time-versus-error comparison: spacing `spacing` h (1 or 2),
    stencil radius 2 or 4, time step `step` dt (1 or 2).  On the 2h grid the sponge is W/2 cells
    with alpha 2 sqrt(step): one step then damps, at the same distance, like `step` fine steps
    (exp(-(alpha_c d/2)^2) = exp(-step (alpha d)^2)).  Every combination keeps the Courant number at
    or below the fine one, so each is stable when the fine grid is."""
    if spacing not in (1, 2) or step not in (1, 2) or radius not in (2, 4):
        raise ValueError("spacing and step must be 1 or 2, radius 2 or 4")
    if spacing == 1:
        return Grid(fine.nx, fine.ny, fine.nz, fine.h, step * fine.dt, radius=radius,
                    sponge_width=fine.sponge_width, sponge_alpha=fine.sponge_alpha * math.sqrt(step),
                    device=fine.device)
    if fine.nx % 2 or fine.ny % 2 or fine.nz % 2:
        raise ValueError("fine grid dimensions must be even")
    return Grid(fine.nx // 2, fine.ny // 2, fine.nz // 2, 2.0 * fine.h, step * fine.dt, radius=radius,
                sponge_width=max(fine.sponge_width // 2, 1), sponge_alpha=fine.sponge_alpha * 2.0 * math.sqrt(step),
                device=fine.device)


def coarse_velocity(v_fine: np.ndarray) -> np.ndarray:
    """Velocity on the coarse grid: the fine model sampled at the coincident cells (2i, 2j, 2k)."""
    return np.ascontiguousarray(np.asarray(v_fine, dtype=np.float32)[::2, ::2, ::2])


def injection_mask(grid, cells, r0: float = 2.0, width: float = 3.0) -> np.ndarray:
    """Compact FP32 (nz, ny, nx) weight of the correction: 0 within r0 cells of any injection cell
    and inside the absorbing sponge, rising linearly over the next `width` cells, 1 elsewhere.  Near
    a point source or a receiver plane the coarse grid cannot carry the fine grid's near field, and
    in the sponge the two grids' absorbing layers differ; correcting either would only launch
    spurious waves, so the corrector is neither trained nor applied there."""
    from scipy.ndimage import distance_transform_edt

    ijk = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    # grid: a Grid, or any object with .shape (nz, ny, nx) and .sponge_width
    hit = np.zeros(grid.shape, dtype=bool)
    hit[ijk[:, 2], ijk[:, 1], ijk[:, 0]] = True
    dist = distance_transform_edt(~hit)
    m = np.clip((dist - r0) / width, 0.0, 1.0)
    W = grid.sponge_width
    for axis, n in enumerate(grid.shape):
        i = np.arange(n)
        edge = np.minimum(i, n - 1 - i).astype(np.float64)
        ramp = np.clip((edge - W + 1) / width, 0.0, 1.0)
        shape = [1, 1, 1]
        shape[axis] = n
        m = m * ramp.reshape(shape)
    return m.astype(np.float32)


# -------------------------------------------------------------------------------------------------
# Network parameters and workspaces
# -------------------------------------------------------------------------------------------------
class CorrectorNet:
    """Three 3x3x3 convolution layers with 16 channels, ReLU after the first two.  FP32 master
    parameters with a BF16 copy of the weights for the kernels; Adam moments; gradients.

    bias=False (the default) keeps the biases at zero: the network is then positively homogeneous,
    net(c x) = c net(x) for c > 0, and maps a zero state to a zero correction, so the correction of a
    quiet region is exactly zero and does not depend on the normalising scale s.  relu=False drops
    the two ReLUs: the network is then linear in its inputs, as the exact correction of a linear
    wave equation is."""

    def __init__(self, seed: int = 0, device="cuda", out_init: float = 0.01, bias: bool = False, relu: bool = True):
        rng = np.random.default_rng(seed)
        p = np.zeros(NPARAM, dtype=np.float32)
        fan = (TAPS * IN_CHANNELS, TAPS * C, TAPS * C)
        for layer in range(3):
            w = np.zeros((TAPS, C, C), dtype=np.float32)
            if layer == 0:
                w[:, :, :IN_CHANNELS] = rng.standard_normal((TAPS, C, IN_CHANNELS)) * math.sqrt(2.0 / fan[0])
            elif layer == 1:
                w[:] = rng.standard_normal((TAPS, C, C)) * math.sqrt(2.0 / fan[1])
            else:
                w[:, :OUT_CHANNELS, :] = rng.standard_normal((TAPS, OUT_CHANNELS, C)) * math.sqrt(1.0 / fan[2]) * out_init
            p[layer * LAYER:layer * LAYER + WEIGHTS] = w.ravel()
        self.device = torch.device(device)
        self.p = torch.from_numpy(p).to(self.device)
        self.p16 = torch.empty(NPARAM, dtype=torch.int16, device=self.device)
        self.grad = torch.zeros_like(self.p)
        self.m1 = torch.zeros_like(self.p)
        self.m2 = torch.zeros_like(self.p)
        self.steps = 0
        self.use_bias = bool(bias)
        self.relu = bool(relu)          # False: a linear network (a learned 7^3 stencil in the inputs)
        self._db_sink = torch.zeros(C, dtype=torch.float32, device=self.device)
        self.sync_bf16()

    def sync_bf16(self, stream=None):
        _abi.rtm_cnn_to_bf16(self.p, self.p16, NPARAM, stream if stream is not None else _cur())

    def w16(self, layer: int) -> torch.Tensor:
        return self.p16[layer * LAYER:layer * LAYER + WEIGHTS]

    def bias(self, layer: int) -> torch.Tensor | None:
        return self.p[layer * LAYER + WEIGHTS:(layer + 1) * LAYER] if self.use_bias else None

    def dw(self, layer: int) -> torch.Tensor:
        return self.grad[layer * LAYER:layer * LAYER + WEIGHTS]

    def db(self, layer: int) -> torch.Tensor:
        """Where the bias gradient goes (a discarded buffer when the biases are off)."""
        return self.grad[layer * LAYER + WEIGHTS:(layer + 1) * LAYER] if self.use_bias else self._db_sink

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        self.steps += 1
        _abi.rtm_cnn_adam(self.p, self.grad, self.m1, self.m2, NPARAM, lr, beta1, beta2, eps, self.steps, self.p16,
                          stream if stream is not None else _cur())

    def layers_host(self):
        """[(w [27, 16, 16], b [16])] as FP64 host arrays of the FP32 master parameters."""
        p = self.p.cpu().numpy().astype(np.float64)
        return [(p[l * LAYER:l * LAYER + WEIGHTS].reshape(TAPS, C, C), p[l * LAYER + WEIGHTS:(l + 1) * LAYER])
                for l in range(3)]

    def state(self) -> np.ndarray:
        return self.p.cpu().numpy().copy()

    def load(self, params: np.ndarray):
        self.p.copy_(torch.from_numpy(np.asarray(params, dtype=np.float32)).to(self.device))
        self.sync_bf16()


class Workspace:
    """Activation buffers for one nx * ny * nz volume.  BF16 volumes carry a one-voxel zero halo
    (written once, here); compact FP32 volumes hold the values the backward pass needs.  A fused
    workspace (inference through the fused first and last layers) has no input or output volume."""

    def __init__(self, nx: int, ny: int, nz: int, train: bool = False, device="cuda", fused: bool = False):
        if nx % 16:
            raise ValueError("the network volume needs nx % 16 == 0")
        if fused and train:
            raise ValueError("a training workspace keeps the input and output volumes")
        self.dims = (int(nx), int(ny), int(nz))
        dev = torch.device(device)
        npad = (nx + 2) * (ny + 2) * (nz + 2) * C
        n = nx * ny * nz * C
        self.x = None if fused else torch.zeros(npad, dtype=torch.int16, device=dev)
        self.h1 = torch.zeros(npad, dtype=torch.int16, device=dev)
        self.h2 = torch.zeros(npad, dtype=torch.int16, device=dev)
        # FP32 output: all 16 channels for training (the loss kernels read that layout), only the two
        # correction channels for inference
        self.out = None if fused else \
            torch.zeros(n if train else nx * ny * nz * OUT_CHANNELS, dtype=torch.float32, device=dev)
        self.out_channels = C if train else OUT_CHANNELS
        self.train = train
        if train:
            self.h1f = torch.zeros(n, dtype=torch.float32, device=dev)
            self.h2f = torch.zeros(n, dtype=torch.float32, device=dev)
            self.target = torch.zeros(n, dtype=torch.float32, device=dev)
            self.dz = torch.zeros(n, dtype=torch.float32, device=dev)
            self.dz16 = torch.zeros(npad, dtype=torch.int16, device=dev)
            self.dh = torch.zeros(n, dtype=torch.float32, device=dev)
            self.wt = torch.zeros(WEIGHTS, dtype=torch.int16, device=dev)
            self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
            # per-workgroup partial sums of the weight gradient (fixed summation order: a training
            # run is reproducible bit for bit)
            self.wpart = torch.empty(_abi.rtm_cnn_wgrad_partials(nx, ny, nz), dtype=torch.float32, device=dev)


def forward(net: CorrectorNet, ws: Workspace, stream=None):
    """ws.out = net(ws.x): three convolutions, ReLU after the first two."""
    if ws.x is None:
        raise ValueError("a fused workspace has no input volume: the Corrector runs the fused layers")
    st = stream if stream is not None else _cur()
    nx, ny, nz = ws.dims
    keep = ws.train
    r = int(net.relu)
    _abi.rtm_cnn_conv3d(nx, ny, nz, ws.x, net.w16(0), net.bias(0), r, ws.h1f if keep else None, ws.h1, st)
    _abi.rtm_cnn_conv3d(nx, ny, nz, ws.h1, net.w16(1), net.bias(1), r, ws.h2f if keep else None, ws.h2, st)
    _abi.rtm_cnn_conv3d(nx, ny, nz, ws.h2, net.w16(2), net.bias(2), 0, ws.out, None, st, y32_channels=ws.out_channels)


def backward(net: CorrectorNet, ws: Workspace, stream=None, weight: float = 1.0, mask=None):
    """net.grad = dL/dparams for L = weight/2 |out - target|^2 over the two output channels (added
    into ws.loss).  Needs the forward pass of the same input with a training workspace."""
    if not ws.train:
        raise ValueError("backward needs a training workspace")
    st = stream if stream is not None else _cur()
    nx, ny, nz = ws.dims
    with torch.cuda.stream(st):
        net.grad.zero_()
    _abi.rtm_cnn_loss_grad(nx, ny, nz, ws.out, ws.target, OUT_CHANNELS, ws.dz, ws.dz16, ws.loss, st, weight=weight,
                           mask=mask)
    acts16 = (ws.x, ws.h1, ws.h2)
    acts32 = (None, ws.h1f, ws.h2f)
    for layer in (2, 1, 0):
        _abi.rtm_cnn_conv3d_wgrad_ordered(nx, ny, nz, acts16[layer], ws.dz, net.dw(layer), net.db(layer), ws.wpart,
                                          ws.wpart.numel(), st)
        if layer == 0:
            break
        _abi.rtm_cnn_weight_flip(net.w16(layer), ws.wt, st)
        _abi.rtm_cnn_conv3d(nx, ny, nz, ws.dz16, ws.wt, None, 0, ws.dh, None, st)
        _abi.rtm_cnn_relu_backward(nx, ny, nz, acts32[layer], ws.dh, int(net.relu), C, ws.dz, ws.dz16, st)


# -------------------------------------------------------------------------------------------------
# Applying the corrector inside a coarse propagation
# -------------------------------------------------------------------------------------------------
class Corrector:
    """Hook for Propagator.run: every `every` coarse levels, u^n and u^{n-1} get the network's
    correction.  A pinned u^{n-1} (a kept snapshot) is left intact: the propagation continues from a
    corrected copy."""

    def __init__(self, net: CorrectorNet, grid: Grid, velocity, every: int):
        if every < 1:
            raise ValueError("every >= 1")
        self.net, self.g, self.every = net, grid, int(every)
        self.ws = Workspace(grid.nx, grid.ny, grid.nz, device=grid.device, fused=True)
        self.scale = torch.zeros(1, dtype=torch.float32, device=grid.device)
        self.applied = 0
        self.mask = None
        self.set_velocity(velocity)

    def set_velocity(self, velocity):
        """Coarse velocity (owned cells, compact, host array or device tensor) of the model."""
        if not isinstance(velocity, torch.Tensor):
            velocity = torch.from_numpy(np.ascontiguousarray(velocity, dtype=np.float32))
        vel = velocity.to(device=self.g.device, dtype=torch.float32).reshape(-1).contiguous()
        if vel.numel() != self.g.points:
            raise ValueError("velocity must cover the coarse grid's owned cells")
        self.vel = vel

    def set_mask(self, mask):
        """Per-cell weight of the correction (compact, host or device; None for 1 everywhere)."""
        if mask is None:
            self.mask = None
            return
        if not isinstance(mask, torch.Tensor):
            mask = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.float32))
        m = mask.to(device=self.g.device, dtype=torch.float32).reshape(-1).contiguous()
        if m.numel() != self.g.points:
            raise ValueError("mask must cover the coarse grid's owned cells")
        self.mask = m

    def apply(self, prop: Propagator):
        g = self.g
        prop.sync()
        st = _cur()
        if prop.u_prv.data_ptr() in prop.pinned:
            fresh = prop.pool.pop() if prop.pool else g.field(fill=None)
            fresh.copy_(prop.u_prv)
            prop.u_prv = fresh
        _abi.rtm_field_absmax(g.c, prop.u_cur, self.scale, st)
        # the network of `forward`, with the input packing fused into the first layer and the
        # correction applied by the last (bitwise the same as pack, forward, apply)
        net, ws, r = self.net, self.ws, int(self.net.relu)
        _abi.rtm_cnn_conv3d_first(g.c, prop.u_cur, prop.u_prv, self.vel, V_REF, V_SCALE, self.scale, net.w16(0),
                                  net.bias(0), r, ws.h1, st)
        _abi.rtm_cnn_conv3d(g.nx, g.ny, g.nz, ws.h1, net.w16(1), net.bias(1), r, None, ws.h2, st)
        _abi.rtm_cnn_conv3d_apply(g.c, ws.h2, net.w16(2), net.bias(2), 0, prop.u_cur, prop.u_prv, self.scale,
                                  mask=self.mask, stream=st)
        prop.exchange_ghosts(prop.u_cur, st)
        if prop.schedule == "overlap":
            prop.level_stream.wait_stream(st)
        self.applied += 1

    def __call__(self, level: int, prop: Propagator):
        if level % self.every == 0:
            self.apply(prop)


# -------------------------------------------------------------------------------------------------
# Training pairs
# -------------------------------------------------------------------------------------------------
def _field_block(grid: Grid, count: int) -> list[torch.Tensor]:
    """`count` padded fields of `grid` carved out of one allocation, each aligned like Grid.field."""
    buf = torch.zeros(count * grid.total + grid._shift, dtype=torch.float32, device=grid.device)
    return [buf[grid._shift + i * grid.total:grid._shift + (i + 1) * grid.total] for i in range(count)]


class Problem:
    """A seeded random velocity model on the fine grid and its coarse companion, with one of two
    kinds of wave source:

    * "source": a Ricker point source at a seeded interior cell (the source side of RTM);
    * "receivers": a plane of receivers (every coarse cell of a seeded depth) re-injecting, time
      reversed, the traces that a point source in the same model left there (the receiver side of
      RTM: the adjoint propagation of recorded data).

    Every source cell is a coarse cell (even fine indices), so both grids inject at the same place."""

    def __init__(self, fine: Grid, coarse: Grid, seed: int, fpeak: float, kind: str = "source",
                 vmin: float = 1500.0, vmax: float = 3000.0, margin: int | None = None, sigma: float = 10.0):
        if kind not in ("source", "receivers"):
            raise ValueError(kind)
        self.seed, self.kind = int(seed), kind
        # smooth media (correlation length of about 2 sigma fine cells): the coarse grid resolves
        # them, as it does the smooth background velocity that RTM migrates with
        self.v = synth.random_smooth_velocity(fine.shape, seed=seed, vmin=vmin, vmax=vmax, sigma=sigma)
        self.vc = coarse_velocity(self.v)
        rng = np.random.default_rng(seed + 7919)
        m = fine.sponge_width + 8 if margin is None else margin
        lo = np.array([m, m, m]) // 2
        hi = np.array([fine.nx - m, fine.ny - m, fine.nz - m]) // 2
        c = rng.integers(lo, np.maximum(hi, lo + 1))          # coarse source cell
        self.src_c = c.reshape(1, 3)
        self.src_f = 2 * self.src_c
        self.fpeak = float(fpeak)
        if kind == "receivers":
            kr = int(rng.integers(lo[2], hi[2]))              # coarse depth of the receiver plane
            jj, ii = np.meshgrid(np.arange(coarse.ny), np.arange(coarse.nx), indexing="ij")
            self.rec_c = np.stack([ii.ravel(), jj.ravel(), np.full(ii.size, kr)], axis=1).astype(np.int64)
            self.rec_f = 2 * self.rec_c
            self.traces = None                                # fine traces, recorded on first use

    def mask(self, coarse: Grid) -> np.ndarray:
        """injection_mask around this problem's injection cells on the coarse grid."""
        return injection_mask(coarse, self.src_c if self.kind == "source" else self.rec_c)

    def _vel_at(self, v, ijk):
        return np.asarray(v)[ijk[:, 2], ijk[:, 1], ijk[:, 0]]

    def fine_sources(self, fine: Grid, nsteps: int) -> Sources:
        if self.kind == "source":
            w = fine.injection_weights(self._vel_at(self.v, self.src_f))
            return Sources(fine, self.src_f, w, fine.ricker(nsteps, self.fpeak)[:, None])
        self._record(fine, nsteps)
        return Sources(fine, self.rec_f, fine.injection_weights(self._vel_at(self.v, self.rec_f)), self.traces,
                       reverse_time=True)

    def coarse_sources(self, coarse: Grid, nsteps: int) -> Sources:
        if self.kind == "source":
            w = coarse.injection_weights(self._vel_at(self.vc, self.src_c))
            return Sources(coarse, self.src_c, w, coarse.ricker(nsteps, self.fpeak)[:, None])
        if self.traces is None or self.traces.shape[0] != 2 * nsteps:
            raise RuntimeError("the fine traces are recorded by fine_sources first")
        # coarse step n injects what fine step 2n does (coarse samples every other fine row)
        return Sources(coarse, self.rec_c, coarse.injection_weights(self._vel_at(self.vc, self.rec_c)),
                       self.traces[1::2].contiguous(), reverse_time=True)

    def _record(self, fine: Grid, nsteps: int):
        if self.traces is not None and self.traces.shape[0] == nsteps:
            return
        kf = fine.kappa_from_velocity(self.v)
        w = fine.injection_weights(self._vel_at(self.v, self.src_f))
        prop = Propagator(fine, kf, sources=Sources(fine, self.src_f, w, fine.ricker(nsteps, self.fpeak)[:, None]),
                          receivers=self.rec_f, schedule="fused")
        self.traces = prop.new_traces(nsteps)
        prop.run(nsteps, self.traces)


class PairSet:
    """Coarse-grid training windows.  For each model, the fine solution is restricted at coarse
    levels 0, K, 2K, ... (and at the level before each).  A window j is the coarse state at level
    (j+1)K (before any correction there) with the restricted fine state at the same level: four
    padded coarse fields, plus the model's coarse velocity and a loss weight.

    Without `net` the window starts from the restricted fine state at level jK (teacher forcing).
    With `net` the coarse solution runs from level 0 with the network applied at every window
    boundary, so the windows carry the corrected solver's own accumulated error (the inputs the
    network meets when it is used, which one-window training never shows it).

    kinds: the source kind of each model ("source" or "receivers", see Problem), cycled over the
    seeds.  Window weights make every window count by its relative error: w = mean(e) / e with e
    the window's squared correction target, clipped to [0.05, 20]."""

    def __init__(self, fine: Grid, coarse: Grid, every: int, nsteps_coarse: int, fpeak, seeds,
                 skip_windows: int = 1, net: CorrectorNet | None = None, kinds=("source",), progress=None):
        self.fine, self.coarse, self.every = fine, coarse, int(every)
        self.nsteps_c = int(nsteps_coarse) // self.every * self.every
        nwin = self.nsteps_c // self.every
        self.seeds = list(seeds)
        self.skip = int(skip_windows)
        self.per_model = nwin - self.skip
        if self.per_model < 1:
            raise ValueError("no windows left")
        count = len(self.seeds) * self.per_model
        self.fields = _field_block(coarse, 4 * count)        # u_cur, u_prv, ref_cur, ref_prv per window
        self.vel = torch.zeros((len(self.seeds), coarse.points), dtype=torch.float32, device=coarse.device)
        self.mask = torch.ones((len(self.seeds), coarse.points), dtype=torch.float32, device=coarse.device)
        self.model_of = np.repeat(np.arange(len(self.seeds)), self.per_model)
        self._ref = _field_block(coarse, 2 * (nwin + 1))
        self._corr = Corrector(net, coarse, self.vel[0], self.every) if net is not None else None
        fps = list(fpeak) if isinstance(fpeak, (list, tuple, np.ndarray)) else [float(fpeak)] * len(self.seeds)
        if len(fps) != len(self.seeds):
            raise ValueError("one peak frequency per model")
        kinds = list(kinds)
        t0 = time.perf_counter()
        for mi, seed in enumerate(self.seeds):
            self._model(mi, seed, float(fps[mi]), kinds[mi % len(kinds)])
            if progress is not None:
                progress(mi)
        torch.cuda.synchronize()
        self.gen_seconds = time.perf_counter() - t0
        del self._ref, self._corr
        self.weights = self._weights()

    def __len__(self):
        return len(self.model_of)

    def window(self, w: int):
        f = self.fields[4 * w:4 * w + 4]
        return f[0], f[1], f[2], f[3], self.vel[self.model_of[w]]

    def window_mask(self, w: int) -> torch.Tensor:
        return self.mask[self.model_of[w]]

    def _weights(self) -> np.ndarray:
        g = self.coarse
        e = np.zeros(len(self))
        for w in range(len(self)):
            u, _, r, _, _ = self.window(w)
            uo, ro = g.owned(u), g.owned(r)
            smax = float(uo.abs().max())
            m = self.window_mask(w).view(g.shape).double()
            e[w] = float((m * (ro - uo).double() ** 2).sum()) / max(smax, 1e-30) ** 2
        e = np.maximum(e, 1e-30)
        return np.clip(e.mean() / e, 0.05, 20.0)

    def _store(self, w: int, u_cur, u_prv, r_cur, r_prv):
        out = self.fields[4 * w:4 * w + 4]
        for dst, src in zip(out, (u_cur, u_prv, r_cur, r_prv)):
            dst.copy_(src)

    def _model(self, mi: int, seed: int, fpeak: float, kind: str):
        fine, coarse, K = self.fine, self.coarse, self.every
        prob = Problem(fine, coarse, seed, fpeak, kind=kind)
        self.vel[mi].copy_(torch.from_numpy(prob.vc.reshape(-1)))
        self.mask[mi].copy_(torch.from_numpy(prob.mask(coarse).reshape(-1)))
        nwin = self.nsteps_c // K
        ref_cur, ref_prv = self._ref[0::2], self._ref[1::2]
        for r in self._ref:
            r.zero_()
        # restricted fine levels at coarse levels jK (cur) and jK - 1 (prv), j = 0..nwin
        kf = fine.kappa_from_velocity(prob.v)
        pf = Propagator(fine, kf, sources=prob.fine_sources(fine, 2 * self.nsteps_c), schedule="fused")

        def grab(level, p):
            if level % (2 * K) == 0:
                _abi.rtm_restrict(fine.c, coarse.c, p.u_cur, ref_cur[level // (2 * K)], _cur(), mode=RESTRICT)
            if (level + 2) % (2 * K) == 0:
                _abi.rtm_restrict(fine.c, coarse.c, p.u_cur, ref_prv[(level + 2) // (2 * K)], _cur(), mode=RESTRICT)

        pf.run(2 * self.nsteps_c, on_level=grab)
        del kf, pf
        kc = coarse.kappa_from_velocity(prob.vc)
        pc = Propagator(coarse, kc, sources=prob.coarse_sources(coarse, self.nsteps_c), schedule="fused")
        if self._corr is None:
            a, b = coarse.field(), coarse.field()
            for j in range(self.skip, nwin):
                a.copy_(ref_cur[j])
                b.copy_(ref_prv[j])
                pc.set_levels(a, b, j * K)
                pc.run(K)
                self._store(mi * self.per_model + (j - self.skip), pc.u_cur, pc.u_prv, ref_cur[j + 1], ref_prv[j + 1])
                a, b = pc.u_prv, pc.u_cur                     # reuse the two buffers
        else:
            self._corr.set_velocity(self.vel[mi])
            self._corr.set_mask(self.mask[mi])

            def hook(level, p):
                if level % K:
                    return
                j = level // K - 1                            # the window that ends here
                if j >= self.skip:
                    self._store(mi * self.per_model + (j - self.skip), p.u_cur, p.u_prv, ref_cur[j + 1],
                                ref_prv[j + 1])
                self._corr.apply(p)

            pc.run(self.nsteps_c, on_level=hook)


def _windows(pairs):
    sets = pairs if isinstance(pairs, (list, tuple)) else [pairs]
    index = [(s, w) for s in sets for w in range(len(s))]
    return sets[0].coarse, index


def train(net: CorrectorNet, pairs, epochs: int, lr: float = 1e-3, seed: int = 0, lr_final: float | None = None,
          noise: float = 0.0, remove_noise: bool = False, weighted: bool = True, log=None, validate=None):
    """Adam over the windows of one PairSet or a list of them, in a seeded random order; returns the
    mean loss per epoch (normalised by the number of voxels and output channels).  noise > 0 adds
    N(0, noise^2) to the normalised wavefield inputs; with remove_noise the target asks the network to
    take it out again, otherwise the target ignores it.  validate(net) -> float, if given, scores the
    network after every epoch (lower is better) and the parameters of the best epoch are kept."""
    g, index = _windows(pairs)
    ws = Workspace(g.nx, g.ny, g.nz, train=True, device=g.device)
    scale = torch.zeros(1, dtype=torch.float32, device=g.device)
    nbuf = torch.zeros(2 * g.points, dtype=torch.float32, device=g.device) if noise > 0 else None
    gen = torch.Generator(device=g.device)
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    st = _cur()
    hist = []
    best = None
    total = epochs * len(index)
    it = 0
    norm = 1.0 / (g.points * OUT_CHANNELS)
    for ep in range(epochs):
        ws.loss.zero_()
        for w in rng.permutation(len(index)):
            ps, k = index[int(w)]
            u_cur, u_prv, r_cur, r_prv, vel = ps.window(k)
            if nbuf is not None:
                nbuf.normal_(0.0, noise, generator=gen)
            _abi.rtm_field_absmax(g.c, u_cur, scale, st)
            _abi.rtm_cnn_pack_input(g.c, u_cur, u_prv, vel, V_REF, V_SCALE, scale, ws.x, noise=nbuf, stream=st)
            _abi.rtm_cnn_target(g.c, r_cur, r_prv, u_cur, u_prv, scale, ws.target,
                                noise=nbuf if remove_noise else None, stream=st)
            forward(net, ws, st)
            backward(net, ws, st, weight=float(ps.weights[k]) if weighted else 1.0, mask=ps.window_mask(k))
            rate = lr if lr_final is None else lr * (lr_final / lr) ** (it / max(total - 1, 1))
            net.adam(rate, stream=st)
            it += 1
        hist.append(float(ws.loss.item()) * norm / len(index))
        if log is not None:
            log(ep, hist[-1])
        if validate is not None:
            score = float(validate(net))
            if log is not None:
                log(ep, hist[-1], score)
            if best is None or score < best[0]:
                best = (score, ep, net.state())
    if validate is not None and best is not None:
        net.load(best[2])
        net.selected_epoch, net.validation_score = best[1], best[0]
    return hist


def window_loss(net: CorrectorNet, pairs) -> tuple[float, float]:
    """(mean loss with the network, mean loss of a zero correction) over all windows."""
    g, index = _windows(pairs)
    ws = Workspace(g.nx, g.ny, g.nz, train=True, device=g.device)
    scale = torch.zeros(1, dtype=torch.float32, device=g.device)
    st = _cur()
    zero = 0.0
    ws.loss.zero_()
    for ps, k in index:
        u_cur, u_prv, r_cur, r_prv, vel = ps.window(k)
        _abi.rtm_field_absmax(g.c, u_cur, scale, st)
        _abi.rtm_cnn_pack_input(g.c, u_cur, u_prv, vel, V_REF, V_SCALE, scale, ws.x, stream=st)
        _abi.rtm_cnn_target(g.c, r_cur, r_prv, u_cur, u_prv, scale, ws.target, stream=st)
        forward(net, ws, st)
        m = ps.window_mask(k)
        _abi.rtm_cnn_loss_grad(g.nx, g.ny, g.nz, ws.out, ws.target, OUT_CHANNELS, ws.dz, ws.dz16, ws.loss, st,
                               mask=m)
        zero += 0.5 * float(torch.sum(m.double()[:, None] * ws.target.view(-1, C)[:, :OUT_CHANNELS].double() ** 2))
    norm = 1.0 / (g.points * OUT_CHANNELS * len(index))
    return float(ws.loss.item()) * norm, zero * norm


# -------------------------------------------------------------------------------------------------
# Evaluation helpers
# -------------------------------------------------------------------------------------------------
def fine_final_restricted(fine: Grid, coarse: Grid, prob: Problem, nsteps_coarse: int) -> torch.Tensor:
    """The fine solution after 2 * nsteps_coarse steps, restricted to the coarse grid."""
    kf = fine.kappa_from_velocity(prob.v)
    pf = Propagator(fine, kf, sources=prob.fine_sources(fine, 2 * nsteps_coarse), schedule="fused")
    pf.run(2 * nsteps_coarse)
    out = coarse.field()
    _abi.rtm_restrict(fine.c, coarse.c, pf.u_cur, out, _cur(), mode=RESTRICT)
    return out


def coarse_final(coarse: Grid, prob: Problem, nsteps_coarse: int, corrector: Corrector | None = None) -> torch.Tensor:
    """The coarse solution after nsteps_coarse steps, with the corrector applied if given."""
    kc = coarse.kappa_from_velocity(prob.vc)
    if corrector is not None:
        corrector.set_velocity(prob.vc)
        corrector.set_mask(prob.mask(coarse))
    pc = Propagator(coarse, kc, sources=prob.coarse_sources(coarse, nsteps_coarse), schedule="fused")
    pc.run(nsteps_coarse, on_level=corrector)
    return pc.u_cur


# -------------------------------------------------------------------------------------------------
# One-shot RTM on the fine grid, the plain coarse grid and the corrected coarse grid
# -------------------------------------------------------------------------------------------------
def _timed(fn, repeats: int = 1):
    """(result of the last call, best wall time in seconds) of fn() with device syncs around."""
    best, out = math.inf, None
    for _ in range(max(1, repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return out, best


PLAIN_VARIANTS = {
    # name: (spacing factor, radius, step factor)
    "2h_r2_2dt": (2, 2, 2),      # the coarse grid the corrector works on, uncorrected
    "2h_r4_2dt": (2, 4, 2),
    "2h_r2_dt": (2, 2, 1),
    "2h_r4_dt": (2, 4, 1),
    "h_r2_dt": (1, 2, 1),
}


def compare_rtm(fine: Grid, v_true, v_bg, src_f, rec_f, nsteps_f: int, fpeak: float, net: CorrectorNet | None,
                every: int, image_every_f: int = 4, repeats: int = 2, schedule: str = "fused",
                snapshots_fine: str | None = None, log=None, plain_variants=(), prolonged: bool = False,
                coarse_radius: int = 2, tune: bool = True):
    """Migrate one shot on the fine grid (the reference) and on the coarse grid without and with the
    learned corrector.  The recorded data are modelled on the fine grid (d_true in v_true, d_bg in
    v_bg) and decimated in time for the coarse runs; sources and receivers sit on even fine cells,
    i.e. on coarse cells.  Returns a dict of images (host arrays on the coarse grid), relative L2
    errors against the fine image (decimated, and full-weighted; over the whole volume and over the
    target zone below the acquisition plane and outside the sponge), and migration wall times.
    snapshots_fine: None (FP32 levels) or "bf16"/"f16" coded snapshots for the fine run (memory).
    plain_variants: names from PLAIN_VARIANTS, further uncorrected solvers timed and scored the same
    way (an image on the fine spacing is restricted to the coarse grid like the reference), the
    points of a time-versus-error curve on which the corrected coarse solver is placed.
    prolonged: also form the plain and corrected coarse images on the fine grid from prolonged
    coarse wavefields (migrate_prolonged) and score them against the fine image on the fine grid.
    tune: first pick the one-launch call's settings for the fine and the coarse grid's shapes
    (tune_grid), so that every solver is timed with its fastest settings."""
    from . import snapshots as snapcodec
    from .rtm import migrate_shot, model_shot

    say = log if log is not None else (lambda msg: None)

    coarse = coarse_grid(fine, coarse_radius)
    if tune:
        say(f"one-launch step tuned: fine {tune_grid(fine)}, coarse {tune_grid(coarse)}")
    src_f = np.asarray(src_f, dtype=np.int64).reshape(-1, 3)
    rec_f = np.asarray(rec_f, dtype=np.int64).reshape(-1, 3)
    if (src_f % 2).any() or (rec_f % 2).any():
        raise ValueError("sources and receivers must sit on even fine cells")
    if nsteps_f % 2 or image_every_f % 2:
        raise ValueError("even step count and imaging interval")
    nsteps_c = nsteps_f // 2
    kt = fine.kappa_from_velocity(v_true)
    kb = fine.kappa_from_velocity(v_bg)
    vs = np.asarray(v_bg)[src_f[:, 2], src_f[:, 1], src_f[:, 0]]
    wav_f = fine.ricker(nsteps_f, fpeak)
    d_true = model_shot(fine, kt, vs, src_f, wav_f, rec_f, nsteps_f, schedule)
    d_bg = model_shot(fine, kb, vs, src_f, wav_f, rec_f, nsteps_f, schedule)
    del kt
    say("fine data modelled")
    codec = snapcodec.make(snapshots_fine)
    snaps_f = codec(fine) if codec is not None else None
    img_f, t_fine = _timed(lambda: migrate_shot(fine, kb, v_bg, src_f, wav_f, rec_f, d_true, d_bg, nsteps_f,
                                                image_every_f, schedule, snaps_f), repeats)
    say(f"fine migration {t_fine:.3f} s")
    ref_full = fine.download(img_f).astype(np.float64) if prolonged else None
    ref_dec = fine.download(img_f)[::2, ::2, ::2].astype(np.float64)
    fw = coarse.field()
    _abi.rtm_restrict(fine.c, coarse.c, img_f, fw, _cur(), mode=_abi.RTM_RESTRICT_FULL)
    ref_fw = coarse.download(fw).astype(np.float64)
    del img_f, kb

    vbc = coarse_velocity(v_bg)
    kbc = coarse.kappa_from_velocity(vbc)
    src_c, rec_c = src_f // 2, rec_f // 2
    wav_c = coarse.ricker(nsteps_c, fpeak)
    # coarse step n records u^{n+1} at time 2(n+1) dt_f: fine trace row 2n + 1
    dc_true = d_true[1::2].contiguous()
    dc_bg = d_bg[1::2].contiguous()
    out = {"t_fine": t_fine, "ref_decimated": ref_dec, "ref_full_weighted": ref_fw}
    # target zone: below the shallowest source or receiver by 6 coarse cells, outside the sponge
    W = coarse.sponge_width
    zt = int(max(src_c[:, 2].max(), rec_c[:, 2].max())) + 6
    zone = (slice(zt, coarse.nz - W), slice(W, coarse.ny - W), slice(W, coarse.nx - W))
    runs = [("plain", None)]
    if net is not None:
        cf, cb = Corrector(net, coarse, vbc, every), Corrector(net, coarse, vbc, every)
        cf.set_mask(injection_mask(coarse, src_c))
        cb.set_mask(injection_mask(coarse, rec_c))
        runs.append(("learned", (cf, cb)))
    for name, corr in runs:
        img, t = _timed(lambda: migrate_shot(coarse, kbc, vbc, src_c, wav_c, rec_c, dc_true, dc_bg, nsteps_c,
                                             image_every_f // 2, schedule, corrector=corr), repeats)
        im = coarse.download(img).astype(np.float64)
        out[f"t_{name}"] = t
        out[f"img_{name}"] = im
        out[f"err_{name}_decimated"] = float(np.linalg.norm(im - ref_dec) / np.linalg.norm(ref_dec))
        out[f"err_{name}_full_weighted"] = float(np.linalg.norm(im - ref_fw) / np.linalg.norm(ref_fw))
        out[f"err_{name}_zone_decimated"] = float(np.linalg.norm((im - ref_dec)[zone]) / np.linalg.norm(ref_dec[zone]))
        out[f"err_{name}_zone_full_weighted"] = float(np.linalg.norm((im - ref_fw)[zone]) /
                                                      np.linalg.norm(ref_fw[zone]))
        say(f"coarse migration ({name}) {t:.3f} s")
        if prolonged:
            zf = tuple(slice(2 * z.start, 2 * z.stop) for z in zone)
            imgp, tp = _timed(lambda: migrate_prolonged(fine, coarse, kbc, vbc, src_c, wav_c, rec_c, dc_true, dc_bg,
                                                        nsteps_c, image_every_f // 2, schedule, corr), repeats)
            imf = fine.download(imgp).astype(np.float64)
            del imgp
            out[f"t_{name}_prolonged"] = tp
            out[f"err_{name}_prolonged_zone"] = float(np.linalg.norm((imf - ref_full)[zf]) /
                                                      np.linalg.norm(ref_full[zf]))
            out[f"err_{name}_prolonged"] = float(np.linalg.norm(imf - ref_full) / np.linalg.norm(ref_full))
            say(f"coarse migration ({name}) imaged on the fine grid: {tp:.3f} s, target-zone error "
                f"{out[f'err_{name}_prolonged_zone']:.3f}")
    for name in plain_variants:
        spacing, radius, step = PLAIN_VARIANTS[name]
        pg = plain_grid(fine, spacing, radius, step)
        if tune:
            tune_grid(pg)
        vp = coarse_velocity(v_bg) if spacing == 2 else np.ascontiguousarray(v_bg, dtype=np.float32)
        kp = pg.kappa_from_velocity(vp)
        sp, rp = src_f // spacing, rec_f // spacing
        # a step of `step` fine steps records u^{n+1} at fine trace row step (n + 1) - 1
        dp_true = d_true[step - 1::step].contiguous()
        dp_bg = d_bg[step - 1::step].contiguous()
        # on the fine spacing the snapshots take the fine run's format (FP32 ones may not fit)
        sn = codec(pg) if (spacing == 1 and codec is not None) else None
        img, t = _timed(lambda: migrate_shot(pg, kp, vp, sp, pg.ricker(nsteps_f // step, fpeak), rp, dp_true, dp_bg,
                                             nsteps_f // step, image_every_f // step, schedule, sn), repeats)
        if spacing == 1:
            fwp = coarse.field()
            _abi.rtm_restrict(pg.c, coarse.c, img, fwp, _cur(), mode=_abi.RTM_RESTRICT_FULL)
            im_fw = coarse.download(fwp).astype(np.float64)
            im_dec = pg.download(img)[::2, ::2, ::2].astype(np.float64)
            del fwp
        else:
            im_fw = im_dec = pg.download(img).astype(np.float64)
        del img, kp
        out[f"t_{name}"] = t
        out[f"err_{name}_zone_full_weighted"] = float(np.linalg.norm((im_fw - ref_fw)[zone]) /
                                                      np.linalg.norm(ref_fw[zone]))
        out[f"err_{name}_zone_decimated"] = float(np.linalg.norm((im_dec - ref_dec)[zone]) /
                                                  np.linalg.norm(ref_dec[zone]))
        say(f"plain {name}: {t:.3f} s, target-zone error {out[f'err_{name}_zone_full_weighted']:.3f} (full-weighted) "
            f"{out[f'err_{name}_zone_decimated']:.3f} (decimated)")
    return out


def migrate_prolonged(fine: Grid, coarse: Grid, kappa_c, v_c, src_c, wav_c, rec_c, d_true, d_bg, nsteps_c: int,
                      image_every_c: int, schedule: str = "fused", corrector=None) -> torch.Tensor:
    """Migrate on the coarse grid but form the image on the fine one: at each imaging level the coarse
    source snapshot and receiver level are prolonged to the fine grid (rtm_prolong, trilinear) and
    correlated there (rtm_image_accumulate).  Returns the fine image field."""
    from .rtm import ShotImager

    imager = ShotImager(coarse, kappa_c, v_c, src_c, wav_c, rec_c, nsteps_c, image_every_c, schedule, None, corrector)
    snaps = imager.forward()
    image = fine.field()
    fa, fb = fine.field(), fine.field()

    def image_fine(snap, r, st):
        _abi.rtm_prolong(coarse.c, fine.c, snap, fa, st)
        _abi.rtm_prolong(coarse.c, fine.c, r, fb, st)
        _abi.rtm_image_accumulate(fine.c, image, fa, fb, 1.0, st)

    imager.backward(snaps, d_true, d_bg, image_fn=image_fine)
    return image


def time_at_error(points, err: float):
    """Time a plain solver needs for image error `err`, read off the time-versus-error curve of
    plain solvers: `points` are (time, error) pairs; the curve is their lower-left frontier (each
    point faster or more accurate than the ones before), interpolated linearly in log error between
    the two frontier points that bracket `err`.  None when err is below every plain error (no plain
    solver measured reaches it); the fastest time when err is above every plain error."""
    pts = sorted((float(t), float(e)) for t, e in points)
    front = []
    for t, e in pts:
        if not front or e < front[-1][1]:
            front.append((t, e))
    if err >= front[0][1]:
        return front[0][0]
    for (t0, e0), (t1, e1) in zip(front, front[1:]):
        if e1 <= err <= e0:
            if e1 <= 0.0:
                return t1
            w = (math.log(e0) - math.log(err)) / (math.log(e0) - math.log(e1))
            return t0 + w * (t1 - t0)
    return None


# -------------------------------------------------------------------------------------------------
# Trained correctors and the fallback rule
# -------------------------------------------------------------------------------------------------
DEFAULTS = {"every": 16, "fpeak": 15.0, "band": (6.0, 16.0), "relu": False}
TRAIN_H, TRAIN_VMIN, TRAIN_VMAX = 10.0, 1500.0, 3000.0


@dataclass
class CorrectorSpec:
    """What a trained corrector is valid for.  It learned the difference between two particular
    discretisations (fine spacing h and step dt, and their coarse companions) over a range of media
    and frequencies; outside them the plain fine grid is the solver to use."""
    h: float
    dt: float
    vmin: float
    vmax: float
    fp_low: float
    fp_high: float
    every: int
    relu: bool
    coarse_radius: int = 2       # stencil radius of the coarse grid the corrector was trained on
    # the fine grid judges the corrector: the target-zone image error of the corrected coarse shot
    # against the plain fine shot, as measured by `compare` (NaN: never measured), and the largest
    # error at which the corrected coarse grid may stand in for the fine one
    image_error: float = float("nan")
    error_bar: float = 1e-2


def save_corrector(path: str, net: CorrectorNet, spec: CorrectorSpec):
    """Parameters and the validity record in one .npz file (plain arrays, no pickles)."""
    np.savez(path, params=net.state(), **{k: np.asarray(v) for k, v in asdict(spec).items()})


def load_corrector(path: str, device="cuda"):
    """(net, spec) from save_corrector's file; a bare .npy of parameters gives spec None."""
    if path.endswith(".npy"):
        params, spec = np.load(path), None
    else:
        with np.load(path) as f:
            params = f["params"]
            spec = CorrectorSpec(**{k: (f[k].item()) for k in CorrectorSpec.__dataclass_fields__ if k in f})
    net = CorrectorNet(device=device, relu=bool(spec.relu) if spec is not None else DEFAULTS["relu"])
    net.load(params)
    return net, spec


def applicable(spec: CorrectorSpec | None, fine, v, fpeak: float, rtol: float = 1e-6, vslack: float = 0.02):
    """(ok, reason): may this corrector stand in for the fine grid on this problem?  The grid must
    have the trained spacing and step, radius 4 and even sizes whose halves suit the network
    (multiple of 16 along x); the velocities must lie in the trained range (within vslack) and the
    peak frequency in the trained band; and the corrector's measured image error against the fine
    solve must lie within its error bar.  Otherwise the fine grid is used."""
    if spec is None:
        return False, "no validity record"
    if not float(spec.image_error) <= float(spec.error_bar):
        if math.isnan(float(spec.image_error)):
            return False, "the corrector's image error against the fine grid was never measured"
        return False, (f"measured image error {float(spec.image_error):.3g} against the fine grid is above the "
                       f"bar {float(spec.error_bar):.3g}")
    if fine.radius != 4:
        return False, "fine grid radius is not 4"
    if abs(fine.h - spec.h) > rtol * spec.h or abs(fine.dt - spec.dt) > rtol * spec.dt:
        return False, f"spacing/step {fine.h}/{fine.dt:.6g} differ from the trained {spec.h}/{spec.dt:.6g}"
    if fine.nx % 2 or fine.ny % 2 or fine.nz % 2 or (fine.nx // 2) % 16:
        return False, "fine sizes must be even with nx / 2 a multiple of 16"
    vmin, vmax = float(np.min(v)), float(np.max(v))
    if vmin < spec.vmin * (1 - vslack) or vmax > spec.vmax * (1 + vslack):
        return False, f"velocities {vmin:.0f}..{vmax:.0f} m/s outside the trained {spec.vmin:.0f}..{spec.vmax:.0f}"
    if not spec.fp_low <= fpeak <= spec.fp_high:
        return False, f"peak frequency {fpeak} Hz outside the trained {spec.fp_low}..{spec.fp_high} Hz"
    return True, "ok"


def migrate(fine: Grid, v_bg, src_f, rec_f, wavelet_fpeak: float, data_true, data_bg, nsteps_f: int,
            image_every_f: int = 4, corrector=None, schedule: str = "fused"):
    """One-shot RTM of recorded data (device traces sampled on the fine step) with the fallback rule:
    the corrected coarse grid when `corrector` = (net, spec) applies to this problem (and its image
    comes out finite), the plain fine grid otherwise.  Returns {"image": padded field, "grid": the
    grid it lives on, "solver": "coarse+corrector" or "fine", "reason": why}."""
    from .rtm import migrate_shot

    src_f = np.asarray(src_f, dtype=np.int64).reshape(-1, 3)
    rec_f = np.asarray(rec_f, dtype=np.int64).reshape(-1, 3)
    net, spec = corrector if corrector is not None else (None, None)
    ok, reason = applicable(spec, fine, v_bg, wavelet_fpeak)
    if ok and ((src_f % 2).any() or (rec_f % 2).any() or nsteps_f % 2 or image_every_f % 2):
        ok, reason = False, "sources, receivers, step count and imaging interval must be even"
    if ok:
        coarse = coarse_grid(fine, int(spec.coarse_radius))
        vbc = coarse_velocity(v_bg)
        cf, cb = Corrector(net, coarse, vbc, spec.every), Corrector(net, coarse, vbc, spec.every)
        cf.set_mask(injection_mask(coarse, src_f // 2))
        cb.set_mask(injection_mask(coarse, rec_f // 2))
        img = migrate_shot(coarse, coarse.kappa_from_velocity(vbc), vbc, src_f // 2,
                           coarse.ricker(nsteps_f // 2, wavelet_fpeak), rec_f // 2, data_true[1::2].contiguous(),
                           data_bg[1::2].contiguous() if data_bg is not None else None, nsteps_f // 2,
                           image_every_f // 2, schedule, corrector=(cf, cb))
        if bool(torch.isfinite(coarse.owned(img)).all()):
            return {"image": img, "grid": coarse, "solver": "coarse+corrector", "reason": reason}
        reason = "the corrected coarse image is not finite"
    img = migrate_shot(fine, fine.kappa_from_velocity(v_bg), v_bg, src_f, fine.ricker(nsteps_f, wavelet_fpeak), rec_f,
                       data_true, data_bg, nsteps_f, image_every_f, schedule)
    return {"image": img, "grid": fine, "solver": "fine", "reason": reason}


# -------------------------------------------------------------------------------------------------
# Command line: train a corrector, compare RTM shots
# -------------------------------------------------------------------------------------------------


def rollout_validator(fine: Grid, coarse: Grid, every: int, nsteps_coarse: int, band, seeds):
    """A validation score for training: held-out models (seeds outside the training set, alternating
    point-source and receiver-plane problems, peak frequencies across `band`), each rolled out for
    nsteps_coarse corrected coarse steps and compared with its restricted fine solution, where the
    corrector acts (relative L2 weighted by the injection mask).  The fine solutions are computed
    once.  Returns score(net) = the mean of the models' errors."""
    seeds = list(seeds)
    freqs = np.linspace(band[0], band[1], len(seeds)) if len(seeds) > 1 else [0.5 * (band[0] + band[1])]
    probs, refs, masks = [], [], []
    for i, (sd, fp) in enumerate(zip(seeds, freqs)):
        prob = Problem(fine, coarse, sd, float(fp), kind="source" if i % 2 == 0 else "receivers")
        probs.append(prob)
        refs.append(coarse.owned(fine_final_restricted(fine, coarse, prob, nsteps_coarse)).double().clone())
        masks.append(torch.from_numpy(prob.mask(coarse)).to(coarse.device).double())

    def score(net: CorrectorNet) -> float:
        errs = []
        for prob, ref, m in zip(probs, refs, masks):
            corr = Corrector(net, coarse, prob.vc, every)
            u = coarse.owned(coarse_final(coarse, prob, nsteps_coarse, corr)).double()
            errs.append(float(torch.linalg.norm(m * (u - ref)) / torch.linalg.norm(m * ref)))
        return float(np.mean(errs))

    return score


def train_corrector(n: int = 96, models: int = 200, first_seed: int = 5000, every: int = DEFAULTS["every"],
                    fpeak=DEFAULTS["fpeak"], nsteps_coarse: int = 300, epochs: int = 10, lr: float = 1e-3,
                    relu: bool = DEFAULTS["relu"], seed: int = 1, log=None, validation_models: int = 4,
                    coarse_radius: int = 2):
    """Train a corrector on `models` seeded fine/coarse pairs (fine n^3, h = 10 m, v in [1500, 3000]
    m/s, alternating point-source and receiver-plane problems).  fpeak: one peak frequency, or a
    (low, high) band from which each model draws its own (seeded).  With validation_models > 0 the
    epoch whose parameters give the lowest rollout error on that many held-out models is kept
    (rollout_validator).  Returns (net, pairs, losses, spec)."""
    fine = Grid(n, n, n, TRAIN_H, Grid.stable_dt(4, TRAIN_H, TRAIN_VMAX))
    coarse = coarse_grid(fine, coarse_radius)
    band = (float(fpeak[0]), float(fpeak[1])) if isinstance(fpeak, (tuple, list)) else (float(fpeak), float(fpeak))
    if isinstance(fpeak, (tuple, list)):
        fpeak = np.random.default_rng(first_seed).uniform(band[0], band[1], models)
    pairs = PairSet(fine, coarse, every, nsteps_coarse, fpeak, range(first_seed, first_seed + models),
                    kinds=("source", "receivers"))
    net = CorrectorNet(seed=seed, relu=relu)
    validate = rollout_validator(fine, coarse, every, nsteps_coarse, band, seeds=range(7000, 7000 + validation_models)) \
        if validation_models > 0 else None
    hist = train(net, pairs, epochs, lr=lr, lr_final=lr / 5, log=log, validate=validate)
    spec = CorrectorSpec(h=fine.h, dt=fine.dt, vmin=TRAIN_VMIN, vmax=TRAIN_VMAX, fp_low=band[0], fp_high=band[1],
                         every=int(every), relu=bool(relu), coarse_radius=int(coarse_radius))
    return net, pairs, hist, spec


def main(argv=None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train", help="train a corrector and save it with its validity record (.npz)")
    t.add_argument("--n", type=int, default=96)
    t.add_argument("--models", type=int, default=200)
    t.add_argument("--every", type=int, default=DEFAULTS["every"])
    t.add_argument("--fp-band", type=float, nargs=2, default=list(DEFAULTS["band"]), metavar=("LOW", "HIGH"),
                   help="band from which each training model draws its peak frequency")
    t.add_argument("--fp", type=float, default=None, help="one peak frequency for every model instead")
    t.add_argument("--steps", type=int, default=300, help="coarse steps per training model")
    t.add_argument("--epochs", type=int, default=10)
    t.add_argument("--relu", action="store_true")
    t.add_argument("--validation-models", type=int, default=4,
                   help="held-out models whose rollout error selects the epoch (0: keep the last epoch)")
    t.add_argument("--seed", type=int, default=1, help="seed of the initial weights")
    t.add_argument("--coarse-radius", type=int, default=2, choices=[2, 4], help="stencil radius of the coarse grid")
    t.add_argument("--out", required=True)
    c = sub.add_parser("compare", help="one RTM shot: fine vs plain coarse vs corrected coarse")
    c.add_argument("--weights", required=True)
    c.add_argument("--n", type=int, default=96)
    c.add_argument("--steps", type=int, default=600, help="fine steps")
    c.add_argument("--every", type=int, default=DEFAULTS["every"], help="used when the weights carry no record")
    c.add_argument("--fp", type=float, default=DEFAULTS["fpeak"])
    c.add_argument("--relu", action="store_true")
    c.add_argument("--image-every", type=int, default=4, help="fine steps between imaging levels")
    c.add_argument("--snapshots", default=None, help="fine snapshot format: bf16 or f16 (default FP32)")
    c.add_argument("--repeats", type=int, default=2)
    c.add_argument("--plain", nargs="*", default=[], choices=sorted(PLAIN_VARIANTS),
                   help="further plain solvers for the time-versus-error curve")
    c.add_argument("--prolonged", action="store_true",
                   help="also image the coarse runs on the fine grid from prolonged wavefields")
    c.add_argument("--record", default=None,
                   help="save the corrector with the measured target-zone image error in its record (.npz)")
    a = ap.parse_args(argv)

    def say(msg):
        print(msg, flush=True)

    if a.cmd == "train":
        t0 = time.perf_counter()
        def logger(e, loss, score=None):
            say(f"epoch {e}: loss {loss:.4e}" if score is None else f"epoch {e}: held-out rollout error {score:.4f}")

        net, pairs, hist, spec = train_corrector(a.n, a.models, every=a.every,
                                                 fpeak=a.fp if a.fp is not None else tuple(a.fp_band),
                                                 nsteps_coarse=a.steps, epochs=a.epochs, relu=a.relu, seed=a.seed,
                                                 log=logger, validation_models=a.validation_models,
                                                 coarse_radius=a.coarse_radius)
        if getattr(net, "selected_epoch", None) is not None:
            say(f"kept epoch {net.selected_epoch} (held-out rollout error {net.validation_score:.4f})")
        with_net, zero = window_loss(net, pairs)
        save_corrector(a.out, net, spec)
        say(json.dumps({"windows": len(pairs), "generation_s": round(pairs.gen_seconds, 2),
                        "train_s": round(time.perf_counter() - t0, 2), "window_loss": with_net,
                        "window_loss_zero_correction": zero, "out": a.out}))
        return 0
    n = a.n
    fine = Grid(n, n, n, TRAIN_H, Grid.stable_dt(4, TRAIN_H, TRAIN_VMAX))
    net, spec = load_corrector(a.weights)
    if spec is None:
        net = CorrectorNet(relu=a.relu)
        net.load(np.load(a.weights))
    z_ref = (fine.sponge_width + 4) // 2 * 2            # source and receivers just below the sponge
    # reflectors 20 to 60 cells below the shot, shallow enough for the recording time; gentler dips on
    # large models keep them inside that depth range across the whole plane
    v_true, v_bg = synth.dipping_reflector_model(fine.shape, 10.0, seed=3, z0_cells=(z_ref + 20, z_ref + 60),
                                                 max_dip_deg=15.0 if n <= 128 else 3.0)
    rec = synth.surface_receivers(n, n, k=z_ref, stride=2)
    src = [(n // 2 // 2 * 2, n // 2 // 2 * 2, z_ref)]
    every = a.every
    if spec is not None:
        every = spec.every
        ok, why = applicable(spec, fine, v_bg, a.fp)
        say(f"fallback rule: corrector {'applies' if ok else 'does not apply'} ({why})")
    say(f"compare: fine {n}^3, {a.steps} steps, {a.fp} Hz, corrector every {every} coarse steps")
    r = compare_rtm(fine, v_true, v_bg, src, rec, a.steps, a.fp, net, every, image_every_f=a.image_every,
                    repeats=a.repeats, snapshots_fine=a.snapshots, log=say, plain_variants=a.plain,
                    prolonged=a.prolonged, coarse_radius=int(spec.coarse_radius) if spec is not None else 2)
    if a.plain and "err_learned_zone_full_weighted" in r:
        # the plain curve: the fine solve (error 0 by definition), the uncorrected coarse grid, the variants
        pts = [(r["t_fine"], 0.0), (r["t_plain"], r["err_plain_zone_full_weighted"])]
        pts += [(r[f"t_{n}"], r[f"err_{n}_zone_full_weighted"]) for n in a.plain]
        t_eq = time_at_error(pts, r["err_learned_zone_full_weighted"])
        r["plain_time_at_learned_error"] = t_eq
        pts_d = [(r["t_fine"], 0.0), (r["t_plain"], r["err_plain_zone_decimated"])]
        pts_d += [(r[f"t_{n}"], r[f"err_{n}_zone_decimated"]) for n in a.plain]
        t_eq_d = time_at_error(pts_d, r["err_learned_zone_decimated"])
        r["plain_time_at_learned_error_decimated"] = t_eq_d
        say(f"learned: {r['t_learned']:.3f} s at target-zone error {r['err_learned_zone_full_weighted']:.3f} "
            f"(full-weighted), {r['err_learned_zone_decimated']:.3f} (decimated); plain solvers reach those errors "
            f"in {t_eq if t_eq is None else round(t_eq, 3)} s and {t_eq_d if t_eq_d is None else round(t_eq_d, 3)} s")
    say(json.dumps({k: v for k, v in r.items() if not k.startswith(("img", "ref"))}))
    if a.record is not None and spec is not None and "err_learned_zone_full_weighted" in r:
        spec = replace(spec, image_error=float(r["err_learned_zone_full_weighted"]))
        save_corrector(a.record, net, spec)
        ok, why = applicable(spec, fine, v_bg, a.fp)
        say(f"recorded image error {spec.image_error:.4g} in {a.record}; fallback rule now: "
            f"{'corrected coarse grid' if ok else 'fine grid'} ({why})")
    return 0


if __name__ == "__main__":
    import sys

    sys.exit(main())
