"""Workload recipes shared by the GPU tests: each side (HIP path and oracle) derives its own
coefficients, time step, sponge, wavelet and kappa from the same seeded synthetic inputs."""
from __future__ import annotations

import math
import os

import numpy as np

import oracle
from paper_1603_03971_amd import synth


def host_threads() -> int:
    """Threads for the oracle's stencil loops: the cores this process may run on (any count gives
    the same bits)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def oracle_forward_problem(v, h, nsteps, src_ijk, fpeak=15.0, rec_ijk=None, sponge_width=16, alpha=0.015,
                           nthreads=None, radius=4, snap_every=0):
    """Oracle run of a forward problem: point sources with the Ricker wavelet."""
    nz, ny, nx = v.shape
    dt = oracle.stable_dt(radius, h, float(np.max(v)))
    kap = oracle.kappa_field(v, dt, h)
    sponge = tuple(oracle.sponge_profile(n, sponge_width, alpha) for n in (nx, ny, nz))
    src_ijk = np.asarray(src_ijk).reshape(-1, 3)
    vs = np.array([v[k, j, i] for i, j, k in src_ijk])
    w = oracle.injection_weight(vs, dt, h)
    amp = np.repeat(oracle.ricker(np.arange(nsteps) * dt, fpeak)[:, None], len(src_ijk), axis=1)
    out = oracle.forward(kap, sponge, nsteps, radius=radius, src_ijk=src_ijk, src_w=w, src_amp=amp, rec_ijk=rec_ijk,
                         nthreads=nthreads or host_threads(), snap_every=snap_every)
    out["dt"] = dt
    return out


def gpu_forward_problem(v, h, nsteps, src_ijk, fpeak=15.0, rec_ijk=None, sponge_width=16, alpha=0.015,
                        schedule="overlap", radius=4, x_align=32, return_prop=False, ghosts="ring", halo="region"):
    """The same problem on the HIP path."""
    import torch

    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    nz, ny, nx = v.shape
    dt = Grid.stable_dt(radius, h, float(np.max(v)))
    g = Grid(nx, ny, nz, h, dt, radius=radius, sponge_width=sponge_width, sponge_alpha=alpha, x_align=x_align)
    kap = g.kappa_from_velocity(v)
    src_ijk = np.asarray(src_ijk).reshape(-1, 3)
    vs = np.array([v[k, j, i] for i, j, k in src_ijk])
    wav = g.ricker(nsteps, fpeak)
    amp = np.repeat(wav[:, None], len(src_ijk), axis=1)
    src = Sources(g, src_ijk, g.injection_weights(vs), amp)
    prop = Propagator(g, kap, sources=src, receivers=rec_ijk, schedule=schedule, ghosts=ghosts, halo=halo)
    traces = prop.new_traces(nsteps)
    prop.run(nsteps, traces)
    torch.cuda.synchronize()
    out = {"u_cur": g.download(prop.u_cur), "u_prv": g.download(prop.u_prv), "traces": traces.cpu().numpy(),
           "dt": dt, "grid": g}
    if return_prop:
        out["prop"] = prop
    return out


def c1_inputs():
    """64^3, h = 10 m, constant 2000 m/s, centre source, 200 steps."""
    n = 64
    v = synth.constant_velocity((n, n, n), 2000.0)
    return v, 10.0, 200, [(32, 32, 32)]


def ragged_inputs(seed=5):
    """Non-tile-multiple box with a layered medium and off-centre sources (several tiles and ragged tails)."""
    shape = (70, 41, 150)   # (nz, ny, nx)
    v = np.array(synth.layered_velocity(shape, 10.0, seed=seed))
    src = [(37, 20, 33), (2, 3, 60), (146, 38, 5)]   # interior source, shell sources
    return v, 10.0, 80, src


def rel_l2(a, b):
    return oracle.rel_l2(a, b)


def plane_standing_wave(nx, ny, nz, h, v, modes):
    kx, ky, kz = (2 * math.pi * m / (n * h) for m, n in zip(modes, (nx, ny, nz)))
    x, y, z = np.arange(nx) * h, np.arange(ny) * h, np.arange(nz) * h
    phase = kx * x[None, None, :] + ky * y[None, :, None] + kz * z[:, None, None]
    return np.cos(phase), (kx, ky, kz)
