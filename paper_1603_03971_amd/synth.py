"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module holds only input generation: velocity models, acquisition geometry and random test
signals.  It contains none of the propagator's arithmetic (no stencil weights, time step, sponge,
wavelet or material coefficient) and imports nothing else from the package, so the CPU oracle and
the HIP path can both be fed from it without sharing any of the method.

All generators use numpy's PCG64 (``default_rng``) and FP64, and return arrays of shape
(nz, ny, nx) with x fastest; grid index (i, j, k) is depth-ordered with k = 0 at the surface.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import gaussian_filter, gaussian_filter1d


def constant_velocity(shape, v: float = 2000.0) -> np.ndarray:
    """Homogeneous medium (the 64^3 point-source workload uses v = 2000 m/s)."""
    return np.full(shape, float(v))


def layered_profile(nz: int, h: float, seed: int, n_layers: int = 20, vmin: float = 1500.0,
                    vmax: float = 4500.0, sigma: float = 3.0) -> np.ndarray:
    """1-D velocity-versus-depth profile of `n_layers` flat layers.

    n_layers - 1 interface depths are drawn uniformly on (0, nz h) and sorted; each layer velocity is
    uniform on [vmin, vmax]; the profile is Gaussian-smoothed with `sigma` cells (mode "nearest")
    and clipped to [vmin, vmax]."""
    rng = np.random.default_rng(seed)
    depths = np.sort(rng.uniform(0.0, nz * h, n_layers - 1))
    vels = rng.uniform(vmin, vmax, n_layers)
    z = np.arange(nz) * h
    layer = np.searchsorted(depths, z, side="right")
    prof = vels[layer]
    if sigma > 0:
        prof = gaussian_filter1d(prof, sigma, mode="nearest")
    return np.clip(prof, vmin, vmax)


def layered_velocity(shape, h: float, seed: int, **kw) -> np.ndarray:
    """Flat layers along z (the 512^3 forward workload: seed 2, 20 layers, 1500-4500 m/s, sigma 3).

    The layers are uniform in x and y, so smoothing the 3-D block equals smoothing the depth profile;
    the result is returned as a read-only broadcast view of that profile."""
    nz, ny, nx = shape
    prof = layered_profile(nz, h, seed, **kw)
    return np.broadcast_to(prof[:, None, None], (nz, ny, nx))


def smooth(v: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian smoothing of a 3-D model (mode "nearest")."""
    return gaussian_filter(np.asarray(v, dtype=np.float64), sigma, mode="nearest")


def dipping_reflector_model(shape, h: float, seed: int, n_planes: int = 3, v0: float = 1500.0,
                            gradient: float = 0.75, z0_cells=(60, 150), max_dip_deg: float = 15.0,
                            thickness_cells: int = 2, dv_range=(200.0, 400.0)):
    """Smooth background v(z) = v0 + gradient * depth plus `n_planes` thin dipping reflectors.

    Each reflector is the set of cells within thickness/2 of the plane z = z0 + a x + b y (cells),
    with z0 uniform in `z0_cells`, dip uniform in [0, max_dip], azimuth uniform, and a velocity jump
    of random sign and magnitude uniform in `dv_range`.  Returns (v_true, v_background)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    zc = np.arange(nz, dtype=np.float64)
    v_bg = v0 + gradient * zc * h
    v_bg3 = np.broadcast_to(v_bg[:, None, None], shape)
    v_true = np.array(v_bg3, dtype=np.float64)
    xs = np.arange(nx, dtype=np.float64)[None, :] - nx / 2
    ys = np.arange(ny, dtype=np.float64)[:, None] - ny / 2
    for _ in range(n_planes):
        z0 = rng.uniform(*z0_cells)
        dip = math.radians(rng.uniform(0.0, max_dip_deg))
        az = rng.uniform(0.0, 2 * math.pi)
        dv = rng.uniform(*dv_range) * (1.0 if rng.uniform() < 0.5 else -1.0)
        a = math.tan(dip) * math.cos(az)
        b = math.tan(dip) * math.sin(az)
        zplane = z0 + a * xs + b * ys                       # (ny, nx), in cells
        half = thickness_cells / 2.0
        mask = np.abs(zc[:, None, None] - zplane[None, :, :]) < half
        v_true[mask] += dv
    return v_true, np.array(v_bg3)


def random_smooth_velocity(shape, seed: int, vmin: float = 1500.0, vmax: float = 4500.0,
                           sigma: float = 4.0) -> np.ndarray:
    """Random heterogeneous medium: white noise smoothed with `sigma` cells, rescaled to [vmin, vmax]."""
    rng = np.random.default_rng(seed)
    f = gaussian_filter(rng.standard_normal(shape), sigma, mode="wrap")
    f = (f - f.min()) / max(f.max() - f.min(), 1e-30)
    return vmin + (vmax - vmin) * f


def surface_receivers(nx: int, ny: int, k: int, stride: int = 2, count_x: int | None = None,
                      count_y: int | None = None) -> np.ndarray:
    """Receiver grid at depth index k: (stride a, stride b, k), a < count_x, b < count_y.
    Returns an (n, 3) int64 array of (i, j, k)."""
    cx = count_x if count_x is not None else (nx + stride - 1) // stride
    cy = count_y if count_y is not None else (ny + stride - 1) // stride
    a, b = np.meshgrid(np.arange(cx) * stride, np.arange(cy) * stride, indexing="xy")
    ijk = np.stack([a.ravel(), b.ravel(), np.full(a.size, k)], axis=1).astype(np.int64)
    return ijk[(ijk[:, 0] < nx) & (ijk[:, 1] < ny)]


def random_positions(n: int, nx: int, ny: int, k: int, seed: int, margin: int = 0) -> np.ndarray:
    """`n` seeded (i, j, k) positions with i, j uniform in [margin, n - margin)."""
    rng = np.random.default_rng(seed)
    i = rng.integers(margin, nx - margin, n)
    j = rng.integers(margin, ny - margin, n)
    return np.stack([i, j, np.full(n, k)], axis=1).astype(np.int64)


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Standard-normal test field (FP64)."""
    return scale * np.random.default_rng(seed).standard_normal(shape)
