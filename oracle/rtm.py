"""FP64 reference of the RTM hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this module.
It shares no code with the HIP library: the stencil loops live in ``rtm_oracle.c`` (plain C,
FP64, no contraction) and the time loops below follow the method's steps in order.

The method (the paper, section II, "Structure of the Application": a high-order stencil applied to
a 3-D block each time step) is written out here as

* coefficients: Taylor weights of the centred second derivative (Fornberg 1988), radius R;
* Laplacian:    L u = sum over axes of [c0 u + sum_m c_m (u(+m) + u(-m))], dimensionless;
* update:       u^{n+1} = g (2 u^n - g u^{n-1} + kappa L u^n), kappa = (v dt / h)^2;
* sponge:       g = gamma(d_x) gamma(d_y) gamma(d_z), gamma(d) = exp(-(alpha d)^2) (Cerjan 1985);
* source:       after the update, u^{n+1}[s] += w_s f(t_n), w_s = (v_s dt)^2 / h^3, t_n = n dt;
* receivers:    trace[n][r] = u^{n+1}[r];
* wavelet:      Ricker, f(t) = (1 - 2 pi^2 fp^2 tau^2) exp(-pi^2 fp^2 tau^2), tau = t - t0;
* RTM:          back-propagate the data with the same update in reverse time and form the
                zero-lag cross-correlation image I = sum_k u^k R^k (Claerbout 1971);
* adjoint:      the exact transpose of the recursion above (Tarantola 1984) and the
                adjoint-state gradient of the least-squares misfit with respect to kappa.

Arrays are numpy float64 of shape (nz, ny, nx) (x fastest).  Where the sponge acts is pinned in
closed form (with kappa = 0 each cell obeys a scalar recurrence with the double root g; with
constant g and kappa a periodic standing wave decays as g^n while it oscillates at the discrete
dispersion frequency; both for the forward and the transposed step).  Parity unpinned: the sponge
constants themselves (alpha, width) are a reading with no closed form; only agreement with the GPU
path covers them.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "rtm_oracle.c"))
    ):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_fd_coefficients.argtypes = [ctypes.c_int, _dp]
    lib.oracle_fd_coefficients.restype = ctypes.c_int
    lib.oracle_laplacian.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, _dp, ctypes.c_int]
    lib.oracle_laplacian.restype = None
    lib.oracle_step.argtypes = [ctypes.c_int] * 5 + [_dp] * 8 + [ctypes.c_int]
    lib.oracle_step.restype = None
    lib.oracle_adjoint_step.argtypes = [ctypes.c_int] * 5 + [_dp] * 9 + [ctypes.c_int]
    lib.oracle_adjoint_step.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------------------------
# Coefficients, time step, sponge, wavelet, material
# ----------------------------------------------------------------------------------------------
def fd_coefficients(radius: int = 4) -> np.ndarray:
    """Centred second-derivative weights c_0..c_R on unit spacing, from Fornberg's recursion."""
    c = np.zeros(radius + 1)
    if _load().oracle_fd_coefficients(int(radius), _ptr(c)) != 0:
        raise ValueError(f"unsupported radius {radius}")
    return c


def stability_limit(radius: int = 4) -> float:
    """Largest Courant number v dt / h for which 3-D leapfrog with this stencil is stable.

    The most negative eigenvalue of the 3-D operator is -3 S with S = |c0| + 2 sum_m |c_m| (the
    checkerboard mode); leapfrog needs kappa * 3 S <= 4, so C* = 2 / sqrt(3 S)."""
    c = fd_coefficients(radius)
    s = abs(c[0]) + 2.0 * np.sum(np.abs(c[1:]))
    return 2.0 / math.sqrt(3.0 * s)


def stable_dt(radius: int, h: float, vmax: float, fraction: float = 0.5) -> float:
    """Time step at `fraction` of the stability limit: dt = fraction * C* * h / vmax."""
    return fraction * stability_limit(radius) * h / vmax


def sponge_profile(n: int, width: int = 16, alpha: float = 0.015) -> np.ndarray:
    """Cerjan taper along one axis: gamma(d) = exp(-(alpha d)^2), d = cells into the sponge."""
    i = np.arange(n, dtype=np.float64)
    d = np.maximum(0.0, np.maximum(width - i, i - (n - 1 - width)))
    if width <= 0:
        d = np.zeros(n)
    return np.exp(-((alpha * d) ** 2))


def ricker(t, fpeak: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet of peak frequency fpeak, unit amplitude, delayed by t0 (default 1.5/fpeak)."""
    if t0 is None:
        t0 = 1.5 / fpeak
    a = (math.pi * fpeak * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def kappa_field(v: np.ndarray, dt: float, h: float) -> np.ndarray:
    """kappa = (v dt / h)^2, the dimensionless coefficient that multiplies L u."""
    v = _f64(v)
    return (v * dt / h) ** 2


def injection_weight(v_s, dt: float, h: float):
    """Weight of a point source: (v_s dt)^2 / h^3 (the grid delta is 1/h^3)."""
    return (np.asarray(v_s, dtype=np.float64) * dt) ** 2 / h**3


# ----------------------------------------------------------------------------------------------
# Stencil operators (the C loops)
# ----------------------------------------------------------------------------------------------
def laplacian(u: np.ndarray, radius: int = 4, periodic: bool = False, nthreads: int = 1) -> np.ndarray:
    u = _f64(u)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    c = fd_coefficients(radius)
    _load().oracle_laplacian(nx, ny, nz, radius, int(periodic), _ptr(c), _ptr(u), _ptr(out), nthreads)
    return out


def _sponge3(sponge, shape):
    nz, ny, nx = shape
    if sponge is None:
        return np.ones(nx), np.ones(ny), np.ones(nz)
    gx, gy, gz = (_f64(s) for s in sponge)
    assert gx.shape == (nx,) and gy.shape == (ny,) and gz.shape == (nz,)
    return gx, gy, gz


def step(u_cur, u_prv, kappa, sponge=None, radius: int = 4, periodic: bool = False,
         nthreads: int = 1, out: np.ndarray | None = None) -> np.ndarray:
    """u^{n+1} = g (2 u^n - g u^{n-1} + kappa L u^n) over the whole box."""
    u_cur, u_prv, kappa = _f64(u_cur), _f64(u_prv), _f64(kappa)
    nz, ny, nx = u_cur.shape
    gx, gy, gz = _sponge3(sponge, u_cur.shape)
    c = fd_coefficients(radius)
    if out is None:
        out = np.empty_like(u_cur)
    _load().oracle_step(nx, ny, nz, radius, int(periodic), _ptr(c), _ptr(kappa), _ptr(gx), _ptr(gy),
                        _ptr(gz), _ptr(u_cur), _ptr(u_prv), _ptr(out), nthreads)
    return out


def adjoint_step(mu_a, mu_b, kappa, sponge=None, radius: int = 4, periodic: bool = False,
                 nthreads: int = 1) -> np.ndarray:
    """mu = 2 g mu_a + L(kappa g mu_a) - g^2 mu_b: one step of the transposed recursion."""
    mu_a, mu_b, kappa = _f64(mu_a), _f64(mu_b), _f64(kappa)
    nz, ny, nx = mu_a.shape
    gx, gy, gz = _sponge3(sponge, mu_a.shape)
    c = fd_coefficients(radius)
    out = np.empty_like(mu_a)
    tmp = np.empty_like(mu_a)
    _load().oracle_adjoint_step(nx, ny, nz, radius, int(periodic), _ptr(c), _ptr(kappa), _ptr(gx),
                                _ptr(gy), _ptr(gz), _ptr(mu_a), _ptr(mu_b), _ptr(out), _ptr(tmp),
                                nthreads)
    return out


# ----------------------------------------------------------------------------------------------
# Time loops
# ----------------------------------------------------------------------------------------------
def _ijk(points):
    p = np.asarray(points, dtype=np.int64).reshape(-1, 3)
    return p[:, 0], p[:, 1], p[:, 2]


def forward(kappa, sponge, nsteps: int, *, radius: int = 4, src_ijk=None, src_w=None, src_amp=None,
            rec_ijk=None, u_cur=None, u_prv=None, snap_every: int = 0, keep_levels: bool = False,
            periodic: bool = False, nthreads: int = 1) -> dict:
    """Run `nsteps` leapfrog steps from (u^0, u^{-1}) (zero by default).

    Each step n = 0..nsteps-1: update (stencil + sponge), then add w_s * src_amp[n, s] at the
    source cells, then record traces[n, r] = u^{n+1} at the receiver cells.  With snap_every = s,
    u^k is kept for every k in 1..nsteps with k % s == 0 (snaps[k // s - 1]).  With keep_levels,
    u^n for n = 0..nsteps-1 is kept (the states the gradient needs).
    """
    kappa = _f64(kappa)
    shape = kappa.shape
    u_cur = np.zeros(shape) if u_cur is None else _f64(u_cur).copy()
    u_prv = np.zeros(shape) if u_prv is None else _f64(u_prv).copy()
    have_src = src_ijk is not None and len(np.asarray(src_ijk).reshape(-1, 3)) > 0
    if have_src:
        si, sj, sk = _ijk(src_ijk)
        src_w = _f64(src_w).reshape(-1)
        src_amp = _f64(src_amp).reshape(nsteps, -1)
    have_rec = rec_ijk is not None and len(np.asarray(rec_ijk).reshape(-1, 3)) > 0
    nrec = len(np.asarray(rec_ijk).reshape(-1, 3)) if have_rec else 0
    if have_rec:
        ri, rj, rk = _ijk(rec_ijk)
    traces = np.zeros((nsteps, nrec))
    snaps = []
    levels = []
    for n in range(nsteps):
        if keep_levels:
            levels.append(u_cur.copy())
        u_nxt = step(u_cur, u_prv, kappa, sponge, radius, periodic, nthreads)
        if have_src:
            np.add.at(u_nxt, (sk, sj, si), src_w * src_amp[n])
        if have_rec:
            traces[n] = u_nxt[rk, rj, ri]
        u_prv, u_cur = u_cur, u_nxt
        if snap_every and (n + 1) % snap_every == 0:
            snaps.append(u_cur.copy())
    out = {"traces": traces, "u_cur": u_cur, "u_prv": u_prv}
    if snap_every:
        out["snaps"] = snaps
    if keep_levels:
        out["levels"] = levels
    return out


def migrate(kappa, sponge, nsteps: int, *, radius: int = 4, src_ijk, src_w, src_amp, rec_ijk, rec_w,
            data, image_every: int = 1, nthreads: int = 1, snapshot_format: str | None = None) -> np.ndarray:
    """Zero-lag cross-correlation image of one shot.

    Forward: the source wavefield u^k, kept at the imaging levels k in T = {k in 1..N : k % s == 0}.
    Backward: the receiver wavefield r with r^0 = r^{-1} = 0 and, for m = 0..N-1,
    r^{m+1} = update(r^m, r^{m-1}) + sum_r w_r data[N-1-m, r]; r^{m+1} is the receiver
    wavefield at forward level k = N - m.  Image: I = sum_{k in T} u^k r^{N+1-k}.  With
    snapshot_format, u^k is stored as 16-bit codes with a per-slab scale and decoded before imaging.
    """
    fwd = forward(kappa, sponge, nsteps, radius=radius, src_ijk=src_ijk, src_w=src_w, src_amp=src_amp,
                  snap_every=image_every, nthreads=nthreads)
    snaps = fwd["snaps"]
    if snapshot_format is not None:
        # snapshots kept in a 16-bit code with one scale per z slab (FP32 decisions), decoded for imaging
        snaps = [snapshot_decode(*snapshot_encode(sn, snapshot_format), snapshot_format).astype(np.float64)
                 for sn in snaps]
    data = _f64(data).reshape(nsteps, -1)
    rec_w = _f64(rec_w).reshape(-1)
    ri, rj, rk = _ijk(rec_ijk)
    shape = _f64(kappa).shape
    image = np.zeros(shape)
    r_cur = np.zeros(shape)
    r_prv = np.zeros(shape)
    for m in range(nsteps):
        r_nxt = step(r_cur, r_prv, kappa, sponge, radius, False, nthreads)
        np.add.at(r_nxt, (rk, rj, ri), rec_w * data[nsteps - 1 - m])
        k = nsteps - m
        if k % image_every == 0:
            image += snaps[k // image_every - 1] * r_nxt
        r_prv, r_cur = r_cur, r_nxt
    return image


def adjoint_sources(kappa, sponge, nsteps: int, *, radius: int = 4, src_ijk, src_w, rec_ijk, y,
                    periodic: bool = False, nthreads: int = 1, return_states: bool = False):
    """Transpose of the map (source series -> traces) of `forward`.

    mu^{N+1} = mu^{N+2} = 0 and, for n = N..1,
        mu^n = 2 g mu^{n+1} + L(kappa g mu^{n+1}) - g^2 mu^{n+2} + R^T y^{n-1};
    the source-side output is x[n, s] = w_s mu^{n+1}[s] for n = 0..N-1.
    """
    kappa = _f64(kappa)
    shape = kappa.shape
    y = _f64(y).reshape(nsteps, -1)
    ri, rj, rk = _ijk(rec_ijk)
    si, sj, sk = _ijk(src_ijk)
    src_w = _f64(src_w).reshape(-1)
    mu_a = np.zeros(shape)   # mu^{n+1}
    mu_b = np.zeros(shape)   # mu^{n+2}
    x = np.zeros((nsteps, len(src_w)))
    states = [None] * (nsteps + 1)
    for n in range(nsteps, 0, -1):
        mu = adjoint_step(mu_a, mu_b, kappa, sponge, radius, periodic, nthreads)
        np.add.at(mu, (rk, rj, ri), y[n - 1])
        x[n - 1] = src_w * mu[sk, sj, si]
        if return_states:
            states[n] = mu
        mu_b, mu_a = mu_a, mu
    if return_states:
        return x, states
    return x


def misfit(traces, observed) -> float:
    """J = 1/2 sum (d - d_obs)^2, accumulated in FP64."""
    r = _f64(traces) - _f64(observed)
    return 0.5 * float(np.sum(r * r))


def gradient_kappa(kappa, sponge, nsteps: int, *, radius: int = 4, src_ijk, src_w, src_amp, rec_ijk,
                   observed, nthreads: int = 1):
    """Adjoint-state gradient of J = 1/2 sum_n sum_r (d^n_r - obs^n_r)^2 with respect to kappa.

    dJ/dkappa = sum_{n=0..N-1} g mu^{n+1} L u^n, with mu driven by the residual traces (the
    injection weights are held fixed).  Returns (J, dJ/dkappa)."""
    kappa = _f64(kappa)
    fwd = forward(kappa, sponge, nsteps, radius=radius, src_ijk=src_ijk, src_w=src_w, src_amp=src_amp,
                  rec_ijk=rec_ijk, keep_levels=True, nthreads=nthreads)
    resid = fwd["traces"] - _f64(observed).reshape(nsteps, -1)
    _, states = adjoint_sources(kappa, sponge, nsteps, radius=radius, src_ijk=src_ijk, src_w=src_w,
                                rec_ijk=rec_ijk, y=resid, nthreads=nthreads, return_states=True)
    gx, gy, gz = _sponge3(sponge, kappa.shape)
    g = gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    grad = np.zeros_like(kappa)
    for n in range(nsteps):
        grad += g * states[n + 1] * laplacian(fwd["levels"][n], radius, False, nthreads)
    return 0.5 * float(np.sum(resid * resid)), grad


# ----------------------------------------------------------------------------------------------
# Reduced-precision snapshots (per-slab scale, 16-bit codes)
# ----------------------------------------------------------------------------------------------
def bf16_rne(x32: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns, round to nearest, ties to even (finite inputs): keep the upper 16
    bits after adding half an ulp of the kept part (0x7FFF plus the lowest kept bit)."""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_to_f32(codes: np.ndarray) -> np.ndarray:
    return (np.asarray(codes, dtype=np.uint32) << 16).astype(np.uint32).view(np.float32)


def snapshot_encode(u, fmt: str):
    """Per-slab (z plane) scale s_k = max |u| over the plane and codes RNE(u / s_k) in BF16 or FP16.
    The quotient and the rounding decision are taken in FP32.  Returns (codes uint16, scales f32)."""
    u32 = np.asarray(u, dtype=np.float32)
    scales = np.max(np.abs(u32), axis=(1, 2)).astype(np.float32)
    safe = np.where(scales > 0, scales, np.float32(1.0)).astype(np.float32)
    q = (u32 / safe[:, None, None]).astype(np.float32)
    q[scales == 0] = 0.0
    if fmt == "bf16":
        codes = bf16_rne(q)
    elif fmt == "f16":
        codes = q.astype(np.float16).view(np.uint16)
    else:
        raise ValueError(fmt)
    return codes, scales


def snapshot_decode(codes, scales, fmt: str) -> np.ndarray:
    vals = bf16_to_f32(codes) if fmt == "bf16" else np.asarray(codes, dtype=np.uint16).view(np.float16).astype(np.float32)
    return vals.astype(np.float32) * np.asarray(scales, dtype=np.float32)[:, None, None]


# ----------------------------------------------------------------------------------------------
# Halo faces and error norms
# ----------------------------------------------------------------------------------------------
def pack_faces(u, radius: int = 4):
    """The six R-thick owned layers -X,+X,-Y,+Y,-Z,+Z, each as its sub-block in x-fastest order."""
    u = _f64(u)
    r = radius
    return [u[:, :, :r].ravel(), u[:, :, -r:].ravel(), u[:, :r, :].ravel(), u[:, -r:, :].ravel(),
            u[:r].ravel(), u[-r:].ravel()]


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2, accumulated in FP64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.sqrt(np.sum(b * b)))
    return float(np.sqrt(np.sum((a - b) ** 2))) / (nb if nb > 0 else 1.0)
