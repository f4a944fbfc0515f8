"""Padded device geometry of one subdomain and helpers that marshal host inputs into it.

A field is a flat FP32 device tensor; owned cell (i, j, k) sits at element
(k + R) * pitch_z + (j + R) * pitch_y + (i + R) (see include/rtm.h).  The allocation is shifted so
that the first interior column (padded x = 2R) of every row starts on an `x_align`-float boundary,
which lets the interior kernel issue aligned float4 loads and whole cache lines.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _abi


def _round_up(a: int, b: int) -> int:
    return (a + b - 1) // b * b


class Grid:
    """Owned box of nx * ny * nz cells with spacing h (m), time step dt (s) and stencil radius R."""

    def __init__(self, nx: int, ny: int, nz: int, h: float, dt: float, radius: int = 4,
                 sponge_width: int = 16, sponge_alpha: float = 0.015, device: str | torch.device = "cuda",
                 x_align: int = 32, pitch_y: int | None = None, sponge_profiles=None):
        """sponge_profiles: optional host arrays (gx [nx], gy [ny], gz [nz]) used instead of the
        profiles computed from sponge_width and sponge_alpha; a subdomain of a decomposed grid passes
        its slices of the global profiles."""
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.h, self.dt, self.radius = float(h), float(dt), int(radius)
        self.device = torch.device(device)
        R = self.radius
        self.x_align = int(x_align)
        self.pitch_y = int(pitch_y) if pitch_y is not None else _round_up(self.nx + 2 * R, self.x_align)
        self.pitch_z = _round_up(self.pitch_y * (self.ny + 2 * R), self.x_align)
        self.total = self.pitch_z * (self.nz + 2 * R)
        # shift so that the float4 holding owned x = 0 (padded element R - R % 4) starts an x_align
        # boundary (allocations are 256 B aligned): with 128-byte lines, a row's owned cells then
        # start a line and the x-strip / interior boundaries fall on line starts, so no call writes a
        # partial line there (the 512^3 halo-first step took 0.614 ms with owned x = 4 line-aligned,
        # 0.547 ms with owned x = 0; the 384^3 radius-2 step 0.324 against 0.285 ms)
        self._shift = (-(R - R % 4)) % self.x_align
        self.sponge_width, self.sponge_alpha = int(sponge_width), float(sponge_alpha)
        if sponge_profiles is None:
            self.gx = self._sponge(self.nx)
            self.gy = self._sponge(self.ny)
            self.gz = self._sponge(self.nz)
        else:
            prof = [np.ascontiguousarray(a, dtype=np.float32) for a in sponge_profiles]
            if [len(a) for a in prof] != [self.nx, self.ny, self.nz]:
                raise ValueError("sponge profiles must have nx, ny and nz entries")
            self.gx, self.gy, self.gz = (torch.from_numpy(a).to(self.device) for a in prof)
        self.c = _abi.rtm_grid_init(self.nx, self.ny, self.nz, R, self.pitch_y, self.pitch_z, self.gx, self.gy,
                                    self.gz)
        off = _abi.rtm_face_layout(self.c)
        self.face_offsets = off[:6]
        self.face_total = off[6]
        self.face_sizes = [off[f + 1] - off[f] for f in range(6)]

    # ------------------------------------------------------------------------------------------
    def _sponge(self, n: int) -> torch.Tensor:
        prof = _abi.rtm_sponge_profile(n, self.sponge_width, self.sponge_alpha)
        return torch.from_numpy(prof).to(self.device)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz

    def field(self, fill: float | None = 0.0) -> torch.Tensor:
        """A padded FP32 field (zero, or uninitialised with fill=None)."""
        n = self.total + self._shift
        buf = torch.empty(n, dtype=torch.float32, device=self.device) if fill is None else \
            torch.full((n,), float(fill), dtype=torch.float32, device=self.device)
        return buf[self._shift:]

    def owned(self, f: torch.Tensor) -> torch.Tensor:
        """Strided (nz, ny, nx) view of the owned cells of a padded field."""
        R = self.radius
        return f.as_strided((self.nz, self.ny, self.nx), (self.pitch_z, self.pitch_y, 1),
                            f.storage_offset() + R * self.pitch_z + R * self.pitch_y + R)

    def padded(self, f: torch.Tensor) -> torch.Tensor:
        """Strided (nz+2R, ny+2R, nx+2R) view including the ghost ring."""
        R = self.radius
        return f.as_strided((self.nz + 2 * R, self.ny + 2 * R, self.nx + 2 * R), (self.pitch_z, self.pitch_y, 1),
                            f.storage_offset())

    def index(self, ijk) -> np.ndarray:
        """Padded linear indices (int64) of owned cells given as an (n, 3) array of (i, j, k)."""
        p = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
        if p.size and (np.any(p < 0) or np.any(p[:, 0] >= self.nx) or np.any(p[:, 1] >= self.ny)
                       or np.any(p[:, 2] >= self.nz)):
            raise ValueError("cell outside the owned box")
        R = self.radius
        return (p[:, 2] + R) * self.pitch_z + (p[:, 1] + R) * self.pitch_y + (p[:, 0] + R)

    def in_halo(self, ijk) -> np.ndarray:
        """True for owned cells that rtm_step_halo updates (the R-shell widened to the halo region
        reported by rtm_halo_region); the rest belong to rtm_step_interior."""
        p = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
        wx, hy, R = _abi.rtm_halo_region(self.c)
        lo = np.array([wx, hy, R])
        hi = np.array([self.nx - wx, self.ny - hy, self.nz - R])
        return np.any((p < lo) | (p >= hi), axis=1)

    def upload(self, host: np.ndarray, f: torch.Tensor | None = None) -> torch.Tensor:
        """Copy a compact (nz, ny, nx) host array into the owned cells of a (new, zeroed) field."""
        if f is None:
            f = self.field()
        src = torch.from_numpy(np.ascontiguousarray(host, dtype=np.float32))
        self.owned(f).copy_(src.to(self.device))
        return f

    def download(self, f: torch.Tensor) -> np.ndarray:
        """Owned cells of a field as a host (nz, ny, nx) float32 array."""
        return self.owned(f).cpu().numpy()

    def kappa_from_velocity(self, v, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """kappa = (v dt / h)^2 on the device; `v` is a host array or a compact device tensor."""
        if not isinstance(v, torch.Tensor):
            v = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(self.device)
        v = v.to(device=self.device, dtype=torch.float32).contiguous()
        if out is None:
            out = self.field()
        _abi.rtm_kappa_from_velocity(self.c, out, v, self.dt / self.h,
                                     stream if stream is not None else torch.cuda.current_stream())
        return out

    def faces(self) -> torch.Tensor:
        return torch.zeros(self.face_total, dtype=torch.float32, device=self.device)

    def face_slots(self, faces: torch.Tensor):
        return [faces[o:o + s] for o, s in zip(self.face_offsets, self.face_sizes)]

    def injection_weights(self, v_at_sources) -> np.ndarray:
        """Point-source weights of this grid's dt and h for the velocities at the source cells
        (rtm_injection_weights)."""
        return _abi.rtm_injection_weights(v_at_sources, self.dt, self.h)

    def ricker(self, nsteps: int, fpeak: float, t0: float | None = None) -> np.ndarray:
        return _abi.rtm_ricker(nsteps, self.dt, fpeak, 1.5 / fpeak if t0 is None else t0)

    @staticmethod
    def stable_dt(radius: int, h: float, vmax: float, fraction: float = 0.5) -> float:
        """dt at `fraction` of the 3-D leapfrog stability limit (rtm_stable_dt)."""
        return _abi.rtm_stable_dt(radius, h, vmax, fraction)

    def bytes_per_field(self) -> int:
        return 4 * self.total

    def __repr__(self):
        return (f"Grid({self.nx}x{self.ny}x{self.nz}, h={self.h}, dt={self.dt:.6g}, R={self.radius}, "
                f"pitch_y={self.pitch_y}, pitch_z={self.pitch_z})")
