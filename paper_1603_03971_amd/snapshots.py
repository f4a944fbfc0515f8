"""Reduced-precision source-wavefield snapshots for imaging.

Each snapshot is a compact x-fastest array of 16-bit codes (BF16 or FP16) of u / s_k plus one FP32
scale s_k = max |u| per z plane (slab); the stencil and the image accumulation stay FP32.  Encoding
(rtm_snapshot_encode) and decoding inside the imaging kernel (rtm_image_accumulate_coded) run in the
library's kernels; this class only owns the buffers.
"""
from __future__ import annotations

import torch

from . import _abi
from .grid import Grid

FORMATS = {"bf16": _abi.RTM_SNAP_BF16, "f16": _abi.RTM_SNAP_F16}


class CodedSnapshots:
    def __init__(self, grid: Grid, fmt: str = "bf16"):
        if fmt not in FORMATS:
            raise ValueError(f"unknown snapshot format {fmt}")
        self.g = grid
        self.fmt = fmt
        self.code = FORMATS[fmt]

    def encode(self, u: torch.Tensor, stream=None):
        g = self.g
        codes = torch.empty(g.points, dtype=torch.int16, device=g.device)
        scales = torch.empty(g.nz, dtype=torch.float32, device=g.device)
        st = stream if stream is not None else torch.cuda.current_stream()
        _abi.rtm_snapshot_encode(g.c, u, codes, scales, self.code, st)
        return codes, scales

    def image_accumulate(self, image, snap, rcv, weight=1.0, stream=None):
        codes, scales = snap
        st = stream if stream is not None else torch.cuda.current_stream()
        _abi.rtm_image_accumulate_coded(self.g.c, image, codes, scales, self.code, rcv, weight, st)

    def bytes_per_snapshot(self) -> int:
        return 2 * self.g.points + 4 * self.g.nz


def make(fmt: str | None):
    """Factory for ShotImager: None keeps FP32 levels (pinned buffers), else a coded format."""
    if fmt is None or fmt == "f32":
        return None
    return lambda grid: CodedSnapshots(grid, fmt)
