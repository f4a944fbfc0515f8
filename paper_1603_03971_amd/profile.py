"""Profiling driver for rocprofv3 and the summary of its output.

  python3 -m paper_1603_03971_amd.profile interior [--n 512] [--launches 10]
      runs the 512^3 layered workload's interior stencil launches (the benchmark's configuration)
      and, for counter calibration, a plain device copy of 1 GiB (reads and writes exactly 1 GiB).
      Run it under `rocprofv3 --pmc FETCH_SIZE` and, separately, `rocprofv3 --pmc WRITE_SIZE`.

  python3 -m paper_1603_03971_amd.profile halo [--n 512] [--launches 10]
      the same for the halo call of the halo-region form (rtm_step_halo_pack_slots: the z slabs,
      y strips and x strips of the halo region, also writing the six faces), for its counters.

  python3 -m paper_1603_03971_amd.profile whole-slots [--n 512] [--launches 10]
      the same for the benchmark's dominant call (the shell form's rtm_step_whole_slots: every
      owned cell, the ghosts read from zero-filled receive slots).

  python3 -m paper_1603_03971_amd.profile conv [--n 384] [--launches 10]
      runs the corrector network's forward pass (three 3x3x3 convolutions, 16 channels, BF16 MFMA)
      on an n^3 volume `launches` times, for a kernel trace of the convolution.

  python3 -m paper_1603_03971_amd.profile corrected [--n 384] [--steps 160] [--every 16]
      runs `steps` coarse-grid steps (radius 2, the coarse companion of a 2n^3 fine grid) of a point
      source in a smooth medium with the dispersion corrector applied every `every` steps, for a
      kernel trace of the corrected coarse propagation (stencil calls, network, glue).

  python3 -m paper_1603_03971_amd.profile shot [--nx 512 --ny 512 --nz 256] [--steps 2000] [--every 4]
      one full-size RTM shot over three dipping reflectors (seed 3; v(z) = 1500 + 0.75 z m/s; source
      at (nx/2, ny/2, 20), receivers every 2 cells at depth 20): models the true and background
      data, then migrates them with FP32, BF16 and FP16 source snapshots (best of --repeats), and
      prints the times, the snapshot memory and each coded image's rel-L2 against the FP32 image.

  python3 -m paper_1603_03971_amd.profile gradient [--n 256] [--shots 8] [--steps 1500] [--every 50]
      the misfit gradient at full size: true model 20 flat layers (seed 4), start model that smoothed
      with sigma = 8 cells, shots at seeded positions at depth 20, receivers every 2 cells at depth
      20; models the observed data, times J and dJ/dv (forward with checkpoints, recomputation,
      adjoint), and checks <dJ/dv, d> against central differences of J: along a smooth direction d,
      and for 1e-3 relative perturbations of --cells seeded cells (signed by the gradient, the
      difference formed from the traces in FP64).

  python3 -m paper_1603_03971_amd.profile summarize --stats DIR --fetch DIR --write DIR --out FILE
      reads rocprofv3 CSV output (kernel stats of a benchmark run, counter collections of the two
      runs above) and writes a short text summary plus the traffic record that bench.py reports
      (keyed by a hash of the kernel source, so stale counters are never reported).

  python3 -m paper_1603_03971_amd.profile summarize-halo --fetch DIR --write DIR --out FILE [--stats DIR]
      the halo call's HBM traffic from the counter runs of `halo` (and its kernel-trace time from the
      benchmark's kernel statistics, if given).

  python3 -m paper_1603_03971_amd.profile summarize-stream --dir DIR --out FILE
      the bandwidth reference from a kernel trace of the stand-alone probe
      (paper_1603_03971_amd/stream_probe, built by build.py: three arrays of 512^3 floats read and one
      written per element, a copy and three reads alone, at several grid sizes), per kernel and grid.

  python3 -m paper_1603_03971_amd.profile summarize-conv --stats DIR --out FILE [--n 384]
  python3 -m paper_1603_03971_amd.profile summarize-corrected --stats DIR --out FILE [--n 384 ...]
      the same for kernel traces of the `conv` and `corrected` runs (per-launch rates; per-step and
      per-correction costs).
  Every summarize mode takes --command (repeatable): the commands recorded in the summary.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30


def run_interior(n: int, launches: int, call: str = "interior"):
    import numpy as np
    import torch

    from . import _abi, synth
    from .grid import Grid

    h = 10.0
    prof = synth.layered_profile(n, h, seed=2)
    g = Grid(n, n, n, h, Grid.stable_dt(4, h, float(prof.max())))
    v = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(prof[:, None, None], (n, n, n)), dtype=np.float32))
    kap = g.kappa_from_velocity(v.cuda())
    u, up = g.field(), g.field()
    g.owned(u).normal_()
    g.owned(up).normal_()
    s = torch.cuda.current_stream()
    faces, recv = g.faces(), g.faces()
    slots = g.face_slots(recv)
    for _ in range(launches):
        if call == "interior":
            _abi.rtm_step_interior(g.c, up, u, up, kap, s)
        elif call == "whole_slots":            # the shell form's call over every owned cell
            _abi.rtm_step_whole_slots(g.c, up, u, up, kap, slots, s)
        else:                                  # the halo-region form's halo call: ghosts from the slots, packs
            _abi.rtm_step_halo_pack_slots(g.c, up, u, up, kap, slots, faces, s)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    wx, hy, R = _abi.rtm_halo_region(g.c)
    interior = (n - 2 * wx) * (n - 2 * hy) * (n - 2 * R)
    points = {"interior": interior, "whole_slots": n**3}.get(call, n**3 - interior)
    print(json.dumps({f"{call}_points": points, "copy_bytes": COPY_BYTES}))


# The hot kernels of the forward, RTM and gradient paths, each launched `launches` times on the n^3
# layered workload (radius 4, line-aligned fields), for counter runs: name -> (kernel-name substring,
# algorithmic bytes per launch as a function of n, what the bytes are).
def interior_cells(n: int) -> int:
    """Cells of the interior call's box on an n^3 grid under the default halo region (64-column x
    strips, 8-row y strips, 4-plane z slabs)."""
    return (n - 2 * 64) * (n - 2 * 8) * (n - 8)


def kernel_table(n: int):
    cells = n ** 3
    interior = interior_cells(n)
    halo = cells - interior
    faces = 6 * 4 * n * n
    shell_cells = n ** 3 - (n - 8) ** 3                    # the owned cells within 4 of a face
    return {
        "interior": ("k_tiled<4, 16, 8, 0, false", 16 * interior, "16 B per interior cell"),
        "halo_pack": ("k_tiled<4, 16, 16, 0, true, 1>", 16 * halo + 4 * faces, "16 B per halo cell + 4 B per face cell"),
        "halo_pack_slots": ("k_tiled<4, 16, 16, 0, true, 5>", 16 * halo + 8 * faces,
                            "16 B per halo cell + 4 B per face cell out + 4 B per ghost cell in"),
        "shell": ("k_shell<13>", 16 * shell_cells + 4 * faces,
                  "16 B per shell cell (12 B in, 4 B to the face buffer) + 4 B per ghost cell in"),
        "whole_slots": ("k_tiled<4, 32, 8, 0, false, 5>", 16 * cells, "16 B per cell"),
        "whole": ("k_tiled<4, 32, 8, 0, false, 1>", 16 * cells, "16 B per cell (also the scaled adjoint step)"),
        "adjoint_direct": ("k_tiled<4, 32, 8, 1, false", 16 * cells, "16 B per cell: mu_a, kappa, mu_b in, mu out"),
        "gradient": ("k_tiled<4, 32, 8, 2, false", 16 * cells, "16 B per cell: u, mu, grad in, grad out"),
        "gradient_scaled": ("k_tiled<4, 32, 8, 3, false", 16 * cells, "16 B per cell: u, w, grad in, grad out"),
        "unpack": ("k_unpack_lines", 8 * faces, "8 B per face cell: slot in, ghost out"),
        "image": ("k_image<true", 16 * cells, "16 B per cell: S, R, I in, I out"),
        "absmax": ("k_plane_absmax<true>", 4 * cells, "4 B per cell"),
        "encode": ("k_encode<true>", 6 * cells, "6 B per cell: u in, 16-bit code out"),
        "image_coded": ("k_image_coded<true", 14 * cells, "14 B per cell: code, R, I in, I out"),
    }


def run_kernels(n: int, launches: int):
    import numpy as np
    import torch

    from . import _abi, synth
    from .grid import Grid
    from .snapshots import CodedSnapshots

    h = 10.0
    prof = synth.layered_profile(n, h, seed=2)
    g = Grid(n, n, n, h, Grid.stable_dt(4, h, float(prof.max())))
    v = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(prof[:, None, None], (n, n, n)), dtype=np.float32))
    kap = g.kappa_from_velocity(v.cuda())
    del v
    a, b, c = g.field(), g.field(), g.field()
    for f in (a, b, c):
        g.owned(f).normal_()
    s = torch.cuda.current_stream()
    send, recv = g.faces(), g.faces()
    slots = g.face_slots(recv)
    dense = (g.faces(), g.faces(), g.faces())
    for src, dst in zip((a, b, kap), dense):
        _abi.rtm_pack_halo(g.c, src, dst, s)
    work = g.field()
    codes = torch.empty(n ** 3, dtype=torch.int16, device="cuda")
    scales = torch.empty(n, dtype=torch.float32, device="cuda")
    calls = {
        "interior": lambda: _abi.rtm_step_interior(g.c, c, a, b, kap, s),
        "halo_pack": lambda: _abi.rtm_step_halo_pack(g.c, c, a, b, kap, send, s),
        "halo_pack_slots": lambda: _abi.rtm_step_halo_pack_slots(g.c, c, a, b, kap, slots, send, s),
        "shell": lambda: _abi.rtm_step_shell_pack(g.c, a, b, kap, slots, send, s, dense=dense),
        "whole_slots": lambda: _abi.rtm_step_whole_slots(g.c, c, a, b, kap, slots, s),
        "whole": lambda: _abi.rtm_step_whole(g.c, c, a, b, kap, s),
        "adjoint_direct": lambda: _abi.rtm_adjoint_step(g.c, c, a, b, kap, work, s),
        "gradient": lambda: _abi.rtm_gradient_accumulate(g.c, c, a, b, s),
        "gradient_scaled": lambda: _abi.rtm_gradient_accumulate_scaled(g.c, c, a, b, s),
        "unpack": lambda: _abi.rtm_unpack_halo(g.c, c, slots, s),
        "image": lambda: _abi.rtm_image_accumulate(g.c, c, a, b, 1.0, s),
        "encode": lambda: _abi.rtm_snapshot_encode(g.c, a, codes, scales, _abi.RTM_SNAP_BF16, s),
        "image_coded": lambda: _abi.rtm_image_accumulate_coded(g.c, c, codes, scales, _abi.RTM_SNAP_BF16, b, 1.0, s),
    }
    for name, fn in calls.items():
        for _ in range(launches):
            fn()
        torch.cuda.synchronize()
        print(f"{name}: {launches} launches", flush=True)
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"n": n, "launches": launches, "copy_bytes": COPY_BYTES}), flush=True)


def summarize_kernels(fetch_dir, write_dir, stats_dir, out, n, commands):
    """Per-kernel HBM traffic (FETCH_SIZE + WRITE_SIZE, calibrated by the 1 GiB copy) against the
    algorithmic bytes of kernel_table, and the kernel-trace duration of the same run."""
    fr, wr = _csv(fetch_dir, "*counter_collection.csv"), _csv(write_dir, "*counter_collection.csv")
    f_cp, _ = _counter(fr, "opy", "FETCH_SIZE", largest=True)
    w_cp, _ = _counter(wr, "opy", "WRITE_SIZE", largest=True)
    kf = COPY_BYTES / (f_cp * 1024.0)
    kw = COPY_BYTES / (w_cp * 1024.0)
    stats = _csv(stats_dir, "*kernel_stats.csv") if stats_dir else []
    lines = [f"# rocprofv3 summary: HBM traffic of the hot kernels, {n}^3 layered workload (radius 4)", "",
             "Commands:"] + [f"    {c}" for c in commands] + [""]
    lines += [f"Counter calibration with a plain 1 GiB device copy: FETCH_SIZE x {kf:.3f}, WRITE_SIZE x {kw:.3f}", "",
              f"    {'call':16s} {'alg MB':>9s} {'read MB':>9s} {'write MB':>9s} {'ratio':>6s} {'avg us':>8s} "
              f"{'alg TB/s':>8s} {'moved TB/s':>10s}  algorithmic bytes"]
    record = {"n": n, "kernel_source_sha256_16": kernel_source_hash(), "fetch_factor": kf, "write_factor": kw,
              "kernels": {}}
    for name, (sub, alg, what) in kernel_table(n).items():
        f, nf = _counter(fr, sub, "FETCH_SIZE")
        w, nw = _counter(wr, sub, "WRITE_SIZE")
        if f is None or w is None:
            continue
        rd, wt = f * 1024.0 * kf, w * 1024.0 * kw
        us = None
        for r in stats:
            if sub in r["Name"]:
                us = float(r["AverageNs"]) / 1e3
                break
        tb_alg = f"{alg / us / 1e6:8.2f}" if us else f"{'-':>8s}"
        tb_mv = f"{(rd + wt) / us / 1e6:10.2f}" if us else f"{'-':>10s}"
        lines.append(f"    {name:16s} {alg / 1e6:9.1f} {rd / 1e6:9.1f} {wt / 1e6:9.1f} {(rd + wt) / alg:6.3f} "
                     f"{(us or 0):8.1f} {tb_alg} {tb_mv}  {what}")
        record["kernels"][name] = {"kernel": sub, "algorithmic_bytes": alg, "read_bytes": rd, "write_bytes": wt,
                                   "avg_us": us, "dispatches": [nf, nw]}
    text = "\n".join(lines) + "\n"
    with open(out, "w") as fo:
        fo.write(text)
    print(text)


def run_conv(n: int, launches: int):
    import torch

    from . import learned

    ws = learned.Workspace(n, n, n, train=False)
    net = learned.CorrectorNet(seed=1, out_init=1.0)
    ws.x.copy_(torch.randn(ws.x.numel(), dtype=torch.bfloat16, device="cuda").view(torch.int16))
    for _ in range(launches):
        learned.forward(net, ws)
    torch.cuda.synchronize()
    flop = 3 * n ** 3 * 27 * 16 * 16 * 2
    print(json.dumps({"voxels": n ** 3, "layers": 3, "algorithmic_flop_per_forward": flop}))


def run_corrected(n: int, steps: int, every: int):
    import numpy as np
    import torch

    from . import learned, synth
    from .grid import Grid
    from .propagator import Propagator, Sources

    fine = Grid(2 * n, 2 * n, 2 * n, learned.TRAIN_H, Grid.stable_dt(4, learned.TRAIN_H, learned.TRAIN_VMAX))
    coarse = learned.coarse_grid(fine)
    del fine
    v = synth.random_smooth_velocity(coarse.shape, seed=11, vmin=1500.0, vmax=3000.0, sigma=5.0).astype(np.float32)
    kap = coarse.kappa_from_velocity(v)
    c = n // 2
    src = Sources(coarse, [(c, c, c)], coarse.injection_weights([v[c, c, c]]), coarse.ricker(steps, 15.0)[:, None])
    net = learned.CorrectorNet(seed=1)
    corr = learned.Corrector(net, coarse, v, every)
    corr.set_mask(learned.injection_mask(coarse, [(c, c, c)]))
    prop = Propagator(coarse, kap, sources=src, schedule="fused")
    prop.run(steps, on_level=corr)
    torch.cuda.synchronize()
    print(json.dumps({"coarse_cells": coarse.points, "steps": steps, "corrections": corr.applied}))


# The radius-4 kernels of the forward step under the default options at 512^3 (prefixes of the
# demangled names): the interior call's tiles (16 x 8 threads), the halo-region call's (16 x 16), the
# shell call (one launch: x-strip rows and 32 x 8 tiles of the z slabs and y strips, faces only),
# the whole-block call with the ghosts from the slots (32 x 8) and the one-launch step's (32 x 8).
INTERIOR_KERNEL = "k_tiled<4, 16, 8, 0, false"
HALO_KERNEL = "k_tiled<4, 16, 16, 0, true"
SHELL_KERNEL = "k_shell<"
WHOLE_SLOTS_KERNEL = "k_tiled<4, 32, 8, 0, false, 5>"
WHOLE_KERNEL = "k_tiled<4, 32, 8, 0, false, 1>"
TILED_R4 = "k_tiled<4, "


def run_shot(nx: int, ny: int, nz: int, steps: int, every: int, repeats: int, schedule: str):
    import time

    import numpy as np
    import torch

    from . import rtm, snapshots, synth
    from .grid import Grid
    from .propagator import tune_grid

    def say(msg):
        print(msg, flush=True)

    h = 10.0
    v_true, v_bg = synth.dipping_reflector_model((nz, ny, nx), h, seed=3)
    dt = Grid.stable_dt(4, h, float(max(v_true.max(), v_bg.max())))
    g = Grid(nx, ny, nz, h, dt)
    src = np.array([[nx // 2, ny // 2, 20]], dtype=np.int64)
    rec = synth.surface_receivers(nx, ny, k=20, stride=2)
    wav = g.ricker(steps, 15.0)
    kap_true, kap_bg = g.kappa_from_velocity(v_true), g.kappa_from_velocity(v_bg)
    vs = v_bg[src[:, 2], src[:, 1], src[:, 0]]
    del v_true
    choice = tune_grid(g)
    say(f"one-launch step tuned for {nx}x{ny}x{nz}: tile variant {choice[0]}, workgroup order {choice[1]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d_true = rtm.model_shot(g, kap_true, vs, src, wav, rec, steps, schedule)
    d_bg = rtm.model_shot(g, kap_bg, vs, src, wav, rec, steps, schedule)
    torch.cuda.synchronize()
    t_model = time.perf_counter() - t0
    del kap_true
    say(f"data modelled: {len(rec)} receivers x {steps} steps, two propagations in {t_model:.3f} s")
    out = {"grid": [nx, ny, nz], "steps": steps, "image_every": every, "receivers": int(len(rec)),
           "schedule": schedule, "tuned": list(choice), "t_model_two_shots_s": round(t_model, 4)}
    images = {}
    for fmt in ("f32", "bf16", "f16"):
        best = None
        for _ in range(max(1, repeats)):
            codec = snapshots.make(fmt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            img = rtm.migrate_shot(g, kap_bg, v_bg, src, wav, rec, d_true, d_bg, steps, every, schedule,
                                   codec(g) if codec is not None else None)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
            images[fmt] = g.download(img).astype(np.float64)
            del img
        torch.cuda.empty_cache()
        nsnap = steps // every
        per = g.bytes_per_field() if fmt == "f32" else snapshots.CodedSnapshots(g, fmt).bytes_per_snapshot()
        out[f"t_migrate_{fmt}_s"] = round(best, 4)
        out[f"snapshot_GB_{fmt}"] = round(nsnap * per / 1e9, 2)
        say(f"migration with {fmt} snapshots: {best:.3f} s ({nsnap} snapshots, {nsnap * per / 1e9:.1f} GB)")
    ref = images["f32"]
    nref = float(np.linalg.norm(ref))
    for fmt in ("bf16", "f16"):
        out[f"image_rel_l2_{fmt}_vs_f32"] = float(np.linalg.norm(images[fmt] - ref) / nref)
    out["image_norm"] = nref
    out["image_finite"] = bool(all(np.isfinite(im).all() for im in images.values()))
    print(json.dumps(out), flush=True)


def run_gradient(n: int, nshots: int, steps: int, every: int, eps: float, cells: int = 0):
    import time

    import numpy as np
    import torch

    from . import synth
    from .adjoint import MisfitProblem, Shot
    from .grid import Grid
    from .propagator import tune_grid

    def say(msg):
        print(msg, flush=True)

    h = 10.0
    shape = (n, n, n)
    v_true = np.ascontiguousarray(synth.layered_velocity(shape, h, seed=4))
    v0 = synth.smooth(v_true, 8.0)
    g = Grid(n, n, n, h, Grid.stable_dt(4, h, float(max(v_true.max(), v0.max()))))
    src = synth.random_positions(nshots, n, n, k=20, seed=4, margin=16)
    rec = synth.surface_receivers(n, n, k=20, stride=2)
    wav = g.ricker(steps, 15.0)
    shots = [Shot([s], g.injection_weights([v0[s[2], s[1], s[0]]]), rec) for s in src]
    prob = MisfitProblem(g, steps, wav, shots, checkpoint_every=every)
    kt = g.kappa_from_velocity(v_true)
    choice = tune_grid(g)
    say(f"one-launch step tuned for {n}^3: tile variant {choice[0]}, workgroup order {choice[1]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sh in shots:
        sh.observed = prob.model(kt, sh)
    torch.cuda.synchronize()
    t_obs = time.perf_counter() - t0
    del kt
    say(f"observed data: {nshots} shots x {steps} steps x {len(rec)} receivers in {t_obs:.3f} s")
    v0_d = torch.from_numpy(v0.astype(np.float32)).cuda()
    prob.misfit_and_gradient(v0_d)                  # warm-up (allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, gv = prob.misfit_and_gradient(v0_d)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    say(f"J and dJ/dv: {t_grad:.3f} s (J = {J:.6e})")
    # central difference along a smooth direction of unit maximum (m/s)
    d = synth.smooth(np.random.default_rng(5).standard_normal(shape), 8.0)
    d = (d / np.abs(d).max()).astype(np.float32)
    dd = torch.from_numpy(d).cuda()
    t0 = time.perf_counter()
    jp = prob.misfit(v0_d + eps * dd)
    jm = prob.misfit(v0_d - eps * dd)
    torch.cuda.synchronize()
    t_fd = time.perf_counter() - t0
    fd = (jp - jm) / (2 * eps)
    ad = float((gv.double() * dd.double()).sum().item())
    cell_check = None
    if cells > 0:
        # 1e-3 relative velocity perturbations on seeded cells of the illuminated zone, each with the
        # sign of its gradient so the contributions add up; J+ - J- = 1/2 <d+ - d-, d+ + d- - 2 d_obs>
        # formed from the traces in FP64, so the two misfits never cancel in floating point
        rng = np.random.default_rng(6)
        ijk = np.stack([rng.integers(16, n - 16, cells), rng.integers(16, n - 16, cells),
                        rng.integers(24, min(n - 16, 100), cells)], axis=1)
        gh = gv.cpu().numpy().astype(np.float64)
        gsel = gh[ijk[:, 2], ijk[:, 1], ijk[:, 0]]
        sign = np.where(gsel >= 0, 1.0, -1.0)
        cell_check = []
        for rel in (1e-3, 1e-2, 3e-2):    # 1e-3 is the specified one; the larger ones lift the signal
            e = np.zeros(shape)           # above the FP32 noise of the traces
            e[ijk[:, 2], ijk[:, 1], ijk[:, 0]] = sign * rel * v0[ijk[:, 2], ijk[:, 1], ijk[:, 0]]
            t0 = time.perf_counter()
            kp = prob.kappa(torch.from_numpy((v0 + e).astype(np.float32)).cuda())
            km = prob.kappa(torch.from_numpy((v0 - e).astype(np.float32)).cuda())
            fd_c = 0.0
            for sh in shots:
                dp = prob.model(kp, sh).cpu().numpy().astype(np.float64)
                dm = prob.model(km, sh).cpu().numpy().astype(np.float64)
                ob = sh.observed.cpu().numpy().astype(np.float64)
                fd_c += 0.5 * float(np.sum((dp - dm) * (dp + dm - 2.0 * ob)))
            fd_c /= 2.0
            ad_c = float(np.sum(gh * e))
            row = {"cells": cells, "relative_perturbation": rel, "t_s": round(time.perf_counter() - t0, 2),
                   "adjoint": ad_c, "fd": fd_c, "rel_diff": abs(ad_c - fd_c) / max(abs(fd_c), 1e-300)}
            cell_check.append(row)
            say(f"{cells}-cell check: {json.dumps(row)}")
    out = {"grid": [n, n, n], "shots": nshots, "steps": steps, "receivers": int(len(rec)), "checkpoint_every": every,
           "schedule": prob.schedule, "t_observed_s": round(t_obs, 4), "t_misfit_and_gradient_s": round(t_grad, 4),
           "t_two_misfits_s": round(t_fd, 4), "J": J, "directional_adjoint": ad, "directional_fd": fd,
           "eps_m_per_s": eps, "rel_diff": abs(ad - fd) / max(abs(fd), 1e-300),
           "gradient_finite": bool(torch.isfinite(gv).all().item()), "cell_check": cell_check}
    print(json.dumps(out), flush=True)


def _csv(d: str, name: str):
    files = glob.glob(os.path.join(d, "**", name), recursive=True)
    if not files:
        raise FileNotFoundError(f"no {name} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _counter(rows, kernel_substr: str, counter: str, largest: bool = False):
    vals = [float(r["Counter_Value"]) for r in rows if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        return None, 0
    return (max(vals) if largest else sum(vals) / len(vals)), len(vals)


def kernel_source_hash() -> str:
    """Hash of what the counted traffic depends on: the kernel source and the field layout."""
    h = hashlib.sha256()
    for part in (("csrc", "rtm.hip"), ("grid.py",)):
        with open(os.path.join(ROOT, "paper_1603_03971_amd", *part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def summarize(stats_dir, fetch_dir, write_dir, out, n, commands, kernel="whole_slots"):
    """Kernel statistics of a benchmark run, the stencil launches by call, and the counter traffic of
    the dominant call (`kernel`: "whole_slots" for the shell form, "interior" for the halo-region
    form); writes the summary and the traffic record that bench.py reads."""
    stats = _csv(stats_dir, "*kernel_stats.csv")
    lines = ["# rocprofv3 summary: 512^3 layered forward workload", ""]
    lines += ["Commands:"] + [f"    {c}" for c in commands] + [""]
    lines.append("Kernel statistics (kernel trace of the benchmark run):")
    lines.append(f"    {'kernel':60s} {'calls':>6s} {'avg us':>10s} {'share %':>8s}")
    for r in stats[:12]:
        name = r["Name"].replace("(anonymous namespace)::", "")[:60]
        avg = float(r["AverageNs"]) / 1e3
        lines.append(f"    {name:60s} {r['Calls']:>6s} {avg:10.2f} {float(r['Percentage']):8.2f}")
    # the radius-4 stencil dispatches of the run by call, from their kernel names
    kinds = [(WHOLE_SLOTS_KERNEL, "rtm_step_whole_slots"), (INTERIOR_KERNEL, "rtm_step_interior"),
             (WHOLE_KERNEL, "rtm_step_whole (fused schedule)"), (SHELL_KERNEL, "rtm_step_shell_pack"),
             (HALO_KERNEL, "rtm_step_halo_pack_slots")]
    trace = _csv(stats_dir, "*kernel_trace.csv")
    calls, grids = {}, {}
    for r in trace:
        for sub, what in kinds:
            if sub in r["Kernel_Name"]:
                calls.setdefault(what, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
                grids.setdefault(what, set()).add(int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]))
                break
    if calls:
        lines += ["", "Radius-4 stencil launches by call (kernel trace):",
                  f"    {'call':34s} {'workgroups':>10s} {'calls':>6s} {'avg us':>10s}"]
        for _, what in kinds:
            d = calls.get(what)
            if d:
                wg = ",".join(str(x) for x in sorted(grids[what]))
                lines.append(f"    {what:34s} {wg:>10s} {len(d):6d} {sum(d) / len(d):10.2f}")
    sub, name, pts = ((WHOLE_SLOTS_KERNEL, "rtm_step_whole_slots", n ** 3) if kernel == "whole_slots"
                      else (INTERIOR_KERNEL, "rtm_step_interior", interior_cells(n)))
    d = calls.get(name, [])
    avg_us = sum(d) / len(d) if d else None
    record = {"n": n, "kernel_source_sha256_16": kernel_source_hash(), "kernel": name, "avg_us_kernel_trace": avg_us}
    if fetch_dir and write_dir:
        fr, wr = _csv(fetch_dir, "*counter_collection.csv"), _csv(write_dir, "*counter_collection.csv")
        f_k, nf = _counter(fr, sub, "FETCH_SIZE")
        w_k, nw = _counter(wr, sub, "WRITE_SIZE")
        # the 1 GiB copy is the largest copy dispatch of the run
        f_cp, _ = _counter(fr, "opy", "FETCH_SIZE", largest=True)
        w_cp, _ = _counter(wr, "opy", "WRITE_SIZE", largest=True)
        kf = COPY_BYTES / (f_cp * 1024.0)
        kw = COPY_BYTES / (w_cp * 1024.0)
        traffic = f_k * 1024.0 * kf + w_k * 1024.0 * kw
        lines += ["", f"HBM traffic of the {name} launch (counters, KiB per dispatch):",
                  f"    FETCH_SIZE {f_k:.0f} KiB ({nf} dispatches), WRITE_SIZE {w_k:.0f} KiB ({nw} dispatches)",
                  f"    calibration with a plain 1 GiB device copy: FETCH x {kf:.3f}, WRITE x {kw:.3f}",
                  f"    traffic per launch {traffic / 1e6:.1f} MB; algorithmic 16 B x {pts} cells = {16 * pts / 1e6:.1f} MB"
                  f" (ratio {traffic / (16 * pts):.3f})"]
        record.update({"fetch_kib": f_k, "write_kib": w_k, "fetch_factor": kf, "write_factor": kw,
                       "hbm_bytes_per_launch": traffic, "algorithmic_bytes_per_launch": 16 * pts})
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    with open(os.path.splitext(out)[0] + "_traffic.txt", "w") as f:
        json.dump(record, f)
        f.write("\n")
    print(text)


def summarize_halo(fetch_dir, write_dir, out, n, commands, stats_dir=None):
    """HBM traffic of the halo call from the FETCH_SIZE / WRITE_SIZE runs of `halo`."""
    fr, wr = _csv(fetch_dir, "*counter_collection.csv"), _csv(write_dir, "*counter_collection.csv")
    f_h, nf = _counter(fr, HALO_KERNEL, "FETCH_SIZE")
    w_h, nw = _counter(wr, HALO_KERNEL, "WRITE_SIZE")
    f_cp, _ = _counter(fr, "opy", "FETCH_SIZE", largest=True)
    w_cp, _ = _counter(wr, "opy", "WRITE_SIZE", largest=True)
    kf = COPY_BYTES / (f_cp * 1024.0)
    kw = COPY_BYTES / (w_cp * 1024.0)
    rd, wt = f_h * 1024.0 * kf, w_h * 1024.0 * kw
    pts = n**3 - interior_cells(n)
    fc = 6 * 4 * n * n                         # face cells the call also writes, ghost cells it reads
    alg_r = 12 * pts + 4 * fc
    alg_w = 4 * (pts + fc)
    lines = [f"# rocprofv3 summary: HBM traffic of the halo call, {n}^3 layered forward workload", "",
             "Commands:"] + [f"    {c}" for c in commands] + [""]
    lines += ["Halo call of the halo-region form (bench.py --halo region; rtm_step_halo_pack_slots: two 4-plane",
              "z slabs, two 8-row y strips, two 64-column x strips; the ghosts read from six receive slots,",
              "the six 4-wide faces written to the face buffer):",
              f"    cells {pts} (the interior call's box is the rest), face cells {fc} (as many ghost cells)",
              f"    FETCH_SIZE {f_h:.0f} KiB ({nf} dispatches), WRITE_SIZE {w_h:.0f} KiB ({nw} dispatches)",
              f"    calibration with a plain 1 GiB device copy: FETCH x {kf:.3f}, WRITE x {kw:.3f}",
              f"    read {rd / 1e6:.1f} MB against 12 B x cells + 4 B x ghost cells = {alg_r / 1e6:.1f} MB "
              f"(ratio {rd / alg_r:.3f})",
              f"    written {wt / 1e6:.1f} MB against 4 B x (cells + face cells) = {alg_w / 1e6:.1f} MB "
              f"(ratio {wt / alg_w:.3f})",
              f"    total {(rd + wt) / 1e6:.1f} MB per launch, {(rd + wt) / (alg_r + alg_w):.3f} x algorithmic"]
    if stats_dir:
        for r in _csv(stats_dir, "*kernel_stats.csv"):
            if HALO_KERNEL in r["Name"]:
                us = float(r["AverageNs"]) / 1e3
                lines.append(f"    kernel trace (--stats run): {us:.1f} us per launch -> "
                             f"{(alg_r + alg_w) / us / 1e6:.2f} TB/s algorithmic, "
                             f"{(rd + wt) / us / 1e6:.2f} TB/s moved")
                break
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    print(text)


STREAM_ARRAYS = {"triad_range": 4, "triad": 4, "copy": 2, "read3": 3}   # arrays of 512^3 floats per launch


def summarize_stream(trace_dir, out, commands):
    """Average duration and bytes per second of each probe kernel at each grid size."""
    rows = _csv(trace_dir, "*kernel_trace.csv")
    groups = {}
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
        if name not in STREAM_ARRAYS:
            continue
        wg = int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])
        groups.setdefault((name, wg), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["# rocprofv3 summary: streaming bandwidth reference on one MI355X (arrays of 512^3 floats)", "",
             "Commands:"] + [f"    {c}" for c in commands] + [""]
    lines += ["triad: out = a + b c (3 reads + 1 write, the stencil's mix; streaming hints on b, c, out),",
              "grid-stride; triad_range: the same, one contiguous range per workgroup; copy: 1 read + 1 write;",
              "read3: 3 reads.  Kernel trace, 21 launches per case (the first is a warm-up):", "",
              f"    {'kernel':12s} {'workgroups':>10s} {'launches':>8s} {'avg us':>9s} {'TB/s':>6s}"]
    best = {}
    for (name, wg), d in sorted(groups.items(), key=lambda kv: (list(STREAM_ARRAYS).index(kv[0][0]), kv[0][1])):
        d = d[1:] if len(d) > 1 else d
        us = sum(d) / len(d)
        tbs = STREAM_ARRAYS[name] * 512 ** 3 * 4 / us / 1e6
        best[name] = max(best.get(name, 0.0), tbs)
        lines.append(f"    {name:12s} {wg:10d} {len(d):8d} {us:9.1f} {tbs:6.2f}")
    lines += ["", "Best per kernel: " + ", ".join(f"{k} {v:.2f} TB/s" for k, v in best.items())]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    print(text)


def summarize_markers(trace_dir, out, commands):
    """Phase sequence of the benchmark's steps from a marker trace (RTM_OPT_MARKERS): the calls of
    one halo-first step in order, host time per call, and the GPU time of the kernels each step
    launched, from the first kernel after the step's first call to the last before the next step."""
    marks = sorted(_csv(trace_dir, "*marker_api_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    kern = sorted(_csv(trace_dir, "*kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    names = {r["Function"] for r in marks}
    first = "rtm_step_shell_pack" if "rtm_step_shell_pack" in names else "rtm_step_halo_pack_slots"
    step_kernel = SHELL_KERNEL if first == "rtm_step_shell_pack" else HALO_KERNEL
    starts = [i for i, r in enumerate(marks) if r["Function"] == first]
    lines = ["# rocprofv3 summary: phase markers of the 512^3 halo-first benchmark step", "", "Commands:"]
    lines += [f"    {c}" for c in commands] + [""]
    if len(starts) < 3:
        lines.append("fewer than three halo-first steps in the trace")
    else:
        seq = [marks[i]["Function"] for i in range(starts[1], starts[2])]
        lines += ["Calls of one halo-first step, in order (host side, each a roctx range):",
                  "    " + " -> ".join(seq), ""]
        stats = {}
        for r in marks[starts[0]:starts[-1]]:
            stats.setdefault(r["Function"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        lines.append(f"    {'call':30s} {'calls':>6s} {'host us per call':>17s}")
        for name, d in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
            lines.append(f"    {name:30s} {len(d):6d} {sum(d) / len(d):17.1f}")
        # the GPU side from the kernel trace alone: a step's kernels run from its halo call's kernel
        # to the next step's (the host enqueues ahead, so host and GPU times do not line up)
        halo = [i for i, k in enumerate(kern) if step_kernel in k["Kernel_Name"]]
        per, rows = [], {}
        for a, b in zip(halo[:-1], halo[1:]):
            per.append((int(kern[b]["Start_Timestamp"]) - int(kern[a]["Start_Timestamp"])) / 1e3)
            prev_end = None
            for pos, k in enumerate(kern[a:b]):
                name = k["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0][:44]
                t0, t1 = int(k["Start_Timestamp"]), int(k["End_Timestamp"])
                gap = (t0 - prev_end) / 1e3 if prev_end is not None else 0.0
                rows.setdefault((pos, name), []).append(((t1 - t0) / 1e3, gap))
                prev_end = t1
        if per:
            med = lambda v: sorted(v)[len(v) // 2]
            lines += ["", f"GPU side, from the kernel trace ({len(per)} steps): median step period {med(per):.1f} us",
                      f"    {'kernel (in launch order)':46s} {'median us':>10s} {'gap before':>11s}"]
            for (pos, name), d in sorted(rows.items()):
                lines.append(f"    {name:46s} {med([x[0] for x in d]):10.1f} {med([x[1] for x in d]):11.1f}")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    print(text)


def summarize_corrected(stats_dir, out, n, steps, every, commands):
    """Per-step and per-correction costs of the `corrected` run from its kernel statistics."""
    rows = _csv(stats_dir, "*kernel_stats.csv")
    lines = [f"# rocprofv3 summary: corrected coarse propagation, {n}^3 coarse grid (radius 2, the companion of a",
             f"# {2 * n}^3 fine grid), point source, {steps} steps in the fused schedule, the corrector applied "
             f"every {every} steps", "", "Commands (from /tmp, TMPDIR=/tmp, PYTHONPATH=<repo root>):"]
    lines += [f"    {c}" for c in commands] + [""]
    lines += ["Kernel statistics (k_conv3d<TY, IN, OUT>: <4, 1, 0> is the first layer reading the wavefield,",
              "<4, 0, 0> the middle layer, <4, 0, 1> the last layer applying the correction to the levels):",
              f"    {'kernel':60s} {'calls':>6s} {'avg us':>9s} {'total ms':>9s} {'share %':>8s}"]
    tot, avg, calls = {}, {}, {}
    for i, r in enumerate(rows):
        name = r["Name"].replace("(anonymous namespace)::", "")
        tot[name] = float(r["TotalDurationNs"]) / 1e3
        avg[name] = float(r["AverageNs"]) / 1e3
        calls[name] = int(r["Calls"])
        if i < 12:
            lines.append(f"    {name[:60]:60s} {r['Calls']:>6s} {avg[name]:9.1f} {tot[name] / 1e3:9.2f} "
                         f"{float(r['Percentage']):8.2f}")

    def total(*subs):
        return sum(v for k, v in tot.items() if any(x in k for x in subs))
    ncorr = max(1, sum(v for k, v in calls.items() if "k_absmax_" in k))   # one scale per correction
    update = [v for k, v in avg.items() if "k_tiled<2," in k]
    step = total("k_tiled<2,", "k_inject", "k_unpack") / steps
    corr = total("k_conv3d", "k_absmax_", "k_zero1", "k_pack(", "k_pack<") / ncorr
    lines += ["", f"Per coarse step (one-launch update, inject, ghost refresh): {step:.0f} us"
                  + (f" (the update {update[0]:.0f} us)" if update else ""),
              f"Per correction (scale, first layer with the input packing, middle layer, last layer applying the "
              f"correction): {corr / 1e3:.2f} ms",
              f"    -> corrected propagation {step + corr / every:.0f} us per coarse step at K = {every}"]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    print(text)


def summarize_conv(stats_dir, out, n, commands):
    """Per-launch time, MFMA rate and traffic of the `conv` run's forward convolutions."""
    rows = _csv(stats_dir, "*kernel_stats.csv")
    lines = [f"# rocprofv3 summary: corrector network forward pass on a {n}^3 volume (three 3x3x3 convolutions,",
             "# 16 -> 16 channels, BF16 MFMA 16x16x32 with FP32 accumulation)", "",
             "Commands (from /tmp, TMPDIR=/tmp, PYTHONPATH=<repo root>):"]
    lines += [f"    {c}" for c in commands] + ["", "Kernel statistics:",
                                                f"    {'kernel':64s} {'calls':>6s} {'avg us':>10s} {'share %':>8s}"]
    calls, total_ns = 0, 0.0
    for i, r in enumerate(rows):
        name = r["Name"].replace("(anonymous namespace)::", "")
        if i < 8:
            lines.append(f"    {name[:64]:64s} {r['Calls']:>6s} {float(r['AverageNs']) / 1e3:10.2f} "
                         f"{float(r['Percentage']):8.2f}")
        if "k_conv3d<" in name:
            calls += int(r["Calls"])
            total_ns += float(r["TotalDurationNs"])
    if calls:
        avg = total_ns / calls / 1e9
        flop = n ** 3 * 27 * 16 * 16 * 2
        nbytes = n ** 3 * 64
        lines += ["", "Derived (per launch, algorithmic; the average over the three layers):",
                  f"    {calls} launches, {avg * 1e6:.1f} us each",
                  f"    work: {n}^3 voxels x 27 taps x 16 x 16 x 2 = {flop / 1e9:.1f} GFLOP -> {flop / avg / 1e12:.0f} "
                  f"TFLOP/s = {100 * flop / avg / 2.5e15:.1f}% of the 2.5 PFLOP/s BF16 dense peak",
                  "    (the MFMA issue count is 10/9 of that: the nine in-plane taps run as five tap pairs)",
                  f"    bytes: 32 B read + 32 B written per voxel (BF16, 16 channels) = {nbytes / 1e9:.2f} GB -> "
                  f"{nbytes / avg / 1e12:.2f} TB/s = {100 * nbytes / avg / 8e12:.0f}% of 8 TB/s",
                  "    (the last layer writes 2 FP32 channels instead; the rim re-read of a 64 x 4 tile adds up to "
                  "1.5x on the input side, partly caught in L2)"]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("interior")
    a.add_argument("--n", type=int, default=512)
    a.add_argument("--launches", type=int, default=10)
    hl = sub.add_parser("halo")
    hl.add_argument("--n", type=int, default=512)
    hl.add_argument("--launches", type=int, default=10)
    ws = sub.add_parser("whole-slots")
    ws.add_argument("--n", type=int, default=512)
    ws.add_argument("--launches", type=int, default=10)
    bh = sub.add_parser("summarize-halo")
    bh.add_argument("--fetch", required=True)
    bh.add_argument("--write", required=True)
    bh.add_argument("--stats")
    bh.add_argument("--out", required=True)
    bh.add_argument("--n", type=int, default=512)
    bh.add_argument("--command", action="append", default=[])
    kn = sub.add_parser("kernels")
    kn.add_argument("--n", type=int, default=512)
    kn.add_argument("--launches", type=int, default=10)
    ss = sub.add_parser("summarize-stream")
    ss.add_argument("--dir", required=True)
    ss.add_argument("--out", required=True)
    ss.add_argument("--command", action="append", default=[])
    sm = sub.add_parser("summarize-markers")
    sm.add_argument("--dir", required=True)
    sm.add_argument("--out", required=True)
    sm.add_argument("--command", action="append", default=[])
    sk = sub.add_parser("summarize-kernels")
    sk.add_argument("--fetch", required=True)
    sk.add_argument("--write", required=True)
    sk.add_argument("--stats")
    sk.add_argument("--out", required=True)
    sk.add_argument("--n", type=int, default=512)
    sk.add_argument("--command", action="append", default=[])
    cv = sub.add_parser("conv")
    cv.add_argument("--n", type=int, default=384)
    cv.add_argument("--launches", type=int, default=10)
    cr = sub.add_parser("corrected")
    cr.add_argument("--n", type=int, default=384)
    cr.add_argument("--steps", type=int, default=160)
    cr.add_argument("--every", type=int, default=16)
    sh = sub.add_parser("shot")
    sh.add_argument("--nx", type=int, default=512)
    sh.add_argument("--ny", type=int, default=512)
    sh.add_argument("--nz", type=int, default=256)
    sh.add_argument("--steps", type=int, default=2000)
    sh.add_argument("--every", type=int, default=4)
    sh.add_argument("--repeats", type=int, default=2)
    sh.add_argument("--schedule", default="fused", choices=["overlap", "serial", "fused"])
    gr = sub.add_parser("gradient")
    gr.add_argument("--n", type=int, default=256)
    gr.add_argument("--shots", type=int, default=8)
    gr.add_argument("--steps", type=int, default=1500)
    gr.add_argument("--every", type=int, default=50)
    gr.add_argument("--eps", type=float, default=2.5, help="central-difference step in m/s")
    gr.add_argument("--cells", type=int, default=64,
                    help="seeded cells perturbed by 1e-3 v for the finite-difference check (0: skip)")
    b = sub.add_parser("summarize")
    b.add_argument("--stats", required=True)
    b.add_argument("--fetch")
    b.add_argument("--write")
    b.add_argument("--out", required=True)
    b.add_argument("--n", type=int, default=512)
    b.add_argument("--kernel", default="whole_slots", choices=["whole_slots", "interior"])
    b.add_argument("--command", action="append", default=[])
    bc = sub.add_parser("summarize-corrected")
    bc.add_argument("--stats", required=True)
    bc.add_argument("--out", required=True)
    bc.add_argument("--n", type=int, default=384)
    bc.add_argument("--steps", type=int, default=160)
    bc.add_argument("--every", type=int, default=16)
    bc.add_argument("--command", action="append", default=[])
    bv = sub.add_parser("summarize-conv")
    bv.add_argument("--stats", required=True)
    bv.add_argument("--out", required=True)
    bv.add_argument("--n", type=int, default=384)
    bv.add_argument("--command", action="append", default=[])
    args = ap.parse_args(argv)
    if args.cmd == "interior":
        run_interior(args.n, args.launches)
    elif args.cmd == "halo":
        run_interior(args.n, args.launches, call="halo")
    elif args.cmd == "whole-slots":
        run_interior(args.n, args.launches, call="whole_slots")
    elif args.cmd == "summarize-halo":
        summarize_halo(args.fetch, args.write, args.out, args.n, args.command, args.stats)
    elif args.cmd == "kernels":
        run_kernels(args.n, args.launches)
    elif args.cmd == "summarize-stream":
        summarize_stream(args.dir, args.out, args.command)
    elif args.cmd == "summarize-markers":
        summarize_markers(args.dir, args.out, args.command)
    elif args.cmd == "summarize-kernels":
        summarize_kernels(args.fetch, args.write, args.stats, args.out, args.n, args.command)
    elif args.cmd == "conv":
        run_conv(args.n, args.launches)
    elif args.cmd == "corrected":
        run_corrected(args.n, args.steps, args.every)
    elif args.cmd == "gradient":
        run_gradient(args.n, args.shots, args.steps, args.every, args.eps, args.cells)
    elif args.cmd == "shot":
        run_shot(args.nx, args.ny, args.nz, args.steps, args.every, args.repeats, args.schedule)
    elif args.cmd == "summarize-conv":
        summarize_conv(args.stats, args.out, args.n, args.command)
    elif args.cmd == "summarize-corrected":
        summarize_corrected(args.stats, args.out, args.n, args.steps, args.every, args.command)
    else:
        summarize(args.stats, args.fetch, args.write, args.out, args.n, args.command, args.kernel)


if __name__ == "__main__":
    sys.exit(main())
