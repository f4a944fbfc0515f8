"""Benchmark: forward propagation at scale on one MI355X.

Workload: 512^3 cells, h = 10 m, seeded layered medium (20 layers, 1500-4500 m/s, Gaussian-smoothed
with sigma = 3 cells, seed 2), radius-4 star stencil with leapfrog, dt at half the stability limit,
15 Hz Ricker point source at the centre, 16-cell sponge, and the halo-first step schedule with all
six 4-wide faces exchanged on the device (one subdomain's share: the faces go out to a send buffer,
and the ghosts come in from six receive slots of a zero-filled receive buffer, as from neighbours
that sent zero faces).  A step is one pass of the whole per-step sequence.  By default (--halo shell):
the shell call (the owned cells within 4 of a face computed into the send buffer, reading the ghosts
from the receive slots), the call over every owned cell (the shell again included, full-width tiles,
the same ghosts), source injection, receiver recording.  With --halo region: the halo call over the
halo region (writing the faces to the send buffer as it goes), source injection, the interior stencil,
recording; with --ghosts ring (and --halo region) the received faces are also unpacked into the ghost
ring by a pass of their own after the interior stencil.

Prints one JSON line: G point-updates/s over the timed steps, the dominant kernel's achieved HBM
bandwidth against the 8 TB/s peak (algorithmic bytes / HIP-event kernel time), and the FP64 CPU
oracle timed on the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT = 16          # read u^n, u^{n-1}, kappa; write u^{n+1} (FP32)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "forward_512_layered_traffic.txt")
# the dominant call (the whole-block call, or the interior call with --halo region) is timed with HIP
# events on every EVENT_EVERY-th timed step counted from the first (100 launches of 1000; at least one
# in any run): each event pair makes the step it brackets about 11 us longer (an event waits for the
# kernel before it and writes back the caches), which the other steps then do not pay
EVENT_EVERY = 10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="cells per axis")
    ap.add_argument("--schedule", default="serial", choices=["overlap", "serial"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--phases", action="store_true", help="also time each phase separately (serial)")
    ap.add_argument("--markers", action="store_true",
                    help="roctx ranges around every per-step call (for rocprofv3 --marker-trace)")
    ap.add_argument("--ghosts", default="slots", choices=["slots", "ring"],
                    help="slots: the halo call reads the ghosts from the receive slots; ring: an unpack pass")
    ap.add_argument("--halo", default=None, choices=["shell", "region"],
                    help="shell (default with --ghosts slots): the halo call computes only the faces and the "
                         "second call every owned cell; region: the halo region, then the interior")
    args = ap.parse_args()
    if args.halo is None:
        args.halo = "shell" if args.ghosts == "slots" else "region"
    if args.halo == "shell" and args.ghosts != "slots":
        ap.error("--halo shell reads the ghosts from the receive slots (--ghosts slots)")
    return args


def kernel_source_hash() -> str:
    """Hash of what the counted traffic depends on: the kernel source and the field layout."""
    h = hashlib.sha256()
    for part in (("csrc", "rtm.hip"), ("grid.py",)):
        with open(os.path.join(ROOT, "paper_1603_03971_amd", *part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def host_threads() -> int:
    """Every core this process may run on (the oracle's result does not depend on the count)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, n)


def cpu_baseline(n: int, h: float, v_prof, target_s: float):
    """FP64 oracle steps on the same 512^3 layered model, on the host cores, for about target_s."""
    import numpy as np

    import oracle

    threads = host_threads()
    v = np.broadcast_to(v_prof[:, None, None], (n, n, n))
    dt = oracle.stable_dt(4, h, float(v_prof.max()))
    kap = oracle.kappa_field(v, dt, h)
    sp = oracle.sponge_profile(n, 16, 0.015)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((n, n, n))
    up = rng.standard_normal((n, n, n))
    out = np.empty_like(u)
    t0 = time.perf_counter()
    steps = 0
    while True:
        oracle.step(u, up, kap, (sp, sp, sp), 4, False, threads, out=out)
        steps += 1
        el = time.perf_counter() - t0
        if el >= target_s or steps >= 200:
            break
    # one more step on a single thread (the multi-threaded step is bitwise the same)
    t1 = time.perf_counter()
    oracle.step(u, up, kap, (sp, sp, sp), 4, False, 1, out=out)
    el1 = time.perf_counter() - t1
    return {"value": n ** 3 * steps / el / 1e9, "unit": "Gpts/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps of the {n}^3 layered workload (random wavefield), "
                      f"{threads} OpenMP threads, {el:.1f} s",
            "single_thread": {"value": n ** 3 / el1 / 1e9, "unit": "Gpts/s", "sample": f"1 step, {el1:.1f} s"},
            "host": {"nproc": os.cpu_count(), "cpu": cpu_model()}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1603_03971_amd import _abi, synth
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    assert torch.cuda.is_available(), "needs a GPU"
    if args.markers:
        _abi.rtm_set_option(_abi.RTM_OPT_MARKERS, 1)
    n, h = args.n, 10.0
    shape = (n, n, n)
    prof = synth.layered_profile(n, h, seed=2)
    vmax = float(prof.max())
    dt = Grid.stable_dt(4, h, vmax)
    g = Grid(n, n, n, h, dt)
    v_dev = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(prof[:, None, None], shape), dtype=np.float32))
    kap = g.kappa_from_velocity(v_dev.cuda())
    del v_dev
    total_steps = args.warmup + args.steps
    c = n // 2
    src = Sources(g, [(c, c, c)], g.injection_weights([prof[c]]), g.ricker(total_steps, 15.0)[:, None])
    rec = synth.surface_receivers(n, n, k=20, stride=16)           # a sparse 32 x 32 surface spread
    prop = Propagator(g, kap, sources=src, receivers=rec, schedule=args.schedule, boundary="zero_faces",
                      ghosts=args.ghosts, halo=args.halo)
    traces = prop.new_traces(total_steps)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        prop.step(traces)
    prop.sync()
    torch.cuda.synchronize()

    prop.interior_events = []
    prop.interior_event_every = EVENT_EVERY
    prop.interior_event_start = prop.n
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prop.step(traces)
    prop.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    finite = bool(torch.isfinite(traces).all().item())
    pts = g.points
    value = pts * args.steps / wall / 1e9
    if args.halo == "shell":
        step_text = ("halo-first: a shell call computing the 6 x 4-wide faces into a send buffer, then one call "
                     "over every owned cell (the shell again included), both reading the ghosts from "
                     "zero-filled receive slots (no unpack pass)")
    elif args.ghosts == "slots":
        step_text = ("halo-first with 6 x 4-wide faces packed to a send buffer and read by the next halo call "
                     "from zero-filled receive slots (no unpack pass)")
    else:
        step_text = ("halo-first with 6 x 4-wide faces packed to a send buffer and unpacked from zero-filled "
                     "receive slots")
    result = {
        "metric": "Gpoint-updates/s", "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"forward {n}^3 layered (20 layers 1500-4500 m/s, sigma 3, seed 2), radius-4 "
                               f"8th-order star, leapfrog, dt at half the stability limit, 15 Hz Ricker at the "
                               f"centre, 16-cell sponge, {step_text}, {args.steps} timed steps",
                   "grid": [n, n, n], "h_m": h, "dt_s": dt, "schedule": args.schedule, "ghosts": args.ghosts,
                   "halo": args.halo,
                   "receivers": int(len(rec))},
        "finite": finite,
    }
    # roofline of the dominant kernel (the whole-block call, or the interior call with --halo region),
    # timed with HIP events on the stream it runs on
    if prop.interior_events:
        ms = [a.elapsed_time(b) for a, b in prop.interior_events]
        avg_s = sum(ms) / len(ms) / 1e3
        if args.halo == "shell":
            kernel, cells = "rtm_step_whole_slots", pts
        else:
            wx, hy, R = _abi.rtm_halo_region(g.c)
            kernel, cells = "rtm_step_interior", (n - 2 * wx) * (n - 2 * hy) * (n - 2 * R)
        achieved = BYTES_PER_POINT * cells / avg_s / 1e9
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            with open(TRAFFIC_FILE) as f:
                t = json.load(f)
            if (t.get("kernel_source_sha256_16") == kernel_source_hash() and t.get("n") == n
                    and t.get("kernel") == kernel):
                traffic = t.get("hbm_bytes_per_launch")
        result["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                              "kernel": kernel, "avg_us": round(avg_s * 1e6, 2),
                              "launches_timed": len(ms),
                              "algorithmic_bytes_per_launch": BYTES_PER_POINT * cells}
        # whole-step roofline with the halo phases, counting the bytes each phase must move: the
        # stencil 16 B per cell; per face cell, the halo call stores the computed value into its
        # send slot (4 B; the value is in registers, not read back) and the received ghost is read
        # from its slot by the next step (4 B), or read and written into the ring by the unpack (8 B,
        # ghosts="ring"); the shell form's second computation of the face cells is not counted
        face_cells = 6 * 4 * n * n
        step_bytes = BYTES_PER_POINT * pts + (8 if args.ghosts == "slots" else 12) * face_cells
        result["step_hbm_frac"] = round(step_bytes / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, 4)
    if args.phases:
        result["phases_us"] = time_phases(g, prop, traces)
    result["device_copy"] = device_copy_rate()
    # the same steps in one launch each (rtm_step_whole, bitwise the same fields): what one GPU with
    # nothing to overlap can do; reported beside the halo-first value, not as it
    del prop
    fused = Propagator(g, kap, sources=src, receivers=rec, schedule="fused")
    fsteps = min(args.steps, 300)
    ftr = fused.new_traces(fsteps + 10)
    fused.run(10, ftr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fused.run(fsteps, ftr)
    torch.cuda.synchronize()
    fwall = time.perf_counter() - t0
    result["fused_schedule"] = {"value": round(pts * fsteps / fwall / 1e9, 3), "unit": "Gpts/s",
                                "ms_per_step": round(fwall / fsteps * 1e3, 4), "steps": fsteps,
                                "what": "one launch per step over all owned cells (rtm_step_whole), then inject "
                                        "and record (the zero ghost ring written once per buffer); bitwise the "
                                        "same fields as the halo-first sequence, which the value measures"}
    del fused
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(n, h, prof, args.cpu_seconds)
    print(json.dumps(result), flush=True)


def device_copy_rate(nbytes: int = 1 << 30, reps: int = 10):
    """Context for the roofline: a plain device-to-device copy (torch's copy, 1 GiB), bytes read plus
    bytes written per second."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return {"GBs": round(2 * nbytes / s / 1e9, 1), "what": "torch device-to-device copy of 1 GiB, read + written "
            "bytes per second (context, not a ceiling)"}


def time_phases(g, prop, traces, reps: int = 20):
    """Per-phase kernel time (the analogue of the paper's per-phase breakdown), one stream."""
    import torch

    from paper_1603_03971_amd import _abi

    st = torch.cuda.current_stream()
    c = g.c
    u_nxt, u_cur, u_prv = prop.u_prv, prop.u_cur, prop.u_prv
    recv = prop._recv_for(prop.n) if prop.ghosts == "slots" else prop.recv
    dense, shell_out = None, prop.send
    if prop.kappa_faces is not None:         # as the next step would run it: its own send buffer
        nb = len(prop.send_bufs)
        dense = (prop.send_bufs[(prop.n - 1) % nb], prop.send_bufs[(prop.n - 2) % nb], prop.kappa_faces)
        shell_out = prop.send_bufs[prop.n % nb]
    phases = {
        "halo": lambda: _abi.rtm_step_halo(c, u_nxt, u_cur, u_prv, prop.kappa, st),
        "pack": lambda: _abi.rtm_pack_halo(c, u_nxt, prop.send, st),
        "halo_pack": lambda: _abi.rtm_step_halo_pack(c, u_nxt, u_cur, u_prv, prop.kappa, prop.send, st),
        "halo_pack_slots": lambda: _abi.rtm_step_halo_pack_slots(c, u_nxt, u_cur, u_prv, prop.kappa, recv,
                                                                 prop.send, st),
        "unpack": lambda: _abi.rtm_unpack_halo(c, u_nxt, prop.recv, st),
        "interior": lambda: _abi.rtm_step_interior(c, u_nxt, u_cur, u_prv, prop.kappa, st),
        "shell_pack": lambda: _abi.rtm_step_shell_pack(c, u_cur, u_prv, prop.kappa, recv, shell_out, st,
                                                       dense=dense),
        "whole_slots": lambda: _abi.rtm_step_whole_slots(c, u_nxt, u_cur, u_prv, prop.kappa, recv, st),
        "record": lambda: _abi.rtm_record(c, u_nxt, prop.rec_idx, traces, prop.nrec, st),
    }
    out = {}
    for name, fn in phases.items():
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        out[name] = round(e0.elapsed_time(e1) / reps * 1e3, 2)
    return out


if __name__ == "__main__":
    main()
