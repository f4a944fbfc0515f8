"""Parity where the interior call really runs: boxes wide enough that rtm_step_interior has full
64 x 8 tiles, several z chunks and the XCD remap, checked against the FP64 oracle cell by cell.

The halo region is x strips of 64 columns and y strips of 8 rows (rtm_halo_region), so any box at
most 128 cells wide in x leaves the interior call nothing to do; the boxes here are wider.
"""
import numpy as np
import pytest

import oracle
from paper_1603_03971_amd import synth
from tests import problems

pytestmark = pytest.mark.gpu


def _parse(schedule):
    """"sched[-ghosts[-halo]]" -> (sched, ghosts, halo), with "ring" and "region" by default."""
    parts = schedule.split("-")
    return parts[0], parts[1] if len(parts) > 1 else "ring", parts[2] if len(parts) > 2 else "region"


def _say(msg):
    print(msg, flush=True)


def _interior_box(shape):
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nz, ny, nx = shape
    g = Grid(nx, ny, nz, 10.0, 1e-3)
    wx, hy, R = _abi.rtm_halo_region(g.c)
    return (wx, nx - wx), (hy, ny - hy), (R, nz - R)


@pytest.fixture(scope="module")
def wide_case():
    """256 x 192 x 160 layered medium (seed 7), sources in the interior box, in an x strip, in a
    z slab, and one on the seam between the interior box and an x strip; 300 steps (0.15 s, past
    the 15 Hz wavelet's peak at 0.1 s), receivers 8-25 cells from the sources, on both sides of
    the seams."""
    shape = (160, 192, 256)
    v = np.array(synth.layered_velocity(shape, 10.0, seed=7))
    src = [(150, 100, 80), (20, 90, 70), (200, 50, 2), (64, 96, 90)]
    rec = [(150, 100, 62), (130, 96, 80), (64, 110, 90), (63, 110, 90), (20, 90, 55), (200, 40, 12),
           (200, 66, 4)]
    nsteps = 300
    _say("wide 256x192x160: oracle")
    ref = problems.oracle_forward_problem(v, 10.0, nsteps, src, rec_ijk=rec)
    return v, src, rec, nsteps, ref


def test_wide_box_exercises_full_interior_tiles(wide_case):
    """The case really gives the interior call full tiles and at least two z chunks."""
    v = wide_case[0]
    (x0, x1), (y0, y1), (z0, z1) = _interior_box(v.shape)
    assert (x1 - x0) % 64 == 0 and (x1 - x0) // 64 >= 2
    assert (y1 - y0) % 8 == 0 and (y1 - y0) // 8 >= 16
    assert z1 - z0 >= 2 * 16
    ref = wide_case[4]["u_cur"]
    inner = np.max(np.abs(ref[z0:z1, y0:y1, x0:x1]))
    assert inner >= 0.3 * np.max(np.abs(ref))       # the wavefield is really there


@pytest.mark.parametrize("schedule", ["serial", "overlap", "fused", "serial-slots", "overlap-slots",
                                      "serial-slots-shell", "overlap-slots-shell"])
def test_wide_box_parity(wide_case, schedule):
    """-slots: the steps with no unpack pass, whose halo calls read the ghosts from the receive slots;
    -shell: the halo call computes only the faces, the second call every owned cell."""
    v, src, rec, nsteps, ref = wide_case
    _say(f"wide {schedule}: gpu")
    sched, ghosts, halo = _parse(schedule)
    gpu = problems.gpu_forward_problem(v, 10.0, nsteps, src, rec_ijk=rec, schedule=sched, ghosts=ghosts, halo=halo)
    e_u = problems.rel_l2(gpu["u_cur"], ref["u_cur"])
    e_p = problems.rel_l2(gpu["u_prv"], ref["u_prv"])
    e_t = problems.rel_l2(gpu["traces"], ref["traces"])
    scale = float(np.max(np.abs(ref["u_cur"])))
    worst = float(np.max(np.abs(gpu["u_cur"] - ref["u_cur"]))) / scale
    (x0, x1), (y0, y1), (z0, z1) = _interior_box(v.shape)
    sub = (slice(z0, z1), slice(y0, y1), slice(x0, x1))
    e_in = problems.rel_l2(gpu["u_cur"][sub], ref["u_cur"][sub])
    _say(f"wide {schedule}: rel-L2 u^N {e_u:.2e} u^N-1 {e_p:.2e} traces {e_t:.2e} interior box {e_in:.2e}, "
         f"max |diff| / max |u| {worst:.2e}")
    assert e_u <= 1e-4 and e_p <= 1e-4 and e_t <= 1e-4 and e_in <= 1e-4
    assert worst <= 1e-5


def test_wide_box_interior_call_alone_matches_oracle(wide_case):
    """One interior call on its own: a seeded random state, the halo call's cells poisoned with NaN in
    the output, so the comparison covers exactly the interior box (full tiles, every z chunk)."""
    import torch

    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    v = wide_case[0]
    nz, ny, nx = v.shape
    dt = Grid.stable_dt(4, 10.0, float(v.max()))
    g = Grid(nx, ny, nz, 10.0, dt)
    u0 = synth.random_field(v.shape, seed=301)
    um = synth.random_field(v.shape, seed=302)
    uc, up = g.upload(u0), g.upload(um)
    kap = g.kappa_from_velocity(v)
    out = g.field(fill=float("nan"))
    _abi.rtm_step_interior(g.c, out, uc, up, kap, torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = g.download(out)
    dto = oracle.stable_dt(4, 10.0, float(v.max()))
    sp = tuple(oracle.sponge_profile(n, 16) for n in (nx, ny, nz))
    ref = oracle.step(u0.astype(np.float32), um.astype(np.float32), oracle.kappa_field(v, dto, 10.0), sp, 4, False,
                      problems.host_threads())
    (x0, x1), (y0, y1), (z0, z1) = _interior_box(v.shape)
    sub = (slice(z0, z1), slice(y0, y1), slice(x0, x1))
    assert np.all(np.isfinite(got[sub]))
    mask = np.ones(v.shape, dtype=bool)
    mask[sub] = False
    assert np.all(np.isnan(got[mask]))           # nothing outside the interior box was written
    e = problems.rel_l2(got[sub], ref[sub])
    worst = float(np.max(np.abs(got[sub] - ref[sub]))) / float(np.max(np.abs(ref[sub])))
    _say(f"interior call alone: rel-L2 {e:.2e}, max |diff| / max {worst:.2e}")
    assert e <= 1e-6 and worst <= 1e-6
