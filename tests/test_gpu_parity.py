"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs.

Bars: FP32 wavefields within 1e-4 relative L2 of the oracle, images within 1e-3; copies (pack,
unpack, record) and schedule/variant comparisons bitwise.
"""
import math

import numpy as np
import pytest

import oracle
from tests import problems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1603_03971_amd import _abi  # noqa: F401  (fails loudly if the library is not built)
    return torch


def _say(msg):
    print(msg, flush=True)


def test_c1_point_source_parity(torch_cuda):
    """64^3 constant-velocity point source, 200 steps: final wavefield and traces vs the oracle."""
    v, h, nsteps, src = problems.c1_inputs()
    rec = [(32, 32, 8), (40, 32, 32), (32, 20, 32), (12, 50, 33)]
    _say("c1: gpu")
    gpu = problems.gpu_forward_problem(v, h, nsteps, src, rec_ijk=rec)
    _say("c1: oracle")
    ref = problems.oracle_forward_problem(v, h, nsteps, src, rec_ijk=rec)
    e_u = problems.rel_l2(gpu["u_cur"], ref["u_cur"])
    e_p = problems.rel_l2(gpu["u_prv"], ref["u_prv"])
    e_t = problems.rel_l2(gpu["traces"], ref["traces"])
    worst = float(np.max(np.abs(gpu["u_cur"] - ref["u_cur"]))) / float(np.max(np.abs(ref["u_cur"])))
    _say(f"c1 rel-L2: u^N {e_u:.3e}  u^N-1 {e_p:.3e}  traces {e_t:.3e}; max |diff| / max |u| {worst:.2e}")
    assert e_u <= 1e-4 and e_p <= 1e-4 and e_t <= 1e-4
    assert worst <= 1e-5


@pytest.mark.parametrize("schedule", ["overlap", "serial"])
def test_ragged_layered_parity(torch_cuda, schedule):
    """150 x 41 x 70 (ragged against every tile size), layered medium, sources inside and in the shell."""
    v, h, nsteps, src = problems.ragged_inputs()
    rec = [(1, 1, 1), (149, 40, 69), (75, 20, 35), (3, 39, 66)]
    _say(f"ragged {schedule}: gpu")
    gpu = problems.gpu_forward_problem(v, h, nsteps, src, rec_ijk=rec, schedule=schedule)
    ref = problems.oracle_forward_problem(v, h, nsteps, src, rec_ijk=rec)
    e_u = problems.rel_l2(gpu["u_cur"], ref["u_cur"])
    e_t = problems.rel_l2(gpu["traces"], ref["traces"])
    worst = float(np.max(np.abs(gpu["u_cur"] - ref["u_cur"]))) / float(np.max(np.abs(ref["u_cur"])))
    _say(f"ragged {schedule} rel-L2: u {e_u:.3e} traces {e_t:.3e}; max |diff| / max |u| {worst:.2e}")
    assert e_u <= 1e-4 and e_t <= 1e-4
    assert worst <= 1e-5


def test_schedules_and_variants_bitwise(torch_cuda):
    """Halo-first on two streams, single stream, the one-launch whole step, every interior and halo
    kernel variant and z chunking, and unaligned pitches (scalar path) all give the same bits."""
    from paper_1603_03971_amd import _abi

    v, h, nsteps, src = problems.ragged_inputs(seed=9)
    nsteps = 30
    base = problems.gpu_forward_problem(v, h, nsteps, src, schedule="serial")["u_cur"]
    runs = {}
    default_variant = _abi.rtm_get_option(_abi.RTM_OPT_INTERIOR_VARIANT)
    try:
        runs["overlap"] = problems.gpu_forward_problem(v, h, nsteps, src, schedule="overlap")["u_cur"]
        runs["fused"] = problems.gpu_forward_problem(v, h, nsteps, src, schedule="fused")["u_cur"]
        runs["fused_unaligned"] = problems.gpu_forward_problem(v, h, nsteps, src, schedule="fused", x_align=1)["u_cur"]
        for var in (0, 1, 2, 3, 4):
            _abi.rtm_set_option(_abi.RTM_OPT_INTERIOR_VARIANT, var)
            runs[f"variant{var}"] = problems.gpu_forward_problem(v, h, nsteps, src)["u_cur"]
            runs[f"variant{var}_fused"] = problems.gpu_forward_problem(v, h, nsteps, src, schedule="fused")["u_cur"]
        _abi.rtm_set_option(_abi.RTM_OPT_INTERIOR_VARIANT, default_variant)
        for var in (1, 2, 4, 5):
            _abi.rtm_set_option(_abi.RTM_OPT_HALO_VARIANT, var)
            runs[f"halo_variant{var}"] = problems.gpu_forward_problem(v, h, nsteps, src)["u_cur"]
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_VARIANT, 0)
        for var in (0, 1, 2, 4, 5):
            _abi.rtm_set_option(_abi.RTM_OPT_WHOLE_VARIANT, var)
            runs[f"whole_variant{var}"] = problems.gpu_forward_problem(v, h, nsteps, src, schedule="fused")["u_cur"]
        _abi.rtm_set_option(_abi.RTM_OPT_WHOLE_VARIANT, 6)
        for zc in (1, 7, 1000):
            _abi.rtm_set_option(_abi.RTM_OPT_ZCHUNK, zc)
            runs[f"zchunk{zc}"] = problems.gpu_forward_problem(v, h, nsteps, src)["u_cur"]
        _abi.rtm_set_option(_abi.RTM_OPT_ZCHUNK, 0)
        _abi.rtm_set_option(_abi.RTM_OPT_XCD_REMAP, 0)
        runs["noremap"] = problems.gpu_forward_problem(v, h, nsteps, src)["u_cur"]
        _abi.rtm_set_option(_abi.RTM_OPT_XCD_REMAP, 1)
        for fl in (0, 1, 2, 3):
            _abi.rtm_set_option(_abi.RTM_OPT_TILE_FLAGS, fl)
            runs[f"tile_flags{fl}"] = problems.gpu_forward_problem(v, h, nsteps, src)["u_cur"]
            runs[f"tile_flags{fl}_fused"] = problems.gpu_forward_problem(v, h, nsteps, src, schedule="fused")["u_cur"]
        _abi.rtm_set_option(_abi.RTM_OPT_TILE_FLAGS, 1)
        runs["x_align4"] = problems.gpu_forward_problem(v, h, nsteps, src, x_align=4)["u_cur"]
        runs["unaligned_pitch"] = problems.gpu_forward_problem(v, h, nsteps, src, x_align=1)["u_cur"]
    finally:
        _abi.rtm_set_option(_abi.RTM_OPT_INTERIOR_VARIANT, default_variant)
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_VARIANT, 0)
        _abi.rtm_set_option(_abi.RTM_OPT_WHOLE_VARIANT, 6)
        _abi.rtm_set_option(_abi.RTM_OPT_ZCHUNK, 0)
        _abi.rtm_set_option(_abi.RTM_OPT_XCD_REMAP, 1)
        _abi.rtm_set_option(_abi.RTM_OPT_TILE_FLAGS, 1)
    assert np.any(base != 0)
    for name, u in runs.items():
        assert np.array_equal(u, base), name


@pytest.mark.parametrize("hz", [0, 8])
def test_halo_and_interior_partition_owned_cells(torch_cuda, hz):
    """NaN-poisoned output: halo then interior write every owned cell exactly once (all finite), and
    neither touches a ghost cell; with the default z slabs (R planes) and with 8-plane slabs."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    _abi.rtm_set_option(_abi.RTM_OPT_HALO_Z_WIDTH, hz)
    try:
        _partition_cases(torch, _abi, Grid, hz)
    finally:
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_Z_WIDTH, 0)


def _partition_cases(torch, _abi, Grid, hz):
    for (nx, ny, nz) in ((150, 41, 70), (8, 8, 8), (9, 21, 13), (64, 64, 64), (200, 19, 12)):
        g = Grid(nx, ny, nz, 10.0, 1e-3)
        rng = np.random.default_rng(nx)
        u = g.upload(rng.standard_normal((nz, ny, nx)))
        up = g.upload(rng.standard_normal((nz, ny, nx)))
        kap = g.upload(rng.uniform(0.01, 0.05, (nz, ny, nx)))
        out = g.field(fill=float("nan"))
        s = torch.cuda.current_stream()
        _abi.rtm_step_halo(g.c, out, u, up, kap, s)
        halo_only = g.owned(out).clone()
        _abi.rtm_step_interior(g.c, out, u, up, kap, s)
        torch.cuda.synchronize()
        own = g.owned(out)
        assert torch.isfinite(own).all(), (nx, ny, nz)
        # the halo call wrote the R-shell widened to x strips of min(64, nx // 2) cells, y strips
        # of min(8, ny // 2) rows and z slabs of R or min(hz, nz // 2) planes
        R, wx, hy = 4, max(4, min(64, nx // 2)), max(4, min(8, ny // 2))
        zs = max(R, min(hz, nz // 2)) if hz else R
        assert _abi.rtm_halo_region(g.c) == (wx, hy, zs)
        shell = torch.zeros((nz, ny, nx), dtype=torch.bool, device=out.device)
        shell[:zs] = True
        shell[-zs:] = True
        shell[:, :hy] = True
        shell[:, -hy:] = True
        shell[:, :, :wx] = True
        shell[:, :, nx - wx:] = True
        assert torch.equal(torch.isfinite(halo_only), shell)
        pad = g.padded(out)
        ghost = torch.ones_like(pad, dtype=torch.bool)
        ghost[R:R + nz, R:R + ny, R:R + nx] = False
        assert torch.isnan(pad[ghost]).all()


def test_pack_unpack_bitwise(torch_cuda):
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nx, ny, nz = 37, 22, 19
    g = Grid(nx, ny, nz, 10.0, 1e-3)
    host = np.random.default_rng(3).standard_normal((nz, ny, nx)).astype(np.float32)
    u = g.upload(host)
    faces = g.faces()
    s = torch.cuda.current_stream()
    _abi.rtm_pack_halo(g.c, u, faces, s)
    torch.cuda.synchronize()
    got = g.face_slots(faces)
    want = oracle.pack_faces(host.astype(np.float64))
    for f in range(6):
        assert np.array_equal(got[f].cpu().numpy(), want[f].astype(np.float32)), f
    # unpack random slots into the ghosts; NULL slots give zeros
    slots = [torch.from_numpy(np.random.default_rng(10 + f).standard_normal(g.face_sizes[f]).astype(np.float32)).cuda()
             for f in range(6)]
    w = g.field(fill=7.0)
    _abi.rtm_unpack_halo(g.c, w, slots, s)
    z = g.field(fill=7.0)
    _abi.rtm_unpack_halo(g.c, z, [None] * 6, s)
    torch.cuda.synchronize()
    pad = g.padded(w).cpu().numpy()
    padz = g.padded(z).cpu().numpy()
    R = 4
    sl = [s_.cpu().numpy() for s_ in slots]
    ghost_blocks = [
        pad[R:R + nz, R:R + ny, 0:R], pad[R:R + nz, R:R + ny, R + nx:],
        pad[R:R + nz, 0:R, R:R + nx], pad[R:R + nz, R + ny:, R:R + nx],
        pad[0:R, R:R + ny, R:R + nx], pad[R + nz:, R:R + ny, R:R + nx],
    ]
    for f in range(6):
        assert np.array_equal(ghost_blocks[f].ravel(), sl[f]), f
    assert np.all(pad[R:R + nz, R:R + ny, R:R + nx] == 7.0)     # owned untouched
    assert pad[0, 0, 0] == 7.0                                    # corners untouched
    assert np.all(padz[R:R + nz, R:R + ny, 0:R] == 0.0)


@pytest.mark.parametrize("shape", [(64, 40, 36), (96, 9, 8), (32, 8, 12)])
def test_unpack_whole_lines(torch_cuda, shape):
    """On the line-aligned layout the x faces are unpacked as whole 128-byte lines (a row's +X ghost,
    its padding, the next row's -X ghost).  Every ghost and owned cell gets the bits of the 16-byte
    unpack; edge and corner ghosts stay untouched (NaN here), with real slots and with NULL ones."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nx, ny, nz = shape
    g = Grid(nx, ny, nz, 10.0, 1e-3)
    assert g.pitch_y == nx + 32                       # the layout the whole-line path needs
    s = torch.cuda.current_stream()
    host = np.random.default_rng(5).standard_normal((nz, ny, nx)).astype(np.float32)
    slots = [torch.from_numpy(np.random.default_rng(20 + f).standard_normal(g.face_sizes[f]).astype(np.float32)).cuda()
             for f in range(6)]
    for recv in (slots, [None] * 6, [slots[0], None, None, slots[3], slots[4], None]):
        out = {}
        for lines in (1, 0):
            _abi.rtm_set_option(_abi.RTM_OPT_UNPACK_LINES, lines)
            try:
                u = g.field(fill=float("nan"))
                g.upload(host, u)
                _abi.rtm_unpack_halo(g.c, u, recv, s)
                torch.cuda.synchronize()
            finally:
                _abi.rtm_set_option(_abi.RTM_OPT_UNPACK_LINES, 1)
            out[lines] = g.padded(u).cpu().numpy()
        assert np.array_equal(out[1], out[0], equal_nan=True)
        assert np.isnan(out[1][0, 0, 0]) and np.isnan(out[1][4, 3, 2]) and np.isnan(out[1][4, 4 + ny, 2])


def test_periodic_standing_wave(torch_cuda):
    """Periodic self-exchange (slot swap): the discrete dispersion relation's closed form and the
    oracle's periodic mode."""
    torch = torch_cuda
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator

    nx, ny, nz, h, v = 48, 24, 40, 10.0, 2000.0
    p0, (kx, ky, kz) = problems.plane_standing_wave(nx, ny, nz, h, v, (3, 2, 5))
    dt = Grid.stable_dt(4, h, v)
    c = [-205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560]
    sym = lambda t: c[0] + 2 * sum(c[m] * math.cos(m * t) for m in range(1, 5))
    lam = sym(kx * h) + sym(ky * h) + sym(kz * h)
    w = 2 / dt * math.asin(v * dt / (2 * h) * math.sqrt(-lam))
    g = Grid(nx, ny, nz, h, dt, sponge_width=0)
    kap = g.kappa_from_velocity(np.full((nz, ny, nx), v))
    nsteps = 200
    for schedule in ("overlap", "serial"):
        prop = Propagator(g, kap, boundary="periodic", schedule=schedule)
        prop.set_state(p0, p0 * math.cos(w * dt))
        prop.run(nsteps)
        torch.cuda.synchronize()
        u = g.download(prop.u_cur).astype(np.float64)
        exact = p0 * math.cos(w * nsteps * dt)
        err = np.max(np.abs(u - exact))
        _say(f"periodic {schedule}: max err vs closed form {err:.3e}")
        assert err < 2e-5
    ref = oracle.forward(oracle.kappa_field(np.full((nz, ny, nx), v), dt, h), None, nsteps, u_cur=p0,
                         u_prv=p0 * math.cos(w * dt), periodic=True, nthreads=8)
    assert problems.rel_l2(u, ref["u_cur"]) < 1e-4


@pytest.mark.parametrize("radius,shape,x_align", [(4, (48, 40, 36), 32), (4, (68, 36, 20), 32),
                                                    (4, (50, 40, 36), 32), (4, (48, 40, 36), 1),
                                                    (2, (48, 24, 20), 32)])
def test_halo_pack_equals_halo_then_pack(torch_cuda, radius, shape, x_align):
    """rtm_step_halo_pack gives the fields and the face buffer of rtm_step_halo then rtm_pack_halo,
    bitwise, for every halo tile shape (the fused path: radius 4, vectorised layout, nx % 4 == 0; the
    other cases take the two calls); after injecting into face, edge and corner cells, rtm_pack_cells
    brings the fused face buffer to what a fresh pack gives."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nx, ny, nz = shape
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(radius, 10.0, 3000.0), radius=radius, sponge_width=3,
             x_align=x_align)
    rng = np.random.default_rng(2100 + nx + radius)
    u, up = g.upload(rng.standard_normal(g.shape)), g.upload(rng.standard_normal(g.shape))
    kap = g.upload(rng.uniform(0.01, 0.05, g.shape))
    st = torch.cuda.current_stream()
    R = radius
    cells = np.array([[0, 5, 7], [nx - 1, ny - 1, nz - 1], [2, 0, nz // 2], [nx // 2, ny - 2, 1],
                      [nx // 2, ny // 2, nz - 3], [R, R, R], [nx // 2, ny // 2, nz // 2]])
    idx = torch.from_numpy(g.index(cells)).cuda()
    w = torch.full((len(cells),), 0.75, dtype=torch.float32, device="cuda")
    amp = torch.linspace(1.0, 2.0, len(cells), dtype=torch.float32, device="cuda")
    default = _abi.rtm_get_option(_abi.RTM_OPT_HALO_VARIANT)
    try:
        for var in (0, 1, 2, 4, 5):
            _abi.rtm_set_option(_abi.RTM_OPT_HALO_VARIANT, var)
            out_a, out_b = g.field(), g.field()
            fa, fb = g.faces(), g.faces()
            _abi.rtm_step_halo(g.c, out_a, u, up, kap, st)
            _abi.rtm_pack_halo(g.c, out_a, fa, st)
            _abi.rtm_step_halo_pack(g.c, out_b, u, up, kap, fb, st)
            torch.cuda.synchronize()
            assert torch.equal(out_a, out_b), var
            assert torch.equal(fa, fb), var
            assert fa.abs().max() > 0
            for out, f, fused in ((out_a, fa, False), (out_b, fb, True)):
                _abi.rtm_inject(g.c, out, idx, w, amp, len(cells), st)
                if fused:
                    _abi.rtm_pack_cells(g.c, out, idx, len(cells), f, st)
                else:
                    _abi.rtm_pack_halo(g.c, out, f, st)
            torch.cuda.synchronize()
            assert torch.equal(fa, fb), var
    finally:
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_VARIANT, default)


def test_periodic_face_sources_schedules_bitwise(torch_cuda):
    """Periodic self-exchange, where the packed faces become the ghosts, with sources in face, edge
    and corner cells: the halo-first schedules (faces packed by the halo call, injected face cells
    re-copied) equal the one-launch schedule (faces packed after the injection), bitwise."""
    torch = torch_cuda
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    nx, ny, nz = 48, 36, 32
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(4, 10.0, 3000.0), sponge_width=0)
    kap = g.kappa_from_velocity(np.random.default_rng(2200).uniform(2000.0, 3000.0, g.shape))
    cells = [(0, 10, 10), (nx - 1, 0, nz - 1), (20, 1, 15), (30, ny - 3, 2), (24, 18, 16)]
    nsteps = 40
    w = g.injection_weights([2500.0] * len(cells))
    amp = np.random.default_rng(2201).standard_normal((nsteps, len(cells))).astype(np.float32)
    out = {}
    for schedule in ("serial", "overlap", "fused"):
        prop = Propagator(g, kap, sources=Sources(g, cells, w, amp), boundary="periodic", schedule=schedule)
        prop.run(nsteps)
        torch.cuda.synchronize()
        out[schedule] = g.download(prop.u_cur)
    assert np.abs(out["fused"]).max() > 0
    for schedule in ("serial", "overlap"):
        assert np.array_equal(out[schedule], out["fused"]), schedule


def test_inject_and_record_exact(torch_cuda):
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    g = Grid(20, 18, 16, 10.0, 1e-3)
    u = g.field()
    cells = np.array([[1, 2, 3], [19, 17, 15], [1, 2, 3], [10, 9, 8]])
    idx = torch.from_numpy(g.index(cells)).cuda()
    w = torch.tensor([0.5, 2.0, 0.25, -1.0], device="cuda")
    amp = torch.tensor([2.0, 3.0, 4.0, 5.0], device="cuda")
    s = torch.cuda.current_stream()
    _abi.rtm_inject(g.c, u, idx, w, amp, 4, s)
    out = torch.zeros(4, device="cuda")
    _abi.rtm_record(g.c, u, idx, out, 4, s)
    bad = torch.tensor([-5, g.total + 10], dtype=torch.int64, device="cuda")
    out2 = torch.full((2,), 9.0, device="cuda")
    _abi.rtm_inject(g.c, u, bad, w[:2], amp[:2], 2, s)       # out-of-range indices are skipped
    _abi.rtm_record(g.c, u, bad, out2, 2, s)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [2.0, 6.0, 2.0, -5.0]      # duplicate cell sums 1.0 + 1.0
    assert out2.cpu().tolist() == [0.0, 0.0]
    host = g.download(u)
    assert np.count_nonzero(host) == 3


def test_image_and_kappa_kernels(torch_cuda):
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nx, ny, nz = 45, 30, 21
    g = Grid(nx, ny, nz, 10.0, 7e-4)
    rng = np.random.default_rng(4)
    a, b, i0 = rng.standard_normal((3, nz, ny, nx))
    img = g.upload(i0)
    _abi.rtm_image_accumulate(g.c, img, g.upload(a), g.upload(b), 0.75, torch.cuda.current_stream())
    vel = rng.uniform(1500, 4500, (nz, ny, nx))
    kap = g.kappa_from_velocity(vel)
    torch.cuda.synchronize()
    a32, b32, i32 = (x.astype(np.float32).astype(np.float64) for x in (a, b, i0))
    np.testing.assert_allclose(g.download(img), i32 + 0.75 * a32 * b32, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(g.download(kap), (vel * 7e-4 / 10.0) ** 2, rtol=5e-7)


def test_row_kernels_vector_and_scalar_paths_bitwise(torch_cuda):
    """The owned-row kernels (imaging, coded imaging, snapshot coding, kappa, velocity gradient) give
    the same bits on a layout that takes their float4 path (aligned rows) and on one that takes the
    scalar path (row pitch not a multiple of 4)."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nx, ny, nz = 68, 30, 21
    rng = np.random.default_rng(14)
    a, b, i0, gk = rng.standard_normal((4, nz, ny, nx))
    vel = rng.uniform(1500, 4500, (nz, ny, nx))
    st = torch.cuda.current_stream()
    outs = []
    for x_align, pitch in ((32, None), (1, nx + 9)):
        g = Grid(nx, ny, nz, 10.0, 7e-4, x_align=x_align, pitch_y=pitch)
        assert (g.pitch_y % 4 == 0) == (x_align == 32)
        img = g.upload(i0)
        _abi.rtm_image_accumulate(g.c, img, g.upload(a), g.upload(b), 0.75, st)
        kap = g.kappa_from_velocity(vel)
        codes = torch.empty(nx * ny * nz, dtype=torch.int16, device="cuda")
        scales = torch.empty(nz, dtype=torch.float32, device="cuda")
        _abi.rtm_snapshot_encode(g.c, g.upload(a), codes, scales, _abi.RTM_SNAP_BF16, st)
        img2 = g.upload(i0)
        _abi.rtm_image_accumulate_coded(g.c, img2, codes, scales, _abi.RTM_SNAP_BF16, g.upload(b), 0.5, st)
        gv = torch.empty(nx * ny * nz, dtype=torch.float32, device="cuda")
        vt = torch.from_numpy(vel.astype(np.float32).reshape(-1)).cuda()
        _abi.rtm_velocity_gradient(g.c, gv, g.upload(gk), vt, 7e-5, st)
        torch.cuda.synchronize()
        outs.append([g.download(img), g.download(kap), codes.cpu().numpy(), scales.cpu().numpy(),
                     g.download(img2), gv.cpu().numpy()])
    for name, x, y in zip(("image", "kappa", "codes", "scales", "coded image", "velocity gradient"), *outs):
        assert np.array_equal(x, y), name


def test_two_subdomain_split_bitwise(torch_cuda):
    """Domain decomposition on one GPU: the box split in x into two subdomains, each stepping with
    its own halo call, pack, interior call and unpack, whose receive slot for the shared face points
    at the neighbour's packed send slot (the exchange, with no copy) and whose outer faces receive
    zero ghosts.  After 60 steps with sources on both sides of the cut, the two halves are bitwise
    the single-domain solution."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi, synth
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Sources

    nx, ny, nz, xs, nsteps = 320, 40, 36, 160, 60       # wide enough for interior calls on both sides
    h = 10.0
    dt = Grid.stable_dt(4, h, 3000.0)
    v = synth.random_smooth_velocity((nz, ny, nx), seed=31, vmin=1500.0, vmax=3000.0)
    whole = Grid(nx, ny, nz, h, dt, sponge_width=6)
    gx, gy, gz = (t.cpu().numpy() for t in (whole.gx, whole.gy, whole.gz))
    parts = [(Grid(xs, ny, nz, h, dt, sponge_profiles=(gx[:xs], gy, gz)), 0, v[:, :, :xs]),
             (Grid(nx - xs, ny, nz, h, dt, sponge_profiles=(gx[xs:], gy, gz)), xs, v[:, :, xs:])]
    src = np.array([[xs - 2, 20, 18], [xs + 1, 10, 10], [250, 30, 25], [5, 33, 30], [100, 20, 18]])
    amp = whole.ricker(nsteps, 20.0)
    w = whole.injection_weights(v[src[:, 2], src[:, 1], src[:, 0]])
    amps = np.repeat(amp[:, None], len(src), axis=1)
    st = torch.cuda.current_stream()

    def run(grids):
        doms = []
        for g, x0, vv in grids:
            sel = (src[:, 0] >= x0) & (src[:, 0] < x0 + g.nx)
            loc = src[sel] - np.array([x0, 0, 0])
            doms.append({"g": g, "kap": g.kappa_from_velocity(vv), "a": g.field(), "b": g.field(),
                         "send": g.faces(), "src": Sources(g, loc, w[sel], amps[:, sel]) if sel.any() else None})
        for i, d in enumerate(doms):
            d["recv"] = [None] * 6
            if i > 0:
                d["recv"][0] = doms[i - 1]["g"].face_slots(doms[i - 1]["send"])[1]
            if i + 1 < len(doms):
                d["recv"][1] = doms[i + 1]["g"].face_slots(doms[i + 1]["send"])[0]
        for n in range(nsteps):
            for d in doms:                                # phase 1-3: halo, shell sources, pack
                g, nxt = d["g"], d["b"]
                _abi.rtm_step_halo(g.c, nxt, d["a"], d["b"], d["kap"], st)
                if d["src"] is not None:
                    d["src"].inject(g, nxt, n, 0, st)
                _abi.rtm_pack_halo(g.c, nxt, d["send"], st)
            for d in doms:                                # interior, interior sources, unpack
                g, nxt = d["g"], d["b"]
                _abi.rtm_step_interior(g.c, nxt, d["a"], d["b"], d["kap"], st)
                if d["src"] is not None:
                    d["src"].inject(g, nxt, n, 1, st)
            for d in doms:
                _abi.rtm_unpack_halo(d["g"].c, d["b"], d["recv"], st)
                d["a"], d["b"] = d["b"], d["a"]
        torch.cuda.synchronize()
        return [(d["g"].download(d["a"]), d["g"].download(d["b"])) for d in doms]

    _say("split: single domain")
    ((ref_cur, ref_prv),) = run([(whole, 0, v)])
    _say("split: two subdomains")
    halves = run(parts)
    cur = np.concatenate([h_[0] for h_ in halves], axis=2)
    prv = np.concatenate([h_[1] for h_ in halves], axis=2)
    assert np.abs(ref_cur).max() > 0
    assert np.array_equal(cur, ref_cur) and np.array_equal(prv, ref_prv)


@pytest.mark.parametrize("fused_pack", [False, True])
def test_2x2x2_subdomain_split_bitwise(torch_cuda, fused_pack):
    """A 2x2x2 decomposition on one GPU: eight subdomains, each with its own halo call, shell
    sources and pack (or the halo call that packs, with injected face cells re-copied), interior call
    and unpack; every face between subdomains receives the neighbour's packed send slot (no copy),
    outer faces zero ghosts.  After 60 steps with sources on the cuts (a corner cell of three faces
    among them), the eight blocks are bitwise the single-domain solution."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi, synth
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Sources

    nx, ny, nz, nsteps = 144, 72, 64, 60
    cut = (64, 40, 28)
    h = 10.0
    dt = Grid.stable_dt(4, h, 3000.0)
    v = synth.random_smooth_velocity((nz, ny, nx), seed=41, vmin=1500.0, vmax=3000.0)
    whole = Grid(nx, ny, nz, h, dt, sponge_width=6)
    gx, gy, gz = (t.cpu().numpy() for t in (whole.gx, whole.gy, whole.gz))
    spans = [((0, cut[0]), (cut[0], nx)), ((0, cut[1]), (cut[1], ny)), ((0, cut[2]), (cut[2], nz))]
    src = np.array([[cut[0] - 1, cut[1] - 1, cut[2] - 1], [cut[0], 20, 10], [30, cut[1], 40], [100, 60, cut[2]],
                    [cut[0] - 3, cut[1] + 2, cut[2] - 2], [20, 15, 12], [120, 55, 50]])
    amp = whole.ricker(nsteps, 20.0)
    w = whole.injection_weights(v[src[:, 2], src[:, 1], src[:, 0]])
    amps = np.repeat(amp[:, None], len(src), axis=1)
    st = torch.cuda.current_stream()

    def run(blocks, fused):
        doms = {}
        for key, (g, o, vv) in blocks.items():
            sel = np.all((src >= o) & (src < o + np.array([g.nx, g.ny, g.nz])), axis=1)
            doms[key] = {"g": g, "kap": g.kappa_from_velocity(vv), "a": g.field(), "b": g.field(),
                         "send": g.faces(), "src": Sources(g, src[sel] - o, w[sel], amps[:, sel]) if sel.any() else None}
        for (ix, iy, iz), d in doms.items():
            d["recv"] = [None] * 6
            for f, (dx, dy, dz, sf) in enumerate([(-1, 0, 0, 1), (1, 0, 0, 0), (0, -1, 0, 3), (0, 1, 0, 2),
                                                  (0, 0, -1, 5), (0, 0, 1, 4)]):
                nb = doms.get((ix + dx, iy + dy, iz + dz))
                if nb is not None:
                    d["recv"][f] = nb["g"].face_slots(nb["send"])[sf]
        for n in range(nsteps):
            for d in doms.values():                       # halo, shell sources, pack
                g, nxt = d["g"], d["b"]
                if fused:
                    _abi.rtm_step_halo_pack(g.c, nxt, d["a"], d["b"], d["kap"], d["send"], st)
                else:
                    _abi.rtm_step_halo(g.c, nxt, d["a"], d["b"], d["kap"], st)
                if d["src"] is not None:
                    d["src"].inject(g, nxt, n, 0, st)
                    if fused:
                        d["src"].repack(g, nxt, n, d["send"], st)
                if not fused:
                    _abi.rtm_pack_halo(g.c, nxt, d["send"], st)
            for d in doms.values():                       # interior, interior sources
                g, nxt = d["g"], d["b"]
                _abi.rtm_step_interior(g.c, nxt, d["a"], d["b"], d["kap"], st)
                if d["src"] is not None:
                    d["src"].inject(g, nxt, n, 1, st)
            for d in doms.values():                       # unpack
                _abi.rtm_unpack_halo(d["g"].c, d["b"], d["recv"], st)
                d["a"], d["b"] = d["b"], d["a"]
        torch.cuda.synchronize()
        return {k: (d["g"].download(d["a"]), d["g"].download(d["b"])) for k, d in doms.items()}

    _say("2x2x2: single domain")
    ((ref_cur, ref_prv),) = run({(0, 0, 0): (whole, np.zeros(3, dtype=np.int64), v)}, False).values()
    blocks = {}
    for ix in range(2):
        for iy in range(2):
            for iz in range(2):
                (x0, x1), (y0, y1), (z0, z1) = spans[0][ix], spans[1][iy], spans[2][iz]
                g = Grid(x1 - x0, y1 - y0, z1 - z0, h, dt, sponge_profiles=(gx[x0:x1], gy[y0:y1], gz[z0:z1]))
                blocks[(ix, iy, iz)] = (g, np.array([x0, y0, z0]), v[z0:z1, y0:y1, x0:x1])
    _say(f"2x2x2: eight subdomains (fused pack {fused_pack})")
    parts = run(blocks, fused_pack)
    assert np.abs(ref_cur).max() > 0
    for (ix, iy, iz), (cur, prv) in parts.items():
        (x0, x1), (y0, y1), (z0, z1) = spans[0][ix], spans[1][iy], spans[2][iz]
        assert np.array_equal(cur, ref_cur[z0:z1, y0:y1, x0:x1]), (ix, iy, iz)
        assert np.array_equal(prv, ref_prv[z0:z1, y0:y1, x0:x1]), (ix, iy, iz)


@pytest.mark.parametrize("radius", [4, 2])
def test_whole_step_equals_halo_then_interior(torch_cuda, radius):
    """rtm_step_whole and rtm_step_halo + rtm_step_interior give the same bits on ragged boxes of
    random fields (ghost ring included), and both leave the ghost ring untouched."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    rng = np.random.default_rng(77 + radius)
    for (nx, ny, nz) in ((150, 41, 70), (9, 21, 13), (130, 9, 40)):
        g = Grid(nx, ny, nz, 10.0, 1e-3, radius=radius, sponge_width=3)
        uc, up, kap = g.field(), g.field(), g.field()
        for f in (uc, up):
            g.padded(f).copy_(torch.from_numpy(rng.standard_normal(g.padded(f).shape).astype(np.float32)))
        g.owned(kap).copy_(torch.from_numpy(rng.uniform(0.01, 0.1, g.shape).astype(np.float32)))
        a, b = g.field(fill=float("nan")), g.field(fill=float("nan"))
        st = torch.cuda.current_stream()
        _abi.rtm_step_halo(g.c, a, uc, up, kap, st)
        _abi.rtm_step_interior(g.c, a, uc, up, kap, st)
        _abi.rtm_step_whole(g.c, b, uc, up, kap, st)
        torch.cuda.synchronize()
        oa, ob = g.download(a), g.download(b)
        assert np.isfinite(ob).all() and np.array_equal(oa, ob), (radius, nx, ny, nz)
        pb = g.padded(b).cpu().numpy()
        R = radius
        ring = np.ones(pb.shape, dtype=bool)
        ring[R:-R, R:-R, R:-R] = False
        assert np.isnan(pb[ring]).all()


@pytest.mark.parametrize("schedule", ["overlap", "serial", "fused"])
def test_radius2_parity(torch_cuda, schedule):
    """The radius-2 (4th-order) path that the coarse grid of the learned corrector runs: a ragged
    layered box with a scaled sponge, sources in the shell and inside, against the FP64 oracle."""
    v = np.array(synth_layered((38, 41, 70)))
    src = [(35, 20, 19), (1, 2, 30), (68, 39, 2)]
    rec = [(2, 2, 2), (69, 40, 37), (35, 20, 10)]
    kw = dict(rec_ijk=rec, sponge_width=8, alpha=0.015 * 2 * math.sqrt(2.0), radius=2)
    gpu = problems.gpu_forward_problem(v, 20.0, 120, src, schedule=schedule, **kw)
    ref = problems.oracle_forward_problem(v, 20.0, 120, src, **kw)
    e_u = problems.rel_l2(gpu["u_cur"], ref["u_cur"])
    e_t = problems.rel_l2(gpu["traces"], ref["traces"])
    _say(f"radius 2 {schedule}: u {e_u:.3e} traces {e_t:.3e}")
    assert e_u <= 1e-4 and e_t <= 1e-4


def test_smallest_boxes_parity(torch_cuda):
    """The smallest legal boxes (2R cells per axis, R = 4 and R = 2): every cell is in the halo
    region, the interior call has nothing to do, and the fused step covers everything."""
    for radius, n in ((4, 8), (2, 4)):
        v = np.full((n, n + 1, n + 2), 2000.0)
        src = [(n // 2, n // 2, n // 2)]
        for schedule in ("serial", "fused"):
            gpu = problems.gpu_forward_problem(v, 10.0, 40, src, sponge_width=0, radius=radius, schedule=schedule)
            ref = problems.oracle_forward_problem(v, 10.0, 40, src, sponge_width=0, radius=radius)
            e = problems.rel_l2(gpu["u_cur"], ref["u_cur"])
            _say(f"smallest box R={radius} {schedule}: {e:.3e}")
            assert e <= 1e-4


def test_empty_problem_stays_zero(torch_cuda):
    """No sources, no receivers, a zero state: every schedule keeps every cell exactly zero (nothing
    reads an unset ghost or stale buffer), and a run of zero steps leaves a given state untouched."""
    torch = torch_cuda
    from paper_1603_03971_amd import synth
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator

    shape = (37, 45, 70)
    g = Grid(shape[2], shape[1], shape[0], 10.0, Grid.stable_dt(4, 10.0, 3000.0))
    kap = g.kappa_from_velocity(synth.random_smooth_velocity(shape, seed=77, vmin=1500, vmax=3000))
    for schedule in ("serial", "overlap", "fused"):
        prop = Propagator(g, kap, schedule=schedule)
        traces = prop.new_traces(7)
        prop.run(7, traces)
        assert int(torch.count_nonzero(prop.u_cur)) == 0 and int(torch.count_nonzero(prop.u_prv)) == 0, schedule
        assert int(torch.count_nonzero(traces)) == 0
        u0, um = synth.random_field(shape, 78), synth.random_field(shape, 79)
        prop.set_state(u0, um)
        prop.run(0)
        assert np.array_equal(g.download(prop.u_cur), u0.astype(np.float32))
        assert np.array_equal(g.download(prop.u_prv), um.astype(np.float32))


def synth_layered(shape):
    from paper_1603_03971_amd import synth

    return synth.layered_velocity(shape, 20.0, seed=12, vmin=1500.0, vmax=3000.0)


@pytest.mark.parametrize("schedule", ["serial", "overlap"])
def test_sources_follow_a_halo_width_change(torch_cuda, schedule):
    """A source whose cell moves from the halo region to the interior when the x-strip width changes
    between steps (64 -> 32 columns) is still added by the call that owns its cell: the run gives the
    one-launch schedule's bits."""
    from paper_1603_03971_amd import _abi, synth
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    torch = torch_cuda
    shape = (36, 40, 200)
    nz, ny, nx = shape
    v = np.array(synth.layered_velocity(shape, 10.0, seed=14))
    src = [(40, 20, 18), (150, 30, 10)]
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(4, 10.0, float(v.max())))
    kap = g.kappa_from_velocity(v)
    vs = np.array([v[k, j, i] for i, j, k in src])
    amp = np.repeat(g.ricker(60, 15.0)[:, None], 2, axis=1)

    def prop_for(sched):
        return Propagator(g, kap, sources=Sources(g, src, g.injection_weights(vs), amp), schedule=sched)

    ref = prop_for("fused")
    ref.run(60)
    prop = prop_for(schedule)
    old = _abi.rtm_get_option(_abi.RTM_OPT_HALO_X_WIDTH)
    try:
        assert bool(g.in_halo([src[0]])[0])
        prop.run(30)
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_X_WIDTH, 32)
        assert not bool(g.in_halo([src[0]])[0])
        prop.run(30)
        torch.cuda.synchronize()
    finally:
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_X_WIDTH, old)
    assert np.any(g.download(ref.u_cur) != 0)
    assert np.array_equal(g.download(prop.u_cur), g.download(ref.u_cur))


@pytest.mark.parametrize("boundary", ["zero_faces", "periodic"])
def test_unpack_aside_bitwise(torch_cuda, boundary):
    """The serial schedule with the unpack on a second stream, concurrent with the interior call,
    gives the bits of the one-stream order (zero-filled receive slots, and the periodic exchange
    whose ghosts carry data)."""
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    torch = torch_cuda
    v, h, nsteps, src = problems.ragged_inputs(seed=11)
    nz, ny, nx = v.shape
    g = Grid(nx, ny, nz, h, Grid.stable_dt(4, h, float(v.max())))
    kap = g.kappa_from_velocity(v)
    vs = np.array([v[k, j, i] for i, j, k in src])
    amp = np.repeat(g.ricker(nsteps, 15.0)[:, None], len(src), axis=1)
    rec = [(1, 1, 1), (149, 40, 69), (75, 20, 35)]
    out = []
    for aside in (False, True):
        p = Propagator(g, kap, sources=Sources(g, src, g.injection_weights(vs), amp), receivers=rec,
                       schedule="serial", boundary=boundary, unpack_aside=aside)
        tr = p.new_traces(nsteps)
        p.run(nsteps, tr)
        torch.cuda.synchronize()
        out.append((g.download(p.u_cur), tr.cpu().numpy()))
    assert np.any(out[0][0] != 0)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("radius", [4, 2])
def test_tuned_one_launch_step_is_bitwise(torch_cuda, radius):
    """rtm_tune_step picks a tile shape and workgroup order for a grid shape; the one-launch step and
    the adjoint step run with it afterwards and give the same bits as before tuning (and as the halo
    and interior calls)."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi, synth
    from paper_1603_03971_amd.grid import Grid

    nx, ny, nz = 136, 72, 60
    v = np.array(synth.layered_velocity((nz, ny, nx), 10.0, seed=17))
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(radius, 10.0, float(v.max())), radius=radius)
    kap = g.kappa_from_velocity(v)
    uc = g.upload(synth.random_field((nz, ny, nx), seed=41))
    up = g.upload(synth.random_field((nz, ny, nx), seed=42))
    work = g.field()
    st = torch.cuda.current_stream()

    def run():
        whole, split, adj = g.field(), g.field(), g.field()
        _abi.rtm_step_whole(g.c, whole, uc, up, kap, st)
        _abi.rtm_step_halo(g.c, split, uc, up, kap, st)
        _abi.rtm_step_interior(g.c, split, uc, up, kap, st)
        _abi.rtm_adjoint_step(g.c, adj, uc, up, kap, work, st)
        torch.cuda.synchronize()
        return g.download(whole), g.download(split), g.download(adj)

    before = run()
    var, remap = _abi.rtm_tune_step(g.c, g.field(), uc, up, kap, reps=2, stream=st)
    _say(f"tuned radius {radius}: variant {var}, workgroup order {remap}")
    assert var in (0, 1, 2, 4, 5) and remap in (0, 1)
    after = run()
    assert np.abs(before[0]).max() > 0
    assert np.array_equal(before[0], before[1])
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
