"""The halo call that reads u_cur's ghost cells from the receive slots (rtm_step_halo_pack_slots) and
the steps built on it (ghosts="slots": no unpack pass).  Everything here is bitwise: the call must give
exactly the fields and faces of rtm_unpack_halo followed by rtm_step_halo_pack, with the ghost ring it
no longer reads poisoned with NaN; the oracle parity of the steps built on it is in
test_gpu_interior.py.
"""
import numpy as np
import pytest

from paper_1603_03971_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1603_03971_amd import _abi  # noqa: F401  (fails loudly if the library is not built)
    return torch


def _say(msg):
    print(msg, flush=True)


def _poison_ring(g, t):
    """Keep the owned cells of a padded field, set everything else (ghost ring, padding) to NaN."""
    owned = g.owned(t).clone()
    t.fill_(float("nan"))
    g.owned(t).copy_(owned)


# (nz, ny, nx): the smallest grids (4-wide x strips, z slabs that meet, odd ny and nz); a box the halo
# region covers whole; ragged x tiles whose last lane loads the +X ghost and y strips whose last tile
# rows are ghost rows (10-row strips); interior boxes with full tiles
@pytest.mark.parametrize("shape,halo_variant,flags", [
    ((8, 8, 8), 0, 1),
    ((13, 9, 20), 0, 1),
    ((40, 36, 64), 0, 1),
    ((30, 20, 100), 0, 1),
    ((30, 20, 100), 2, 0),
    ((70, 41, 200), 0, 1),
    ((70, 41, 200), 0, 0),
    ((50, 72, 256), 1, 1),
    ((50, 72, 256), 2, 1),
    ((50, 72, 256), 4, 1),
    ((50, 72, 256), 5, 1),
])
def test_halo_pack_slots_matches_unpack_then_halo_pack(torch_cuda, shape, halo_variant, flags):
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nz, ny, nx = shape
    _say(f"halo_pack_slots {shape} halo variant {halo_variant} flags {flags}")
    v = np.array(synth.layered_velocity(shape, 10.0, seed=3))
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(4, 10.0, float(v.max())))
    kap = g.kappa_from_velocity(v)
    u0 = synth.random_field(shape, seed=11)
    um = synth.random_field(shape, seed=12)
    rng = np.random.default_rng(13)
    recv_buf = torch.from_numpy(rng.standard_normal(g.face_total).astype(np.float32)).cuda()
    recv = g.face_slots(recv_buf)
    st = torch.cuda.current_stream()
    old = (_abi.rtm_get_option(_abi.RTM_OPT_HALO_VARIANT), _abi.rtm_get_option(_abi.RTM_OPT_TILE_FLAGS))
    try:
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_VARIANT, halo_variant)
        _abi.rtm_set_option(_abi.RTM_OPT_TILE_FLAGS, flags)
        # reference: the received faces unpacked into the ghost ring, then the halo call that packs
        uc_r, up = g.upload(u0), g.upload(um)
        _abi.rtm_unpack_halo(g.c, uc_r, recv, st)
        out_r, faces_r = g.field(), g.faces()
        _abi.rtm_step_halo_pack(g.c, out_r, uc_r, up, kap, faces_r, st)
        # the same from the slots, with u_cur's ring (and u_prv's) poisoned
        uc_s, up_s = g.upload(u0), g.upload(um)
        _poison_ring(g, uc_s)
        _poison_ring(g, up_s)
        out_s, faces_s = g.field(), g.faces()
        _abi.rtm_step_halo_pack_slots(g.c, out_s, uc_s, up_s, kap, recv, faces_s, st)
        torch.cuda.synchronize()
    finally:
        _abi.rtm_set_option(_abi.RTM_OPT_HALO_VARIANT, old[0])
        _abi.rtm_set_option(_abi.RTM_OPT_TILE_FLAGS, old[1])
    assert torch.isfinite(out_s).all()
    assert torch.count_nonzero(out_r) > 0
    assert torch.equal(out_s, out_r)            # every cell of the padded block, ring and interior box too
    assert torch.equal(faces_s, faces_r)


def _problem(shape, seed=21):
    """Layered medium, sources in the interior box, in a face layer (re-packed after injection), in a
    z slab and near a corner; receivers spread over the regions."""
    v = np.array(synth.layered_velocity(shape, 10.0, seed=seed))
    nz, ny, nx = shape
    src = [(nx // 2, ny // 2, nz // 2), (2, ny // 2, nz // 3), (nx // 3, 5, 1), (nx - 2, ny - 3, nz - 2)]
    rec = [(nx // 2 + 7, ny // 2, nz // 2), (1, 1, 1), (nx - 1, ny - 1, nz - 1), (nx // 3, 3, 2), (70, 20, 20)]
    return v, src, rec


def _run(v, src, rec, nsteps, schedule, boundary, ghosts, poison=False, pin_at=None, halo="region"):
    import torch

    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    nz, ny, nx = v.shape
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(4, 10.0, float(v.max())), sponge_width=8)
    kap = g.kappa_from_velocity(v)
    vs = np.array([v[k, j, i] for i, j, k in src])
    amp = np.repeat(g.ricker(nsteps, 25.0)[:, None], len(src), axis=1)
    s = Sources(g, src, g.injection_weights(vs), amp)
    prop = Propagator(g, kap, sources=s, receivers=rec, schedule=schedule, boundary=boundary, ghosts=ghosts,
                      debug=poison, halo=halo)
    prop.set_state(synth.random_field(v.shape, seed=31, scale=1e-3), synth.random_field(v.shape, seed=32, scale=1e-3))
    if poison:
        torch.cuda.synchronize()
        _poison_ring(g, prop.u_cur)
        _poison_ring(g, prop.u_prv)
    traces = prop.new_traces(nsteps)
    pinned = []

    def on_level(k, p):
        if k == pin_at:
            pinned.append(p.pin_current())     # the next levels go to fresh (NaN, in debug) buffers
    prop.run(nsteps, traces, on_level=on_level)
    torch.cuda.synchronize()
    return prop, g, traces.cpu().numpy()


@pytest.mark.parametrize("halo", ["region", "shell"])
@pytest.mark.parametrize("boundary", ["zero", "zero_faces", "periodic"])
@pytest.mark.parametrize("schedule", ["serial", "overlap"])
def test_slots_steps_bitwise(torch_cuda, schedule, boundary, halo):
    """40 steps with ghosts="slots" (the level buffers' ghost rings NaN throughout, and a level pinned
    half-way so that later levels land in fresh NaN buffers), with the halo region or the shell form of
    the halo call, against ghosts="ring": the same bits."""
    v, src, rec = _problem((44, 40, 200))
    _say(f"slots {schedule} {boundary} {halo}")
    pr, g, tr = _run(v, src, rec, 40, schedule, boundary, "ring", pin_at=20)
    ps, _, ts = _run(v, src, rec, 40, schedule, boundary, "slots", poison=True, pin_at=20, halo=halo)
    a_cur, a_prv = g.download(pr.u_cur), g.download(pr.u_prv)
    b_cur, b_prv = g.download(ps.u_cur), g.download(ps.u_prv)
    assert np.all(np.isfinite(b_cur)) and np.abs(a_cur).max() > 0
    assert np.array_equal(a_cur, b_cur) and np.array_equal(a_prv, b_prv)
    assert np.array_equal(tr, ts)


@pytest.mark.parametrize("boundary", ["zero_faces", "periodic"])
def test_fill_ghosts_then_whole_step_bitwise(torch_cuda, boundary):
    """After a slots run, fill_ghosts() writes the newest level's ring; one rtm_step_whole from it
    gives the same bits as from the ring run's level."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi

    v, src, rec = _problem((36, 40, 160), seed=22)
    pr, g, _ = _run(v, src, rec, 25, "serial", boundary, "ring")
    ps, _, _ = _run(v, src, rec, 25, "serial", boundary, "slots")
    ps.fill_ghosts()
    st = torch.cuda.current_stream()
    outs = []
    for p in (pr, ps):
        out = g.field()
        _abi.rtm_step_whole(g.c, out, p.u_cur, p.u_prv, p.kappa, st)
        outs.append(out)
    torch.cuda.synchronize()
    a, b = g.download(outs[0]), g.download(outs[1])
    assert np.abs(a).max() > 0 and np.array_equal(a, b)


def test_two_subdomain_split_slots_bitwise(torch_cuda):
    """The x split of a 320 x 40 x 36 box into two subdomains with no unpack pass: each halo call reads
    its ghosts from the receive slots (the neighbour's face buffer of the previous step for the shared
    face, a zero buffer for the outer ones), each subdomain alternating between two face buffers.
    After 60 steps with sources on both sides of the cut, bitwise the single-domain solution."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Sources

    nx, ny, nz, xs, nsteps = 320, 40, 36, 160, 60
    h = 10.0
    dt = Grid.stable_dt(4, h, 3000.0)
    v = synth.random_smooth_velocity((nz, ny, nx), seed=31, vmin=1500.0, vmax=3000.0)
    whole = Grid(nx, ny, nz, h, dt, sponge_width=6)
    gx, gy, gz = (t.cpu().numpy() for t in (whole.gx, whole.gy, whole.gz))
    parts = [(Grid(xs, ny, nz, h, dt, sponge_profiles=(gx[:xs], gy, gz)), 0, v[:, :, :xs]),
             (Grid(nx - xs, ny, nz, h, dt, sponge_profiles=(gx[xs:], gy, gz)), xs, v[:, :, xs:])]
    src = np.array([[xs - 2, 20, 18], [xs + 1, 10, 10], [250, 30, 25], [5, 33, 30], [100, 20, 18]])
    w = whole.injection_weights(v[src[:, 2], src[:, 1], src[:, 0]])
    amps = np.repeat(whole.ricker(nsteps, 20.0)[:, None], len(src), axis=1)
    st = torch.cuda.current_stream()

    def run(grids, slots):
        doms = []
        for g, x0, vv in grids:
            sel = (src[:, 0] >= x0) & (src[:, 0] < x0 + g.nx)
            loc = src[sel] - np.array([x0, 0, 0])
            doms.append({"g": g, "kap": g.kappa_from_velocity(vv), "a": g.field(), "b": g.field(),
                         "send": [g.faces(), g.faces()], "zero": g.faces(),
                         "src": Sources(g, loc, w[sel], amps[:, sel]) if sel.any() else None})
        if slots:
            for d in doms:
                _poison_ring(d["g"], d["a"])
                _poison_ring(d["g"], d["b"])

        def recv(i, b):
            """Receive slots of subdomain i's level made by a step that packed into buffer b."""
            d = doms[i]
            r = [d["g"].face_slots(d["zero"])[f] if slots else None for f in range(6)]
            if i > 0:
                r[0] = doms[i - 1]["g"].face_slots(doms[i - 1]["send"][b])[1]
            if i + 1 < len(doms):
                r[1] = doms[i + 1]["g"].face_slots(doms[i + 1]["send"][b])[0]
            return r

        for n in range(nsteps):
            b = n % 2
            for i, d in enumerate(doms):                  # halo call (+ ghosts from slots) and pack
                g, nxt = d["g"], d["b"]
                if slots:
                    _abi.rtm_step_halo_pack_slots(g.c, nxt, d["a"], d["b"], d["kap"], recv(i, 1 - b), d["send"][b], st)
                else:
                    _abi.rtm_step_halo_pack(g.c, nxt, d["a"], d["b"], d["kap"], d["send"][b], st)
                if d["src"] is not None:
                    d["src"].inject(g, nxt, n, 0, st)
                    d["src"].repack(g, nxt, n, d["send"][b], st)
            for d in doms:                                # interior call and interior sources
                g, nxt = d["g"], d["b"]
                _abi.rtm_step_interior(g.c, nxt, d["a"], d["b"], d["kap"], st)
                if d["src"] is not None:
                    d["src"].inject(g, nxt, n, 1, st)
            for i, d in enumerate(doms):
                if not slots:
                    _abi.rtm_unpack_halo(d["g"].c, d["b"], recv(i, b), st)
                d["a"], d["b"] = d["b"], d["a"]
        torch.cuda.synchronize()
        return [(d["g"].download(d["a"]), d["g"].download(d["b"])) for d in doms]

    _say("split slots: single domain, ring")
    ((ref_cur, ref_prv),) = run([(whole, 0, v)], False)
    _say("split slots: two subdomains, slots")
    halves = run(parts, True)
    cur = np.concatenate([h_[0] for h_ in halves], axis=2)
    prv = np.concatenate([h_[1] for h_ in halves], axis=2)
    assert np.abs(ref_cur).max() > 0 and np.all(np.isfinite(cur))
    assert np.array_equal(cur, ref_cur) and np.array_equal(prv, ref_prv)
