"""The shell form of the halo-first step (section II phases 1, 2 and 4): rtm_step_shell_pack computes the
owned cells within R of a face into the face buffer only, rtm_step_whole_slots updates every owned cell
with the ghosts read from the receive slots.  Together they must give the same bits as the ring path
(the received faces unpacked into u_cur's ghost ring, the one-launch step, the faces packed from its
result), on grids from the smallest up to several tiles with ragged tails."""
import numpy as np
import pytest

from paper_1603_03971_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_03971_amd import _abi  # noqa: F401  (fails loudly if the library is not built)
    return torch


def _say(msg):
    print(msg, flush=True)


def _poison_ring(g, t):
    owned = g.owned(t).clone()
    t.fill_(float("nan"))
    g.owned(t).copy_(owned)


# (nz, ny, nx): the smallest grids (faces that meet, x strips whose inside neighbour is the other face),
# odd ny and nz, ragged x tiles, deep boxes with several z chunks
@pytest.mark.parametrize("shape,dense,flags", [
    ((8, 8, 8), True, 1),
    ((9, 13, 8), True, 1),
    ((13, 9, 20), True, 1),
    ((13, 9, 20), False, 1),
    ((40, 36, 64), True, 1),
    ((30, 20, 100), True, 0),
    ((30, 20, 100), False, 0),
    ((70, 41, 200), True, 1),
    ((70, 41, 200), False, 1),
    ((50, 72, 256), True, 1),
])
def test_shell_pack_and_whole_slots_match_ring_path(torch_cuda, shape, dense, flags):
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nz, ny, nx = shape
    _say(f"shell {shape} dense {dense} flags {flags}")
    v = np.array(synth.layered_velocity(shape, 10.0, seed=3))
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(4, 10.0, float(v.max())))
    kap = g.kappa_from_velocity(v)
    u0 = synth.random_field(shape, seed=11)
    um = synth.random_field(shape, seed=12)
    rng = np.random.default_rng(13)
    recv_buf = torch.from_numpy(rng.standard_normal(g.face_total).astype(np.float32)).cuda()
    recv = g.face_slots(recv_buf)
    st = torch.cuda.current_stream()
    old = _abi.rtm_get_option(_abi.RTM_OPT_TILE_FLAGS)
    try:
        _abi.rtm_set_option(_abi.RTM_OPT_TILE_FLAGS, flags)
        # reference: the received faces unpacked into the ghost ring, the one-launch step, the pack
        uc_r, up_r = g.upload(u0), g.upload(um)
        _abi.rtm_unpack_halo(g.c, uc_r, recv, st)
        out_r, faces_r = g.field(), g.faces()
        _abi.rtm_step_whole(g.c, out_r, uc_r, up_r, kap, st)
        _abi.rtm_pack_halo(g.c, out_r, faces_r, st)
        # the shell call and the whole-block call from the slots, u_cur's and u_prv's rings poisoned;
        # the dense face copies packed from the levels and from kappa
        uc_s, up_s = g.upload(u0), g.upload(um)
        copies = None
        if dense:
            copies = (g.faces(), g.faces(), g.faces())
            for src, dst in zip((uc_s, up_s, kap), copies):
                _abi.rtm_pack_halo(g.c, src, dst, st)
        _poison_ring(g, uc_s)
        _poison_ring(g, up_s)
        faces_s = g.faces().fill_(float("nan"))
        _abi.rtm_step_shell_pack(g.c, uc_s, up_s, kap, recv, faces_s, st, dense=copies)
        out_s = g.field(float("nan"))
        _abi.rtm_step_whole_slots(g.c, out_s, uc_s, up_s, kap, recv, st)
        torch.cuda.synchronize()
    finally:
        _abi.rtm_set_option(_abi.RTM_OPT_TILE_FLAGS, old)
    assert torch.count_nonzero(faces_r) > 0
    assert torch.equal(faces_s, faces_r)                     # every face cell written, the same bits
    assert torch.isfinite(g.owned(out_s)).all()
    assert torch.equal(g.owned(out_s), g.owned(out_r))


def test_whole_slots_in_place(torch_cuda):
    """u_nxt = u_prv (the two-buffer rotation of the serial schedule): the same bits."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    shape = (40, 36, 128)
    nz, ny, nx = shape
    v = np.array(synth.layered_velocity(shape, 10.0, seed=4))
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(4, 10.0, float(v.max())))
    kap = g.kappa_from_velocity(v)
    u0, um = synth.random_field(shape, seed=41), synth.random_field(shape, seed=42)
    recv = g.face_slots(torch.randn(g.face_total, device="cuda"))
    st = torch.cuda.current_stream()
    a, b, out = g.upload(u0), g.upload(um), g.field()
    _abi.rtm_step_whole_slots(g.c, out, a, b, kap, recv, st)
    _abi.rtm_step_whole_slots(g.c, b, a, b, kap, recv, st)
    torch.cuda.synchronize()
    assert torch.equal(g.owned(out), g.owned(b))


def test_two_subdomain_split_shell_bitwise(torch_cuda):
    """The x split of a 320 x 40 x 36 box into two subdomains in the shell form: each shell call reads its
    ghosts from the receive slots (the neighbour's face buffer of the previous step for the shared face,
    a zero buffer for the outer ones) and the faces of its own last two levels from its face buffers
    (three, rotating), each whole-block call the same slots; sources on both sides of the cut, those in
    face cells re-copied into the faces.  After 60 steps, bitwise the single-domain solution."""
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

    def doms_for(grids):
        doms = []
        for g, x0, vv in grids:
            sel = (src[:, 0] >= x0) & (src[:, 0] < x0 + g.nx)
            loc = src[sel] - np.array([x0, 0, 0])
            kap = g.kappa_from_velocity(vv)
            kf = g.faces()
            _abi.rtm_pack_halo(g.c, kap, kf, st)
            doms.append({"g": g, "kap": kap, "kf": kf, "a": g.field(), "b": g.field(),
                         "send": [g.faces(), g.faces(), g.faces()], "zero": g.faces(),
                         "src": Sources(g, loc, w[sel], amps[:, sel]) if sel.any() else None})
        return doms

    def recv(doms, i, b):
        """Receive slots of subdomain i's level whose faces are in face buffer b."""
        d = doms[i]
        r = list(d["g"].face_slots(d["zero"]))
        if i > 0:
            r[0] = doms[i - 1]["g"].face_slots(doms[i - 1]["send"][b])[1]
        if i + 1 < len(doms):
            r[1] = doms[i + 1]["g"].face_slots(doms[i + 1]["send"][b])[0]
        return r

    def run_ring(grids):
        (d,) = doms_for(grids)
        g = d["g"]
        for n in range(nsteps):
            _abi.rtm_step_whole(g.c, d["b"], d["a"], d["b"], d["kap"], st)
            if d["src"] is not None:
                d["src"].inject(g, d["b"], n, 2, st)
            _abi.rtm_unpack_halo(g.c, d["b"], [None] * 6, st)
            d["a"], d["b"] = d["b"], d["a"]
        torch.cuda.synchronize()
        return g.download(d["a"]), g.download(d["b"])

    def run_shell(grids):
        doms = doms_for(grids)
        for d in doms:                 # levels 0 and -1 are zero: so are their faces (buffers 2 and 1)
            _poison_ring(d["g"], d["a"])
            _poison_ring(d["g"], d["b"])
        for n in range(nsteps):
            b, bc, bp = n % 3, (n - 1) % 3, (n - 2) % 3
            for i, d in enumerate(doms):                  # shell calls: the faces of level n + 1
                g = d["g"]
                _abi.rtm_step_shell_pack(g.c, d["a"], d["b"], d["kap"], recv(doms, i, bc), d["send"][b], st,
                                         dense=(d["send"][bc], d["send"][bp], d["kf"]))
            for i, d in enumerate(doms):                  # whole-block calls, sources, re-copy
                g = d["g"]
                _abi.rtm_step_whole_slots(g.c, d["b"], d["a"], d["b"], d["kap"], recv(doms, i, bc), st)
                if d["src"] is not None:
                    d["src"].inject(g, d["b"], n, 2, st)
                    d["src"].repack(g, d["b"], n, d["send"][b], st)
            for d in doms:
                d["a"], d["b"] = d["b"], d["a"]
        torch.cuda.synchronize()
        return [(d["g"].download(d["a"]), d["g"].download(d["b"])) for d in doms]

    _say("split shell: single domain, ring")
    ref_cur, ref_prv = run_ring([(whole, 0, v)])
    _say("split shell: two subdomains")
    halves = run_shell(parts)
    cur = np.concatenate([h_[0] for h_ in halves], axis=2)
    prv = np.concatenate([h_[1] for h_ in halves], axis=2)
    assert np.abs(ref_cur).max() > 0 and np.all(np.isfinite(cur))
    assert np.array_equal(cur, ref_cur) and np.array_equal(prv, ref_prv)


@pytest.mark.parametrize("nsrc,nrec", [(1, 1024), (5, 0), (0, 300), (3, 4093), (40, 1000), (40, 5000)])
def test_inject_record_matches_the_two_calls(torch_cuda, nsrc, nrec):
    """rtm_inject_record against rtm_inject then rtm_record: the same field and samples, bit for bit,
    with a receiver on a source cell, a source given twice and indices outside the block; up to 4096
    items in one workgroup, more in the two launches."""
    torch = torch_cuda
    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    g = Grid(40, 36, 30, 10.0, 1e-3)
    rng = np.random.default_rng(nsrc * 1000 + nrec)
    u0 = g.upload(synth.random_field((30, 36, 40), seed=5))
    total = int(g.total)
    sidx = rng.integers(0, total, size=nsrc).astype(np.int64)
    if nsrc >= 3:
        sidx[1] = sidx[0]                                   # twice: two adds
        sidx[2] = total + 7                                 # outside: ignored
    ridx = rng.integers(0, total, size=nrec).astype(np.int64)
    if nrec >= 2 and nsrc >= 1:
        ridx[0] = sidx[0]                                   # on a source cell: records the injected value
        ridx[1] = -3                                        # outside: 0
    w = rng.uniform(0.5, 2.0, nsrc).astype(np.float32)
    amp = rng.standard_normal(nsrc).astype(np.float32)
    dev = lambda a: torch.from_numpy(a).cuda() if a.size else None
    si, ri, wd, ad = dev(sidx), dev(ridx), dev(w), dev(amp)
    st = torch.cuda.current_stream()
    ua, ub = u0.clone(), u0.clone()
    oa = torch.full((max(nrec, 1),), float("nan"), device="cuda")
    ob = oa.clone()
    if nsrc:
        _abi.rtm_inject(g.c, ua, si, wd, ad, nsrc, st)
    if nrec:
        _abi.rtm_record(g.c, ua, ri, oa, nrec, st)
    _abi.rtm_inject_record(g.c, ub, si, wd, ad, nsrc, ri, ob if nrec else None, nrec, st)
    torch.cuda.synchronize()
    if nsrc >= 3:
        # the cell given twice takes two atomic adds, whose order is not fixed: equal up to rounding
        d = int(sidx[0])
        assert torch.allclose(ua[d], ub[d], rtol=1e-6, atol=0.0)
        ua[d] = ub[d] = 0.0
        if nrec >= 1:
            assert torch.allclose(oa[0], ob[0], rtol=1e-6, atol=0.0)
            oa[0] = ob[0] = 0.0
    assert torch.equal(ua, ub)
    if nrec:
        assert not torch.isnan(ob).any()                   # every sample written
        assert torch.equal(oa, ob)
    if nsrc >= 3 and nrec >= 2:
        assert ob[1].item() == 0.0 and ub[int(ridx[2])].item() == ob[2].item()


def test_refresh_kappa_after_in_place_change(torch_cuda):
    """A medium changed in place half-way (kappa scaled in a block touching the -x face): with
    refresh_kappa() the shell form stays bitwise the halo-region form, which reads kappa itself."""
    torch = torch_cuda
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    shape = (36, 40, 96)
    nz, ny, nx = shape
    v = np.array(synth.layered_velocity(shape, 10.0, seed=8))
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(4, 10.0, float(v.max()) * 1.1), sponge_width=6)
    runs = []
    for halo in ("region", "shell"):
        kap = g.kappa_from_velocity(v)
        src = Sources(g, [(30, 20, 18)], g.injection_weights([v[18, 20, 30]]), g.ricker(60, 20.0)[:, None])
        p = Propagator(g, kap, sources=src, schedule="serial", boundary="zero_faces", ghosts="slots", halo=halo)
        p.run(30)
        p.sync()
        g.owned(kap)[4:20, 5:30, 0:12] *= 1.2          # in place, x from 0: the shell call's x strips
        p.refresh_kappa()
        p.run(30)
        torch.cuda.synchronize()
        runs.append(g.download(p.u_cur))
    assert np.abs(runs[0]).max() > 0 and np.array_equal(runs[0], runs[1])
