"""Grids of more than 2^32 cells: every kernel on the path must index with 64-bit offsets, and every
elementwise launch must stride past the 2^32 work-items one launch dimension holds.

1664^3 owned cells (4.61e9) in padded fields of 4.74e9 elements (19 GB each).  A seeded random block
near the far corner, a source and receivers there, 12 steps: the disturbance cannot reach beyond 48
cells of the block, so the oracle on the 96^3 corner box (zero outside it, as the real field is) is
exact for the whole box, and every other cell must still be exactly zero (an offset that wrapped at
2^32 would write far from the corner).  The one-launch schedule must give the same bits, and the
imaging and snapshot-coding kernels are checked over every owned cell.
"""
import numpy as np
import pytest

import oracle
from paper_1603_03971_amd import synth

pytestmark = pytest.mark.gpu

N = 1664
H = 10.0
STEPS = 12
BOX = 96          # corner box the oracle steps: the block plus 4 * STEPS cells, and margin
BLK = 24          # random block [N - 40, N - 16) on every axis


def _say(msg):
    print(msg, flush=True)


def test_more_than_2_32_cells():
    import torch

    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.propagator import Propagator, Sources

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 140 * 2**30:
        pytest.skip(f"needs about 140 GB of device memory, {free / 2**30:.0f} GiB free")
    st = torch.cuda.current_stream()
    prof = synth.layered_profile(N, H, seed=6)
    dt = Grid.stable_dt(4, H, float(prof.max()))
    g = Grid(N, N, N, H, dt)
    assert N**3 > 2**32 and g.total > 2**32
    _say(f"maxsize: {N}^3 owned cells, padded fields of {g.total} elements")

    # kappa over every owned cell (the elementwise kernel strides 18 times over its capped grid)
    v = torch.from_numpy(prof.astype(np.float32)).cuda()[:, None, None].expand(N, N, N).contiguous()
    kap = g.kappa_from_velocity(v)
    del v
    torch.cuda.empty_cache()
    ko = g.owned(kap)
    s32 = np.float32(dt / H)
    for k in (0, 1551, 1552, N - 1):
        a = np.float32(prof[k]) * s32
        assert float(ko[k, N - 1, N - 1]) == float(a * a) and float(ko[k, 0, 0]) == float(a * a), k

    lo = N - BOX
    c0 = N - 40
    u0 = synth.random_field((BLK, BLK, BLK), seed=61)
    um = synth.random_field((BLK, BLK, BLK), seed=62)
    amp = synth.random_field((STEPS, 1, 1), seed=63).reshape(STEPS, 1)
    src = (N - 10, N - 30, N - 20)
    rec = [(N - 1, N - 1, N - 1), (N - 5, N - 28, N - 33), (N - 20, N - 20, N - 2), (N - 60, N - 61, N - 62)]

    def run(schedule):
        sources = Sources(g, [src], g.injection_weights([prof[src[2]]]), amp.astype(np.float32))
        prop = Propagator(g, kap, sources=sources, receivers=rec, schedule=schedule)
        blk = slice(c0, c0 + BLK)
        g.owned(prop.u_cur)[blk, blk, blk].copy_(torch.from_numpy(u0.astype(np.float32)).cuda())
        g.owned(prop.u_prv)[blk, blk, blk].copy_(torch.from_numpy(um.astype(np.float32)).cuda())
        traces = prop.new_traces(STEPS)
        prop.run(STEPS, traces)
        torch.cuda.synchronize()
        return prop, traces

    _say("maxsize: serial halo-first schedule")
    prop, traces = run("serial")
    uo = g.owned(prop.u_cur)
    corner = uo[lo:, lo:, lo:].cpu().numpy().astype(np.float64)
    nonzero_all = int(torch.count_nonzero(uo))
    nonzero_corner = int(np.count_nonzero(corner))
    assert nonzero_corner > 0 and nonzero_all == nonzero_corner, (nonzero_all, nonzero_corner)

    _say("maxsize: oracle on the corner box")
    sp = oracle.sponge_profile(N, 16, 0.015)[lo:]
    vv = np.broadcast_to(prof[lo:, None, None], (BOX, BOX, BOX))
    dto = oracle.stable_dt(4, H, float(prof.max()))
    assert abs(dto - dt) < 1e-15
    U0 = np.zeros((BOX, BOX, BOX))
    UM = np.zeros((BOX, BOX, BOX))
    b0 = c0 - lo
    U0[b0:b0 + BLK, b0:b0 + BLK, b0:b0 + BLK] = u0.astype(np.float32)
    UM[b0:b0 + BLK, b0:b0 + BLK, b0:b0 + BLK] = um.astype(np.float32)
    ref = oracle.forward(oracle.kappa_field(vv, dto, H), (sp, sp, sp), STEPS,
                         src_ijk=[tuple(a - lo for a in src)], src_w=oracle.injection_weight([prof[src[2]]], dto, H),
                         src_amp=amp.astype(np.float32).astype(np.float64),
                         rec_ijk=[tuple(a - lo for a in r) for r in rec], u_cur=U0, u_prv=UM, nthreads=16)
    scale = float(np.max(np.abs(ref["u_cur"])))
    err = float(np.max(np.abs(corner - ref["u_cur"]))) / scale
    terr = float(np.max(np.abs(traces.cpu().numpy() - ref["traces"]))) / float(np.max(np.abs(ref["traces"])))
    _say(f"maxsize: corner box max error / scale {err:.2e}, traces {terr:.2e}")
    assert err <= 1e-5 and terr <= 1e-5

    _say("maxsize: one-launch schedule")
    fprop, ftraces = run("fused")
    assert bool(torch.equal(g.owned(fprop.u_cur), uo)) and bool(torch.equal(ftraces, traces))
    del fprop, ftraces
    torch.cuda.empty_cache()

    _say("maxsize: image accumulation over every owned cell")
    img = g.field()
    _abi.rtm_image_accumulate(g.c, img, prop.u_cur, prop.u_prv, 0.5, st)
    torch.cuda.synchronize()
    want = (0.5 * uo) * g.owned(prop.u_prv)
    assert bool(torch.equal(g.owned(img), want))
    assert int(torch.count_nonzero(img)) == int(torch.count_nonzero(want))     # no ghost written
    del img, want
    torch.cuda.empty_cache()

    _say("maxsize: BF16 snapshot coding over every owned cell")
    # plane k = P * 2^(k mod 7 - 3): exact scalings, so every plane has P's codes and scale * 2^e
    plane = synth.random_field((1, N, N), seed=64).astype(np.float32)
    f = torch.tensor([2.0 ** (k % 7 - 3) for k in range(N)], dtype=torch.float32, device="cuda")
    field = prop.u_cur
    g.owned(field).copy_(torch.from_numpy(plane).cuda().expand(N, N, N) * f[:, None, None])
    codes = torch.empty(N * N * N, dtype=torch.int16, device="cuda")
    scales = torch.empty(N, dtype=torch.float32, device="cuda")
    _abi.rtm_snapshot_encode(g.c, field, codes, scales, _abi.RTM_SNAP_BF16, st)
    torch.cuda.synchronize()
    pc, ps = oracle.snapshot_encode(plane, "bf16")
    want_scales = torch.from_numpy(ps.astype(np.float32)).cuda() * f
    assert bool(torch.equal(scales, want_scales))
    want_codes = torch.from_numpy(pc.reshape(-1).view(np.int16).copy()).cuda()
    assert bool(torch.equal(codes.view(N, N * N), want_codes.expand(N, N * N)))

    _say("maxsize: imaging with the coded snapshot")
    img = g.field()
    _abi.rtm_image_accumulate_coded(g.c, img, codes, scales, _abi.RTM_SNAP_BF16, prop.u_prv, 1.0, st)
    torch.cuda.synchronize()
    dec = (codes.view(torch.bfloat16).float().view(N, N, N)) * scales[:, None, None]
    assert bool(torch.equal(g.owned(img), dec * g.owned(prop.u_prv)))
    del img, dec, codes, scales, prop, kap
    torch.cuda.empty_cache()


def test_faces_beyond_2_31_elements():
    """A flat 23200 x 23200 x 8 grid: its z faces hold 2.15e9 > 2^31 cells each, so pack and unpack
    take their 64-bit counters.  Every slot must be the owned face, in the slot order the faces are
    documented in, and every ghost face must receive its slot."""
    import torch

    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 110 * 2**30:
        pytest.skip(f"needs about 110 GB of device memory, {free / 2**30:.0f} GiB free")
    nx = ny = 23200
    nz = 8
    R = 4
    g = Grid(nx, ny, nz, H, 1e-3)
    assert max(g.face_sizes) >= 2**31
    _say(f"faces: {nx} x {ny} x {nz}, largest slot {max(g.face_sizes)} cells")
    st = torch.cuda.current_stream()
    u = g.field()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(65)
    g.owned(u).uniform_(-1.0, 1.0, generator=gen)
    faces = g.faces()
    _abi.rtm_pack_halo(g.c, u, faces, st)
    torch.cuda.synchronize()
    o = g.owned(u)
    owned_faces = [o[:, :, :R], o[:, :, nx - R:], o[:, :R, :], o[:, ny - R:, :], o[:R], o[nz - R:]]
    slots = g.face_slots(faces)
    for f in range(6):
        assert bool(torch.equal(slots[f].view(owned_faces[f].shape), owned_faces[f])), f
    _say("faces: pack checked")
    w = g.field()
    _abi.rtm_unpack_halo(g.c, w, slots, st)
    torch.cuda.synchronize()
    pad = g.padded(w)
    ghosts = [pad[R:R + nz, R:R + ny, :R], pad[R:R + nz, R:R + ny, nx + R:],
              pad[R:R + nz, :R, R:R + nx], pad[R:R + nz, ny + R:, R:R + nx],
              pad[:R, R:R + ny, R:R + nx], pad[nz + R:, R:R + ny, R:R + nx]]
    for f in range(6):
        assert bool(torch.equal(ghosts[f], owned_faces[f])), f
    assert int(torch.count_nonzero(g.owned(w))) == 0
    _say("faces: unpack checked")
    del u, w, faces, slots, owned_faces, ghosts, pad, o
    torch.cuda.empty_cache()
