"""The fused first and last corrector layers against the separate calls they stand for, bit for bit.

rtm_cnn_conv3d_first must give the BF16 volume of rtm_cnn_pack_input followed by rtm_cnn_conv3d, and
rtm_cnn_conv3d_apply the levels of rtm_cnn_conv3d (two FP32 output channels) followed by
rtm_cnn_apply_correction; the separate calls are checked against the oracle in test_gpu_cnn.  Grids
are radius-2 coarse grids with ragged x, y and z tiles (64-voxel x tiles, 4-row y tiles)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
C = 16
GRIDS = [(48, 13, 11), (80, 7, 5), (16, 4, 4)]


def _say(msg):
    print(msg, flush=True)


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _grid(shape):
    from paper_1603_03971_amd.grid import Grid

    nx, ny, nz = shape
    return Grid(nx, ny, nz, 20.0, Grid.stable_dt(2, 20.0, 3000.0), radius=2, sponge_width=2)


def _bf16(a):
    return oracle.bf16_rne(np.asarray(a, dtype=np.float32)).view(np.int16)


def _state(g, seed):
    from paper_1603_03971_amd import synth

    a = synth.random_field(g.shape, seed)
    b = a + 0.1 * synth.random_field(g.shape, seed + 1)
    vel = synth.random_smooth_velocity(g.shape, seed + 2, 1500, 3000).astype(np.float32)
    return a, b, vel


@pytest.mark.parametrize("shape", GRIDS)
@pytest.mark.parametrize("relu", [0, 1])
@pytest.mark.parametrize("zero_scale", [False, True])
def test_conv3d_first_is_pack_then_conv(shape, relu, zero_scale):
    import torch

    from paper_1603_03971_amd import _abi, learned

    g = _grid(shape)
    nx, ny, nz = shape
    st = torch.cuda.current_stream()
    a, b, vel = _state(g, 1200 + nx + relu)
    ua, ub, dv = g.upload(a), g.upload(b), _dev(vel.reshape(-1))
    s = torch.zeros(1, dtype=torch.float32, device="cuda")
    if not zero_scale:
        _abi.rtm_field_absmax(g.c, ua, s, st)
    rng = np.random.default_rng(1300 + nx)
    w = _dev(_bf16(rng.standard_normal((27, C, C)) * 0.2).reshape(-1))
    bias = _dev(rng.standard_normal(C).astype(np.float32))
    npad = (nx + 2) * (ny + 2) * (nz + 2) * C
    x = torch.zeros(npad, dtype=torch.int16, device="cuda")
    y_ref = torch.zeros(npad, dtype=torch.int16, device="cuda")
    y = torch.zeros(npad, dtype=torch.int16, device="cuda")
    _say(f"conv3d_first {shape} relu={relu} zero_scale={zero_scale}")
    _abi.rtm_cnn_pack_input(g.c, ua, ub, dv, learned.V_REF, learned.V_SCALE, s, x, stream=st)
    _abi.rtm_cnn_conv3d(nx, ny, nz, x, w, bias, relu, None, y_ref, st)
    _abi.rtm_cnn_conv3d_first(g.c, ua, ub, dv, learned.V_REF, learned.V_SCALE, s, w, bias, relu, y, st)
    torch.cuda.synchronize()
    assert torch.equal(y, y_ref)
    # the levels and the velocity are only read
    assert np.array_equal(g.download(ua), a.astype(np.float32))
    assert np.array_equal(g.download(ub), b.astype(np.float32))
    if zero_scale:
        # s = 0: zero input, so the output is the bias (through the ReLU)
        h = y.cpu().numpy().reshape(nz + 2, ny + 2, nx + 2, C)[1:-1, 1:-1, 1:-1]
        bb = bias.cpu().numpy()
        assert np.array_equal(h, np.broadcast_to(_bf16(np.maximum(bb, 0) if relu else bb), h.shape))
    else:
        assert x.any() and y.any()


@pytest.mark.parametrize("shape", GRIDS)
@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("with_bias", [False, True])
def test_conv3d_apply_is_conv_then_apply(shape, masked, with_bias):
    import torch

    from paper_1603_03971_amd import _abi

    g = _grid(shape)
    nx, ny, nz = shape
    st = torch.cuda.current_stream()
    a, b, _ = _state(g, 1400 + nx)
    rng = np.random.default_rng(1500 + nx + 2 * masked + with_bias)
    h = np.zeros((nz + 2, ny + 2, nx + 2, C), dtype=np.int16)
    h[1:-1, 1:-1, 1:-1] = _bf16(rng.standard_normal((nz, ny, nx, C)))
    x = _dev(h.reshape(-1))
    w = _dev(_bf16(rng.standard_normal((27, C, C)) * 0.1).reshape(-1))
    bias = _dev(rng.standard_normal(C).astype(np.float32)) if with_bias else None
    mask = None
    if masked:
        # per-cell weights in [0, 1], a fifth of them 0 (cells the correction must leave untouched)
        mk = rng.uniform(0.0, 1.0, g.points).astype(np.float32)
        mk[rng.uniform(size=g.points) < 0.2] = 0.0
        mask = _dev(mk)
    s = torch.full((1,), 0.37, dtype=torch.float32, device="cuda")
    ref_cur, ref_prv, cur, prv = g.upload(a), g.upload(b), g.upload(a), g.upload(b)
    out = torch.zeros(g.points * 2, dtype=torch.float32, device="cuda")
    _say(f"conv3d_apply {shape} masked={masked} bias={with_bias}")
    _abi.rtm_cnn_conv3d(nx, ny, nz, x, w, bias, 0, out, None, st, y32_channels=2)
    _abi.rtm_cnn_apply_correction(g.c, ref_cur, ref_prv, out, s, st, out_channels=2, mask=mask)
    _abi.rtm_cnn_conv3d_apply(g.c, x, w, bias, 0, cur, prv, s, mask=mask, stream=st)
    torch.cuda.synchronize()
    # whole padded fields: the owned cells bitwise, the ghost ring untouched
    assert torch.equal(cur, ref_cur)
    assert torch.equal(prv, ref_prv)
    assert not np.array_equal(g.download(cur), a.astype(np.float32))


def test_corrector_fused_equals_separate_calls():
    """Corrector.apply (absmax, fused first layer, middle layer, fused last layer) against absmax,
    pack, the three-layer forward and apply on a copy of the same state."""
    import torch

    from paper_1603_03971_amd import _abi, learned
    from paper_1603_03971_amd.propagator import Propagator

    g = _grid((48, 13, 11))
    st = torch.cuda.current_stream()
    a, b, vel = _state(g, 1600)
    for relu in (False, True):
        net = learned.CorrectorNet(seed=7, relu=relu, out_init=0.3)
        corr = learned.Corrector(net, g, vel, every=1)
        corr.set_mask(learned.injection_mask(g, [(20, 6, 5)]))
        prop = Propagator(g, g.field(0.1), schedule="serial")
        prop.u_cur.copy_(g.upload(a))
        prop.u_prv.copy_(g.upload(b))
        ref_cur, ref_prv = g.upload(a), g.upload(b)
        corr.apply(prop)
        ws = learned.Workspace(g.nx, g.ny, g.nz)
        s = torch.zeros(1, dtype=torch.float32, device="cuda")
        _abi.rtm_field_absmax(g.c, ref_cur, s, st)
        _abi.rtm_cnn_pack_input(g.c, ref_cur, ref_prv, corr.vel, learned.V_REF, learned.V_SCALE, s, ws.x, stream=st)
        learned.forward(net, ws, st)
        _abi.rtm_cnn_apply_correction(g.c, ref_cur, ref_prv, ws.out, s, st, out_channels=ws.out_channels,
                                      mask=corr.mask)
        torch.cuda.synchronize()
        _say(f"corrector relu={relu}: max change {float((prop.u_cur - g.upload(a)).abs().max()):.3e}")
        assert torch.equal(g.owned(prop.u_cur), g.owned(ref_cur))
        assert torch.equal(g.owned(prop.u_prv), g.owned(ref_prv))
        assert not np.array_equal(g.download(prop.u_cur), a.astype(np.float32))


def test_fused_layer_argument_checks():
    import torch

    from paper_1603_03971_amd import _abi, learned

    g = _grid((48, 13, 11))
    st = torch.cuda.current_stream()
    u, v = g.field(), g.field()
    s = torch.ones(1, dtype=torch.float32, device="cuda")
    vel = torch.full((g.points,), 2000.0, dtype=torch.float32, device="cuda")
    w = torch.zeros(27 * C * C, dtype=torch.int16, device="cuda")
    y = torch.zeros(50 * 15 * 13 * C, dtype=torch.int16, device="cuda")
    with pytest.raises(RuntimeError):
        _abi.rtm_cnn_conv3d_first(g.c, u, v, vel, learned.V_REF, 0.0, s, w, None, 0, y, st)     # v_scale
    with pytest.raises(RuntimeError):
        _abi.rtm_cnn_conv3d_first(g.c, u, v, vel, learned.V_REF, 1.0, s, w[1:], None, 0, y, st)  # w misaligned
    with pytest.raises(RuntimeError):
        _abi.rtm_cnn_conv3d_apply(g.c, y, w, None, 0, u, u, s, stream=st)                       # u_cur == u_prv
    with pytest.raises(RuntimeError):
        _abi.rtm_cnn_conv3d_apply(g.c, y, w, None, 0, u, v, None, stream=st)                    # no scale
    g17 = _grid((17, 8, 8))
    with pytest.raises(RuntimeError):
        _abi.rtm_cnn_conv3d_apply(g17.c, y, w, None, 0, g17.field(), g17.field(), s, stream=st)  # nx % 16
