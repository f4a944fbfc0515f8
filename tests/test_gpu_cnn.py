"""GPU CNN kernels (BF16 MFMA, FP32 accumulation) against the FP64 oracle.

Inputs are quantised to BF16 on the host (round to nearest even, by the oracle's own codec) and the
oracle receives the same quantised values, so each kernel differs from the oracle only by FP32
summation order; the whole network, whose activations the GPU rounds to BF16 between layers, is
compared at a BF16-level tolerance."""
import numpy as np
import pytest

import oracle
from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu
C = 16


def _say(msg):
    print(msg, flush=True)


def _q(a):
    """(BF16 codes as int16, their FP64 values) of an FP32-rounded array."""
    codes = oracle.bf16_rne(np.asarray(a, dtype=np.float32))
    return codes.view(np.int16), oracle.bf16_to_f32(codes).astype(np.float64)


def _with_halo(codes):
    nz, ny, nx, c = codes.shape
    out = np.zeros((nz + 2, ny + 2, nx + 2, c), dtype=np.int16)
    out[1:-1, 1:-1, 1:-1] = codes
    return out


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return oracle.rel_l2(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))


SHAPES = [(5, 7, 48), (3, 9, 80), (1, 1, 16)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("relu", [0, 1])
def test_conv3d_forward(shape, relu):
    import torch

    from paper_1603_03971_amd import _abi

    nz, ny, nx = shape
    rng = np.random.default_rng(400 + nx + relu)
    xc, xv = _q(rng.standard_normal((nz, ny, nx, C)))
    wc, wv = _q(rng.standard_normal((27, C, C)) * 0.2)
    b = rng.standard_normal(C).astype(np.float32)
    _say(f"conv3d {shape} relu={relu}")
    x = _dev(_with_halo(xc).reshape(-1))
    w = _dev(wc.reshape(-1))
    y32 = torch.zeros(nz * ny * nx * C, dtype=torch.float32, device="cuda")
    y16 = torch.zeros((nz + 2) * (ny + 2) * (nx + 2) * C, dtype=torch.int16, device="cuda")
    _abi.rtm_cnn_conv3d(nx, ny, nz, x, w, _dev(b), relu, y32, y16, torch.cuda.current_stream())
    torch.cuda.synchronize()
    ref = ocnn.conv3d(xv, wv, b.astype(np.float64), relu=bool(relu))
    got = y32.cpu().numpy().reshape(nz, ny, nx, C)
    e = _rel(got, ref)
    _say(f"  rel-L2 {e:.2e}, max abs {np.max(np.abs(got - ref)):.2e}")
    assert e <= 1e-6
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))
    # BF16 output: the kernel's rounding of its own FP32 result, bit for bit, and an untouched halo
    h = y16.cpu().numpy().reshape(nz + 2, ny + 2, nx + 2, C)
    assert np.array_equal(h[1:-1, 1:-1, 1:-1], oracle.bf16_rne(got).view(np.int16))
    h[1:-1, 1:-1, 1:-1] = 0
    assert not h.any()


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3d_weight_gradient(shape):
    import torch

    from paper_1603_03971_amd import _abi

    nz, ny, nx = shape
    rng = np.random.default_rng(500 + nx)
    xc, xv = _q(rng.standard_normal((nz, ny, nx, C)))
    dz = rng.standard_normal((nz, ny, nx, C)).astype(np.float32)
    _, dzq = _q(dz)
    dw0 = rng.standard_normal((27, C, C)).astype(np.float32)
    db0 = rng.standard_normal(C).astype(np.float32)
    _say(f"wgrad {shape}")
    dw = _dev(dw0.reshape(-1))
    db = _dev(db0)
    _abi.rtm_cnn_conv3d_wgrad(nx, ny, nz, _dev(_with_halo(xc).reshape(-1)), _dev(dz.reshape(-1)), dw, db,
                              torch.cuda.current_stream())
    torch.cuda.synchronize()
    ref_w, _ = ocnn.conv3d_wgrad(xv, dzq)
    _, ref_b = ocnn.conv3d_wgrad(xv, dz.astype(np.float64))
    gw = dw.cpu().numpy().reshape(27, C, C) - dw0.astype(np.float64)
    gb = db.cpu().numpy() - db0.astype(np.float64)
    ew, eb = _rel(gw, ref_w), _rel(gb, ref_b)
    _say(f"  dW rel-L2 {ew:.2e}, db rel-L2 {eb:.2e}")
    assert ew <= 1e-5 and eb <= 1e-5
    # the fixed-order variant: the same sums to the same tolerance, and the same bits on every call
    npart = _abi.rtm_cnn_wgrad_partials(nx, ny, nz)
    part = torch.full((npart,), float("nan"), device="cuda")
    xd, dzd = _dev(_with_halo(xc).reshape(-1)), _dev(dz.reshape(-1))
    outs = []
    for _ in range(2):
        dw2, db2 = _dev(dw0.reshape(-1)), _dev(db0)
        _abi.rtm_cnn_conv3d_wgrad_ordered(nx, ny, nz, xd, dzd, dw2, db2, part, npart, torch.cuda.current_stream())
        torch.cuda.synchronize()
        outs.append((dw2.cpu().numpy(), db2.cpu().numpy()))
    gw2 = outs[0][0].reshape(27, C, C) - dw0.astype(np.float64)
    gb2 = outs[0][1] - db0.astype(np.float64)
    assert _rel(gw2, ref_w) <= 1e-5 and _rel(gb2, ref_b) <= 1e-5
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("shape", SHAPES[:2])
def test_data_gradient_by_flipped_convolution(shape):
    import torch

    from paper_1603_03971_amd import _abi

    nz, ny, nx = shape
    rng = np.random.default_rng(600 + nx)
    wc, wv = _q(rng.standard_normal((27, C, C)) * 0.2)
    y = rng.standard_normal((nz, ny, nx, C)).astype(np.float32)
    dy = rng.standard_normal((nz, ny, nx, C)).astype(np.float32)
    st = torch.cuda.current_stream()
    n, npad = nz * ny * nx * C, (nz + 2) * (ny + 2) * (nx + 2) * C
    dz32 = torch.zeros(n, dtype=torch.float32, device="cuda")
    dz16 = torch.zeros(npad, dtype=torch.int16, device="cuda")
    wt = torch.zeros(27 * C * C, dtype=torch.int16, device="cuda")
    dx = torch.zeros(n, dtype=torch.float32, device="cuda")
    _say(f"dgrad {shape}")
    _abi.rtm_cnn_relu_backward(nx, ny, nz, _dev(y.reshape(-1)), _dev(dy.reshape(-1)), 1, C, dz32, dz16, st)
    _abi.rtm_cnn_weight_flip(_dev(wc.reshape(-1)), wt, st)
    _abi.rtm_cnn_conv3d(nx, ny, nz, dz16, wt, None, 0, dx, None, st)
    torch.cuda.synchronize()
    dz_ref = np.where(y > 0, dy, np.float32(0.0))            # +0 where the ReLU is off, like the kernel
    assert np.array_equal(dz32.cpu().numpy().reshape(nz, ny, nx, C), dz_ref)
    dzc, dzv = _q(dz_ref)
    assert np.array_equal(dz16.cpu().numpy().reshape(nz + 2, ny + 2, nx + 2, C)[1:-1, 1:-1, 1:-1], dzc)
    ref = ocnn.conv3d_dgrad(dzv, wv)
    e = _rel(dx.cpu().numpy().reshape(nz, ny, nx, C), ref)
    _say(f"  dx rel-L2 {e:.2e}")
    assert e <= 1e-6


def test_loss_gradient_and_adam():
    import torch

    from paper_1603_03971_amd import _abi

    nz, ny, nx = 3, 5, 32
    rng = np.random.default_rng(700)
    out = rng.standard_normal((nz, ny, nx, C)).astype(np.float32)
    tgt = rng.standard_normal((nz, ny, nx, C)).astype(np.float32)
    n, npad = out.size, (nz + 2) * (ny + 2) * (nx + 2) * C
    dz32 = torch.zeros(n, dtype=torch.float32, device="cuda")
    dz16 = torch.zeros(npad, dtype=torch.int16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    _abi.rtm_cnn_loss_grad(nx, ny, nz, _dev(out.reshape(-1)), _dev(tgt.reshape(-1)), 2, dz32, dz16, loss,
                           torch.cuda.current_stream())
    torch.cuda.synchronize()
    d = np.zeros_like(out)
    d[..., :2] = out[..., :2] - tgt[..., :2]
    assert np.array_equal(dz32.cpu().numpy().reshape(out.shape), d)
    ref_loss = 0.5 * np.sum(d.astype(np.float64) ** 2)
    assert abs(float(loss.item()) - ref_loss) <= 1e-12 * ref_loss
    loss.zero_()
    _abi.rtm_cnn_loss_grad(nx, ny, nz, _dev(out.reshape(-1)), _dev(tgt.reshape(-1)), 2, dz32, dz16, loss,
                           torch.cuda.current_stream(), weight=0.25)
    torch.cuda.synchronize()
    assert np.array_equal(dz32.cpu().numpy().reshape(out.shape), np.float32(0.25) * d)
    assert abs(float(loss.item()) - 0.25 * ref_loss) <= 1e-12 * ref_loss
    # per-voxel mask: w = weight * mask
    mk = rng.uniform(0.0, 1.0, (nz, ny, nx)).astype(np.float32)
    loss.zero_()
    _abi.rtm_cnn_loss_grad(nx, ny, nz, _dev(out.reshape(-1)), _dev(tgt.reshape(-1)), 2, dz32, dz16, loss,
                           torch.cuda.current_stream(), weight=0.5, mask=_dev(mk.reshape(-1)))
    torch.cuda.synchronize()
    wv = (np.float32(0.5) * mk)[..., None]
    assert np.array_equal(dz32.cpu().numpy().reshape(out.shape), wv * d)
    ref_m = 0.5 * np.sum(wv.astype(np.float64) * d.astype(np.float64) ** 2)
    assert abs(float(loss.item()) - ref_m) <= 1e-5 * ref_m
    # Adam: three steps against the update rule written out in FP64
    p0 = rng.standard_normal(1000).astype(np.float32)
    p = _dev(p0.copy())
    m1 = torch.zeros_like(p)
    m2 = torch.zeros_like(p)
    p16 = torch.zeros(1000, dtype=torch.int16, device="cuda")
    P, M, V = p0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in (1, 2, 3):
        g = rng.standard_normal(1000).astype(np.float32)
        _abi.rtm_cnn_adam(p, _dev(g), m1, m2, 1000, 1e-2, 0.9, 0.999, 1e-8, step, p16, torch.cuda.current_stream())
        M = 0.9 * M + 0.1 * g
        V = 0.999 * V + 0.001 * g.astype(np.float64) ** 2
        P = P - 1e-2 * (M / (1 - 0.9 ** step)) / (np.sqrt(V / (1 - 0.999 ** step)) + 1e-8)
    torch.cuda.synchronize()
    got = p.cpu().numpy()
    assert np.max(np.abs(got - P)) <= 1e-5
    assert np.array_equal(p16.cpu().numpy(), oracle.bf16_rne(got).view(np.int16))


def test_network_gradient_matches_oracle():
    """Forward and backward of the three-layer network through the library against the FP64
    oracle with the same (BF16-rounded) weights; the GPU also rounds activations and output
    gradients to BF16 between layers, hence the BF16-level tolerance."""
    import torch

    from paper_1603_03971_amd import learned

    nz, ny, nx = 6, 9, 32
    net = learned.CorrectorNet(seed=3, out_init=1.0, bias=True)
    rng = np.random.default_rng(800)
    p = net.state()
    for layer in range(3):
        p[layer * learned.LAYER + learned.WEIGHTS:(layer + 1) * learned.LAYER] = rng.standard_normal(C) * 0.1
    net.load(p)
    xin = np.zeros((nz, ny, nx, C), dtype=np.float32)
    xin[..., :4] = rng.standard_normal((nz, ny, nx, 4))
    xc, xv = _q(xin)
    tgt = np.zeros((nz, ny, nx, C), dtype=np.float32)
    tgt[..., :2] = rng.standard_normal((nz, ny, nx, 2)) * 0.5
    ws = learned.Workspace(nx, ny, nz, train=True)
    ws.x.copy_(_dev(_with_halo(xc).reshape(-1)))
    ws.target.copy_(_dev(tgt.reshape(-1)))
    learned.forward(net, ws)
    learned.backward(net, ws)
    torch.cuda.synchronize()
    layers = net.layers_host()
    params = [(oracle.bf16_to_f32(oracle.bf16_rne(w.astype(np.float32))).astype(np.float64), b) for w, b in layers]
    loss, grads = ocnn.loss_and_grads(xv, tgt, params)
    out_ref, _ = ocnn.forward(xv, params)
    out = ws.out.cpu().numpy().reshape(nz, ny, nx, C)
    eo = _rel(out[..., :2], out_ref[..., :2])
    el = abs(float(ws.loss.item()) - loss) / loss
    _say(f"network: out rel-L2 {eo:.2e}, loss rel {el:.2e}")
    assert eo <= 1e-2 and el <= 1e-2
    g = net.grad.cpu().numpy().astype(np.float64)
    for layer in range(3):
        gw = g[layer * learned.LAYER:layer * learned.LAYER + learned.WEIGHTS].reshape(27, C, C)
        gb = g[layer * learned.LAYER + learned.WEIGHTS:(layer + 1) * learned.LAYER]
        ew, eb = _rel(gw, grads[layer][0]), _rel(gb, grads[layer][1])
        cos = float(np.sum(gw * grads[layer][0]) / (np.linalg.norm(gw) * np.linalg.norm(grads[layer][0])))
        _say(f"  layer {layer}: dW rel-L2 {ew:.2e} (cos {cos:.6f}), db rel-L2 {eb:.2e}")
        assert ew <= 2e-2 and eb <= 2e-2 and cos >= 0.999


@pytest.mark.parametrize("relu,masked", [(False, True), (False, False)])
def test_trained_network_loss_and_gradients_match_oracle(relu, masked):
    """The network the corrector trains (linear, the default) with its masked, weighted window loss:
    forward, loss and every parameter group's gradient through the library against the FP64 oracle
    (oracle/cnn.py with the same relu flag, mask and weight), at the BF16-level tolerance of the
    whole network (activations rounded to BF16 between layers).  The ReLU network is covered by
    test_network_gradient_matches_oracle; with ReLU the two sides take the ReLU decisions on values
    of different precision (FP32 from BF16 operands against FP64), so its gradients differ more."""
    import torch

    from paper_1603_03971_amd import learned

    nz, ny, nx = 6, 9, 32
    net = learned.CorrectorNet(seed=5, out_init=1.0, bias=False, relu=relu)
    rng = np.random.default_rng(801)
    xin = np.zeros((nz, ny, nx, C), dtype=np.float32)
    xin[..., :4] = rng.standard_normal((nz, ny, nx, 4))
    xc, xv = _q(xin)
    tgt = np.zeros((nz, ny, nx, C), dtype=np.float32)
    tgt[..., :2] = rng.standard_normal((nz, ny, nx, 2)) * 0.5
    weight = 0.37
    mask = None
    if masked:
        mask = rng.uniform(0.0, 1.0, (nz, ny, nx)).astype(np.float32)
        mask[:, :2] = 0.0                                   # a masked-off band, as near injection cells
    ws = learned.Workspace(nx, ny, nz, train=True)
    ws.x.copy_(_dev(_with_halo(xc).reshape(-1)))
    ws.target.copy_(_dev(tgt.reshape(-1)))
    learned.forward(net, ws)
    learned.backward(net, ws, weight=weight, mask=None if mask is None else _dev(mask.reshape(-1)))
    torch.cuda.synchronize()
    params = [(oracle.bf16_to_f32(oracle.bf16_rne(w.astype(np.float32))).astype(np.float64), b)
              for w, b in net.layers_host()]
    loss, grads = ocnn.loss_and_grads(xv, tgt, params, relu=relu, mask=mask, weight=weight)
    out_ref, _ = ocnn.forward(xv, params, relu=relu)
    out = ws.out.cpu().numpy().reshape(nz, ny, nx, C)
    eo = _rel(out[..., :2], out_ref[..., :2])
    el = abs(float(ws.loss.item()) - loss) / loss
    _say(f"network relu={relu} masked={masked}: out rel-L2 {eo:.2e}, loss rel {el:.2e}")
    assert eo <= 1e-2 and el <= 1e-2
    g = net.grad.cpu().numpy().astype(np.float64)
    for layer in range(3):
        gw = g[layer * learned.LAYER:layer * learned.LAYER + learned.WEIGHTS].reshape(27, C, C)
        ew = _rel(gw, grads[layer][0])
        cos = float(np.sum(gw * grads[layer][0]) / (np.linalg.norm(gw) * np.linalg.norm(grads[layer][0])))
        _say(f"  layer {layer}: dW rel-L2 {ew:.2e} (cos {cos:.6f})")
        assert ew <= 2e-2 and cos >= 0.999


def test_restrict_absmax_pack_target_apply():
    import torch

    from paper_1603_03971_amd import _abi, learned, synth
    from paper_1603_03971_amd.grid import Grid

    fine = Grid(64, 36, 22, 10.0, Grid.stable_dt(4, 10.0, 3000.0), sponge_width=4)
    coarse = learned.coarse_grid(fine)
    assert (coarse.nx, coarse.ny, coarse.nz, coarse.radius, coarse.sponge_width) == (32, 18, 11, 2, 2)
    st = torch.cuda.current_stream()
    uf = synth.random_field(fine.shape, 900)
    a, b = synth.random_field(coarse.shape, 901), synth.random_field(coarse.shape, 902)
    ra, rb = synth.random_field(coarse.shape, 903), synth.random_field(coarse.shape, 904)
    vel = synth.random_smooth_velocity(coarse.shape, 905, 1500, 3000).astype(np.float32)
    fu = fine.upload(uf)
    cu = coarse.field()
    _abi.rtm_restrict(fine.c, coarse.c, fu, cu, st)
    cfw = coarse.field()
    _abi.rtm_restrict(fine.c, coarse.c, fu, cfw, st, mode=_abi.RTM_RESTRICT_FULL)
    s = torch.zeros(1, dtype=torch.float32, device="cuda")
    fa, fb = coarse.upload(a), coarse.upload(b)
    _abi.rtm_field_absmax(coarse.c, fa, s, st)
    x = torch.zeros(34 * 20 * 13 * C, dtype=torch.int16, device="cuda")
    _abi.rtm_cnn_pack_input(coarse.c, fa, fb, _dev(vel.reshape(-1)), learned.V_REF, learned.V_SCALE, s, x, stream=st)
    tgt = torch.zeros(coarse.points * C, dtype=torch.float32, device="cuda")
    _abi.rtm_cnn_target(coarse.c, coarse.upload(ra), coarse.upload(rb), fa, fb, s, tgt, stream=st)
    torch.cuda.synchronize()
    assert np.array_equal(coarse.download(cu), uf.astype(np.float32)[::2, ::2, ::2])
    # full weighting: the (1/4, 1/2, 1/4)^3 average around (2i, 2j, 2k), zero ghosts outside the box
    pad = np.pad(uf.astype(np.float32).astype(np.float64), 1)
    wts = (0.25, 0.5, 0.25)
    ref_fw = np.zeros(coarse.shape)
    nzc, nyc, nxc = coarse.shape
    for oz in range(3):
        for oy in range(3):
            for ox in range(3):
                ref_fw += wts[oz] * wts[oy] * wts[ox] * pad[oz:oz + 2 * nzc:2, oy:oy + 2 * nyc:2, ox:ox + 2 * nxc:2]
    assert oracle.rel_l2(coarse.download(cfw), ref_fw) <= 1e-6
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    smax = np.float32(np.max(np.abs(a32)))
    assert float(s.item()) == smax
    inv = np.float32(1.0) / smax
    xs = x.cpu().numpy().reshape(13, 20, 34, C)[1:-1, 1:-1, 1:-1]
    xa, xd = a32 * inv, (a32 - b32) * inv
    assert np.array_equal(xs[..., 0], oracle.bf16_rne(xa).view(np.int16))
    assert np.array_equal(xs[..., 1], oracle.bf16_rne(xd).view(np.int16))
    m = (vel - np.float32(learned.V_REF)) * (np.float32(1.0) / np.float32(learned.V_SCALE))
    assert np.array_equal(xs[..., 2], oracle.bf16_rne(m * xa).view(np.int16))
    assert np.array_equal(xs[..., 3], oracle.bf16_rne(m * xd).view(np.int16))
    assert not xs[..., 4:].any()
    t = tgt.cpu().numpy().reshape(coarse.shape + (C,))
    ra32, rb32 = ra.astype(np.float32), rb.astype(np.float32)
    assert np.array_equal(t[..., 0], (ra32 - a32) * inv)
    assert np.array_equal(t[..., 1], ((ra32 - rb32) - (a32 - b32)) * inv)
    assert not t[..., 2:].any()
    out = np.zeros(coarse.shape + (C,), dtype=np.float32)
    out[..., :2] = np.random.default_rng(906).standard_normal(coarse.shape + (2,))
    _abi.rtm_cnn_apply_correction(coarse.c, fa, fb, _dev(out.reshape(-1)), s, st, out_channels=C)
    torch.cuda.synchronize()
    ref = np.float64(smax) * out[..., 0] + a32              # exact product, then one FP64 rounding
    got = coarse.download(fa).astype(np.float64)
    assert np.all(np.abs(got - ref) <= np.spacing(np.abs(ref).astype(np.float32)))
    refb = np.float64(smax) * (out[..., 0] - out[..., 1]) + b32     # u^{n-1} += s (o0 - o1)
    gotb = coarse.download(fb).astype(np.float64)
    assert np.all(np.abs(gotb - refb) <= np.spacing(np.abs(refb).astype(np.float32)))
    # with a mask the correction is scaled per cell (0 leaves the cell untouched)
    mk = learned.injection_mask(coarse, [(5, 6, 4)])
    assert mk[4, 6, 5] == 0.0 and mk.max() == 1.0
    before = coarse.download(fa)
    _abi.rtm_cnn_apply_correction(coarse.c, fa, fb, _dev(out.reshape(-1)), s, st, out_channels=C,
                                  mask=_dev(mk.reshape(-1)))
    torch.cuda.synchronize()
    after = coarse.download(fa)
    assert np.array_equal(after[mk == 0], before[mk == 0])
    c32 = np.float32(smax) * mk                                     # the kernel's FP32 factor
    ref2 = c32.astype(np.float64) * out[..., 0] + before            # then one rounding, like fmaf
    ulp = np.spacing(np.abs(ref2).astype(np.float32))
    assert float(np.max(np.abs(after - ref2) / ulp)) <= 1.0


def test_conv3d_partial_output_channels_and_noise_inputs():
    """y32 with only the first 2 of 16 channels (the correction layer's inference layout), and the
    noise arguments of the input packing and target kernels."""
    import torch

    from paper_1603_03971_amd import _abi, learned, synth
    from paper_1603_03971_amd.grid import Grid

    nz, ny, nx = 4, 6, 96
    rng = np.random.default_rng(950)
    xc, xv = _q(rng.standard_normal((nz, ny, nx, C)))
    wc, wv = _q(rng.standard_normal((27, C, C)) * 0.2)
    y2 = torch.full((nz * ny * nx * 2,), -7.0, dtype=torch.float32, device="cuda")
    _abi.rtm_cnn_conv3d(nx, ny, nz, _dev(_with_halo(xc).reshape(-1)), _dev(wc.reshape(-1)), None, 0, y2, None,
                        torch.cuda.current_stream(), y32_channels=2)
    torch.cuda.synchronize()
    ref = ocnn.conv3d(xv, wv)[..., :2]
    assert _rel(y2.cpu().numpy().reshape(nz, ny, nx, 2), ref) <= 1e-6

    g = Grid(32, 10, 7, 20.0, 1e-3, radius=2, sponge_width=3)
    a, b, ra, rb = (synth.random_field(g.shape, s) for s in (951, 952, 953, 954))
    vel = np.full(g.shape, 3000.0, dtype=np.float32)
    noise = (rng.standard_normal(g.shape + (2,)) * 0.01).astype(np.float32)
    st = torch.cuda.current_stream()
    s_ = torch.tensor([2.0], dtype=torch.float32, device="cuda")
    x = torch.zeros(34 * 12 * 9 * C, dtype=torch.int16, device="cuda")
    tgt = torch.zeros(g.points * C, dtype=torch.float32, device="cuda")
    fa, fb = g.upload(a), g.upload(b)
    nd = _dev(noise.reshape(-1))
    _abi.rtm_cnn_pack_input(g.c, fa, fb, _dev(vel.reshape(-1)), learned.V_REF, learned.V_SCALE, s_, x, noise=nd,
                            stream=st)
    _abi.rtm_cnn_target(g.c, g.upload(ra), g.upload(rb), fa, fb, s_, tgt, noise=nd, stream=st)
    torch.cuda.synchronize()
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    half = np.float32(0.5)
    xa = a32 * half + noise[..., 0]
    xd = (a32 - b32) * half + noise[..., 1]
    xs = x.cpu().numpy().reshape(9, 12, 34, C)[1:-1, 1:-1, 1:-1]
    assert np.array_equal(xs[..., 0], oracle.bf16_rne(xa).view(np.int16))
    assert np.array_equal(xs[..., 1], oracle.bf16_rne(xd).view(np.int16))
    m = (np.float32(3000.0) - np.float32(learned.V_REF)) * (np.float32(1.0) / np.float32(learned.V_SCALE))
    assert np.array_equal(xs[..., 2], oracle.bf16_rne(m * xa).view(np.int16))
    t = tgt.cpu().numpy().reshape(g.shape + (C,))
    ra32, rb32 = ra.astype(np.float32), rb.astype(np.float32)
    assert np.array_equal(t[..., 0], (ra32 - a32) * half - noise[..., 0])
    assert np.array_equal(t[..., 1], ((ra32 - rb32) - (a32 - b32)) * half - noise[..., 1])


@pytest.mark.parametrize("radius,shape", [(2, (37, 5, 48)), (4, (9, 70, 64)), (2, (4, 4, 16))])
def test_field_absmax_covers_every_owned_cell_and_no_ghost(radius, shape):
    """rtm_field_absmax on ragged grids: the extreme sits in turn at each corner cell (one of them
    negative), while the ghost ring holds larger values that must not count."""
    import torch

    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    nz, ny, nx = shape
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(radius, 10.0, 3000.0), radius=radius, sponge_width=2)
    st = torch.cuda.current_stream()
    base = np.random.default_rng(1700 + nx).uniform(-1.0, 1.0, g.shape).astype(np.float32)
    s = torch.zeros(1, dtype=torch.float32, device="cuda")
    corners = [(k, j, i) for k in (0, nz - 1) for j in (0, ny - 1) for i in (0, nx - 1)]
    for n, (k, j, i) in enumerate(corners):
        a = base.copy()
        peak = np.float32(3.0 + n) * (np.float32(-1.0) if n % 2 else np.float32(1.0))
        a[k, j, i] = peak
        f = g.upload(a)
        pad = g.padded(f)
        pad[0].fill_(1e6)                       # a ghost plane below the box
        pad[:, :, 0].fill_(-1e6)                # a ghost column
        g.owned(f).copy_(torch.from_numpy(a).cuda())
        _abi.rtm_field_absmax(g.c, f, s, st)
        torch.cuda.synchronize()
        assert float(s.item()) == abs(float(peak)), (k, j, i)
