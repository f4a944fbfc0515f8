"""GPU reduced-precision snapshots: codes bit-exact against the oracle's FP32 decisions, and the RTM
image with BF16 / FP16 snapshots against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1603_03971_amd import synth
from tests.test_gpu_rtm import gpu_rtm, oracle_rtm, small_rtm_inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_encode_bitexact(fmt):
    import torch

    from paper_1603_03971_amd.grid import Grid
    from paper_1603_03971_amd.snapshots import CodedSnapshots

    nx, ny, nz = 37, 22, 19
    g = Grid(nx, ny, nz, 10.0, 1e-3)
    scale = np.exp(np.random.default_rng(8).uniform(-30, 10, nz))
    scale[5] = 0.0
    u = (synth.random_field((nz, ny, nx), seed=61) * scale[:, None, None]).astype(np.float32)
    codec = CodedSnapshots(g, fmt)
    codes, scales = codec.encode(g.upload(u))
    torch.cuda.synchronize()
    want_codes, want_scales = oracle.snapshot_encode(u, fmt)
    assert np.array_equal(scales.cpu().numpy(), want_scales)
    got = codes.cpu().numpy().view(np.uint16).reshape(nz, ny, nx)
    assert np.array_equal(got, want_codes)


@pytest.fixture(scope="module")
def case():
    v_true, v_bg, src, rec = small_rtm_inputs()
    args = (v_true, v_bg, src, rec, 320, 20.0, 4)
    exact = oracle_rtm(*args)[0]
    return args, exact


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_coded_snapshot_image(case, fmt):
    """The coded path against the oracle with the same coding (parity of the path, 1e-3), and the
    image error that the coding costs against the exact FP64 image (reported; bounded by the code's
    relative precision, 2^-8 for BF16 and 2^-10 for FP16, on the image norm)."""
    from paper_1603_03971_amd import snapshots

    args, exact = case
    img = gpu_rtm(*args, snapshots=snapshots.make(fmt))[0]
    v_true, v_bg, src, rec, nsteps, fpeak, s = args
    h = 10.0
    dt = oracle.stable_dt(4, h, float(max(v_true.max(), v_bg.max())))
    sp = tuple(oracle.sponge_profile(n, 8) for n in (v_true.shape[2], v_true.shape[1], v_true.shape[0]))
    src = np.asarray(src)
    rec = np.asarray(rec)
    ws = oracle.injection_weight(v_bg[src[:, 2], src[:, 1], src[:, 0]], dt, h)
    wr = oracle.injection_weight(v_bg[rec[:, 2], rec[:, 1], rec[:, 0]], dt, h)
    amp = oracle.ricker(np.arange(nsteps) * dt, fpeak)[:, None]
    kt, kb = oracle.kappa_field(v_true, dt, h), oracle.kappa_field(v_bg, dt, h)
    d_t = oracle.forward(kt, sp, nsteps, src_ijk=src, src_w=ws, src_amp=amp, rec_ijk=rec, nthreads=8)["traces"]
    d_b = oracle.forward(kb, sp, nsteps, src_ijk=src, src_w=ws, src_amp=amp, rec_ijk=rec, nthreads=8)["traces"]
    coded_ref = oracle.migrate(kb, sp, nsteps, src_ijk=src, src_w=ws, src_amp=amp, rec_ijk=rec, rec_w=wr,
                               data=d_t - d_b, image_every=s, nthreads=8, snapshot_format=fmt)
    e_path = oracle.rel_l2(img, coded_ref)
    e_cost = oracle.rel_l2(img, exact)
    e_cost_oracle = oracle.rel_l2(coded_ref, exact)
    _say(f"{fmt} snapshots: image vs coded oracle {e_path:.3e}; vs exact FP64 image {e_cost:.3e} "
         f"(oracle's own coding cost {e_cost_oracle:.3e})")
    assert e_path <= 1e-3
    assert e_cost <= (2.0 ** -8 if fmt == "bf16" else 2.0 ** -10)


def test_f32_snapshot_image_cost(case):
    args, exact = case
    img = gpu_rtm(*args)[0]
    e = oracle.rel_l2(img, exact)
    _say(f"f32 snapshots: image vs exact FP64 image {e:.3e}")
    assert e <= 1e-3
