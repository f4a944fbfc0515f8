"""CPU checks of the C ABI: the library loads, exports every declared symbol, validates arguments
before touching a device, and its host helpers agree with the oracle's independent definitions."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "rtm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rtm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_1603_03971_amd import _abi
    return _abi


def test_exports_every_declared_symbol(abi):
    names = _declared_functions()
    assert "rtm_step_halo" in names and "rtm_image_accumulate" in names
    for name in names:
        assert hasattr(abi.lib, name), name
    assert abi.rtm_abi_version() == 1


def test_python_binding_has_same_names(abi):
    for name in _declared_functions():
        assert callable(getattr(abi, name)), name


def test_strerror(abi):
    for code in (0, -1, -2, -3, -4):
        assert abi.rtm_strerror(code)
    assert "unknown" in abi.rtm_strerror(-99)


def _grid(abi, nx=16, ny=12, nz=10, radius=4, pitch_y=None, pitch_z=None, sponge=True):
    py = pitch_y if pitch_y is not None else nx + 2 * radius
    pz = pitch_z if pitch_z is not None else py * (ny + 2 * radius)
    fake = 0x1000 if sponge else None  # host-side validation never dereferences the sponge pointers
    return abi.rtm_grid_init(nx, ny, nz, radius, py, pz, fake, fake, fake)


def test_grid_init_coefficients(abi):
    g = _grid(abi)
    np.testing.assert_allclose(np.array(g.c), oracle.fd_coefficients(4).astype(np.float32), rtol=0, atol=0)
    g2 = _grid(abi, radius=2)
    np.testing.assert_allclose(np.array(g2.c)[:3], oracle.fd_coefficients(2).astype(np.float32), rtol=0, atol=0)


@pytest.mark.parametrize("kw", [dict(radius=3), dict(nx=7), dict(nz=3, radius=2), dict(pitch_y=20),
                                dict(pitch_z=100), dict(sponge=False)])
def test_grid_init_rejects(abi, kw):
    with pytest.raises(abi.RTMError) as e:
        _grid(abi, **kw)
    assert e.value.status == abi.RTM_EINVAL


def test_validation_before_device(abi):
    """Argument errors are reported without any device call (these run on a machine with no GPU)."""
    g = _grid(abi)
    L = abi.lib
    gp = ctypes.byref(g)
    assert L.rtm_step_halo(None, 16, 32, 48, 64, None) == abi.RTM_EINVAL
    assert L.rtm_step_halo(gp, None, 32, 48, 64, None) == abi.RTM_EINVAL
    assert L.rtm_step_interior(gp, 16, 16, 48, 64, None) == abi.RTM_EALIAS          # u_nxt == u_cur
    total = g.pitch_z * (g.nz + 8)
    assert L.rtm_step_interior(gp, 4096, 4096 + 8, 4096 * 1000, 4096 * 2000, None) == abi.RTM_EALIAS
    assert L.rtm_pack_halo(gp, None, 4096, None) == abi.RTM_EINVAL
    assert L.rtm_pack_halo(gp, 4096, 4096 + 4 * total - 64, None) == abi.RTM_EALIAS
    assert L.rtm_step_halo_pack(gp, 4096, 1 << 36, 1 << 37, 1 << 38, None, None) == abi.RTM_EINVAL
    assert L.rtm_step_halo_pack(gp, 4096, 1 << 36, 1 << 37, 1 << 38, 4096 + 4 * total - 64, None) == abi.RTM_EALIAS
    assert L.rtm_step_halo_pack(gp, None, 1 << 36, 1 << 37, 1 << 38, 1 << 39, None) == abi.RTM_EINVAL
    # the halo call that reads u_cur's ghosts from six receive slots
    slots = (ctypes.c_void_p * 6)(*[(1 << 40) + 4096 * f for f in range(6)])
    one_null = (ctypes.c_void_p * 6)(*([1 << 40] * 5 + [None]))
    odd = (ctypes.c_void_p * 6)(*([1 << 40] * 5 + [(1 << 40) + 8]))              # not 16-byte aligned
    hps = L.rtm_step_halo_pack_slots
    assert hps(gp, 4096, 1 << 36, 1 << 37, 1 << 38, one_null, 1 << 39, None) == abi.RTM_EINVAL
    assert hps(gp, 4096, 1 << 36, 1 << 37, 1 << 38, odd, 1 << 39, None) == abi.RTM_EINVAL
    assert hps(gp, 4096, 1 << 36, 1 << 37, 1 << 38, None, 1 << 39, None) == abi.RTM_EINVAL
    assert hps(gp, 4096, 1 << 36, 1 << 37, 1 << 38, slots, None, None) == abi.RTM_EINVAL
    assert hps(gp, 4096, 1 << 36, 1 << 37, 1 << 38, slots, (1 << 40) + 8192, None) == abi.RTM_EALIAS  # slot 2
    assert hps(gp, (1 << 40) + 4096 * 5, 1 << 36, 1 << 37, 1 << 38, slots, 1 << 39, None) == abi.RTM_EALIAS
    assert hps(gp, 4096, 1 << 36, 1 << 37, 1 << 38, slots, 4096 + 64, None) == abi.RTM_EALIAS   # faces over u_nxt
    g2 = _grid(abi, radius=2)
    assert hps(ctypes.byref(g2), 4096, 1 << 36, 1 << 37, 1 << 38, slots, 1 << 39, None) == abi.RTM_EINVAL
    # the shell call (faces only, optional dense face copies) and the whole-block call with slots
    shp, wsl = L.rtm_step_shell_pack, L.rtm_step_whole_slots
    F = 1 << 39
    assert shp(gp, 1 << 36, 1 << 37, 1 << 38, None, None, None, slots, None, None) == abi.RTM_EINVAL      # no faces
    assert shp(gp, None, 1 << 37, 1 << 38, None, None, None, slots, F, None) == abi.RTM_EINVAL           # no u_cur
    assert shp(gp, 1 << 36, 1 << 37, 1 << 38, None, None, None, one_null, F, None) == abi.RTM_EINVAL
    assert shp(gp, 1 << 36, 1 << 37, 1 << 38, F + (1 << 30), None, None, slots, F, None) == abi.RTM_EINVAL  # 1 of 3
    assert shp(gp, 1 << 36, 1 << 37, 1 << 38, F + 8 + (1 << 30), F + (2 << 30), F + (3 << 30), slots, F,
               None) == abi.RTM_EINVAL                                                                # misaligned copy
    assert shp(gp, 1 << 36, 1 << 37, 1 << 38, F + 64, F + (2 << 30), F + (3 << 30), slots, F,
               None) == abi.RTM_EALIAS                                                                # copy over faces
    assert shp(gp, 1 << 36, 1 << 37, 1 << 38, None, None, None, slots, (1 << 40) + 8192, None) == abi.RTM_EALIAS
    assert shp(gp, 1 << 36, 1 << 37, 1 << 38, None, None, None, slots, (1 << 36) + 64, None) == abi.RTM_EALIAS
    assert shp(ctypes.byref(g2), 1 << 36, 1 << 37, 1 << 38, None, None, None, slots, F, None) == abi.RTM_EINVAL
    assert wsl(gp, 4096, 1 << 36, 1 << 37, 1 << 38, None, None) == abi.RTM_EINVAL
    assert wsl(gp, 4096, 1 << 36, 1 << 37, 1 << 38, one_null, None) == abi.RTM_EINVAL
    assert wsl(gp, None, 1 << 36, 1 << 37, 1 << 38, slots, None) == abi.RTM_EINVAL
    assert wsl(gp, (1 << 40) + 4096 * 5, 1 << 36, 1 << 37, 1 << 38, slots, None) == abi.RTM_EALIAS   # slot in u_nxt
    assert wsl(ctypes.byref(g2), 4096, 1 << 36, 1 << 37, 1 << 38, slots, None) == abi.RTM_EINVAL
    # the tuning call: reps in 1..1000, and u_nxt is scratch, never u_prv
    assert L.rtm_tune_step(gp, 4096, 1 << 36, 1 << 37, 1 << 38, 0, None, None) == abi.RTM_EINVAL
    assert L.rtm_tune_step(gp, 4096, 1 << 36, 1 << 37, 1 << 38, 1001, None, None) == abi.RTM_EINVAL
    assert L.rtm_tune_step(gp, 1 << 37, 1 << 36, 1 << 37, 1 << 38, 3, None, None) == abi.RTM_EALIAS
    assert L.rtm_tune_step(None, 4096, 1 << 36, 1 << 37, 1 << 38, 3, None, None) == abi.RTM_EINVAL
    g3 = _grid(abi, nx=18, pitch_y=28)                                                  # nx % 4 != 0
    assert hps(ctypes.byref(g3), 4096, 1 << 36, 1 << 37, 1 << 38, slots, 1 << 39, None) == abi.RTM_EINVAL
    assert shp(ctypes.byref(g3), 1 << 36, 1 << 37, 1 << 38, None, None, None, slots, F, None) == abi.RTM_EINVAL
    assert wsl(ctypes.byref(g3), 4096, 1 << 36, 1 << 37, 1 << 38, slots, None) == abi.RTM_EINVAL
    assert L.rtm_pack_cells(gp, 4096, 64, -1, 1 << 39, None) == abi.RTM_EINVAL
    assert L.rtm_pack_cells(gp, 4096, 64, 0, 1 << 39, None) == abi.RTM_OK             # nothing to do
    assert L.rtm_pack_cells(gp, 4096, 64, 3, None, None) == abi.RTM_EINVAL
    assert L.rtm_pack_cells(gp, 4096, 64, 3, 4096 + 16, None) == abi.RTM_EALIAS
    assert L.rtm_inject(gp, 4096, 64, 64, 64, -1, None) == abi.RTM_EINVAL
    assert L.rtm_inject(gp, 4096, 64, 64, 64, 0, None) == abi.RTM_OK                # nothing to do
    assert L.rtm_record(gp, 4096, 64, 64, -5, None) == abi.RTM_EINVAL
    # injection and recording in one call
    ir = L.rtm_inject_record
    assert ir(gp, 4096, 64, 64, 64, -1, 64, 64, 1, None) == abi.RTM_EINVAL
    assert ir(gp, 4096, 64, 64, 64, 1, 64, 64, -1, None) == abi.RTM_EINVAL
    assert ir(gp, 4096, None, 64, 64, 1, 64, 64, 1, None) == abi.RTM_EINVAL
    assert ir(gp, 4096, 64, 64, 64, 1, None, 64, 1, None) == abi.RTM_EINVAL
    assert ir(gp, 4096, 64, 64, 64, 1, 64, None, 1, None) == abi.RTM_EINVAL
    assert ir(gp, None, None, None, None, 0, None, None, 0, None) == abi.RTM_OK       # nothing to do
    assert ir(None, 4096, 64, 64, 64, 1, 64, 64, 1, None) == abi.RTM_EINVAL
    assert L.rtm_record(gp, None, None, None, 0, None) == abi.RTM_OK               # nothing to do
    assert L.rtm_misfit_residual_chunks(64, 128, 256, 10, 512, 0, 1024, None) == abi.RTM_EINVAL   # no chunks
    assert L.rtm_misfit_residual_chunks(64, 128, 256, 10, None, 4, 1024, None) == abi.RTM_EINVAL  # no partials
    assert L.rtm_misfit_residual_chunks(None, None, None, 0, None, 4, None, None) == abi.RTM_OK    # nothing to do
    assert L.rtm_misfit_residual_chunks(1 << 20, 1 << 21, 1 << 22, 10, 1 << 30, 4, 1 << 30, None) == abi.RTM_EALIAS
    assert L.rtm_cnn_wgrad_partials(64, 8, 4) == 1 * 2 * 4 * (27 * 16 * 16 + 16)
    assert L.rtm_cnn_wgrad_partials(60, 8, 4) == abi.RTM_EINVAL                     # nx % 16 != 0
    need = L.rtm_cnn_wgrad_partials(64, 8, 4)
    assert L.rtm_cnn_conv3d_wgrad_ordered(64, 8, 4, 4096, 8192, 16384, 32768, 1 << 20, need - 1, None) == abi.RTM_EINVAL
    assert L.rtm_cnn_conv3d_wgrad_ordered(64, 8, 4, 4096, 8192, 16384, 32768, None, need, None) == abi.RTM_EINVAL
    assert L.rtm_cnn_conv3d_wgrad_ordered(64, 8, 4, 1 << 30, 1 << 31, 1 << 32, 1 << 33, 1 << 32, need, None) == \
        abi.RTM_EALIAS                                                               # partials over dw
    assert L.rtm_inject(gp, None, None, None, None, 0, None) == abi.RTM_OK
    assert L.rtm_image_accumulate(gp, 4096, 4096, 1 << 40, 1.0, None) == abi.RTM_EALIAS
    assert L.rtm_set_option(99, 0) == abi.RTM_EINVAL
    assert L.rtm_set_option(abi.RTM_OPT_INTERIOR_VARIANT, 7) == abi.RTM_EINVAL
    assert L.rtm_get_option(99) == abi.RTM_EINVAL
    assert L.rtm_get_option(abi.RTM_OPT_INTERIOR_VARIANT) == 2          # the 16x8 tile by default
    assert L.rtm_get_option(abi.RTM_OPT_WHOLE_VARIANT) == 6             # the tile shape chosen by radius
    assert L.rtm_set_option(abi.RTM_OPT_WHOLE_VARIANT, 3) == abi.RTM_EINVAL
    assert L.rtm_get_option(abi.RTM_OPT_ZCHUNK) == 0
    assert L.rtm_get_option(abi.RTM_OPT_HALO_VARIANT) == 0
    assert L.rtm_get_option(abi.RTM_OPT_HALO_Z_WIDTH) == 0              # z slabs of R planes
    assert L.rtm_set_option(abi.RTM_OPT_HALO_Z_WIDTH, -1) == abi.RTM_EINVAL
    assert L.rtm_get_option(abi.RTM_OPT_MARKERS) == 0
    assert L.rtm_set_option(abi.RTM_OPT_MARKERS, 2) == abi.RTM_EINVAL
    assert L.rtm_set_option(abi.RTM_OPT_MARKERS, 1) == abi.RTM_OK       # roctx is installed here
    g0 = _grid(abi)
    assert L.rtm_step_halo(ctypes.byref(g0), None, 32, 48, 64, None) == abi.RTM_EINVAL   # marked, still checked
    assert L.rtm_set_option(abi.RTM_OPT_MARKERS, 0) == abi.RTM_OK
    assert L.rtm_set_option(abi.RTM_OPT_HALO_VARIANT, 3) == abi.RTM_EINVAL   # no scalar halo variant


def test_face_layout_and_index(abi):
    g = _grid(abi, nx=16, ny=12, nz=10)
    off = abi.rtm_face_layout(g)
    R = 4
    sizes = [R * 12 * 10, R * 12 * 10, 16 * R * 10, 16 * R * 10, 16 * 12 * R, 16 * 12 * R]
    assert off == list(np.concatenate([[0], np.cumsum(sizes)]))
    assert abi.rtm_index(g, 0, 0, 0) == R * g.pitch_z + R * g.pitch_y + R
    assert abi.rtm_index(g, 3, 2, 1) - abi.rtm_index(g, 0, 0, 0) == 3 + 2 * g.pitch_y + g.pitch_z


def test_host_helpers_match_oracle(abi):
    for r in (2, 4):
        assert abs(abi.rtm_stability_limit(r) - oracle.stability_limit(r)) < 1e-15
    assert abi.rtm_stability_limit(3) == 0.0
    for n, w, a in ((64, 16, 0.015), (40, 0, 0.015), (100, 30, 0.02)):
        np.testing.assert_allclose(abi.rtm_sponge_profile(n, w, a), oracle.sponge_profile(n, w, a).astype(np.float32),
                                   rtol=0, atol=0)
    dt = 1.1321388e-3
    t = np.arange(300) * dt
    np.testing.assert_allclose(abi.rtm_ricker(300, dt, 15.0, 0.1), oracle.ricker(t, 15.0, 0.1).astype(np.float32),
                               rtol=0, atol=2e-7)


def test_stable_dt_and_injection_weights_match_oracle(abi):
    """dt and the point-source weights come from the library (the C ABI) and agree with the oracle's
    own formulas; bad arguments are RTM_EINVAL."""
    for r, h, vmax in ((4, 10.0, 2000.0), (4, 10.0, 4500.0), (2, 20.0, 3000.0)):
        dt = abi.rtm_stable_dt(r, h, vmax, 0.5)
        assert abs(dt - oracle.stable_dt(r, h, vmax)) <= 1e-15 * dt
        assert abs(abi.rtm_stable_dt(r, h, vmax, 0.99) - 0.99 * oracle.stability_limit(r) * h / vmax) <= 1e-15 * dt
    # C1: dt = 0.5 C* h / v = 1.132139 ms
    assert abs(abi.rtm_stable_dt(4, 10.0, 2000.0, 0.5) - 1.132139e-3) < 1e-9
    for bad in ((3, 10.0, 2000.0, 0.5), (4, 0.0, 2000.0, 0.5), (4, 10.0, -1.0, 0.5), (4, 10.0, 2000.0, 0.0)):
        with pytest.raises(abi.RTMError) as e:
            abi.rtm_stable_dt(*bad)
        assert e.value.status == abi.RTM_EINVAL
    v = np.array([1500.0, 2000.0, 4500.0, 3217.5])
    dt, h = 5.389e-4, 10.0
    w = abi.rtm_injection_weights(v, dt, h)
    ref = oracle.injection_weight(v, dt, h)
    assert w.dtype == np.float32
    np.testing.assert_array_equal(w, ref.astype(np.float32))
    assert len(abi.rtm_injection_weights([], dt, h)) == 0
    with pytest.raises(abi.RTMError):
        abi.rtm_injection_weights(v, -dt, h)


def test_injection_mask():
    """The corrector's weight: 0 at and near injection cells and in the sponge, 1 in the clear
    interior, a linear ramp between."""
    from types import SimpleNamespace

    from paper_1603_03971_amd.learned import injection_mask

    g = SimpleNamespace(shape=(20, 24, 32), sponge_width=2)
    m = injection_mask(g, [(16, 12, 10)], r0=2.0, width=3.0)
    assert m.dtype == np.float32 and m.shape == (20, 24, 32)
    assert m[10, 12, 16] == 0.0 and m[10, 12, 18] == 0.0          # within r0
    assert abs(m[10, 12, 19] - 1.0 / 3.0) < 1e-6                   # distance 3: one third up the ramp
    assert m[10, 12, 24] == 1.0                                    # clear of source and sponge
    assert (m[:, :, 0] == 0).all() and (m[:, :, 1] == 0).all()     # sponge cells
    assert abs(m[10, 12, 2] - 1.0 / 3.0) < 1e-6                    # first cell past the sponge
    plane = np.stack(np.meshgrid(np.arange(32), np.arange(24), indexing="xy"), -1).reshape(-1, 2)
    rec = np.concatenate([plane, np.full((len(plane), 1), 6)], axis=1)
    mp = injection_mask(g, rec)
    assert (mp[6] == 0).all() and (mp[8] == 0).all() and mp[14, 12, 16] == 1.0


def test_corrector_fallback_rule():
    """learned.applicable: the corrected coarse grid stands in for the fine one only inside the
    corrector's validity record."""
    from types import SimpleNamespace

    from paper_1603_03971_amd.learned import CorrectorSpec, applicable

    from dataclasses import replace

    spec = CorrectorSpec(h=10.0, dt=7.5e-4, vmin=1500.0, vmax=3000.0, fp_low=6.0, fp_high=16.0, every=16,
                         relu=False, image_error=0.008)
    fine = SimpleNamespace(h=10.0, dt=7.5e-4, radius=4, nx=96, ny=64, nz=70)
    v = np.full((70, 64, 96), 2000.0)
    assert applicable(spec, fine, v, 15.0) == (True, "ok")
    # the fine grid judges the corrector: no measured error, or one above the bar, means the fine grid
    ok, why = applicable(replace(spec, image_error=float("nan")), fine, v, 15.0)
    assert not ok and "never measured" in why
    ok, why = applicable(replace(spec, image_error=0.21), fine, v, 15.0)
    assert not ok and "above the bar" in why
    assert applicable(replace(spec, image_error=0.21, error_bar=0.25), fine, v, 15.0)[0]
    assert not applicable(None, fine, v, 15.0)[0]
    assert not applicable(spec, fine, v, 20.0)[0]                                   # frequency
    assert not applicable(spec, fine, np.full_like(v, 4000.0), 15.0)[0]             # velocity
    assert not applicable(spec, SimpleNamespace(**{**vars(fine), "dt": 5e-4}), v, 15.0)[0]
    assert not applicable(spec, SimpleNamespace(**{**vars(fine), "nx": 80}), v, 15.0)[0]   # 40 % 16
    assert not applicable(spec, SimpleNamespace(**{**vars(fine), "radius": 2}), v, 15.0)[0]


def test_time_at_error_reads_the_plain_frontier():
    """The plain solvers' time at a given image error: the lower-left frontier of (time, error)
    points, interpolated in log error; dominated points do not count."""
    from paper_1603_03971_amd.learned import time_at_error

    pts = [(3.2, 0.0), (0.25, 0.29), (0.26, 0.12), (0.30, 0.2), (0.5, 0.05), (0.9, 0.02)]
    assert time_at_error(pts, 0.5) == 0.25            # above every error: the fastest solver
    assert time_at_error(pts, 0.12) == 0.26
    t = time_at_error(pts, 0.2)                       # between 0.29 and 0.12 on the frontier
    w = (np.log(0.29) - np.log(0.2)) / (np.log(0.29) - np.log(0.12))
    assert abs(t - (0.25 + w * 0.01)) < 1e-12
    assert time_at_error(pts, 0.01) == 3.2            # only the fine solve reaches it
    assert time_at_error([(0.2, 0.3), (0.4, 0.1)], 0.05) is None


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and says so, before touching a device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""

