"""ctypes binding of librtm.so: the same names and arguments as include/rtm.h.

Argument marshalling only.  Field arguments accept a torch tensor (its data_ptr is passed), a raw
integer device address, or None (NULL).  Streams accept a torch.cuda.Stream, a raw hipStream_t
integer, or None (the null stream).  A nonzero status raises RTMError.  If the library has not been
built, importing the binding fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtm.so")

RTM_OK, RTM_EINVAL, RTM_EALIAS, RTM_ELAUNCH, RTM_EDEVICE = 0, -1, -2, -3, -4
RTM_SNAP_BF16, RTM_SNAP_F16 = 1, 2
RTM_RESTRICT_INJECT, RTM_RESTRICT_FULL = 0, 1
RTM_OPT_INTERIOR_VARIANT, RTM_OPT_ZCHUNK, RTM_OPT_XCD_REMAP, RTM_OPT_HALO_X_WIDTH, RTM_OPT_HALO_Y_WIDTH = 1, 2, 3, 4, 5
RTM_OPT_HALO_VARIANT, RTM_OPT_WHOLE_VARIANT, RTM_OPT_UNPACK_LINES, RTM_OPT_TILE_FLAGS = 6, 7, 8, 9
RTM_OPT_HALO_Z_WIDTH, RTM_OPT_MARKERS = 10, 11


class RTMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib.rtm_strerror(status).decode()} (status {status})")


class rtm_grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("radius", ctypes.c_int32),
        ("pitch_y", ctypes.c_int64), ("pitch_z", ctypes.c_int64),
        ("c", ctypes.c_float * 5),
        ("gx", ctypes.c_void_p), ("gy", ctypes.c_void_p), ("gz", ctypes.c_void_p),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_1603_03971_amd/build.py` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    gp = ctypes.POINTER(rtm_grid)
    sig = {
        "rtm_abi_version": ([], ctypes.c_int),
        "rtm_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "rtm_grid_init": ([gp, i32, i32, i32, i32, i64, i64, vp, vp, vp], ctypes.c_int),
        "rtm_stability_limit": ([i32], f64),
        "rtm_stable_dt": ([i32, f64, f64, f64, ctypes.POINTER(f64)], ctypes.c_int),
        "rtm_injection_weights": ([i32, vp, f64, f64, vp], ctypes.c_int),
        "rtm_sponge_profile": ([i32, i32, f64, vp], ctypes.c_int),
        "rtm_ricker": ([i32, f64, f64, f64, vp], ctypes.c_int),
        "rtm_face_layout": ([gp, ctypes.POINTER(i64)], ctypes.c_int),
        "rtm_index": ([gp, i32, i32, i32], i64),
        "rtm_set_option": ([i32, i32], ctypes.c_int),
        "rtm_get_option": ([i32], ctypes.c_int),
        "rtm_halo_region": ([gp, ctypes.POINTER(i32)], ctypes.c_int),
        "rtm_step_halo": ([gp, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_step_interior": ([gp, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_step_whole": ([gp, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_tune_step": ([gp, vp, vp, vp, vp, i32, ctypes.POINTER(i32), vp], ctypes.c_int),
        "rtm_pack_halo": ([gp, vp, vp, vp], ctypes.c_int),
        "rtm_step_halo_pack": ([gp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_step_halo_pack_slots": ([gp, vp, vp, vp, vp, ctypes.POINTER(vp), vp, vp], ctypes.c_int),
        "rtm_inject_record": ([gp, vp, vp, vp, vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp], ctypes.c_int),
        "rtm_step_shell_pack": ([gp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp), vp, vp], ctypes.c_int),
        "rtm_step_whole_slots": ([gp, vp, vp, vp, vp, ctypes.POINTER(vp), vp], ctypes.c_int),
        "rtm_pack_cells": ([gp, vp, vp, i32, vp, vp], ctypes.c_int),
        "rtm_unpack_halo": ([gp, vp, ctypes.POINTER(vp), vp], ctypes.c_int),
        "rtm_inject": ([gp, vp, vp, vp, vp, i32, vp], ctypes.c_int),
        "rtm_record": ([gp, vp, vp, vp, i32, vp], ctypes.c_int),
        "rtm_kappa_from_velocity": ([gp, vp, vp, f32, vp], ctypes.c_int),
        "rtm_image_accumulate": ([gp, vp, vp, vp, f32, vp], ctypes.c_int),
        "rtm_count_nonfinite": ([gp, vp, vp, vp], ctypes.c_int),
        "rtm_snapshot_encode": ([gp, vp, vp, vp, i32, vp], ctypes.c_int),
        "rtm_adjoint_step": ([gp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_gradient_accumulate": ([gp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_gradient_accumulate_scaled": ([gp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_scaled_adjoint_factors": ([gp, vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "rtm_record_weighted": ([gp, vp, vp, vp, vp, i32, vp], ctypes.c_int),
        "rtm_velocity_gradient_scaled": ([gp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_misfit_residual": ([vp, vp, vp, i64, vp, vp], ctypes.c_int),
        "rtm_misfit_residual_chunks": ([vp, vp, vp, i64, vp, i32, vp, vp], ctypes.c_int),
        "rtm_misfit_residual_chunks_noalloc": ([vp, vp, vp, i64, i32, vp, vp], ctypes.c_int),
        "rtm_velocity_gradient": ([gp, vp, vp, vp, f32, vp], ctypes.c_int),
        "rtm_image_accumulate_coded": ([gp, vp, vp, vp, i32, vp, f32, vp], ctypes.c_int),
        "rtm_cnn_conv3d": ([i32, i32, i32, vp, vp, vp, i32, vp, i32, vp, vp], ctypes.c_int),
        "rtm_cnn_conv3d_wgrad": ([i32, i32, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_cnn_conv3d_wgrad_ordered": ([i32, i32, i32, vp, vp, vp, vp, vp, i64, vp], ctypes.c_int),
        "rtm_cnn_wgrad_partials": ([i32, i32, i32], i64),
        "rtm_cnn_relu_backward": ([i32, i32, i32, vp, vp, i32, i32, vp, vp, vp], ctypes.c_int),
        "rtm_cnn_loss_grad": ([i32, i32, i32, vp, vp, i32, f32, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_cnn_weight_flip": ([vp, vp, vp], ctypes.c_int),
        "rtm_cnn_adam": ([vp, vp, vp, vp, i32, f32, f32, f32, f32, i32, vp, vp], ctypes.c_int),
        "rtm_cnn_to_bf16": ([vp, vp, i32, vp], ctypes.c_int),
        "rtm_cnn_pack_input": ([gp, vp, vp, vp, f32, f32, vp, vp, vp, vp], ctypes.c_int),
        "rtm_cnn_apply_correction": ([gp, vp, vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "rtm_cnn_conv3d_first": ([gp, vp, vp, vp, f32, f32, vp, vp, vp, i32, vp, vp], ctypes.c_int),
        "rtm_cnn_conv3d_apply": ([gp, vp, vp, vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_cnn_target": ([gp, vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "rtm_restrict": ([gp, gp, vp, vp, i32, vp], ctypes.c_int),
        "rtm_prolong": ([gp, gp, vp, vp, vp], ctypes.c_int),
        "rtm_field_absmax": ([gp, vp, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
lib = _lib


def _p(x) -> int | None:
    """Device address of a tensor / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _s(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status: int, where: str):
    if status != RTM_OK:
        raise RTMError(status, where)


def rtm_abi_version() -> int:
    return _lib.rtm_abi_version()


def rtm_strerror(status: int) -> str:
    return _lib.rtm_strerror(status).decode()


def rtm_grid_init(nx, ny, nz, radius, pitch_y, pitch_z, gx, gy, gz) -> rtm_grid:
    g = rtm_grid()
    _check(_lib.rtm_grid_init(ctypes.byref(g), nx, ny, nz, radius, pitch_y, pitch_z, _p(gx), _p(gy), _p(gz)),
           "rtm_grid_init")
    return g


def rtm_stability_limit(radius: int) -> float:
    return _lib.rtm_stability_limit(radius)


def rtm_stable_dt(radius: int, h: float, vmax: float, fraction: float = 0.5) -> float:
    dt = ctypes.c_double()
    _check(_lib.rtm_stable_dt(radius, h, vmax, fraction, ctypes.byref(dt)), "rtm_stable_dt")
    return dt.value


def rtm_injection_weights(v, dt: float, h: float):
    import numpy as np

    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
    out = np.empty(len(v), dtype=np.float32)
    _check(_lib.rtm_injection_weights(len(v), v.ctypes.data if len(v) else None, dt, h,
                                      out.ctypes.data if len(v) else None), "rtm_injection_weights")
    return out


def rtm_sponge_profile(n: int, width: int, alpha: float):
    import numpy as np

    out = np.empty(n, dtype=np.float32)
    _check(_lib.rtm_sponge_profile(n, width, alpha, out.ctypes.data), "rtm_sponge_profile")
    return out


def rtm_ricker(nsteps: int, dt: float, fpeak: float, t0: float):
    import numpy as np

    out = np.empty(nsteps, dtype=np.float32)
    _check(_lib.rtm_ricker(nsteps, dt, fpeak, t0, out.ctypes.data), "rtm_ricker")
    return out


def rtm_face_layout(grid: rtm_grid):
    off = (ctypes.c_int64 * 7)()
    _check(_lib.rtm_face_layout(ctypes.byref(grid), off), "rtm_face_layout")
    return list(off)


def rtm_index(grid: rtm_grid, i: int, j: int, k: int) -> int:
    return _lib.rtm_index(ctypes.byref(grid), i, j, k)


def rtm_set_option(option: int, value: int):
    _check(_lib.rtm_set_option(option, value), "rtm_set_option")


def rtm_get_option(option: int) -> int:
    v = _lib.rtm_get_option(option)
    if v < 0:
        raise RTMError(v, "rtm_get_option")
    return v


def rtm_halo_region(grid):
    """(wx, hy, R): widths of the halo region's x strips, y strips and z slabs."""
    w = (ctypes.c_int32 * 3)()
    _check(_lib.rtm_halo_region(ctypes.byref(grid), w), "rtm_halo_region")
    return tuple(w)


def rtm_step_halo(grid, u_nxt, u_cur, u_prv, kappa, stream=None):
    _check(_lib.rtm_step_halo(ctypes.byref(grid), _p(u_nxt), _p(u_cur), _p(u_prv), _p(kappa), _s(stream)),
           "rtm_step_halo")


def rtm_step_interior(grid, u_nxt, u_cur, u_prv, kappa, stream=None):
    _check(_lib.rtm_step_interior(ctypes.byref(grid), _p(u_nxt), _p(u_cur), _p(u_prv), _p(kappa), _s(stream)),
           "rtm_step_interior")


def rtm_step_whole(grid, u_nxt, u_cur, u_prv, kappa, stream=None):
    _check(_lib.rtm_step_whole(ctypes.byref(grid), _p(u_nxt), _p(u_cur), _p(u_prv), _p(kappa), _s(stream)),
           "rtm_step_whole")


def rtm_tune_step(grid, u_nxt, u_cur, u_prv, kappa, reps=3, stream=None):
    """Tune the one-launch call for this grid shape (waits for the device); returns the chosen
    (tile variant, workgroup order), or (-1, -1) when there is nothing to tune."""
    choice = (ctypes.c_int32 * 2)()
    _check(_lib.rtm_tune_step(ctypes.byref(grid), _p(u_nxt), _p(u_cur), _p(u_prv), _p(kappa), int(reps), choice,
                              _s(stream)), "rtm_tune_step")
    return int(choice[0]), int(choice[1])


def rtm_pack_halo(grid, u, faces, stream=None):
    _check(_lib.rtm_pack_halo(ctypes.byref(grid), _p(u), _p(faces), _s(stream)), "rtm_pack_halo")


def rtm_step_halo_pack(grid, u_nxt, u_cur, u_prv, kappa, faces, stream=None):
    _check(_lib.rtm_step_halo_pack(ctypes.byref(grid), _p(u_nxt), _p(u_cur), _p(u_prv), _p(kappa), _p(faces),
                                   _s(stream)), "rtm_step_halo_pack")


def rtm_step_halo_pack_slots(grid, u_nxt, u_cur, u_prv, kappa, recv, faces, stream=None):
    """`recv`: six receive-slot addresses (tensor or int) holding u_cur's ghost faces."""
    arr = (ctypes.c_void_p * 6)(*[_p(f) for f in recv])
    _check(_lib.rtm_step_halo_pack_slots(ctypes.byref(grid), _p(u_nxt), _p(u_cur), _p(u_prv), _p(kappa), arr,
                                         _p(faces), _s(stream)), "rtm_step_halo_pack_slots")


def rtm_inject_record(grid, u, src_idx, w, amp, nsrc, rec_idx, out, nrec, stream=None):
    _check(_lib.rtm_inject_record(ctypes.byref(grid), _p(u), _p(src_idx), _p(w), _p(amp), int(nsrc), _p(rec_idx),
                                  _p(out), int(nrec), _s(stream)), "rtm_inject_record")


def rtm_step_shell_pack(grid, u_cur, u_prv, kappa, recv, faces, stream=None, dense=None):
    """`recv`: six receive-slot addresses (tensor or int) holding u_cur's ghost faces.  `dense`: None or
    the face buffers (faces_cur, faces_prv, faces_kappa) of u_cur, u_prv and kappa."""
    arr = (ctypes.c_void_p * 6)(*[_p(f) for f in recv])
    fc, fp, fk = dense if dense is not None else (None, None, None)
    _check(_lib.rtm_step_shell_pack(ctypes.byref(grid), _p(u_cur), _p(u_prv), _p(kappa), _p(fc), _p(fp), _p(fk),
                                    arr, _p(faces), _s(stream)), "rtm_step_shell_pack")


def rtm_step_whole_slots(grid, u_nxt, u_cur, u_prv, kappa, recv, stream=None):
    """`recv`: six receive-slot addresses (tensor or int) holding u_cur's ghost faces."""
    arr = (ctypes.c_void_p * 6)(*[_p(f) for f in recv])
    _check(_lib.rtm_step_whole_slots(ctypes.byref(grid), _p(u_nxt), _p(u_cur), _p(u_prv), _p(kappa), arr,
                                     _s(stream)), "rtm_step_whole_slots")


def rtm_pack_cells(grid, u, idx, n, faces, stream=None):
    _check(_lib.rtm_pack_cells(ctypes.byref(grid), _p(u), _p(idx), int(n), _p(faces), _s(stream)),
           "rtm_pack_cells")


def rtm_unpack_halo(grid, u, faces, stream=None):
    """`faces`: six slot addresses (tensor, int or None for a zero/physical boundary)."""
    arr = (ctypes.c_void_p * 6)(*[_p(f) for f in faces])
    _check(_lib.rtm_unpack_halo(ctypes.byref(grid), _p(u), arr, _s(stream)), "rtm_unpack_halo")


def rtm_inject(grid, u, idx, w, amp, n, stream=None):
    _check(_lib.rtm_inject(ctypes.byref(grid), _p(u), _p(idx), _p(w), _p(amp), n, _s(stream)), "rtm_inject")


def rtm_record(grid, u, idx, out, n, stream=None):
    _check(_lib.rtm_record(ctypes.byref(grid), _p(u), _p(idx), _p(out), n, _s(stream)), "rtm_record")


def rtm_kappa_from_velocity(grid, kappa, v, dt_over_h, stream=None):
    _check(_lib.rtm_kappa_from_velocity(ctypes.byref(grid), _p(kappa), _p(v), dt_over_h, _s(stream)),
           "rtm_kappa_from_velocity")


def rtm_image_accumulate(grid, image, src, rcv, weight=1.0, stream=None):
    _check(_lib.rtm_image_accumulate(ctypes.byref(grid), _p(image), _p(src), _p(rcv), weight, _s(stream)),
           "rtm_image_accumulate")


def rtm_count_nonfinite(grid, u, count, stream=None):
    _check(_lib.rtm_count_nonfinite(ctypes.byref(grid), _p(u), _p(count), _s(stream)), "rtm_count_nonfinite")


def rtm_snapshot_encode(grid, u, codes, scales, fmt, stream=None):
    _check(_lib.rtm_snapshot_encode(ctypes.byref(grid), _p(u), _p(codes), _p(scales), fmt, _s(stream)),
           "rtm_snapshot_encode")


def rtm_image_accumulate_coded(grid, image, codes, scales, fmt, rcv, weight=1.0, stream=None):
    _check(_lib.rtm_image_accumulate_coded(ctypes.byref(grid), _p(image), _p(codes), _p(scales), fmt, _p(rcv),
                                           weight, _s(stream)), "rtm_image_accumulate_coded")


def rtm_adjoint_step(grid, mu_out, mu_a, mu_b, kappa, work, stream=None):
    _check(_lib.rtm_adjoint_step(ctypes.byref(grid), _p(mu_out), _p(mu_a), _p(mu_b), _p(kappa), _p(work), _s(stream)),
           "rtm_adjoint_step")


def rtm_gradient_accumulate(grid, grad, u, mu, stream=None):
    _check(_lib.rtm_gradient_accumulate(ctypes.byref(grid), _p(grad), _p(u), _p(mu), _s(stream)),
           "rtm_gradient_accumulate")


def rtm_misfit_residual(d, obs, resid, n, misfit, stream=None):
    _check(_lib.rtm_misfit_residual(_p(d), _p(obs), _p(resid), n, _p(misfit), _s(stream)), "rtm_misfit_residual")


def rtm_misfit_residual_chunks(d, obs, resid, n, partials, nchunks, misfit, stream=None):
    _check(_lib.rtm_misfit_residual_chunks(_p(d), _p(obs), _p(resid), n, _p(partials), nchunks, _p(misfit),
                                           _s(stream)), "rtm_misfit_residual_chunks")


def rtm_misfit_residual_chunks_noalloc(d, obs, resid, n, nchunks, misfit, stream=None):
    _check(_lib.rtm_misfit_residual_chunks_noalloc(_p(d), _p(obs), _p(resid), n, nchunks, _p(misfit), _s(stream)),
           "rtm_misfit_residual_chunks_noalloc")


def rtm_gradient_accumulate_scaled(grid, grad, u, w, stream=None):
    _check(_lib.rtm_gradient_accumulate_scaled(ctypes.byref(grid), _p(grad), _p(u), _p(w), _s(stream)),
           "rtm_gradient_accumulate_scaled")


def rtm_scaled_adjoint_factors(grid, kappa, idx, n, kg, inv_kg, stream=None):
    _check(_lib.rtm_scaled_adjoint_factors(ctypes.byref(grid), _p(kappa), _p(idx), n, _p(kg), _p(inv_kg),
                                           _s(stream)), "rtm_scaled_adjoint_factors")


def rtm_record_weighted(grid, u, idx, w, out, n, stream=None):
    _check(_lib.rtm_record_weighted(ctypes.byref(grid), _p(u), _p(idx), _p(w), _p(out), n, _s(stream)),
           "rtm_record_weighted")


def rtm_velocity_gradient_scaled(grid, grad_v, G, v, stream=None):
    _check(_lib.rtm_velocity_gradient_scaled(ctypes.byref(grid), _p(grad_v), _p(G), _p(v), _s(stream)),
           "rtm_velocity_gradient_scaled")


def rtm_velocity_gradient(grid, grad_v, grad_kappa, v, dt_over_h, stream=None):
    _check(_lib.rtm_velocity_gradient(ctypes.byref(grid), _p(grad_v), _p(grad_kappa), _p(v), dt_over_h, _s(stream)),
           "rtm_velocity_gradient")


def rtm_cnn_conv3d(nx, ny, nz, x, w, bias, relu, y32, y16, stream=None, y32_channels=16):
    _check(_lib.rtm_cnn_conv3d(nx, ny, nz, _p(x), _p(w), _p(bias), int(relu), _p(y32), y32_channels, _p(y16),
                               _s(stream)), "rtm_cnn_conv3d")


def rtm_cnn_conv3d_wgrad(nx, ny, nz, x, dz, dw, db, stream=None):
    _check(_lib.rtm_cnn_conv3d_wgrad(nx, ny, nz, _p(x), _p(dz), _p(dw), _p(db), _s(stream)), "rtm_cnn_conv3d_wgrad")


def rtm_cnn_wgrad_partials(nx, ny, nz) -> int:
    n = int(_lib.rtm_cnn_wgrad_partials(nx, ny, nz))
    if n < 0:
        raise RTMError(n, "rtm_cnn_wgrad_partials")
    return n


def rtm_cnn_conv3d_wgrad_ordered(nx, ny, nz, x, dz, dw, db, partials, partials_len, stream=None):
    _check(_lib.rtm_cnn_conv3d_wgrad_ordered(nx, ny, nz, _p(x), _p(dz), _p(dw), _p(db), _p(partials), partials_len,
                                             _s(stream)), "rtm_cnn_conv3d_wgrad_ordered")


def rtm_cnn_relu_backward(nx, ny, nz, y, dy, relu, channels, dz32, dz16, stream=None):
    _check(_lib.rtm_cnn_relu_backward(nx, ny, nz, _p(y), _p(dy), int(relu), channels, _p(dz32), _p(dz16), _s(stream)),
           "rtm_cnn_relu_backward")


def rtm_cnn_loss_grad(nx, ny, nz, out, target, channels, dz32, dz16, loss=None, stream=None, weight=1.0, mask=None):
    _check(_lib.rtm_cnn_loss_grad(nx, ny, nz, _p(out), _p(target), channels, weight, _p(mask), _p(dz32), _p(dz16),
                                  _p(loss), _s(stream)), "rtm_cnn_loss_grad")


def rtm_cnn_weight_flip(w, wt, stream=None):
    _check(_lib.rtm_cnn_weight_flip(_p(w), _p(wt), _s(stream)), "rtm_cnn_weight_flip")


def rtm_cnn_adam(param, grad, m1, m2, n, lr, beta1, beta2, eps, step, param_bf16=None, stream=None):
    _check(_lib.rtm_cnn_adam(_p(param), _p(grad), _p(m1), _p(m2), n, lr, beta1, beta2, eps, step, _p(param_bf16),
                             _s(stream)), "rtm_cnn_adam")


def rtm_cnn_to_bf16(a, b, n, stream=None):
    _check(_lib.rtm_cnn_to_bf16(_p(a), _p(b), n, _s(stream)), "rtm_cnn_to_bf16")


def rtm_cnn_pack_input(grid, u_cur, u_prv, velocity, v_ref, v_scale, scale, x, noise=None, stream=None):
    _check(_lib.rtm_cnn_pack_input(ctypes.byref(grid), _p(u_cur), _p(u_prv), _p(velocity), v_ref, v_scale, _p(scale),
                                   _p(noise), _p(x), _s(stream)), "rtm_cnn_pack_input")


def rtm_cnn_apply_correction(grid, u_cur, u_prv, out, scale, stream=None, out_channels=16, mask=None):
    _check(_lib.rtm_cnn_apply_correction(ctypes.byref(grid), _p(u_cur), _p(u_prv), _p(out), out_channels, _p(mask),
                                         _p(scale), _s(stream)), "rtm_cnn_apply_correction")


def rtm_cnn_conv3d_first(grid, u_cur, u_prv, velocity, v_ref, v_scale, scale, w, bias, relu, y16, stream=None):
    _check(_lib.rtm_cnn_conv3d_first(ctypes.byref(grid), _p(u_cur), _p(u_prv), _p(velocity), v_ref, v_scale,
                                     _p(scale), _p(w), _p(bias), int(relu), _p(y16), _s(stream)),
           "rtm_cnn_conv3d_first")


def rtm_cnn_conv3d_apply(grid, x, w, bias, relu, u_cur, u_prv, scale, mask=None, stream=None):
    _check(_lib.rtm_cnn_conv3d_apply(ctypes.byref(grid), _p(x), _p(w), _p(bias), int(relu), _p(u_cur), _p(u_prv),
                                     _p(mask), _p(scale), _s(stream)), "rtm_cnn_conv3d_apply")


def rtm_cnn_target(grid, ref_cur, ref_prv, u_cur, u_prv, scale, target, noise=None, stream=None):
    _check(_lib.rtm_cnn_target(ctypes.byref(grid), _p(ref_cur), _p(ref_prv), _p(u_cur), _p(u_prv), _p(scale),
                               _p(noise), _p(target), _s(stream)), "rtm_cnn_target")


def rtm_restrict(fine, coarse, u_fine, u_coarse, stream=None, mode=None):
    mode = RTM_RESTRICT_INJECT if mode is None else mode
    _check(_lib.rtm_restrict(ctypes.byref(fine), ctypes.byref(coarse), _p(u_fine), _p(u_coarse), mode, _s(stream)),
           "rtm_restrict")


def rtm_prolong(coarse, fine, u_coarse, u_fine, stream=None):
    _check(_lib.rtm_prolong(ctypes.byref(coarse), ctypes.byref(fine), _p(u_coarse), _p(u_fine), _s(stream)),
           "rtm_prolong")


def rtm_field_absmax(grid, u, out, stream=None):
    _check(_lib.rtm_field_absmax(ctypes.byref(grid), _p(u), _p(out), _s(stream)), "rtm_field_absmax")
