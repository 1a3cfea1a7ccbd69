"""ctypes binding of libges.so (include/ges.h).

Argument marshalling only: every function here converts torch tensors to device
pointers and calls the C entry point of the same name; all arithmetic runs in the
HIP kernels.  The library must have been built (``paper_2402_10128_amd.build``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libges.so")

GES_OK = 0
GRAD2D_STRIDE = 12   # GES_GRAD2D_STRIDE: binary64 slots per splat in the 2-D gradient rows
STATUS_NAMES = {0: "OK", 1: "INVALID_ARGUMENT", 2: "CAPACITY", 3: "OUT_OF_MEMORY", 4: "DEVICE", 5: "BUSY",
                6: "NOT_FOUND", 7: "INTERNAL"}
FALLOFF_PHI, FALLOFF_GEF, FALLOFF_PHI_EXACT = 0, 1, 2
TILES_SQUARE, TILES_ELLIPSE = 0, 1
TILE = 16


class GESError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ges_splats(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("beta", C.c_void_p)]


class ges_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("near_z", C.c_float)]


class ges_raster_params(C.Structure):
    _fields_ = [("falloff", C.c_int32), ("tile_cull", C.c_int32), ("rho", C.c_float), ("bg", C.c_float * 3),
                ("flags", C.c_uint32)]


class ges_splat_grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta")]


class ges_frame_view(C.Structure):
    _fields_ = [("records", C.c_void_p), ("tile_ranges", C.c_void_p), ("sorted_pairs", C.c_void_p),
                ("sorted_tiles", C.c_void_p), ("final_T", C.c_void_p), ("n_contrib", C.c_void_p),
                ("grad2d", C.c_void_p), ("stats", C.c_void_p), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("tile_work", C.c_void_p), ("group_order", C.c_void_p), ("row_marks", C.c_void_p)]


class ges_serve_config(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("queue_capacity", C.c_int32), ("falloff", C.c_int32),
                ("tile_cull", C.c_int32), ("rho", C.c_float), ("bg", C.c_float * 3), ("sequential", C.c_int32)]


class ges_adam_group(C.Structure):
    _fields_ = [("params", C.c_void_p), ("grads", C.c_void_p), ("exp_avg", C.c_void_p), ("exp_avg_sq", C.c_void_p),
                ("count", C.c_int64), ("lr", C.c_float)]


class ges_adam_splats(C.Structure):
    _fields_ = [("exp_avg", C.c_void_p * 6), ("exp_avg_sq", C.c_void_p * 6), ("lr", C.c_float * 6),
                ("step", C.c_int64), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("grad_accum", C.c_void_p), ("grad_count", C.c_void_p), ("grads_in", C.c_void_p * 6)]


class ges_splat_set(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("beta", C.c_void_p)]


class ges_mix_problem(C.Structure):
    _fields_ = [("model", C.c_int32), ("n", C.c_int32), ("positive", C.c_int32), ("target", C.c_int32)]


class ges_request_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("t_submit_ns", C.c_uint64), ("t_start_ns", C.c_uint64),
                ("t_done_ns", C.c_uint64), ("num_keys", C.c_uint64), ("batch_size", C.c_int32)]


# exported entry points and their argument types
_SIGS = {
    "ges_abi_version": (C.c_uint32, []),
    "ges_last_error": (C.c_char_p, []),
    "ges_workspace_query": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "ges_key_workspace_query": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "ges_preprocess": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.POINTER(ges_raster_params),
                                 C.c_void_p, C.c_size_t, C.POINTER(C.c_uint64), C.c_void_p]),
    "ges_render_forward": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.POINTER(ges_raster_params),
                                     C.c_void_p, C.c_void_p, C.c_size_t, C.c_uint64, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "ges_render_backward": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.POINTER(ges_raster_params),
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(ges_splat_grads),
                                      C.c_void_p]),
    "ges_frame_view_get": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64,
                                     C.c_void_p, C.POINTER(ges_frame_view)]),
    "ges_views_workspace_query": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t),
                                            C.POINTER(C.c_size_t)]),
    "ges_preprocess_views": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.c_int32,
                                       C.POINTER(ges_raster_params), C.c_void_p, C.c_size_t, C.POINTER(C.c_uint64),
                                       C.c_void_p]),
    "ges_render_forward_views": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.c_int32,
                                           C.POINTER(ges_raster_params), C.c_void_p, C.c_void_p, C.c_size_t,
                                           C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ges_render_backward_views": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.c_int32,
                                            C.POINTER(ges_raster_params), C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.POINTER(ges_splat_grads), C.c_int32, C.c_void_p,
                                            C.c_void_p, C.c_void_p]),
    "ges_render_backward_views_adam": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.c_int32,
                                                 C.POINTER(ges_raster_params), C.c_void_p, C.c_void_p, C.c_void_p,
                                                 C.c_void_p, C.POINTER(ges_splat_grads), C.POINTER(ges_adam_splats),
                                                 C.c_void_p]),
    "ges_frame_view_get_views": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.c_uint64, C.c_void_p, C.c_int32, C.POINTER(ges_frame_view)]),
    "ges_profile_enable": (C.c_int, [C.c_int32]),
    "ges_profile_select": (C.c_int, [C.c_uint32]),
    "ges_profile_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]),
    "ges_mask_scratch_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "ges_freq_mask": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ges_loss_scratch_bytes": (C.c_size_t, []),
    "ges_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_float, C.c_float,
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ges_ssim_scratch_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "ges_ssim_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_float, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p]),
    "ges_render_backward_adam": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera), C.POINTER(ges_raster_params),
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.POINTER(ges_splat_grads), C.POINTER(ges_adam_splats), C.c_void_p]),
    "ges_prune_scratch_bytes": (C.c_size_t, [C.c_int64]),
    "ges_prune_splats": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(ges_splat_set), C.POINTER(ges_splat_set), C.c_int32,
                                   C.c_double, C.c_double, C.c_void_p, C.c_size_t, C.POINTER(C.c_int64), C.c_void_p]),
    "ges_shape_reset": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p]),
    "ges_mix_fit": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_float, C.c_float,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_float,
                              C.c_float, C.c_float, C.c_void_p]),
    "ges_render_backward_accumulate": (C.c_int, [C.POINTER(ges_splats), C.POINTER(ges_camera),
                                                 C.POINTER(ges_raster_params), C.c_void_p, C.c_void_p, C.c_void_p,
                                                 C.c_void_p, C.POINTER(ges_splat_grads), C.c_void_p, C.c_void_p,
                                                 C.c_void_p]),
    "ges_densify_scratch_bytes": (C.c_size_t, [C.c_int64]),
    "ges_densify": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(ges_splat_set), C.POINTER(ges_splat_set), C.c_int32,
                              C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                              C.c_size_t, C.POINTER(C.c_int64), C.c_void_p]),
    "ges_opacity_reset": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_void_p]),
    "ges_adam_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "ges_expon_lr": (C.c_double, [C.c_int64, C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_double]),
    "ges_loss_schedule": (C.c_int, [C.c_int64, C.c_int64, C.c_float, C.c_float, C.POINTER(C.c_float),
                                    C.POINTER(C.c_float)]),
    "ges_serve_create": (C.c_int, [C.POINTER(ges_serve_config), C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "ges_serve_create_simulated": (C.c_int, [C.POINTER(ges_serve_config), C.c_size_t, C.c_uint64, C.c_uint64,
                                             C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
    "ges_serve_add_scene": (C.c_int, [C.c_void_p, C.POINTER(ges_splats), C.POINTER(C.c_int32)]),
    "ges_serve_submit": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(ges_camera), C.c_void_p, C.POINTER(C.c_uint64)]),
    "ges_serve_submit_inspect": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(ges_camera), C.c_void_p, C.c_void_p,
                                           C.c_size_t, C.POINTER(C.c_uint64)]),
    "ges_serve_inspect_bytes": (C.c_size_t, [C.c_int64, C.c_int32, C.c_int32, C.c_uint64]),
    "ges_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(ges_request_info)]),
    "ges_serve_drain": (C.c_int, [C.c_void_p]),
    "ges_serve_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def lib():
    """Load libges.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2402_10128_amd.build.build()")
        _lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(_lib, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
    return _lib


def _check(status):
    if status != GES_OK:
        raise GESError(status, lib().ges_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def camera_struct(cam) -> ges_camera:
    c = ges_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).ravel()]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).ravel()]
    c.fx, c.fy, c.cx, c.cy, c.near_z = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy, cam.near))
    return c


RASTER_KEEP_GRAD2D = 1


def params_struct(falloff=FALLOFF_PHI, tile_cull=TILES_SQUARE, rho=0.1, bg=(0.0, 0.0, 0.0), flags=0) -> ges_raster_params:
    p = ges_raster_params()
    p.falloff, p.tile_cull, p.rho = int(falloff), int(tile_cull), float(rho)
    p.bg[:] = [float(b) for b in bg]
    p.flags = int(flags)
    return p


def splats_struct(means, log_scales, quats, opacity_logits, sh, beta) -> ges_splats:
    s = ges_splats()
    s.n = int(means.shape[0])
    k = int(sh.shape[1]) if sh.dim() == 3 else 1
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[k]
    s.sh_degree = deg
    for name, t in (("means", means), ("log_scales", log_scales), ("quats", quats),
                    ("opacity_logits", opacity_logits), ("sh", sh), ("beta", beta)):
        if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        setattr(s, name, t.data_ptr())
    return s


# ---- thin wrappers with the C names --------------------------------------------------------------------
def ges_abi_version() -> int:
    return lib().ges_abi_version()


def ges_workspace_query(n, width, height):
    a, b = C.c_size_t(0), C.c_size_t(0)
    _check(lib().ges_workspace_query(int(n), int(width), int(height), C.byref(a), C.byref(b)))
    return a.value, b.value


def ges_key_workspace_query(num_keys, n, width, height):
    a = C.c_size_t(0)
    _check(lib().ges_key_workspace_query(int(num_keys), int(n), int(width), int(height), C.byref(a)))
    return a.value


def ges_preprocess(splats, cam, params, splat_ws, read_num_keys=True, stream=None):
    k = C.c_uint64(0)
    _check(lib().ges_preprocess(C.byref(splats), C.byref(cam), C.byref(params), _ptr(splat_ws),
                                splat_ws.numel(), C.byref(k) if read_num_keys else None, _stream(stream)))
    return k.value if read_num_keys else None


def ges_render_forward(splats, cam, params, splat_ws, key_ws, num_keys, pixel_ws, out_rgb, stream=None):
    _check(lib().ges_render_forward(C.byref(splats), C.byref(cam), C.byref(params), _ptr(splat_ws), _ptr(key_ws),
                                    0 if key_ws is None else key_ws.numel(), int(num_keys), _ptr(pixel_ws),
                                    _ptr(out_rgb), _stream(stream)))


def ges_render_backward(splats, cam, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads: dict, stream=None):
    g = ges_splat_grads()
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta"):
        t = grads.get(k)
        setattr(g, k, None if t is None else t.data_ptr())
    _check(lib().ges_render_backward(C.byref(splats), C.byref(cam), C.byref(params), _ptr(splat_ws), _ptr(key_ws),
                                     _ptr(pixel_ws), _ptr(dL_drgb), C.byref(g), _stream(stream)))


def ges_frame_view_get(n, width, height, splat_ws, key_ws, num_keys, pixel_ws, views=1, view=0) -> ges_frame_view:
    v = ges_frame_view()
    _check(lib().ges_frame_view_get_views(int(n), int(views), int(width), int(height), _ptr(splat_ws), _ptr(key_ws),
                                          int(num_keys), _ptr(pixel_ws), int(view), C.byref(v)))
    return v


# ---- several views of one scene per launch sequence -----------------------------------------------------
def _cams(cams):
    return (ges_camera * len(cams))(*cams)


def ges_views_workspace_query(n, views, width, height):
    a, b = C.c_size_t(0), C.c_size_t(0)
    _check(lib().ges_views_workspace_query(int(n), int(views), int(width), int(height), C.byref(a), C.byref(b)))
    return a.value, b.value


def ges_preprocess_views(splats, cams, params, splat_ws, read_num_keys=True, stream=None):
    """cams: list of ges_camera (one resolution).  Returns the batch's slot count when read_num_keys."""
    k = C.c_uint64(0)
    _check(lib().ges_preprocess_views(C.byref(splats), _cams(cams), len(cams), C.byref(params), _ptr(splat_ws),
                                      splat_ws.numel(), C.byref(k) if read_num_keys else None, _stream(stream)))
    return k.value if read_num_keys else None


def ges_render_forward_views(splats, cams, params, splat_ws, key_ws, num_keys, pixel_ws, out_rgb, stream=None):
    """out_rgb: [len(cams), H, W, 3] float32."""
    _check(lib().ges_render_forward_views(C.byref(splats), _cams(cams), len(cams), C.byref(params), _ptr(splat_ws),
                                          _ptr(key_ws), 0 if key_ws is None else key_ws.numel(), int(num_keys),
                                          _ptr(pixel_ws), _ptr(out_rgb), _stream(stream)))


def _grads_struct(grads):
    g = ges_splat_grads()
    if grads is not None:
        for name in SPLAT_PARAMS:
            t = grads.get(name)
            setattr(g, name, None if t is None else t.data_ptr())
    return g


def ges_render_backward_views(splats, cams, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads: dict,
                              accumulate=False, grad_accum=None, grad_count=None, stream=None):
    """Summed parameter gradients of the views (dL_drgb: [len(cams), H, W, 3]) written to (or added to) grads."""
    _check(lib().ges_render_backward_views(C.byref(splats), _cams(cams), len(cams), C.byref(params), _ptr(splat_ws),
                                           _ptr(key_ws), _ptr(pixel_ws), _ptr(dL_drgb), C.byref(_grads_struct(grads)),
                                           1 if accumulate else 0, _ptr(grad_accum), _ptr(grad_count),
                                           _stream(stream)))


def ges_render_backward_views_adam(splats, cams, params, splat_ws, key_ws, pixel_ws, dL_drgb, exp_avg: dict,
                                   exp_avg_sq: dict, lrs: dict, step, beta1=0.9, beta2=0.999, eps=1e-15, grads=None,
                                   grad_accum=None, grad_count=None, stream=None):
    """Fused Adam over the views' summed gradients (grads: required with more than one view; receives the sum)."""
    opt = _adam_struct(exp_avg, exp_avg_sq, lrs, step, beta1, beta2, eps, grad_accum, grad_count, None)
    _check(lib().ges_render_backward_views_adam(C.byref(splats), _cams(cams), len(cams), C.byref(params),
                                                _ptr(splat_ws), _ptr(key_ws), _ptr(pixel_ws), _ptr(dL_drgb),
                                                C.byref(_grads_struct(grads)), C.byref(opt), _stream(stream)))


STAGES = ["preprocess", "depth_sort", "key_scan", "duplicate", "tile_sort", "raster_forward", "raster_backward",
          "preprocess_backward", "zero", "loss", "adam", "ssim", "mix_fit", "row_reduce"]


def ges_profile_enable(on: bool):
    _check(lib().ges_profile_enable(1 if on else 0))


def ges_profile_select(stages):
    """Time only the named stages (names of STAGES); an empty list switches timing off."""
    mask = 0
    for st in stages:
        mask |= 1 << STAGES.index(st)
    _check(lib().ges_profile_select(mask))


def ges_profile_read(reset=True):
    ms = (C.c_double * len(STAGES))()
    n = (C.c_int64 * len(STAGES))()
    _check(lib().ges_profile_read(ms, n, 1 if reset else 0))
    return {STAGES[k]: (ms[k], n[k]) for k in range(len(STAGES))}


def ges_freq_mask(target, omega, mask=None, stream=None):
    H, W = int(target.shape[0]), int(target.shape[1])
    scratch = torch.empty(lib().ges_mask_scratch_bytes(W, H), dtype=torch.uint8, device=target.device)
    if mask is None:
        mask = torch.empty((H, W), dtype=torch.uint8, device=target.device)
    _check(lib().ges_freq_mask(_ptr(target), W, H, float(omega), _ptr(scratch), _ptr(mask), _stream(stream)))
    return mask


def ges_freq_mask_static(target, omega, mask=None, stream=None):
    """The frequency mask with the library's own scratch array (no scratch buffer is allocated)."""
    H, W = int(target.shape[0]), int(target.shape[1])
    if mask is None:
        mask = torch.empty((H, W), dtype=torch.uint8, device=target.device)
    _check(lib().ges_freq_mask_static(_ptr(target), W, H, float(omega), _ptr(mask), _stream(stream)))
    return mask


def ges_loss(img, target, mask, lam_l1, lam_w, dL_dimg=None, loss_out=None, scratch=None, stream=None):
    H, W = int(img.shape[0]), int(img.shape[1])
    if dL_dimg is None:
        dL_dimg = torch.empty_like(img)
    if loss_out is None:
        loss_out = torch.empty((), dtype=torch.float32, device=img.device)
    if scratch is None:
        scratch = torch.empty(lib().ges_loss_scratch_bytes(), dtype=torch.uint8, device=img.device)
    _check(lib().ges_loss(_ptr(img), _ptr(target), _ptr(mask), W, H, float(lam_l1), float(lam_w), _ptr(scratch),
                          _ptr(loss_out), _ptr(dL_dimg), _stream(stream)))
    return loss_out, dL_dimg


def ges_ssim_loss(img, target, lam_ssim, loss_inout, dL_dimg, scratch=None, stream=None):
    """loss_inout += lam_ssim (1 - mean SSIM); dL_dimg += lam_ssim dL_ssim/dimg (both accumulated in place)."""
    H, W = int(img.shape[0]), int(img.shape[1])
    if scratch is None:
        scratch = torch.empty(lib().ges_ssim_scratch_bytes(W, H), dtype=torch.uint8, device=img.device)
    _check(lib().ges_ssim_loss(_ptr(img), _ptr(target), W, H, float(lam_ssim), _ptr(scratch), _ptr(loss_inout),
                               _ptr(dL_dimg), _stream(stream)))
    return loss_inout, dL_dimg


ADAM_MAX_GROUPS = 8


def ges_adam_step(groups, step, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """In-place Adam step; groups: list of (params, grads, exp_avg, exp_avg_sq, lr) with float32 CUDA tensors."""
    arr = (ges_adam_group * max(1, len(groups)))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        for t in (p, g, m, v):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != p.numel():
                raise ValueError("Adam groups take contiguous float32 tensors of one size")
        arr[k] = ges_adam_group(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(), float(lr))
    _check(lib().ges_adam_step(arr, len(groups), int(step), float(beta1), float(beta2), float(eps), _stream(stream)))


SPLAT_PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh", "beta")


def ges_render_backward_adam(splats, cam, params, splat_ws, key_ws, pixel_ws, dL_drgb, exp_avg: dict,
                             exp_avg_sq: dict, lrs: dict, step, beta1=0.9, beta2=0.999, eps=1e-15, grads=None,
                             grad_accum=None, grad_count=None, grads_in=None, stream=None):
    """Backward pass with Adam fused in: updates the tensors behind ``splats`` and the moments in place; with
    grad_accum/grad_count also accumulates the densification statistic; grads_in (dict) holds other views'
    gradients added to this view's before the update."""
    opt = _adam_struct(exp_avg, exp_avg_sq, lrs, step, beta1, beta2, eps, grad_accum, grad_count, grads_in)
    _check(lib().ges_render_backward_adam(C.byref(splats), C.byref(cam), C.byref(params), _ptr(splat_ws),
                                          _ptr(key_ws), _ptr(pixel_ws), _ptr(dL_drgb), C.byref(_grads_struct(grads)),
                                          C.byref(opt), _stream(stream)))


def _adam_struct(exp_avg, exp_avg_sq, lrs, step, beta1, beta2, eps, grad_accum, grad_count, grads_in):
    opt = ges_adam_splats()
    for k, name in enumerate(SPLAT_PARAMS):
        opt.grads_in[k] = None if grads_in is None else grads_in[name].data_ptr()
    opt.grad_accum = None if grad_accum is None else grad_accum.data_ptr()
    opt.grad_count = None if grad_count is None else grad_count.data_ptr()
    for k, name in enumerate(SPLAT_PARAMS):
        opt.exp_avg[k] = exp_avg[name].data_ptr()
        opt.exp_avg_sq[k] = exp_avg_sq[name].data_ptr()
        opt.lr[k] = float(lrs[name])
    opt.step, opt.beta1, opt.beta2, opt.eps = int(step), float(beta1), float(beta2), float(eps)
    return opt


def _splat_set(d: dict | None) -> ges_splat_set:
    st = ges_splat_set()
    for name in SPLAT_PARAMS:
        t = None if d is None else d.get(name)
        setattr(st, name, None if t is None else t.data_ptr())
    return st


def ges_prune_splats(src_sets: list, dst_sets: list, sh_degree: int, min_opacity: float, min_beta: float,
                     scratch=None, stream=None) -> int:
    """Compact the survivors of every set in src_sets into dst_sets (dicts of float32 CUDA tensors; set 0
    holds the parameters); returns the survivor count (waits for the stream)."""
    n = int(src_sets[0]["beta"].shape[0])
    k = len(src_sets)
    src = (ges_splat_set * k)(*[_splat_set(d) for d in src_sets])
    dst = (ges_splat_set * k)(*[_splat_set(d) for d in dst_sets])
    if scratch is None:
        scratch = torch.empty(lib().ges_prune_scratch_bytes(n), dtype=torch.uint8, device=src_sets[0]["beta"].device)
    kept = C.c_int64(0)
    _check(lib().ges_prune_splats(n, int(sh_degree), src, dst, k, float(min_opacity), float(min_beta), _ptr(scratch),
                                  scratch.numel(), C.byref(kept), _stream(stream)))
    return kept.value


def ges_densify(src_sets: list, dst_sets: list, sh_degree: int, grad_accum, grad_count, normals,
                grad_threshold: float, scale_threshold: float, scratch=None, stream=None) -> int:
    """Clone/split into dst_sets (dicts of float32 CUDA tensors with room for the result); returns the new
    count (waits for the stream).  Raises GESError (capacity) when dst is too small."""
    n = int(src_sets[0]["beta"].shape[0])
    cap = int(dst_sets[0]["beta"].shape[0])
    k = len(src_sets)
    src = (ges_splat_set * k)(*[_splat_set(d) for d in src_sets])
    dst = (ges_splat_set * k)(*[_splat_set(d) for d in dst_sets])
    if scratch is None:
        scratch = torch.empty(lib().ges_densify_scratch_bytes(n), dtype=torch.uint8, device=src_sets[0]["beta"].device)
    out = C.c_int64(0)
    _check(lib().ges_densify(n, int(sh_degree), src, dst, k, cap, _ptr(grad_accum), _ptr(grad_count), _ptr(normals),
                             float(grad_threshold), float(scale_threshold), _ptr(scratch), scratch.numel(),
                             C.byref(out), _stream(stream)))
    return out.value


def ges_opacity_reset(opacity_logits, exp_avg=None, exp_avg_sq=None, max_opacity=0.01, stream=None):
    _check(lib().ges_opacity_reset(_ptr(opacity_logits), _ptr(exp_avg), _ptr(exp_avg_sq), int(opacity_logits.numel()),
                                   float(max_opacity), _stream(stream)))


def ges_shape_reset(beta, exp_avg=None, exp_avg_sq=None, value=2.0, stream=None):
    _check(lib().ges_shape_reset(_ptr(beta), _ptr(exp_avg), _ptr(exp_avg_sq), int(beta.numel()), float(value),
                                 _stream(stream)))


MIX_MODELS = {"gmm": 0, "dog": 1, "log": 2, "gef": 3}
MIX_MAX_COMPONENTS = 128


def ges_mix_fit(problems, targets, x0, dx, params, epochs, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_out=None,
                final_loss=None, order="largest_first", stream=None):
    """problems: int32 CUDA tensor [P, 4] (model, n, positive, target); targets [T, m]; params [P, 128, 4]
    updated in place.  order: "largest_first" (workgroups take the problems by decreasing n), None (in
    order) or an int32 CUDA permutation.  Returns final_loss [P]."""
    P = int(problems.shape[0])
    if problems.dtype != torch.int32 or problems.dim() != 2 or problems.shape[1] != 4 or not problems.is_contiguous():
        raise ValueError("problems must be a contiguous int32 [P, 4] tensor")
    if params.shape != (P, MIX_MAX_COMPONENTS, 4) or params.dtype != torch.float32 or not params.is_contiguous():
        raise ValueError("params must be a contiguous float32 [P, 128, 4] tensor")
    if final_loss is None:
        final_loss = torch.empty(P, dtype=torch.float32, device=params.device)
    if isinstance(order, str):
        # a stable sort on the device: the table is an input, the order only schedules it
        order = torch.argsort(-problems[:, 1].to(torch.int64), stable=True).to(torch.int32)
    _check(lib().ges_mix_fit(_ptr(problems), P, _ptr(targets), int(targets.shape[0]), int(targets.shape[1]),
                             float(x0), float(dx), _ptr(params), _ptr(grad_out), _ptr(final_loss), _ptr(order),
                             int(epochs),
                             float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))
    return final_loss


def ges_render_backward_accumulate(splats, cam, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads: dict,
                                   grad_accum=None, grad_count=None, stream=None):
    """Backward pass of one more view: its parameter gradients are added to ``grads``."""
    g = ges_splat_grads()
    for k in SPLAT_PARAMS:
        t = grads.get(k)
        setattr(g, k, None if t is None else t.data_ptr())
    _check(lib().ges_render_backward_accumulate(C.byref(splats), C.byref(cam), C.byref(params), _ptr(splat_ws),
                                                _ptr(key_ws), _ptr(pixel_ws), _ptr(dL_drgb), C.byref(g),
                                                _ptr(grad_accum), _ptr(grad_count), _stream(stream)))


def ges_expon_lr(step, lr_init, lr_final, max_steps, delay_steps=0, delay_mult=1.0) -> float:
    return lib().ges_expon_lr(int(step), float(lr_init), float(lr_final), int(max_steps), int(delay_steps),
                              float(delay_mult))


def ges_loss_schedule(iteration, total_iterations, lam_ssim, lam_omega):
    """(omega, lam_l1) of an iteration: the mask strength and the L1 weight (binary32)."""
    w, l1 = C.c_float(0.0), C.c_float(0.0)
    _check(lib().ges_loss_schedule(int(iteration), int(total_iterations), float(lam_ssim), float(lam_omega),
                                   C.byref(w), C.byref(l1)))
    return w.value, l1.value


# ---- a frame: owns the workspaces of one (scene, camera) render --------------------------------------
@dataclass
class Frame:
    """Workspaces and results of one render; re-usable across calls with the same sizes."""
    n: int
    width: int
    height: int
    splat_ws: torch.Tensor
    pixel_ws: torch.Tensor
    key_ws: torch.Tensor | None = None
    num_keys: int = 0        # the slot count (or capacity) the frame was rendered with
    key_capacity: int = 0    # slots the current key workspace holds
    views: int = 1           # views of one scene rendered together (the ..._views calls)

    @staticmethod
    def create(n, width, height, device="cuda", views=1):
        sb, pb = ges_views_workspace_query(n, views, width, height)
        return Frame(n, width, height, torch.empty(sb, dtype=torch.uint8, device=device),
                     torch.empty(pb, dtype=torch.uint8, device=device), views=views)

    def ensure_keys(self, num_keys):
        if self.key_ws is None or self.key_capacity < num_keys:
            # grow with headroom so that small changes of the key count do not reallocate
            cap = max(int(num_keys * 1.25), num_keys + 1024)
            need = ges_key_workspace_query(cap, self.n, self.width, self.height)
            self.key_ws = torch.empty(need, dtype=torch.uint8, device=self.splat_ws.device)
            self.key_capacity = cap
        self.num_keys = num_keys

    def view(self, v=0) -> ges_frame_view:
        return ges_frame_view_get(self.n, self.width, self.height, self.splat_ws, self.key_ws, self.num_keys,
                                  self.pixel_ws, self.views, v)


def frame_arrays(frame: Frame, n: int, view=0) -> dict:
    """Copies of a frame's inspection arrays (of view `view` of a multi-view frame) as numpy (tests)."""
    v = frame.view(view)
    out = {}
    ws = frame.splat_ws

    def sl(ptr, nbytes, tensor):
        off = ptr - tensor.data_ptr()
        return tensor[off:off + nbytes]

    out["records"] = sl(v.records, 64 * n, ws).view(torch.float32).reshape(n, 16).cpu().numpy()
    T = v.tiles_x * v.tiles_y
    out["ranges"] = sl(v.tile_ranges, 8 * T, ws).view(torch.int32).reshape(T, 2).cpu().numpy().view(np.uint32)
    out["grad2d"] = sl(v.grad2d, 8 * GRAD2D_STRIDE * n, ws).view(torch.float64).reshape(n, GRAD2D_STRIDE).cpu().numpy()
    out["stats"] = sl(v.stats, 32, ws).view(torch.int64).cpu().numpy()
    out["keys"] = int(out["stats"][0])
    out["tile_work"] = sl(v.tile_work, 4 * T, ws).view(torch.int32).cpu().numpy().view(np.uint32)
    out["group_order"] = sl(v.group_order, 4 * ((T + 7) // 8), ws).view(torch.int32).cpu().numpy().view(np.uint32)
    if frame.key_ws is not None and frame.num_keys > 0:
        K = out["keys"]
        if frame.views > 1:   # the sorted pairs cover every view of the batch
            K = sum(int(sl(frame.view(u).stats, 8, ws).view(torch.int64).cpu()[0]) for u in range(frame.views))
        K = min(K, frame.num_keys)
        pairs = sl(v.sorted_pairs, 8 * K, frame.key_ws).view(torch.int32).reshape(K, 2).cpu().numpy().view(np.uint32)
        out["sorted_ids"] = pairs[:, 0].copy()
        out["sorted_slots"] = pairs[:, 1].copy()
        out["sorted_tiles"] = sl(v.sorted_tiles, 4 * K, frame.key_ws).view(torch.int32).cpu().numpy().view(np.uint32)
        marks = sl(v.row_marks, 4 * ((frame.num_keys + 31) // 32), frame.key_ws).cpu().numpy()
        out["rows_stored"] = int(np.unpackbits(marks).sum())
    px = frame.width * frame.height
    out["final_T"] = sl(v.final_T, 4 * px, frame.pixel_ws).view(torch.float32).reshape(frame.height, frame.width).cpu().numpy()
    out["n_contrib"] = sl(v.n_contrib, 4 * px, frame.pixel_ws).view(torch.int32).reshape(
        frame.height, frame.width).cpu().numpy().view(np.uint32)
    return out


def render(scene: dict, cam, falloff=FALLOFF_PHI, tile_cull=TILES_SQUARE, rho=0.1, bg=(0.0, 0.0, 0.0), frame=None,
           out=None, stream=None):
    """Preprocess + forward render of one view.  scene: dict of CUDA float32 tensors."""
    s = splats_struct(scene["means"], scene["log_scales"], scene["quats"], scene["opacity_logits"], scene["sh"],
                      scene["beta"])
    c = camera_struct(cam)
    p = params_struct(falloff, tile_cull, rho, bg)
    if frame is None:
        frame = Frame.create(s.n, c.width, c.height, scene["means"].device)
    k = ges_preprocess(s, c, p, frame.splat_ws, True, stream)
    frame.ensure_keys(k)
    if out is None:
        out = torch.empty((c.height, c.width, 3), dtype=torch.float32, device=scene["means"].device)
    ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, out, stream)
    return out, frame
