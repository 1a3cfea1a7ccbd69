"""ctypes wrapper around the C++ CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline leg
of the benchmark.  It shares no code with the HIP library and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

MODE_F32, MODE_F64 = 0, 1
FALLOFF_PHI, FALLOFF_GEF, FALLOFF_PHI_EXACT = 0, 1, 2
TILES_SQUARE, TILES_ELLIPSE = 0, 1
TILE = 16


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (no fast-math, no FMA contraction)."""
    src = os.path.join(HERE, "ges_oracle.cpp")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", LIB_PATH + ".tmp", src]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Splats(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("beta", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("near_z", C.c_float)]


class _Params(C.Structure):
    _fields_ = [("falloff", C.c_int32), ("tile_cull", C.c_int32), ("rho", C.c_float), ("bg", C.c_float * 3)]


class _Record(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("u", "v", "depth", "conic", "qmax", "opacity", "rgb", "beta", "radius",
                                          "rect", "tiles_touched", "clamp_bits")]


class _Stats(C.Structure):
    _fields_ = [("pairs_examined", C.c_int64), ("pairs_skipped", C.c_int64), ("pairs_blended", C.c_int64),
                ("pixels_flagged", C.c_int64), ("decision_hash", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB_PATH)
        for name in ("oc_preprocess", "oc_splat_in_tile", "oc_tile_counts", "oc_build_keys", "oc_tile_list",
                     "oc_render", "oc_render_untiled", "oc_backward", "oc_backward_untiled", "oc_num_threads"):
            getattr(_lib, name).restype = C.c_int
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


@dataclass
class Record:
    u: np.ndarray
    v: np.ndarray
    depth: np.ndarray
    conic: np.ndarray
    qmax: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray
    beta: np.ndarray
    radius: np.ndarray
    rect: np.ndarray
    tiles_touched: np.ndarray
    clamp_bits: np.ndarray

    @staticmethod
    def empty(n):
        return Record(np.zeros(n), np.zeros(n), np.zeros(n), np.zeros((n, 3)), np.zeros(n), np.zeros(n),
                      np.zeros((n, 3)), np.zeros(n), np.zeros(n, np.int32), np.zeros((n, 4), np.int32),
                      np.zeros(n, np.int64), np.zeros(n, np.uint8))

    @property
    def n(self):
        return self.u.shape[0]

    def c(self):
        r = _Record()
        for k, _ in _Record._fields_:
            setattr(r, k, _p(getattr(self, k)))
        return r


def camera_struct(cam) -> _Camera:
    c = _Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).ravel()]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).ravel()]
    c.fx, c.fy, c.cx, c.cy, c.near_z = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy, cam.near))
    return c


def params_struct(falloff=FALLOFF_PHI, tile_cull=TILES_SQUARE, rho=0.1, bg=(0.0, 0.0, 0.0)) -> _Params:
    p = _Params()
    p.falloff, p.tile_cull, p.rho = int(falloff), int(tile_cull), float(rho)
    p.bg[:] = [float(b) for b in bg]
    return p


class Oracle:
    """One scene + camera + parameters, evaluated on the CPU."""

    def __init__(self, scene_arrays: dict, sh_degree: int, cam, falloff=FALLOFF_PHI, tile_cull=TILES_SQUARE,
                 rho=0.1, bg=(0.0, 0.0, 0.0)):
        self.arr = {k: _f32(v) for k, v in scene_arrays.items()}
        self.n = int(self.arr["means"].shape[0])
        self.sh_degree = int(sh_degree)
        self.cam = cam
        self.W, self.H = int(cam.width), int(cam.height)
        self.TX, self.TY = (self.W + TILE - 1) // TILE, (self.H + TILE - 1) // TILE
        self.cs = camera_struct(cam)
        self.ps = params_struct(falloff, tile_cull, rho, bg)
        self.falloff, self.tile_cull, self.rho, self.bg = falloff, tile_cull, rho, tuple(bg)

    def _splats(self):
        s = _Splats()
        s.n, s.sh_degree = self.n, self.sh_degree
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "beta"):
            setattr(s, k, _p(self.arr[k]))
        return s

    def preprocess(self, mode=MODE_F32) -> Record:
        rec = Record.empty(self.n)
        rc = rec.c()
        s = self._splats()
        rv = lib().oc_preprocess(mode, C.byref(s), C.byref(self.cs), C.byref(self.ps), C.byref(rc))
        assert rv == 0, rv
        return rec

    def tile_counts(self, rec: Record, mode=MODE_F32):
        counts = np.zeros(self.TX * self.TY, np.int64)
        rc = rec.c()
        lib().oc_tile_counts(mode, C.byref(rc), C.c_int64(rec.n), C.byref(self.cs), C.byref(self.ps), _p(counts))
        return counts

    def build_keys(self, rec: Record, mode=MODE_F32):
        K = int(rec.tiles_touched.sum())
        keys = np.zeros(max(K, 1), np.uint64)
        vals = np.zeros(max(K, 1), np.uint32)
        ranges = np.zeros((self.TX * self.TY, 2), np.int64)
        rc = rec.c()
        rv = lib().oc_build_keys(mode, C.byref(rc), C.c_int64(rec.n), C.byref(self.cs), C.byref(self.ps), _p(keys),
                                 _p(vals), C.c_int64(K), _p(ranges))
        assert rv == 0, rv
        return keys[:K], vals[:K], ranges

    def tile_list(self, rec: Record, tile: int, mode=MODE_F32):
        rc = rec.c()
        ln = C.c_int64(0)
        cap = 1 << 16
        while True:
            out = np.zeros(cap, np.uint32)
            lib().oc_tile_list(mode, C.byref(rc), C.c_int64(rec.n), C.byref(self.cs), C.byref(self.ps),
                               C.c_int32(tile), _p(out), C.c_int64(cap), C.byref(ln))
            if ln.value <= cap:
                return out[:ln.value].copy()
            cap = ln.value

    def render(self, rec: Record, values, ranges, tiles=None, mode=MODE_F32):
        img = np.zeros((self.H, self.W, 3))
        alt = np.zeros((self.H, self.W, 3))
        fT = np.zeros((self.H, self.W))
        nc = np.zeros((self.H, self.W), np.int32)
        fl = np.zeros((self.H, self.W), np.uint8)
        st = _Stats()
        rc = rec.c()
        tl = None if tiles is None else np.ascontiguousarray(tiles, np.int32)
        values = np.ascontiguousarray(values, np.uint32)
        ranges = np.ascontiguousarray(ranges, np.int64)
        rv = lib().oc_render(mode, C.byref(rc), C.c_int64(rec.n), C.byref(self.cs), C.byref(self.ps), _p(values),
                             _p(ranges), _p(tl), C.c_int64(0 if tl is None else len(tl)), _p(img), _p(fT), _p(nc),
                             _p(fl), _p(alt), C.byref(st))
        assert rv == 0, rv
        return dict(img=img, final_T=fT, n_contrib=nc, flags=fl, alt=alt, stats=_stats_dict(st))

    def render_untiled(self, rec: Record, mode=MODE_F32):
        img = np.zeros((self.H, self.W, 3))
        alt = np.zeros((self.H, self.W, 3))
        fT = np.zeros((self.H, self.W))
        nc = np.zeros((self.H, self.W), np.int32)
        fl = np.zeros((self.H, self.W), np.uint8)
        st = _Stats()
        rc = rec.c()
        rv = lib().oc_render_untiled(mode, C.byref(rc), C.c_int64(rec.n), C.byref(self.cs), C.byref(self.ps),
                                     _p(img), _p(fT), _p(nc), _p(fl), _p(alt), C.byref(st))
        assert rv == 0, rv
        return dict(img=img, final_T=fT, n_contrib=nc, flags=fl, alt=alt, stats=_stats_dict(st))

    def backward2d(self, rec: Record, dL_dimg, values=None, ranges=None, tiles=None, mode=MODE_F32,
                   with_delta=False):
        """Per-splat gradient of <dL_dimg, image> w.r.t. (u,v,a,b,c,opacity,r,g,b,beta).

        with_delta: also return, per splat and component, the allowance from floating-point-ambiguous
        decisions (delta), the sum of |per-pixel contribution| (mass) and the first-order bound on the
        binary32 evaluation error of the contributions (ebound): (g2d, delta, mass, ebound, stats)."""
        g2d = np.zeros((rec.n, 10))
        delta = np.zeros((rec.n, 10)) if with_delta else None
        mass = np.zeros((rec.n, 10)) if with_delta else None
        ebound = np.zeros((rec.n, 10)) if with_delta else None
        d = np.ascontiguousarray(dL_dimg, np.float64)
        st = _Stats()
        rc = rec.c()
        if values is None:
            rv = lib().oc_backward_untiled(mode, C.byref(rc), C.c_int64(rec.n), C.byref(self.cs), C.byref(self.ps),
                                           _p(d), _p(g2d), _p(delta), _p(mass), _p(ebound), C.byref(st))
        else:
            tl = None if tiles is None else np.ascontiguousarray(tiles, np.int32)
            rv = lib().oc_backward(mode, C.byref(rc), C.c_int64(rec.n), C.byref(self.cs), C.byref(self.ps),
                                   _p(np.ascontiguousarray(values, np.uint32)),
                                   _p(np.ascontiguousarray(ranges, np.int64)), _p(tl),
                                   C.c_int64(0 if tl is None else len(tl)), _p(d), _p(g2d), _p(delta), _p(mass),
                                   _p(ebound), C.byref(st))
        assert rv == 0, rv
        if with_delta:
            return g2d, delta, mass, ebound, _stats_dict(st)
        return g2d, _stats_dict(st)


def _stats_dict(st):
    return dict(pairs_examined=st.pairs_examined, pairs_skipped=st.pairs_skipped, pairs_blended=st.pairs_blended,
                pixels_flagged=st.pixels_flagged, decision_hash=st.decision_hash)


def exp_c(x):
    x = _f32(x).ravel()
    y = np.empty_like(x)
    lib().oc_exp_c(_p(x), _p(y), C.c_int64(x.size))
    return y


def log_c(x):
    x = _f32(x).ravel()
    y = np.empty_like(x)
    lib().oc_log_c(_p(x), _p(y), C.c_int64(x.size))
    return y


def lgamma_c(x):
    x = _f32(x).ravel()
    y = np.empty_like(x)
    lib().oc_lgamma_c(_p(x), _p(y), C.c_int64(x.size))
    return y


def num_threads():
    return lib().oc_num_threads()


def set_num_threads(n: int):
    lib().oc_set_num_threads(int(n))
