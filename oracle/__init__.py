"""FP64 CPU oracle for the Fourier PlenOctree render and fine-tune path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library and never imports the HIP package: the arithmetic lives in
`fpo_oracle.c` (plain C, FP64) and in the numpy checkers `brute.py` and
`codec.py`.

Python here only marshals numpy arrays into the C functions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpo_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm", "-lpthread"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("fwd", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fov_y_deg", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("time", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("n_sigma", ctypes.c_int32), ("n_sh_fourier", ctypes.c_int32),
                ("period", ctypes.c_double), ("sigma_scale", ctypes.c_double),
                ("stop_T", ctypes.c_double), ("band", ctypes.c_double),
                ("bg", ctypes.c_double * 3)]


_P = ctypes.c_void_p


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        L.or_basis.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P]
        L.or_sh9.argtypes = [_P, _P]
        L.or_camera_ray.argtypes = [ctypes.POINTER(_Camera), ctypes.c_int32, ctypes.c_int32, _P, _P]
        L.or_camera_rays.argtypes = [ctypes.POINTER(_Camera), ctypes.c_int64, _P, _P, _P, _P]
        L.or_tree_build.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.or_tree_build.restype = ctypes.c_void_p
        L.or_tree_free.argtypes = [ctypes.c_void_p]
        L.or_tree_locate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.or_tree_locate.restype = ctypes.c_int64
        L.or_trace.argtypes = [ctypes.c_void_p, _P, _P, ctypes.c_int64, _P, _P, _P]
        L.or_trace.restype = ctypes.c_int64
        L.or_render_rays.argtypes = [ctypes.c_void_p, _P, _P, ctypes.POINTER(_Params), _P, ctypes.c_int32,
                                     _P, _P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P, _P, _P]
        L.or_render_rays.restype = ctypes.c_int32
        L.or_render_grad.argtypes = [ctypes.c_void_p, _P, ctypes.POINTER(_Params), _P, ctypes.c_int32,
                                     _P, _P, _P, ctypes.c_int64, _P, ctypes.c_int32, _P, _P]
        L.or_render_grad.restype = ctypes.c_int32
        L.or_bake.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(_Params), _P, ctypes.c_int32, ctypes.c_int32, _P]
        L.or_ray_labels.argtypes = [ctypes.c_void_p, _P, ctypes.POINTER(_Params), _P, ctypes.c_int32,
                                    _P, _P, _P, ctypes.c_int64, _P]
        L.or_ray_labels.restype = ctypes.c_int32
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
def basis(t: float, period: float, n: int) -> np.ndarray:
    """Eq. 8 real Fourier basis values IDFT_i(t), i < n."""
    out = np.zeros(n, dtype=np.float64)
    lib().or_basis(float(t), float(period), int(n), _ptr(out))
    return out


def sh9(d) -> np.ndarray:
    """Real SH basis (degree <= 2) of a unit direction, 9 values."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(9, dtype=np.float64)
    lib().or_sh9(_ptr(d), _ptr(out))
    return out


def _camera_struct(cam) -> _Camera:
    c = _Camera()
    c.eye[:] = [float(v) for v in cam.eye]
    c.fwd[:] = [float(v) for v in cam.fwd]
    c.up[:] = [float(v) for v in cam.up]
    c.fov_y_deg = float(cam.fov_y_deg)
    c.width = int(cam.width)
    c.height = int(cam.height)
    c.time = float(cam.time)
    return c


def camera_rays(cam, px: Optional[np.ndarray] = None, py: Optional[np.ndarray] = None):
    """FP64 pinhole rays.  Without px/py: every pixel, row-major [H*W]."""
    if px is None:
        yy, xx = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
        px, py = xx.reshape(-1), yy.reshape(-1)
    c = _camera_struct(cam)
    px = np.ascontiguousarray(px, dtype=np.int32)
    py = np.ascontiguousarray(py, dtype=np.int32)
    n = len(px)
    o = np.zeros((n, 3))
    d = np.zeros((n, 3))
    lib().or_camera_rays(ctypes.byref(c), n, _ptr(px), _ptr(py), _ptr(o), _ptr(d))
    return o, d


class OracleTree:
    """Leaves (depth, i, j, k) in caller order, located by a hash of their keys."""

    def __init__(self, leaf_dijk: np.ndarray, max_depth: int):
        self.dijk = np.ascontiguousarray(leaf_dijk, dtype=np.int32)
        self.max_depth = int(max_depth)
        err = ctypes.c_int32(0)
        self._h = lib().or_tree_build(_ptr(self.dijk), self.dijk.shape[0], self.max_depth,
                                      ctypes.byref(err))
        self.error = int(err.value)
        if not self._h:
            raise ValueError(f"invalid leaf set (oracle error {self.error})")

    def close(self):
        if getattr(self, "_h", None):
            lib().or_tree_free(self._h)
            self._h = None

    __del__ = close

    @property
    def n_leaves(self) -> int:
        return int(self.dijk.shape[0])

    def locate(self, x: int, y: int, z: int) -> int:
        return int(lib().or_tree_locate(self._h, int(x), int(y), int(z)))

    def trace(self, o, d):
        """Segment list (leaf, t0, t1) of one ray; d is normalised first."""
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        d = d / np.linalg.norm(d)
        cap = 3 * (1 << self.max_depth) + 8
        leaf = np.zeros(cap, dtype=np.int64)
        t0 = np.zeros(cap)
        t1 = np.zeros(cap)
        n = lib().or_trace(self._h, _ptr(o), _ptr(d), cap, _ptr(leaf), _ptr(t0), _ptr(t1))
        return leaf[:n].copy(), t0[:n].copy(), t1[:n].copy()


def make_params(n_sigma=31, n_sh_fourier=5, period=60.0, sigma_scale=64.0, stop_T=0.0,
                band=1e-3, bg=(0.0, 0.0, 0.0)) -> _Params:
    p = _Params()
    p.n_sigma = n_sigma
    p.n_sh_fourier = n_sh_fourier
    p.period = period
    p.sigma_scale = sigma_scale
    p.stop_T = stop_T
    p.band = band
    p.bg[:] = [float(v) for v in bg]
    return p


def render_rays(tree: OracleTree, coeffs: Optional[np.ndarray], params: _Params, times: Sequence[float],
                o: np.ndarray, d: np.ndarray, t_idx: np.ndarray, n_threads: int = 1,
                snapshot: Optional[np.ndarray] = None):
    """Render rays in FP64.  Returns a dict with both early-termination outcomes.

    rgb: [n][2][3] (outcome 0 stops at threshold tau(1+band), outcome 1 at
    tau(1-band)); T: [n][2]; n_seg: [n][2] composited segments; n_opaque:
    [n][2] composited segments with positive optical depth; n_cells: [n]
    segments crossed without early stop.
    """
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    t_idx = np.ascontiguousarray(t_idx, dtype=np.int32)
    times = np.ascontiguousarray(times, dtype=np.float64)
    n = o.shape[0]
    c = None if coeffs is None else np.ascontiguousarray(coeffs, dtype=np.float64)
    s = None if snapshot is None else np.ascontiguousarray(snapshot, dtype=np.float64)
    rgb = np.zeros((n, 2, 3))
    T = np.zeros((n, 2))
    n_seg = np.zeros((n, 2), dtype=np.int64)
    n_opaque = np.zeros((n, 2), dtype=np.int64)
    n_cells = np.zeros(n, dtype=np.int64)
    st = lib().or_render_rays(tree._h, _ptr(c), _ptr(s), ctypes.byref(params), _ptr(times), len(times),
                              _ptr(o), _ptr(d), _ptr(t_idx), n, int(n_threads),
                              _ptr(rgb), _ptr(T), _ptr(n_seg), _ptr(n_opaque), _ptr(n_cells))
    if st != 0:
        raise MemoryError("oracle render failed")
    return {"rgb": rgb, "T": T, "n_seg": n_seg, "n_opaque": n_opaque, "n_cells": n_cells}


def render_grad(tree: OracleTree, coeffs: np.ndarray, params: _Params, times: Sequence[float],
                o: np.ndarray, d: np.ndarray, t_idx: np.ndarray, grad_rgb: np.ndarray, n_threads: int = 8):
    """dL/dk for dL/dC = grad_rgb, FP64.  Returns (grad [L][ncoeff], rgb [n][3]).
    The sums are formed in ray order for any thread count."""
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    t_idx = np.ascontiguousarray(t_idx, dtype=np.int32)
    times = np.ascontiguousarray(times, dtype=np.float64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    g = np.ascontiguousarray(grad_rgb, dtype=np.float64)
    grad = np.zeros_like(c)
    rgb = np.zeros((o.shape[0], 3))
    st = lib().or_render_grad(tree._h, _ptr(c), ctypes.byref(params), _ptr(times), len(times),
                              _ptr(o), _ptr(d), _ptr(t_idx), o.shape[0], _ptr(g), int(n_threads), _ptr(grad),
                              _ptr(rgb))
    if st != 0:
        raise MemoryError("oracle gradient failed")
    return grad, rgb


def bake(coeffs: np.ndarray, params: _Params, times: Sequence[float], n_threads: int = 1) -> np.ndarray:
    """Eq. 7 / Eq. 9 at every time: [n_t][28][L] FP64."""
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    times = np.ascontiguousarray(times, dtype=np.float64)
    out = np.zeros((len(times), 28, c.shape[0]))
    lib().or_bake(_ptr(c), c.shape[0], ctypes.byref(params), _ptr(times), len(times), int(n_threads), _ptr(out))
    return out


def ray_labels(tree: OracleTree, coeffs: np.ndarray, params: _Params, times: Sequence[float],
               o: np.ndarray, d: np.ndarray, t_idx: np.ndarray) -> np.ndarray:
    """Proposal labels [n][3] = (hit, s_in, s_out) from the plain walk."""
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    t_idx = np.ascontiguousarray(t_idx, dtype=np.int32)
    times = np.ascontiguousarray(times, dtype=np.float64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    out = np.zeros((o.shape[0], 3))
    st = lib().or_ray_labels(tree._h, _ptr(c), ctypes.byref(params), _ptr(times), len(times),
                             _ptr(o), _ptr(d), _ptr(t_idx), o.shape[0], _ptr(out))
    if st != 0:
        raise MemoryError("oracle labels failed")
    return out
