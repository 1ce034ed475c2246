"""ctypes binding of libfpo (include/fpo.h).

Argument marshalling only: every step of the render / fine-tune path runs in
the library (host C++ for tree building and the FP64 time basis, HIP kernels
on the device for everything else).  PyTorch provides device memory and the
current HIP stream.  If libfpo.so has not been built, importing the library
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfpo.so")

FPO_OK, FPO_E_INVALID, FPO_E_UNSUPPORTED, FPO_E_DEVICE, FPO_E_CAPACITY, FPO_E_NOMEM = range(6)
FPO_F32, FPO_BF16, FPO_FP8_E4M3 = 0, 1, 2
N_SIGMA, N_SH_FOURIER, SH_DEGREE, N_SH = 31, 5, 2, 9
N_COEFF = 166
N_BAKED = 28
BASIS_STRIDE = 32
CAMERA_FLOATS = 16
MAX_DEPTH = 10
COEFFS_PER_WORD = {FPO_F32: 4, FPO_BF16: 8, FPO_FP8_E4M3: 16}
RECORD_WORDS = {FPO_F32: 48, FPO_BF16: 24, FPO_FP8_E4M3: 16}   # 16-byte words per leaf record
SNAP_VALUES = 32
NOALLOC_SCRATCH_BYTES = 32 << 20   # fpo_render_noalloc's static device scratch


def record_words(dtype: int) -> int:
    return RECORD_WORDS[dtype]


class FpoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libfpo status {status}: {msg}")
        self.status = status


class Layout(ctypes.Structure):
    _fields_ = [("n_sigma", ctypes.c_int32), ("n_sh_fourier", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32), ("period", ctypes.c_float),
                ("sigma_scale", ctypes.c_float)]


class TreeView(ctypes.Structure):
    _fields_ = [("children", ctypes.c_void_p), ("n_nodes", ctypes.c_int64),
                ("max_depth", ctypes.c_int32), ("coeffs", ctypes.c_void_p),
                ("leaf_scale", ctypes.c_void_p), ("dtype", ctypes.c_int),
                ("n_leaves", ctypes.c_int64), ("leaf_stride", ctypes.c_int64),
                ("layout", Layout), ("grandchildren", ctypes.c_void_p), ("n_grandchild_rows", ctypes.c_int64),
                ("level_offsets", ctypes.c_void_p), ("bounds", ctypes.c_void_p)]


class CameraC(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("fwd", ctypes.c_float * 3),
                ("up", ctypes.c_float * 3), ("fov_y_deg", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("time", ctypes.c_double)]


FIELD_MAX_GAUSS = 8
FUSION_ACC = 32


class FieldC(ctypes.Structure):
    _fields_ = [("mu", (ctypes.c_float * 3) * FIELD_MAX_GAUSS), ("w", ctypes.c_float * FIELD_MAX_GAUSS),
                ("a", ctypes.c_float * FIELD_MAX_GAUSS), ("n_gauss", ctypes.c_int32),
                ("u", (ctypes.c_float * 3) * 3), ("v", (ctypes.c_float * 3) * 3), ("b", ctypes.c_float * 3)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("bg", ctypes.c_float * 3), ("stop_T", ctypes.c_float),
                ("snapshot", ctypes.c_void_p), ("snapshot_dtype", ctypes.c_int),
                ("snapshot_cam_stride", ctypes.c_int64), ("flags", ctypes.c_int32),
                ("coarse_bits", ctypes.c_void_p), ("proposal", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_int64)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_lib = None

# name -> argtypes; every function returns fpo_status (int)
_SIGS = {
    "fpo_build_tree": [_P, _I64, _I32, _P, _I64, _P, _P],
    "fpo_leaf_bounds": [_P, _I64, _I32, _P],
    "fpo_time_basis": [_P, _I32, ctypes.POINTER(Layout), _P],
    "fpo_camera_pack": [ctypes.POINTER(CameraC), _I32, _P],
    "fpo_pack_coeffs": [_P, _P, _I64, _I64, ctypes.POINTER(Layout), _P, _P],
    "fpo_render": [ctypes.POINTER(TreeView), ctypes.POINTER(CameraC), _I32,
                   ctypes.POINTER(RenderOpts), _P, _P, _P],
    "fpo_render_noalloc": [ctypes.POINTER(TreeView), ctypes.POINTER(CameraC), _I32,
                           ctypes.POINTER(RenderOpts), _P, _P, _P],
    "fpo_camera_rays": [_P, _I32, _P, _P, _P, _I64, _P, _P, _P],
    "fpo_render_rays": [ctypes.POINTER(TreeView), _P, _P, _P, _P, _I32, _I64,
                        ctypes.POINTER(RenderOpts), _P, _P, _P],
    "fpo_trace_rays": [ctypes.POINTER(TreeView), _P, _P, _I64, _I32, _P, _P, _P, _P],
    "fpo_render_backward": [ctypes.POINTER(TreeView), _P, _P, _P, _P, _I32, _I64,
                            ctypes.POINTER(RenderOpts), _P, _P, _P, _P],
    "fpo_l2_loss": [_P, _P, _I32, _I32, _I32, _P, _P, _P, _I64, _P, _P, _P],
    "fpo_adam_step": [_P, _P, _P, _P, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float, _I32, _P],
    "fpo_adam_step_dev": [_P, _P, _P, _P, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float, _P, _P],
    "fpo_adam_step_touched": [_P, _P, _P, _P, _I64, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, _I32, _P, _P],
    "fpo_quantize": [_P, _I64, _I64, ctypes.POINTER(Layout), ctypes.c_int, _P, _P, _P],
    "fpo_bake_times": [ctypes.POINTER(TreeView), _P, _I32, ctypes.c_int, _P, _P, _P],
    "fpo_coarse_occupancy": [_P, _I64, _I32, _P],
    "fpo_ray_labels": [ctypes.POINTER(TreeView), _P, _P, _P, _P, _P, _I32, _I64,
                       ctypes.POINTER(RenderOpts), _P, _P, _P],
    "fpo_mlp_forward": [_P, _P, _I64, _P, _P],
    "fpo_mlp_loss_grad": [_P, _P, _P, _P, _I64, _P, _P, _P, _P],
    "fpo_mlp_pack": [_P, _P, _P],
    "fpo_mlp_infer": [_P, _P, _I64, _P, _P],
    "fpo_union_leaves": [_P, _I64, _I32, _P, _I64, _P],
    "fpo_frame_values": [ctypes.POINTER(TreeView), _P, _P, _P, _I64, _P, _P, _P],
    "fpo_dft_frames": [_P, _I32, _I64, _I64, _I32, _P, _P, _P],
    "fpo_prune_leaves": [_P, _I64, ctypes.c_float, _P, _P],
    "fpo_fusion_observe": [ctypes.POINTER(TreeView), _P, ctypes.POINTER(CameraC), ctypes.POINTER(FieldC),
                           ctypes.c_float, _P, _P],
    "fpo_fusion_apply": [_P, _P, _P, _P, _I64, _P],
    "fpo_prune_at": [ctypes.POINTER(TreeView), _P, ctypes.c_int, _I64, _I32, _P, _P],
    "fpo_prune_at_sigma": [ctypes.POINTER(TreeView), _P, _I64, _I32, _P, _P],
    "fpo_grandchild_tables": [_P, _I64, _I32, _I64, _P, _P],
    "fpo_coarse_occupancy_at": [_P, _I64, _I32, _P, ctypes.c_int, ctypes.c_float, _P, _P],
}
# functions with another return type
_OTHER = {"fpo_mlp_workspace_floats": ([_I64], ctypes.c_int64)}


def lib():
    """Load libfpo.so (raises if it is missing: build it with build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2202_08614_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        for name, (args, res) in _OTHER.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        L.fpo_last_error.argtypes = []
        L.fpo_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    return list(_SIGS) + list(_OTHER) + ["fpo_last_error"]


def _check(st: int):
    if st != FPO_OK:
        raise FpoError(st, lib().fpo_last_error().decode())


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _t_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_layout(period: float = 60.0, sigma_scale: float = 64.0, n_sigma: int = N_SIGMA,
                n_sh_fourier: int = N_SH_FOURIER) -> Layout:
    return Layout(int(n_sigma), int(n_sh_fourier), SH_DEGREE, float(period), float(sigma_scale))


def layout_record_words(n_sigma: int, n_sh_fourier: int, dtype: int = FPO_F32) -> int:
    """16-byte words of a record of `dtype` for the layout (n1, n2): whole
    128-byte lines."""
    per_word = {FPO_F32: 4, FPO_BF16: 8, FPO_FP8_E4M3: 16}[dtype]
    return ((n_sigma + 27 * n_sh_fourier + per_word - 1) // per_word + 7) // 8 * 8


def camera_struct(cams) -> ctypes.Array:
    arr = (CameraC * len(cams))()
    for i, c in enumerate(cams):
        arr[i].eye[:] = [float(v) for v in c.eye]
        arr[i].fwd[:] = [float(v) for v in c.fwd]
        arr[i].up[:] = [float(v) for v in c.up]
        arr[i].fov_y_deg = float(c.fov_y_deg)
        arr[i].width = int(c.width)
        arr[i].height = int(c.height)
        arr[i].time = float(c.time)
    return arr


def make_opts(bg=(0.0, 0.0, 0.0), stop_T: float = 0.0, snapshot=None, snapshot_dtype: int = FPO_F32,
              snapshot_cam_stride: int = 0, flags: int = 0, coarse_bits=None, proposal=None,
              workspace=None) -> RenderOpts:
    """Render options.  Tensors passed here must outlive every call using them."""
    o = RenderOpts()
    o.bg[:] = [float(v) for v in bg]
    o.stop_T = float(stop_T)
    o.snapshot = None if snapshot is None else snapshot.data_ptr()
    o.snapshot_dtype = int(snapshot_dtype)
    o.snapshot_cam_stride = int(snapshot_cam_stride)
    o.flags = int(flags)
    o.coarse_bits = None if coarse_bits is None else coarse_bits.data_ptr()
    o.proposal = None if proposal is None else proposal.data_ptr()
    o.workspace = None if workspace is None else workspace.data_ptr()
    o.workspace_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    return o


def skip_workspace(n_cams: int, height: int, width: int, device):
    """Scratch for the skip modes of fpo_render."""
    import torch
    return torch.empty((min(n_cams, 16) * height * width * 2,), dtype=torch.float32, device=device)


def record_workspace(n_rays: int, cap: int, device):
    """Workspace for FPO_RAYS_RECORD: int32 counts of n_rays, then cap records
    of RECORD_BYTES per ray from the next 256-byte boundary."""
    import torch
    head = (4 * n_rays + 255) // 256 * 256
    nbytes = head + n_rays * cap * RECORD_BYTES
    return torch.empty((nbytes // 4,), dtype=torch.int32, device=device)


def record_counts(workspace, n_rays: int):
    """The per-ray record counts the forward left (-1: overflow)."""
    return workspace[:n_rays]


# ---------------------------------------------------------------------------
# host calls
# ---------------------------------------------------------------------------
def build_tree(leaf_dijk: np.ndarray, max_depth: int):
    """fpo_build_tree -> (children [n_nodes][8] int32, perm [L] int64)."""
    dijk = np.ascontiguousarray(leaf_dijk, dtype=np.int32)
    n = dijk.shape[0]
    n_nodes = ctypes.c_int64(0)
    _check(lib().fpo_build_tree(_np_ptr(dijk), n, int(max_depth), None, 0, ctypes.byref(n_nodes), None))
    children = np.zeros((n_nodes.value, 8), dtype=np.int32)
    perm = np.zeros(n, dtype=np.int64)
    _check(lib().fpo_build_tree(_np_ptr(dijk), n, int(max_depth), _np_ptr(children), n_nodes.value,
                                ctypes.byref(n_nodes), _np_ptr(perm)))
    return children, perm


def leaf_bounds(leaf_dijk: np.ndarray, max_depth: int) -> np.ndarray:
    """fpo_leaf_bounds -> int32 [6]: lo x, y, z, hi x, y, z on the finest lattice."""
    dijk = np.ascontiguousarray(leaf_dijk, dtype=np.int32)
    out = np.zeros(6, dtype=np.int32)
    _check(lib().fpo_leaf_bounds(_np_ptr(dijk), dijk.shape[0], int(max_depth), _np_ptr(out)))
    return out


def time_basis(times: Sequence[float], layout: Optional[Layout] = None) -> np.ndarray:
    layout = layout or make_layout()
    t = np.ascontiguousarray(times, dtype=np.float64)
    out = np.zeros((len(t), BASIS_STRIDE), dtype=np.float32)
    _check(lib().fpo_time_basis(_np_ptr(t), len(t), ctypes.byref(layout), _np_ptr(out)))
    return out


def camera_pack(cams) -> np.ndarray:
    arr = camera_struct(cams)
    out = np.zeros((len(cams), CAMERA_FLOATS), dtype=np.float32)
    _check(lib().fpo_camera_pack(arr, len(cams), _np_ptr(out)))
    return out


# ---------------------------------------------------------------------------
# device tree
# ---------------------------------------------------------------------------
class DeviceTree:
    """A tree resident on the GPU: child table, leaf records of coefficients
    ([leaf_stride][record_words][16 bytes]) and, for quantised stores, per-leaf
    scales."""

    def __init__(self, children, n_nodes: int, max_depth: int, coeffs, scale, dtype: int,
                 n_leaves: int, leaf_stride: int, perm: np.ndarray, layout: Layout,
                 n_upper: Optional[int] = None, grandchildren=None, levels: Optional[np.ndarray] = None,
                 bounds: Optional[np.ndarray] = None):
        self.children = children
        # host int32 [6]: lattice box holding every leaf (fpo_leaf_bounds), or None (the unit cube)
        self.bounds = None if bounds is None else np.ascontiguousarray(bounds, dtype=np.int32)
        # host int64 [max_depth + 1]: first node of each depth (fpo_build_tree's numbering), or None
        self.levels = None if levels is None else np.ascontiguousarray(levels, dtype=np.int64)
        # nodes that have an internal child (numbered first, breadth first); None: not known yet
        self.n_upper = n_upper
        # two-level table of `children` (fpo_grandchild_tables), or None
        self.grandchildren = grandchildren
        self.n_nodes = int(n_nodes)
        self.max_depth = int(max_depth)
        self.coeffs = coeffs
        self.scale = scale
        self.dtype = int(dtype)
        self.n_leaves = int(n_leaves)
        self.leaf_stride = int(leaf_stride)
        self.perm = perm
        self.layout = layout

    @classmethod
    def from_leaves(cls, leaf_dijk: np.ndarray, coeffs: np.ndarray, max_depth: int,
                    device="cuda", period: float = 60.0, sigma_scale: float = 64.0,
                    leaf_stride: Optional[int] = None, n_sigma: int = N_SIGMA,
                    n_sh_fourier: int = N_SH_FOURIER, clip: bool = True) -> "DeviceTree":
        """clip: camera renders start each ray on the leaves' bounds
        (fpo_leaf_bounds) instead of the unit cube."""
        import torch
        children, perm = build_tree(leaf_dijk, max_depth)
        n = int(leaf_dijk.shape[0])
        stride = int(leaf_stride or n)
        layout = make_layout(period, sigma_scale, n_sigma, n_sh_fourier)
        src = torch.from_numpy(np.ascontiguousarray(coeffs, dtype=np.float32)).to(device)
        perm_d = torch.from_numpy(perm).to(device)
        recs = torch.empty((stride, layout_record_words(n_sigma, n_sh_fourier), 4), dtype=torch.float32,
                           device=device)
        pack_coeffs(src, perm_d, n, stride, recs, layout)
        del src
        return cls(torch.from_numpy(children).to(device), children.shape[0], max_depth, recs, None,
                   FPO_F32, n, stride, perm, layout, n_upper=upper_rows(children),
                   levels=level_offsets(children, max_depth),
                   bounds=leaf_bounds(leaf_dijk, max_depth) if clip else None)

    def with_store(self, coeffs, scale, dtype: int) -> "DeviceTree":
        return DeviceTree(self.children, self.n_nodes, self.max_depth, coeffs, scale, dtype,
                          self.n_leaves, self.leaf_stride, self.perm, self.layout, self.n_upper,
                          self.grandchildren, self.levels, self.bounds)

    def upper(self) -> int:
        """Nodes with an internal child (computed from the child table once)."""
        if self.n_upper is None:
            self.n_upper = upper_rows(self.children.cpu().numpy())
        return self.n_upper

    def view(self) -> TreeView:
        v = TreeView()
        v.children = self.children.data_ptr()
        v.n_nodes = self.n_nodes
        v.max_depth = self.max_depth
        v.coeffs = None if self.coeffs is None else self.coeffs.data_ptr()
        v.leaf_scale = None if self.scale is None else self.scale.data_ptr()
        v.dtype = self.dtype
        v.n_leaves = self.n_leaves
        v.leaf_stride = self.leaf_stride
        v.layout = self.layout
        if self.grandchildren is not None:
            v.grandchildren = self.grandchildren.data_ptr()
            v.n_grandchild_rows = int(self.grandchildren.shape[-3])
        if self.levels is not None:
            v.level_offsets = self.levels.ctypes.data
        if self.bounds is not None:
            v.bounds = self.bounds.ctypes.data
        return v


def level_offsets(children: np.ndarray, max_depth: int) -> Optional[np.ndarray]:
    """First node of each depth, [max_depth + 1] int64 ending at n_nodes, for a
    child table numbered level by level (fpo_build_tree's order: the internal
    children of depth-L nodes are exactly the next rows, each once); None if
    the table is not numbered so."""
    ch = np.asarray(children)
    n = int(ch.shape[0])
    off = np.zeros(max_depth + 1, dtype=np.int64)
    lo, hi = 0, min(n, 1)                 # depth 0: the root
    for L in range(max_depth):
        off[L] = lo
        kids = ch[lo:hi]
        kids = kids[kids > 0].astype(np.int64)
        if kids.size and (kids.min() != hi or kids.max() != hi + kids.size - 1 or np.unique(kids).size != kids.size):
            return None
        lo, hi = hi, hi + kids.size
    if lo != hi or hi != n:               # no internal node at depth max_depth; every row reached
        return None
    off[max_depth] = n
    return off


def upper_rows(children: np.ndarray) -> int:
    """1 + the last node that has an internal child: with breadth-first
    numbering those nodes are exactly 0 .. n - 1 (a child table of a pruned
    time has no more of them)."""
    has = (np.asarray(children) > 0).any(axis=1)
    return int(np.nonzero(has)[0][-1]) + 1 if has.any() else 0


# ---------------------------------------------------------------------------
# device calls
# ---------------------------------------------------------------------------
def pack_coeffs(src, perm, n_leaves: int, leaf_stride: int, dst, layout: Optional[Layout] = None):
    _check(lib().fpo_pack_coeffs(_t_ptr(src), _t_ptr(perm), int(n_leaves), int(leaf_stride),
                                 None if layout is None else ctypes.byref(layout), _t_ptr(dst), _stream()))


def render(tree: DeviceTree, cams, opts: Optional[RenderOpts] = None, rgb=None, T=None, want_T: bool = False):
    """fpo_render -> (rgb [n][H][W][3], T [n][H][W] or None)."""
    import torch
    opts = opts or make_opts()
    n, H, W = len(cams), int(cams[0].height), int(cams[0].width)
    dev = tree.children.device
    if rgb is None:
        rgb = torch.empty((n, H, W, 3), dtype=torch.float32, device=dev)
    if T is None and want_T:
        T = torch.empty((n, H, W), dtype=torch.float32, device=dev)
    tv = tree.view()
    arr = camera_struct(cams)
    _check(lib().fpo_render(ctypes.byref(tv), arr, n, ctypes.byref(opts), _t_ptr(rgb), _t_ptr(T), _stream()))
    return rgb, T


def render_noalloc(tree: DeviceTree, cams, opts: Optional[RenderOpts] = None, rgb=None, T=None,
                   want_T: bool = False):
    """fpo_render_noalloc: fpo_render with the skip scratch in the library's
    static device array (opts.workspace is ignored)."""
    import torch
    opts = opts or make_opts()
    n, H, W = len(cams), int(cams[0].height), int(cams[0].width)
    dev = tree.children.device
    if rgb is None:
        rgb = torch.empty((n, H, W, 3), dtype=torch.float32, device=dev)
    if T is None and want_T:
        T = torch.empty((n, H, W), dtype=torch.float32, device=dev)
    tv = tree.view()
    arr = camera_struct(cams)
    _check(lib().fpo_render_noalloc(ctypes.byref(tv), arr, n, ctypes.byref(opts), _t_ptr(rgb), _t_ptr(T),
                                    _stream()))
    return rgb, T


def camera_rays(cam_table, cam, py, px, o=None, d=None):
    import torch
    n = int(cam.numel())
    dev = cam.device
    o = o if o is not None else torch.empty((n, 3), dtype=torch.float32, device=dev)
    d = d if d is not None else torch.empty((n, 3), dtype=torch.float32, device=dev)
    _check(lib().fpo_camera_rays(_t_ptr(cam_table), int(cam_table.shape[0]), _t_ptr(cam), _t_ptr(py), _t_ptr(px),
                                 n, _t_ptr(o), _t_ptr(d), _stream()))
    return o, d


def render_rays(tree: DeviceTree, o, d, t_idx, basis, opts: Optional[RenderOpts] = None, rgb=None, T=None,
                want_T: bool = False):
    import torch
    opts = opts or make_opts()
    n = int(o.shape[0])
    dev = o.device
    if rgb is None:
        rgb = torch.empty((n, 3), dtype=torch.float32, device=dev)
    if T is None and want_T:
        T = torch.empty((n,), dtype=torch.float32, device=dev)
    tv = tree.view()
    _check(lib().fpo_render_rays(ctypes.byref(tv), _t_ptr(o), _t_ptr(d), _t_ptr(t_idx), _t_ptr(basis),
                                 int(basis.shape[0]), n, ctypes.byref(opts), _t_ptr(rgb), _t_ptr(T), _stream()))
    return rgb, T


def trace_rays(tree: DeviceTree, o, d, max_visits: int):
    """fpo_trace_rays -> (leaf_ids [n][cap], t01 [n][cap][2], n_visits [n])."""
    import torch
    n = int(o.shape[0])
    dev = o.device
    ids = torch.full((n, max_visits), -1, dtype=torch.int32, device=dev)
    t01 = torch.zeros((n, max_visits, 2), dtype=torch.float32, device=dev)
    nv = torch.zeros((n,), dtype=torch.int32, device=dev)
    tv = tree.view()
    _check(lib().fpo_trace_rays(ctypes.byref(tv), _t_ptr(o), _t_ptr(d), n, int(max_visits), _t_ptr(ids),
                                _t_ptr(t01), _t_ptr(nv), _stream()))
    return ids, t01, nv


def render_backward(tree: DeviceTree, o, d, t_idx, basis, rgb_fwd, grad_rgb, grad_coeffs,
                    opts: Optional[RenderOpts] = None):
    """fpo_render_backward: adds dL/dk into grad_coeffs (F32 leaf records)."""
    opts = opts or make_opts()
    tv = tree.view()
    _check(lib().fpo_render_backward(ctypes.byref(tv), _t_ptr(o), _t_ptr(d), _t_ptr(t_idx), _t_ptr(basis),
                                     int(basis.shape[0]), int(o.shape[0]), ctypes.byref(opts), _t_ptr(rgb_fwd),
                                     _t_ptr(grad_rgb), _t_ptr(grad_coeffs), _stream()))
    return grad_coeffs


def l2_loss(rgb, images, image_idx, py, px, grad_rgb=None, loss=None):
    """fpo_l2_loss -> (grad_rgb [n][3], loss [1])."""
    import torch
    n = int(rgb.shape[0])
    if grad_rgb is None:
        grad_rgb = torch.empty_like(rgb)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=rgb.device)
    _check(lib().fpo_l2_loss(_t_ptr(rgb), _t_ptr(images), int(images.shape[0]), int(images.shape[2]),
                             int(images.shape[1]), _t_ptr(image_idx), _t_ptr(py), _t_ptr(px), n,
                             _t_ptr(grad_rgb), _t_ptr(loss), _stream()))
    return grad_rgb, loss


def adam_step(params, grad, m, v, step: int, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    _check(lib().fpo_adam_step(_t_ptr(params), _t_ptr(grad), _t_ptr(m), _t_ptr(v), int(params.numel()),
                               float(lr), float(beta1), float(beta2), float(eps), int(step), _stream()))


def adam_step_dev(params, grad, m, v, state, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8):
    """fpo_adam_step_dev: the step count in `state` (device int32[4], zeroed
    before the first step) advances by one per call or graph replay."""
    _check(lib().fpo_adam_step_dev(_t_ptr(params), _t_ptr(grad), _t_ptr(m), _t_ptr(v), int(params.numel()),
                                   float(lr), float(beta1), float(beta2), float(eps), _t_ptr(state), _stream()))


def adam_step_touched(params, grad, m, v, step: int = 0, lr: float = 1e-2, beta1: float = 0.9,
                      beta2: float = 0.999, eps: float = 1e-8, record_floats: int = 4 * RECORD_WORDS[FPO_F32],
                      state=None):
    """fpo_adam_step_touched over records of `record_floats` floats: records
    with an all-zero gradient are left untouched (lazy Adam)."""
    n = int(params.numel())
    if n % record_floats:
        raise ValueError("params is not a whole number of records")
    _check(lib().fpo_adam_step_touched(_t_ptr(params), _t_ptr(grad), _t_ptr(m), _t_ptr(v), n // record_floats,
                                       int(record_floats), float(lr), float(beta1), float(beta2), float(eps),
                                       int(step), _t_ptr(state), _stream()))


def quantize(tree: DeviceTree, dtype: int) -> DeviceTree:
    """fpo_quantize: a BF16 / FP8 copy of an F32 tree (same structure)."""
    import torch
    if tree.dtype != FPO_F32:
        raise ValueError("quantize needs an F32 tree")
    dev = tree.coeffs.device
    lay = tree.layout
    q = torch.zeros((tree.leaf_stride, layout_record_words(lay.n_sigma, lay.n_sh_fourier, dtype), 4),
                    dtype=torch.int32, device=dev)
    scale = torch.empty((tree.leaf_stride,), dtype=torch.float32, device=dev)
    _check(lib().fpo_quantize(_t_ptr(tree.coeffs), tree.n_leaves, tree.leaf_stride, ctypes.byref(lay), int(dtype),
                              _t_ptr(q), _t_ptr(scale), _stream()))
    return tree.with_store(q, scale, dtype)


def bake_times(tree: DeviceTree, basis, out_dtype: int = FPO_F32, out=None, sigma_out=None):
    """fpo_bake_times -> out [n_t][leaf_stride][32] snapshot records (float32 or
    bfloat16).  sigma_out: None, or a float32 [n_t][leaf_stride] tensor that
    receives value 0 of every record as FP32 (the density plane)."""
    import torch
    n_t = int(basis.shape[0])
    if out is None:
        dt = torch.float32 if out_dtype == FPO_F32 else torch.bfloat16
        out = torch.empty((n_t, tree.leaf_stride, SNAP_VALUES), dtype=dt, device=basis.device)
    if sigma_out is not None and (sigma_out.dtype != torch.float32 or tuple(sigma_out.shape) != (n_t, tree.leaf_stride)
                                  or not sigma_out.is_contiguous()):
        raise ValueError("sigma_out must be a contiguous float32 [n_t][leaf_stride] tensor")
    tv = tree.view()
    _check(lib().fpo_bake_times(ctypes.byref(tv), _t_ptr(basis), n_t, int(out_dtype), _t_ptr(out),
                                None if sigma_out is None else _t_ptr(sigma_out), _stream()))
    return out


# ---------------------------------------------------------------------------
# learned proposal
# ---------------------------------------------------------------------------
MLP_N_IN = 7
FPO_RENDER_SKIP_COARSE = 1
FPO_RENDER_SKIP_PROPOSAL = 2
FPO_RAYS_RECORD = 4
RECORD_BYTES = 32
MLP_N_PARAMS = 9795
MLP_N_PARAMS_PADDED = 9796
MLP_PACKED_BYTES = 23056
COARSE_WORDS = 8192


def coarse_occupancy(leaf_dijk: np.ndarray, max_depth: int) -> np.ndarray:
    """fpo_coarse_occupancy -> uint32 [8192] (host)."""
    dijk = np.ascontiguousarray(leaf_dijk, dtype=np.int32)
    bits = np.zeros(COARSE_WORDS, np.uint32)
    _check(lib().fpo_coarse_occupancy(_np_ptr(dijk), int(dijk.shape[0]), int(max_depth), _np_ptr(bits)))
    return bits


def ray_labels(tree: DeviceTree, o, d, t_idx, basis, tau, opts: Optional[RenderOpts] = None):
    """fpo_ray_labels -> (labels [n][3], inputs [n][7])."""
    import torch
    opts = opts or make_opts()
    n = int(o.shape[0])
    labels = torch.empty((n, 3), dtype=torch.float32, device=o.device)
    inputs = torch.empty((n, MLP_N_IN), dtype=torch.float32, device=o.device)
    tv = tree.view()
    _check(lib().fpo_ray_labels(ctypes.byref(tv), _t_ptr(o), _t_ptr(d), _t_ptr(t_idx), _t_ptr(basis), _t_ptr(tau),
                                int(basis.shape[0]), n, ctypes.byref(opts), _t_ptr(labels), _t_ptr(inputs),
                                _stream()))
    return labels, inputs


def mlp_forward(params, inputs, out=None):
    import torch
    n = int(inputs.shape[0])
    out = out if out is not None else torch.empty((n, 3), dtype=torch.float32, device=inputs.device)
    _check(lib().fpo_mlp_forward(_t_ptr(params), _t_ptr(inputs), n, _t_ptr(out), _stream()))
    return out


def mlp_workspace(n: int, device):
    import torch
    return torch.empty((int(lib().fpo_mlp_workspace_floats(int(n))),), dtype=torch.float32, device=device)


def mlp_loss_grad(params, inputs, labels, grad, loss, workspace, idx=None, n: Optional[int] = None):
    """fpo_mlp_loss_grad: adds the batch gradient into grad and the loss into loss[0]."""
    n = int(idx.numel()) if idx is not None else (int(n) if n is not None else int(inputs.shape[0]))
    _check(lib().fpo_mlp_loss_grad(_t_ptr(params), _t_ptr(inputs), _t_ptr(labels), _t_ptr(idx), n,
                                   _t_ptr(workspace), _t_ptr(grad), _t_ptr(loss), _stream()))


def mlp_pack(params, out=None):
    import torch
    out = out if out is not None else torch.empty((MLP_PACKED_BYTES,), dtype=torch.uint8, device=params.device)
    _check(lib().fpo_mlp_pack(_t_ptr(params), _t_ptr(out), _stream()))
    return out


def mlp_infer(packed, inputs, out=None):
    import torch
    n = int(inputs.shape[0])
    out = out if out is not None else torch.empty((n, 3), dtype=torch.float32, device=inputs.device)
    _check(lib().fpo_mlp_infer(_t_ptr(packed), _t_ptr(inputs), n, _t_ptr(out), _stream()))
    return out


# ---------------------------------------------------------------------------
# building an FPO from per-frame octrees
# ---------------------------------------------------------------------------
MAX_FRAMES = 120
PRUNE_SIGMA = 1e-3


def union_leaves(cells: np.ndarray, max_depth: int) -> np.ndarray:
    """fpo_union_leaves -> [n_union][4] int32 (Morton order)."""
    c = np.ascontiguousarray(cells, dtype=np.int32)
    n = ctypes.c_int64(0)
    _check(lib().fpo_union_leaves(_np_ptr(c), int(c.shape[0]), int(max_depth), None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, 4), dtype=np.int32)
    _check(lib().fpo_union_leaves(_np_ptr(c), int(c.shape[0]), int(max_depth), _np_ptr(out), n.value,
                                  ctypes.byref(n)))
    return out


class FrameTree:
    """Structure of one frame's octree on the device (no coefficients)."""

    def __init__(self, leaf_dijk: np.ndarray, max_depth: int, device):
        import torch
        children, perm = build_tree(leaf_dijk, max_depth)
        self.children = torch.from_numpy(children).to(device)
        self.perm = torch.from_numpy(perm).to(device)
        self.n_nodes = children.shape[0]
        self.n_leaves = int(leaf_dijk.shape[0])
        self.max_depth = int(max_depth)

    def view(self) -> TreeView:
        v = TreeView()
        v.children = self.children.data_ptr()
        v.n_nodes = self.n_nodes
        v.max_depth = self.max_depth
        v.n_leaves = self.n_leaves
        v.leaf_stride = self.n_leaves
        v.layout = make_layout()
        return v


def frame_values(frame: FrameTree, values, union_cells_slot, out, n_bad):
    """fpo_frame_values: values [n_f][32] (caller order) onto the union slots."""
    tv = frame.view()
    _check(lib().fpo_frame_values(ctypes.byref(tv), _t_ptr(frame.perm), _t_ptr(values), _t_ptr(union_cells_slot),
                                  int(union_cells_slot.shape[0]), _t_ptr(out), _t_ptr(n_bad), _stream()))


def dft_frames(frames, n_leaves: int, literal: bool = False, coeffs=None, sigma_max=None):
    """fpo_dft_frames: frames [T][stride][32] -> (F32 records [stride][48][4], sigma_max [stride])."""
    import torch
    T, stride = int(frames.shape[0]), int(frames.shape[1])
    if coeffs is None:
        coeffs = torch.zeros((stride, record_words(FPO_F32), 4), dtype=torch.float32, device=frames.device)
    if sigma_max is None:
        sigma_max = torch.zeros((stride,), dtype=torch.float32, device=frames.device)
    _check(lib().fpo_dft_frames(_t_ptr(frames), T, int(n_leaves), stride, 1 if literal else 0, _t_ptr(coeffs),
                                _t_ptr(sigma_max), _stream()))
    return coeffs, sigma_max


def prune_leaves(sigma_max: np.ndarray, threshold: float = PRUNE_SIGMA) -> np.ndarray:
    sm = np.ascontiguousarray(sigma_max, dtype=np.float32)
    keep = np.zeros(sm.shape[0], dtype=np.int64)
    n = ctypes.c_int64(0)
    _check(lib().fpo_prune_leaves(_np_ptr(sm), int(sm.shape[0]), float(threshold), _np_ptr(keep), ctypes.byref(n)))
    return keep[:n.value]


# ---------------------------------------------------------------------------
# PlenOctree fusion
# ---------------------------------------------------------------------------
def field_struct(field) -> FieldC:
    """fpo_field from an object with mu [G][3], w [G], a [G], u, v [3][3], b [3]."""
    f = FieldC()
    n = len(field.w)
    if n > FIELD_MAX_GAUSS:
        raise ValueError(f"at most {FIELD_MAX_GAUSS} Gaussians")
    for g in range(n):
        for c in range(3):
            f.mu[g][c] = float(field.mu[g][c])
        f.w[g] = float(field.w[g])
        f.a[g] = float(field.a[g])
    f.n_gauss = n
    for c in range(3):
        for k in range(3):
            f.u[c][k] = float(field.u[c][k])
            f.v[c][k] = float(field.v[c][k])
        f.b[c] = float(field.b[c])
    return f


def fusion_observe(tree: DeviceTree, values, cam, field, acc, tau: float = 1e-3):
    """fpo_fusion_observe: values [leaf_stride][32] F32 (slot order), acc
    [leaf_stride][32] F32 (added to)."""
    tv = tree.view()
    cs = camera_struct([cam])
    fs = field_struct(field) if not isinstance(field, FieldC) else field
    _check(lib().fpo_fusion_observe(ctypes.byref(tv), _t_ptr(values), cs, ctypes.byref(fs), float(tau),
                                    _t_ptr(acc), _stream()))


def fusion_apply(values, weight, count, acc, n_leaves: int):
    """fpo_fusion_apply over the first n_leaves slots."""
    _check(lib().fpo_fusion_apply(_t_ptr(values), _t_ptr(weight), _t_ptr(count), _t_ptr(acc), int(n_leaves),
                                  _stream()))


# ---------------------------------------------------------------------------
# occupancy at one time
# ---------------------------------------------------------------------------
def prune_at(tree: DeviceTree, snapshots, snapshot_dtype: int = FPO_F32, out=None):
    """fpo_prune_at: per-time child tables [n_t][n_nodes][8] from snapshots
    [n_t][leaf_stride][32] (or one [leaf_stride][32])."""
    import torch
    snaps = snapshots if snapshots.dim() == 3 else snapshots[None]
    n_t = int(snaps.shape[0])
    if out is None:
        out = torch.empty((n_t, tree.n_nodes, 8), dtype=torch.int32, device=snaps.device)
    tv = tree.view()
    _check(lib().fpo_prune_at(ctypes.byref(tv), _t_ptr(snaps), int(snapshot_dtype), int(snaps.shape[1]), n_t,
                              _t_ptr(out), _stream()))
    return out


def prune_at_sigma(tree: DeviceTree, sigma, out=None):
    """fpo_prune_at_sigma: per-time child tables [n_t][n_nodes][8] from a
    density plane [n_t][stride] float32 (bake_times sigma_out)."""
    import torch
    sg = sigma if sigma.dim() == 2 else sigma[None]
    n_t = int(sg.shape[0])
    if out is None:
        out = torch.empty((n_t, tree.n_nodes, 8), dtype=torch.int32, device=sg.device)
    tv = tree.view()
    _check(lib().fpo_prune_at_sigma(ctypes.byref(tv), _t_ptr(sg), int(sg.shape[1]), n_t, _t_ptr(out), _stream()))
    return out


def tree_with_children(tree: DeviceTree, children, grandchildren=None) -> "DeviceTree":
    """The same tree (coefficients, leaves) walked through another child table
    of the same shape, e.g. one time of prune_at's output, and optionally that
    table's two-level table (one time of grandchild_tables' output)."""
    if tuple(children.shape) != (tree.n_nodes, 8):
        raise ValueError("child table shape differs")
    if grandchildren is not None and (grandchildren.dim() != 3 or tuple(grandchildren.shape[1:]) != (64, 2)):
        raise ValueError("grandchildren must be [rows][64][2]")
    return DeviceTree(children, tree.n_nodes, tree.max_depth, tree.coeffs, tree.scale, tree.dtype, tree.n_leaves,
                      tree.leaf_stride, tree.perm, tree.layout, tree.n_upper, grandchildren, tree.levels,
                      tree.bounds)


def grandchild_tables(tree: DeviceTree, children=None, n_rows: Optional[int] = None, out=None):
    """fpo_grandchild_tables of `children` ([n_t][n_nodes][8], default: the
    tree's own table) over its first n_rows nodes (default: the nodes with an
    internal child) -> [n_t][n_rows][64][2] int32."""
    import torch
    ch = tree.children if children is None else children
    ch3 = ch if ch.dim() == 3 else ch[None]
    n_t = int(ch3.shape[0])
    rows = int(n_rows if n_rows is not None else tree.upper())
    if rows < 1:
        raise ValueError("no node has an internal child")
    if out is None:
        out = torch.empty((n_t, rows, 64, 2), dtype=torch.int32, device=ch3.device)
    _check(lib().fpo_grandchild_tables(_t_ptr(ch3), tree.n_nodes, n_t, rows, _t_ptr(out), _stream()))
    return out


def leaf_cells_slot_order(leaf_dijk: np.ndarray, perm: np.ndarray, device):
    """(depth, i, j, k) of every leaf slot, as fpo_coarse_occupancy_at takes them."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(leaf_dijk, np.int32)[perm])).to(device)


def coarse_occupancy_at(leaf_cells, max_depth: int, snapshot, snapshot_dtype: int = FPO_F32,
                        sigma_scale: float = 64.0, out=None):
    import torch
    if out is None:
        out = torch.empty((8192,), dtype=torch.int32, device=snapshot.device)
    _check(lib().fpo_coarse_occupancy_at(_t_ptr(leaf_cells), int(leaf_cells.shape[0]), int(max_depth),
                                         _t_ptr(snapshot), int(snapshot_dtype), float(sigma_scale), _t_ptr(out),
                                         _stream()))
    return out
