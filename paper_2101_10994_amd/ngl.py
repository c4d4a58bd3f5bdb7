"""Python binding of libngl.so (the gfx950 neural geometric LOD library).

Argument marshalling only: every step of the path runs in the library's
HIP kernels; PyTorch provides device memory and the current stream.  The
names mirror the C ABI in include/ngl.h.  There is no fallback: if the
library is not built, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libngl.so")

MAX_LODS = 8
MAX_DEPTH = MAX_LODS + 2
F32, F16, BF16 = 0, 1, 2
MISS, HIT, MAX_STEPS, FAR, STALLED, INVALID = range(6)

_TORCH_DTYPE = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}
_DTYPE_CODE = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}

_lock = threading.Lock()
_lib = None

P = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64


class NGLError(RuntimeError):
    pass


class ngl_model(C.Structure):
    _fields_ = [("num_lods", i32), ("feat_dim", i32), ("hidden", i32), ("with_xyz", i32),
                ("feat_dtype", i32), ("w_dtype", i32),
                ("nvox", i64 * MAX_DEPTH), ("ncorner", i64 * MAX_LODS),
                ("cell", P * MAX_DEPTH), ("child_mask", P * MAX_DEPTH), ("first_child", P * MAX_DEPTH),
                ("parent", P * MAX_DEPTH), ("corners", P * MAX_LODS), ("feat", P * MAX_LODS),
                ("W1", P * MAX_LODS), ("b1", P * MAX_LODS), ("w2", P * MAX_LODS), ("b2", P),
                ("corner_adj_off", P * MAX_LODS), ("corner_adj", P * MAX_LODS), ("W1_packed", P * MAX_LODS)]


class ngl_octree_host(C.Structure):
    _fields_ = [("cell", P * MAX_DEPTH), ("child_mask", P * MAX_DEPTH), ("first_child", P * MAX_DEPTH),
                ("parent", P * MAX_DEPTH), ("corners", P * MAX_LODS), ("corner_cell", P * MAX_LODS),
                ("corner_adj_off", P * MAX_LODS), ("corner_adj", P * MAX_LODS)]


class ngl_view(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3), ("fov_y_deg", C.c_float),
                ("width", i32), ("height", i32), ("lod", i32), ("alpha", C.c_float)]


class ngl_trace_params(C.Structure):
    _fields_ = [("max_steps", i32), ("delta", C.c_float), ("t_far", C.c_float), ("osc_check", i32),
                ("analytic", i32), ("sphere", C.c_float * 4), ("image_width", i32)]


class ngl_shape(C.Structure):
    _fields_ = [("n_spheres", i32), ("n_tori", i32), ("spheres", P), ("tori", P)]


class ngl_adam_params(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("step", i32)]


class ngl_lod_select(C.Structure):
    _fields_ = [("d_near", C.c_float), ("d_far", C.c_float), ("lod_near", C.c_float), ("lod_far", C.c_float)]


EXPORTS = {
    "ngl_status_str": (C.c_char_p, [C.c_int]),
    "ngl_last_error": (C.c_char_p, []),
    "ngl_version": (C.c_int, []),
    "ngl_set_option": (C.c_int, [C.c_int, C.c_int]),
    "ngl_get_option": (C.c_int, [C.c_int, P]),
    "ngl_octree_plan": (C.c_int, [P, i64, i32, P, P]),
    "ngl_octree_fill": (C.c_int, [P, i64, i32, P]),
    "ngl_octree_build_device_workspace": (C.c_int, [i64, i32, P]),
    "ngl_octree_build_device": (C.c_int, [P, i64, i32, P, P, C.c_size_t, P]),
    "ngl_query_sdf": (C.c_int, [P, P, i64, i32, C.c_float, P, P, P, P, P]),
    "ngl_query_sdf_all_lods": (C.c_int, [P, P, i64, P, P]),
    "ngl_decode_sdf": (C.c_int, [P, i32, P, P, i32, i64, P, P]),
    "ngl_sdf_normals": (C.c_int, [P, P, P, P, P, P, i64, i32, C.c_float, C.c_float, P, P]),
    "ngl_camera_rays": (C.c_int, [P, P, P, C.c_float, i32, i32, P, P, P]),
    "ngl_trace_octree_workspace": (C.c_int, [i64, i64, P]),
    "ngl_trace_octree": (C.c_int, [P, P, P, i64, i32, i64, P, C.c_size_t, P, P, P, P, P, P, P]),
    "ngl_sphere_trace": (C.c_int, [P, P, P, i64, i32, C.c_float, P, P, P, P, P, P, P, P, P, P, C.c_size_t, P]),
    "ngl_sphere_trace_workspace": (C.c_int, [P]),
    "ngl_sphere_trace_workspace_rays": (C.c_int, [C.c_int64, P]),
    "ngl_sphere_trace_lod_workspace": (C.c_int, [i64, P]),
    "ngl_sphere_trace_lod": (C.c_int, [P, P, P, i64, i32, P, P, P, P, P, P, P, P, P, P, P, P, C.c_size_t, P]),
    "ngl_model_table_bytes": (C.c_int, [i32, P]),
    "ngl_model_table_upload": (C.c_int, [P, i32, P, P]),
    "ngl_render_batch_workspace": (C.c_int, [P, i32, i64, P]),
    "ngl_render_batch": (C.c_int, [P, P, P, i32, P, i64, P, C.c_size_t, P, P, P, P, P, P, P]),
    "ngl_train_workspace": (C.c_int, [P, i64, P]),
    "ngl_backward_all_lods": (C.c_int, [P, P, i64, P, P, P, P, P, P, P, C.c_size_t, P]),
    "ngl_train_fwd_bwd": (C.c_int, [P, P, P, i64, P, P, P, P, P, P, P, P, C.c_size_t, P]),
    "ngl_train_fwd_bwd_lods": (C.c_int, [P, P, P, i64, P, P, P, P, P, P, P, P, P, C.c_size_t, P]),
    "ngl_shape_sdf": (C.c_int, [P, P, i64, P, P]),
    "ngl_sample_surface_workspace": (C.c_int, [i64, P]),
    "ngl_sample_surface": (C.c_int, [P, P, i64, i32, C.c_float, P, P, P, C.c_size_t, P]),
    "ngl_training_points": (C.c_int, [P, P, i64, i64, P, i64, i64, C.c_float, P, P, P]),
    "ngl_adam_step": (C.c_int, [P, i32, P, P, P, P, P, P]),
    "ngl_packed_decoder_bytes": (C.c_int, [P, P]),
    "ngl_pack_decoders": (C.c_int, [P, P, C.c_size_t, P]),
    "ngl_workspace_bytes": (C.c_int, [C.c_int, P, i64, i64, P]),
    "ngl_sphere_trace_static": (C.c_int, [P, P, P, i64, i32, C.c_float, P, P, P, P, P, P, P, P, P, P]),
}

# ngl_workspace_bytes operations
(OP_TRACE_OCTREE, OP_SPHERE_TRACE, OP_SPHERE_TRACE_LOD, OP_TRAIN, OP_SAMPLE_SURFACE, OP_OCTREE_BUILD_DEVICE,
 OP_PACK_DECODERS) = range(7)


def workspace_bytes(op: int, model=None, n: int = 0, aux: int = 0) -> int:
    """Device bytes the call `op` needs (ngl_workspace_bytes)."""
    b = C.c_size_t()
    _check(lib().ngl_workspace_bytes(int(op), model.ref if model is not None else None, int(n), int(aux),
                                     C.addressof(b)))
    return int(b.value)


def lib():
    """Load libngl.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise NGLError("libngl.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2101_10994_amd.build)")
            h = C.CDLL(LIB_PATH)
            for name, (res, args) in EXPORTS.items():
                f = getattr(h, name)
                f.restype = res
                f.argtypes = args
            _lib = h
    return _lib


(OPT_F32_DECODER, OPT_TRACE_WAVES, OPT_TRACE_BLOCKS_PER_CU, OPT_TRACE_PAUSE1, OPT_TRACE_PAUSE2,
 OPT_TRACE_WIDE, OPT_COOP_GATHER, OPT_QUERY_BLOCKS_PER_CU) = 0, 1, 2, 3, 4, 5, 6, 7
MAX_BATCH = 32


def set_option(key: int, value: int):
    """Library option (see ngl_set_option): OPT_F32_DECODER 0 = VALU, 1 = matrix cores."""
    _check(lib().ngl_set_option(int(key), int(value)))


def get_option(key: int) -> int:
    v = C.c_int()
    _check(lib().ngl_get_option(int(key), C.addressof(v)))
    return int(v.value)


def _check(rc: int):
    if rc != 0:
        L = lib()
        raise NGLError("%s: %s" % (L.ngl_status_str(rc).decode(), L.ngl_last_error().decode()))


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype=None):
    if not t.is_cuda:
        raise NGLError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise NGLError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise NGLError("expected a contiguous tensor")
    return t


# ---------------------------------------------------------------------------
# 1. Octree
# ---------------------------------------------------------------------------
class Octree:
    """Canonical sparse voxel octree: host arrays from ngl_octree_fill and
    their device copies."""

    def __init__(self, ijk: np.ndarray, num_lods: int, device="cuda"):
        L = lib()
        ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
        self.num_lods = int(num_lods)
        self.depth = self.num_lods + 1
        nv = np.zeros(MAX_DEPTH, np.int64)
        nc = np.zeros(MAX_LODS, np.int64)
        _check(L.ngl_octree_plan(_ptr(ijk), ijk.shape[0], self.num_lods, _ptr(nv), _ptr(nc)))
        self.nvox = nv[: self.depth + 1].copy()
        self.ncorner = nc[: self.num_lods].copy()
        D = self.depth
        self.cell = [np.zeros(int(self.nvox[d]), np.uint32) for d in range(D + 1)]
        self.child_mask = [np.zeros(int(self.nvox[d]), np.uint8) for d in range(D + 1)]
        self.first_child = [np.zeros(int(self.nvox[d]), np.int32) for d in range(D + 1)]
        self.parent = [np.zeros(int(self.nvox[d]), np.int32) for d in range(D + 1)]
        self.corners = [np.zeros((int(self.nvox[lv + 1]), 8), np.int32) for lv in range(1, D)]
        self.corner_cell = [np.zeros((int(self.ncorner[lv - 1]), 3), np.int32) for lv in range(1, D)]
        self.corner_adj_off = [np.zeros(int(self.ncorner[lv - 1]) + 1, np.int32) for lv in range(1, D)]
        self.corner_adj = [np.zeros(8 * int(self.nvox[lv + 1]), np.int32) for lv in range(1, D)]
        h = ngl_octree_host()
        for d in range(D + 1):
            h.cell[d] = _ptr(self.cell[d])
            h.child_mask[d] = _ptr(self.child_mask[d])
            h.first_child[d] = _ptr(self.first_child[d])
            h.parent[d] = _ptr(self.parent[d])
        for lv in range(self.num_lods):
            h.corners[lv] = _ptr(self.corners[lv])
            h.corner_cell[lv] = _ptr(self.corner_cell[lv])
            h.corner_adj_off[lv] = _ptr(self.corner_adj_off[lv])
            h.corner_adj[lv] = _ptr(self.corner_adj[lv])
        _check(L.ngl_octree_fill(_ptr(ijk), ijk.shape[0], self.num_lods, C.addressof(h)))
        self.device = device
        self.d_cell = self.d_child_mask = self.d_first_child = self.d_parent = self.d_corners = None
        if device is not None:
            self.to(device)

    def to(self, device):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.d_cell = [t(a.view(np.int32)) for a in self.cell]
        self.d_child_mask = [t(a) for a in self.child_mask]
        self.d_first_child = [t(a) for a in self.first_child]
        self.d_parent = [t(a) for a in self.parent]
        self.d_corners = [t(a) for a in self.corners]
        self.d_corner_adj_off = [t(a) for a in self.corner_adj_off]
        self.d_corner_adj = [t(a) for a in self.corner_adj]
        self.device = device
        return self

    def cell_ijk(self, d: int) -> np.ndarray:
        c = self.cell[d].astype(np.int64)
        return np.stack([c & 1023, (c >> 10) & 1023, (c >> 20) & 1023], 1).astype(np.int32)

    def corner_positions(self) -> List[np.ndarray]:
        return [-1.0 + self.corner_cell[lv].astype(np.float64) * (2.0 / 2 ** (lv + 2))
                for lv in range(self.num_lods)]


class ngl_octree_device(C.Structure):
    _fields_ = [("cell", P * MAX_DEPTH), ("child_mask", P * MAX_DEPTH), ("first_child", P * MAX_DEPTH),
                ("parent", P * MAX_DEPTH), ("corners", P * MAX_LODS), ("corner_cell", P * MAX_LODS),
                ("corner_adj_off", P * MAX_LODS), ("corner_adj", P * MAX_LODS), ("nvox", P), ("ncorner", P),
                ("bad", P)]


class DeviceOctree:
    """The canonical octree built on the device (ngl_octree_build_device),
    with the attributes a Model reads; device arrays are trimmed views of
    upper-bound allocations (one synchronisation reads the sizes)."""

    def __init__(self, ijk: torch.Tensor, num_lods: int):
        if ijk.dtype != torch.int32 or not ijk.is_cuda:
            raise NGLError("ijk must be an int32 device tensor [n][3]")
        ijk = ijk.reshape(-1, 3).contiguous()
        n = ijk.shape[0]
        dev = ijk.device
        self.num_lods = L = int(num_lods)
        self.depth = D = L + 1
        nb = C.c_size_t()
        _check(lib().ngl_octree_build_device_workspace(n, L, C.addressof(nb)))
        ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=dev)
        cap = [max(1, min(n, 8 ** d)) for d in range(D + 1)]
        e32 = lambda k: torch.empty(k, dtype=torch.int32, device=dev)
        self.d_cell = [e32(cap[d]) for d in range(D + 1)]
        self.d_child_mask = [torch.empty(cap[d], dtype=torch.uint8, device=dev) for d in range(D + 1)]
        self.d_first_child = [e32(cap[d]) for d in range(D + 1)]
        self.d_parent = [e32(cap[d]) for d in range(D + 1)]
        self.d_corners = [e32(8 * cap[lv + 1]) for lv in range(1, D)]
        self.d_corner_cell = [e32(3 * 8 * cap[lv + 1]) for lv in range(1, D)]
        self.d_corner_adj_off = [e32(8 * cap[lv + 1] + 1) for lv in range(1, D)]
        self.d_corner_adj = [e32(8 * cap[lv + 1]) for lv in range(1, D)]
        counts = torch.zeros(MAX_DEPTH + MAX_LODS + 1, dtype=torch.int64, device=dev)
        o = ngl_octree_device()
        for d in range(D + 1):
            o.cell[d], o.child_mask[d] = _ptr(self.d_cell[d]), _ptr(self.d_child_mask[d])
            o.first_child[d], o.parent[d] = _ptr(self.d_first_child[d]), _ptr(self.d_parent[d])
        for lv in range(L):
            o.corners[lv], o.corner_cell[lv] = _ptr(self.d_corners[lv]), _ptr(self.d_corner_cell[lv])
            o.corner_adj_off[lv], o.corner_adj[lv] = _ptr(self.d_corner_adj_off[lv]), _ptr(self.d_corner_adj[lv])
        base = counts.data_ptr()
        o.nvox, o.ncorner, o.bad = base, base + 8 * MAX_DEPTH, base + 8 * (MAX_DEPTH + MAX_LODS)
        self._keep = (ijk, ws, counts, o)
        self.rebuild()
        c = counts.cpu().numpy()
        if c[MAX_DEPTH + MAX_LODS] > 0:
            raise NGLError("%d cells outside [0, %d)^3" % (int(c[MAX_DEPTH + MAX_LODS]), 1 << D))
        self.nvox = c[: D + 1].copy()
        self.ncorner = c[MAX_DEPTH: MAX_DEPTH + L].copy()
        nv, nc = self.nvox, self.ncorner
        self.d_cell = [t[: int(nv[d])] for d, t in enumerate(self.d_cell)]
        self.d_child_mask = [t[: int(nv[d])] for d, t in enumerate(self.d_child_mask)]
        self.d_first_child = [t[: int(nv[d])] for d, t in enumerate(self.d_first_child)]
        self.d_parent = [t[: int(nv[d])] for d, t in enumerate(self.d_parent)]
        self.d_corners = [t[: 8 * int(nv[lv + 2])].view(-1, 8) for lv, t in enumerate(self.d_corners)]
        self.d_corner_cell = [t[: 3 * int(nc[lv])].view(-1, 3) for lv, t in enumerate(self.d_corner_cell)]
        self.d_corner_adj_off = [t[: int(nc[lv]) + 1] for lv, t in enumerate(self.d_corner_adj_off)]
        self.d_corner_adj = [t[: 8 * int(nv[lv + 2])] for lv, t in enumerate(self.d_corner_adj)]
        self.device = dev

    def rebuild(self):
        """Enqueue the build again into the same buffers (no allocation, no
        synchronisation): for timing."""
        ijk, ws, counts, o = self._keep
        _check(lib().ngl_octree_build_device(_ptr(ijk), ijk.shape[0], self.num_lods, C.addressof(o), _ptr(ws),
                                             ws.numel(), _stream()))

    def corner_positions(self) -> List[np.ndarray]:
        return [-1.0 + self.d_corner_cell[lv].cpu().numpy().astype(np.float64) * (2.0 / 2 ** (lv + 2))
                for lv in range(self.num_lods)]


# ---------------------------------------------------------------------------
# Model
# ---------------------------------------------------------------------------
class Model:
    """Octree + corner features + per-LOD decoders as device tensors.

    feats[l]: [ncorner_l][m] (float32/float16/bfloat16); W1[l]: [h][din]
    (float32 or bfloat16); b1[l], w2[l]: [h] float32; b2: [L] float32."""

    def __init__(self, tree: Octree, feats: Sequence[torch.Tensor], W1: Sequence[torch.Tensor],
                 b1: Sequence[torch.Tensor], w2: Sequence[torch.Tensor], b2: torch.Tensor, with_xyz: bool = True,
                 pack: bool = False):
        self.tree = tree
        self._packed = None
        self.num_lods = tree.num_lods
        assert len(feats) == self.num_lods and len(W1) == self.num_lods
        self.feats = [_dev(f) for f in feats]
        self.W1 = [_dev(w) for w in W1]
        self.b1 = [_dev(b, torch.float32) for b in b1]
        self.w2 = [_dev(w, torch.float32) for w in w2]
        self.b2 = _dev(b2, torch.float32)
        self.m = int(self.feats[0].shape[1])
        self.hidden = int(self.W1[0].shape[0])
        self.with_xyz = bool(with_xyz)
        self.feat_dtype = _DTYPE_CODE[self.feats[0].dtype]
        self.w_dtype = _DTYPE_CODE[self.W1[0].dtype]
        din = self.m + (3 if self.with_xyz else 0)
        for lv in range(self.num_lods):
            nc = int(tree.ncorner[lv])
            f = self.feats[lv]
            if tuple(f.shape) != (nc, self.m) and not (nc == 0 and f.shape[1] == self.m):
                raise NGLError("feats[%d] has shape %s, expected (%d, %d)" % (lv, tuple(f.shape), nc, self.m))
            if _DTYPE_CODE[f.dtype] != self.feat_dtype:
                raise NGLError("all feature levels must share one dtype")
            if tuple(self.W1[lv].shape) != (self.hidden, din) or _DTYPE_CODE[self.W1[lv].dtype] != self.w_dtype:
                raise NGLError("W1[%d] must be [%d][%d] of one dtype" % (lv, self.hidden, din))
            if tuple(self.b1[lv].shape) != (self.hidden,) or tuple(self.w2[lv].shape) != (self.hidden,):
                raise NGLError("b1[%d]/w2[%d] must have %d entries" % (lv, lv, self.hidden))
        if tuple(self.b2.shape) != (self.num_lods,):
            raise NGLError("b2 must have num_lods entries")
        self._struct = self._make_struct()
        if pack:
            self.pack()

    def pack(self):
        """Pre-pack the decoders' first layers in matrix-core fragment order
        (ngl_pack_decoders); kernels then copy them instead of rebuilding
        them per block.  Call again after W1 or b1 change (refresh() does)."""
        nb = C.c_size_t()
        _check(lib().ngl_packed_decoder_bytes(self.ref, C.addressof(nb)))
        if self._packed is None or self._packed.numel() < nb.value:
            self._packed = torch.empty(int(nb.value), dtype=torch.uint8, device=self.b2.device)
        _check(lib().ngl_pack_decoders(self.ref, _ptr(self._packed), int(nb.value), _stream()))

    def unpack(self):
        """Drop the packed decoders (kernels build fragments from W1, b1)."""
        self._packed = None
        for lv in range(MAX_LODS):
            self._struct.W1_packed[lv] = None

    @property
    def packed(self) -> bool:
        return self._packed is not None

    def _make_struct(self):
        s = ngl_model()
        t = self.tree
        s.num_lods, s.feat_dim, s.hidden, s.with_xyz = self.num_lods, self.m, self.hidden, int(self.with_xyz)
        s.feat_dtype, s.w_dtype = self.feat_dtype, self.w_dtype
        for d in range(t.depth + 1):
            s.nvox[d] = int(t.nvox[d])
            s.cell[d] = _ptr(t.d_cell[d]) if t.nvox[d] else None
            s.child_mask[d] = _ptr(t.d_child_mask[d]) if t.nvox[d] else None
            s.first_child[d] = _ptr(t.d_first_child[d]) if t.nvox[d] else None
            s.parent[d] = _ptr(t.d_parent[d]) if t.nvox[d] else None
        for lv in range(self.num_lods):
            s.ncorner[lv] = int(t.ncorner[lv])
            s.corners[lv] = _ptr(t.d_corners[lv]) if t.nvox[lv + 2] else None
            s.feat[lv] = _ptr(self.feats[lv]) if self.feats[lv].numel() else None
            s.W1[lv] = _ptr(self.W1[lv])
            s.b1[lv] = _ptr(self.b1[lv])
            s.w2[lv] = _ptr(self.w2[lv])
            s.corner_adj_off[lv] = _ptr(t.d_corner_adj_off[lv])
            s.corner_adj[lv] = _ptr(t.d_corner_adj[lv]) if t.nvox[lv + 2] else None
        s.b2 = _ptr(self.b2)
        return s

    @property
    def ref(self):
        return C.addressof(self._struct)

    def refresh(self):
        """Rebuild the C view after parameters were reassigned (and re-pack
        the decoders if they were packed)."""
        self._struct = self._make_struct()
        if self._packed is not None:
            self.pack()


# ---------------------------------------------------------------------------
# 2. Queries
# ---------------------------------------------------------------------------
def query_sdf(model: Model, x: torch.Tensor, lod: int, alpha: float = 0.0, alpha_pp: torch.Tensor = None,
              want_valid: bool = False, want_vox: bool = False, out: torch.Tensor = None):
    """SDF at LOD `lod` (+alpha) for points x [3][P] (float32, device)."""
    _dev(x, torch.float32)
    Pn = x.shape[1]
    dev = x.device
    sdf = out if out is not None else torch.empty(Pn, dtype=torch.float32, device=dev)
    blend = alpha_pp is not None or alpha > 0.0
    Lp = lod + 1 if blend else lod
    valid = torch.empty(Pn, dtype=torch.uint8, device=dev) if want_valid else None
    vox = torch.empty((Lp, Pn), dtype=torch.int32, device=dev) if want_vox else None
    if alpha_pp is not None:
        _dev(alpha_pp, torch.float32)
    _check(lib().ngl_query_sdf(model.ref, _ptr(x), Pn, int(lod), float(alpha), _ptr(alpha_pp), _ptr(sdf),
                               _ptr(valid), _ptr(vox), _stream()))
    res = {"sdf": sdf}
    if want_valid:
        res["valid"] = valid
    if want_vox:
        res["vox"] = vox
    return res


def query_sdf_all_lods(model: Model, x: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    _dev(x, torch.float32)
    Pn = x.shape[1]
    o = out if out is not None else torch.empty((model.num_lods, Pn), dtype=torch.float32, device=x.device)
    _check(lib().ngl_query_sdf_all_lods(model.ref, _ptr(x), Pn, _ptr(o), _stream()))
    return o


def decode_sdf(model: Model, lod: int, z: torch.Tensor, x: torch.Tensor = None, out: torch.Tensor = None):
    """Decoder `lod` on given inputs: z [P][m] (float32 or bfloat16 rows,
    device), x [3][P] float32 when the model reads the position."""
    if z.dtype not in (torch.float32, torch.bfloat16) or not z.is_cuda or not z.is_contiguous():
        raise NGLError("z must be a contiguous float32 or bfloat16 device tensor")
    Pn = z.shape[0]
    if x is not None:
        _dev(x, torch.float32)
    sdf = out if out is not None else torch.empty(Pn, dtype=torch.float32, device=z.device)
    zt = BF16 if z.dtype == torch.bfloat16 else F32
    _check(lib().ngl_decode_sdf(model.ref, int(lod), _ptr(x), _ptr(z), zt, Pn, _ptr(sdf), _stream()))
    return sdf


def default_normal_step(model: "Model") -> float:
    """Finite-difference step: 1/16 of the finest voxel's edge."""
    return 2.0 / (4 << (model.num_lods - 1)) / 16.0


def sdf_normals(model: Model, lod: int, alpha: float = 0.0, h: float = None, x: torch.Tensor = None,
                rays=None, out: torch.Tensor = None) -> torch.Tensor:
    """Unit normals [3][P] by central differences of the SDF at LOD lod
    (+alpha), either at points x [3][P] or at the hit points of rays =
    (o, d, t_hit, status) (zero for rays that did not hit)."""
    h = default_normal_step(model) if h is None else h
    if rays is not None:
        o, d, t_hit, status = rays
        for a in (o, d):
            _dev(a, torch.float32)
        _dev(t_hit, torch.float32)
        _dev(status, torch.uint8)
        Pn = t_hit.shape[0]
        dev = t_hit.device
        args = (None, _ptr(o), _ptr(d), _ptr(t_hit), _ptr(status))
    else:
        _dev(x, torch.float32)
        Pn = x.shape[1]
        dev = x.device
        args = (_ptr(x), None, None, None, None)
    n = out if out is not None else torch.empty((3, Pn), dtype=torch.float32, device=dev)
    _check(lib().ngl_sdf_normals(model.ref, *args, Pn, int(lod), float(alpha), float(h), _ptr(n), _stream()))
    return n


# ---------------------------------------------------------------------------
# 3. Rays
# ---------------------------------------------------------------------------
def camera_rays(eye, target, up, fov_y_deg: float, width: int, height: int, device="cuda", out=None):
    R = width * height
    if out is None:
        o = torch.empty((3, R), dtype=torch.float32, device=device)
        d = torch.empty((3, R), dtype=torch.float32, device=device)
    else:
        o, d = out
    e = np.asarray(eye, np.float32)
    t = np.asarray(target, np.float32)
    u = np.asarray(up, np.float32)
    _check(lib().ngl_camera_rays(_ptr(e), _ptr(t), _ptr(u), float(fov_y_deg), int(width), int(height), _ptr(o),
                                 _ptr(d), _stream()))
    return o, d


class TraceBuffers:
    """Workspace and outputs of ngl_trace_octree for R rays at a capacity."""

    def __init__(self, R: int, capacity: int, device="cuda"):
        nb = C.c_size_t()
        _check(lib().ngl_trace_octree_workspace(R, capacity, C.addressof(nb)))
        self.R, self.capacity = R, capacity
        self.ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=device)
        self.ray = torch.empty(max(capacity, 1), dtype=torch.int32, device=device)
        self.vox = torch.empty(max(capacity, 1), dtype=torch.int32, device=device)
        self.t_in = torch.empty(max(capacity, 1), dtype=torch.float32, device=device)
        self.t_out = torch.empty(max(capacity, 1), dtype=torch.float32, device=device)
        self.ray_off = torch.empty(R + 1, dtype=torch.int32, device=device)
        self.counts = torch.zeros(2, dtype=torch.int64, device=device)


def trace_octree_into(model: Model, o, d, target_depth: int, buf: TraceBuffers):
    """Enqueue the ray-octree intersection into preallocated buffers (no sync)."""
    R = o.shape[1]
    assert buf.R == R
    _check(lib().ngl_trace_octree(model.ref, _ptr(o), _ptr(d), R, int(target_depth), buf.capacity, _ptr(buf.ws),
                                  buf.ws.numel(), _ptr(buf.ray), _ptr(buf.vox), _ptr(buf.t_in), _ptr(buf.t_out),
                                  _ptr(buf.ray_off), _ptr(buf.counts), _stream()))


def trace_octree(model: Model, o: torch.Tensor, d: torch.Tensor, target_depth: int, capacity: int = None,
                 buffers: TraceBuffers = None):
    """Front-to-back hit lists at `target_depth`.  Reads the device counts
    (one stream synchronisation) and retries with a larger capacity while a
    list overflowed."""
    _dev(o, torch.float32)
    _dev(d, torch.float32)
    R = o.shape[1]
    cap = capacity if capacity is not None else max(8 * R, 1 << 16)
    buf = buffers if buffers is not None and buffers.capacity >= cap else TraceBuffers(R, cap, o.device)
    trace_octree_into(model, o, d, target_depth, buf)
    counts = buf.counts.cpu()
    # After an overflow the sizes of deeper lists are lower bounds: grow
    # (at least doubling) until every list fits.
    while int(counts[1]) > buf.capacity:
        buf = TraceBuffers(R, max(int(counts[1]), 2 * buf.capacity), o.device)
        trace_octree_into(model, o, d, target_depth, buf)
        counts = buf.counts.cpu()
    n = int(counts[0])
    return dict(ray=buf.ray[:n], vox=buf.vox[:n], t_in=buf.t_in[:n], t_out=buf.t_out[:n], ray_off=buf.ray_off,
                count=n, max_list=int(counts[1]), buffers=buf)


def trace_params(max_steps: int, delta: float, t_far: float = 5.0, osc_check: bool = False, analytic_sphere=None,
                 image_width: int = 0):
    p = ngl_trace_params()
    p.image_width = int(image_width)
    p.max_steps = int(max_steps)
    p.delta = float(delta)
    p.t_far = float(t_far)
    p.osc_check = int(osc_check)
    p.analytic = int(analytic_sphere is not None)
    if analytic_sphere is not None:
        for k in range(4):
            p.sphere[k] = float(analytic_sphere[k])
    return p


def sphere_trace(model: Model, o, d, lod: int, alpha: float, hits: dict, max_steps: int, delta: float,
                 t_far: float = 5.0, osc_check: bool = False, analytic_sphere=None, out=None, phased: bool = True,
                 image_width: int = 0):
    """Sphere trace one view (ngl_sphere_trace).  `phased` sizes the
    workspace for the phased form (same results, long rays compacted);
    image_width > 0 serves the rays of that row-major image in 8x8 tiles
    (same results)."""
    R = o.shape[1]
    dev = o.device
    if out is None:
        out = dict(t=torch.empty(R, dtype=torch.float32, device=dev),
                   status=torch.empty(R, dtype=torch.uint8, device=dev),
                   steps=torch.empty(R, dtype=torch.int32, device=dev),
                   hit_vox=torch.empty(R, dtype=torch.int32, device=dev))
    prm = trace_params(max_steps, delta, t_far, osc_check, analytic_sphere, image_width)
    if "ws" not in out:
        nb = C.c_size_t()
        if phased:
            _check(lib().ngl_sphere_trace_workspace_rays(R, C.addressof(nb)))
        else:
            _check(lib().ngl_sphere_trace_workspace(C.addressof(nb)))
        out["ws"] = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    _check(lib().ngl_sphere_trace(model.ref, _ptr(o), _ptr(d), R, int(lod), float(alpha), _ptr(hits["vox"]),
                                  _ptr(hits["t_in"]), _ptr(hits["t_out"]), _ptr(hits["ray_off"]), C.addressof(prm),
                                  _ptr(out["t"]), _ptr(out["status"]), _ptr(out["steps"]), _ptr(out["hit_vox"]),
                                  _ptr(out["ws"]), out["ws"].numel(), _stream()))
    return out


STATIC_TRACE_MAX_RAYS = 1 << 21


def sphere_trace_static(model: Model, o, d, lod: int, alpha: float, hits: dict, max_steps: int, delta: float,
                        t_far: float = 5.0, osc_check: bool = False, out=None):
    """Sphere trace one view without a caller workspace
    (ngl_sphere_trace_static: the library's per-GPU array, no allocation in
    the call; calls on one GPU must not overlap)."""
    R = o.shape[1]
    dev = o.device
    if out is None:
        out = dict(t=torch.empty(R, dtype=torch.float32, device=dev),
                   status=torch.empty(R, dtype=torch.uint8, device=dev),
                   steps=torch.empty(R, dtype=torch.int32, device=dev),
                   hit_vox=torch.empty(R, dtype=torch.int32, device=dev))
    prm = trace_params(max_steps, delta, t_far, osc_check)
    _check(lib().ngl_sphere_trace_static(model.ref, _ptr(o), _ptr(d), R, int(lod), float(alpha), _ptr(hits["vox"]),
                                         _ptr(hits["t_in"]), _ptr(hits["t_out"]), _ptr(hits["ray_off"]),
                                         C.addressof(prm), _ptr(out["t"]), _ptr(out["status"]), _ptr(out["steps"]),
                                         _ptr(out["hit_vox"]), _stream()))
    return out


def lod_select(d_near: float, d_far: float, lod_near: float, lod_far: float) -> ngl_lod_select:
    s = ngl_lod_select()
    s.d_near, s.d_far, s.lod_near, s.lod_far = float(d_near), float(d_far), float(lod_near), float(lod_far)
    return s


def sphere_trace_lod(model: Model, o, d, pair_depth: int, sel: ngl_lod_select, hits: dict, max_steps: int,
                     delta: float, t_far: float = 5.0, osc_check: bool = False, out=None):
    """Sphere trace with per-pixel LOD selection (ngl_sphere_trace_lod);
    hits at pair_depth.  Returns t, status, steps, hit_vox and each ray's
    continuous LOD."""
    R = o.shape[1]
    dev = o.device
    if out is None:
        out = dict(t=torch.empty(R, dtype=torch.float32, device=dev),
                   status=torch.empty(R, dtype=torch.uint8, device=dev),
                   steps=torch.empty(R, dtype=torch.int32, device=dev),
                   hit_vox=torch.empty(R, dtype=torch.int32, device=dev),
                   lod=torch.empty(R, dtype=torch.float32, device=dev))
    prm = trace_params(max_steps, delta, t_far, osc_check)
    if "ws" not in out:
        nb = C.c_size_t()
        _check(lib().ngl_sphere_trace_lod_workspace(R, C.addressof(nb)))
        out["ws"] = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    _check(lib().ngl_sphere_trace_lod(model.ref, _ptr(o), _ptr(d), R, int(pair_depth), C.addressof(sel),
                                      _ptr(hits["vox"]), _ptr(hits["t_in"]), _ptr(hits["t_out"]),
                                      _ptr(hits["ray_off"]), C.addressof(prm), _ptr(out["t"]), _ptr(out["status"]),
                                      _ptr(out["steps"]), _ptr(out["hit_vox"]), _ptr(out.get("lod")),
                                      _ptr(out["ws"]), out["ws"].numel(), _stream()))
    return out


# ---------------------------------------------------------------------------
# 3b. Batched rendering
# ---------------------------------------------------------------------------
def make_view(eye, width, height, lod, alpha=0.0, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fov_y_deg=45.0):
    v = ngl_view()
    for a in range(3):
        v.eye[a], v.target[a], v.up[a] = float(eye[a]), float(target[a]), float(up[a])
    v.fov_y_deg = float(fov_y_deg)
    v.width, v.height, v.lod, v.alpha = int(width), int(height), int(lod), float(alpha)
    return v


class BatchRenderer:
    """Device model table, workspace and outputs for ngl_render_batch over a
    fixed list of models (all of one format) and view sizes."""

    def __init__(self, models: Sequence[Model], views: Sequence[ngl_view], pair_capacity: int, device="cuda"):
        L = lib()
        self.models = list(models)
        self.n = len(self.models)
        if not 1 <= self.n <= MAX_BATCH:
            raise NGLError("between 1 and %d models" % MAX_BATCH)
        self.h_models = (ngl_model * self.n)(*[m._struct for m in self.models])
        nb = C.c_size_t()
        _check(L.ngl_model_table_bytes(self.n, C.addressof(nb)))
        self.table = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        _check(L.ngl_model_table_upload(C.addressof(self.h_models), self.n, _ptr(self.table), _stream()))
        self.set_views(views, pair_capacity, device)

    def set_views(self, views, pair_capacity, device="cuda"):
        self.views = (ngl_view * self.n)(*views)
        self.sizes = [v.width * v.height for v in views]
        self.base = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.capacity = int(pair_capacity)
        nb = C.c_size_t()
        _check(lib().ngl_render_batch_workspace(C.addressof(self.views), self.n, self.capacity, C.addressof(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        R = int(self.base[-1])
        self.t = torch.empty(R, dtype=torch.float32, device=device)
        self.status = torch.empty(R, dtype=torch.uint8, device=device)
        self.steps = torch.empty(R, dtype=torch.int32, device=device)
        self.hit_vox = torch.empty(R, dtype=torch.int32, device=device)
        self.counts = torch.zeros((self.n, 2), dtype=torch.int64, device=device)
        self.clock = torch.zeros(self.n + 1, dtype=torch.int64, device=device)

    def render(self, max_steps: int, delta: float, t_far: float = 5.0, osc_check: bool = False):
        """Enqueue one batched render (no synchronisation)."""
        self._prm = trace_params(max_steps, delta, t_far, osc_check)
        _check(lib().ngl_render_batch(C.addressof(self.h_models), _ptr(self.table), C.addressof(self.views), self.n,
                                      C.addressof(self._prm), self.capacity, _ptr(self.ws), self.ws.numel(),
                                      _ptr(self.t), _ptr(self.status), _ptr(self.steps), _ptr(self.hit_vox),
                                      _ptr(self.counts), _ptr(self.clock), _stream()))

    def overflowed(self) -> bool:
        return bool((self.counts[:, 1] > self.capacity).any().item())

    def view_slice(self, i: int) -> slice:
        return slice(int(self.base[i]), int(self.base[i + 1]))

    def frame_ms(self):
        """Per-view end time after the batch start (device wall clock, 100 MHz)."""
        c = self.clock.cpu().numpy().astype(np.float64)
        return (c[1:] - c[0]) * 1e-5


# ---------------------------------------------------------------------------
# 4. Training
# ---------------------------------------------------------------------------
class Grads:
    """FP32 gradient buffers laid out like the model's parameters."""

    def __init__(self, model: Model):
        dev = model.b2.device
        self.dfeat = [torch.empty(f.shape, dtype=torch.float32, device=dev) for f in model.feats]
        self.dW1 = [torch.empty(w.shape, dtype=torch.float32, device=dev) for w in model.W1]
        self.db1 = [torch.empty_like(b) for b in model.b1]
        self.dw2 = [torch.empty_like(w) for w in model.w2]
        self.db2 = torch.empty_like(model.b2)
        arr = lambda lst: (P * MAX_LODS)(*[_ptr(t) if t.numel() else None for t in lst])
        self._arrays = [arr(self.dfeat), arr(self.dW1), arr(self.db1), arr(self.dw2)]
        self.ptrs = [C.addressof(a) for a in self._arrays]


def train_workspace(model: Model, P_: int, device="cuda") -> torch.Tensor:
    nb = C.c_size_t()
    _check(lib().ngl_train_workspace(model.ref, int(P_), C.addressof(nb)))
    return torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=device)


def train_fwd_bwd(model: Model, x: torch.Tensor, target: torch.Tensor, grads: Grads = None, ws: torch.Tensor = None,
                  sdf_all: torch.Tensor = None, loss: torch.Tensor = None):
    _dev(x, torch.float32)
    _dev(target, torch.float32)
    Pn = x.shape[1]
    g = grads if grads is not None else Grads(model)
    w = ws if ws is not None else train_workspace(model, Pn, x.device)
    ls = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().ngl_train_fwd_bwd(model.ref, _ptr(x), _ptr(target), Pn, _ptr(ls), _ptr(sdf_all), g.ptrs[0],
                                   g.ptrs[1], g.ptrs[2], g.ptrs[3], _ptr(g.db2), _ptr(w), w.numel(), _stream()))
    return ls, g


def backward_all_lods(model: Model, x: torch.Tensor, grad_sdf: torch.Tensor, grads: Grads = None,
                      ws: torch.Tensor = None) -> Grads:
    _dev(x, torch.float32)
    _dev(grad_sdf, torch.float32)
    Pn = x.shape[1]
    g = grads if grads is not None else Grads(model)
    w = ws if ws is not None else train_workspace(model, Pn, x.device)
    _check(lib().ngl_backward_all_lods(model.ref, _ptr(x), Pn, _ptr(grad_sdf), g.ptrs[0], g.ptrs[1], g.ptrs[2],
                                       g.ptrs[3], _ptr(g.db2), _ptr(w), w.numel(), _stream()))
    return g


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
class NGLODSdf(torch.autograd.Function):
    """sdf_all = [f_theta_L([x, z_L(x)]) for L = 1..Lmax] (Eq. 2) with the
    library's backward (FP32 model).  Usage:
        sdf_all = NGLODSdf.apply(model, x, *model.parameters())
    Gradients flow to the corner features and decoder parameters (not to x)."""

    @staticmethod
    def forward(ctx, model: Model, x: torch.Tensor, *params):
        ctx.model = model
        ctx.save_for_backward(x)
        return query_sdf_all_lods(model, x.contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        (x,) = ctx.saved_tensors
        model = ctx.model
        g = backward_all_lods(model, x.contiguous(), grad_out.contiguous().float())
        return (None, None, *g.dfeat, *g.dW1, *g.db1, *g.dw2, g.db2)


def parameters(model: Model):
    """The model's tensors in the order NGLODSdf.backward returns gradients."""
    return [*model.feats, *model.W1, *model.b1, *model.w2, model.b2]


# ---------------------------------------------------------------------------
# 5. Fitting pieces: analytic shapes, samplers, Adam, per-LOD loss weights
# ---------------------------------------------------------------------------
class DeviceShape:
    """A sphere/torus union (spheres [n][4], tori [n][6]) in device memory."""

    def __init__(self, spheres, tori, device="cuda"):
        sph = torch.tensor(np.asarray(spheres, np.float64).reshape(-1, 4), dtype=torch.float32, device=device)
        tor = torch.tensor(np.asarray(tori, np.float64).reshape(-1, 6), dtype=torch.float32, device=device)
        self.spheres, self.tori = sph.contiguous(), tor.contiguous()
        self.s = ngl_shape()
        self.s.n_spheres, self.s.n_tori = sph.shape[0], tor.shape[0]
        self.s.spheres, self.s.tori = _ptr(self.spheres), _ptr(self.tori)
        self.ref = C.addressof(self.s)

    def host(self):
        """The FP32-rounded primitives as float64 arrays."""
        return (self.spheres.double().cpu().numpy().reshape(-1, 4), self.tori.double().cpu().numpy().reshape(-1, 6))


def shape_sdf(shape: DeviceShape, x: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    _dev(x, torch.float32)
    o = out if out is not None else torch.empty(x.shape[1], dtype=torch.float32, device=x.device)
    _check(lib().ngl_shape_sdf(shape.ref, _ptr(x), x.shape[1], _ptr(o), _stream()))
    return o


def sample_surface(shape: DeviceShape, u: torch.Tensor, max_steps: int, delta: float, out: dict = None) -> dict:
    """SDF surface sampler: u [5][n] uniforms; returns pts [3][n] (the first
    `count` columns are the hits, in ray order) and a device count."""
    _dev(u, torch.float32)
    n = u.shape[1]
    dev = u.device
    if out is None:
        nb = C.c_size_t()
        _check(lib().ngl_sample_surface_workspace(n, C.addressof(nb)))
        out = dict(pts=torch.empty((3, n), dtype=torch.float32, device=dev),
                   count=torch.zeros(1, dtype=torch.int64, device=dev),
                   ws=torch.empty(max(int(nb.value), 4), dtype=torch.uint8, device=dev))
    _check(lib().ngl_sample_surface(shape.ref, _ptr(u), n, int(max_steps), float(delta), _ptr(out["pts"]),
                                    _ptr(out["count"]), _ptr(out["ws"]), out["ws"].numel(), _stream()))
    return out


def training_points(shape: DeviceShape, surface: torch.Tensor, n_surface: int, uniforms: torch.Tensor, batch: int,
                    sigma: float = 0.01, x: torch.Tensor = None, target: torch.Tensor = None):
    """2:2:1 training set: x [N/batch][3][batch] and targets [N]."""
    _dev(surface, torch.float32)
    _dev(uniforms, torch.float32)
    N = uniforms.shape[1]
    dev = uniforms.device
    x = x if x is not None else torch.empty((N // batch, 3, batch), dtype=torch.float32, device=dev)
    target = target if target is not None else torch.empty(N, dtype=torch.float32, device=dev)
    _check(lib().ngl_training_points(shape.ref, _ptr(surface), int(n_surface), surface.shape[1], _ptr(uniforms), N,
                                     int(batch), float(sigma), _ptr(x), _ptr(target), _stream()))
    return x, target


class AdamGroup:
    """Pointer tables of one set of tensors for ngl_adam_step, built once."""

    def __init__(self, params, grads, m, v):
        self.n = len(params)
        arr = lambda lst: (P * max(self.n, 1))(*[_ptr(t) for t in lst])
        self.numel = (i64 * max(self.n, 1))(*[t.numel() for t in params])
        self.arrays = [arr(params), arr(grads), arr(m), arr(v)]
        self.addr = [C.addressof(a) for a in self.arrays]
        self.prm = ngl_adam_params()

    def step(self, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        p = self.prm
        p.lr, p.beta1, p.beta2, p.eps, p.step = float(lr), float(beta1), float(beta2), float(eps), int(step)
        _check(lib().ngl_adam_step(C.addressof(p), self.n, *self.addr, C.addressof(self.numel), _stream()))


def adam_step(params, grads, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Fused Adam over lists of FP32 device tensors (in place)."""
    AdamGroup(params, grads, m, v).step(step, lr, beta1, beta2, eps)


def train_fwd_bwd_lods(model: Model, x: torch.Tensor, target: torch.Tensor, lod_weight, grads: Grads = None,
                       ws: torch.Tensor = None, loss: torch.Tensor = None, sdf_all: torch.Tensor = None):
    """Eq. 4 with per-LOD weights (host list of num_lods floats)."""
    _dev(x, torch.float32)
    _dev(target, torch.float32)
    Pn = x.shape[1]
    g = grads if grads is not None else Grads(model)
    w = ws if ws is not None else train_workspace(model, Pn, x.device)
    ls = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=x.device)
    lw = (C.c_float * MAX_LODS)(*([float(v) for v in lod_weight] + [0.0] * (MAX_LODS - len(lod_weight))))
    _check(lib().ngl_train_fwd_bwd_lods(model.ref, _ptr(x), _ptr(target), Pn, C.addressof(lw), _ptr(ls),
                                        _ptr(sdf_all), g.ptrs[0], g.ptrs[1], g.ptrs[2], g.ptrs[3], _ptr(g.db2),
                                        _ptr(w), w.numel(), _stream()))
    return ls, g

