"""FP64 CPU oracle (test infrastructure only).

Plain, slow, obviously correct restatement of the neural geometric LOD
hot path (arXiv 2101.10994).  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
uses it.  It shares no code with the GPU library (`oracle.c` includes
nothing from it).

Entry points and the passage each one follows:

* ``Octree``          -- sparse voxel octree from occupancy (Sec. 3.2; App. A.1)
* ``query``           -- SDF at LOD L (Eq. 2) or continuous L+alpha (Eq. 3)
* ``decode``          -- the per-LOD decoder of Eq. 2 alone, on given [x, z]
* ``trace_octree``    -- ray-octree hit lists (Sec. 3.4, Alg. 1, App. C)
* ``camera_rays``     -- pinhole primary rays (the ray set of Alg. 1)
* ``sphere_trace``    -- adaptive-stepping sphere tracing (Sec. 3.4, Fig. 3;
                         stopping rules of App. A.4)
* ``lod_select``      -- per-pixel LOD from distance (Sec. 3.4, LOD Selection)
* ``sphere_trace_pp`` -- sphere tracing with a LOD and blend weight per ray
* ``normals``         -- surface normals by central finite differences of
                         ``query`` (App. A.4), at points or ray hit points
* ``train_fwd_bwd``   -- Eq. 4 loss and its gradient (Sec. 3.3)

Every entry point is pinned by CPU tests against closed forms, brute force
or finite differences (see tests/test_oracle_*.py); none is "parity
unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

MAXL = 10
MISS, HIT, MAX_STEPS, FAR, STALLED, INVALID = range(6)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = C.CDLL(_LIB)
            _setup(_lib)
    return _lib


P = C.c_void_p
i64 = C.c_int64


class _Model(C.Structure):
    _fields_ = [("num_lods", C.c_int), ("m", C.c_int), ("hidden", C.c_int), ("with_xyz", C.c_int),
                ("feat", P * MAXL), ("W1", P * MAXL), ("b1", P * MAXL), ("w2", P * MAXL),
                ("b2", P)]


class _TraceParams(C.Structure):
    _fields_ = [("max_steps", C.c_int), ("delta", C.c_double), ("t_far", C.c_double),
                ("osc_check", C.c_int), ("analytic", C.c_int), ("sphere", C.c_double * 4),
                ("margin_sdf", C.c_double), ("margin_t", C.c_double)]


def _setup(lib):
    lib.orc_octree_build.restype = P
    lib.orc_octree_build.argtypes = [P, i64, C.c_int]
    lib.orc_octree_free.argtypes = [P]
    lib.orc_octree_counts.argtypes = [P, P, P]
    lib.orc_octree_export_depth.argtypes = [P, C.c_int, P, P, P, P]
    lib.orc_octree_export_corners.argtypes = [P, C.c_int, P, P]
    lib.orc_decode.restype = C.c_int
    lib.orc_decode.argtypes = [P, C.c_int, P, P, i64, P, P, P]
    lib.orc_query.restype = C.c_int
    lib.orc_query.argtypes = [P, P, P, i64, C.c_int, C.c_double, P, P, P, P, P, P]
    lib.orc_ray_box.restype = C.c_int
    lib.orc_ray_box.argtypes = [P, P, C.c_int, P, P, P]
    lib.orc_trace_octree.restype = i64
    lib.orc_trace_octree.argtypes = [P, P, P, i64, C.c_int, i64, P, P, P, P, P]
    lib.orc_camera_rays.argtypes = [P, P, P, C.c_double, C.c_int, C.c_int, P, P]
    lib.orc_sphere_trace.restype = C.c_int
    lib.orc_sphere_trace.argtypes = [P, P, P, P, i64, C.c_int, C.c_double, P, P, P, P, P,
                                     P, P, P, P, P]
    lib.orc_sphere_trace_pp.restype = C.c_int
    lib.orc_sphere_trace_pp.argtypes = [P, P, P, P, i64, C.c_int, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_lod_select.argtypes = [C.c_float, C.c_float, C.c_float, C.c_float, C.c_int, C.c_float, P, P, P]
    lib.orc_train_fwd_bwd_w.restype = C.c_int
    lib.orc_train_fwd_bwd_w.argtypes = [P, P, P, P, i64, P, P, P, P, P, P, P, P]
    lib.orc_shape_sdf_many.argtypes = [C.c_int, P, C.c_int, P, P, i64, P]
    lib.orc_sample_surface.argtypes = [C.c_int, P, C.c_int, P, P, i64, C.c_int, C.c_double, C.c_double, C.c_double,
                                       P, P, P]
    lib.orc_training_points.restype = C.c_int
    lib.orc_training_points.argtypes = [C.c_int, P, C.c_int, P, P, i64, P, i64, C.c_double, P, P]
    lib.orc_train_fwd_bwd.restype = C.c_int
    lib.orc_train_fwd_bwd.argtypes = [P, P, P, P, i64, P, P, P, P, P, P, P]


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int):
    """Set the OpenMP thread count used by the oracle (via libgomp)."""
    _load()
    gomp = C.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(int(n))


def max_threads() -> int:
    _load()
    gomp = C.CDLL("libgomp.so.1")
    gomp.omp_get_max_threads.restype = C.c_int
    return int(gomp.omp_get_max_threads())


class Octree:
    """Canonical sparse voxel octree (sorted Morton codes per depth)."""

    def __init__(self, ijk: np.ndarray, num_lods: int):
        lib = _load()
        ijk = _c(np.asarray(ijk).reshape(-1, 3), np.int32)
        h = lib.orc_octree_build(_ptr(ijk), ijk.shape[0], int(num_lods))
        if not h:
            raise ValueError("invalid occupancy for the oracle octree")
        self._h = h
        self.num_lods = int(num_lods)
        self.depth = self.num_lods + 1
        nv = np.zeros(self.depth + 1, np.int64)
        nc = np.zeros(self.num_lods, np.int64)
        lib.orc_octree_counts(h, _ptr(nv), _ptr(nc))
        self.nvox = nv
        self.ncorner = nc

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_octree_free(self._h)
            self._h = None

    def export_depth(self, d: int):
        n = int(self.nvox[d])
        ijk = np.zeros((n, 3), np.int32)
        cm = np.zeros(n, np.uint8)
        fc = np.zeros(n, np.int32)
        par = np.zeros(n, np.int32)
        _load().orc_octree_export_depth(self._h, d, _ptr(ijk), _ptr(cm), _ptr(fc), _ptr(par))
        return dict(ijk=ijk, child_mask=cm, first_child=fc, parent=par)

    def export_corners(self, lvl: int):
        nv = int(self.nvox[lvl + 1])
        nc = int(self.ncorner[lvl - 1])
        corners = np.zeros((nv, 8), np.int32)
        cijk = np.zeros((nc, 3), np.int32)
        _load().orc_octree_export_corners(self._h, lvl, _ptr(corners), _ptr(cijk))
        return corners, cijk

    def corner_positions(self):
        """Corner positions in [-1,1]^3 per feature level (float64)."""
        out = []
        for lvl in range(1, self.num_lods + 1):
            _, cijk = self.export_corners(lvl)
            r = 2 ** (lvl + 1)
            out.append(-1.0 + cijk.astype(np.float64) * (2.0 / r))
        return out


class Model:
    """Parameters in float64 (features per level, decoders per LOD)."""

    def __init__(self, feats, W1, b1, w2, b2, with_xyz=True):
        self.num_lods = len(feats)
        self.feats = [_c(f, np.float64) for f in feats]
        self.W1 = [_c(w, np.float64) for w in W1]
        self.b1 = [_c(w, np.float64) for w in b1]
        self.w2 = [_c(w, np.float64) for w in w2]
        self.b2 = _c(b2, np.float64)
        self.m = self.feats[0].shape[1]
        self.hidden = self.W1[0].shape[0]
        self.with_xyz = bool(with_xyz)
        assert self.W1[0].shape[1] == self.m + (3 if with_xyz else 0)

    def struct(self):
        s = _Model()
        s.num_lods, s.m, s.hidden, s.with_xyz = self.num_lods, self.m, self.hidden, int(self.with_xyz)
        for lvl in range(self.num_lods):
            s.feat[lvl] = _ptr(self.feats[lvl])
            s.W1[lvl] = _ptr(self.W1[lvl])
            s.b1[lvl] = _ptr(self.b1[lvl])
            s.w2[lvl] = _ptr(self.w2[lvl])
        s.b2 = _ptr(self.b2)
        return s

    def param_count_per_lod(self):
        return self.W1[0].size + self.b1[0].size + self.w2[0].size + 1


def query(tree: Octree, model: Model, x_soa: np.ndarray, lod: int, alpha: float = 0.0,
          alpha_pp: np.ndarray = None, want_vox: bool = False):
    """SDF at LOD `lod` (+alpha).  x_soa: float32 [3][P].
    Returns dict(sdf, scale, scale1, valid, vox); scale and scale1 are the
    magnitude scales used in error bounds (see decode in oracle.c)."""
    x = _c(x_soa, np.float32)
    Pn = x.shape[1]
    ap = None if alpha_pp is None else _c(alpha_pp, np.float32)
    blend = ap is not None or alpha > 0.0
    Lp = lod + 1 if blend else lod
    sdf = np.zeros(Pn)
    scale = np.zeros(Pn)
    scale1 = np.zeros(Pn)
    valid = np.zeros(Pn, np.uint8)
    vox = np.zeros((Lp, Pn), np.int32) if want_vox else None
    ms = model.struct()
    rc = _load().orc_query(tree._h, C.addressof(ms), _ptr(x), Pn, int(lod), float(alpha), _ptr(ap),
                           _ptr(sdf), _ptr(scale), _ptr(scale1), _ptr(valid), _ptr(vox))
    if rc != 0:
        raise ValueError("oracle query: invalid arguments")
    return dict(sdf=sdf, scale=scale, scale1=scale1, valid=valid, vox=vox)


def decode(model: Model, lod: int, z, x_soa=None):
    """Decoder `lod` (Eq. 2's MLP) on inputs z [P][m] (float64 values) and
    x [3][P] float32.  Returns dict(sdf, scale, scale1)."""
    zz = _c(z, np.float64)
    Pn = zz.shape[0]
    x = _c(x_soa if x_soa is not None else np.zeros((3, Pn)), np.float32)
    sdf, scale, scale1 = np.zeros(Pn), np.zeros(Pn), np.zeros(Pn)
    ms = model.struct()
    rc = _load().orc_decode(C.addressof(ms), int(lod), _ptr(x), _ptr(zz), Pn, _ptr(sdf), _ptr(scale), _ptr(scale1))
    if rc != 0:
        raise ValueError("oracle decode: invalid arguments")
    return dict(sdf=sdf, scale=scale, scale1=scale1)


def fma_f32(a, b, c):
    """a*b + c for float32 arrays, rounded once to float32 (IEEE fused
    multiply-add, round to nearest even)."""
    a64 = np.asarray(a, np.float32).astype(np.float64)
    b64 = np.asarray(b, np.float32).astype(np.float64)
    c64 = np.asarray(c, np.float32).astype(np.float64)
    p = a64 * b64                      # exact: 24 + 24 bits fit in 53
    s = p + c64
    bv = s - p                         # two-sum: s + e == p + c exactly
    e = (p - (s - bv)) + (c64 - bv)
    r = s.astype(np.float32)
    # s rounds like the exact sum unless s is a float32 midpoint and e != 0.
    toward = np.where(s > r.astype(np.float64), np.float32(np.inf), np.float32(-np.inf)).astype(np.float32)
    r2 = np.nextafter(r, toward)
    mid = (r.astype(np.float64) + r2.astype(np.float64)) * 0.5
    tie = (s == mid) & (e != 0.0) & (s != r.astype(np.float64))
    pick2 = tie & ((e > 0.0) == (r2 > r))
    return np.where(pick2, r2, r).astype(np.float32)


def normals(tree: Octree, model: Model, lod: int, alpha: float, h: float, x_soa=None, rays=None):
    """Unit surface normals by central differences (App. A.4 names finite
    differences; the central form and the step h are this library's
    reading).  For each point x and axis a, f(x + h e_a) and f(x - h e_a)
    are SDF values at LOD lod (+alpha) of the float32 points x_a +- h, and
    g_a = (f+ - f-) / (2h); the normal is g / |g| (zero when |g| = 0).
    With rays = (o, d, t_hit, status) the points are fma(t_hit, d, o) for
    rays with status HIT, zero normals elsewhere.  Also returns g and
    per-axis (scale, scale1) sums of the six queries for error bounds."""
    h32 = np.float32(h)
    if rays is not None:
        o, d, t, st = rays
        o = _c(o, np.float32)
        d = _c(d, np.float32)
        t = np.asarray(t, np.float32)
        x = np.stack([fma_f32(t, d[a], o[a]) for a in range(3)])
        act = np.asarray(st) == HIT
    else:
        x = _c(x_soa, np.float32)
        act = np.ones(x.shape[1], bool)
    Pn = x.shape[1]
    g = np.zeros((3, Pn))
    fsum = np.zeros((3, Pn))
    ssum = np.zeros((3, Pn))
    s1sum = np.zeros((3, Pn))
    for a in range(3):
        for sgn in (1.0, -1.0):
            xs = x.copy()
            xs[a] = (x[a] + np.float32(sgn) * h32).astype(np.float32)
            q = query(tree, model, xs, lod, alpha)
            g[a] += sgn * q["sdf"]
            fsum[a] += np.abs(q["sdf"])
            ssum[a] += q["scale"]
            s1sum[a] += q["scale1"]
    g /= 2.0 * float(h32)
    g[:, ~act] = 0.0
    ln = np.sqrt((g * g).sum(0))
    n = np.where(ln > 0.0, g / np.where(ln > 0.0, ln, 1.0), 0.0)
    return dict(n=n, g=g, points=x, active=act, fsum=fsum, scale=ssum, scale1=s1sum)


def ray_box(o, d, depth, cell):
    """FP32 slab predicate of one ray against one cell: (hit, t_in, t_out)."""
    o = _c(o, np.float32)
    d = _c(d, np.float32)
    c = _c(cell, np.int32)
    ti = C.c_float()
    to = C.c_float()
    h = _load().orc_ray_box(_ptr(o), _ptr(d), int(depth), _ptr(c), C.addressof(ti), C.addressof(to))
    return bool(h), ti.value, to.value


def trace_octree(tree: Octree, o_soa, d_soa, target_depth: int):
    """Front-to-back hit lists at octree depth `target_depth`."""
    o = _c(o_soa, np.float32)
    d = _c(d_soa, np.float32)
    R = o.shape[1]
    off = np.zeros(R + 1, np.int64)
    lib = _load()
    total = lib.orc_trace_octree(tree._h, _ptr(o), _ptr(d), R, int(target_depth), 0, None, None, None, None,
                                 _ptr(off))
    if total < 0:
        raise ValueError("oracle trace_octree: invalid arguments")
    ray = np.zeros(total, np.int32)
    vox = np.zeros(total, np.int32)
    tin = np.zeros(total, np.float32)
    tout = np.zeros(total, np.float32)
    lib.orc_trace_octree(tree._h, _ptr(o), _ptr(d), R, int(target_depth), int(total), _ptr(ray), _ptr(vox),
                         _ptr(tin), _ptr(tout), _ptr(off))
    return dict(ray=ray, vox=vox, t_in=tin, t_out=tout, ray_off=off)


def camera_rays(eye, target, up, fov_y_deg, width, height):
    """FP64 pinhole rays, SoA [3][W*H] (origin, direction)."""
    R = width * height
    o = np.zeros((3, R))
    d = np.zeros((3, R))
    e = _c(eye, np.float64)
    t = _c(target, np.float64)
    u = _c(up, np.float64)
    _load().orc_camera_rays(_ptr(e), _ptr(t), _ptr(u), float(fov_y_deg), int(width), int(height), _ptr(o), _ptr(d))
    return o, d


def sphere_trace(tree: Octree, model: Model, o_soa, d_soa, lod: int, alpha: float, hits: dict,
                 max_steps: int, delta: float, t_far: float = 5.0, osc_check: bool = False,
                 analytic_sphere=None, margin_sdf: float = 0.0, margin_t: float = 0.0):
    """Adaptive-stepping sphere trace over precomputed hit lists `hits`
    (as returned by trace_octree at depth lod+1, or lod+2 when alpha > 0)."""
    o = _c(o_soa, np.float32)
    d = _c(d_soa, np.float32)
    R = o.shape[1]
    prm = _TraceParams()
    prm.max_steps = int(max_steps)
    prm.delta = float(delta)
    prm.t_far = float(t_far)
    prm.osc_check = int(osc_check)
    prm.analytic = int(analytic_sphere is not None)
    if analytic_sphere is not None:
        for k in range(4):
            prm.sphere[k] = float(analytic_sphere[k])
    prm.margin_sdf = float(margin_sdf)
    prm.margin_t = float(margin_t)
    t_hit = np.zeros(R)
    status = np.zeros(R, np.uint8)
    steps = np.zeros(R, np.int32)
    hv = np.zeros(R, np.int32)
    marg = np.zeros(R, np.uint8)
    ms = model.struct() if model is not None else _Model()
    rc = _load().orc_sphere_trace(tree._h, C.addressof(ms), _ptr(o), _ptr(d), R, int(lod), float(alpha),
                                  _ptr(hits["vox"]), _ptr(hits["t_in"]), _ptr(hits["t_out"]),
                                  _ptr(_c(hits["ray_off"], np.int64)), C.addressof(prm), _ptr(t_hit),
                                  _ptr(status), _ptr(steps), _ptr(hv), _ptr(marg))
    if rc != 0:
        raise ValueError("oracle sphere_trace: invalid arguments")
    return dict(t=t_hit, status=status, steps=steps, hit_vox=hv, marginal=marg)


def lod_select(d_near: float, d_far: float, lod_near: float, lod_far: float, num_lods: int, dist):
    """Per-ray continuous LOD from a distance, in FP32 (see orc_lod_select).
    Returns (lod_cont float32, lod_int int32, alpha float32) arrays."""
    dist = np.atleast_1d(np.asarray(dist, np.float32))
    Lc = np.zeros(len(dist), np.float32)
    Li = np.zeros(len(dist), np.int32)
    al = np.zeros(len(dist), np.float32)
    lib = _load()
    out_c, out_i, out_a = C.c_float(), C.c_int32(), C.c_float()
    for k, v in enumerate(dist):
        lib.orc_lod_select(float(d_near), float(d_far), float(lod_near), float(lod_far), int(num_lods), float(v),
                           C.byref(out_c), C.byref(out_i), C.byref(out_a))
        Lc[k], Li[k], al[k] = out_c.value, out_i.value, out_a.value
    return Lc, Li, al


def first_pair_distance(hits: dict, R: int, t_far: float):
    """Entry distance of each ray's first pair (t_far when it has none)."""
    off = np.asarray(hits["ray_off"], np.int64)
    t_in = np.asarray(hits["t_in"], np.float32)
    has = off[1:] > off[:-1]
    dist = np.full(R, np.float32(t_far), np.float32)
    dist[has] = t_in[off[:-1][has]]
    return dist


def sphere_trace_pp(tree: Octree, model: Model, o_soa, d_soa, pair_depth: int, lod_pp, alpha_pp, hits: dict,
                    max_steps: int, delta: float, t_far: float = 5.0, osc_check: bool = False,
                    margin_sdf: float = 0.0, margin_t: float = 0.0):
    """Sphere trace with per-ray LOD and blend weight over hit lists at
    `pair_depth` (see orc_sphere_trace_pp)."""
    o = _c(o_soa, np.float32)
    d = _c(d_soa, np.float32)
    R = o.shape[1]
    prm = _TraceParams()
    prm.max_steps = int(max_steps)
    prm.delta = float(delta)
    prm.t_far = float(t_far)
    prm.osc_check = int(osc_check)
    prm.analytic = 0
    prm.margin_sdf = float(margin_sdf)
    prm.margin_t = float(margin_t)
    t_hit = np.zeros(R)
    status = np.zeros(R, np.uint8)
    steps = np.zeros(R, np.int32)
    hv = np.zeros(R, np.int32)
    marg = np.zeros(R, np.uint8)
    ms = model.struct()
    lp = _c(lod_pp, np.int32)
    ap = _c(alpha_pp, np.float32)
    rc = _load().orc_sphere_trace_pp(tree._h, C.addressof(ms), _ptr(o), _ptr(d), R, int(pair_depth), _ptr(lp),
                                     _ptr(ap), _ptr(hits["vox"]), _ptr(hits["t_in"]), _ptr(hits["t_out"]),
                                     _ptr(_c(hits["ray_off"], np.int64)), C.addressof(prm), _ptr(t_hit),
                                     _ptr(status), _ptr(steps), _ptr(hv), _ptr(marg))
    if rc != 0:
        raise ValueError("oracle sphere_trace_pp: invalid arguments")
    return dict(t=t_hit, status=status, steps=steps, hit_vox=hv, marginal=marg)


def train_fwd_bwd(tree: Octree, model: Model, x_soa, target, want_sdf=False, grads=True, lod_weight=None):
    """Eq. 4 loss and gradients (float64), laid out like the parameters;
    lod_weight (optional, [L]) weights each LOD's term."""
    x = _c(x_soa, np.float32)
    tg = _c(target, np.float32)
    Pn = x.shape[1]
    L = model.num_lods
    loss = np.zeros(1)
    out = dict()
    if grads:
        dF = [np.zeros_like(f) for f in model.feats]
        dW1 = [np.zeros_like(w) for w in model.W1]
        db1 = [np.zeros_like(w) for w in model.b1]
        dw2 = [np.zeros_like(w) for w in model.w2]
        db2 = np.zeros(L)
        arr = lambda lst: (P * L)(*[_ptr(a) for a in lst])
        pF, pW1, pb1, pw2 = arr(dF), arr(dW1), arr(db1), arr(dw2)
        out.update(dfeat=dF, dW1=dW1, db1=db1, dw2=dw2, db2=db2)
    else:
        pF = pW1 = pb1 = pw2 = None
        db2 = None
    sdf_all = np.zeros((L, Pn)) if want_sdf else None
    ms = model.struct()
    lw = None if lod_weight is None else _c(lod_weight, np.float64)
    rc = _load().orc_train_fwd_bwd_w(tree._h, C.addressof(ms), _ptr(x), _ptr(tg), Pn, _ptr(lw), _ptr(loss),
                                     pF, pW1, pb1, pw2, _ptr(db2), _ptr(sdf_all))
    if rc != 0:
        raise ValueError("oracle train_fwd_bwd: invalid arguments")
    out["loss"] = float(loss[0])
    if want_sdf:
        out["sdf_all"] = sdf_all
    return out


def loss(tree: Octree, model: Model, x_soa, target) -> float:
    return train_fwd_bwd(tree, model, x_soa, target, grads=False)["loss"]


# ---------------------------------------------------------------------------
# Fitting (training appendix): analytic shapes, samplers, Adam
# ---------------------------------------------------------------------------
def _shape_arrays(spheres, tori):
    sph = _c(np.asarray(spheres, np.float64).reshape(-1, 4), np.float64)
    tor = _c(np.asarray(tori, np.float64).reshape(-1, 6), np.float64)
    return sph, tor


def shape_sdf(spheres, tori, x_soa):
    """Exact union SDF (float64) at float32 points [3][P]."""
    sph, tor = _shape_arrays(spheres, tori)
    x = _c(x_soa, np.float32)
    out = np.zeros(x.shape[1])
    _load().orc_shape_sdf_many(len(sph), _ptr(sph), len(tor), _ptr(tor), _ptr(x), x.shape[1], _ptr(out))
    return out


def sample_surface(spheres, tori, u, max_steps: int, delta: float, margin_box: float = 0.0, margin_sdf: float = 0.0):
    """SDF surface sampler (see orc_sample_surface); u: [5][n] float32."""
    sph, tor = _shape_arrays(spheres, tori)
    uu = _c(u, np.float32)
    n = uu.shape[1]
    pts = np.zeros((3, n))
    hit = np.zeros(n, np.uint8)
    marg = np.zeros(n, np.uint8)
    _load().orc_sample_surface(len(sph), _ptr(sph), len(tor), _ptr(tor), _ptr(uu), n, int(max_steps), float(delta),
                               float(margin_box), float(margin_sdf), _ptr(pts), _ptr(hit), _ptr(marg))
    return dict(points=pts, hit=hit.astype(bool), marginal=marg.astype(bool))


def training_points(spheres, tori, surface_pts, uni, sigma: float = 0.01):
    """2:2:1 surface/near/uniform training set (see orc_training_points).
    surface_pts: [3][ns] float64, uni: [4][N] float32.  Returns float32
    points [3][N] and float64 targets [N]."""
    sph, tor = _shape_arrays(spheres, tori)
    S = _c(surface_pts, np.float64)
    un = _c(uni, np.float32)
    N = un.shape[1]
    xs = np.zeros((3, N), np.float32)
    tg = np.zeros(N)
    rc = _load().orc_training_points(len(sph), _ptr(sph), len(tor), _ptr(tor), _ptr(S), S.shape[1], _ptr(un), N,
                                     float(sigma), _ptr(xs), _ptr(tg))
    if rc != 0:
        raise ValueError("oracle training_points: no surface samples")
    return xs, tg


def adam_step(params, grads, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) in float64, in
    place on lists of arrays: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
    c1 = 1.0 / (1.0 - beta1 ** step)
    c2 = 1.0 / (1.0 - beta2 ** step)
    for th, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1.0 - beta1) * g
        vv *= beta2
        vv += (1.0 - beta2) * g * g
        th -= lr * (mm * c1) / (np.sqrt(vv * c2) + eps)

