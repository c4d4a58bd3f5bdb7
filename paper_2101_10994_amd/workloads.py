"""Seeded synthetic inputs for the neural-SDF octree path.

This module produces *inputs only*: analytic shapes (unions of spheres and
tori), the finest-level occupancy they induce, query points, training
targets, camera descriptions, random rays and randomly initialised
parameters.  It contains none of the method's own arithmetic (no octree
construction, no traversal, no interpolation, no decoder), so it can feed
both the GPU library and the CPU oracle without coupling them.

Shapes stand in for the paper's meshes (ShapeNet / Thingi / TurboSquid,
Section 4.1), which are not available; the recipes:

* occupancy: a finest voxel is occupied iff |SDF(centre)| is strictly below
  the voxel diagonal (a voxel exists only where there is surface, Sec. 3.2);
* features ~ N(0, 0.01^2) (App. A.1); decoder weights and biases
  ~ N(0, 1/fan_in);
* query points: uniform in [-1,1]^3, surface samples and surface samples
  perturbed by N(0, 0.01^2) (App. A.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Independent random streams per input kind (numpy SeedSequence.spawn).
STREAM_SHAPE, STREAM_FEAT, STREAM_DEC, STREAM_QUERY, STREAM_CAMERA, STREAM_EXTRA = range(6)


def rngs(seed: int, n: int = 6) -> List[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


# --------------------------------------------------------------------------
# Analytic shapes (exact SDFs of the primitives; union = min)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Shape:
    spheres: np.ndarray  # [ns, 4]  cx cy cz R
    tori: np.ndarray     # [nt, 6]  cx cy cz R r axis(0=x,1=y,2=z)

    def sdf(self, p: np.ndarray) -> np.ndarray:
        """Exact signed distance of the union (float64), p: [n, 3]."""
        p = np.asarray(p, dtype=np.float64)
        out = np.full(p.shape[0], np.inf)
        for cx, cy, cz, rad in self.spheres:
            q = p - np.array([cx, cy, cz])
            out = np.minimum(out, np.sqrt((q * q).sum(1)) - rad)
        for cx, cy, cz, big, small, axis in self.tori:
            q = p - np.array([cx, cy, cz])
            a = int(axis)
            ax = [(1, 2), (0, 2), (0, 1)][a]
            ring = np.sqrt(q[:, ax[0]] ** 2 + q[:, ax[1]] ** 2) - big
            out = np.minimum(out, np.sqrt(ring * ring + q[:, a] ** 2) - small)
        return out

    def surface_area(self):
        sa = [4 * math.pi * r * r for r in self.spheres[:, 3]]
        ta = [4 * math.pi * math.pi * big * small for big, small in self.tori[:, 3:5]]
        return np.array(sa + ta, dtype=np.float64)


def sphere_shape(radius=0.6, centre=(0.0, 0.0, 0.0)) -> Shape:
    return Shape(np.array([[*centre, radius]], dtype=np.float64), np.zeros((0, 6)))


def random_union(rng: np.random.Generator, n_spheres: int, n_tori: int,
                 fixed_torus: Optional[tuple] = None) -> Shape:
    """Seeded union: sphere radii U[0.1,0.4], centres U[-0.6,0.6]^3; random tori
    with centre U[-0.6,0.6]^3, R~U[0.2,0.5], r~U[0.05,0.15], axis in {x,y,z}."""
    sph = np.zeros((n_spheres, 4))
    sph[:, :3] = rng.uniform(-0.6, 0.6, size=(n_spheres, 3))
    sph[:, 3] = rng.uniform(0.1, 0.4, size=n_spheres)
    tor = []
    if fixed_torus is not None:
        tor.append(list(fixed_torus))
    for _ in range(n_tori):
        c = rng.uniform(-0.6, 0.6, size=3)
        tor.append([*c, rng.uniform(0.2, 0.5), rng.uniform(0.05, 0.15), float(rng.integers(0, 3))])
    return Shape(sph, np.array(tor, dtype=np.float64).reshape(-1, 6))


def occupancy_ijk(shape: Shape, res: int) -> np.ndarray:
    """Finest-level occupied cells: |SDF(centre)| < sqrt(3)*(2/res), strict, float64.

    Candidates are pruned coarse-to-fine with the 1-Lipschitz bound of the
    union SDF (a coarse cell is dropped only if no finer centre inside it can
    pass the test), then the exact rule is applied to every survivor.
    Returns int32 [n, 3] (x, y, z cell indices), lexicographically sorted.
    """
    diag_f = math.sqrt(3.0) * 2.0 / res
    cells = np.zeros((1, 3), dtype=np.int64)
    r = 1
    while r < res:
        r *= 2
        # children of surviving cells at resolution r
        off = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.int64)
        cells = (cells[:, None, :] * 2 + off[None]).reshape(-1, 3)
        centre = -1.0 + (cells + 0.5) * (2.0 / r)
        d = np.abs(shape.sdf(centre))
        if r < res:
            half_diag_r = 0.5 * math.sqrt(3.0) * 2.0 / r
            keep = d < diag_f + half_diag_r + 1e-9
        else:
            keep = d < diag_f
        cells = cells[keep]
    if res == 1:
        centre = np.zeros((1, 3))
        cells = cells[np.abs(shape.sdf(centre)) < diag_f]
    order = np.lexsort((cells[:, 2], cells[:, 1], cells[:, 0]))
    return np.ascontiguousarray(cells[order].astype(np.int32))


# --------------------------------------------------------------------------
# Point samplers (App. A.2)
# --------------------------------------------------------------------------
def uniform_points(rng, n) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=(n, 3))


def points_in_cells(rng, ijk: np.ndarray, res: int, n: int) -> np.ndarray:
    """Uniform points inside uniformly chosen cells of an occupancy set."""
    pick = rng.integers(0, ijk.shape[0], size=n)
    u = rng.uniform(0.0, 1.0, size=(n, 3))
    return -1.0 + (ijk[pick].astype(np.float64) + u) * (2.0 / res)


def surface_points(rng, shape: Shape, n: int) -> np.ndarray:
    """Area-weighted samples on the primitives' surfaces, keeping only points on
    the union's boundary (|SDF_union| <= 1e-9)."""
    out = []
    area = shape.surface_area()
    prob = area / area.sum()
    ns = shape.spheres.shape[0]
    need = n
    while need > 0:
        m = max(2 * need, 1024)
        prim = rng.choice(len(prob), size=m, p=prob)
        pts = np.zeros((m, 3))
        for k in np.unique(prim):
            sel = prim == k
            cnt = int(sel.sum())
            if k < ns:
                cx, cy, cz, rad = shape.spheres[k]
                v = rng.normal(size=(cnt, 3))
                v /= np.linalg.norm(v, axis=1, keepdims=True)
                pts[sel] = np.array([cx, cy, cz]) + rad * v
            else:
                cx, cy, cz, big, small, axis = shape.tori[k - ns]
                # area element of a torus ~ (R + r cos v): rejection-sample v
                uu = rng.uniform(0, 2 * math.pi, size=cnt)
                vv = np.empty(cnt)
                filled = 0
                while filled < cnt:
                    cand = rng.uniform(0, 2 * math.pi, size=2 * cnt)
                    acc = rng.uniform(0, 1, size=2 * cnt) < (big + small * np.cos(cand)) / (big + small)
                    cand = cand[acc][: cnt - filled]
                    vv[filled:filled + cand.size] = cand
                    filled += cand.size
                ring = big + small * np.cos(vv)
                local = np.stack([ring * np.cos(uu), ring * np.sin(uu), small * np.sin(vv)], 1)
                a = int(axis)
                ax = [(1, 2), (0, 2), (0, 1)][a]
                world = np.zeros_like(local)
                # local z is the torus axis (world axis a); the ring lies in
                # the plane of the other two axes, as in Shape.sdf
                world[:, ax[0]] = local[:, 0]
                world[:, ax[1]] = local[:, 1]
                world[:, a] = local[:, 2]
                pts[sel] = np.array([cx, cy, cz]) + world
        keep = np.abs(shape.sdf(pts)) <= 1e-9
        keep &= np.all(np.abs(pts) <= 1.0, axis=1)
        pts = pts[keep][:need]
        out.append(pts)
        need -= pts.shape[0]
    return np.concatenate(out, 0)


def near_points(rng, shape: Shape, n: int, sigma: float = 0.01) -> np.ndarray:
    """Surface samples plus isotropic N(0, sigma^2) offsets, resampled until
    they fall inside [-1,1]^3."""
    out = np.zeros((0, 3))
    while out.shape[0] < n:
        m = n - out.shape[0]
        p = surface_points(rng, shape, m) + rng.normal(0.0, sigma, size=(m, 3))
        p = p[np.all(np.abs(p) <= 1.0, axis=1)]
        out = np.concatenate([out, p], 0)
    return out[:n]


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
def features(rng, ncorner_per_lod, m: int, sigma: float = 0.01) -> List[np.ndarray]:
    """Corner features per feature level, N(0, sigma^2), float64 [nc, m]."""
    return [rng.normal(0.0, sigma, size=(int(nc), m)) for nc in ncorner_per_lod]


def decoders(rng, num_lods: int, din: int, hidden: int):
    """Per-LOD one-hidden-layer decoders, weights and biases ~ N(0, 1/fan_in).
    W1: [L][hidden][din] (input order: x, y, z, then features), b1: [L][hidden],
    w2: [L][hidden], b2: [L]."""
    s1 = 1.0 / math.sqrt(din)
    s2 = 1.0 / math.sqrt(hidden)
    return dict(
        W1=rng.normal(0.0, s1, size=(num_lods, hidden, din)),
        b1=rng.normal(0.0, s1, size=(num_lods, hidden)),
        w2=rng.normal(0.0, s2, size=(num_lods, hidden)),
        b2=rng.normal(0.0, s2, size=(num_lods,)),
    )


def embedded_features(rng, shape: Shape, corner_pos_per_lod, m: int, sigma: float = 0.01):
    """'SDF-embedded' features for timed renders: at level l (1-based) channel
    l-1 holds the exact SDF at the level's corners, the same channel is zero on
    every other level, and all remaining channels are N(0, sigma^2)."""
    L = len(corner_pos_per_lod)
    assert m >= L
    out = []
    for lvl, pos in enumerate(corner_pos_per_lod):
        f = rng.normal(0.0, sigma, size=(pos.shape[0], m))
        f[:, :L] = 0.0
        f[:, lvl] = shape.sdf(pos)
        out.append(f)
    return out


def embedded_decoders(rng, num_lods: int, m: int, hidden: int, with_xyz: bool = True):
    """Decoders whose output is channel L-1 of the summed feature: hidden units
    0 and 1 are ReLU(+z) and ReLU(-z) of that channel with output weights +1/-1;
    all other hidden units keep random first-layer weights but have zero output
    weight, so the full first layer is still evaluated."""
    din = m + (3 if with_xyz else 0)
    off = 3 if with_xyz else 0
    d = decoders(rng, num_lods, din, hidden)
    for L in range(num_lods):
        d["W1"][L, 0, :] = 0.0
        d["W1"][L, 1, :] = 0.0
        d["W1"][L, 0, off + L] = 1.0
        d["W1"][L, 1, off + L] = -1.0
        d["b1"][L, :2] = 0.0
        d["w2"][L, :] = 0.0
        d["w2"][L, 0] = 1.0
        d["w2"][L, 1] = -1.0
        d["b2"][L] = 0.0
    return d


def spread_decoders(rng, num_lods: int, m: int, hidden: int, with_xyz: bool = True, noise: float = 0.05):
    """Decoders that read channel L-1 of the summed feature like
    embedded_decoders, but through every hidden unit: units come in pairs
    (u_k, -u_k) with output weights (+c_k, -c_k), so the pair contributes
    c_k (ReLU(u_k) - ReLU(-u_k)) = c_k u_k.  Each u_k = a_k z_{L-1} + r_k .
    [x, z_other] + b_k has random weights on every input; the last pair's
    r and b are chosen so that sum_k c_k r_k = 0 and sum_k c_k b_k = 0, and
    sum_k c_k a_k = 1, so in exact arithmetic the output is z_{L-1} (and
    b2 = 0).  The cancellation spreads the result over all hidden units
    with terms much larger than the output, so the accumulation order and
    the rounding of the weights, positions and features reach the result.
    Returns float64 arrays with the layout of decoders()."""
    din = m + (3 if with_xyz else 0)
    off = 3 if with_xyz else 0
    K = hidden // 2
    W1 = np.zeros((num_lods, hidden, din))
    b1 = np.zeros((num_lods, hidden))
    w2 = np.zeros((num_lods, hidden))
    for L in range(num_lods):
        c = rng.uniform(0.5, 1.5, size=K) * rng.choice([-1.0, 1.0], size=K) / K
        a = rng.uniform(0.5, 1.5, size=K) * np.sign(c)
        a /= float(np.dot(c, a))
        r = rng.normal(0.0, noise, size=(K, din))
        r[:, off + L] = 0.0
        b = rng.normal(0.0, noise, size=K)
        r[K - 1] = -np.dot(c[:K - 1], r[:K - 1]) / c[K - 1]
        b[K - 1] = -np.dot(c[:K - 1], b[:K - 1]) / c[K - 1]
        u = r.copy()
        u[:, off + L] = a
        W1[L, 0::2] = u
        W1[L, 1::2] = -u
        b1[L, 0::2] = b
        b1[L, 1::2] = -b
        w2[L, 0::2] = c
        w2[L, 1::2] = -c
    return dict(W1=W1, b1=b1, w2=w2, b2=np.zeros(num_lods))


# --------------------------------------------------------------------------
# Cameras and rays
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    eye: tuple
    target: tuple = (0.0, 0.0, 0.0)
    up: tuple = (0.0, 1.0, 0.0)
    fov_y_deg: float = 45.0
    width: int = 64
    height: int = 64


def camera_on_sphere(rng, radius: float, width: int, height: int) -> Camera:
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    if abs(v[1]) > 0.95:  # keep away from the up vector
        v[1] = 0.95 * np.sign(v[1])
        v /= np.linalg.norm(v)
    return Camera(eye=tuple(float(a) for a in radius * v), width=width, height=height)


def random_rays(rng, n: int, origin_radius=(1.2, 3.0), aim_radius=0.9):
    """Rays from origins on a shell outside the box, aimed at random points
    inside it; directions normalised in float64 then rounded to float32.
    Returns (o [3][n], d [3][n]) float32 SoA."""
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    o = v * rng.uniform(*origin_radius, size=(n, 1))
    tgt = rng.uniform(-aim_radius, aim_radius, size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return (np.ascontiguousarray(o.T.astype(np.float32)), np.ascontiguousarray(d.T.astype(np.float32)))


def axis_rays(rng, n: int, res: int):
    """Axis-parallel rays along +/-x, +/-y, +/-z through the centres of random
    columns of a resolution-`res` grid, starting outside the box."""
    axis = rng.integers(0, 3, size=n)
    sign = rng.choice([-1.0, 1.0], size=n)
    cols = rng.integers(0, res, size=(n, 3))
    o = -1.0 + (cols + 0.5) * (2.0 / res)
    d = np.zeros((n, 3))
    for k in range(n):
        o[k, axis[k]] = -1.5 * sign[k]
        d[k, axis[k]] = sign[k]
    return (np.ascontiguousarray(o.T.astype(np.float32)), np.ascontiguousarray(d.T.astype(np.float32)))


# --------------------------------------------------------------------------
# Configurations
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Config:
    name: str
    num_lods: int
    feat_dim: int
    hidden: int
    n_query: int
    width: int
    height: int
    max_steps: int
    delta: float
    eye: tuple = (0.0, 0.0, 2.5)
    query_lod: int = 0          # 0 -> num_lods
    feat_dtype: str = "f32"
    w_dtype: str = "f32"


TINY = Config("tiny-sphere-3lod-m8", 3, 8, 32, 4096, 64, 64, 32, 3e-4)
PAPER = Config("union8s1t-5lod-m32", 5, 32, 128, 1 << 20, 1024, 1024, 100, 1e-4,
               eye=(0.9, 0.6, 2.2))
TRAIN = Config("union8s1t-5lod-m32-train", 5, 32, 128, 1 << 19, 0, 0, 0, 0.0)
PREC = Config("union32s4t-7lod-m32-half", 7, 32, 128, 1 << 22, 1920, 1080, 100, 1e-4,
              eye=(0.9, 0.6, 2.2), query_lod=5, feat_dtype="f16", w_dtype="bf16")


def tiny_shape() -> Shape:
    return sphere_shape(0.6)


def paper_shape(seed: int = 0) -> Shape:
    r = rngs(seed)[STREAM_SHAPE]
    return random_union(r, 8, 0, fixed_torus=(0.0, 0.0, 0.0, 0.5, 0.15, 2.0))


def prec_shape(seed: int = 0) -> Shape:
    r = rngs(seed)[STREAM_SHAPE]
    return random_union(r, 32, 4)


def paper_queries(seed: int, shape: Shape, n: int) -> np.ndarray:
    """Half uniform in the box, half surface samples + N(0, 0.01^2)."""
    r = rngs(seed)[STREAM_QUERY]
    nu = n // 2
    p = np.concatenate([uniform_points(r, nu), near_points(r, shape, n - nu)], 0)
    return p[r.permutation(n)]


def train_points(seed: int, shape: Shape, n: int):
    """1/3 uniform, 2/3 near-surface (sigma 0.01); targets = exact union SDF."""
    r = rngs(seed)[STREAM_QUERY]
    nu = n // 3
    p = np.concatenate([uniform_points(r, nu), near_points(r, shape, n - nu)], 0)
    p = p[r.permutation(n)]
    p32 = p.astype(np.float32)
    return p32, shape.sdf(p32.astype(np.float64)).astype(np.float32)


def soa(p: np.ndarray, dtype=np.float32) -> np.ndarray:
    """[n,3] -> contiguous [3][n]."""
    return np.ascontiguousarray(np.asarray(p).T.astype(dtype))


# --------------------------------------------------------------------------
# Batched rendering: 16 seeded shapes with 3..7 LODs
# --------------------------------------------------------------------------
BATCH = Config("batch16-3to7lod-m32-half", 0, 32, 128, 0, 512, 512, 100, 1e-4, feat_dtype="f16", w_dtype="bf16")


def batch_scene(seed: int = 0, n: int = 16, width: int = 512, height: int = 512):
    """n seeded sphere/torus unions; shape s has 3 + s % 5 LODs, a camera on a
    radius-3 sphere looking at the origin, and renders at LOD num_lods - s % 2.
    Returns a list of dicts (shape, num_lods, camera, lod)."""
    r = rngs(seed)
    out = []
    for s in range(n):
        L = 3 + s % 5
        shape = random_union(r[STREAM_SHAPE], 2 + s % 5, 1 + s % 2)
        cam = camera_on_sphere(r[STREAM_CAMERA], 3.0, width, height)
        out.append(dict(shape=shape, num_lods=L, camera=cam, lod=max(1, L - s % 2)))
    return out
