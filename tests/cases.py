"""Shared test cases: one set of seeded parameters, stored in the precision
the GPU reads them, handed to both the GPU library and the oracle (which
reads the same stored values in float64)."""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
from paper_2101_10994_amd import workloads as W

try:
    import torch
except Exception:  # pragma: no cover
    torch = None


@dataclasses.dataclass
class Case:
    ijk: np.ndarray
    L: int
    m: int
    H: int
    with_xyz: bool
    feats: list      # stored values, float64 arrays
    W1: list
    b1: list
    w2: list
    b2: np.ndarray
    feat_dtype: str = "f32"
    w_dtype: str = "f32"
    shape: object = None
    otree: object = None

    def oracle_model(self):
        return oracle.Model(self.feats, self.W1, self.b1, self.w2, self.b2, with_xyz=self.with_xyz)

    def gpu_model(self, device="cuda"):
        from paper_2101_10994_amd import ngl
        tree = ngl.Octree(self.ijk, self.L, device=device)
        fd = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
        feats = [torch.tensor(f, dtype=torch.float64).to(fd[self.feat_dtype]).to(device) for f in self.feats]
        W1 = [torch.tensor(w, dtype=torch.float64).to(fd[self.w_dtype]).to(device) for w in self.W1]
        f32 = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=device)
        return ngl.Model(tree, feats, W1, [f32(b) for b in self.b1], [f32(w) for w in self.w2], f32(self.b2),
                         with_xyz=self.with_xyz)


def _round(a, dtype):
    """Round float64 values to a storage dtype and back (exactly representable)."""
    if dtype == "f32":
        return np.asarray(a, np.float32).astype(np.float64)
    if dtype == "f16":
        return np.asarray(a, np.float16).astype(np.float64)
    if dtype == "bf16":
        t = torch.tensor(np.asarray(a), dtype=torch.float64).to(torch.bfloat16)
        return t.to(torch.float64).numpy()
    raise ValueError(dtype)


def make_case(shape, res, L, m, H, seed=0, sigma=0.01, with_xyz=True, feat_dtype="f32", w_dtype="f32",
              embedded=False, spread=False):
    """embedded: SDF-embedded features with the two-unit embedded decoder;
    spread: the same features read through every hidden unit
    (workloads.spread_decoders)."""
    ijk = W.occupancy_ijk(shape, res)
    otree = oracle.Octree(ijk, L)
    rs = W.rngs(seed)
    if embedded or spread:
        feats = W.embedded_features(rs[W.STREAM_FEAT], shape, otree.corner_positions(), m, sigma)
        if spread:
            dec = W.spread_decoders(rs[W.STREAM_DEC], L, m, H, with_xyz)
        else:
            dec = W.embedded_decoders(rs[W.STREAM_DEC], L, m, H, with_xyz)
    else:
        feats = W.features(rs[W.STREAM_FEAT], otree.ncorner, m, sigma)
        dec = W.decoders(rs[W.STREAM_DEC], L, m + (3 if with_xyz else 0), H)
    return Case(ijk=ijk, L=L, m=m, H=H, with_xyz=with_xyz,
                feats=[_round(f, feat_dtype) for f in feats],
                W1=[_round(w, w_dtype) for w in dec["W1"]],
                b1=[_round(b, "f32") for b in dec["b1"]],
                w2=[_round(w, "f32") for w in dec["w2"]],
                b2=_round(dec["b2"], "f32"), feat_dtype=feat_dtype, w_dtype=w_dtype, shape=shape, otree=otree)


def tiny_case(**kw):
    return make_case(W.tiny_shape(), 16, 3, 8, 32, **kw)


def paper_case(**kw):
    return make_case(W.paper_shape(0), 64, 5, 32, 128, **kw)


def edge_points(ijk, res, L, rng, n_in=4096, n_uniform=1024):
    """Points inside occupied finest cells, uniform points, lattice points of
    every level and their float32 neighbours, the box corners and a few
    points outside the box."""
    pts = [W.points_in_cells(rng, ijk, res, n_in), W.uniform_points(rng, n_uniform)]
    for lvl in range(1, L + 1):
        r = 2 ** (lvl + 1)
        pts.append(-1.0 + rng.integers(0, r + 1, size=(64, 3)) * (2.0 / r))
    p = np.concatenate(pts, 0).astype(np.float32)
    lat = p[n_in + n_uniform:]
    p = np.concatenate([p, np.nextafter(lat, np.float32(-2)), np.nextafter(lat, np.float32(2)),
                        np.array([[1, 1, 1], [-1, -1, -1], [1, -1, 1], [1.5, 0, 0], [0, -1.25, 0]], np.float32)])
    return W.soa(p)
