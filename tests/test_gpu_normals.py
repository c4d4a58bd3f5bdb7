"""GPU parity: finite-difference surface normals (App. A.4) against the
FP64 oracle on the same float32 points (or the same rays and hit
distances).  Each difference quotient inherits the query bound of its two
probes: |dg_a| <= (tol * (s+ + s-) + 2^-22 (|f+| + |f-|)) / (2h), and a unit
vector moves by at most 2 |dg| / |g|."""
import numpy as np
import pytest

import oracle
from paper_2101_10994_amd import workloads as W

from cases import edge_points, make_case, paper_case, tiny_case

pytestmark = pytest.mark.gpu
TOL = 1e-5
TOL16 = 5e-5  # BF16 weights: the query bound against s1 (BF16 bars of the query tests)


def check(n_gpu, o, h, tol=TOL, scale="scale"):
    n_gpu = n_gpu.astype(np.float64)
    act = o["active"]
    assert np.all(n_gpu[:, ~act] == 0.0)
    h32 = float(np.float32(h))
    dg = (tol * o[scale] + 2.0 ** -22 * o["fsum"]) / (2.0 * h32)
    dgn = np.sqrt((dg * dg).sum(0))
    gn = np.sqrt((o["g"] ** 2).sum(0))
    bound = np.where(gn > 0, 2.0 * dgn / np.maximum(gn, 1e-300), 2.0) + 2e-6
    err = np.sqrt(((n_gpu - o["n"]) ** 2).sum(0))
    bad = np.nonzero(act & (err > bound))[0]
    assert bad.size == 0, (bad[:10], err[bad[:10]], bound[bad[:10]])
    unit = act & (gn > 0)
    np.testing.assert_allclose(np.sqrt((n_gpu[:, unit] ** 2).sum(0)), 1.0, atol=2e-6)
    return float(np.median(err[act])) if act.any() else 0.0


def points_both(case, x, lod, alpha, h):
    import torch
    from paper_2101_10994_amd import ngl
    gm = case.gpu_model()
    n = ngl.sdf_normals(gm, lod, alpha, h, x=torch.from_numpy(x).cuda()).cpu().numpy()
    o = oracle.normals(case.otree, case.oracle_model(), lod, alpha, h, x_soa=x)
    return n, o


@pytest.mark.parametrize("lod", [1, 2, 3])
def test_tiny_points(lod, f32_decoder):
    case = tiny_case(sigma=0.1)
    x = edge_points(case.ijk, 16, 3, np.random.default_rng(lod))
    h = 2.0 ** -7
    n, o = points_both(case, x, lod, 0.0, h)
    check(n, o, h)


def test_tiny_blend_and_small_step(f32_decoder):
    case = tiny_case(sigma=0.2)
    x = edge_points(case.ijk, 16, 3, np.random.default_rng(11))
    for h in (2.0 ** -7, 1e-3):
        n, o = points_both(case, x, 2, 0.37, h)
        check(n, o, h)


@pytest.mark.parametrize("fdt,wdt", [("f16", "f32"), ("bf16", "f32"), ("f32", "bf16"), ("bf16", "bf16")])
def test_tiny_half_precision(fdt, wdt):
    case = tiny_case(sigma=0.1, feat_dtype=fdt, w_dtype=wdt)
    x = edge_points(case.ijk, 16, 3, np.random.default_rng(12))
    h = 2.0 ** -7
    n, o = points_both(case, x, 3, 0.0, h)
    if wdt == "bf16":
        check(n, o, h, TOL16, "scale1")
    else:
        check(n, o, h)


def hits_of(case, eye, width, height, lod, alpha, sample_every=1):
    """Oracle camera rays and oracle sphere-trace hits (float32 distances)."""
    co, cd = oracle.camera_rays(eye, (0, 0, 0), (0, 1, 0), 45.0, width, height)
    o = np.ascontiguousarray(co.astype(np.float32)[:, ::sample_every])
    d = np.ascontiguousarray(cd.astype(np.float32)[:, ::sample_every])
    depth = (lod + 1 if alpha > 0 else lod) + 1
    oh = oracle.trace_octree(case.otree, o, d, depth)
    r = oracle.sphere_trace(case.otree, case.oracle_model(), o, d, lod, alpha, oh, 128, 3e-4)
    return o, d, r["t"].astype(np.float32), r["status"]


def rays_both(case, rays, lod, alpha, h):
    import torch
    from paper_2101_10994_amd import ngl
    gm = case.gpu_model()
    o, d, t, st = rays
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (o, d, t, st)]
    n = ngl.sdf_normals(gm, lod, alpha, h, rays=tuple(dev)).cpu().numpy()
    on = oracle.normals(case.otree, case.oracle_model(), lod, alpha, h, rays=rays)
    return n, on


def test_paper_scale_hit_points(f32_decoder):
    """5 LODs at 64^3, SDF-embedded model, hit points of a camera frame."""
    case = paper_case(embedded=True)
    rays = hits_of(case, W.PAPER.eye, 192, 160, 5, 0.0, sample_every=3)
    assert (rays[3] == oracle.HIT).sum() > 3000
    h = 2.0 / 64 / 16
    n, o = rays_both(case, rays, 5, 0.0, h)
    check(n, o, h)
    # lower LOD with a blend, random features on top of the embedding
    case = paper_case(embedded=True, sigma=0.05)
    rays = hits_of(case, W.PAPER.eye, 128, 128, 3, 0.5, sample_every=2)
    n, o = rays_both(case, rays, 3, 0.5, h)
    check(n, o, h)


def test_empty_and_argument_errors():
    import torch
    from paper_2101_10994_amd import ngl
    case = tiny_case()
    gm = case.gpu_model()
    x = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    assert ngl.sdf_normals(gm, 2, x=x).shape == (3, 0)
    x = torch.zeros((3, 8), dtype=torch.float32, device="cuda")
    for kw in ({"lod": 0}, {"lod": 4}, {"lod": 3, "alpha": 0.5}, {"lod": 2, "h": 0.0}, {"lod": 2, "h": -1.0}):
        with pytest.raises(ngl.NGLError):
            ngl.sdf_normals(gm, x=x, **kw)
    n = ngl.sdf_normals(gm, 2, x=x)
    assert torch.isfinite(n).all()



NORMAL_CASES = {
    "m32-f32-spread": lambda: make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True),
    "m32-bf16-spread": lambda: make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True, feat_dtype="f16",
                                         w_dtype="bf16"),
    "m8": lambda: make_case(W.paper_shape(0), 32, 4, 8, 32, embedded=True),
    "m64": lambda: make_case(W.paper_shape(0), 32, 4, 64, 64, embedded=True, with_xyz=False),
}


@pytest.mark.parametrize("name", list(NORMAL_CASES))
def test_cooperative_normals_are_the_one_lane_bits(name, f32_decoder):
    """The cooperative normal kernel (each probe gathered tile-wise, four
    lanes per point) gives the bits of the one-lane-per-point kernel: hit
    points of a frame and scattered points (some outside the box), steps
    from far below to above a finest cell, discrete and blended LODs."""
    import torch
    from paper_2101_10994_amd import ngl
    gm = NORMAL_CASES[name]().gpu_model()
    L = gm.num_lods
    o, d = ngl.camera_rays(W.PAPER.eye, (0, 0, 0), (0, 1, 0), 45.0, 256, 192)
    rng = np.random.default_rng(11)
    x = torch.from_numpy(rng.uniform(-1.1, 1.1, (3, 20011)).astype(np.float32)).cuda()
    old = ngl.get_option(ngl.OPT_COOP_GATHER)
    try:
        for lod, alpha in ((L, 0.0), (L - 2, 0.4)):
            hits = ngl.trace_octree(gm, o, d, (lod + 1 if alpha > 0 else lod) + 1)
            tr = ngl.sphere_trace(gm, o, d, lod, alpha, hits, 100, 1e-4)
            assert int((tr["status"] == ngl.HIT).sum()) > 2000
            rays = (o, d, tr["t"], tr["status"])
            for h in (2.0 ** -14, 2.0 ** -9, 2.0 ** -5):
                got = {}
                for coop in (1, 0):
                    ngl.set_option(ngl.OPT_COOP_GATHER, coop)
                    got[coop] = (ngl.sdf_normals(gm, lod, alpha, h, rays=rays), ngl.sdf_normals(gm, lod, alpha, h, x=x))
                for a, b in zip(got[1], got[0]):
                    assert torch.equal(a, b), (lod, alpha, h)
    finally:
        ngl.set_option(ngl.OPT_COOP_GATHER, old)
