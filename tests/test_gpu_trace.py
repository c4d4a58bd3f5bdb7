"""GPU parity: adaptive-stepping sphere tracing (Sec. 3.4, Fig. 3; App. A.4)
against the FP64 oracle on the same hit lists.  Several stopping points are
correct (any t in the delta band), so the comparison is toleranced: hit/miss
must agree on every ray the oracle does not flag as marginal, and hit
distances agree to a small fraction of the finest voxel."""
import numpy as np
import pytest

import oracle
from paper_2101_10994_amd import workloads as W

from cases import make_case, paper_case, tiny_case
from tracecmp import check, report, summary, trace_both

pytestmark = pytest.mark.gpu


def test_analytic_sphere_matches_oracle_and_closed_form():
    case = tiny_case()
    g, r = trace_both(case, (0.3, 0.2, 2.5), 128, 128, 3, 0.0, 200, 3e-4, analytic=(0, 0, 0, 0.6))
    nhit, _ = check(g, r, 2 / 16)
    assert nhit > 4000


def test_tiny_random_model(f32_decoder):
    case = tiny_case(sigma=0.1)
    g, r = trace_both(case, (0.0, 0.0, 2.5), 64, 64, 3, 0.0, 32, 3e-4)
    check(g, r, 2 / 16)


def test_tiny_embedded_model_all_lods(f32_decoder):
    case = make_case(W.tiny_shape(), 16, 3, 8, 32, embedded=True)
    for lod in (1, 2, 3):
        g, r = trace_both(case, (0.4, -0.3, 2.4), 96, 80, lod, 0.0, 100, 3e-4)
        nhit, _ = check(g, r, 2 / 16)
        assert nhit > 1000
    g, r = trace_both(case, (0.4, -0.3, 2.4), 96, 80, 2, 0.45, 100, 3e-4)
    check(g, r, 2 / 16)


def test_paper_scale_embedded_sampled(f32_decoder):
    """1024x1024 render of the 5-LOD union on the GPU; 32,768 sampled rays
    traced by the oracle."""
    case = make_case(W.paper_shape(0), 64, 5, 32, 128, embedded=True)
    idx = np.random.default_rng(0).choice(1024 * 1024, 32768, replace=False)
    g, r = trace_both(case, W.PAPER.eye, 1024, 1024, 5, 0.0, 100, 1e-4, sample=idx)
    # ~10 steps per ray across 1/32-wide voxels: about 1-2% of rays have a
    # step within 1e-5 of a voxel bound
    nhit, nmarg = check(g, r, 2 / 64, max_marginal=0.03)
    report("trace_paper_embedded_f32_%s" % ["valu", "mfma"][f32_decoder], summary(g, r, 2 / 64))
    assert nhit > 10000


def test_paper_scale_spread_decoder_sampled(f32_decoder):
    """1024x1024 render of the 5-LOD union through a decoder whose output
    depends on every hidden unit (workloads.spread_decoders), FP32 weights:
    32,768 sampled rays traced by the oracle.  Unlike the embedded decoder,
    the accumulation order of the first and second layers reaches the
    result here."""
    case = make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True)
    idx = np.random.default_rng(4).choice(1024 * 1024, 32768, replace=False)
    g, r = trace_both(case, W.PAPER.eye, 1024, 1024, 5, 0.0, 100, 1e-4, sample=idx)
    nhit, nmarg = check(g, r, 2 / 64, max_marginal=0.03)
    report("trace_paper_spread_f32_%s" % ["valu", "mfma"][f32_decoder], summary(g, r, 2 / 64))
    assert nhit > 10000


def test_paper_scale_spread_decoder_bf16_sampled():
    """As above with FP16 features and BF16 weights on the matrix cores,
    blended (L = 4 + 0.35) and at LOD 5."""
    case = make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True, feat_dtype="f16", w_dtype="bf16")
    for lod, alpha in ((5, 0.0), (4, 0.35)):
        idx = np.random.default_rng(5 + lod).choice(1024 * 1024, 16384, replace=False)
        g, r = trace_both(case, W.PAPER.eye, 1024, 1024, lod, alpha, 100, 1e-4, sample=idx)
        nhit, nmarg = check(g, r, 2 / 64, max_marginal=0.03)
        report("trace_paper_spread_bf16_lod%d_a%g" % (lod, alpha), summary(g, r, 2 / 64))
        assert nhit > 4000


def test_stop_rules_and_invalid_rays():
    import torch
    from paper_2101_10994_amd import ngl
    case = tiny_case()
    gm = case.gpu_model()
    o, d = ngl.camera_rays((0, 0, 2.5), (0, 0, 0), (0, 1, 0), 45.0, 16, 16)
    hits = ngl.trace_octree(gm, o, d, 4)
    has = (hits["ray_off"][1:] > hits["ray_off"][:-1]).cpu().numpy()
    g0 = ngl.sphere_trace(gm, o, d, 3, 0.0, hits, 0, 3e-4)
    st = g0["status"].cpu().numpy()
    assert np.all(st[has] == ngl.MAX_STEPS) and np.all(st[~has] == ngl.MISS)
    gf = ngl.sphere_trace(gm, o, d, 3, 0.0, hits, 100, 3e-4, t_far=0.5, analytic_sphere=(0, 0, 0, 0.6))
    assert np.all(gf["status"].cpu().numpy()[has] == ngl.FAR)
    o2 = o.clone()
    o2[0, 5] = float("nan")
    gi = ngl.sphere_trace(gm, o2, d, 3, 0.0, hits, 10, 3e-4)
    assert int(gi["status"][5]) == ngl.INVALID


def test_bf16_decoder_embedded_trace():
    """FP16 features + BF16 decoder on the matrix cores, tiny and paper-scale
    (sampled) renders against the oracle on the same stored parameters."""
    case = make_case(W.tiny_shape(), 16, 3, 8, 32, embedded=True, feat_dtype="f16", w_dtype="bf16")
    for lod, alpha in ((3, 0.0), (2, 0.45)):
        g, r = trace_both(case, (0.4, -0.3, 2.4), 96, 80, lod, alpha, 100, 3e-4)
        check(g, r, 2 / 16)
    case = make_case(W.paper_shape(0), 64, 5, 32, 128, embedded=True, feat_dtype="f16", w_dtype="bf16")
    idx = np.random.default_rng(3).choice(1024 * 1024, 16384, replace=False)
    g, r = trace_both(case, W.PAPER.eye, 1024, 1024, 5, 0.0, 100, 1e-4, sample=idx)
    nhit, nmarg = check(g, r, 2 / 64, max_marginal=0.03)
    report("trace_paper_embedded_bf16_lod5", summary(g, r, 2 / 64))


PHASE_CASES = {
    "m32-f32": lambda: make_case(W.paper_shape(0), 64, 5, 32, 128, embedded=True),
    "m32-bf16": lambda: make_case(W.paper_shape(0), 64, 5, 32, 128, embedded=True, feat_dtype="f16",
                                  w_dtype="bf16"),
    "m8": lambda: make_case(W.paper_shape(0), 32, 4, 8, 32, embedded=True),
    "m16-bf16": lambda: make_case(W.paper_shape(0), 32, 4, 16, 32, embedded=True, feat_dtype="bf16",
                                  w_dtype="bf16"),
    "m64": lambda: make_case(W.paper_shape(0), 32, 4, 64, 64, embedded=True, with_xyz=False),
    "m32-spread-bf16": lambda: make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True, feat_dtype="f16",
                                         w_dtype="bf16"),
}


@pytest.mark.parametrize("name", list(PHASE_CASES))
def test_phased_trace_is_bitwise_the_single_launch(name, f32_decoder):
    """The phased tracer parks rays still running at the pause counts and
    resumes them from their saved state, the last phase optionally with a
    group of lanes per ray: every output equals the single launch's, bit for
    bit, for any pause counts (blended LODs too)."""
    import torch
    from paper_2101_10994_amd import ngl
    case = PHASE_CASES[name]()
    gm = case.gpu_model()
    L = gm.num_lods
    o, d = ngl.camera_rays(W.PAPER.eye, (0, 0, 0), (0, 1, 0), 45.0, 384, 384)
    keys = (ngl.OPT_TRACE_PAUSE1, ngl.OPT_TRACE_PAUSE2, ngl.OPT_TRACE_WIDE)
    old = [ngl.get_option(k) for k in keys]
    try:
        for lod, alpha in ((L, 0.0), (L - 2, 0.4)):
            hits = ngl.trace_octree(gm, o, d, (lod + 1 if alpha > 0 else lod) + 1)
            ref = ngl.sphere_trace(gm, o, d, lod, alpha, hits, 100, 1e-4, phased=False)
            st = ref["steps"].cpu().numpy()
            assert (st > 8).sum() > 50  # some rays are parked
            for cfg in ((16, 0, 1), (16, 40, 0), (16, 40, 1), (1, 2, 1), (8, 0, 0), (0, 30, 1), (99, 0, 1),
                        (5, 5, 1), (2, 0, 1)):
                for k, v in zip(keys, cfg):
                    ngl.set_option(k, v)
                g = ngl.sphere_trace(gm, o, d, lod, alpha, hits, 100, 1e-4)
                assert g["ws"].numel() > 256
                for key in ("t", "status", "steps", "hit_vox"):
                    assert torch.equal(g[key], ref[key]), (lod, alpha, cfg, key)
    finally:
        for k, v in zip(keys, old):
            ngl.set_option(k, v)


@pytest.mark.parametrize("name", ["m32-f32", "m32-spread-bf16", "m8"])
def test_tile_order_is_bitwise_the_ray_order(name, f32_decoder):
    """Serving an image's rays in 8x8 pixel tiles (image_width > 0) changes
    only which rays share a wavefront: every output is the same bits, one
    phase or phased, blended or not; widths that do not tile are rejected."""
    import torch
    from paper_2101_10994_amd import ngl
    gm = PHASE_CASES[name]().gpu_model()
    L = gm.num_lods
    o, d = ngl.camera_rays(W.PAPER.eye, (0, 0, 0), (0, 1, 0), 45.0, 384, 256)
    for lod, alpha in ((L, 0.0), (L - 2, 0.4)):
        hits = ngl.trace_octree(gm, o, d, (lod + 1 if alpha > 0 else lod) + 1)
        for phased in (False, True):
            ref = ngl.sphere_trace(gm, o, d, lod, alpha, hits, 100, 1e-4, phased=phased)
            got = ngl.sphere_trace(gm, o, d, lod, alpha, hits, 100, 1e-4, phased=phased, image_width=384)
            for key in ("t", "status", "steps", "hit_vox"):
                assert torch.equal(got[key], ref[key]), (lod, alpha, phased, key)
    for bad in (100, 388, -8, 96 * 5):
        with pytest.raises(ngl.NGLError):
            ngl.sphere_trace(gm, o, d, L, 0.0, hits, 100, 1e-4, image_width=bad)
