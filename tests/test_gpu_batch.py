"""Batched persistent rendering: several models (different octree depths,
cameras and LODs) traced by one launch.  Every view is checked against the
oracle directly (its own camera rays, hit lists and trace at the view's LOD
and alpha), and must equal the single-view path (camera rays, ray-octree
intersection, sphere trace) bit for bit; every ray must end, and the
per-view clocks must be ordered."""
import numpy as np
import pytest

from paper_2101_10994_amd import workloads as W

import oracle

from cases import make_case
from tracecmp import check, oracle_reference, report, summary

pytestmark = pytest.mark.gpu


def batch_cases():
    rs = W.rngs(11)
    shapes = [W.tiny_shape(), W.paper_shape(0), W.random_union(rs[0], 4, 1), W.random_union(rs[1], 6, 2)]
    lods = [3, 4, 2, 5]
    cases = []
    for s, L in zip(shapes, lods):
        cases.append(make_case(s, 2 ** (L + 1), L, 32, 128, embedded=True, feat_dtype="f16", w_dtype="bf16"))
    return cases


@pytest.mark.parametrize("alphas", [(0.0, 0.0, 0.0, 0.0), (0.0, 0.5, 0.0, 0.25)])
def test_batch_equals_single_view(alphas):
    import torch
    from paper_2101_10994_amd import ngl
    cases = batch_cases()
    models = [c.gpu_model() for c in cases]
    rng = np.random.default_rng(3)
    views = []
    for i, c in enumerate(cases):
        cam = W.camera_on_sphere(rng, 2.6, 96 + 16 * i, 80 + 8 * i)
        lod = c.L if alphas[i] == 0.0 else c.L - 1
        views.append(ngl.make_view(cam.eye, cam.width, cam.height, lod, alphas[i]))
    br = ngl.BatchRenderer(models, views, pair_capacity=1 << 20)
    br.status.fill_(255)
    br.render(100, 1e-4)
    torch.cuda.synchronize()
    assert not br.overflowed()
    assert int((br.status == 255).sum()) == 0
    fm = br.frame_ms()
    assert np.all(fm > 0)
    for i, (m, v) in enumerate(zip(models, views)):
        o, d = ngl.camera_rays(tuple(v.eye), (0, 0, 0), (0, 1, 0), 45.0, v.width, v.height)
        depth = (v.lod + 1 if v.alpha > 0 else v.lod) + 1
        hits = ngl.trace_octree(m, o, d, depth)
        single = ngl.sphere_trace(m, o, d, v.lod, v.alpha, hits, 100, 1e-4)
        sl = br.view_slice(i)
        for key, out in (("t", br.t), ("status", br.status), ("steps", br.steps), ("hit_vox", br.hit_vox)):
            a = single[key].cpu().numpy()
            b = out[sl].cpu().numpy()
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (i, key)
        assert int((single["status"] == ngl.HIT).sum()) > 100


@pytest.mark.parametrize("alphas", [(0.0, 0.0, 0.0, 0.0), (0.0, 0.5, 0.0, 0.25)])
def test_batch_views_match_oracle(alphas):
    """Each view of one batched launch against the oracle: the oracle builds
    the view's float32 camera rays itself (the GPU's agree to 5e-7), traces
    them at the view's LOD and alpha, and a ray is also marginal when its
    status changes under a 2e-6 turn of its direction."""
    import torch
    from paper_2101_10994_amd import ngl
    cases = batch_cases()
    models = [c.gpu_model() for c in cases]
    rng = np.random.default_rng(13)
    views = []
    for i, c in enumerate(cases):
        cam = W.camera_on_sphere(rng, 2.6, 112 + 16 * i, 96 + 8 * i)
        lod = c.L if alphas[i] == 0.0 else c.L - 1
        views.append(ngl.make_view(cam.eye, cam.width, cam.height, lod, alphas[i]))
    br = ngl.BatchRenderer(models, views, pair_capacity=1 << 20)
    br.render(100, 1e-4)
    torch.cuda.synchronize()
    assert not br.overflowed()
    out = {}
    for i, (c, v) in enumerate(zip(cases, views)):
        co, cd = oracle.camera_rays(tuple(v.eye), (0, 0, 0), (0, 1, 0), 45.0, v.width, v.height)
        o32, d32 = np.ascontiguousarray(co.astype(np.float32)), np.ascontiguousarray(cd.astype(np.float32))
        r = oracle_reference(c, o32, d32, v.lod, v.alpha, 100, 1e-4, dir_eps=2e-6)
        sl = br.view_slice(i)
        g = {"t": br.t[sl].cpu().numpy(), "status": br.status[sl].cpu().numpy(),
             "hit_vox": br.hit_vox[sl].cpu().numpy()}
        voxel = 2.0 / 2 ** (c.L + 1)
        nhit, nmarg = check(g, r, voxel, max_marginal=0.03)
        out["view%d_L%d_a%g" % (i, v.lod, v.alpha)] = summary(g, r, voxel)
        assert nhit > 100
    report("batch_vs_oracle_" + "_".join("%g" % a for a in alphas), out)


def test_batch_rejects_mixed_formats():
    from paper_2101_10994_amd import ngl
    cases = batch_cases()[:2]
    m0 = cases[0].gpu_model()
    c1 = make_case(W.tiny_shape(), 16, 3, 16, 64, feat_dtype="f16", w_dtype="bf16")
    views = [ngl.make_view((0, 0, 2.5), 32, 32, 3), ngl.make_view((0, 0, 2.5), 32, 32, 3)]
    br = ngl.BatchRenderer([m0, c1.gpu_model()], views, pair_capacity=1 << 16)
    with pytest.raises(ngl.NGLError):
        br.render(10, 1e-4)


def test_graph_replay_matches_eager():
    """The batched render captured in a graph replays to the eager result,
    with eager work between replays."""
    import torch
    from paper_2101_10994_amd import ngl
    cases = batch_cases()
    models = [c.gpu_model() for c in cases]
    rng = np.random.default_rng(9)
    views = []
    for c in cases:
        cam = W.camera_on_sphere(rng, 2.8, 64, 48)
        views.append(ngl.make_view(cam.eye, cam.width, cam.height, c.L))
    br = ngl.BatchRenderer(models, views, pair_capacity=1 << 18)
    br.render(60, 1e-4)
    torch.cuda.synchronize()
    ref = {k: getattr(br, k).clone() for k in ("t", "status", "steps", "hit_vox")}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        br.render(60, 1e-4)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        br.t.fill_(-1.0)
        br.status.fill_(255)
        br.steps.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in ref.items():
            assert torch.equal(getattr(br, k), v), (rep, k)
        assert np.all(br.frame_ms() >= 0)


def test_autotuner_applies_a_valid_config(tmp_path):
    import torch
    from paper_2101_10994_amd import autotune, ngl
    cases = batch_cases()[:2]
    models = [c.gpu_model() for c in cases]
    views = [ngl.make_view((0.3, 0.2, 2.6), 64, 64, c.L) for c in cases]
    br = ngl.BatchRenderer(models, views, pair_capacity=1 << 18)
    saved = autotune.current()
    br.render(40, 1e-4)
    torch.cuda.synchronize()
    ref = [x.clone() for x in (br.t, br.status, br.steps, br.hit_vox)]
    try:
        res = autotune.tune("test-batch", lambda: br.render(40, 1e-4), fp32_model=False, repeats=1,
                            path=str(tmp_path / "tune.json"))
        assert res["config"] == autotune.current()
        assert len(res["trials"]) >= 36 and res["ms"] > 0
        again = autotune.tune("test-batch", lambda: br.render(40, 1e-4), fp32_model=False,
                              path=str(tmp_path / "tune.json"))
        assert again["cached"] and again["config"] == res["config"]
        br.render(40, 1e-4)
        torch.cuda.synchronize()
        # the options change the launch schedule only: same bits as before
        for a, b in zip(ref, (br.t, br.status, br.steps, br.hit_vox)):
            assert torch.equal(a, b)
    finally:
        autotune.apply(saved)


def phased_batch_run():
    import torch
    from paper_2101_10994_amd import ngl
    cases = batch_cases()
    models = [c.gpu_model() for c in cases]
    rng = np.random.default_rng(5)
    views = []
    for i, c in enumerate(cases):
        cam = W.camera_on_sphere(rng, 2.6, 128, 96)
        views.append(ngl.make_view(cam.eye, cam.width, cam.height, c.L - 1, 0.5 if i % 2 else 0.0))
    br = ngl.BatchRenderer(models, views, pair_capacity=1 << 20)
    br.render(100, 1e-4)
    torch.cuda.synchronize()
    assert not br.overflowed()
    assert int((br.steps > 4).sum()) > 100
    return {"t": br.t.clone(), "status": br.status.clone(), "steps": br.steps.clone(), "hit_vox": br.hit_vox.clone()}


def test_phased_batch_is_bitwise_the_single_launch():
    """The batched render parks rays at the pause count per view and
    finishes them eight lanes per ray: outputs equal the one-phase launch
    bit for bit."""
    import torch
    from paper_2101_10994_amd import ngl
    keys = (ngl.OPT_TRACE_PAUSE1, ngl.OPT_TRACE_WIDE)
    old = [ngl.get_option(k) for k in keys]
    try:
        ngl.set_option(ngl.OPT_TRACE_PAUSE1, 0)
        ref = phased_batch_run()
        ngl.set_option(ngl.OPT_TRACE_WIDE, 1)
        for pause in (24, 4):
            ngl.set_option(ngl.OPT_TRACE_PAUSE1, pause)
            got = phased_batch_run()
            for key in ("t", "status", "steps", "hit_vox"):
                assert torch.equal(got[key], ref[key]), (pause, key)
    finally:
        for k, v in zip(keys, old):
            ngl.set_option(k, v)
