"""GPU parity: camera rays and the breadth-first ray-octree intersection
(Sec. 3.4, Alg. 1, App. C) against the oracle's per-ray depth-first search.
Hit lists (ray, voxel, order), t_in/t_out and ray offsets are bit-exact."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2101_10994_amd import workloads as W

pytestmark = pytest.mark.gpu


def gpu_tree(ijk, L):
    import torch
    from paper_2101_10994_amd import ngl
    tree = ngl.Octree(ijk, L, device="cuda")
    m = ngl.Model(tree, [torch.zeros((int(tree.ncorner[lv]), 8), device="cuda") for lv in range(L)],
                  [torch.zeros((16, 11), device="cuda")] * L,
                  [torch.zeros(16, device="cuda")] * L, [torch.zeros(16, device="cuda")] * L,
                  torch.zeros(L, device="cuda"))
    return tree, m


def compare_lists(m, otree, o, d, depth, capacity=None):
    import torch
    from paper_2101_10994_amd import ngl
    g = ngl.trace_octree(m, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), depth, capacity=capacity)
    ref = oracle.trace_octree(otree, o, d, depth)
    n = len(ref["vox"])
    assert g["count"] == n
    assert np.array_equal(g["ray"].cpu().numpy(), ref["ray"])
    assert np.array_equal(g["vox"].cpu().numpy(), ref["vox"])
    assert np.array_equal(g["t_in"].cpu().numpy().view(np.int32), ref["t_in"].view(np.int32))
    assert np.array_equal(g["t_out"].cpu().numpy().view(np.int32), ref["t_out"].view(np.int32))
    assert np.array_equal(g["ray_off"].cpu().numpy().astype(np.int64), ref["ray_off"])
    return g, ref


def test_camera_rays_match_oracle():
    import torch
    from paper_2101_10994_amd import ngl
    for (eye, W_, H_) in [((0.0, 0.0, 2.5), 64, 64), ((0.9, 0.6, 2.2), 333, 127)]:
        o, d = ngl.camera_rays(eye, (0, 0, 0), (0, 1, 0), 45.0, W_, H_)
        ro, rd = oracle.camera_rays(eye, (0, 0, 0), (0, 1, 0), 45.0, W_, H_)
        assert np.array_equal(o.cpu().numpy(), ro.astype(np.float32))
        assert np.abs(d.cpu().numpy() - rd).max() < 5e-7


def test_tiny_all_depths():
    ijk = W.occupancy_ijk(W.tiny_shape(), 16)
    otree = oracle.Octree(ijk, 3)
    _, m = gpu_tree(ijk, 3)
    rng = np.random.default_rng(0)
    co, cd = oracle.camera_rays((0.0, 0.0, 2.5), (0, 0, 0), (0, 1, 0), 45.0, 64, 64)
    ro, rd = W.random_rays(rng, 2000)
    ao, ad = W.axis_rays(rng, 500, 16)
    io = rng.uniform(-1, 1, size=(3, 300)).astype(np.float32)  # origins inside the box
    o = np.ascontiguousarray(np.concatenate([co.astype(np.float32), ro, ao, io], 1))
    d = np.ascontiguousarray(np.concatenate([cd.astype(np.float32), rd, ad, rd[:, :300]], 1))
    for depth in range(0, 5):
        compare_lists(m, otree, o, d, depth)


def test_paper_scale_camera():
    """1024x1024 camera at the finest depth of the 5-LOD octree: full lists."""
    ijk = W.occupancy_ijk(W.paper_shape(0), 64)
    otree = oracle.Octree(ijk, 5)
    _, m = gpu_tree(ijk, 5)
    co, cd = oracle.camera_rays(W.PAPER.eye, (0, 0, 0), (0, 1, 0), 45.0, 1024, 1024)
    o, d = co.astype(np.float32), cd.astype(np.float32)
    g, ref = compare_lists(m, otree, o, d, 6)
    assert g["count"] > 1_000_000
    # and at an intermediate depth
    compare_lists(m, otree, o, d, 4)


def test_random_octrees():
    rng = np.random.default_rng(5)
    for L in (1, 2, 4):
        r = 2 ** (L + 1)
        ijk = rng.integers(0, r, size=(int(rng.integers(1, 300)), 3)).astype(np.int32)
        otree = oracle.Octree(ijk, L)
        _, m = gpu_tree(ijk, L)
        o, d = W.random_rays(rng, 3000)
        compare_lists(m, otree, o, d, L + 1)


def test_capacity_overflow_is_reported_and_bounded():
    import torch
    from paper_2101_10994_amd import ngl
    ijk = W.occupancy_ijk(W.tiny_shape(), 16)
    _, m = gpu_tree(ijk, 3)
    co, cd = oracle.camera_rays((0.0, 0.0, 2.5), (0, 0, 0), (0, 1, 0), 45.0, 64, 64)
    o = torch.from_numpy(co.astype(np.float32)).cuda()
    d = torch.from_numpy(cd.astype(np.float32)).cuda()
    cap, guard = 1000, 4096
    R = o.shape[1]
    nb = C.c_size_t()
    ngl.lib().ngl_trace_octree_workspace(R, cap, C.addressof(nb))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    bufs = [torch.full((cap + guard,), -7, dtype=torch.int32, device="cuda") for _ in range(4)]
    off = torch.empty(R + 1, dtype=torch.int32, device="cuda")
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    rc = ngl.lib().ngl_trace_octree(m.ref, o.data_ptr(), d.data_ptr(), R, 4, cap, ws.data_ptr(), ws.numel(),
                                    *[b.data_ptr() for b in bufs], off.data_ptr(), counts.data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(counts[1]) > cap
    for b in bufs:
        assert torch.all(b[cap:] == -7)
    # the wrapper retries with the reported size and matches the oracle
    compare_lists(m, oracle.Octree(ijk, 3), co.astype(np.float32), cd.astype(np.float32), 4, capacity=cap)


def test_empty_tree_and_no_rays():
    import torch
    from paper_2101_10994_amd import ngl
    _, m = gpu_tree(np.zeros((0, 3), np.int32), 2)
    o, d = W.random_rays(np.random.default_rng(1), 100)
    g = ngl.trace_octree(m, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), 3)
    assert g["count"] == 0 and torch.all(g["ray_off"] == 0)
    _, m = gpu_tree(W.occupancy_ijk(W.tiny_shape(), 16), 3)
    g = ngl.trace_octree(m, torch.zeros((3, 0), device="cuda"), torch.zeros((3, 0), device="cuda"), 4)
    assert g["count"] == 0
