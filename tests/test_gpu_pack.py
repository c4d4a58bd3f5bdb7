"""Decoders pre-packed in matrix-core fragment order (ngl_pack_decoders)
give the same bits as fragments built from W1 and b1 inside the kernels:
queries (discrete and blended), the phased trace, normals, the decoder
alone and the batched render, for BF16 and FP32 weights and several
widths.  Re-packing after a weight change takes the new weights."""
import numpy as np
import pytest

from paper_2101_10994_amd import workloads as W

from cases import edge_points, make_case

pytestmark = pytest.mark.gpu

CASES = {
    "m32-bf16": lambda: make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True, feat_dtype="f16", w_dtype="bf16"),
    "m32-f32": lambda: make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True),
    "m8-noxyz-f32": lambda: make_case(W.tiny_shape(), 16, 3, 8, 32, sigma=0.1, with_xyz=False),
    "m64-bf16": lambda: make_case(W.tiny_shape(), 16, 3, 64, 64, sigma=0.1, feat_dtype="bf16", w_dtype="bf16"),
}


def outputs(gm, case, x, o, d):
    import torch
    from paper_2101_10994_amd import ngl
    L = case.L
    out = {}
    out["q"] = ngl.query_sdf(gm, x, L, want_valid=True)["sdf"]
    out["qa"] = ngl.query_sdf(gm, x, L - 1, alpha=0.4)["sdf"]
    hits = ngl.trace_octree(gm, o, d, L + 1)
    tr = ngl.sphere_trace(gm, o, d, L, 0.0, hits, 100, 1e-4)
    out.update({"t_" + k: tr[k] for k in ("t", "status", "steps", "hit_vox")})
    out["n"] = ngl.sdf_normals(gm, L, 0.0, 2.0 ** -9, x=x)
    z = torch.randn((4099, case.m), generator=torch.Generator(device="cuda").manual_seed(3), device="cuda")
    out["dec"] = ngl.decode_sdf(gm, L, z.contiguous(), x=x[:, :4099].contiguous() if case.with_xyz else None)
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_packed_equals_unpacked(name, f32_decoder):
    import torch
    from paper_2101_10994_amd import ngl
    case = CASES[name]()
    gm = case.gpu_model()
    x = torch.from_numpy(edge_points(case.ijk, 2 ** (case.L + 1), case.L, np.random.default_rng(1))).cuda()
    o, d = ngl.camera_rays((0.9, 0.6, 2.2), (0, 0, 0), (0, 1, 0), 45.0, 192, 160)
    ref = outputs(gm, case, x, o, d)
    gm.pack()
    assert gm.packed
    got = outputs(gm, case, x, o, d)
    for k in ref:
        assert torch.equal(ref[k], got[k]), (name, k)


def test_repack_after_weight_change_and_batch():
    import torch
    from paper_2101_10994_amd import ngl
    case = CASES["m32-bf16"]()
    gm = case.gpu_model()
    gm.pack()
    x = torch.from_numpy(W.soa(W.points_in_cells(np.random.default_rng(2), case.ijk, 64, 20000))).cuda()
    a = ngl.query_sdf(gm, x, 5)["sdf"]
    # scale W1 of LOD 5 in place: the packed copy is stale until refresh()
    with torch.no_grad():
        gm.W1[4].mul_(2.0)
    gm.refresh()
    b = ngl.query_sdf(gm, x, 5)["sdf"]
    gm.unpack()
    c = ngl.query_sdf(gm, x, 5)["sdf"]
    assert torch.equal(b, c) and not torch.equal(a, b)
    # batched render: packed models give the unpacked bits
    with torch.no_grad():
        gm.W1[4].mul_(0.5)
    gm.refresh()
    views = [ngl.make_view((0.9, 0.6, 2.2), 96, 80, 5), ngl.make_view((-1.5, 0.8, 2.0), 64, 64, 4, 0.3)]
    res = []
    for packed in (False, True):
        if packed:
            gm.pack()
        br = ngl.BatchRenderer([gm, gm], views, pair_capacity=1 << 20)
        br.render(100, 1e-4)
        torch.cuda.synchronize()
        res.append((br.t.clone(), br.status.clone(), br.steps.clone()))
    for u, v in zip(res[0], res[1]):
        assert torch.equal(u, v)


def test_pack_arguments():
    import torch
    from paper_2101_10994_amd import ngl
    case = CASES["m8-noxyz-f32"]()
    gm = case.gpu_model()
    nb = ngl.workspace_bytes(ngl.OP_PACK_DECODERS, gm)
    assert nb % 256 == 0 and nb > 0
    buf = torch.empty(nb + 512, dtype=torch.uint8, device="cuda")
    lib = ngl.lib()
    assert lib.ngl_pack_decoders(gm.ref, buf.data_ptr(), nb - 1, None) == 1  # too small
    assert lib.ngl_pack_decoders(gm.ref, buf.data_ptr() + 16, nb, None) == 1  # misaligned
    assert lib.ngl_pack_decoders(gm.ref, None, nb, None) == 1
    assert all(gm._struct.W1_packed[i] is None for i in range(ngl.MAX_LODS))
