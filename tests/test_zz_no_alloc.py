"""The allocation-free sphere trace (ngl_sphere_trace_static, for callers
that cannot allocate device memory) against ngl_sphere_trace with a caller
workspace: the same bits on two calls in a row, the second with fewer rays
(the library's array keeps the first call's contents), through the C ABI;
more rays than the array holds are rejected."""
import ctypes as C

import numpy as np
import pytest

from paper_2101_10994_amd import workloads as W

from cases import make_case

pytestmark = pytest.mark.gpu


def trace_static(ngl, gm, o, d, lod, alpha, hits, prm):
    import torch
    R = o.shape[1]
    out = dict(t=torch.empty(R, dtype=torch.float32, device="cuda"),
               status=torch.empty(R, dtype=torch.uint8, device="cuda"),
               steps=torch.empty(R, dtype=torch.int32, device="cuda"),
               hit_vox=torch.empty(R, dtype=torch.int32, device="cuda"))
    rc = ngl.lib().ngl_sphere_trace_static(
        gm.ref, o.data_ptr(), d.data_ptr(), R, lod, alpha, hits["vox"].data_ptr(), hits["t_in"].data_ptr(),
        hits["t_out"].data_ptr(), hits["ray_off"].data_ptr(), C.addressof(prm), out["t"].data_ptr(),
        out["status"].data_ptr(), out["steps"].data_ptr(), out["hit_vox"].data_ptr(),
        torch.cuda.current_stream().cuda_stream)
    assert rc == 0, ngl.lib().ngl_last_error()
    return out


def test_static_trace_equals_workspace_trace():
    import torch
    from paper_2101_10994_amd import ngl
    case = make_case(W.paper_shape(0), 64, 5, 32, 128, spread=True)
    gm = case.gpu_model()
    prm = ngl.trace_params(100, 1e-4, 5.0, False, None)
    for (w, h), (lod, alpha) in (((768, 640), (5, 0.0)), ((160, 120), (4, 0.3))):
        o, d = ngl.camera_rays(W.PAPER.eye, (0, 0, 0), (0, 1, 0), 45.0, w, h)
        hits = ngl.trace_octree(gm, o, d, (lod + 1 if alpha > 0 else lod) + 1)
        ref = ngl.sphere_trace(gm, o, d, lod, alpha, hits, 100, 1e-4)
        got = trace_static(ngl, gm, o, d, lod, alpha, hits, prm)
        torch.cuda.synchronize()
        for k in ("t", "status", "steps", "hit_vox"):
            assert torch.equal(got[k], ref[k]), (w, h, k)
        assert int((ref["steps"] > 24).sum()) > 0  # some rays take the phased path


def test_static_trace_rejects_too_many_rays():
    from paper_2101_10994_amd import ngl
    case = make_case(W.tiny_shape(), 16, 3, 8, 32)
    gm = case.gpu_model()
    prm = ngl.trace_params(10, 1e-4, 5.0, False, None)
    R = ngl.STATIC_TRACE_MAX_RAYS + 1
    # rejected before any device access: the pointers are never read
    rc = ngl.lib().ngl_sphere_trace_static(gm.ref, 16, 16, R, 3, 0.0, 16, 16, 16, 16, C.addressof(prm), 16, 16, 16,
                                           16, None)
    assert rc == 2 and b"NGL_STATIC_TRACE_MAX_RAYS" in ngl.lib().ngl_last_error()
