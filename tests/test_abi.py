"""The C-ABI library loads and exports every symbol include/ngl.h declares;
host-only entry points (octree build, argument checks) run without a GPU."""
import os
import re

import numpy as np
import pytest

from paper_2101_10994_amd import ngl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ngl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ngl_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ngl.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
        assert n in ngl.EXPORTS, n


def test_status_strings():
    lib = ngl.lib()
    assert lib.ngl_status_str(0) == b"ok"
    assert lib.ngl_status_str(1) == b"invalid argument"
    assert lib.ngl_version() >= 1


def test_struct_layout_matches_header():
    import ctypes as C
    # 6 int32 + 10+8 int64 + 4*10 + 5*8 + 1 + 2*8 + 8 pointers
    assert C.sizeof(ngl.ngl_model) == 6 * 4 + 18 * 8 + (4 * 10 + 5 * 8 + 1 + 2 * 8 + 8) * 8
    assert C.sizeof(ngl.ngl_trace_params) == 4 * 6 + 16


def test_plan_rejects_bad_input():
    lib = ngl.lib()
    nv = np.zeros(10, np.int64)
    nc = np.zeros(8, np.int64)
    bad = np.array([[16, 0, 0]], np.int32)
    assert lib.ngl_octree_plan(bad.ctypes.data, 1, 3, nv.ctypes.data, nc.ctypes.data) == 1
    assert b"outside" in lib.ngl_last_error()
    ok = np.array([[15, 0, 0]], np.int32)
    assert lib.ngl_octree_plan(ok.ctypes.data, 1, 0, nv.ctypes.data, nc.ctypes.data) == 1
    assert lib.ngl_octree_plan(ok.ctypes.data, 1, 9, nv.ctypes.data, nc.ctypes.data) == 1
    assert lib.ngl_octree_plan(ok.ctypes.data, 1, 3, nv.ctypes.data, nc.ctypes.data) == 0
    assert list(nv[:5]) == [1, 1, 1, 1, 1]


def test_device_calls_validate_before_launch():
    lib = ngl.lib()
    import ctypes as C
    m = ngl.ngl_model()
    m.num_lods = 0
    assert lib.ngl_query_sdf(C.addressof(m), None, 0, 1, 0.0, None, None, None, None, None) == 1
    assert lib.ngl_sdf_normals(C.addressof(m), None, None, None, None, None, 0, 1, 0.0, 0.01, None, None) == 1
    m.num_lods = 2
    assert lib.ngl_trace_octree(C.addressof(m), None, None, 0, 7, 0, None, 0, None, None, None, None, None, None,
                                None) == 1
    assert b"target_depth" in lib.ngl_last_error()


def test_options():
    from paper_2101_10994_amd import ngl
    assert ngl.get_option(ngl.OPT_F32_DECODER) in (0, 1)
    old = ngl.get_option(ngl.OPT_F32_DECODER)
    ngl.set_option(ngl.OPT_F32_DECODER, 0)
    assert ngl.get_option(ngl.OPT_F32_DECODER) == 0
    ngl.set_option(ngl.OPT_F32_DECODER, old)
    with pytest.raises(ngl.NGLError):
        ngl.set_option(ngl.OPT_F32_DECODER, 7)
    with pytest.raises(ngl.NGLError):
        ngl.set_option(99, 0)
    for key in (ngl.OPT_TRACE_PAUSE1, ngl.OPT_TRACE_PAUSE2):
        with pytest.raises(ngl.NGLError):
            ngl.set_option(key, 5000)
        with pytest.raises(ngl.NGLError):
            ngl.set_option(key, -1)
    with pytest.raises(ngl.NGLError):
        ngl.set_option(ngl.OPT_TRACE_WIDE, 2)


def test_phased_trace_workspace_sizes():
    """Workspace queries of the phased tracers: 256 B of counters plus one
    256-byte-aligned array per parked-state field and id list (host only)."""
    import ctypes as C
    from paper_2101_10994_amd import ngl
    lib = ngl.lib()
    al = lambda b: (b + 255) // 256 * 256
    for R in (0, 1, 1000, 1 << 20):
        nb = C.c_size_t()
        assert lib.ngl_sphere_trace_workspace_rays(R, C.addressof(nb)) == 0
        assert nb.value == 256 + 6 * al(4 * R)
        assert lib.ngl_sphere_trace_lod_workspace(R, C.addressof(nb)) == 0
        assert nb.value == 256 + 2 * al(4 * R) + al(R) + 5 * al(4 * R)
    nb = C.c_size_t()
    assert lib.ngl_sphere_trace_workspace_rays(-1, C.addressof(nb)) == 1
    assert lib.ngl_sphere_trace_lod_workspace(-1, C.addressof(nb)) == 1


def test_workspace_bytes_matches_each_query():
    """ngl_workspace_bytes returns the value of each call's own size query
    (host only); unknown ops and negative sizes are rejected."""
    import ctypes as C
    from paper_2101_10994_amd import ngl
    lib = ngl.lib()

    def own(fn, *args):
        nb = C.c_size_t()
        assert getattr(lib, fn)(*args, C.addressof(nb)) == 0
        return nb.value

    for n in (0, 1, 1000, 1 << 20):
        assert ngl.workspace_bytes(ngl.OP_TRACE_OCTREE, None, n, 4 * n + 7) == own("ngl_trace_octree_workspace", n,
                                                                                  4 * n + 7)
        assert ngl.workspace_bytes(ngl.OP_SPHERE_TRACE, None, n) == own("ngl_sphere_trace_workspace_rays", n)
        assert ngl.workspace_bytes(ngl.OP_SPHERE_TRACE_LOD, None, n) == own("ngl_sphere_trace_lod_workspace", n)
        assert ngl.workspace_bytes(ngl.OP_SAMPLE_SURFACE, None, n) == own("ngl_sample_surface_workspace", n)
        for L in (1, 5, 8):
            assert ngl.workspace_bytes(ngl.OP_OCTREE_BUILD_DEVICE, None, n, L) == own(
                "ngl_octree_build_device_workspace", n, L)
    with pytest.raises(ngl.NGLError):
        ngl.workspace_bytes(99, None, 1)
    with pytest.raises(ngl.NGLError):
        ngl.workspace_bytes(ngl.OP_SPHERE_TRACE, None, -1)
    with pytest.raises(ngl.NGLError):
        ngl.workspace_bytes(ngl.OP_TRAIN, None, 10)
    with pytest.raises(ngl.NGLError):
        ngl.workspace_bytes(ngl.OP_OCTREE_BUILD_DEVICE, None, 10, 0)


def test_packed_decoder_bytes():
    """Per LOD: (h/16) fragments per K-step of 64 lanes, 16 B (BF16: one step
    per 32 features + the position/bias step) or 4 B (FP32: ceil((din+1)/4)
    steps), rounded up to 256 B (host only: a model view with null device
    pointers is enough for the size)."""
    import ctypes as C
    from paper_2101_10994_amd import ngl
    lib = ngl.lib()
    for m, h, xyz, wdt, L in ((32, 128, 1, 2, 5), (32, 128, 1, 0, 5), (8, 32, 0, 0, 3), (64, 64, 1, 2, 7),
                              (16, 16, 1, 0, 2)):
        s = ngl.ngl_model()
        s.num_lods, s.feat_dim, s.hidden, s.with_xyz, s.feat_dtype, s.w_dtype = L, m, h, xyz, 0, wdt
        dummy = C.c_float(0.0)
        for lv in range(L):
            s.W1[lv] = s.b1[lv] = s.w2[lv] = C.addressof(dummy)
        s.b2 = C.addressof(dummy)
        nb = C.c_size_t()
        assert lib.ngl_packed_decoder_bytes(C.addressof(s), C.addressof(nb)) == 0, lib.ngl_last_error()
        if wdt == 2:
            per = (h // 16) * ((m + 31) // 32 + 1) * 64 * 16
        else:
            per = (h // 16) * ((m + 3 * xyz + 1 + 3) // 4) * 64 * 4
        assert nb.value == L * ((per + 255) // 256 * 256)
