"""Pins for the oracle's ray-octree intersection (Sec. 3.4, Alg. 1, App. C)
and its FP32 slab predicate: exact rational arithmetic, brute force over
every target-depth voxel, closed-form hit lists for axis-parallel rays, the
root-only tree, and front-to-back order."""
from fractions import Fraction

import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from paper_2101_10994_amd import workloads as W


def exact_slab(o, d, lo, hi):
    """Exact (rational) intersection of {o + t d, t >= 0} with the closed box.
    Returns (hit, margin, t_enter, t_exit)."""
    tmin, tmax = None, None
    for a in range(3):
        oa, da = Fraction(float(o[a])), Fraction(float(d[a]))
        la, ha = Fraction(float(lo[a])), Fraction(float(hi[a]))
        if da == 0:
            if not (la <= oa <= ha):
                return False, None, None, None
            continue
        t0, t1 = (la - oa) / da, (ha - oa) / da
        n, f = min(t0, t1), max(t0, t1)
        tmin = n if tmin is None or n > tmin else tmin
        tmax = f if tmax is None or f < tmax else tmax
    if tmin is None:
        return True, None, Fraction(0), None
    enter = max(tmin, Fraction(0))
    return tmax >= enter, tmax - enter, enter, tmax


def test_slab_predicate_vs_exact():
    rng = np.random.default_rng(0)
    n_marginal = 0
    n = 3000
    for k in range(n):
        depth = int(rng.integers(0, 6))
        r = 2 ** depth
        cell = rng.integers(0, r, size=3)
        lo = -1.0 + cell * (2.0 / r)
        hi = lo + 2.0 / r
        o = rng.uniform(-2, 2, size=3).astype(np.float32)
        # aim near the box so that many tests are close calls
        tgt = lo + rng.uniform(-0.2, 1.2, size=3) * (2.0 / r)
        d = (tgt - o)
        if k % 7 == 0:
            d[rng.integers(0, 3)] = 0.0
        d = (d / np.linalg.norm(d)).astype(np.float32)
        hit, ti, to = oracle.ray_box(o, d, depth, cell)
        ex, margin, te, tx = exact_slab(o, d, lo, hi)
        scale = 1.0 + abs(float(te or 0)) + abs(float(tx or 0))
        if margin is not None and abs(float(margin)) <= 1e-5 * scale:
            n_marginal += 1
            continue
        assert hit == ex, (o, d, depth, cell)
        if hit and tx is not None:
            assert abs(ti - float(te)) <= 1e-5 * scale
            assert abs(to - float(tx)) <= 1e-5 * scale
    assert n_marginal < n * 0.02


def test_slab_parallel_axes():
    # parallel to x inside the slab of y/z -> depends on x only
    o = np.array([-1.5, 0.1, 0.1], np.float32)
    d = np.array([1.0, 0.0, 0.0], np.float32)
    assert oracle.ray_box(o, d, 1, [0, 1, 1]) == (True, 0.5, 1.5)
    assert oracle.ray_box(o, d, 1, [1, 1, 1]) == (True, 1.5, 2.5)
    assert oracle.ray_box(o, d, 1, [1, 0, 1])[0] is False
    # touching a face counts (closed box)
    o2 = np.array([-1.5, 0.0, 0.5], np.float32)
    assert oracle.ray_box(o2, d, 1, [0, 0, 1])[0] is True
    assert oracle.ray_box(o2, d, 1, [0, 1, 1])[0] is True
    # grazing an edge: entry == exit at a single point still counts
    o3 = np.array([-0.5, 0.5, -0.5], np.float32)
    d3 = np.array([1.0, -1.0, 0.0], np.float32)
    assert oracle.ray_box(o3, d3, 1, [0, 0, 0]) == (True, 0.5, 0.5)
    assert oracle.ray_box(o3, d3, 1, [0, 1, 0]) == (True, 0.0, 0.5)
    # pointing away
    assert oracle.ray_box(o, -d, 1, [0, 1, 1])[0] is False
    # origin inside: t_in = 0
    assert oracle.ray_box(np.array([0.5, 0.5, 0.5], np.float32), d, 1, [1, 1, 1]) == (True, 0.0, 0.5)


def brute_hits(t, o, d, depth):
    """Every voxel at `depth` tested with the slab predicate, per ray."""
    e = t.export_depth(depth)
    out = []
    for i in range(o.shape[1]):
        hits = {}
        for v in range(len(e["ijk"])):
            h, ti, to = oracle.ray_box(o[:, i], d[:, i], depth, e["ijk"][v])
            if h:
                hits[v] = (ti, to)
        out.append(hits)
    return out


def check_lists(t, o, d, depth):
    res = oracle.trace_octree(t, o, d, depth)
    brute = brute_hits(t, o, d, depth)
    off = res["ray_off"]
    for i in range(o.shape[1]):
        seg = slice(off[i], off[i + 1])
        assert np.all(res["ray"][seg] == i)
        vox = res["vox"][seg]
        assert set(vox.tolist()) == set(brute[i].keys())
        assert len(set(vox.tolist())) == len(vox)
        for k, v in enumerate(vox):
            assert (res["t_in"][seg][k], res["t_out"][seg][k]) == brute[i][v]
        # front to back: FP32 entry distances never decrease along the list
        assert np.all(np.diff(res["t_in"][seg]) >= 0)
    return res


def test_dfs_equals_brute_force_tiny_sphere():
    ijk = W.occupancy_ijk(W.tiny_shape(), 16)
    t = oracle.Octree(ijk, 3)
    rng = np.random.default_rng(1)
    o, d = W.random_rays(rng, 60)
    for depth in range(0, 5):
        check_lists(t, o, d, depth)


@settings(max_examples=20, deadline=None)
@given(st.integers(1, 2), st.integers(0, 2 ** 31 - 1))
def test_dfs_equals_brute_force_random(L, seed):
    rng = np.random.default_rng(seed)
    r = 2 ** (L + 1)
    ijk = rng.integers(0, r, size=(int(rng.integers(1, 40)), 3)).astype(np.int32)
    t = oracle.Octree(ijk, L)
    o, d = W.random_rays(rng, 20)
    # some rays starting inside the box and some axis-parallel ones
    o2 = rng.uniform(-1, 1, size=(3, 5)).astype(np.float32)
    d2 = d[:, :5].copy()
    oa, da = W.axis_rays(rng, 5, r)
    o = np.concatenate([o, o2, oa], 1)
    d = np.concatenate([d, d2, da], 1)
    check_lists(t, o, d, L + 1)


def test_axis_column_closed_form():
    """Rays along +/-z through a column centre hit exactly that column's
    occupied cells, in order, entering at the cell face."""
    ijk = W.occupancy_ijk(W.tiny_shape(), 16)
    t = oracle.Octree(ijk, 3)
    occ = set(map(tuple, ijk.tolist()))
    e = t.export_depth(4)
    index = {tuple(c): v for v, c in enumerate(e["ijk"].tolist())}
    for (i, j) in [(8, 8), (3, 7), (0, 0), (7, 12)]:
        for sgn in (1.0, -1.0):
            o = np.array([[-1 + (i + 0.5) / 8], [-1 + (j + 0.5) / 8], [-1.5 * sgn]], np.float32)
            d = np.array([[0.0], [0.0], [sgn]], np.float32)
            res = oracle.trace_octree(t, o, d, 4)
            ks = [k for k in range(16) if (i, j, k) in occ]
            if sgn < 0:
                ks = ks[::-1]
            assert res["vox"].tolist() == [index[(i, j, k)] for k in ks]
            lo = np.array([-1 + k / 8 for k in ks])
            tin = lo + 1.5 if sgn > 0 else 1.5 - (lo + 1 / 8)
            np.testing.assert_array_equal(res["t_in"], tin.astype(np.float32))


def test_root_only_and_empty():
    t = oracle.Octree(np.array([[0, 0, 0]], np.int32), 1)
    rng = np.random.default_rng(3)
    o, d = W.random_rays(rng, 50, aim_radius=1.5)
    res = oracle.trace_octree(t, o, d, 0)
    for i in range(50):
        h = oracle.ray_box(o[:, i], d[:, i], 0, [0, 0, 0])[0]
        assert res["ray_off"][i + 1] - res["ray_off"][i] == int(h)
    assert np.all(res["vox"] == 0)
    te = oracle.Octree(np.zeros((0, 3), np.int32), 1)
    res = oracle.trace_octree(te, o, d, 2)
    assert len(res["vox"]) == 0 and np.all(res["ray_off"] == 0)


def test_camera_rays_closed_form():
    W_, H_ = 65, 33
    o, d = oracle.camera_rays((0.0, 0.0, 2.5), (0, 0, 0), (0, 1, 0), 45.0, W_, H_)
    np.testing.assert_allclose(np.linalg.norm(d, axis=0), 1.0, atol=1e-15)
    assert np.all(o[2] == 2.5)
    c = (H_ // 2) * W_ + W_ // 2
    np.testing.assert_allclose(d[:, c], [0, 0, -1], atol=1e-15)
    # top-centre pixel: vertical angle atan(tan(22.5 deg) * (1 - 1/H))
    top = W_ // 2
    ang = np.arctan2(d[1, top], -d[2, top])
    np.testing.assert_allclose(ang, np.arctan(np.tan(np.radians(22.5)) * (1 - 1 / H_)), atol=1e-14)
    # right-centre pixel: horizontal angle with aspect W/H; +x is to the right
    right = c + W_ // 2
    ang = np.arctan2(d[0, right], -d[2, right])
    np.testing.assert_allclose(ang, np.arctan(np.tan(np.radians(22.5)) * W_ / H_ * (1 - 1 / W_)), atol=1e-14)
