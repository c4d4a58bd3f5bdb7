"""Pins for the oracle's fitting pieces (training appendix): the analytic
union SDF at closed-form points, the SDF surface sampler (hits lie on the
surface, origins inside a sphere always hit, directions uniform), the 2:2:1
training set (structure, uniform and Gaussian statistics, exact targets),
per-LOD loss weights (linearity, all-ones is Eq. 4) and Adam (closed-form
first step and constant-gradient steps)."""
import math

import numpy as np

import oracle
from paper_2101_10994_amd import workloads as W

NO_TORI = np.zeros((0, 6))


def test_shape_sdf_closed_forms():
    # dyadic centre, radius and points: the distances are exact
    sph = [[0.125, -0.25, 0.375, 0.5]]
    x = np.array([[0.125, -0.25, 0.375], [0.875, -0.25, 0.375], [0.125, -0.25, -0.375],
                  [0.125 + 0.75, -0.25 + 0.5, 0.375], [0.125 + 0.375, -0.25, 0.375 + 0.5]], np.float32).T
    got = oracle.shape_sdf(sph, NO_TORI, x)
    assert got.tolist() == [-0.5, 0.25, 0.25, math.sqrt(0.75 ** 2 + 0.25) - 0.5, 0.625 - 0.5]
    # torus R = 0.5, r = 0.125 around axis z at the origin: -r on the ring,
    # sqrt(R^2 + h^2) - r on the axis, and the axis choice rotates it
    for a in range(3):
        tor = [[0, 0, 0, 0.5, 0.125, a]]
        u, v = [(1, 2), (0, 2), (0, 1)][a]
        ring = np.zeros((3, 1), np.float32)
        ring[u, 0] = 0.5
        axis_pt = np.zeros((3, 1), np.float32)
        axis_pt[a, 0] = 0.25
        assert oracle.shape_sdf(np.zeros((0, 4)), tor, ring)[0] == -0.125
        np.testing.assert_allclose(oracle.shape_sdf(np.zeros((0, 4)), tor, axis_pt)[0],
                                   math.sqrt(0.25 + 0.0625) - 0.125, atol=1e-15)
    # the union is the minimum
    both = oracle.shape_sdf(sph, [[0, 0, 0, 0.5, 0.125, 2]], x)
    np.testing.assert_array_equal(both, np.minimum(got, oracle.shape_sdf(np.zeros((0, 4)), [[0, 0, 0, 0.5, 0.125, 2]], x)))
    # agrees with the workload generator's float64 SDF on a random union
    shape = W.paper_shape(0)
    pts = np.random.default_rng(0).uniform(-1, 1, (2000, 3)).astype(np.float32)
    np.testing.assert_allclose(oracle.shape_sdf(shape.spheres, shape.tori, W.soa(pts)),
                               shape.sdf(pts.astype(np.float64)), atol=1e-14)


def test_surface_sampler_on_a_sphere():
    rho, delta = 0.6, 1e-5
    rng = np.random.default_rng(1)
    u = rng.uniform(0, 1, (5, 20000)).astype(np.float32)
    r = oracle.sample_surface([[0, 0, 0, rho]], NO_TORI, u, 200, delta)
    p = r["points"][:, r["hit"]]
    # every hit lies within delta of the sphere
    assert np.all(np.abs(np.linalg.norm(p, axis=0) - rho) < delta)
    # origins inside the ball always hit; origins outside hit iff the
    # forward ray passes within rho (and stays in the box, which a ray from
    # inside the box towards a ball inside the box does)
    o = -1.0 + 2.0 * u[:3].astype(np.float64)
    z = 1.0 - 2.0 * u[3].astype(np.float64)
    phi = 2 * np.pi * u[4].astype(np.float64)
    d = np.stack([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z])
    inside = np.linalg.norm(o, axis=0) < rho
    assert np.all(r["hit"][inside])
    b = (o * d).sum(0)
    closest = np.sqrt(np.maximum((o * o).sum(0) - b * b, 0))
    forward_hit = ~inside & (b < 0) & (closest < rho - 1e-3)
    clear_miss = ~inside & ((b > 0) | (closest > rho + 1e-3))
    assert np.all(r["hit"][forward_hit]) and not np.any(r["hit"][clear_miss])
    # directions are uniform on the sphere: E[d] = 0, E[d d^T] = I/3
    assert np.all(np.abs(d.mean(1)) < 0.03)
    np.testing.assert_allclose((d @ d.T) / d.shape[1], np.eye(3) / 3, atol=0.02)


def test_training_points_structure_and_statistics():
    shape = W.paper_shape(0)
    rng = np.random.default_rng(2)
    u = rng.uniform(0, 1, (5, 40000)).astype(np.float32)
    s = oracle.sample_surface(shape.spheres, shape.tori, u, 200, 1e-6)
    S = s["points"][:, s["hit"]]
    N = 50000
    uni = rng.uniform(0, 1, (4, N)).astype(np.float32)
    sigma = 0.01
    xs, tg = oracle.training_points(shape.spheres, shape.tori, S, uni, sigma)
    c = np.arange(N) % 5
    q = np.arange(N) // 5
    k = {0: 2 * q, 1: 2 * q + 1, 2: 2 * q, 3: 2 * q + 1}
    for cc in (0, 1):
        sel = c == cc
        np.testing.assert_array_equal(xs[:, sel], S[:, k[cc][sel] % S.shape[1]].astype(np.float32))
        assert np.all(np.abs(tg[sel]) < 2e-6)
    sel = c == 4
    np.testing.assert_array_equal(xs[:, sel], (-1.0 + 2.0 * uni[:3, sel].astype(np.float64)).astype(np.float32))
    g = np.concatenate([(xs[:, c == cc].astype(np.float64) - S[:, k[cc][c == cc] % S.shape[1]]) / sigma
                        for cc in (2, 3)], 1)
    assert np.all(np.abs(g.mean(1)) < 0.03)
    np.testing.assert_allclose(g.var(1), 1.0, atol=0.04)
    np.testing.assert_allclose(oracle.shape_sdf(shape.spheres, shape.tori, xs), tg, atol=0)
    # near points sit about sigma from the surface
    assert 0.5 * sigma < np.median(np.abs(tg[(c == 2) | (c == 3)])) < 1.5 * sigma


def test_near_offsets_are_isotropic_standard_normal():
    """The near-surface offsets (training appendix, Sampling: surface points
    moved by isotropic Gaussian noise) are sigma times a standard normal
    vector in R^3: independent N(0,1) components.  Each check below is one
    the two-value Box-Muller pairing can get wrong while every per-axis
    mean and variance stays right (a reused angle correlates two axes, a
    reused radius couples the squared components of all three)."""
    from scipy import stats
    shape = W.paper_shape(0)
    rng = np.random.default_rng(5)
    u = rng.uniform(0, 1, (5, 40000)).astype(np.float32)
    s = oracle.sample_surface(shape.spheres, shape.tori, u, 200, 1e-6)
    S = s["points"][:, s["hit"]]
    N = 100000
    uni = rng.uniform(0, 1, (4, N)).astype(np.float32)
    sigma = 0.25  # large against FP32 rounding of the stored points
    xs, _ = oracle.training_points(shape.spheres, shape.tori, S, uni, sigma)
    c = np.arange(N) % 5
    q = np.arange(N) // 5
    near = (c == 2) | (c == 3)
    k = (2 * q + (c - 2))[near] % S.shape[1]
    g = (xs[:, near].astype(np.float64) - S[:, k]) / sigma
    n = g.shape[1]
    # FP32 storage of x moves g by at most 2^-24 |x| / sigma < 1e-6
    se = 1.0 / np.sqrt(n)
    # covariance = identity (a shared angle gives correlation +-1)
    cov = g @ g.T / n
    np.testing.assert_allclose(np.diag(cov), 1.0, atol=8 * np.sqrt(2) * se)
    off = cov[~np.eye(3, dtype=bool)]
    assert np.all(np.abs(off) < 6 * se), off
    # squared components uncorrelated: cov(g_a^2, g_b^2) = 0 for independent
    # normals (a shared radius gives E r^4 / 4 - 1 = 1); each estimate has
    # standard error sqrt(8 / n)
    g2 = g * g
    c2 = np.cov(g2)
    assert np.all(np.abs(c2[~np.eye(3, dtype=bool)]) < 6 * np.sqrt(8.0) * se), c2
    # |g|^2 follows chi-square with 3 degrees of freedom: mean 3, variance 6
    r2 = g2.sum(0)
    assert abs(r2.mean() - 3.0) < 6 * np.sqrt(6.0) * se
    assert abs(r2.var() - 6.0) < 0.3
    assert stats.kstest(r2, stats.chi2(3).cdf).pvalue > 1e-4
    # the direction g/|g| is uniform on the sphere: E[n n^T] = I/3
    nd = g / np.sqrt(r2)
    np.testing.assert_allclose(nd @ nd.T / n, np.eye(3) / 3, atol=6 * se)
    # offsets do not depend on which surface sample they perturb
    for a in range(3):
        assert abs(np.corrcoef(g[a], k)[0, 1]) < 6 * se


def test_lod_weights_are_linear():
    ijk = W.occupancy_ijk(W.tiny_shape(), 16)
    t = oracle.Octree(ijk, 3)
    rng = np.random.default_rng(3)
    d = W.decoders(rng, 3, 11, 32)
    feats = [rng.normal(0, 0.1, size=(int(n), 8)) for n in t.ncorner]
    mdl = oracle.Model(feats, list(d["W1"]), list(d["b1"]), list(d["w2"]), d["b2"])
    x = W.soa(W.points_in_cells(rng, ijk, 16, 300))
    y = rng.normal(0, 0.1, 300).astype(np.float32)
    ref = oracle.train_fwd_bwd(t, mdl, x, y)
    ones = oracle.train_fwd_bwd(t, mdl, x, y, lod_weight=[1.0, 1.0, 1.0])
    parts = [oracle.train_fwd_bwd(t, mdl, x, y, lod_weight=np.eye(3)[L]) for L in range(3)]
    w = np.array([0.0, 0.5, 2.0])
    mix = oracle.train_fwd_bwd(t, mdl, x, y, lod_weight=w)
    for key in ("dfeat", "dW1", "db1", "dw2"):
        for L in range(3):
            np.testing.assert_array_equal(ones[key][L], ref[key][L])
            lin = sum(w[j] * parts[j][key][L] for j in range(3))
            np.testing.assert_allclose(mix[key][L], lin, rtol=1e-12, atol=1e-15)
    assert ones["loss"] == ref["loss"]
    np.testing.assert_allclose(mix["loss"], sum(w[j] * parts[j]["loss"] for j in range(3)), rtol=1e-12)
    # a zero-weight LOD's decoder receives no gradient
    assert np.all(parts[2]["dW1"][0] == 0) and np.all(parts[2]["db2"][:2] == 0)


def test_adam_closed_forms():
    rng = np.random.default_rng(4)
    lr, eps = 1e-3, 1e-8
    th0 = rng.normal(size=50)
    g = rng.normal(size=50)
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    oracle.adam_step([th], [g], [m], [v], 1, lr=lr, eps=eps)
    # first step: bias-corrected moments are g and g^2
    np.testing.assert_allclose(th, th0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    for t in range(2, 30):
        before = th.copy()
        oracle.adam_step([th], [g], [m], [v], t, lr=lr, eps=eps)
        np.testing.assert_allclose(th - before, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-18)
    # zero gradient after one step: the moments decay, the step keeps its sign
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    oracle.adam_step([th], [g], [m], [v], 1, lr=lr, eps=eps)
    before = th.copy()
    oracle.adam_step([th], [np.zeros(50)], [m], [v], 2, lr=lr, eps=eps)
    b1, b2 = 0.9, 0.999
    mh = b1 * (1 - b1) * g / (1 - b1 ** 2)
    vh = b2 * (1 - b2) * g * g / (1 - b2 ** 2)
    np.testing.assert_allclose(th - before, -lr * mh / (np.sqrt(vh) + eps), rtol=1e-12)
