"""GPU parity of the fitting pieces (training appendix) against the FP64
oracle on the same inputs (uniforms drawn on the host): the analytic shape
SDF, the SDF surface sampler, the 2:2:1 training set, per-LOD loss weights,
the fused Adam step, and the fitting loop itself (a few steps from the same
start, same surface samples and uniforms)."""
import numpy as np
import pytest

import oracle
from paper_2101_10994_amd import workloads as W

from cases import make_case, tiny_case
from test_gpu_train import compare, gpu_train, points

pytestmark = pytest.mark.gpu


def dshape(shape):
    from paper_2101_10994_amd import ngl
    return ngl.DeviceShape(shape.spheres, shape.tori)


def test_shape_sdf():
    import torch
    from paper_2101_10994_amd import ngl
    shape = W.prec_shape(0)
    ds = dshape(shape)
    sph, tor = ds.host()
    x = W.soa(np.random.default_rng(0).uniform(-1.1, 1.1, (20000, 3)))
    g = ngl.shape_sdf(ds, torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    r = oracle.shape_sdf(sph, tor, x)
    assert np.abs(g - r).max() <= 2e-6


@pytest.mark.parametrize("shape_fn", [W.tiny_shape, lambda: W.paper_shape(0)])
def test_surface_sampler(shape_fn):
    import torch
    from paper_2101_10994_amd import ngl
    shape = shape_fn()
    ds = dshape(shape)
    sph, tor = ds.host()
    n, delta = 30000, 1e-4
    u = np.random.default_rng(1).uniform(0, 1, (5, n)).astype(np.float32)
    g = ngl.sample_surface(ds, torch.from_numpy(u).cuda(), 256, delta)
    cnt = int(g["count"].item())
    pts = g["pts"][:, :cnt].cpu().numpy()
    r = oracle.sample_surface(sph, tor, u, 256, delta, margin_box=2e-5)
    # every GPU sample lies on the surface (FP64 SDF)
    assert np.all(np.abs(oracle.shape_sdf(sph, tor, pts)) < delta + 2e-6)
    # marginal rays: near a box face, or hit/miss changes for delta +- 2%
    lo = oracle.sample_surface(sph, tor, u, 256, delta * 0.98)
    hi = oracle.sample_surface(sph, tor, u, 256, delta * 1.02)
    marg = r["marginal"] | (lo["hit"] != r["hit"]) | (hi["hit"] != r["hit"])
    assert marg.mean() < 0.01
    assert abs(cnt - int(r["hit"].sum())) <= int(marg.sum())
    # ray order: up to the first marginal ray the two sample lists align;
    # where FP32 rounding moves the stopping step by one the point moves by
    # at most about delta
    first = int(np.argmax(marg)) if marg.any() else n
    k = int(r["hit"][:first].sum())
    assert k > 500
    ref = r["points"][:, :first][:, r["hit"][:first]]
    d = np.abs(pts[:, :k] - ref).max(0)
    assert d.max() <= 2.5 * delta
    assert np.mean(d > 5e-5) <= 0.01


def test_training_points():
    import torch
    from paper_2101_10994_amd import ngl
    shape = W.paper_shape(0)
    ds = dshape(shape)
    sph, tor = ds.host()
    rng = np.random.default_rng(2)
    S = W.surface_points(rng, shape, 3000).T.astype(np.float32)
    N, B = 10000, 500
    uni = rng.uniform(0, 1, (4, N)).astype(np.float32)
    uni[0, :7] = 0.0   # radius inputs of 0 read as 1
    x, t = ngl.training_points(ds, torch.from_numpy(np.ascontiguousarray(S)).cuda(), S.shape[1],
                               torch.from_numpy(uni).cuda(), B, 0.01)
    xg = x.cpu().numpy().transpose(1, 0, 2).reshape(3, N)  # batch-major -> [3][N]
    xo, to = oracle.training_points(sph, tor, S.astype(np.float64), uni, 0.01)
    c = np.arange(N) % 5
    exact = (c < 2) | (c == 4)
    np.testing.assert_array_equal(xg[:, exact], xo[:, exact])
    assert np.abs(xg[:, ~exact].astype(np.float64) - xo[:, ~exact]).max() <= 2e-6
    assert np.abs(t.cpu().numpy() - to).max() <= 4e-6


def test_adam_step():
    import torch
    from paper_2101_10994_amd import ngl
    rng = np.random.default_rng(3)
    shapes = [(7,), (33, 5), (1,), (0,), (1000,)]
    th = [rng.normal(size=s) for s in shapes]
    m = [rng.normal(size=s) * 0.01 for s in shapes]
    v = [np.abs(rng.normal(size=s)) * 1e-4 for s in shapes]
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    th, m, v = [f32(a) for a in th], [f32(a) for a in m], [f32(a) for a in v]
    dt = lambda lst: [torch.tensor(a, dtype=torch.float32, device="cuda") for a in lst]
    gth, gm, gv = dt(th), dt(m), dt(v)
    # the hyper-parameters as the FP32 values the kernel receives
    lr, b1, b2, eps = (float(np.float32(c)) for c in (2e-3, 0.9, 0.999, 1e-8))
    for step in (1, 2, 7):
        g = [f32(rng.normal(size=s)) for s in shapes]
        # cancellation scale of m' = b1 m + (1 - b1) g, before the update
        mscale = [b1 * np.abs(mm) + (1 - b1) * np.abs(gg) for mm, gg in zip(m, g)]
        ngl.adam_step(gth, dt(g), gm, gv, step, lr=lr, beta1=b1, beta2=b2, eps=eps)
        oracle.adam_step(th, g, m, v, step, lr=lr, beta1=b1, beta2=b2, eps=eps)
        c1, c2 = 1 / (1 - b1 ** step), 1 / (1 - b2 ** step)
        for a, b, ms, vv in zip(gth, th, mscale, v):
            upd = lr * c1 * ms / (np.sqrt(vv * c2) + eps)
            assert np.all(np.abs(a.cpu().numpy() - b) <= 1e-6 * np.abs(b) + 1e-6 * upd + 1e-12)
        for a, b, ms in zip(gm, m, mscale):
            assert np.all(np.abs(a.cpu().numpy() - b) <= 4 * 2.0 ** -24 * ms + 1e-30)
        for a, b in zip(gv, v):
            assert np.all(np.abs(a.cpu().numpy() - b) <= 1e-6 * np.abs(b) + 1e-30)
        th = [a.cpu().numpy().astype(np.float64) for a in gth]
        m = [a.cpu().numpy().astype(np.float64) for a in gm]
        v = [a.cpu().numpy().astype(np.float64) for a in gv]


def test_lod_weighted_training():
    import torch
    from paper_2101_10994_amd import ngl
    case = tiny_case(sigma=0.1)
    x, tgt = points(case, np.random.default_rng(4), 3000, 16)
    gm = case.gpu_model()
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda()
    w = [1.0, 0.0, 0.5]
    loss, g = ngl.train_fwd_bwd_lods(gm, xd, td, w)
    got = dict(loss=float(loss.item()), dfeat=[t.cpu().numpy() for t in g.dfeat],
               dW1=[t.cpu().numpy() for t in g.dW1], db1=[t.cpu().numpy() for t in g.db1],
               dw2=[t.cpu().numpy() for t in g.dw2], db2=g.db2.cpu().numpy())
    r = oracle.train_fwd_bwd(case.otree, case.oracle_model(), x, tgt, lod_weight=w)
    for key in ("dW1", "db1", "dw2"):
        assert np.all(got[key][1] == 0)
        got[key][1] = r[key][1]  # exact zeros on both sides; compare() skips nothing
    compare(got, r)
    # all-ones weights are the plain Eq. 4 step, bitwise
    l1, g1 = ngl.train_fwd_bwd_lods(gm, xd, td, [1.0, 1.0, 1.0])
    ref = gpu_train(case, x, tgt)
    assert float(l1.item()) == ref["loss"]
    for a, b in zip(g1.dfeat, ref["dfeat"]):
        assert np.array_equal(a.cpu().numpy(), b)


def fit_case():
    case = make_case(W.sphere_shape(0.55), 16, 3, 8, 32, seed=5, sigma=0.01)
    return case


def test_fit_loop_matches_oracle_steps():
    """Two epochs of 5 batches (10 Adam steps) from the same start with the
    same surface samples and uniforms: parameters agree with the FP64
    oracle's loop (differences come from FP32 gradients, bounded by the
    Adam step size per step)."""
    import torch
    from paper_2101_10994_amd import fit, ngl
    case = fit_case()
    gm = case.gpu_model()
    shape = case.shape
    ds = dshape(shape)
    sph, tor = ds.host()
    rng = np.random.default_rng(6)
    S = np.ascontiguousarray(W.surface_points(rng, shape, 800).T.astype(np.float32))
    N, B, lr = 1000, 200, 1e-3
    unis = [rng.uniform(0, 1, (4, N)).astype(np.float32) for _ in range(2)]
    it = iter(unis)
    f = fit.Fitter(gm, ds, points=N, batch=B, lr=lr, surface=torch.from_numpy(S).cuda(),
                   uniforms=lambda rows, n: torch.from_numpy(next(it)).cuda())
    losses = [f.run_epoch() for _ in range(2)]
    # oracle loop
    om = case.oracle_model()
    params = [*om.feats, *om.W1, *om.b1, *om.w2, om.b2]
    ms = [np.zeros_like(p) for p in params]
    vs = [np.zeros_like(p) for p in params]
    step = 0
    olosses = []
    for e in range(2):
        xo, to = oracle.training_points(sph, tor, S.astype(np.float64), unis[e], 0.01)
        to32 = to.astype(np.float32)
        bl = []
        for b in range(N // B):
            xb = np.ascontiguousarray(xo[:, b * B:(b + 1) * B])
            r = oracle.train_fwd_bwd(case.otree, om, xb, to32[b * B:(b + 1) * B])
            grads = [*r["dfeat"], *r["dW1"], *r["db1"], *r["dw2"], r["db2"]]
            step += 1
            oracle.adam_step(params, grads, ms, vs, step, lr=lr)
            bl.append(r["loss"])
        olosses.append(float(np.mean(bl)))
    np.testing.assert_allclose(losses, olosses, rtol=1e-3)
    got = [t.detach().double().cpu().numpy() for t in ngl.parameters(gm)]
    for a, b in zip(got, params):
        d = np.abs(a - b)
        assert d.max() <= 2 * lr * step
        assert np.median(d) <= 1e-5


def test_fit_reduces_loss_and_schedules():
    import torch
    from paper_2101_10994_amd import fit, ngl
    case = fit_case()
    ds = dshape(case.shape)
    gm = case.gpu_model()
    f = fit.Fitter(gm, ds, points=20000, batch=500, lr=1e-3, seed=1)
    first = f.run_epoch()
    for _ in range(4):
        last = f.run_epoch()
    assert last < 0.5 * first
    # progressive: before the coarser LODs are added their features stay put
    gm2 = case.gpu_model()
    f2 = fit.Fitter(gm2, ds, points=5000, batch=500, schedule="progressive", grow_every=2, seed=2)
    before = [t.clone() for t in gm2.feats]
    assert f2.active_lods() == [3]
    f2.run_epoch()
    assert torch.equal(gm2.feats[0], before[0]) and torch.equal(gm2.feats[1], before[1])
    assert not torch.equal(gm2.feats[2], before[2])
    f2.run_epoch()
    assert f2.active_lods() == [2, 3]
    # frozen decoders: only features move
    gm3 = case.gpu_model()
    f3 = fit.Fitter(gm3, ds, points=5000, batch=500, freeze_decoders=True, seed=3)
    dec = [t.clone() for t in (*gm3.W1, *gm3.b1, *gm3.w2, gm3.b2)]
    f3.run_epoch()
    for a, b in zip(dec, (*gm3.W1, *gm3.b1, *gm3.w2, gm3.b2)):
        assert torch.equal(a, b)
