"""Benchmark of the neural geometric LOD hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input on
the paper-scale workload (union of 8 spheres and a torus, 5 LODs at
resolutions 4..64, 32-dim corner features, 35->128->1 decoders):
  * 2^20 SDF queries at LOD 5 (half uniform, half near-surface);
  * one 1024x1024 frame: camera rays, breadth-first ray-octree
    intersection down to the finest depth, adaptive-stepping sphere trace
    (<= 100 SDF evaluations per ray, hit threshold 1e-4);
  * one training forward+backward of Eq. 4 on 2^19 points;
  * the same queries and trace in the BF16-MFMA form (FP16 features, BF16
    first decoder layer with FP32 accumulation) next to the plain FP32 form.
Prints one JSON line.  `value` is octree SDF queries per second of the
query batch; frame rate and training points per second are reported next
to it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "octree SDF queries/s, 1024^2 sphere-trace fps, fwd+bwd points/s at fixed err"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 (packed vector / matrix) peak

# Algorithmic work per SDF evaluation at LOD 5 with m = 32, h = 128:
# gather 5 levels x (8 corner rows x 32 x 4 B + 8 corner ids x 4 B) = 5,280 B;
# a query adds its 12 B point and 4 B result, a trace step about 28 B of
# ray/pair state.  Flops: trilinear 5 x 8 x 32 x 2 + decoder 2 x (35 x 128 +
# 128) + 2 x 128.
GATHER_BYTES = 5 * (8 * 32 * 4 + 8 * 4)
QUERY_BYTES = GATHER_BYTES + 16
TRACE_STEP_BYTES = GATHER_BYTES + 28
EVAL_FLOPS = 5 * 8 * 32 * 2 + 2 * (35 * 128 + 128) + 2 * 128
# Traversal: 16 B per slab-tested candidate (8 B pair read, 8 B per emitted
# child written; ray and voxel records amortised over their pairs).
TRAVERSAL_BYTES = 16

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs
# of this bench (KiB per dispatch), each scaled by the reading of the same
# counter for a plain 256 MiB device copy (FETCH_SIZE reads 131,088 KiB,
# WRITE_SIZE 262,144 KiB).  Valid only while the kernel's sources hash to
# the recorded value; otherwise traffic is reported as null.
COUNTERS = {
    # both launches of the phased FP32 trace (first 24 evaluations, then the wide kernel)
    "k_sphere_trace": {"sources": ["ngl_trace_impl.h", "ngl_device.h", "ngl_mfma.h"],
                       "sha256": "f3eea318163c0b52781a9996e82e8ca1242b8c3f5a5dbe11ab5de26d506966ef",
                       "fetch_kib": 312591.9 + 22987.4, "write_kib": 33450.7 + 3516.8},
    # every launch of one traversal to depth 6 (root and six child passes,
    # ray inverses, segment offsets)
    "traverse": {"sources": ["ngl_traverse.hip", "ngl_device.h"],
                 "sha256": "d1c4196cc585dd988bfdc7542ad8170f78014f558a7bdd22b721f7c9ab6091b1",
                 "fetch_kib": 348071.9, "write_kib": 380740.2},
    # k_query_coop, FP32 features and matrix-core decoder
    "k_query": {"sources": ["ngl_query_impl.h", "ngl_device.h", "ngl_mfma.h"],
                "sha256": "3cfbe96b6ca4fb74ed93a90f236ee5dcc1c33da45d08b2c9b227385948328b9c",
                "fetch_kib": 105003.0, "write_kib": 4096.0},
}
FETCH_SCALE = (256 << 10) / 131087.9
WRITE_SCALE = (256 << 10) / 262144.0


def traversal_candidates(ngl, model, o, d, target):
    """Slab tests of one traversal to `target`: the root test of every ray
    plus every occupied child of every hit pair at depths 0..target-1."""
    pop = np.array([bin(i).count("1") for i in range(256)], np.int64)
    cand = o.shape[1]
    for dd in range(target):
        vox = ngl.trace_octree(model, o, d, dd)["vox"].cpu().numpy()
        cand += int(pop[model.tree.child_mask[dd][vox]].sum())
    return cand


def sources_sha256(names):
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2101_10994_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch, or None if the sources changed."""
    c = COUNTERS.get(kernel)
    if c is None or sources_sha256(c["sources"]) != c["sha256"]:
        return None
    return (c["fetch_kib"] * FETCH_SCALE + c["write_kib"] * WRITE_SCALE) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(device):
    import torch
    from paper_2101_10994_amd import ngl
    from paper_2101_10994_amd import workloads as W

    cfg = W.PAPER
    shape = W.paper_shape(0)
    res = 2 ** (cfg.num_lods + 1)
    ijk = W.occupancy_ijk(shape, res)
    tree = ngl.Octree(ijk, cfg.num_lods, device=device)
    rs = W.rngs(0)
    feats = W.embedded_features(rs[W.STREAM_FEAT], shape, tree.corner_positions(), cfg.feat_dim)
    dec = W.spread_decoders(rs[W.STREAM_DEC], cfg.num_lods, cfg.feat_dim, cfg.hidden)
    f32 = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=device)
    model = ngl.Model(tree, [f32(f) for f in feats], [f32(w) for w in dec["W1"]], [f32(b) for b in dec["b1"]],
                      [f32(w) for w in dec["w2"]], f32(dec["b2"]), pack=True)
    # the BF16-MFMA form of the same model: FP16 features, BF16 first layer
    half = ngl.Model(tree, [f32(f).half() for f in feats], [f32(w).bfloat16() for w in dec["W1"]],
                     [f32(b) for b in dec["b1"]], [f32(w) for w in dec["w2"]], f32(dec["b2"]), pack=True)
    xq = W.soa(W.paper_queries(0, shape, cfg.n_query))
    xt, tg = W.train_points(1, shape, W.TRAIN.n_query)
    return dict(cfg=cfg, shape=shape, ijk=ijk, tree=tree, model=model, half=half, feats=feats, dec=dec,
                xq_host=xq, xq=torch.from_numpy(xq).to(device), xt_host=W.soa(xt), tg_host=tg,
                xt=torch.from_numpy(W.soa(xt)).to(device), tg=torch.from_numpy(tg).to(device))


class Timer:
    """HIP events on the current stream around one component."""

    def __init__(self):
        self.ms = []

    def __enter__(self):
        import torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self._pending = (self.a, self.b)
        self.ms.append(self._pending)

    def values(self):
        return [a.elapsed_time(b) for a, b in self.ms]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="approximate CPU-baseline budget")
    ap.add_argument("--no-batch", action="store_true", help="skip the 16-shape batched render")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the decoder-alone, LOD-selection, fitting and octree-build components")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, run one plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--only", choices=["query", "frame", "train", "half", "decoder", "precision", "fit", "batch"], default=None,
                    help="run a single component (profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the hot path is single-GPU (one process per GPU would replicate the "
              "octree and shard rays/points; that form is not implemented). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2101_10994_amd import ngl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda"
    S = setup(dev)
    cfg, model = S["cfg"], S["model"]
    W_, H_ = cfg.width, cfg.height
    R = W_ * H_
    lod = cfg.num_lods
    eye = cfg.eye

    # buffers
    sdf = torch.empty(cfg.n_query, dtype=torch.float32, device=dev)
    o = torch.empty((3, R), dtype=torch.float32, device=dev)
    d = torch.empty((3, R), dtype=torch.float32, device=dev)
    ngl.camera_rays(eye, (0, 0, 0), (0, 1, 0), 45.0, W_, H_, out=(o, d))
    first = ngl.trace_octree(model, o, d, lod + 1)  # sizes the pair lists once
    buf = ngl.TraceBuffers(R, first["max_list"], dev)
    hits = dict(vox=buf.vox, t_in=buf.t_in, t_out=buf.t_out, ray_off=buf.ray_off)
    tr = dict(t=torch.empty(R, dtype=torch.float32, device=dev),
              status=torch.empty(R, dtype=torch.uint8, device=dev),
              steps=torch.empty(R, dtype=torch.int32, device=dev),
              hit_vox=torch.empty(R, dtype=torch.int32, device=dev))
    have_train = True
    try:
        grads = ngl.Grads(model)
        tws = ngl.train_workspace(model, S["xt"].shape[1], dev)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    except ngl.NGLError:
        have_train = False

    do_q = args.only in (None, "query")
    do_f = args.only in (None, "frame")
    do_t = args.only in (None, "train") and have_train
    do_h = args.only in (None, "half")
    do_v = args.only is None
    f32_mode = ngl.get_option(ngl.OPT_F32_DECODER)
    tvq, tvs = Timer(), Timer()
    sdf_v = torch.empty(cfg.n_query, dtype=torch.float32, device=dev)
    tr_v = dict(t=torch.empty(R, dtype=torch.float32, device=dev),
                status=torch.empty(R, dtype=torch.uint8, device=dev),
                steps=torch.empty(R, dtype=torch.int32, device=dev),
                hit_vox=torch.empty(R, dtype=torch.int32, device=dev))
    tq, tc, tt, ts, ttr = Timer(), Timer(), Timer(), Timer(), Timer()
    thq, ths, tn, thn = Timer(), Timer(), Timer(), Timer()
    h_fd = ngl.default_normal_step(model)
    nrm = torch.empty((3, R), dtype=torch.float32, device=dev)
    nrm_h = torch.empty((3, R), dtype=torch.float32, device=dev)
    half = S["half"]
    sdf_h = torch.empty(cfg.n_query, dtype=torch.float32, device=dev)
    tr_h = dict(t=torch.empty(R, dtype=torch.float32, device=dev),
                status=torch.empty(R, dtype=torch.uint8, device=dev),
                steps=torch.empty(R, dtype=torch.int32, device=dev),
                hit_vox=torch.empty(R, dtype=torch.int32, device=dev))

    def step(timed):
        if do_q:
            if timed:
                with tq:
                    ngl.query_sdf(model, S["xq"], lod, out=sdf)
            else:
                ngl.query_sdf(model, S["xq"], lod, out=sdf)
        if do_f:
            if timed:
                with tc:
                    ngl.camera_rays(eye, (0, 0, 0), (0, 1, 0), 45.0, W_, H_, out=(o, d))
                with tt:
                    ngl.trace_octree_into(model, o, d, lod + 1, buf)
                with ts:
                    ngl.sphere_trace(model, o, d, lod, 0.0, hits, cfg.max_steps, cfg.delta, out=tr, image_width=W_)
                with tn:
                    ngl.sdf_normals(model, lod, 0.0, h_fd, rays=(o, d, tr["t"], tr["status"]), out=nrm)
            else:
                ngl.camera_rays(eye, (0, 0, 0), (0, 1, 0), 45.0, W_, H_, out=(o, d))
                ngl.trace_octree_into(model, o, d, lod + 1, buf)
                ngl.sphere_trace(model, o, d, lod, 0.0, hits, cfg.max_steps, cfg.delta, out=tr, image_width=W_)
                ngl.sdf_normals(model, lod, 0.0, h_fd, rays=(o, d, tr["t"], tr["status"]), out=nrm)
        if do_v:
            # FP32 decoder on the vector ALUs (the per-lane form), for comparison
            ngl.set_option(ngl.OPT_F32_DECODER, 0)
            if timed:
                with tvq:
                    ngl.query_sdf(model, S["xq"], lod, out=sdf_v)
                with tvs:
                    ngl.sphere_trace(model, o, d, lod, 0.0, hits, cfg.max_steps, cfg.delta, out=tr_v, image_width=W_)
            else:
                ngl.query_sdf(model, S["xq"], lod, out=sdf_v)
                ngl.sphere_trace(model, o, d, lod, 0.0, hits, cfg.max_steps, cfg.delta, out=tr_v, image_width=W_)
            ngl.set_option(ngl.OPT_F32_DECODER, f32_mode)
        if do_h:
            # BF16-MFMA form: same queries; the trace reuses the frame's hit lists
            if not do_f:
                ngl.camera_rays(eye, (0, 0, 0), (0, 1, 0), 45.0, W_, H_, out=(o, d))
                ngl.trace_octree_into(model, o, d, lod + 1, buf)
            if timed:
                with thq:
                    ngl.query_sdf(half, S["xq"], lod, out=sdf_h)
                with ths:
                    ngl.sphere_trace(half, o, d, lod, 0.0, hits, cfg.max_steps, cfg.delta, out=tr_h, image_width=W_)
                with thn:
                    ngl.sdf_normals(half, lod, 0.0, h_fd, rays=(o, d, tr_h["t"], tr_h["status"]), out=nrm_h)
            else:
                ngl.query_sdf(half, S["xq"], lod, out=sdf_h)
                ngl.sphere_trace(half, o, d, lod, 0.0, hits, cfg.max_steps, cfg.delta, out=tr_h, image_width=W_)
                ngl.sdf_normals(half, lod, 0.0, h_fd, rays=(o, d, tr_h["t"], tr_h["status"]), out=nrm_h)
        if do_t:
            if timed:
                with ttr:
                    ngl.train_fwd_bwd(model, S["xt"], S["tg"], grads=grads, ws=tws, loss=loss)
            else:
                ngl.train_fwd_bwd(model, S["xt"], S["tg"], grads=grads, ws=tws, loss=loss)

    for k in range(args.warmup):
        step(False)
        log("warmup step %d done" % k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log("timed %d steps: %.3f ms/step" % (args.steps, ms_per_step))
    if do_f:
        cnt = buf.counts.cpu()
        assert int(cnt[1]) <= buf.capacity, "pair list overflowed during timing"

    mean = lambda tm: float(np.mean(tm.values())) if tm.ms else None
    comp = {}
    qps = None
    if do_q:
        q_ms = mean(tq)
        qps = cfg.n_query / (q_ms * 1e-3)
        comp["query"] = {"ms": q_ms, "queries_per_s": qps, "points": cfg.n_query, "lod": lod}
    if do_f:
        status = tr["status"].cpu().numpy()
        steps_arr = tr["steps"].cpu().numpy()
        frame_ms = mean(tc) + mean(tt) + mean(ts) + mean(tn)
        n_cand = traversal_candidates(ngl, model, o, d, lod + 1)
        trav_gbs = TRAVERSAL_BYTES * n_cand / (mean(tt) * 1e6)
        n_eval = int(steps_arr.sum())
        comp["frame"] = {"ms": frame_ms, "fps": 1e3 / frame_ms, "rays_per_s": R / (frame_ms * 1e-3),
                         "camera_ms": mean(tc), "traverse_ms": mean(tt), "trace_ms": mean(ts),
                         "normals_ms": mean(tn), "normal_step": h_fd,
                         "traverse_candidates": n_cand, "traverse_algorithmic_GBps": trav_gbs,
                         "traverse_hbm_frac": trav_gbs / HBM_PEAK_GBS,
                         "visible_px": int((status == ngl.HIT).sum()), "rays_with_voxels": int(
                             (buf.ray_off[1:] > buf.ray_off[:-1]).sum()),
                         "final_pairs": int(buf.counts[0]), "sdf_evals": n_eval,
                         "sdf_evals_per_s": n_eval / (mean(ts) * 1e-3)}
    if do_h:
        hq_ms, hs_ms = mean(thq), mean(ths)
        st_h = tr_h["status"].cpu().numpy()
        n_eval_h = int(tr_h["steps"].cpu().numpy().sum())
        comp["bf16_form"] = {"features": "f16", "decoder": "bf16 MFMA, fp32 accumulate",
                             "query_ms": hq_ms, "queries_per_s": cfg.n_query / (hq_ms * 1e-3),
                             "trace_ms": hs_ms, "sdf_evals": n_eval_h, "sdf_evals_per_s": n_eval_h / (hs_ms * 1e-3),
                             "visible_px": int((st_h == ngl.HIT).sum()),
                             "normals_ms": mean(thn),
                             "frame_ms": (mean(tc) + mean(tt) + hs_ms + mean(thn)) if do_f else None}
        if do_q:
            comp["bf16_form"]["max_abs_diff_vs_fp32"] = float((sdf_h - sdf).abs().max())
    if do_v:
        comp["fp32_valu_form"] = {"decoder": "fp32 per lane on the vector ALUs", "query_ms": mean(tvq),
                                  "queries_per_s": cfg.n_query / (mean(tvq) * 1e-3), "trace_ms": mean(tvs),
                                  "max_abs_diff_vs_mfma": float((sdf_v - sdf).abs().max())}
    if do_t:
        tr_ms = mean(ttr)
        comp["train"] = {"ms": tr_ms, "points_per_s": S["xt"].shape[1] / (tr_ms * 1e-3), "points": S["xt"].shape[1]}

    # Roofline of the kernel behind `value` (the cooperative query kernel,
    # one launch per batch, timed alone with HIP events on its stream).  Its
    # binding roof is FP32 compute: the measured HBM traffic per launch gives
    # an arithmetic intensity whose HBM roof (intensity x 8 TB/s) lies above
    # the FP32 peak, and the feature table is served from the caches.  All
    # flops (first layer on the FP32 matrix cores, trilinear weights and the
    # second layer on the vector ALUs) are priced at the FP32 peak.  The
    # HBM-priced view (algorithmic bytes, which the caches absorb, and the
    # measured traffic) is kept beside it.
    roof = None
    if do_q:
        ms = comp["query"]["ms"]
        nbytes, flops = QUERY_BYTES * cfg.n_query, EVAL_FLOPS * cfg.n_query
        traffic = measured_traffic("k_query")
        tfl = flops / (ms * 1e-3) / 1e12
        comp["query"]["algorithmic_GBps"] = nbytes / (ms * 1e6)
        comp["query"]["hbm_traffic_bytes"] = traffic
        roof = {"kernel": "k_query_coop", "bound": "mfma", "achieved": tfl, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tfl / FP32_PEAK_TFLOPS, "traffic": traffic,
                "flops_per_launch": flops, "flops_per_query": EVAL_FLOPS,
                "hbm": {"algorithmic_bytes_per_launch": nbytes, "algorithmic_GBps": nbytes / (ms * 1e6),
                        "measured_GBps": traffic / (ms * 1e6) if traffic else None,
                        "measured_frac": traffic / (ms * 1e6) / HBM_PEAK_GBS if traffic else None,
                        "hbm_roof_tflops": (flops / traffic) * HBM_PEAK_GBS / 1e3 if traffic else None},
                "targets": {"gather_hbm_frac": 0.5, "decoder_mfma_frac": 0.4}}
    if do_f:
        ev = comp["frame"]["sdf_evals"]
        tms = comp["frame"]["trace_ms"]
        traffic = measured_traffic("k_sphere_trace")
        tfl = EVAL_FLOPS * ev / (tms * 1e-3) / 1e12
        comp["frame"]["trace_roofline"] = {
            "kernels": "k_sphere_trace + k_sphere_trace_wide", "bound": "mfma", "achieved": tfl,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tfl / FP32_PEAK_TFLOPS,
            "algorithmic_GBps": TRACE_STEP_BYTES * ev / (tms * 1e6), "traffic": traffic,
            "measured_hbm_frac": traffic / (tms * 1e6) / HBM_PEAK_GBS if traffic else None}
        comp["frame"]["trace_algorithmic_GBps"] = TRACE_STEP_BYTES * ev / (tms * 1e6)
        comp["frame"]["trace_hbm_traffic_bytes"] = traffic
        ttr = measured_traffic("traverse")
        trms = comp["frame"]["traverse_ms"]
        comp["frame"]["traverse_hbm_traffic_bytes"] = ttr
        comp["frame"]["traverse_measured_hbm_frac"] = ttr / (trms * 1e6) / HBM_PEAK_GBS if ttr else None

    if args.calibrate_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # calibrate the HBM-traffic counters of the kernels above
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only == "batch" or (args.only is None and not args.no_batch):
        comp["batch"] = run_batch(dev, args.steps, args.warmup)
    if args.only == "decoder" or (args.only is None and not args.no_extras):
        comp["decoder_bf16"] = run_decoder(S, dev, args.steps, args.warmup)
    if args.only is None and not args.no_extras:
        comp["frame_lod_select"] = run_lod_select(model, cfg, o, d, buf, args.steps, args.warmup)
    if args.only == "precision" or (args.only is None and not args.no_extras):
        comp["precision"] = run_precision(dev, max(3, args.steps // 2), 1)
    if args.only == "fit" or (args.only is None and not args.no_extras):
        comp["fit"] = run_fit(S, dev)
    if args.only is None and not args.no_extras:
        comp["octree_build"] = run_octree_build(dev, args.steps)
        if do_h:
            hq = comp["bf16_form"]["queries_per_s"] * DEC_MFMA_FLOPS / 1e12
            # computed from the query rate (the counters of the fused kernel are in profiles/)
            comp["bf16_form"]["fused_decoder_mfma_frac_computed"] = hq / BF16_PEAK_TFLOPS

    cpu = None
    if not args.no_cpu and do_q:
        cpu = cpu_baseline(S, args.cpu_seconds)

    out = {"metric": METRIC, "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "f32_decoder": ["vector ALU", "matrix cores (v_mfma_f32_16x16x4f32)"][f32_mode],
           "config": {"workload": "union8s1t-5lod-m32: 2^20 queries at LOD 5 + 1024x1024 frame "
                                  "(<=100 steps, delta 1e-4, FD normals at hits)" + (" + 2^19-point train step" if do_t else ""),
                      "lods": cfg.num_lods, "feat_dim": cfg.feat_dim, "hidden": cfg.hidden,
                      "queries": cfg.n_query, "image": [W_, H_], "train_points": S["xt"].shape[1]},
           "roofline": roof, "cpu_baseline": cpu, "components": comp}
    print(json.dumps(out), flush=True)


BF16_PEAK_TFLOPS = 2500.0     # MI355X dense BF16 matrix peak
DEC_MFMA_FLOPS = 2 * 32 * 128  # MFMA-eligible flops of one decoder on z (m = 32, h = 128)


def run_decoder(S, dev, steps, warmup):
    """The decoder alone (BF16 weights of the step's half-precision model)
    on 2^20 points whose BF16 z rows (64 MB) and positions are resident on
    the device: the split form of the query, for the matrix-core
    utilisation of the decoder."""
    import torch
    from paper_2101_10994_amd import ngl
    half, cfg = S["half"], S["cfg"]
    P = cfg.n_query
    g = torch.Generator(device=dev)
    g.manual_seed(1234)
    z = (0.3 * torch.randn((P, cfg.feat_dim), generator=g, device=dev)).to(torch.bfloat16)
    x = S["xq"]
    out = torch.empty(P, dtype=torch.float32, device=dev)
    for _ in range(warmup):
        ngl.decode_sdf(half, cfg.num_lods, z, x=x, out=out)
    tm = Timer()
    for _ in range(steps):
        with tm:
            ngl.decode_sdf(half, cfg.num_lods, z, x=x, out=out)
    torch.cuda.synchronize()
    ms = float(np.median(tm.values()))
    tf = DEC_MFMA_FLOPS * P / (ms * 1e-3) / 1e12
    return {"points": P, "ms": ms, "points_per_s": P / (ms * 1e-3), "z_bytes": P * cfg.feat_dim * 2,
            "mfma_tflops": tf, "mfma_frac_bf16": tf / BF16_PEAK_TFLOPS,
            "note": "2*32*128 flops per point (first layer on z); inputs 80 B per point"}


LOD_SELECT = (2.0, 3.0, 5.0, 2.0)  # d_near, d_far, lod_near, lod_far


def run_precision(dev, steps, warmup):
    """The precision workload: 7 LODs (resolutions 4..256) over a seeded union
    of 32 spheres and 4 tori, 32-dim FP16 features, BF16 decoders on the
    matrix cores (SDF-embedded features read through every hidden unit),
    packed.  Timed: 2^22 queries (half uniform, half near-surface) at
    L = 5 + alpha with alpha ~ U[0,1) per query, and one 1920x1080 frame
    (camera, traversal to depth 7, trace at L = 5 + alpha for one seeded
    alpha, FD normals at the hits).  The FP32 form of the same stored values
    (FP32 matrix-core decoder) runs the same queries and frame once for the
    BF16 form's error."""
    import torch
    from paper_2101_10994_amd import ngl
    from paper_2101_10994_amd import workloads as W
    cfg = W.PREC
    t0 = time.perf_counter()
    shape = W.prec_shape(0)
    ijk = W.occupancy_ijk(shape, 256)
    tree = ngl.Octree(ijk, cfg.num_lods, device=dev)
    rs = W.rngs(0)
    feats = W.embedded_features(rs[W.STREAM_FEAT], shape, tree.corner_positions(), cfg.feat_dim)
    dec = W.spread_decoders(rs[W.STREAM_DEC], cfg.num_lods, cfg.feat_dim, cfg.hidden)
    f32 = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    b1, w2, b2 = [f32(b) for b in dec["b1"]], [f32(w) for w in dec["w2"]], f32(dec["b2"])
    half = ngl.Model(tree, [f32(f).half() for f in feats], [f32(w).bfloat16() for w in dec["W1"]], b1, w2, b2,
                     pack=True)
    full = ngl.Model(tree, [f.float() for f in half.feats], [w.float() for w in half.W1], b1, w2, b2, pack=True)
    x = torch.from_numpy(W.soa(W.paper_queries(0, shape, cfg.n_query))).to(dev)
    app = torch.from_numpy(np.random.default_rng(5).uniform(0, 1, cfg.n_query).astype(np.float32)).to(dev)
    alpha = float(np.float32(np.random.default_rng(1080).uniform(0.0, 1.0)))
    lod = cfg.query_lod
    depth = lod + 2
    R = cfg.width * cfg.height
    o = torch.empty((3, R), dtype=torch.float32, device=dev)
    d = torch.empty((3, R), dtype=torch.float32, device=dev)
    ngl.camera_rays(cfg.eye, (0, 0, 0), (0, 1, 0), 45.0, cfg.width, cfg.height, out=(o, d))
    first = ngl.trace_octree(half, o, d, depth)
    buf = ngl.TraceBuffers(R, first["max_list"], dev)
    hits = dict(vox=buf.vox, t_in=buf.t_in, t_out=buf.t_out, ray_off=buf.ray_off)
    mk = lambda: dict(t=torch.empty(R, dtype=torch.float32, device=dev),
                      status=torch.empty(R, dtype=torch.uint8, device=dev),
                      steps=torch.empty(R, dtype=torch.int32, device=dev),
                      hit_vox=torch.empty(R, dtype=torch.int32, device=dev))
    tr, tr32 = mk(), mk()
    sdf = torch.empty(cfg.n_query, dtype=torch.float32, device=dev)
    nrm = torch.empty((3, R), dtype=torch.float32, device=dev)
    h_fd = 2.0 / 256 / 16.0
    setup_s = time.perf_counter() - t0
    tq, tc, tt, ts, tn = Timer(), Timer(), Timer(), Timer(), Timer()
    for k in range(warmup + steps):
        timed = k >= warmup
        with (tq if timed else Timer()):
            ngl.query_sdf(half, x, lod, alpha_pp=app, out=sdf)
        with (tc if timed else Timer()):
            ngl.camera_rays(cfg.eye, (0, 0, 0), (0, 1, 0), 45.0, cfg.width, cfg.height, out=(o, d))
        with (tt if timed else Timer()):
            ngl.trace_octree_into(half, o, d, depth, buf)
        with (ts if timed else Timer()):
            ngl.sphere_trace(half, o, d, lod, alpha, hits, cfg.max_steps, cfg.delta, out=tr, image_width=cfg.width)
        with (tn if timed else Timer()):
            ngl.sdf_normals(half, lod, alpha, h_fd, rays=(o, d, tr["t"], tr["status"]), out=nrm)
    torch.cuda.synchronize()
    assert int(buf.counts[1]) <= buf.capacity, "pair list overflowed during timing"
    med = lambda tm: float(np.median(tm.values()))
    sdf32 = ngl.query_sdf(full, x, lod, alpha_pp=app)["sdf"]
    ngl.sphere_trace(full, o, d, lod, alpha, hits, cfg.max_steps, cfg.delta, out=tr32, image_width=cfg.width)
    torch.cuda.synchronize()
    st, st32 = tr["status"].cpu().numpy(), tr32["status"].cpu().numpy()
    both = (st == ngl.HIT) & (st32 == ngl.HIT)
    dt = np.abs(tr["t"].cpu().numpy()[both].astype(np.float64) - tr32["t"].cpu().numpy()[both]) / (2.0 / 256)
    err = (sdf - sdf32).abs()
    frame_ms = med(tc) + med(tt) + med(ts) + med(tn)
    return {"lods": cfg.num_lods, "finest_res": 256, "voxels": int(tree.nvox.sum()), "corners": int(tree.ncorner.sum()),
            "features": "f16", "decoder": "bf16 MFMA (activations as bf16 hi+lo), fp32 accumulate",
            "queries": cfg.n_query, "query_lod": "5 + alpha, alpha ~ U[0,1) per query",
            "query_ms": med(tq), "queries_per_s": cfg.n_query / (med(tq) * 1e-3),
            "image": [cfg.width, cfg.height], "frame_alpha": alpha, "frame_ms": frame_ms, "fps": 1e3 / frame_ms,
            "camera_ms": med(tc), "traverse_ms": med(tt), "trace_ms": med(ts), "normals_ms": med(tn),
            "final_pairs": int(buf.counts[0]), "visible_px": int((st == ngl.HIT).sum()),
            "sdf_evals": int(tr["steps"].sum()),
            "vs_fp32_form": {"max_abs_sdf_diff": float(err.max()), "median_abs_sdf_diff": float(err.median()),
                             "status_agree_frac": float((st == st32).mean()),
                             "hit_dt_finest_voxels_p50": float(np.median(dt)) if dt.size else None,
                             "hit_dt_finest_voxels_p999": float(np.quantile(dt, 0.999)) if dt.size else None,
                             "hit_dt_finest_voxels_max": float(dt.max()) if dt.size else None},
            "setup_s": setup_s}


def run_lod_select(model, cfg, o, d, buf, steps, warmup):
    """The step's 1024^2 frame with per-pixel LOD selection: LOD 5 up to
    distance 2.0 from the eye (the nearest surfaces are at about 1.6), LOD 2
    from 3.0 on, linear in between (the traversal runs to the LOD-5 depth;
    rays are grouped by LOD on the device and each group is traced with its
    two decoders)."""
    import torch
    from paper_2101_10994_amd import ngl
    sel = ngl.lod_select(*LOD_SELECT)
    hits = dict(vox=buf.vox, t_in=buf.t_in, t_out=buf.t_out, ray_off=buf.ray_off)
    tt, ts = Timer(), Timer()
    out = None
    for k in range(warmup + steps):
        if k < warmup:
            ngl.trace_octree_into(model, o, d, cfg.num_lods + 1, buf)
            out = ngl.sphere_trace_lod(model, o, d, cfg.num_lods + 1, sel, hits, cfg.max_steps, cfg.delta, out=out)
            continue
        with tt:
            ngl.trace_octree_into(model, o, d, cfg.num_lods + 1, buf)
        with ts:
            out = ngl.sphere_trace_lod(model, o, d, cfg.num_lods + 1, sel, hits, cfg.max_steps, cfg.delta, out=out)
    torch.cuda.synchronize()
    lod = out["lod"].cpu().numpy()
    st = out["status"].cpu().numpy()
    hit = st == ngl.HIT
    trav, trace = float(np.mean(tt.values())), float(np.mean(ts.values()))
    return {"selection": dict(zip(("d_near", "d_far", "lod_near", "lod_far"), LOD_SELECT)),
            "traverse_ms": trav, "trace_ms": trace, "ms": trav + trace, "visible_px": int(hit.sum()),
            "sdf_evals": int(out["steps"].sum()), "mean_lod_of_hits": float(lod[hit].mean()) if hit.any() else None,
            "rays_per_lod": {str(L): int(((np.floor(lod) == L) | ((L == 5) & (lod >= 5))).sum()) for L in (2, 3, 4, 5)}}


def run_fit(S, dev):
    """The fitting loop of the training appendix on the paper-scale shape
    and octree, from a random FP32 init: 500,000 points per epoch in the
    2:2:1 split (surface samples from the SDF sampler), Adam at lr 1e-3,
    all LODs jointly; one warm-up epoch, then one timed epoch at the
    paper's batch of 512 and one at a batch of 16,384."""
    import torch
    from paper_2101_10994_amd import fit, ngl
    from paper_2101_10994_amd import workloads as W
    cfg, tree, shape = S["cfg"], S["tree"], S["shape"]
    rs = W.rngs(7)
    feats = W.features(rs[W.STREAM_FEAT], tree.ncorner, cfg.feat_dim)
    dec = W.decoders(rs[W.STREAM_DEC], cfg.num_lods, cfg.feat_dim + 3, cfg.hidden)
    f32 = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    model = ngl.Model(tree, [f32(f) for f in feats], [f32(w) for w in dec["W1"]], [f32(b) for b in dec["b1"]],
                      [f32(w) for w in dec["w2"]], f32(dec["b2"]))
    ds = ngl.DeviceShape(shape.spheres, shape.tori, device=dev)
    out = {"points_per_epoch": 500000, "lr": 1e-3, "schedule": "joint"}
    for batch in (512, 16384):
        f = fit.Fitter(model, ds, points=500000, batch=batch, seed=batch)
        first = f.run_epoch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = f.run_epoch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out["batch_%d" % batch] = {
            "epoch_ms": ms, "points_per_s": f.N / (ms * 1e-3), "steps": f.N // batch, "loss_epoch1": first,
            "loss_epoch2": last, "surface_samples": int(f.sampler["count"].item())}
    return out


def run_octree_build(dev, steps):
    """Device octree build (the initialisation pass) from the 7-LOD
    occupancy of the 32-sphere/4-torus union (res 256), against the host
    build of the same cells."""
    import torch
    from paper_2101_10994_amd import ngl
    from paper_2101_10994_amd import workloads as W
    ijk = W.occupancy_ijk(W.prec_shape(0), 256)
    t0 = time.perf_counter()
    ngl.Octree(ijk, 7, device=None)
    host_ms = (time.perf_counter() - t0) * 1e3
    dt = ngl.DeviceOctree(torch.from_numpy(ijk.astype(np.int32)).to(dev), 7)
    tm = Timer()
    for _ in range(steps):
        with tm:
            dt.rebuild()
    torch.cuda.synchronize()
    ms = float(np.median(tm.values()))
    return {"cells": int(len(ijk)), "lods": 7, "voxels": int(dt.nvox.sum()), "corners": int(dt.ncorner.sum()),
            "device_ms": ms, "host_ms": host_ms, "cells_per_s": len(ijk) / (ms * 1e-3)}


def run_batch(dev, steps, warmup):
    """16 seeded shapes (3..7 LODs, FP16 features, BF16 decoders), one
    512x512 view each at its own camera and LOD, traced by one persistent
    launch per frame; launch shape picked by the autotuner; the frame is
    captured in a graph and timed by replaying it."""
    import torch
    from paper_2101_10994_amd import autotune, ngl
    from paper_2101_10994_amd import workloads as W
    cfg = W.BATCH
    t0 = time.perf_counter()
    scene = W.batch_scene(0, 16, cfg.width, cfg.height)
    models, views = [], []
    for i, it in enumerate(scene):
        L = it["num_lods"]
        ijk = W.occupancy_ijk(it["shape"], 2 ** (L + 1))
        tree = ngl.Octree(ijk, L, device=dev)
        rs = W.rngs(100 + i)
        feats = W.embedded_features(rs[W.STREAM_FEAT], it["shape"], tree.corner_positions(), cfg.feat_dim)
        dec = W.spread_decoders(rs[W.STREAM_DEC], L, cfg.feat_dim, cfg.hidden)
        f32 = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
        models.append(ngl.Model(tree, [f32(f).half() for f in feats], [f32(w).bfloat16() for w in dec["W1"]],
                                [f32(b) for b in dec["b1"]], [f32(w) for w in dec["w2"]], f32(dec["b2"]),
                                pack=True))
        views.append(ngl.make_view(it["camera"].eye, cfg.width, cfg.height, it["lod"]))
    setup_s = time.perf_counter() - t0
    cap = 1 << 22
    br = ngl.BatchRenderer(models, views, cap, dev)
    br.render(cfg.max_steps, cfg.delta)
    torch.cuda.synchronize()
    while br.overflowed():
        cap = max(2 * cap, int(br.counts[:, 1].max().item()))
        br = ngl.BatchRenderer(models, views, cap, dev)
        br.render(cfg.max_steps, cfg.delta)
        torch.cuda.synchronize()
    log("batch setup %.1fs, pair capacity %d" % (setup_s, cap))
    untuned = autotune.current()
    tuned = autotune.tune("batch16x512-f16-bf16", lambda: br.render(cfg.max_steps, cfg.delta), fp32_model=False,
                          repeats=3, use_cache=False)
    log("autotuned batch launch: %s (%.3f ms)" % (tuned["config"], tuned["ms"]))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        br.render(cfg.max_steps, cfg.delta)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(max(1, warmup)):
        g.replay()
    torch.cuda.synchronize()
    ev = []
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        ev.append((a, b))
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    assert not br.overflowed(), "pair list overflowed during timing"
    R = sum(cfg.width * cfg.height for _ in views)
    status = br.status.cpu().numpy()
    steps_arr = br.steps.cpu().numpy()
    fm = br.frame_ms()
    out = {"shapes": len(views), "image": [cfg.width, cfg.height], "lods": [it["num_lods"] for it in scene],
           "view_lods": [it["lod"] for it in scene], "ms": ms, "rays": R, "rays_per_s": R / (ms * 1e-3),
           "frame_ms_per_shape": [round(float(x), 4) for x in fm],
           "visible_px": int((status == ngl.HIT).sum()), "sdf_evals": int(steps_arr.sum()),
           "graph": True, "tuned": tuned["config"], "tuned_ms": tuned["ms"],
           "untuned_ms": tuned.get("default_ms"), "setup_s": setup_s}
    autotune.apply(untuned)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(S, budget_s):
    """The FP64 oracle on a bounded sample of the same workload, timed on the
    host cores (median of 3 runs after one warm-up, and once on one thread);
    scaled to the metric's unit."""
    import oracle
    cfg = S["cfg"]
    t0 = time.perf_counter()
    otree = oracle.Octree(S["ijk"], cfg.num_lods)
    feats = S["feats"]
    dec = S["dec"]
    om = oracle.Model([np.asarray(f, np.float32).astype(np.float64) for f in feats],
                      [np.asarray(w, np.float32).astype(np.float64) for w in dec["W1"]],
                      [np.asarray(b, np.float32).astype(np.float64) for b in dec["b1"]],
                      [np.asarray(w, np.float32).astype(np.float64) for w in dec["w2"]],
                      np.asarray(dec["b2"], np.float32).astype(np.float64))
    build_s = time.perf_counter() - t0
    cores = oracle.max_threads()

    def median3(fn):
        fn()
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    def one_thread(fn):
        oracle.set_threads(1)
        try:
            t = time.perf_counter()
            fn()
            return time.perf_counter() - t
        finally:
            oracle.set_threads(cores)

    # queries: grow the sample until one run takes about a twelfth of the budget
    n = 4096
    xq = S["xq_host"]
    while True:
        t0 = time.perf_counter()
        oracle.query(otree, om, np.ascontiguousarray(xq[:, :n]), cfg.num_lods)
        dt = time.perf_counter() - t0
        if dt > budget_s / 12 or n >= xq.shape[1]:
            break
        n = min(xq.shape[1], n * 4)
    xs = np.ascontiguousarray(xq[:, :n])
    qps = n / median3(lambda: oracle.query(otree, om, xs, cfg.num_lods))
    n1 = max(1024, n // max(cores, 1))
    x1 = np.ascontiguousarray(xq[:, :n1])
    qps1 = n1 / one_thread(lambda: oracle.query(otree, om, x1, cfg.num_lods))
    # frame: every k-th ray of the 1024^2 camera, scaled to the full frame
    co, cd = oracle.camera_rays(cfg.eye, (0, 0, 0), (0, 1, 0), 45.0, cfg.width, cfg.height)
    h_fd = 2.0 / (4 << (cfg.num_lods - 1)) / 16.0

    def frame(stride):
        idx = np.arange(0, cfg.width * cfg.height, stride)
        o = np.ascontiguousarray(co[:, idx].astype(np.float32))
        d = np.ascontiguousarray(cd[:, idx].astype(np.float32))

        def run():
            hits = oracle.trace_octree(otree, o, d, cfg.num_lods + 1)
            r = oracle.sphere_trace(otree, om, o, d, cfg.num_lods, 0.0, hits, cfg.max_steps, cfg.delta)
            oracle.normals(otree, om, cfg.num_lods, 0.0, h_fd, rays=(o, d, r["t"].astype(np.float32), r["status"]))
        return run

    stride = 16
    frame_s = median3(frame(stride)) * stride
    stride1 = stride * max(cores, 1)
    frame1_s = one_thread(frame(stride1)) * stride1
    # training step on a sample
    nt = 8192
    xt = np.ascontiguousarray(S["xt_host"][:, :nt])
    tp = nt / median3(lambda: oracle.train_fwd_bwd(otree, om, xt, S["tg_host"][:nt]))
    nt1 = 1024
    xt1 = np.ascontiguousarray(S["xt_host"][:, :nt1])
    tp1 = nt1 / one_thread(lambda: oracle.train_fwd_bwd(otree, om, xt1, S["tg_host"][:nt1]))
    return {"value": qps, "unit": "queries/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d of the 2^20 queries at LOD 5; frame from every %dth ray of the 1024^2 camera "
                      "(traversal + trace + normals), scaled x%d; training on %d points; median of 3 runs "
                      "after a warm-up; one-thread runs on %d queries, every %dth ray, %d training points"
                      % (n, stride, stride, nt, n1, stride1, nt1),
            "fps_1024": 1.0 / frame_s, "train_points_per_s": tp, "octree_build_s": build_s,
            "one_thread": {"queries_per_s": qps1, "fps_1024": 1.0 / frame1_s, "train_points_per_s": tp1}}


if __name__ == "__main__":
    main()
