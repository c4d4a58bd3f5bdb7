"""Autotuner for the tracers' launch shape.

Candidates are combinations of the library options that change how the
persistent tracers are launched, never what they compute:
  * NGL_OPT_TRACE_WAVES          wavefronts per block (4, 2, 1);
  * NGL_OPT_TRACE_BLOCKS_PER_CU  resident blocks per compute unit (0 = the
                                 occupancy limit, or a smaller cap);
  * NGL_OPT_TRACE_PAUSE1         evaluation count at which the phased tracer
                                 parks the rays still running and finishes
                                 them with a group of lanes per ray (24, 12,
                                 48; 0 = one phase);
  * NGL_OPT_F32_DECODER          FP32 decoder on the vector ALUs or the matrix
                                 cores (FP32 models only).
Each candidate is timed with HIP events on the current stream (median of a
few runs after one warm-up) and the fastest is kept, per device and workload
signature, in a JSON cache ($NGL_TUNE_CACHE, default ~/.cache/ngl_tune.json).
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Callable, Dict, Iterable, Optional

import torch

from . import ngl

_KEYS = {"waves": ngl.OPT_TRACE_WAVES, "blocks_per_cu": ngl.OPT_TRACE_BLOCKS_PER_CU,
         "pause": ngl.OPT_TRACE_PAUSE1, "f32_decoder": ngl.OPT_F32_DECODER}


def cache_path() -> str:
    return os.environ.get("NGL_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ngl_tune.json"))


def current() -> Dict[str, int]:
    return {k: ngl.get_option(v) for k, v in _KEYS.items()}


def apply(config: Dict[str, int]) -> None:
    for k, v in config.items():
        ngl.set_option(_KEYS[k], int(v))


def candidates(fp32_model: bool) -> Iterable[Dict[str, int]]:
    dec = (1, 0) if fp32_model else (1,)
    for w, b, p, f in itertools.product((0, 2, 1), (0, 4, 2), (24, 12, 48, 0), dec):
        yield {"waves": w, "blocks_per_cu": b, "pause": p, "f32_decoder": f}


def time_ms(fn: Callable[[], None], repeats: int = 3) -> float:
    fn()  # warm-up (also fills the library's per-kernel occupancy caches)
    ts = []
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(signature: str, fn: Callable[[], None], fp32_model: bool, repeats: int = 3,
         path: Optional[str] = None, use_cache: bool = True) -> dict:
    """Return {"config": best options, "ms": its time, "trials": [...]},
    applying the best configuration.  Cached per device and signature."""
    path = path or cache_path()
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    key = "%s|%s" % (dev, signature)
    cache = _load_cache(path) if use_cache else {}
    if key in cache:
        apply(cache[key]["config"])
        return dict(cache[key], cached=True)
    saved = current()
    trials = []
    for cfg in candidates(fp32_model):
        apply(cfg)
        trials.append({"config": cfg, "ms": time_ms(fn, repeats)})
    best = min(trials, key=lambda t: t["ms"])
    apply(best["config"])
    result = {"config": best["config"], "ms": best["ms"], "trials": trials, "default_ms": next(
        (t["ms"] for t in trials if t["config"] == {**saved, "f32_decoder": t["config"]["f32_decoder"]}), None)}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache[key] = {"config": best["config"], "ms": best["ms"]}
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return dict(result, cached=False)
