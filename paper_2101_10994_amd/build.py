"""Build the gfx950 HIP library (libngl.so) in-tree with hipcc.

Every source under csrc/ is compiled for gfx950 only, with packed-FP32
instruction selection disabled, and linked into one shared object whose
exported symbols are the C ABI declared in include/ngl.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libngl.so")
OBJDIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-std=c++17", "-O3", "-fPIC", "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-function"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
          # matrix-core results in ordinary VGPRs (no accumulator-register copies)
          "-mllvm", "-amdgpu-mfma-vgpr-form"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def _includes(path: str, seen: set) -> set:
    """The project headers `path` includes, directly or not."""
    import re
    with open(path) as f:
        for name in re.findall(r'^\s*#\s*include\s+"([^"]+)"', f.read(), flags=re.M):
            for d in (CSRC, INCLUDE):
                h = os.path.join(d, name)
                if os.path.exists(h) and h not in seen:
                    seen.add(h)
                    _includes(h, seen)
                    break
    return seen


def _stale(src: str) -> bool:
    """The object is missing or older than its source or a header it includes."""
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    deps = [src] + sorted(_includes(src, set()))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, changed_only: bool = False) -> str:
    """Compile the sources and link libngl.so.  Rebuilds everything unless
    changed_only, which recompiles only stale objects."""
    srcs = sources()
    todo = [s for s in srcs if _stale(s)] if changed_only else srcs
    if todo:
        with cf.ThreadPoolExecutor(max_workers=min(8, len(todo))) as ex:
            list(ex.map(_compile, todo))
    objs = [os.path.join(OBJDIR, os.path.basename(s) + ".o") for s in srcs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, changed_only="--changed" in sys.argv[1:])
    sys.exit(0)
