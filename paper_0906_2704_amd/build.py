"""Build libht.so (the HIP library behind include/ht.h) in-tree for gfx950.

Each HIP source is compiled to its own object in parallel (one hipcc process per file,
objects under _build/), then the objects are linked into paper_0906_2704_amd/libht.so.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["ht_plan.hip", "ht_transform.hip", "ht_spectral.hip", "ht_batch.hip", "ht_batch_k_scan.hip",
           "ht_batch_k_features.hip", "ht_batch_k_learned.hip", "ht_batch_k_fused.hip", "ht_mlp.hip", "ht_gemm.hip",
           "ht_learn.hip"]
LIB = os.path.join(HERE, "libht.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed FP32 instructions in any HIP code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def _stale(src, obj):
    """True if obj is missing or older than its source or any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src, os.path.join(ROOT, "include", "ht.h")]
    deps += [os.path.join(HERE, "csrc", h) for h in os.listdir(os.path.join(HERE, "csrc")) if h.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose=False, jobs=None, incremental=False):
    """Compile every source (incremental=True: only those whose object is out of date)
    and link libht.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs, cmds = [], []
    for s in SOURCES:
        src = os.path.join(HERE, "csrc", s)
        obj = os.path.join(OBJDIR, s.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and not _stale(src, obj):
            continue
        cmds.append([hipcc()] + HIPCC_FLAGS + inc + ["-c", src, "-o", obj])
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        codes = list(ex.map(lambda c: _run(c, verbose), cmds))
    if any(codes):
        raise RuntimeError("hipcc failed compiling libht sources")
    tmp = LIB + ".tmp"
    if _run([hipcc()] + HIPCC_FLAGS + ["-shared"] + objs + ["-o", tmp], verbose):
        raise RuntimeError("hipcc failed linking libht.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="-i" in sys.argv[1:]))
