"""Build libnnm.so (gfx950) in-tree with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled
(``-target-feature -packed-fp32-ops``); objects go to ``_build/`` and the shared
library to ``paper_2201_09147_amd/libnnm.so``.
"""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libnnm.so")

ARCH = os.environ.get("NNM_OFFLOAD_ARCH", "gfx950")
SOURCES = ["nnm_api.cpp", "trace_kernels.hip", "trace_ws.hip", "fit_kernels.hip", "nesting_kernels.hip",
           "mesh_kernels.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def _compile(src: str, verbose: bool, defines=(), build_dir=BUILD_DIR, host_flags=()) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    host = [x for f in host_flags for x in ("-Xarch_host", f)]
    cmd = [_hipcc(), *COMMON, *host, *[f"-D{d}" for d in defines], "-x", "hip", "-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if verbose and err:
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False, defines=(), out=LIB, build_dir=BUILD_DIR, host_flags=(), link_flags=()) -> str:
    """Compile every source and link libnnm.so; returns the library path.

    ``defines`` (e.g. ["NNM_RING_LOWP=6"]) and ``out`` build a variant;
    ``host_flags`` go to the host compilation only (each after -Xarch_host),
    ``link_flags`` to the link."""
    os.makedirs(build_dir, exist_ok=True)
    sources = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(len(sources), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, defines, build_dir, host_flags), sources))
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, *link_flags, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
