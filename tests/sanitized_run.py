"""Run the CPU test suite against AddressSanitizer + UndefinedBehaviorSanitizer
builds of the host code: the C oracle (oracle/*.c, built with clang) and
libnnm's host side (validation, Lipschitz bounds, weight packing, network
files, nesting thresholds, argument checks; the device code is built as
usual).  Both builds go to _build/asan/; pytest then runs in a child process
with clang's ASan runtime preloaded, so the first invalid access or undefined
operation in either library aborts the run with a report.

    python tests/sanitized_run.py [extra pytest arguments]

Exit status: pytest's.  CPU only; nothing here touches a GPU.
"""

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

OUT = os.path.join(ROOT, "_build", "asan")
CLANG = "/opt/rocm/llvm/bin/clang"
# each -fsanitize= is its own flag so the HIP build can put -Xarch_host before it
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    res = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                         check=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not found:
            raise FileNotFoundError("clang's ASan runtime (libclang_rt.asan-x86_64.so) not found")
        path = found[0]
    return path


def build_oracle_sanitized() -> str:
    from oracle.build import SOURCES
    lib = os.path.join(OUT, "libnnm_oracle_asan.so")
    cmd = [CLANG, "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared", *SAN,
           "-shared-libsan", "-o", lib, *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    return lib


def build_nnm_sanitized() -> str:
    from paper_2201_09147_amd import build as nnm_build
    return nnm_build.build(out=os.path.join(OUT, "libnnm_asan.so"), build_dir=OUT,
                           host_flags=["-g", *SAN], link_flags=["-shared-libsan", "-fsanitize=address",
                                                                 "-fsanitize=undefined"])


def main(argv) -> int:
    os.makedirs(OUT, exist_ok=True)
    oracle_lib = build_oracle_sanitized()
    nnm_lib = build_nnm_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan_runtime()
    # Python's own allocations are never freed at exit: leak reports would be noise
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:allocator_may_return_null=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu",
           f"--oracle-lib={oracle_lib}", f"--nnm-lib={nnm_lib}", *argv]
    print("sanitized run:", " ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
