"""Build the HIP library libswalign.so for gfx950 with hipcc (in-tree)."""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswalign.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["sw_kernels.hip", "sw_tracker.hip", "sw_trace.hip", "sw_filter.hip", "sw_index.hip", "sw_peak.hip", "sw_serve.hip", "sw_api.cpp", "sw_ctx.cpp", "sw_server.cpp", "sw_seed.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# No packed-fp32 instructions anywhere in device code (this code has no float math).
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mcode-object-version=5"]


def _compile(src, obj):
    lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    from concurrent.futures import ThreadPoolExecutor
    jobs = []
    with ThreadPoolExecutor(max_workers=10) as ex:
        for s in SOURCES:
            obj = os.path.join(BUILD, os.path.splitext(s)[0] + ".o")
            objs.append(obj)
            jobs.append((s, ex.submit(_compile, s, obj)))
        for s, j in jobs:
            t0 = time.time()
            err = j.result()
            if verbose:
                print(f"compiled {s}", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t = time.time()
    print(build(verbose=True), f"{time.time() - t:.1f}s")
