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


def _stale(src, obj):
    """An object older than its source or than any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "sw_align.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, changed_only: bool = False) -> str:
    """Compile every source (changed_only: only objects older than their inputs) and link."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    from concurrent.futures import ThreadPoolExecutor
    jobs = []
    with ThreadPoolExecutor(max_workers=10) as ex:
        for s in SOURCES:
            obj = os.path.join(BUILD, os.path.splitext(s)[0] + ".o")
            objs.append(obj)
            if changed_only and not _stale(s, obj):
                continue
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
    print(build(verbose=True, changed_only="--changed" in sys.argv), f"{time.time() - t:.1f}s")
