"""Host test of the served path on the CPU: the server's scheduler, admission,
staging and finisher threads, with its gather/scatter kernels run by a CPU
stand-in of the HIP runtime (tests/host_serve/fake_hip) and the scoring calls
replaced by a deterministic function of each read and CAL.

The stand-in runtime is asynchronous like the real one: every stream's work
runs later, on a worker thread of its own, with random delays; an event
completes when the worker reaches it; a queued copy aborts if the host changed
its source in the meantime; hipFree does not wait.  Free arena blocks are
poisoned for the address sanitizer.  So a block released or re-staged while a
queued step still reads it, a step header rewritten before its copy ran, or a
buffer freed under queued work, all fail the test.

Several client threads submit requests under a small staging budget (admission
waits, arena blocks reused, requests split over steps, both scoring paths), with
read layouts that are tight, gapped and shuffled, or arbitrary; and the served
benchmark's own configuration is replayed (4 GiB budget, 1024 chunks, 65536
reads and 1 M CALs per step, 3.2 and 2.7 Gbp references, a 300-request pool
submitted twice from four client threads (the benchmark submits it eight
times; the number of rounds changes no code path), then three Poisson load phases
with waits, timestamps and releases).  Every output must belong to its own
request, read, CAL and strand.  Built with the host address and
undefined-behaviour sanitizers (and the thread sanitizer where ROCm's clang
provides it)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "host_serve", f) for f in ("driver.cpp", "stubs.cpp", "serve_kernels.cpp")] + \
      [os.path.join(ROOT, "paper_1805_00106_amd", "csrc", "sw_server.cpp")]
INC = ["-I" + os.path.join(HERE, "host_serve", "fake_hip"),
       "-include", os.path.join(HERE, "host_serve", "mark_block.h")]


def _build(tmp_path, compiler, sanitize):
    exe = str(tmp_path / f"host_serve_{os.path.basename(compiler)}")
    cmd = [compiler, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", *sanitize, *INC,
           "-o", exe, *SRC]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "mismatches 0" in r.stdout, r.stdout
    return r.stdout


@pytest.fixture(scope="module")
def asan_exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    return _build(tmp_path_factory.mktemp("hs"), gxx,
                  ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])


@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("seed", [1, 2])
def test_served_routing_under_asan(asan_exe, seed, layout):
    out = _run(asan_exe, seed, 4, 60, layout)
    assert "submit errors 0, failed 0" in out


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_served_routing_steps_in_flight(asan_exe, depth):
    """Fixed numbers of steps in flight (the default, 0, is the adaptive rule)."""
    out = _run(asan_exe, 3, 4, 60, 2, 0, depth)
    assert "submit errors 0, failed 0" in out


def test_served_routing_at_benchmark_scale(asan_exe):
    """The served benchmark's step sizes (1024 chunks, 65536 reads and 1 M CALs per
    step) and request sizes (1..10000 reads of up to 250 bases, up to 32 CALs)."""
    out = _run(asan_exe, 11, 4, 120, 2, 1)
    assert "submit errors 0, failed 0" in out


def test_served_benchmark_configuration(asan_exe):
    """The served benchmark's configuration end to end (the pool submitted twice,
    load phases shortened to 120 requests each)."""
    out = _run(asan_exe, "bench", 7, 300, 2, 120)
    assert "submit errors 0, failed 0" in out


def test_served_threads_under_tsan(tmp_path):
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ not found")
    exe = _build(tmp_path, clang, ["-fsanitize=thread"])
    _run(exe, 5, 4, 40, 2)
    _run(exe, 12, 4, 60, 0, 1)
