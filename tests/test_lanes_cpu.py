"""The 64-bit lane broadcast the one-wavefront-per-task kernel uses for a task's
window start (csrc/sw_lanes.h), compiled for the host with a stand-in 32-bit
shuffle over 64 simulated lanes: every value comes back unchanged, including
reference positions at and past 2^31 and 2^32, where a sign-extended low half
used to turn the window start negative."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r'''
#include <stdio.h>
#include <stdint.h>
#include "sw_lanes.h"
int main() {
  const int64_t vals[] = {0, 1, 15, 2147483647LL, 2147483648LL, 2147483663LL, 3000000000LL, 3199999999LL,
                          4294967295LL, 4294967296LL, 4294967311LL, 5900000000LL, (1LL << 40) + 12345,
                          -1, -2147483648LL, (int64_t)0x7FFFFFFFFFFFFFFFLL};
  int bad = 0;
  for (int64_t v : vals)
    for (int src = 0; src < 64; src += 21) {
      // 64 lanes: lane `src` holds v, the others other values; each lane's 32-bit
      // halves are what a hardware shuffle would read from it
      int lo[64], hi[64];
      for (int l = 0; l < 64; ++l) {
        const int64_t x = l == src ? v : (int64_t)0x5A5A5A5A5A5A5A5ALL ^ l;
        lo[l] = (int)(uint32_t)(uint64_t)x;
        hi[l] = (int)(uint32_t)((uint64_t)x >> 32);
      }
      // lane 5 asks for lane src's value: the first shuffle moves low halves, the second high ones
      int call = 0;
      auto shfl32 = [&](int, int s) { return (call++ == 0 ? lo : hi)[s]; };
      const int64_t mine = (int64_t)0x5A5A5A5A5A5A5A5ALL ^ 5;
      const int64_t got = swk::shfl_i64(shfl32, src == 5 ? v : mine, src);
      if (got != v) {
        printf("lane %d value %lld came back as %lld\n", src, (long long)v, (long long)got);
        ++bad;
      }
    }
  printf("bad %d\n", bad);
  return bad ? 1 : 0;
}
'''


def test_shfl_i64_keeps_positions_past_2_31(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    src = tmp_path / "lanes.cpp"
    src.write_text(PROG)
    exe = tmp_path / "lanes"
    r = subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_1805_00106_amd", "csrc"),
                        "-o", str(exe), str(src)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "bad 0" in r.stdout, r.stdout
