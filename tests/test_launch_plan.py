"""CPU tests of the launch-planning rules (csrc/plan.h), compiled with g++.

A dispatch counts its work-items in 32 bits, so every launcher whose grid
grows with the batch splits it into launches of whole transforms below 2^31
work-items; and a launch's dynamic plus static LDS must fit one workgroup
(a 160 KiB dynamic request beside 16 bytes of static LDS faulted once);
and the hard sweeps' LDS histogram rows are padded to a skewed odd pitch
that still fits two 128-bin tables per CU.
These are host rules; the GPU tests cover the launchers that apply them.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_10690_amd", "csrc")

PROGRAM = r"""
#include "plan.h"
#include <stdio.h>
using namespace gemi;
int main() {
  int bad = 0;
  // grids of every launcher at the largest batch the entry points accept
  // (2^24 transforms): hard sweeps (256/512/1024 threads, up to a few
  // thousand workgroups per transform), Parzen sweeps (chunks x bands, 512),
  // MI reduction and dMI/dp (up to 32 slices of 256 threads), the final
  // merge (1 x 64)
  const long long wgs[] = {1, 8, 32, 2048, 2736, 5464, 32768, 1 << 20, 1 << 21};
  const int threads[] = {64, 256, 512, 1024};
  const long long ns[] = {1, 1000, 1 << 23, 1 << 24};
  for (long long wg : wgs)
    for (int th : threads)
      for (long long n : ns) {
        const int step = transforms_per_launch(wg, th);
        if (step < 1) { printf("step < 1 for wg=%lld th=%d\n", wg, th); ++bad; }
        if (wg * th <= kMaxWorkItemsPerLaunch && (long long)step * wg * th > kMaxWorkItemsPerLaunch) {
          printf("launch of %d transforms x %lld x %d passes 2^31\n", step, wg, th); ++bad;
        }
        long long covered = 0, launches = 0;
        for (long long t0 = 0; t0 < n; t0 += step) {
          const long long part = n - t0 < step ? n - t0 : step;
          if (part * wg * th > kMaxWorkItemsPerLaunch && part > 1) { ++bad; break; }
          covered += part;
          ++launches;
        }
        if (covered != n) { printf("batch of %lld covered %lld\n", n, covered); ++bad; }
      }
  // the worst reduction grid at 2^24 transforms needs several launches
  if ((1LL << 24) / transforms_per_launch(32, 256) < 2) { printf("reduction not split\n"); ++bad; }
  // LDS: the case that faulted, limits exactly met, and overflow-safe sums
  const size_t K = 1024;
  if (lds_fits(160 * K, 16, 160 * K, 160 * K)) { printf("160K + 16 accepted\n"); ++bad; }
  if (!lds_fits(64 * K, 1536, 64 * K, 160 * K)) { printf("64K + 1536 refused\n"); ++bad; }
  if (!lds_fits(160 * K, 0, 160 * K, 160 * K)) { printf("160K + 0 refused\n"); ++bad; }
  if (lds_fits(64 * K + 1, 0, 64 * K, 160 * K)) { printf("above the configured maximum accepted\n"); ++bad; }
  if (lds_fits(0, 200 * K, 160 * K, 160 * K)) { printf("static above the device maximum accepted\n"); ++bad; }
  if (lds_fits((size_t)-1, 16, (size_t)-1, 160 * K)) { printf("wrapped sum accepted\n"); ++bad; }
  // hard-sweep LDS histograms: rows padded to an odd pitch with a skew of 3
  // banks or more for widths that are multiples of 32, at least the row's
  // counters; two u32 128-bin tables per CU, and a 256-bin packed one with
  // the pairs kernel's 8-byte slot within that kernel's 150 KiB
  for (int B = 2; B <= 256; ++B)
    for (int pk = 0; pk < 2; ++pk) {
      const int w = hist_row_words(B, pk), used = pk ? (B + 1) / 2 : B;
      if (w % 2 != 1 || w < used + 3 || w > used + 4) { printf("pitch %d for B=%d pk=%d\n", w, B, pk); ++bad; }
      if (used % 32 == 0 && (w % 32 == 1 || w % 32 == 31)) { printf("unit skew B=%d pk=%d\n", B, pk); ++bad; }
      if (hist_lds_bytes(B, pk) != (size_t)B * w * 4) { printf("bytes B=%d\n", B); ++bad; }
    }
  if (2 * hist_lds_bytes(128, false) > 160 * K) { printf("two 128-bin u32 tables do not fit a CU\n"); ++bad; }
  if (hist_lds_bytes(256, true) + 16 > 150 * K) { printf("256-bin packed table too large\n"); ++bad; }
  printf(bad ? "FAIL %d\n" : "OK\n", bad);
  return bad ? 1 : 0;
}
"""


def test_launch_plan_rules(tmp_path):
    src = tmp_path / "plan_test.cpp"
    exe = tmp_path / "plan_test"
    src.write_text(PROGRAM)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, "-o", str(exe), str(src)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK")


def test_launchers_use_the_guard():
    """Every launch with dynamic LDS goes through lds_guard, and every batch
    launcher through transforms_per_launch (source check of the launchers)."""
    for name, guards in (("hard.hip", 2), ("parzen.hip", 3), ("pairs.hip", 1)):
        text = open(os.path.join(CSRC, name)).read()
        assert text.count("lds_guard(") >= guards, name
    for name in ("hard.hip", "parzen.hip", "reduce.hip"):
        assert "transforms_per_launch(" in open(os.path.join(CSRC, name)).read(), name


if __name__ == "__main__":
    pytest.main([__file__, "-q"])
