"""CPU test of the fixed-volume walk of the sweep kernels (GroupWalk in
csrc/plan.h, the same constexpr code the kernels run), compiled with g++.

Every 4-row group of the fixed volume must be visited exactly once over the
slabs and the waves that share each slab (contiguous shares per wave, or
the waves taking the groups in turn), and at every visited group the
walk's incrementally stepped row coordinates must equal the matrix applied
to the group's first row exactly (Q32 integers: any drift would move every
count after it).
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_10690_amd", "csrc")

PROGRAM = r"""
#include "plan.h"
#include <algorithm>
#include <stdio.h>
#include <vector>
using namespace gemi;

static int bad = 0;
static long long checked = 0;
// a matrix with entries of Q32 size and all different (no symmetric
// mistake cancels)
static const int64_t M[12] = {4294967296LL + 12345, -987654321, 55555555, 7LL << 32,
                              -123456789, 4294967296LL - 777, 31415926, -(3LL << 32),
                              2718281, -1414213, 4294967296LL + 999, 11LL << 32};

// Walks every slab with every wave and checks each visited group.
template <typename Walk>
static void check(const char* name, int fny, int fnz, int chunks, int nw, bool interleave) {
  const int G = (fny + kTileY - 1) / kTileY;
  std::vector<int> seen((size_t)G * fnz, 0);
  for (int c = 0; c < chunks; ++c)
    for (int w = 0; w < nw; ++w) {
      Walk walk;
      walk.init(M, fny, fnz, chunks, (uint32_t)c, w, nw, 5, 2, interleave);
      for (; walk.g < walk.g1; walk.next()) {
        const int64_t g = walk.g;
        if (g < 0 || g >= (int64_t)seen.size()) { printf("%s: group %lld out of range\n", name, (long long)g); ++bad; return; }
        ++seen[g];
        if (walk.k != g / G || walk.j0 != (int)(g % G) * kTileY) {
          printf("%s fny %d fnz %d: group %lld at k %d j0 %d\n", name, fny, fnz, (long long)g, walk.k, walk.j0); ++bad;
        }
        for (int a = 0; a < 3; ++a) {
          const int64_t want = M[4 * a + 1] * walk.j0 + M[4 * a + 2] * walk.k + M[4 * a + 3];
          if (walk.r[a] != want) { printf("%s: row coordinate drift at group %lld\n", name, (long long)g); ++bad; }
        }
        ++checked;
      }
    }
  for (size_t g = 0; g < seen.size(); ++g)
    if (seen[g] != 1) {
      printf("%s fny %d fnz %d chunks %d waves %d: group %zu visited %d times\n", name, fny, fnz, chunks, nw, g, seen[g]);
      ++bad;
      return;
    }
}

int main() {
  const int fnys[] = {1, 3, 4, 5, 8, 63, 64, 256};
  const int fnzs[] = {1, 2, 7, 180};
  const int chunk_counts[] = {1, 8, 120};
  const int wave_counts[] = {1, 4, 16};
  for (int fny : fnys)
    for (int fnz : fnzs)
      for (int chunks : chunk_counts)
        for (int nw : wave_counts) {
          check<GroupWalk>("contiguous", fny, fnz, chunks, nw, false);
          check<GroupWalkFlex>("flex contiguous", fny, fnz, chunks, nw, false);
          check<GroupWalkFlex>("flex interleaved", fny, fnz, chunks, nw, true);
        }
  printf("checked %lld groups, %d failures\n", checked, bad);
  return bad ? 1 : 0;
}
"""


def test_walk_visits_every_group_once_with_exact_rows(tmp_path):
    src = tmp_path / "walk.cpp"
    exe = tmp_path / "walk"
    src.write_text(PROGRAM)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, "-o", str(exe), str(src)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
