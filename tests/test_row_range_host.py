"""CPU test of the x ranges of a row group (range_lane, range_value and
row_spans in csrc/plan.h, the same constexpr code the hard sweeps run),
compiled with g++.

For a row group of the 16 x 4 tile, the hard sweeps run the x iterations
where every lane lies inside the moving volume without the per-voxel bounds
test, and leave out (excluding boundary) the iterations where no lane can.
Against brute force over every lane and iteration, on matrices that land
exactly on the volume's faces, have zero and negative x steps, rotate,
scale, and on matrices too large for the exact bound arithmetic:
  * every iteration of the every-lane range has all 64 lanes inside;
  * no iteration left out has any lane inside;
  * the every-lane range misses at most one iteration of the exact range
    at each end (a bound that is an exact integer, a face hit exactly, is
    moved inward by the margin), and the some-lane range adds at most one past the exact
    necessary range at each end.
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_10690_amd", "csrc")

PROGRAM = r"""
#include "plan.h"
#include <math.h>
#include <stdio.h>
#include <random>
using namespace gemi;

static int bad = 0;
static long long groups = 0, core_iters = 0, skipped_iters = 0, fallback = 0;

static bool inside(const int64_t* M, const int64_t* top, int64_t x, int64_t y, int64_t z) {
  for (int a = 0; a < 3; ++a) {
    const int64_t q = M[4 * a] * x + M[4 * a + 1] * y + M[4 * a + 2] * z + M[4 * a + 3];
    if (q < 0 || q > top[a]) return false;
  }
  return true;
}

// The device's sixteen lanes and their group minima, on the host.
static RowSpans spans_of(const int64_t* M, const int64_t* top, int j0, int k, int full, bool skip, bool* exact) {
  int vmin[4] = {1 << 30, 1 << 30, 1 << 30, 1 << 30};
  *exact = true;
  for (int lane = 0; lane < 64; ++lane) {
    const int ax = lane & 3, a = ax < 3 ? ax : 0;
    const RangeLane c = range_lane(lane, (double)M[4 * a], (double)M[4 * a + 1], (double)M[4 * a + 2], (double)M[4 * a + 3],
                                   (double)top[a]);
    if (!c.exact) *exact = false;
    const int v = range_value(c, j0, k);
    if (lane < 16) vmin[lane >> 2] = v < vmin[lane >> 2] ? v : vmin[lane >> 2];
  }
  if (!*exact) return RowSpans{0, full, full, full};
  return row_spans(vmin[0], vmin[1], vmin[2], vmin[3], full, skip);
}

static void check(const char* name, const int64_t* M, const int64_t* top, int fnx, int fny, int fnz) {
  const int full = fnx / kTileX;
  for (int k = 0; k < fnz; k += (fnz > 8 ? 5 : 1))
    for (int j0 = 0; j0 < fny; j0 += kTileY)
      for (int skip = 0; skip < 2; ++skip) {
        bool exact;
        const RowSpans s = spans_of(M, top, j0, k, full, skip, &exact);
        ++groups;
        if (!exact) { ++fallback; }
        if (s.u0 < 0 || s.u0 > s.c0 || s.c0 > s.c1 || s.c1 > s.u1 || s.u1 > full || (!skip && (s.u0 != 0 || s.u1 != full))) {
          printf("%s: bad spans %d %d %d %d (full %d)\n", name, s.u0, s.c0, s.c1, s.u1, full); ++bad; return;
        }
        int ex_lo = full, ex_hi = -1, nec_lo = full, nec_hi = -1;
        for (int it = 0; it < full; ++it) {
          bool all = true, any = false;
          for (int dy = 0; dy < kTileY; ++dy)
            for (int dx = 0; dx < kTileX; ++dx) {
              const bool in = inside(M, top, dx + kTileX * it, j0 + dy, k);
              all = all && in;
              any = any || in;
            }
          // the per-axis necessary condition of the some-lane range
          bool nec = true;
          for (int a = 0; a < 3; ++a) {
            int64_t lo = INT64_MAX, hi = INT64_MIN;
            for (int dy = 0; dy < kTileY; ++dy)
              for (int dx = 0; dx < kTileX; dx += kTileX - 1) {
                const int64_t q = M[4 * a] * (dx + kTileX * it) + M[4 * a + 1] * (j0 + dy) + M[4 * a + 2] * k + M[4 * a + 3];
                lo = q < lo ? q : lo; hi = q > hi ? q : hi;
              }
            nec = nec && hi >= 0 && lo <= top[a];
          }
          if (all) { ex_lo = it < ex_lo ? it : ex_lo; ex_hi = it; }
          if (nec) { nec_lo = it < nec_lo ? it : nec_lo; nec_hi = it; }
          const bool in_core = it >= s.c0 && it < s.c1;
          const bool left_out = it < s.u0 || it >= s.u1;
          core_iters += in_core;
          skipped_iters += left_out;
          if (in_core && !all) { printf("%s j0 %d k %d it %d: unchecked iteration has a lane outside\n", name, j0, k, it); ++bad; return; }
          if (left_out && any) { printf("%s j0 %d k %d it %d: left-out iteration has a lane inside\n", name, j0, k, it); ++bad; return; }
        }
        if (!exact) continue;
        for (int it = ex_lo + 1; it < ex_hi; ++it)
          if (it < s.c0 || it >= s.c1) {
            printf("%s j0 %d k %d: every-lane range [%d, %d) against exact [%d, %d]\n", name, j0, k, s.c0, s.c1, ex_lo, ex_hi); ++bad; return;
          }
        if (skip && nec_hi >= nec_lo && (s.u0 < nec_lo - 1 || s.u1 > nec_hi + 2)) {
          printf("%s j0 %d k %d: some-lane range [%d, %d) against [%d, %d]\n", name, j0, k, s.u0, s.u1, nec_lo, nec_hi); ++bad; return;
        }
        if (skip && nec_hi < nec_lo && s.u1 - s.u0 > 2) {
          printf("%s j0 %d k %d: some-lane range [%d, %d) where no lane can be inside\n", name, j0, k, s.u0, s.u1); ++bad; return;
        }
      }
}

static const double Q = 4294967296.0;
static void q32(const double* A, int64_t* M) { for (int e = 0; e < 12; ++e) M[e] = (int64_t)llrint(A[e] * Q); }

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  const int fnx = 96, fny = 40, fnz = 12;
  // moving volumes of the fixed size, smaller and larger
  const int dims[][3] = {{96, 40, 12}, {64, 32, 9}, {130, 70, 20}};
  for (const auto& d : dims) {
    const int64_t top[3] = {(int64_t)(d[0] - 1) << 32, (int64_t)(d[1] - 1) << 32, (int64_t)(d[2] - 1) << 32};
    // integer translations: coordinates land exactly on the faces
    for (int tx = -20; tx <= 20; tx += 5)
      for (int ty = -6; ty <= 6; ty += 3) {
        const double A[12] = {1, 0, 0, (double)tx, 0, 1, 0, (double)ty, 0, 0, 1, (double)(tx % 3)};
        int64_t M[12]; q32(A, M); check("translation", M, top, fnx, fny, fnz);
      }
    // quarter turns and mirrors about z (zero and negative x steps)
    const double turns[][12] = {
        {0, -1, 0, 39, 1, 0, 0, 0, 0, 0, 1, 0}, {-1, 0, 0, 95, 0, -1, 0, 39, 0, 0, 1, 0},
        {0, 1, 0, 0, -1, 0, 0, 95, 0, 0, 1, 0}, {-1, 0, 0, 63.5, 0, 1, 0, 0.25, 0, 0, -1, 11},
        {0, 0, 1, 0, 0, 1, 0, 0, 1, 0, 0, 0}, {0, 0, 0, 5, 0, 1, 0, 0, 0, 0, 1, 0}};
    for (const auto& A : turns) { int64_t M[12]; q32(A, M); check("quarter turn", M, top, fnx, fny, fnz); }
    // random rotations, scales and shears with sub-voxel translations
    for (int n = 0; n < 60; ++n) {
      double A[12];
      for (int e = 0; e < 12; ++e) A[e] = (e % 4 == 3) ? 12.0 * U(rng) : ((e % 4) == e / 4 ? 1.0 : 0.0) + 0.3 * U(rng);
      int64_t M[12]; q32(A, M); check("random", M, top, fnx, fny, fnz);
    }
    // steps of one Q32 unit: the bounds lie far outside every row
    const int64_t tiny[12] = {1, 0, 0, 7LL << 32, 0, (int64_t)1 << 32, 0, 0, -1, 0, (int64_t)1 << 32, 0};
    check("tiny steps", tiny, top, fnx, fny, fnz);
  }
  // entries beyond the exact bound arithmetic: every voxel checked
  const int64_t top[3] = {(int64_t)95 << 32, (int64_t)39 << 32, (int64_t)11 << 32};
  const double big[12] = {1, 0, 0, 2e6, 0, 1, 0, 0, 0, 0, 1, 0};
  int64_t M[12]; q32(big, M); check("large", M, top, fnx, fny, fnz);
  printf("%lld groups, %lld unchecked and %lld left-out iterations, %lld fallbacks, %d failures\n", groups, core_iters,
         skipped_iters, fallback, bad);
  return bad || fallback == 0 || core_iters == 0 || skipped_iters == 0 ? 1 : 0;
}
"""


def test_row_ranges_against_brute_force(tmp_path):
    src = tmp_path / "ranges.cpp"
    exe = tmp_path / "ranges"
    src.write_text(PROGRAM)
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-Wall", "-I", CSRC, "-o", str(exe), str(src)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert " 0 failures" in out.stdout
