// Launch-planning arithmetic of libgemi.so: pure host functions with no HIP
// dependency, shared by the launchers and compiled on its own by the CPU
// unit test of the planning rules.  Internal; not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace gemi {

// A dispatch counts its work-items in 32 bits: a grid of n x (workgroups
// per transform) x threads beyond that wraps without an error and leaves
// transforms unevaluated.  Every launcher whose grid grows with the number
// of transforms issues launches of whole transforms, each below 2^31
// work-items.
constexpr int64_t kMaxWorkItemsPerLaunch = 0x7FFFFFFF;

// Transforms per launch for a kernel of `workgroups_per_transform`
// workgroups of `threads` threads (at least 1).
inline int32_t transforms_per_launch(int64_t workgroups_per_transform, int32_t threads) {
  const int64_t per = workgroups_per_transform * threads;
  const int64_t m = per > 0 ? kMaxWorkItemsPerLaunch / per : 1;
  return (int32_t)(m < 1 ? 1 : (m > 0x7FFFFFFF ? 0x7FFFFFFF : m));
}

// 32-bit words per fixed-bin row of a hard sweep's LDS histogram: the row's
// counters (u32, or two 16-bit ones per word when packed) and a pad that
// makes the row width odd and not 1 modulo 32.  Unpadded rows of a
// power-of-two width would put every cell of one moving bin in one of the
// 32 LDS banks, and the counts of one wave, whose fixed bins differ by
// noise, would queue on that bank; a skew of 3 banks per row spreads them
// over the banks (a plain +1 skew would line up the anti-diagonals).
constexpr int32_t hist_row_words(int32_t bins, bool packed) {
  const int32_t w = (packed ? (bins + 1) / 2 : bins) + 3;
  return (w & 1) ? w : w + 1;
}
constexpr size_t hist_lds_bytes(int32_t bins, bool packed) {
  return (size_t)bins * (size_t)hist_row_words(bins, packed) * 4;
}

// Whether a launch's LDS fits: its dynamic request within the dynamic
// maximum the kernel was configured for, and dynamic plus the kernel's
// static arrays within what one workgroup of the device may hold.  A launch
// past the second limit fails at dispatch (as an invalid allocation that
// the runtime may report only at a later call), so the launchers test it
// before launching.
inline bool lds_fits(size_t dynamic_bytes, size_t static_bytes, size_t configured_dynamic_max,
                     size_t device_max) {
  return dynamic_bytes <= configured_dynamic_max && static_bytes <= device_max &&
         dynamic_bytes <= device_max - static_bytes;
}

// ---------------------------------------------------------------------------
// the fixed-volume walk shared by the sweep kernels
// ---------------------------------------------------------------------------

constexpr int kTileX = 16, kTileY = 4;  // a wave64 covers 16 x 4 fixed voxels at a time

// One wave's walk over its share of a slab: groups of kTileY consecutive
// rows of one slice with exact Q32 row coordinates.  Either each wave takes
// a contiguous share of the slab's row groups (GroupWalk), or the waves
// take them in turn (wave w: groups w, w + NW, ...; GroupWalkFlex with
// `interleave`, chosen at run time).  Where the
// work per row group is even (a hard sweep; the background band of a Parzen
// sweep) contiguous shares keep each wave on neighbouring rows; where it is
// concentrated in a few rows (a Parzen band of rare slots, the skull of a
// CT), contiguous shares leave most waves idle while the few that hold those
// rows finish, and interleaving spreads them over all waves.
// Lane (dx, dy) of the 16 x 4 tile starts at r + lane_off and steps by
// `step` = 16 M[:,0] along x.
// (Constexpr members, so the same code runs in the kernels and in the CPU
// test of the walk.)
template <bool FLEX>
struct GroupWalkT {
  int64_t g, g1;
  int32_t j0, k, G, stride;
  int64_t r[3], lane_off[3], step[3], adv[3], wrap[3];

  constexpr void init(const int64_t* Mq, int32_t fny, int32_t fnz, int32_t chunks, uint32_t chunk, int wave,
                      int nwaves, int dx, int dy, bool interleave = false) {
    G = (fny + kTileY - 1) / kTileY;
    const int64_t groups = (int64_t)G * fnz;
    const int64_t s0 = groups * chunk / chunks, s1 = groups * (chunk + 1) / chunks;
    if (FLEX && interleave) {
      g = s0 + wave;
      g1 = s1;
      stride = nwaves;
    } else {
      g = s0 + (s1 - s0) * wave / nwaves;
      g1 = s0 + (s1 - s0) * (wave + 1) / nwaves;
      stride = 1;
    }
    k = (int32_t)(g / G);
    j0 = (int32_t)(g - (int64_t)k * G) * kTileY;
    for (int a = 0; a < 3; ++a) {
      const int64_t m0 = Mq[4 * a], m1 = Mq[4 * a + 1], m2 = Mq[4 * a + 2], m3 = Mq[4 * a + 3];
      r[a] = m1 * j0 + m2 * k + m3;
      lane_off[a] = m0 * dx + m1 * dy;
      step[a] = m0 * kTileX;
      adv[a] = m1 * (FLEX ? (int64_t)kTileY * stride : (int64_t)kTileY);
      wrap[a] = m2 - m1 * ((int64_t)G * kTileY);
    }
  }

  constexpr void next() {
    const int32_t st = FLEX ? stride : 1;
    g += st;
    j0 += st * kTileY;
    for (int a = 0; a < 3; ++a) r[a] += adv[a];
    if constexpr (FLEX) {
      while (j0 >= G * kTileY) {  // into the next slice (more than once when a slice has fewer groups than waves)
        j0 -= G * kTileY;
        ++k;
        for (int a = 0; a < 3; ++a) r[a] += wrap[a];
      }
    } else if (j0 >= G * kTileY) {
      j0 = 0;
      ++k;
      for (int a = 0; a < 3; ++a) r[a] += wrap[a];
    }
  }
};
using GroupWalk = GroupWalkT<false>;
using GroupWalkFlex = GroupWalkT<true>;

// ---------------------------------------------------------------------------
// x ranges of a row group: where every lane of the tile lies inside the
// moving volume, and where some lane can
// ---------------------------------------------------------------------------
//
// Along a row group the 64 lanes of the tile step together by
// step_a = 16 m0_a per x iteration, so at iteration `it` the least and the
// greatest coordinate over the tile on axis a are R_a + omin_a + it step_a
// and R_a + omax_a + it step_a, where R_a = m1_a j0 + m2_a k + m3_a is the
// coordinate of the group's first voxel and omin_a, omax_a are the extreme
// lane offsets m0_a dx + m1_a dy.  Every lane lies in [0, top_a] on every
// axis exactly when six inequalities A + it S >= 0 hold: A = R + omin with
// S = step, and A = top - R - omax with S = -step, for each axis.  Some lane
// can lie inside only when the six with omin and omax exchanged hold.  One
// with S > 0 bounds `it` from below (it >= ceil(-A / S)), one with S < 0
// from above (it <= floor(A / -S)), and one with S = 0 holds for every `it`
// or for none.
//
// Sixteen lanes evaluate the twelve bounds of a row group at once.  Lane l
// takes axis l % 4 (none when 3) of group l / 4: lower bounds of the
// every-lane range, its upper bounds, lower bounds of the some-lane range,
// its upper bounds.  It forms v = floor((A + D) / |S|), which is the upper
// bound itself, or minus the lower bound, so that each group's bound is the
// least v of its four lanes.  The margin D = -/+ (ceil(|S| / 64) + 1) (every-
// lane / some-lane range) is an integer of at least |S| / 64, so A + D stays
// an exact integer in double (below 2^53), and the division and the
// rounding to float err by far less than D / |S|: the every-lane range can
// only come out narrower than exact, the some-lane range only wider, by one
// iteration where a bound lies within D / |S| of an integer (a face hit
// exactly is one such case).  When a transform's entries are too large for
// A to be exact the lane says so (`exact` false) and the caller checks
// every voxel.

// range_lane and range_value use math builtins and so cannot be constexpr;
// compiled as HIP they are marked for both sides.
#ifdef __HIP__
#define GEMI_HOST_DEVICE __attribute__((host, device))
#else
#define GEMI_HOST_DEVICE
#endif

struct RangeLane {
  double a1, a2, a0;  // A + D = a1 j0 + a2 k + a0
  double inv;         // v = floor((A + D) inv)
  bool exact;
};

constexpr float kRangeClamp = 1048576.0f;  // |v| <= 2^20, far past any row's iterations

// The constants of lane `lane` (0..63), given the Q32 entries (m0, m1, m2,
// m3) of the matrix row of its axis (lane % 4; any values for the lanes that
// take no bound) and that axis's upper moving coordinate top = (n - 1) 2^32,
// all as doubles (integers; exact below 2^53).  Everything is formed in
// double: while |m0| < 2^47, |m1|, |m2| < 2^38 and |m3| < 2^49 (`exact`)
// every value below is an integer below 2^53 (a half-integer below 2^51
// when S = 0, which makes m0 = 0) and so exact.
GEMI_HOST_DEVICE inline RangeLane range_lane(int lane, double m0, double m1, double m2, double m3, double top) {
  RangeLane c{0.0, 0.0, 1073741824.0, 1.0, true};  // no bound: v clamps to 2^20
  if (lane >= 16 || (lane & 3) == 3) return c;
  const int group = lane >> 2;
  const bool every = group < 2, lower = (group & 1) == 0;
  const double step = m0 * kTileX;
  const double ox = m0 * (kTileX - 1), oy = m1 * (kTileY - 1);
  const double omin = (ox < 0 ? ox : 0.0) + (oy < 0 ? oy : 0.0);
  const double omax = (ox > 0 ? ox : 0.0) + (oy > 0 ? oy : 0.0);
  // "lo": R + o_lo + it step >= 0; "hi": top - R - o_hi - it step >= 0
  const double o_lo = every ? omin : omax, o_hi = every ? omax : omin;
  const bool lo = lower == (step >= 0);
  const double mag = __builtin_fabs(step);
  const double margin = __builtin_floor(mag * (1.0 / 64.0)) + 2.0;  // ceil(|S| / 64) + 1 at least
  const double cst = lo ? m3 + o_lo : top - o_hi - m3;
  c.a1 = lo ? m1 : -m1;
  c.a2 = lo ? m2 : -m2;
  // S = 0: v is +-2^20 by the sign of A + 1/2 (no margin: A is an integer)
  c.a0 = step == 0 ? cst + 0.5 : cst + (every ? -margin : margin);
  c.inv = step == 0 ? 1152921504606846976.0 : 1.0 / mag;  // 2^60 when S = 0
  // j0, k < 2^12: |A + D| < 2^50 + 2^50 + |m3| + 15 |m0| + 3 |m1| + top + margin < 2^53
  c.exact = __builtin_fabs(m0) < 140737488355328.0 && __builtin_fabs(m1) < 274877906944.0 &&
            __builtin_fabs(m2) < 274877906944.0 && __builtin_fabs(m3) < 562949953421312.0;
  return c;
}

// v of one lane for the row group whose first row is j0 in slice k.
GEMI_HOST_DEVICE inline int32_t range_value(const RangeLane& c, int32_t j0, int32_t k) {
  const double A = __builtin_fma((double)j0, c.a1, __builtin_fma((double)k, c.a2, c.a0));
  const float t = __builtin_fminf(__builtin_fmaxf((float)(A * c.inv), -kRangeClamp), kRangeClamp);
  return (int32_t)__builtin_floorf(t);
}

// Iterations of a row group of `full` x steps: checked [u0, c0), every lane
// inside [c0, c1), checked [c1, u1); none left out when `skip` is false
// (CLAMP counts every voxel).  The arguments are the least v of the four
// groups of lanes.
struct RowSpans {
  int32_t u0, c0, c1, u1;
};
constexpr RowSpans row_spans(int32_t v_every_lo, int32_t v_every_hi, int32_t v_some_lo, int32_t v_some_hi,
                             int32_t full, bool skip) {
  RowSpans s{0, 0, 0, full};
  if (skip) {
    s.u0 = -v_some_lo > 0 ? (-v_some_lo < full ? -v_some_lo : full) : 0;
    s.u1 = v_some_hi + 1 < full ? v_some_hi + 1 : full;
    if (s.u1 < s.u0) s.u1 = s.u0;
  }
  s.c0 = -v_every_lo > s.u0 ? -v_every_lo : s.u0;
  s.c1 = v_every_hi + 1 < s.u1 ? v_every_hi + 1 : s.u1;
  if (s.c1 <= s.c0) s.c0 = s.c1 = s.u1;
  return s;
}

}  // namespace gemi
