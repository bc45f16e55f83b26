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

}  // namespace gemi
