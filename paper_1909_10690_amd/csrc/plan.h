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

}  // namespace gemi
