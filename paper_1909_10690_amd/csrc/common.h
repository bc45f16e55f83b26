// Internal declarations shared by the HIP translation units of libgemi.so.
// Nothing here is part of the public ABI (include/gemi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gemi {

constexpr int kMaxQ = 16;
constexpr int kBlock = 256;  // threads per workgroup of the reduction kernels (4 wave64)

// Entropic indices passed by value to the reduction kernels.
struct QList {
  double q[kMaxQ];
  int32_t n;
  int32_t pseudo;  // 1 = pseudo-additive Tsallis MI
};

// Exact floor(X / R) for 0 <= X < 2^24 as (X * m) >> s (Granlund and
// Montgomery, "Division by invariant integers using multiplication", PLDI
// 1994, Thm 4.2 with N = 24, l = ceil(log2 R), m = ceil(2^(N+l) / R)).
struct Divider {
  uint32_t m;
  uint32_t s;
};

inline Divider make_divider(uint32_t R) {
  uint32_t l = 0;
  while ((1u << l) < R) ++l;
  const uint64_t num = 1ull << (24 + l);
  Divider d;
  d.m = (uint32_t)((num + R - 1) / R);
  d.s = 24 + l;
  return d;
}

__device__ __forceinline__ uint32_t div_small(uint32_t x, Divider d) {
  return (uint32_t)(((uint64_t)x * d.m) >> d.s);
}

// Q32 quantisation of one index-space 3x4 transform: Mq = rne(M * 2^32).
// A transform is usable when every entry is finite, linear entries are
// within +-2^16 and translations within +-2^24 (so that every coordinate of
// a volume of at most 4096 voxels per axis fits in int64).
__device__ __forceinline__ bool quantize_transform(const double* __restrict__ M, int64_t* Mq) {
  bool ok = true;
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    const double m = M[e];
    const double lim = (e % 4 == 3) ? 16777216.0 : 65536.0;
    ok = ok && (fabs(m) <= lim);  // false for NaN and infinities
    Mq[e] = __double2ll_rn(m * 4294967296.0);
  }
  return ok;
}

// Host-side launch descriptions.
struct VolumeDesc {
  const void* data;
  int32_t nx, ny, nz, dtype;
  double lo, hi;
};

struct HardLaunch {
  const double* transforms;  // [n][12]
  const uint8_t* fbins;      // fixed-volume bins, [fnz][fny][fnx]
  const uint2* quads;        // moving quad volume, [mnz+1][mny][mnx]
  VolumeDesc fixed, moving;
  uint32_t* hist;  // [n][B][B]
  int32_t n, bins, clamp;
  int32_t chunks;  // workgroups per transform, multiple of 8
  int32_t packed;  // 1: two 16-bit counters per LDS word (bins > 128)
  int32_t block;   // threads per workgroup: 256, 512 or 1024
  int32_t slab_major;  // workgroup order: 1 slab-major, 0 transform-major
};

// Bytes of the moving quad volume of an nx x ny x nz volume (< 2^32 for
// at most 2^28 voxels).
inline size_t quad_volume_bytes(int32_t nx, int32_t ny, int32_t nz) {
  return (size_t)nx * (size_t)ny * (size_t)(nz + 1) * 8;
}

struct ReduceLaunch {
  const uint32_t* hist;  // [n][B][B] counts, or NULL when `table` is used
  const double* table;   // [n][B][B] Parzen masses, or NULL
  const uint64_t* count; // [n] normaliser for Parzen tables
  const double* transforms;
  int32_t n, bins;
  QList q;
  double* mi_out;        // [n][n_q]
  uint64_t* overlap_out; // [n] or NULL
};

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t value, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, hipStream_t s);
hipError_t launch_prebin_fixed(const VolumeDesc& f, int bins, uint8_t* out, hipStream_t s);
hipError_t launch_pack_quads(const VolumeDesc& m, uint2* out, hipStream_t s);
hipError_t launch_hist_hard(const HardLaunch& L, hipStream_t s);
hipError_t launch_mi_reduce(const ReduceLaunch& L, hipStream_t s);
hipError_t configure_kernels();

}  // namespace gemi
