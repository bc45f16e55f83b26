// Random subsampling of the fixed volume (Discussion: Mattes' MI draws its
// voxels at random where MI over all voxels does not, and the paper leaves
// the effect of that sampling open).
//
// Fixed voxel i (linear index z ny nx + y nx + x) takes part when the top 32
// bits of the SplitMix64 output for counter i are below the threshold
// floor(fraction 2^32) (every voxel for a fraction of 1 or more).  SplitMix64
// (Steele, Lea and Flood, OOPSLA 2014) is written here from its published
// definition: output i of the stream seeded with s mixes s + (i + 1) gamma,
// gamma = 0x9E3779B97F4A7C15, through two xor-shift-multiply rounds and a
// final xor-shift.  The decision depends only on (seed, i), so any thread
// order gives the same sample.
//
// The kept voxels are compacted into a list of 8-byte entries
// {x | y << 12 | fixed bin << 24, z} (edges <= 4096, bins <= 256); the
// sampled sweeps read it instead of walking the volume.  Entries are placed
// with one atomic per wave, so their order varies from run to run; the
// histograms built from them do not (integer counts and the Parzen path's
// fixed-point sums commute).
#include "common.h"

namespace gemi {

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int kListThreads = 256;

// `thr` = floor(fraction 2^32), or 2^32 to keep every voxel.
__global__ __launch_bounds__(kListThreads) void sample_list_kernel(const uint8_t* __restrict__ fbins,
                                                                   int32_t nx, int32_t ny, int64_t nvox,
                                                                   uint64_t seed, uint64_t thr,
                                                                   uint2* __restrict__ list,
                                                                   unsigned long long* __restrict__ n_list) {
  const int64_t stride = (int64_t)gridDim.x * kListThreads;
  // every lane runs the same number of rounds (the ballot needs the whole wave)
  const int64_t rounds = (nvox + stride - 1) / stride;
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t i = r * stride + blockIdx.x * (int64_t)kListThreads + threadIdx.x;
    const bool keep = i < nvox && (splitmix64(seed, (uint64_t)i) >> 32) < thr;
    const uint64_t mask = __ballot(keep);
    if (mask == 0) continue;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(n_list, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0, 64);
    if (keep) {
      // fixed voxels < 2^28: 32-bit divisions
      const uint32_t iu = (uint32_t)i;
      const uint32_t z = iu / plane, rem = iu - z * plane;
      const uint32_t y = rem / (uint32_t)nx, x = rem - y * (uint32_t)nx;
      list[base + below] = make_uint2(x | (y << 12) | ((uint32_t)fbins[i] << 24), z);
    }
  }
}

hipError_t launch_sample_list(const uint8_t* fbins, int32_t nx, int32_t ny, int32_t nz, double fraction,
                              uint64_t seed, uint2* list, unsigned long long* n_list, hipStream_t s) {
  const int64_t nvox = (int64_t)nx * ny * nz;
  const uint64_t thr = fraction >= 1.0 ? (1ull << 32) : (uint64_t)floor(fraction * 4294967296.0);
  int64_t g = (nvox + kListThreads - 1) / kListThreads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(sample_list_kernel, dim3((unsigned)g), dim3(kListThreads), 0, s, fbins, nx, ny, nvox, seed,
                     thr, list, n_list);
  return hipGetLastError();
}

}  // namespace gemi
