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
// sampled sweeps read it instead of walking the volume.  Each workgroup
// writes its range of voxels in ascending order at a place reserved with
// one atomic, so the order of the ranges varies from run to run.  Hard
// histograms built from the list do not (integer counts commute).  Parzen
// tables may, in the last bits: a workgroup's share of the list depends on
// that order, and its exact fixed-point partial sums are rounded to fp64
// and merged with fp64 atomics in scheduling order.
#include "common.h"

namespace gemi {

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int kListThreads = 256;
constexpr int kListWaves = kListThreads / 64;

__device__ __forceinline__ bool kept(uint64_t seed, uint64_t thr, int64_t i, int64_t nvox) {
  return i < nvox && (splitmix64(seed, (uint64_t)i) >> 32) < thr;
}

// Each workgroup takes a contiguous range of fixed voxels: it counts the
// kept ones, reserves their places in the list with one atomic, and writes
// them in ascending order (one atomic per workgroup: a counter shared by
// every wave serialised the whole pass).  `thr` = floor(fraction 2^32), or
// 2^32 to keep every voxel.
__global__ __launch_bounds__(kListThreads) void sample_list_kernel(const uint8_t* __restrict__ fbins,
                                                                   int32_t nx, int32_t ny, int64_t nvox,
                                                                   uint64_t seed, uint64_t thr,
                                                                   uint2* __restrict__ list,
                                                                   unsigned long long* __restrict__ n_list) {
  __shared__ uint32_t wave_count[kListWaves];
  __shared__ unsigned long long block_base;
  const int64_t per = ((nvox + gridDim.x - 1) / gridDim.x + kListThreads - 1) / kListThreads * kListThreads;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < nvox ? b0 + per : nvox;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // pass 1: count
  uint32_t mine = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kListThreads) mine += kept(seed, thr, i, nvox);
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
  if (lane == 0) wave_count[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t total = 0;
    for (int w = 0; w < kListWaves; ++w) total += wave_count[w];
    block_base = total ? atomicAdd(n_list, (unsigned long long)total) : 0ull;
  }
  __syncthreads();
  // pass 2: write, one round of kListThreads voxels at a time
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  unsigned long long run = block_base;
  for (int64_t r0 = b0; r0 < b1; r0 += kListThreads) {
    const int64_t i = r0 + threadIdx.x;
    const bool keep = i < b1 && kept(seed, thr, i, nvox);
    const uint64_t mask = __ballot(keep);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    __syncthreads();  // the previous round's counts have been read
    if (lane == 0) wave_count[wave] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kListWaves; ++w) {
      before += (uint32_t)w < wave ? wave_count[w] : 0u;
      total += wave_count[w];
    }
    if (keep) {
      // fixed voxels < 2^28: 32-bit divisions
      const uint32_t iu = (uint32_t)i;
      const uint32_t z = iu / plane, rem = iu - z * plane;
      const uint32_t y = rem / (uint32_t)nx, x = rem - y * (uint32_t)nx;
      list[run + before + below] = make_uint2(x | (y << 12) | ((uint32_t)fbins[i] << 24), z);
    }
    run += total;
  }
}

hipError_t launch_sample_list(const uint8_t* fbins, int32_t nx, int32_t ny, int32_t nz, double fraction,
                              uint64_t seed, uint2* list, unsigned long long* n_list, hipStream_t s) {
  const int64_t nvox = (int64_t)nx * ny * nz;
  const uint64_t thr = fraction >= 1.0 ? (1ull << 32) : (uint64_t)floor(fraction * 4294967296.0);
  // about 16 rounds of kListThreads voxels per workgroup, at most 4096 workgroups
  int64_t g = (nvox + 16 * kListThreads - 1) / (16 * kListThreads);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(sample_list_kernel, dim3((unsigned)g), dim3(kListThreads), 0, s, fbins, nx, ny, nvox, seed,
                     thr, list, n_list);
  return hipGetLastError();
}

}  // namespace gemi
