// Measurement probe: the peak rate of LDS atomic adds on this device, the
// ceiling against which the histogram sweeps' LDS-atomic rate is reported.
// Each lane adds into its own 32-bit LDS word (consecutive lanes in
// consecutive banks, so no bank conflicts and no same-address
// serialisation) in an unrolled loop; the result is written out so the
// adds cannot be dropped.
#include "common.h"

namespace gemi {

constexpr int kProbeThreads = 1024;

__global__ __launch_bounds__(kProbeThreads) void lds_atomic_probe_kernel(uint32_t* __restrict__ out,
                                                                          int32_t iters) {
  __shared__ uint32_t words[kProbeThreads];
  words[threadIdx.x] = 0;
  __syncthreads();
  uint32_t* w = &words[threadIdx.x];
  for (int i = 0; i < iters; i += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) atomicAdd(w, 1u + (uint32_t)k);
  }
  __syncthreads();
  out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = words[threadIdx.x];
}

hipError_t launch_lds_atomic_probe(uint32_t* out, int32_t blocks, int32_t iters, hipStream_t s) {
  hipLaunchKernelGGL(lds_atomic_probe_kernel, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s, out, iters);
  return hipGetLastError();
}

}  // namespace gemi
