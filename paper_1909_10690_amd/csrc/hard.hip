// Hard-binned joint histogram of fixed vs. transformed moving volume
// (Transform + Metric blocks of Fig. 1; "full histogram over all voxels",
// Discussion), for gfx950.
//
// One workgroup = one transform x one slab of fixed rows.  Each wave64
// sweeps a fixed row with its 64 lanes on consecutive x (coalesced fixed
// reads), stepping the exact Q32 moving coordinate by 64 * M[:,0] per
// iteration.  Each lane gathers its 2x2x2 moving neighbourhood, forms the
// exact 16-bit-weight trilinear value in integers, bins it, and adds one
// count to the workgroup's private joint histogram in LDS.  At the end the
// non-zero LDS bins are added once into the transform's HBM histogram.
#include "common.h"

namespace gemi {

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_f64_kernel(double* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

static unsigned fill_grid(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g == 0) g = 1;
  return (unsigned)g;
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t value, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fixed-volume binning, once per call
// ---------------------------------------------------------------------------

template <typename T>
__global__ void prebin_int_kernel(const T* __restrict__ u, size_t nvox, int32_t lo, int32_t hi,
                                  uint32_t bins, Divider div, uint8_t* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
       i += (size_t)gridDim.x * blockDim.x) {
    int32_t v = (int32_t)u[i];
    v = v < lo ? lo : (v > hi ? hi : v);
    out[i] = (uint8_t)div_small((uint32_t)(v - lo) * bins, div);
  }
}

__global__ void prebin_f32_kernel(const float* __restrict__ u, size_t nvox, double lo, double hi,
                                  int32_t bins, uint8_t* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = (double)u[i];
    v = v < lo ? lo : (v > hi ? hi : v);
    // floor(((v - lo) / (hi - lo)) * B), each step one IEEE fp64 operation
    const double r = __ddiv_rn(__dsub_rn(v, lo), __dsub_rn(hi, lo));
    int32_t b = (int32_t)floor(__dmul_rn(r, (double)bins));
    out[i] = (uint8_t)(b > bins - 1 ? bins - 1 : (b < 0 ? 0 : b));
  }
}

hipError_t launch_prebin_fixed(const VolumeDesc& f, int bins, uint8_t* out, hipStream_t s) {
  const size_t nvox = (size_t)f.nx * f.ny * f.nz;
  const unsigned grid = fill_grid(nvox);
  if (f.dtype == 3) {
    hipLaunchKernelGGL(prebin_f32_kernel, dim3(grid), dim3(256), 0, s, (const float*)f.data, nvox,
                       f.lo, f.hi, bins, out);
  } else {
    const int32_t lo = (int32_t)f.lo, hi = (int32_t)f.hi;
    const Divider d = make_divider((uint32_t)(hi - lo + 1));
    if (f.dtype == 0)
      hipLaunchKernelGGL(prebin_int_kernel<uint8_t>, dim3(grid), dim3(256), 0, s,
                         (const uint8_t*)f.data, nvox, lo, hi, (uint32_t)bins, d, out);
    else if (f.dtype == 1)
      hipLaunchKernelGGL(prebin_int_kernel<uint16_t>, dim3(grid), dim3(256), 0, s,
                         (const uint16_t*)f.data, nvox, lo, hi, (uint32_t)bins, d, out);
    else
      hipLaunchKernelGGL(prebin_int_kernel<int16_t>, dim3(grid), dim3(256), 0, s,
                         (const int16_t*)f.data, nvox, lo, hi, (uint32_t)bins, d, out);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the histogram sweep
// ---------------------------------------------------------------------------

struct HardArgs {
  const double* transforms;
  const uint8_t* fbins;
  const void* moving;
  uint32_t* hist;
  int32_t fnx, fny, fnz;
  int32_t mnx, mny, mnz;
  int32_t mlo, mhi;
  int32_t bins, chunks;
  Divider div;  // floor(X / R_moving)
};

// Maps workgroup id -> (transform, slab).  Workgroups are dealt round-robin
// to the 8 XCDs, so XCD x receives ids x, x+8, ...; those all take slabs
// from the x-th eighth of the fixed volume, whose moving footprint then
// stays in that XCD's L2 across transforms.
__device__ __forceinline__ void block_work(int32_t chunks, uint32_t& t, uint32_t& chunk) {
  const uint32_t bid = blockIdx.x;
  const uint32_t xcd = bid & 7u, slot = bid >> 3;
  const uint32_t c8 = (uint32_t)chunks >> 3;
  t = slot / c8;
  chunk = xcd * c8 + (slot - t * c8);
}

template <typename T>
__device__ __forceinline__ uint32_t clamp_offset(T v, int32_t lo, int32_t hi) {
  int32_t x = (int32_t)v;
  x = x < lo ? lo : (x > hi ? hi : x);
  return (uint32_t)(x - lo);
}

template <typename T, bool CLAMP, bool PACKED>
__global__ __launch_bounds__(kBlock) void hist_hard_kernel(HardArgs a) {
  extern __shared__ uint32_t lds_hist[];
  const int B = a.bins;
  const int words = PACKED ? (B * B + 1) / 2 : B * B;
  for (int e = threadIdx.x; e < words; e += kBlock) lds_hist[e] = 0;

  uint32_t t, chunk;
  block_work(a.chunks, t, chunk);
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)t, Mq);
  __syncthreads();
  if (!ok) return;  // unusable transform: histogram stays zero

  const int64_t rows = (int64_t)a.fny * a.fnz;
  const int64_t r0 = rows * chunk / a.chunks, r1 = rows * (chunk + 1) / a.chunks;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t topx = (uint64_t)(a.mnx - 1) << 32;
  const uint64_t topy = (uint64_t)(a.mny - 1) << 32;
  const uint64_t topz = (uint64_t)(a.mnz - 1) << 32;
  const uint32_t sy_full = (uint32_t)a.mnx, sz_full = (uint32_t)a.mnx * (uint32_t)a.mny;
  const T* __restrict__ mv = (const T*)a.moving;
  const int64_t stepx = Mq[0] * 64, stepy = Mq[4] * 64, stepz = Mq[8] * 64;

  for (int64_t r = r0 + wave; r < r1; r += kBlock / 64) {
    const int64_t k = r / a.fny, j = r - k * a.fny;
    int64_t qx = Mq[0] * lane + Mq[1] * j + Mq[2] * k + Mq[3];
    int64_t qy = Mq[4] * lane + Mq[5] * j + Mq[6] * k + Mq[7];
    int64_t qz = Mq[8] * lane + Mq[9] * j + Mq[10] * k + Mq[11];
    const uint8_t* __restrict__ frow = a.fbins + r * a.fnx;
    for (int x = lane; x < a.fnx; x += 64, qx += stepx, qy += stepy, qz += stepz) {
      uint64_t cx = (uint64_t)qx, cy = (uint64_t)qy, cz = (uint64_t)qz;
      if (CLAMP) {
        cx = qx < 0 ? 0 : (cx > topx ? topx : cx);
        cy = qy < 0 ? 0 : (cy > topy ? topy : cy);
        cz = qz < 0 ? 0 : (cz > topz ? topz : cz);
      } else {
        // 0 <= q <= top, with negative q wrapping to huge unsigned values
        if (cx > topx || cy > topy || cz > topz) continue;
      }
      uint32_t ix = (uint32_t)(cx >> 32), iy = (uint32_t)(cy >> 32), iz = (uint32_t)(cz >> 32);
      uint32_t wx = (uint32_t)cx >> 16, wy = (uint32_t)cy >> 16, wz = (uint32_t)cz >> 16;
      // On the last sample of an axis the fraction is 0: take the cell one
      // below with full weight on its upper corner (x), or point the upper
      // corner at the sample itself (y, z); the exact sum is unchanged.
      if (ix == (uint32_t)a.mnx - 1) {
        ix -= 1;
        wx = 65536;
      }
      const uint32_t sy = (iy == (uint32_t)a.mny - 1) ? 0u : sy_full;
      const uint32_t sz = (iz == (uint32_t)a.mnz - 1) ? 0u : sz_full;
      const uint32_t i0 = (iz * (uint32_t)a.mny + iy) * (uint32_t)a.mnx + ix;
      const uint32_t v000 = clamp_offset(mv[i0], a.mlo, a.mhi);
      const uint32_t v100 = clamp_offset(mv[i0 + 1], a.mlo, a.mhi);
      const uint32_t v010 = clamp_offset(mv[i0 + sy], a.mlo, a.mhi);
      const uint32_t v110 = clamp_offset(mv[i0 + sy + 1], a.mlo, a.mhi);
      const uint32_t v001 = clamp_offset(mv[i0 + sz], a.mlo, a.mhi);
      const uint32_t v101 = clamp_offset(mv[i0 + sz + 1], a.mlo, a.mhi);
      const uint32_t v011 = clamp_offset(mv[i0 + sy + sz], a.mlo, a.mhi);
      const uint32_t v111 = clamp_offset(mv[i0 + sy + sz + 1], a.mlo, a.mhi);
      const uint32_t ux = 65536u - wx, uy = 65536u - wy, uz = 65536u - wz;
      // x: < 2^32; y: < 2^48; z: < 2^64 -- all exact
      const uint32_t a00 = v000 * ux + v100 * wx;
      const uint32_t a10 = v010 * ux + v110 * wx;
      const uint32_t a01 = v001 * ux + v101 * wx;
      const uint32_t a11 = v011 * ux + v111 * wx;
      const uint64_t b0 = (uint64_t)a00 * uy + (uint64_t)a10 * wy;
      const uint64_t b1 = (uint64_t)a01 * uy + (uint64_t)a11 * wy;
      const uint64_t V = b0 * uz + b1 * wz;
      // floor(V * B / (R 2^48)) = floor(X / R), X = floor(V * B / 2^48) < 2^24
      const uint32_t X = (uint32_t)(V >> 48) * (uint32_t)B +
                         (uint32_t)(((V & 0xFFFFFFFFFFFFull) * (uint64_t)B) >> 48);
      const uint32_t bm = div_small(X, a.div);
      const uint32_t cell = (uint32_t)frow[x] * (uint32_t)B + bm;
      if (PACKED)
        atomicAdd(&lds_hist[cell >> 1], 1u << ((cell & 1u) * 16u));
      else
        atomicAdd(&lds_hist[cell], 1u);
    }
  }
  __syncthreads();
  uint32_t* __restrict__ out = a.hist + (size_t)t * B * B;
  for (int e = threadIdx.x; e < words; e += kBlock) {
    const uint32_t v = lds_hist[e];
    if (v == 0) continue;
    if (PACKED) {
      if (v & 0xFFFFu) atomicAdd(&out[2 * e], v & 0xFFFFu);
      if (v >> 16) atomicAdd(&out[2 * e + 1], v >> 16);  // never set past the last bin
    } else {
      atomicAdd(&out[e], v);
    }
  }
}

template <typename T, bool CLAMP, bool PACKED>
static hipError_t launch_typed(const HardArgs& a, int n, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((hist_hard_kernel<T, CLAMP, PACKED>), dim3((unsigned)(n * a.chunks)),
                     dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_dtype(const HardArgs& a, int n, bool clamp, bool packed, size_t lds,
                               hipStream_t s) {
  if (clamp)
    return packed ? launch_typed<T, true, true>(a, n, lds, s) : launch_typed<T, true, false>(a, n, lds, s);
  return packed ? launch_typed<T, false, true>(a, n, lds, s) : launch_typed<T, false, false>(a, n, lds, s);
}

hipError_t launch_hist_hard(const HardLaunch& L, hipStream_t s) {
  if (L.n == 0) return hipSuccess;
  HardArgs a;
  a.transforms = L.transforms;
  a.fbins = L.fbins;
  a.moving = L.moving.data;
  a.hist = L.hist;
  a.fnx = L.fixed.nx;
  a.fny = L.fixed.ny;
  a.fnz = L.fixed.nz;
  a.mnx = L.moving.nx;
  a.mny = L.moving.ny;
  a.mnz = L.moving.nz;
  a.mlo = (int32_t)L.moving.lo;
  a.mhi = (int32_t)L.moving.hi;
  a.bins = L.bins;
  a.chunks = L.chunks;
  a.div = make_divider((uint32_t)(a.mhi - a.mlo + 1));
  const size_t lds = L.packed ? (((size_t)L.bins * L.bins + 1) / 2) * 4 : (size_t)L.bins * L.bins * 4;
  switch (L.moving.dtype) {
  case 0: return launch_dtype<uint8_t>(a, L.n, L.clamp, L.packed, lds, s);
  case 1: return launch_dtype<uint16_t>(a, L.n, L.clamp, L.packed, lds, s);
  case 2: return launch_dtype<int16_t>(a, L.n, L.clamp, L.packed, lds, s);
  default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t allow_big_lds() {
  const int bytes = 160 * 1024;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)hist_hard_kernel<T, false, false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)hist_hard_kernel<T, true, false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)hist_hard_kernel<T, false, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)hist_hard_kernel<T, true, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t configure_hard_kernels() {
  hipError_t e;
  if ((e = allow_big_lds<uint8_t>()) != hipSuccess) return e;
  if ((e = allow_big_lds<uint16_t>()) != hipSuccess) return e;
  return allow_big_lds<int16_t>();
}

}  // namespace gemi
