// Hard-binned joint histogram of fixed vs. transformed moving volume
// (Transform + Metric blocks of Fig. 1; "full histogram over all voxels",
// Discussion), for gfx950.
//
// Per call, the fixed volume is reduced to one bin byte per voxel and the
// moving volume to an "oct volume": each 16-byte element holds the clamped,
// offset intensities of a voxel's whole 2x2x2 trilinear neighbourhood as
// 16-bit values, so a lane gathers its neighbourhood with one aligned
// 128-bit load.  The sweep is limited by gather instruction issue about as
// much as by arithmetic, so one 16-byte gather beats two 8-byte gathers of
// the same bytes.
//
// One workgroup = one transform x one slab of fixed rows.  Each wave64
// walks its own run of 4-row groups with scalar coordinates; its 64 lanes
// cover a 16 x 4 tile of fixed voxels (a compact footprint in the moving
// volume even under rotation, so few cache lines per load) and step the
// exact Q32 moving coordinate by 16 * M[:,0] per iteration.  Each lane forms the exact
// 16-bit-weight trilinear value: x-lerps with v_dot2_u32_u16 in integers
// (< 2^32), y-lerps in fp64 (exact: integers < 2^48), the z-lerp as one
// fp64 fma (the exact value rounded once).  The bin floor(V B / (R 2^48))
// is read off the rounded value unless it lies within 2^-29 of a bin edge;
// those lanes redo the sum in 64-bit integers, so every bin is exact.  One
// count goes to the workgroup's private joint histogram in LDS; at the end
// the non-zero LDS bins are added once into the transform's HBM histogram.
#include "common.h"
#include "sweep.h"

#include <mutex>
#include <utility>
#include <vector>

#pragma clang fp contract(off)

namespace gemi {

// ---------------------------------------------------------------------------
// LDS guard
// ---------------------------------------------------------------------------

namespace {
std::mutex g_lds_mu;
std::vector<std::pair<const void*, size_t>> g_lds_static;  // kernel -> static LDS bytes
size_t g_lds_device_max = 0;                               // LDS one workgroup may hold
}  // namespace

hipError_t lds_register(const void* kernel) {
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, kernel);
  if (e != hipSuccess) return e;
  int dev = 0, max_block = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&max_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
    return e;
  std::lock_guard<std::mutex> g(g_lds_mu);
  g_lds_device_max = (size_t)max_block;
  for (auto& k : g_lds_static)
    if (k.first == kernel) {
      k.second = attr.sharedSizeBytes;
      return hipSuccess;
    }
  g_lds_static.emplace_back(kernel, attr.sharedSizeBytes);
  return hipSuccess;
}

hipError_t lds_guard(const void* kernel, size_t dynamic, size_t configured_max, bool at_zero) {
  for (int pass = 0; pass < 2; ++pass) {
    {
      std::lock_guard<std::mutex> g(g_lds_mu);
      for (const auto& k : g_lds_static)
        if (k.first == kernel)
          return lds_fits(dynamic, k.second, configured_max, g_lds_device_max) && (!at_zero || k.second == 0)
                     ? hipSuccess
                     : hipErrorInvalidValue;
    }
    if (pass == 0) {
      const hipError_t e = lds_register(kernel);
      if (e != hipSuccess) return e;
    }
  }
  return hipErrorInvalidValue;
}

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
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (uint8_t)fixed_bin_int((int32_t)u[i], lo, hi, bins, div);
}

__global__ void prebin_f32_kernel(const float* __restrict__ u, size_t nvox, double lo, double hi,
                                  int32_t bins, uint8_t* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (uint8_t)fixed_bin_real((double)u[i], lo, hi, bins);
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
// moving oct volume, once per call
// ---------------------------------------------------------------------------

// out[z][y][x] holds the eight 16-bit clamped, offset intensities
// v' = clamp(v, lo, hi) - lo of the voxel's 2x2x2 neighbourhood, so one
// 16-byte load fetches all trilinear corners: word 2 dz + dy packs
// (x, y+dy, z+dz) in its low half and (x1, y+dy, z+dz) in its high half,
// with x1 = min(x+1, nx-1) and y+1, z+1 likewise clamped.  A neighbour
// index is thus clamped to the volume, as in the trilinear rule; on those
// corners the hard path's weight is 0, and the Parzen path's derivative
// along that axis vanishes.
template <typename T>
__global__ void pack_octs_kernel(const T* __restrict__ v, int32_t nx, int32_t ny, int32_t nz,
                                 int32_t lo, int32_t hi, uint4* __restrict__ out) {
  const int32_t y = blockIdx.y, z = blockIdx.z;
  uint4* __restrict__ orow = out + ((size_t)z * ny + y) * nx;
  const T* __restrict__ r00 = v + ((size_t)z * ny + y) * nx;
  const T* __restrict__ r10 = r00 + (y + 1 < ny ? nx : 0);
  const size_t dz = z + 1 < nz ? (size_t)nx * ny : 0;
  const T* __restrict__ r01 = r00 + dz;
  const T* __restrict__ r11 = r10 + dz;
  auto c = [&](T raw) -> uint32_t { return clamp_offset((int32_t)raw, lo, hi); };
  for (int32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nx; x += gridDim.x * blockDim.x) {
    const int32_t x1 = x + 1 < nx ? x + 1 : nx - 1;
    orow[x] = make_uint4(c(r00[x]) | (c(r00[x1]) << 16), c(r10[x]) | (c(r10[x1]) << 16),
                         c(r01[x]) | (c(r01[x1]) << 16), c(r11[x]) | (c(r11[x1]) << 16));
  }
}

// The same neighbourhood with 8-bit corners (moving range R <= 256): byte
// 4 dz + 2 dy + dx' of the element holds (x + dx', y + dy, z + dz), dx' = 0
// for x and 1 for x1.
template <typename T>
__global__ void pack_oct8_kernel(const T* __restrict__ v, int32_t nx, int32_t ny, int32_t nz,
                                 int32_t lo, int32_t hi, uint2* __restrict__ out) {
  const int32_t y = blockIdx.y, z = blockIdx.z;
  uint2* __restrict__ orow = out + ((size_t)z * ny + y) * nx;
  const T* __restrict__ r00 = v + ((size_t)z * ny + y) * nx;
  const T* __restrict__ r10 = r00 + (y + 1 < ny ? nx : 0);
  const size_t dz = z + 1 < nz ? (size_t)nx * ny : 0;
  const T* __restrict__ r01 = r00 + dz;
  const T* __restrict__ r11 = r10 + dz;
  auto c = [&](T raw) -> uint32_t { return clamp_offset((int32_t)raw, lo, hi); };
  for (int32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nx; x += gridDim.x * blockDim.x) {
    const int32_t x1 = x + 1 < nx ? x + 1 : nx - 1;
    orow[x] = make_uint2(c(r00[x]) | (c(r00[x1]) << 8) | (c(r10[x]) << 16) | (c(r10[x1]) << 24),
                         c(r01[x]) | (c(r01[x1]) << 8) | (c(r11[x]) << 16) | (c(r11[x1]) << 24));
  }
}

hipError_t launch_pack_oct8(const VolumeDesc& m, uint2* out, hipStream_t s) {
  const dim3 grid((unsigned)((m.nx + 255) / 256), (unsigned)m.ny, (unsigned)m.nz);
  const int32_t lo = (int32_t)m.lo, hi = (int32_t)m.hi;
  if (m.dtype == 0)
    hipLaunchKernelGGL(pack_oct8_kernel<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 1)
    hipLaunchKernelGGL(pack_oct8_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 2)
    hipLaunchKernelGGL(pack_oct8_kernel<int16_t>, grid, dim3(256), 0, s, (const int16_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_pack_octs(const VolumeDesc& m, uint4* out, hipStream_t s) {
  const dim3 grid((unsigned)((m.nx + 255) / 256), (unsigned)m.ny, (unsigned)m.nz);
  const int32_t lo = (int32_t)m.lo, hi = (int32_t)m.hi;
  if (m.dtype == 0)
    hipLaunchKernelGGL(pack_octs_kernel<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 1)
    hipLaunchKernelGGL(pack_octs_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 2)
    hipLaunchKernelGGL(pack_octs_kernel<int16_t>, grid, dim3(256), 0, s, (const int16_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the histogram sweep
// ---------------------------------------------------------------------------

// Dynamic LDS limit of the hard sweeps (a u32 table up to 128 bins, 16-bit
// pairs above: at most 128 KiB), within the 160 KiB of a workgroup.
constexpr size_t kHardLdsMax = 160 * 1024;

struct HardArgs {
  const double* transforms;
  uint32_t* hist;
  HardGeom geom;
  int32_t n, chunks;
  int32_t slab_major;     // 1: consecutive workgroups of an XCD share a slab
  const uint32_t* order;  // processing order (absolute indices) or NULL
  uint32_t order_base;    // absolute index of this launch's first transform
};

// 1024-thread workgroups are held to 64 VGPRs (a few row-loop values spill to
// scratch) so that two of them, 8 waves per SIMD, share a CU next to two
// 64 KiB LDS histograms; the sweep waits on its gathers and gains from the
// extra waves.  Smaller workgroups keep their registers.
// BRICK: slabs as bricks (GroupWalkBrick) rather than thin slabs.
template <bool CLAMP, bool PACKED, bool OCT8, int NT, bool BRICK = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 1024 ? 8 : 1)))
void hist_hard_kernel(HardArgs a) {
  extern __shared__ uint32_t lds_hist[];
  const int B = a.geom.bins;
  clear_hist<PACKED, NT>(lds_hist, B);
  uint32_t t, chunk, band;
  block_work(a.chunks, a.n, 1, a.slab_major, t, chunk, band);
  if (a.order) t = a.order[t] - a.order_base;
  const double* Md = a.transforms + 12 * (size_t)t;
  int64_t Mq[12];
  const bool ok = quantize_transform_wave(Md, Mq);
  __syncthreads();
  if (ok) {
    if (BRICK)  // bricks keep the per-voxel test (row ranges measured 0.7% slower on rotation maps)
      sweep_hard<CLAMP, PACKED, OCT8, NT / 64, GroupWalkBrick, false>(a.geom, Md, Mq, a.chunks, chunk, lds_hist);
    else
      sweep_hard<CLAMP, PACKED, OCT8, NT / 64>(a.geom, Md, Mq, a.chunks, chunk, lds_hist);
  }
  __syncthreads();
  if (ok) flush_hist<PACKED, NT>(lds_hist, B, a.hist + (size_t)t * B * B, false);
}

// Sampled sweep: the workgroup's share of the sample list (entries
// {x | y << 12 | fixed bin << 24, z}) for one transform, each sample's Q32
// coordinates formed straight from the matrix.  With 16-bit counters the
// share is counted in spans of at most 65535 samples, each flushed before
// the next, so no counter can overflow whatever the sample count.
template <bool CLAMP, bool PACKED, bool OCT8, int NT>
__global__ __launch_bounds__(NT) void hist_sampled_kernel(HardArgs a, const uint2* __restrict__ list,
                                                          const unsigned long long* __restrict__ n_list) {
  extern __shared__ uint32_t lds_hist[];
  const int B = a.geom.bins;
  clear_hist<PACKED, NT>(lds_hist, B);
  uint32_t t, chunk, band;
  block_work(a.chunks, a.n, 1, a.slab_major, t, chunk, band);
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)t, Mq);
  const int64_t ns = (int64_t)*n_list;
  const int64_t s0 = ns * chunk / a.chunks, s1 = ns * (chunk + 1) / a.chunks;
  const int64_t span = PACKED ? 65535 : s1 - s0;
  const HardStep hs(a.geom, lds_hist, OCT8);
  uint32_t* out = a.hist + (size_t)t * B * B;
  for (int64_t p0 = s0; p0 < s1; p0 += span) {
    const int64_t p1 = p0 + span < s1 ? p0 + span : s1;
    __syncthreads();
    if (ok) {
      for (int64_t e = p0 + threadIdx.x; e < p1; e += NT) {
        const uint2 en = list[e];
        const int64_t x = en.x & 0xFFFu, y = (en.x >> 12) & 0xFFFu, z = en.y;
        const uint32_t fb = en.x >> 24;
        const int64_t qx = Mq[0] * x + Mq[1] * y + Mq[2] * z + Mq[3];
        const int64_t qy = Mq[4] * x + Mq[5] * y + Mq[6] * z + Mq[7];
        const int64_t qz = Mq[8] * x + Mq[9] * y + Mq[10] * z + Mq[11];
        hs.count<CLAMP, PACKED, OCT8>(qx, qy, qz, [&] { return fb; }, lds_hist);
      }
    }
    __syncthreads();
    if (ok) flush_hist<PACKED, NT>(lds_hist, B, out, true);
  }
}

constexpr int kSampledBlock = 512;

template <bool CLAMP, bool PACKED, bool OCT8>
static hipError_t launch_sampled_variant(const HardArgs& a, const uint2* list, const unsigned long long* n_list,
                                         size_t lds, hipStream_t s) {
  const hipError_t e =
      lds_guard((const void*)hist_sampled_kernel<CLAMP, PACKED, OCT8, kSampledBlock>, lds, kHardLdsMax, true);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((hist_sampled_kernel<CLAMP, PACKED, OCT8, kSampledBlock>), dim3((unsigned)(a.n * a.chunks)),
                     dim3(kSampledBlock), lds, s, a, list, n_list);
  return hipGetLastError();
}

template <bool CLAMP, bool PACKED, bool OCT8, int NT, bool BRICK>
static hipError_t launch_variant(const HardArgs& a, int n, size_t lds, hipStream_t s) {
  const hipError_t e =
      lds_guard((const void*)hist_hard_kernel<CLAMP, PACKED, OCT8, NT, BRICK>, lds, kHardLdsMax, true);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((hist_hard_kernel<CLAMP, PACKED, OCT8, NT, BRICK>), dim3((unsigned)(n * a.chunks)),
                     dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <bool OCT8, int NT, bool BRICK>
static hipError_t launch_layout(const HardArgs& a, int n, bool clamp, bool packed, size_t lds,
                                hipStream_t s) {
  if (clamp)
    return packed ? launch_variant<true, true, OCT8, NT, BRICK>(a, n, lds, s)
                  : launch_variant<true, false, OCT8, NT, BRICK>(a, n, lds, s);
  return packed ? launch_variant<false, true, OCT8, NT, BRICK>(a, n, lds, s)
                : launch_variant<false, false, OCT8, NT, BRICK>(a, n, lds, s);
}

template <int NT, bool BRICK = false>
static hipError_t launch_nt(const HardArgs& a, int n, bool clamp, bool packed, size_t lds,
                            hipStream_t s) {
  return a.geom.oct8 ? launch_layout<true, NT, BRICK>(a, n, clamp, packed, lds, s)
                     : launch_layout<false, NT, BRICK>(a, n, clamp, packed, lds, s);
}

HardGeom make_hard_geom(const VolumeDesc& fixed, const VolumeDesc& moving, const uint8_t* fbins,
                        const void* octs, int32_t bins) {
  HardGeom g;
  g.fbins = fbins;
  g.octs = octs;
  g.fnx = fixed.nx;
  g.fny = fixed.ny;
  g.fnz = fixed.nz;
  g.mnx = moving.nx;
  g.mny = moving.ny;
  g.mnz = moving.nz;
  g.oct8 = oct8_range(moving.lo, moving.hi) ? 1 : 0;
  g.oct_bytes = (uint32_t)(g.oct8 ? oct8_volume_bytes(moving.nx, moving.ny, moving.nz)
                                  : oct_volume_bytes(moving.nx, moving.ny, moving.nz));
  g.bins = bins;
  const uint32_t R = (uint32_t)((int32_t)moving.hi - (int32_t)moving.lo + 1);
  g.scale = ldexp((double)bins / (double)R, -48);
  g.div = make_divider(R);
  return g;
}

hipError_t launch_hist_hard(const HardLaunch& L, hipStream_t s) {
  if (L.n == 0) return hipSuccess;
  HardArgs a;
  a.transforms = L.transforms;
  a.hist = L.hist;
  a.geom = make_hard_geom(L.fixed, L.moving, L.fbins, L.octs, L.bins);
  a.n = L.n;
  a.chunks = L.chunks;
  a.slab_major = L.slab_major;
  a.order = nullptr;
  a.order_base = 0;
  const size_t lds = hist_lds_bytes(L.bins, L.packed);
  if (L.block != 256 && L.block != 512 && L.block != 1024) return hipErrorInvalidValue;
  int32_t step = transforms_per_launch(L.chunks, L.block);
  // with an order, launches start at multiples of its sorted blocks
  const bool ordered = L.order && step >= kOrderBlock;
  if (ordered) step -= step % kOrderBlock;
  for (int32_t t0 = 0; t0 < L.n; t0 += step) {
    HardArgs b = a;
    b.n = L.n - t0 < step ? L.n - t0 : step;
    b.transforms = a.transforms + 12 * (size_t)t0;
    b.hist = a.hist + (size_t)t0 * L.bins * L.bins;
    if (ordered) {
      b.order = L.order + t0;
      b.order_base = (uint32_t)(L.order_t0 + t0);
    }
    hipError_t e;
    switch (L.block) {
    case 256: e = launch_nt<256>(b, b.n, L.clamp, L.packed, lds, s); break;
    case 512: e = launch_nt<512>(b, b.n, L.clamp, L.packed, lds, s); break;
    default:  // 1024; bricks only with the default 1024-thread shape
      e = L.brick ? launch_nt<1024, true>(b, b.n, L.clamp, L.packed, lds, s)
                  : launch_nt<1024>(b, b.n, L.clamp, L.packed, lds, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_hist_sampled(const HardLaunch& L, const uint2* list, const unsigned long long* n_list,
                               hipStream_t s) {
  if (L.n == 0) return hipSuccess;
  HardArgs a;
  a.transforms = L.transforms;
  a.hist = L.hist;
  a.geom = make_hard_geom(L.fixed, L.moving, L.fbins, L.octs, L.bins);
  a.n = L.n;
  a.chunks = L.chunks;
  a.slab_major = 1;
  a.order = nullptr;  // the sampled sweep keeps the batch order
  a.order_base = 0;
  const size_t lds = hist_lds_bytes(L.bins, L.packed);
  const bool o8 = a.geom.oct8 != 0;
  auto one = [&](const HardArgs& b) -> hipError_t {
    if (L.clamp) {
      if (L.packed) return o8 ? launch_sampled_variant<true, true, true>(b, list, n_list, lds, s)
                              : launch_sampled_variant<true, true, false>(b, list, n_list, lds, s);
      return o8 ? launch_sampled_variant<true, false, true>(b, list, n_list, lds, s)
                : launch_sampled_variant<true, false, false>(b, list, n_list, lds, s);
    }
    if (L.packed) return o8 ? launch_sampled_variant<false, true, true>(b, list, n_list, lds, s)
                            : launch_sampled_variant<false, true, false>(b, list, n_list, lds, s);
    return o8 ? launch_sampled_variant<false, false, true>(b, list, n_list, lds, s)
              : launch_sampled_variant<false, false, false>(b, list, n_list, lds, s);
  };
  const int32_t step = transforms_per_launch(L.chunks, kSampledBlock);
  for (int32_t t0 = 0; t0 < L.n; t0 += step) {
    HardArgs b = a;
    b.n = L.n - t0 < step ? L.n - t0 : step;
    b.transforms = a.transforms + 12 * (size_t)t0;
    b.hist = a.hist + (size_t)t0 * L.bins * L.bins;
    const hipError_t e = one(b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NT, bool BRICK = false>
static hipError_t allow_big_lds() {
  const int bytes = (int)kHardLdsMax;
  const void* fns[8] = {(const void*)hist_hard_kernel<false, false, false, NT, BRICK>,
                        (const void*)hist_hard_kernel<true, false, false, NT, BRICK>,
                        (const void*)hist_hard_kernel<false, true, false, NT, BRICK>,
                        (const void*)hist_hard_kernel<true, true, false, NT, BRICK>,
                        (const void*)hist_hard_kernel<false, false, true, NT, BRICK>,
                        (const void*)hist_hard_kernel<true, false, true, NT, BRICK>,
                        (const void*)hist_hard_kernel<false, true, true, NT, BRICK>,
                        (const void*)hist_hard_kernel<true, true, true, NT, BRICK>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess || (e = lds_register(f)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t configure_hard_kernels() {
  hipError_t e;
  const void* sampled[8] = {
      (const void*)hist_sampled_kernel<false, false, false, kSampledBlock>,
      (const void*)hist_sampled_kernel<true, false, false, kSampledBlock>,
      (const void*)hist_sampled_kernel<false, true, false, kSampledBlock>,
      (const void*)hist_sampled_kernel<true, true, false, kSampledBlock>,
      (const void*)hist_sampled_kernel<false, false, true, kSampledBlock>,
      (const void*)hist_sampled_kernel<true, false, true, kSampledBlock>,
      (const void*)hist_sampled_kernel<false, true, true, kSampledBlock>,
      (const void*)hist_sampled_kernel<true, true, true, kSampledBlock>};
  for (const void* f : sampled)
    if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kHardLdsMax)) != hipSuccess ||
        (e = lds_register(f)) != hipSuccess)
      return e;
  if ((e = allow_big_lds<256>()) != hipSuccess) return e;
  if ((e = allow_big_lds<512>()) != hipSuccess) return e;
  if ((e = allow_big_lds<1024, true>()) != hipSuccess) return e;
  return allow_big_lds<1024>();
}


// ---------------------------------------------------------------------------
// processing order of a batch
// ---------------------------------------------------------------------------

// A thin slab of the fixed volume spans every x and y, so its image in the
// moving volume is set by the moving z that each transform assigns to it:
// workgroups that sweep one slab for transforms of similar z rows read the
// same moving slices, which then stay in the XCD's L2.  Transforms are
// keyed by four features of the index-space z row (M[2][.]) in moving
// voxels: the image depth of the fixed centre, and how much that depth
// changes across the fixed volume's z, x and y extents; the quantised
// features are interleaved bit by bit (a Morton code), with the index in
// the low bits, and each block of kOrderBlock transforms is sorted by that
// key (bitonic, in LDS).  The histograms do not depend on the order.
__global__ __launch_bounds__(1024) void order_transforms_kernel(const double* __restrict__ M, int32_t n,
                                                                float cx, float cy, float cz, float ex, float ey,
                                                                float ez, uint32_t* __restrict__ order) {
  __shared__ unsigned long long key[kOrderBlock];
  const int32_t base = (int32_t)blockIdx.x * kOrderBlock;
  const int32_t m = min(kOrderBlock, n - base);
  int32_t p = 1;
  while (p < m) p <<= 1;
  auto quant = [](float f) -> uint32_t {  // 13 bits, 2 moving voxels per step
    const float v = floorf(f * 0.5f) + 4096.0f;
    return (uint32_t)fminf(fmaxf(v, 0.0f), 8191.0f);
  };
  for (int32_t i = threadIdx.x; i < p; i += blockDim.x) {
    unsigned long long k = ~0ull;
    if (i < m) {
      const double* r = M + 12 * (size_t)(base + i) + 8;  // z row
      const float f[4] = {(float)(r[0] * cx + r[1] * cy + r[2] * cz + r[3]), (float)(r[2] * ez),
                          (float)(r[0] * ex), (float)(r[1] * ey)};
      uint32_t q[4];
      for (int j = 0; j < 4; ++j) q[j] = quant(f[j]);
      unsigned long long code = 0;
      for (int b = 12; b >= 0; --b)
        for (int j = 0; j < 4; ++j) code = (code << 1) | ((q[j] >> b) & 1u);
      k = (code << 12) | (unsigned long long)i;  // 52-bit code, 12-bit index
    }
    key[i] = k;
  }
  __syncthreads();
  for (int32_t size = 2; size <= p; size <<= 1)
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = threadIdx.x; i < p; i += blockDim.x) {
        const int32_t j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const unsigned long long a = key[i], b = key[j];
          if ((a > b) == up) {
            key[i] = b;
            key[j] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int32_t i = threadIdx.x; i < m; i += blockDim.x) order[base + i] = (uint32_t)(base + (key[i] & 0xFFFu));
}

hipError_t launch_order_transforms(const double* M, int32_t n, int32_t fnx, int32_t fny, int32_t fnz, uint32_t* order,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + kOrderBlock - 1) / kOrderBlock);
  hipLaunchKernelGGL(order_transforms_kernel, dim3(blocks), dim3(1024), 0, s, M, n, 0.5f * (float)(fnx - 1),
                     0.5f * (float)(fny - 1), 0.5f * (float)(fnz - 1), (float)(fnx - 1), (float)(fny - 1),
                     (float)(fnz - 1), order);
  return hipGetLastError();
}

}  // namespace gemi
