// Parzen-windowed (cubic B-spline) joint histogram, its MI gradient table
// and the backward sweep, for gfx950.
//
// The fixed side keeps its hard bin; the moving side spreads each voxel
// over 4 bins with the centred cubic B-spline beta3 at
// s = 1 + (v - lo)/(hi - lo) * (B - 4), v the trilinear moving value.  The
// table p = h / N makes MI a smooth function of the transform, so a
// gradient optimiser of Eq. (3) can use d MI / d M, the derivative with
// respect to the 12 entries of the index-space matrix:
//   d MI/d M[r][c] = (ds/dv) / N * sum_x w(x) * dv/dy_r(x) * x~_c,
//   w(x) = -sum_kappa G(bf(x), kappa) * beta3'(kappa - s(x)),
// with G = d MI / d p (per entropy) built once per transform from the
// forward table.  The backward sweep recomputes every voxel's taps rather
// than storing them.
//
// Both sweeps walk the fixed volume like the hard-binned one (16 x 4 voxel
// wave tiles, slab-major workgroup order).  The moving volume is read from
// a quad volume: the four (x, y) corners of the voxel's neighbourhood in a
// slice per element, two loads (slices z and z + 1) per voxel; 8-byte
// elements of exact 16-bit integers for an integer volume, 16-byte fp32
// elements for a float one.  A
// workgroup accumulates one band of table rows (fixed bins) in LDS; bands
// keep large tables within LDS, and a voxel outside the band costs only
// its fixed-bin read.  Workgroup partials are merged into fp64 in HBM.
#include "common.h"

namespace gemi {

// ---------------------------------------------------------------------------
// fp32 quad volume for float moving volumes
// ---------------------------------------------------------------------------

// out[z][y][x] (z <= nz) = (v'(x,y), v'(x1,y), v'(x,y1), v'(x1,y1)),
// v' = clamp(v, lo, hi) - lo, neighbour indices clamped, slice nz = nz-1.
__global__ void pack_quads_f32_kernel(const float* __restrict__ v, int32_t nx, int32_t ny,
                                      int32_t nz, float lo, float hi, float4* __restrict__ out) {
  const int32_t y = blockIdx.y, z = blockIdx.z;
  float4* __restrict__ orow = out + ((size_t)z * ny + y) * nx;
  const int32_t zs = z < nz ? z : nz - 1;
  const float* __restrict__ r0 = v + ((size_t)zs * ny + y) * nx;
  const float* __restrict__ r1 = r0 + (y + 1 < ny ? nx : 0);
  auto c = [&](float a) -> float { return fminf(fmaxf(a, lo), hi) - lo; };
  for (int32_t x = threadIdx.x; x < nx; x += blockDim.x) {
    const int32_t x1 = x + 1 < nx ? x + 1 : nx - 1;
    orow[x] = make_float4(c(r0[x]), c(r0[x1]), c(r1[x]), c(r1[x1]));
  }
}

// out[z][y][x] (z <= nz) = (v'(x,y) | v'(x1,y) << 16, v'(x,y1) | v'(x1,y1) << 16)
// for an integer volume, v' = clamp(v, lo, hi) - lo < 2^16, neighbour
// indices clamped, slice nz = nz-1.
template <typename T>
__global__ void pack_quads16_kernel(const T* __restrict__ v, int32_t nx, int32_t ny, int32_t nz, int32_t lo,
                                    int32_t hi, uint2* __restrict__ out) {
  const int32_t y = blockIdx.y, z = blockIdx.z;
  uint2* __restrict__ orow = out + ((size_t)z * ny + y) * nx;
  const int32_t zs = z < nz ? z : nz - 1;
  const T* __restrict__ r0 = v + ((size_t)zs * ny + y) * nx;
  const T* __restrict__ r1 = r0 + (y + 1 < ny ? nx : 0);
  auto c = [&](int32_t a) -> uint32_t { return (uint32_t)((a < lo ? lo : (a > hi ? hi : a)) - lo); };
  for (int32_t x = threadIdx.x; x < nx; x += blockDim.x) {
    const int32_t x1 = x + 1 < nx ? x + 1 : nx - 1;
    orow[x] = make_uint2(c(r0[x]) | (c(r0[x1]) << 16), c(r1[x]) | (c(r1[x1]) << 16));
  }
}

hipError_t launch_pack_quads16(const VolumeDesc& m, uint2* out, hipStream_t s) {
  const dim3 grid(1, (unsigned)m.ny, (unsigned)m.nz + 1);
  const int32_t lo = (int32_t)m.lo, hi = (int32_t)m.hi;
  switch (m.dtype) {
  case 0: hipLaunchKernelGGL(pack_quads16_kernel<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)m.data, m.nx, m.ny,
                             m.nz, lo, hi, out); break;
  case 1: hipLaunchKernelGGL(pack_quads16_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)m.data, m.nx,
                             m.ny, m.nz, lo, hi, out); break;
  default: hipLaunchKernelGGL(pack_quads16_kernel<int16_t>, grid, dim3(256), 0, s, (const int16_t*)m.data, m.nx,
                              m.ny, m.nz, lo, hi, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_pack_quads_f32(const VolumeDesc& m, float4* out, hipStream_t s) {
  const dim3 grid(1, (unsigned)m.ny, (unsigned)m.nz + 1);
  hipLaunchKernelGGL(pack_quads_f32_kernel, grid, dim3(256), 0, s, (const float*)m.data, m.nx,
                     m.ny, m.nz, (float)m.lo, (float)m.hi, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// occupied fixed-bin rows
// ---------------------------------------------------------------------------

// used[b] = 1 for every bin b that some fixed voxel falls in.  Each thread
// scans 16 consecutive voxels and marks a bin only where it differs from
// the previous voxel and is not yet marked, so long runs of one bin (air)
// cost no LDS writes.
__global__ __launch_bounds__(256) void rows_used_kernel(const uint8_t* __restrict__ fb, size_t n,
                                                        uint32_t* __restrict__ used) {
  __shared__ uint32_t u[256];
  u[threadIdx.x] = 0;
  __syncthreads();
  const size_t n16 = n / 16;
  const uint4* __restrict__ v = (const uint4*)fb;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x) {
    const uint4 w = v[i];
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    uint32_t prev = 0x100u;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t b = (words[k >> 2] >> ((k & 3) * 8)) & 0xFFu;
      if (b != prev && !u[b]) u[b] = 1u;
      prev = b;
    }
  }
  if (blockIdx.x == 0)
    for (size_t i = n16 * 16 + threadIdx.x; i < n; i += blockDim.x) u[fb[i]] = 1u;
  __syncthreads();
  if (u[threadIdx.x]) used[threadIdx.x] = 1u;
}

// Slots: rank of each occupied row among the occupied rows (one workgroup).
__global__ __launch_bounds__(256) void row_map_kernel(RowMap* m, int32_t bins) {
  __shared__ uint32_t pre[256];
  const int r = threadIdx.x;
  const uint32_t used = (r < bins && m->used[r]) ? 1u : 0u;
  pre[r] = used;
  __syncthreads();
  if (r == 0) {
    uint32_t sum = 0;
    for (int i = 0; i < 256; ++i) {
      const uint32_t u = pre[i];
      pre[i] = sum;
      sum += u;
    }
    m->n_slots = sum;
  }
  __syncthreads();
  m->slot_of_row[r] = used ? pre[r] : 0u;
  if (used) m->row_of_slot[pre[r]] = (uint32_t)r;
}

// fbins[i] <- slot of fbins[i], 16 voxels per thread.
__global__ __launch_bounds__(256) void remap_rows_kernel(uint8_t* __restrict__ fb, size_t n,
                                                         const RowMap* __restrict__ m) {
  __shared__ uint32_t slot[256];
  slot[threadIdx.x] = m->slot_of_row[threadIdx.x];
  __syncthreads();
  const size_t n16 = n / 16;
  uint4* __restrict__ v = (uint4*)fb;
  auto map4 = [&](uint32_t w) -> uint32_t {
    return slot[w & 0xFFu] | (slot[(w >> 8) & 0xFFu] << 8) | (slot[(w >> 16) & 0xFFu] << 16) |
           (slot[w >> 24] << 24);
  };
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x) {
    const uint4 w = v[i];
    v[i] = make_uint4(map4(w.x), map4(w.y), map4(w.z), map4(w.w));
  }
  if (blockIdx.x == 0)
    for (size_t i = n16 * 16 + threadIdx.x; i < n; i += blockDim.x) fb[i] = (uint8_t)slot[fb[i]];
}

hipError_t launch_row_map(uint8_t* fbins, size_t nvox, int32_t bins, RowMap* m, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u32(m->used, 256, 0u, s)) != hipSuccess) return e;
  const size_t blocks = (nvox / 16 + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks));
  hipLaunchKernelGGL(rows_used_kernel, dim3(grid), dim3(256), 0, s, (const uint8_t*)fbins, nvox, m->used);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(row_map_kernel, dim3(1), dim3(256), 0, s, m, bins);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(remap_rows_kernel, dim3(grid), dim3(256), 0, s, fbins, nvox, (const RowMap*)m);
  return hipGetLastError();
}

// One thread per wave tile (kTileX x kTileY voxels of one slice): the OR of
// the slot groups of its voxels.
__global__ __launch_bounds__(256) void tile_mask_kernel(const uint8_t* __restrict__ slots, int32_t nx, int32_t ny,
                                                        int32_t nz, uint32_t* __restrict__ mask) {
  const int32_t XT = (nx + kTileX - 1) / kTileX, G = (ny + kTileY - 1) / kTileY;
  const int64_t tiles = (int64_t)G * nz * XT;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tiles; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = t / XT;
    const int32_t xt = (int32_t)(t - g * XT);
    const int32_t k = (int32_t)(g / G), j0 = (int32_t)(g - (int64_t)k * G) * kTileY;
    const int32_t x0 = xt * kTileX, x1 = min(nx, x0 + kTileX);
    uint32_t m = 0;
    for (int32_t j = j0; j < min(ny, j0 + kTileY); ++j) {
      const uint8_t* row = slots + ((int64_t)k * ny + j) * nx;
      for (int32_t x = x0; x < x1; ++x) m |= 1u << (row[x] / kSlotGroup);
    }
    mask[t] = m;
  }
}

// One thread per row group: the OR of its tiles' masks, after the tiles.
__global__ __launch_bounds__(256) void row_mask_kernel(int32_t XT, int64_t groups, uint32_t* __restrict__ mask) {
  const uint32_t* __restrict__ tiles = mask;
  uint32_t* __restrict__ rows = mask + groups * XT;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < groups; g += (int64_t)gridDim.x * blockDim.x) {
    uint32_t m = 0;
    for (int32_t t = 0; t < XT; ++t) m |= tiles[g * XT + t];
    rows[g] = m;
  }
}

hipError_t launch_tile_mask(const uint8_t* slots, int32_t nx, int32_t ny, int32_t nz, uint32_t* mask, hipStream_t s) {
  const int64_t tiles = parzen_tiles(nx, ny, nz);
  const int64_t blocks = (tiles + 255) / 256;
  hipLaunchKernelGGL(tile_mask_kernel, dim3((unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192)), dim3(256),
                     0, s, slots, nx, ny, nz, mask);
  const int64_t groups = parzen_row_groups(ny, nz);
  const int64_t gblocks = (groups + 255) / 256;
  hipLaunchKernelGGL(row_mask_kernel, dim3((unsigned)(gblocks < 8192 ? (gblocks > 0 ? gblocks : 1) : 8192)),
                     dim3(256), 0, s, (int32_t)((nx + kTileX - 1) / kTileX), groups, mask);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-voxel sample shared by the forward and backward sweeps
// ---------------------------------------------------------------------------

typedef unsigned int uint4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

typedef unsigned int uint2_t __attribute__((ext_vector_type(2)));

// Corner values c[z][y][x] of the 2x2x2 neighbourhood: two quads, slices z
// and z + 1 (`slice_bytes` apart), fp32 (FQ, 16 bytes each) or 16-bit
// integers (8 bytes each).
template <bool FQ>
__device__ __forceinline__ void gather(const __amdgpu_buffer_rsrc_t& rsrc, uint32_t idx,
                                       int32_t slice_bytes, float c[2][2][2]) {
  if (FQ) {
    const float4_t a = __builtin_bit_cast(float4_t, __builtin_amdgcn_raw_buffer_load_b128(rsrc, idx * 16u, 0, 0));
    const float4_t b = __builtin_bit_cast(float4_t, __builtin_amdgcn_raw_buffer_load_b128(rsrc, idx * 16u, slice_bytes, 0));
    c[0][0][0] = a.x; c[0][0][1] = a.y; c[0][1][0] = a.z; c[0][1][1] = a.w;
    c[1][0][0] = b.x; c[1][0][1] = b.y; c[1][1][0] = b.z; c[1][1][1] = b.w;
  } else {
    const uint2_t a = __builtin_amdgcn_raw_buffer_load_b64(rsrc, idx * 8u, 0, 0);
    const uint2_t b = __builtin_amdgcn_raw_buffer_load_b64(rsrc, idx * 8u, slice_bytes, 0);
    c[0][0][0] = (float)(a.x & 0xFFFFu); c[0][0][1] = (float)(a.x >> 16);
    c[0][1][0] = (float)(a.y & 0xFFFFu); c[0][1][1] = (float)(a.y >> 16);
    c[1][0][0] = (float)(b.x & 0xFFFFu); c[1][0][1] = (float)(b.x >> 16);
    c[1][1][0] = (float)(b.y & 0xFFFFu); c[1][1][1] = (float)(b.y >> 16);
  }
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

// The four B-spline weights beta3(kappa0 + i - s), kappa0 = floor(s) - 1,
// as polynomials in the fraction f = s - floor(s).
__device__ __forceinline__ void bspline_weights(float f, float w[4]) {
  const float f2 = f * f, f3 = f2 * f, g = 1.0f - f;
  w[0] = g * g * g * (1.0f / 6.0f);
  w[1] = fmaf(0.5f, f3, 2.0f / 3.0f - f2);
  w[2] = (fmaf(-3.0f, f3, fmaf(3.0f, f2, fmaf(3.0f, f, 1.0f)))) * (1.0f / 6.0f);
  w[3] = f3 * (1.0f / 6.0f);
}

// Their derivatives beta3'(kappa0 + i - s).
__device__ __forceinline__ void bspline_slopes(float f, float d[4]) {
  const float g = 1.0f - f;
  d[0] = 0.5f * g * g;
  d[1] = f * fmaf(-1.5f, f, 2.0f);
  d[2] = g * fmaf(1.5f, g, -2.0f);
  d[3] = -0.5f * f * f;
}

// floor(w * 2^40) for a weight w in [0, 2/3], as hi * 2^32 + lo with
// hi = floor(w * 2^8) < 2^8 and lo the next 32 bits of w * 2^8.
__device__ __forceinline__ unsigned long long fixed40(float w) {
  const float a = w * 256.0f;
  const uint32_t hi = (uint32_t)a;
  const uint32_t lo = (uint32_t)(__builtin_amdgcn_fractf(a) * 4294967296.0f);
  return ((unsigned long long)hi << 32) | lo;
}

// Dynamic LDS limit of the Parzen sweeps: band budgets up to 128 KiB (the
// launch shape picks one), with room for the static arrays beside them
// within the 160 KiB a workgroup may hold.
constexpr size_t kParzenLdsMax = 144 * 1024;

// Sweep geometry of one workgroup.
struct SweepCtx {
  uint32_t t, chunk, band;
  int32_t r_lo, r_hi;  // slots (occupied fixed-bin rows) of this band
};

// ---------------------------------------------------------------------------
// forward: Parzen table
// ---------------------------------------------------------------------------

// The band's table is accumulated in LDS as unsigned 24.40 fixed point: each
// voxel adds its four B-spline weights scaled by 2^40, with the largest
// derived by subtraction so that the voxel's mass is exactly 2^40 (the
// four cubic B-spline weights at any shift sum to one: partition of
// unity).  Integer adds commute, so the table does
// not depend on the order of the atomics.  The 2^-40 step keeps the tiny
// taps (w ~ f^3 / 6) accurate to ~1e-12, below the fp32 rounding of the
// weights themselves; a coarser step biases the near-empty cells that
// dominate the Tsallis gradient for q < 1.  A 64-bit cell cannot overflow:
// a workgroup covers fewer than 2^24 voxels (2^28 voxels at most, split
// into at least 32 workgroups per transform).  64-bit LDS atomics need an
// 8-byte aligned address, hence the alignment of the table.
//
// Slot 0, the lowest occupied fixed bin, is the background of a medical
// volume (air, most of a CT): whole waves add their taps into a handful of
// its cells, and same-address and same-bank LDS atomics serialise.  The
// band holding it keeps kHotCopies bank-skewed copies of the row's first
// parzen_hot_cols(B) columns (common.h), lane l adding into copy
// l % kHotCopies; the copies are summed at the flush.
// Cell index and 32-bit fraction of an exact Q32 coordinate q on an axis of
// n samples, q clamped to [0, (n - 1) 2^32]: the index is the high word held
// to [0, n - 1]; the fraction is the low word while the high word lies in
// [0, n - 2], and zero otherwise (at or past either end the clamped
// coordinate is a whole sample).  The high word fits 32 bits for every
// usable matrix (linear entries <= 2^16, translations <= 2^24).
__device__ __forceinline__ void clamp_q32(int64_t q, int32_t n, uint32_t& cell, uint32_t& frac) {
  const int32_t hi = (int32_t)(q >> 32);
  cell = (uint32_t)min(max(hi, 0), n - 1);
  frac = (uint32_t)hi < (uint32_t)(n - 1) ? (uint32_t)q : 0u;
}

// Where a fixed voxel reads the moving volume: gather index, 32-bit
// fractions per axis, and whether it takes part (EXCLUDE drops voxels
// outside the volume).
struct Loc {
  uint32_t idx, frac[3];
  bool inside;
};

// A voxel's moving neighbourhood as loaded: two quads, a: slice z, b:
// slice z + 1 (fp32: all four words; 16-bit integers: .x and .y).
struct Raw {
  uint4_t a, b;
};

// Corner values c[z][y][x] of a loaded neighbourhood.
template <bool FQ>
__device__ __forceinline__ void unpack(const Raw& d, float c[2][2][2]) {
  if (FQ) {
    const float4_t a = __builtin_bit_cast(float4_t, d.a), b = __builtin_bit_cast(float4_t, d.b);
    c[0][0][0] = a.x; c[0][0][1] = a.y; c[0][1][0] = a.z; c[0][1][1] = a.w;
    c[1][0][0] = b.x; c[1][0][1] = b.y; c[1][1][0] = b.z; c[1][1][1] = b.w;
  } else {
    c[0][0][0] = (float)(d.a.x & 0xFFFFu); c[0][0][1] = (float)(d.a.x >> 16);
    c[0][1][0] = (float)(d.a.y & 0xFFFFu); c[0][1][1] = (float)(d.a.y >> 16);
    c[1][0][0] = (float)(d.b.x & 0xFFFFu); c[1][0][1] = (float)(d.b.x >> 16);
    c[1][1][0] = (float)(d.b.y & 0xFFFFu); c[1][1][1] = (float)(d.b.y >> 16);
  }
}

// The tiles of a row group that hold slots of a band, 64 tiles at a time:
// lane i reads tile base + i's mask and a ballot gathers the wave's
// answers, so the walk visits only those tiles and a tile without the
// band's slots costs no load (bands other than the background's find their
// slots in a few percent of the tiles).
struct ActiveTiles {
  uint64_t bits;  // tile base + i holds slots of the band (uniform)
  int32_t base;

  __device__ __forceinline__ ActiveTiles(const uint32_t* __restrict__ tmask, int32_t tb, int32_t XT, int lane,
                                         uint32_t band_groups) {
    const int32_t t = tb + lane;
    const uint32_t m = t < XT ? tmask[t] : 0u;
    bits = __ballot((m & band_groups) != 0u);
    base = tb;
  }
  __device__ __forceinline__ bool any() const { return bits != 0; }
  // the first tile, taken off the set
  __device__ __forceinline__ int32_t first() {
    const int32_t t = base + (int32_t)__builtin_ctzll(bits);
    bits &= bits - 1;
    return t;
  }
  // the next tile, taken off the set, or -1
  __device__ __forceinline__ int32_t next() {
    if (!bits) return -1;
    return first();
  }
};

// Slot of the fixed voxel at x of a lane's row, or -1 past the row.
__device__ __forceinline__ int32_t fixed_slot(const uint8_t* __restrict__ frow, bool row_ok, int32_t x, int32_t nx) {
  return row_ok && x < nx ? (int32_t)frow[x] : -1;
}

// Calls f(q, slot, x) for the voxels of a lane's row in a row group: x its
// column, q its exact Q32 moving coordinates, slot its fixed slot (-1 past
// the row), loaded one visited tile ahead.  A band that holds every slot
// visits every tile in order; any other band only the tiles with its slots.
template <typename F>
__device__ __forceinline__ void row_tiles(const GroupWalkFlex& w, const uint32_t* __restrict__ tmask, int32_t XT,
                                          int lane, int dx, uint32_t band_groups, bool every,
                                          const uint8_t* __restrict__ frow, bool row_ok, int32_t nx, F&& f) {
  if (every) {
    int64_t q[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = w.r[r] + w.lane_off[r];
    int32_t fb_next = fixed_slot(frow, row_ok, dx, nx);
    for (int32_t ti = 0; ti < XT; ++ti) {
      const int32_t x = ti * kTileX + dx;
      const int32_t fbv = fb_next;
      if (ti + 1 < XT) fb_next = fixed_slot(frow, row_ok, x + kTileX, nx);
      f(q, fbv, x);
#pragma unroll
      for (int r = 0; r < 3; ++r) q[r] += w.step[r];
    }
    return;
  }
  for (int32_t tb = 0; tb < XT; tb += 64) {
    ActiveTiles at(tmask, tb, XT, lane, band_groups);
    if (!at.any()) continue;
    int32_t ti = at.first();
    int64_t q[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = w.r[r] + w.lane_off[r] + w.step[r] * ti;
    int32_t fb_next = fixed_slot(frow, row_ok, ti * kTileX + dx, nx);
    for (;;) {
      const int32_t fbv = fb_next;
      const int32_t tn = at.next();
      if (tn >= 0) fb_next = fixed_slot(frow, row_ok, tn * kTileX + dx, nx);
      f(q, fbv, ti * kTileX + dx);
      if (tn < 0) break;
      // to the next visited tile one step at a time (a skipped tile costs
      // three adds; a jump would need 64-bit products)
      do {
#pragma unroll
        for (int r = 0; r < 3; ++r) q[r] += w.step[r];
      } while (++ti < tn);
    }
  }
}

// Per-launch constants of the forward step of one fixed voxel.
struct ParzenFwdStep {
  __amdgpu_buffer_rsrc_t rsrc;
  uint64_t top[3];
  int32_t n[3];
  uint32_t NY, MX;
  int32_t SZ;  // bytes to the next slice of quads
  int B, pitch;
  float sscale, smax;

  template <bool FQ>
  __device__ __forceinline__ static ParzenFwdStep make(const ParzenArgs& a) {
    ParzenFwdStep p;
    p.top[0] = (uint64_t)(a.mnx - 1) << 32;
    p.top[1] = (uint64_t)(a.mny - 1) << 32;
    p.top[2] = (uint64_t)(a.mnz - 1) << 32;
    p.n[0] = a.mnx;
    p.n[1] = a.mny;
    p.n[2] = a.mnz;
    p.NY = (uint32_t)a.mny;
    p.MX = (uint32_t)a.mnx;
    p.SZ = (FQ ? 16 : 8) * a.mnx * a.mny;
    p.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)a.gvol, (short)0, (int)a.gvol_bytes, 0x00020000);
    p.B = a.bins;
    p.pitch = parzen_pitch(a.bins);
    p.sscale = a.sscale;
    p.smax = (float)(p.B - 3);
    return p;
  }

  // Where a fixed voxel at exact Q32 moving coordinates q reads the moving
  // volume: clamped (CLAMP) or dropped outside [0, n - 1].
  template <bool CLAMP>
  __device__ __forceinline__ Loc locate(const int64_t q[3]) const {
    Loc l;
    l.inside = true;
    uint32_t cix[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (CLAMP) {
        clamp_q32(q[r], n[r], cix[r], l.frac[r]);
      } else {
        l.inside = l.inside && (uint64_t)q[r] <= top[r];
        cix[r] = (uint32_t)(q[r] >> 32);
        l.frac[r] = (uint32_t)q[r];
      }
    }
    l.idx = mad24(mad24(cix[2], NY, cix[1]), MX, cix[0]);
    return l;
  }

  // The voxel's 2x2x2 moving neighbourhood as stored: two float4 quads
  // (FQ), one 16-bit oct (OCT: all eight corners in one 16-byte record, as
  // the hard path stores them), or two 16-bit quads.
  template <bool FQ, bool OCT = false>
  __device__ __forceinline__ Raw fetch(uint32_t idx) const {
    Raw d;
    if (OCT) {
      const uint4_t o = __builtin_amdgcn_raw_buffer_load_b128(rsrc, idx * 16u, 0, 0);
      d.a = uint4_t{o.x, o.y, 0u, 0u};
      d.b = uint4_t{o.z, o.w, 0u, 0u};
    } else if (FQ) {
      d.a = __builtin_amdgcn_raw_buffer_load_b128(rsrc, idx * 16u, 0, 0);
      d.b = __builtin_amdgcn_raw_buffer_load_b128(rsrc, idx * 16u, SZ, 0);
    } else {
      const uint2_t lo = __builtin_amdgcn_raw_buffer_load_b64(rsrc, idx * 8u, 0, 0);
      const uint2_t hi = __builtin_amdgcn_raw_buffer_load_b64(rsrc, idx * 8u, SZ, 0);
      d.a = uint4_t{lo.x, lo.y, 0u, 0u};
      d.b = uint4_t{hi.x, hi.y, 0u, 0u};
    }
    return d;
  }

  // The four B-spline taps of a located, fetched voxel of slot fb (in the
  // band) into the LDS table.
  template <bool FQ>
  __device__ __forceinline__ void taps(const Raw& d, const Loc& l, int32_t fb, const SweepCtx& sc, int cells,
                                       int copy, unsigned long long* lds_tab) const {
    float c[2][2][2];
    unpack<FQ>(d, c);
    const float tx = (float)l.frac[0] * 2.3283064365386963e-10f;
    const float ty = (float)l.frac[1] * 2.3283064365386963e-10f;
    const float tz = (float)l.frac[2] * 2.3283064365386963e-10f;
    const float v0 = lerpf(lerpf(c[0][0][0], c[0][0][1], tx), lerpf(c[0][1][0], c[0][1][1], tx), ty);
    const float v1 = lerpf(lerpf(c[1][0][0], c[1][0][1], tx), lerpf(c[1][1][0], c[1][1][1], tx), ty);
    const float v = lerpf(v0, v1, tz);
    const float s = fminf(fmaxf(fmaf(v, sscale, 1.0f), 1.0f), smax);
    const float fl = floorf(s);
    float wt[4];
    bspline_weights(s - fl, wt);
    const unsigned long long q0 = fixed40(wt[0]), q2 = fixed40(wt[2]), q3 = fixed40(wt[3]);
    const unsigned long long q1 = (1ull << 40) - q0 - q2 - q3;  // w1 >= 1/6
    const int32_t col0 = (int32_t)fl - 1;
    int base = (int)__umul24((uint32_t)(fb - sc.r_lo), (uint32_t)pitch) + col0;  // fb >= r_lo
    // slot 0 (in band 0 only): the lane's copy of the row's hot columns
    if (fb == 0 && col0 + 3 < parzen_hot_cols(B)) base = cells + copy * parzen_hot_stride(B) + col0;
    unsigned long long* cell = lds_tab + base;
    atomicAdd(cell + 0, q0);
    atomicAdd(cell + 1, q1);
    atomicAdd(cell + 2, q2);
    atomicAdd(cell + 3, q3);
  }

  // One fixed voxel at exact Q32 moving coordinates q: if it lies inside
  // (or CLAMP) and its slot falls in the band's rows, its four B-spline taps
  // go into the LDS table.  Returns whether the voxel took part in this band
  // (each voxel belongs to one band, so the bands' counts add up to N).
  template <bool FQ, bool CLAMP, bool OCT = false>
  __device__ __forceinline__ bool add(const int64_t q[3], int32_t fb, const SweepCtx& sc, int cells, int copy,
                                      unsigned long long* lds_tab) const {
    const Loc l = locate<CLAMP>(q);
    if (!l.inside || fb < sc.r_lo || fb >= sc.r_hi) return false;
    taps<FQ>(fetch<FQ, OCT>(l.idx), l, fb, sc, cells, copy, lds_tab);
    return true;
  }
};

// Adds the band's LDS table into the transform's HBM table (fp64) and the
// count of the band's voxels that took part.
template <int NT>
__device__ __forceinline__ void flush_parzen(const ParzenArgs& a, const SweepCtx& sc, int cells, int hot_cells,
                                             const unsigned long long* lds_tab, uint32_t lds_count) {
  const int B = a.bins, pitch = parzen_pitch(B);
  double* __restrict__ out = a.table + (size_t)sc.t * B * B;
  const int hot_cols = hot_cells ? parzen_hot_cols(B) : 0, hot_stride = parzen_hot_stride(B);
  // a wave per band row, a lane per column: the row's table row is read
  // once per wave, and no cell index is divided by the pitch
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int rr = wave; rr < sc.r_hi - sc.r_lo; rr += NT / 64) {
    double* __restrict__ orow = out + (size_t)a.rows->row_of_slot[sc.r_lo + rr] * B;
    for (int c = lane; c < B; c += 64) {
      unsigned long long v = lds_tab[rr * pitch + c];
      if (rr == 0 && c < hot_cols)  // slot 0's row is the band's first
        for (int k = 0; k < kHotCopies; ++k) v += lds_tab[cells + k * hot_stride + c];
      if (v) atomicAdd(&orow[c], (double)v * 9.094947017729282379150390625e-13);  // 2^-40
    }
  }
  if (threadIdx.x == 0 && lds_count)
    atomicAdd((unsigned long long*)&a.count[sc.t], (unsigned long long)lds_count);
}

template <bool FQ, bool CLAMP, int NT>
__global__ __launch_bounds__(NT) void parzen_fwd_kernel(ParzenArgs a) {
  extern __shared__ __align__(16) unsigned long long lds_tab[];
  __shared__ uint32_t lds_count;
  const int B = a.bins;
  SweepCtx sc;
  block_work(a.chunks, a.n, a.bands, a.slab_major, sc.t, sc.chunk, sc.band);
  const int32_t n_slots = (int32_t)a.rows->n_slots;
  sc.r_lo = (int32_t)sc.band * a.band_rows;
  if (sc.r_lo >= n_slots) return;  // a band past the occupied rows (whole workgroup)
  sc.r_hi = min(n_slots, sc.r_lo + a.band_rows);
  const int cells = (sc.r_hi - sc.r_lo) * parzen_pitch(B);
  const int hot_cells = sc.r_lo == 0 ? parzen_hot_cells(B) : 0;  // copies of slot 0's hot columns
  for (int e = threadIdx.x; e < cells + hot_cells; e += NT) lds_tab[e] = 0ull;
  if (threadIdx.x == 0) lds_count = 0;
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)sc.t, Mq);
  __syncthreads();
  uint32_t taken = 0;
  const int copy = (threadIdx.x & (kHotCopies - 1));  // this lane's copy of slot 0
  if (ok) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int dx = lane & (kTileX - 1), dy = lane / kTileX;
    // bands of rare slots (not the background's) interleave their waves
    GroupWalkFlex w;
    w.init(Mq, a.fny, a.fnz, a.chunks, sc.chunk, wave, NT / 64, dx, dy, sc.r_lo > 0);
    const ParzenFwdStep ps = ParzenFwdStep::template make<FQ>(a);
    const int32_t XT = (a.fnx + kTileX - 1) / kTileX;
    const uint32_t band_groups = slot_group_mask(sc.r_lo, sc.r_hi);
    const bool every = sc.r_lo == 0 && sc.r_hi >= n_slots;  // the band holds every slot
    for (; w.g < w.g1; w.next()) {
      if (!(a.row_mask[w.g] & band_groups)) continue;  // no slot of this band in the row group
      const int32_t j = w.j0 + dy;
      const bool row_ok = j < a.fny;
      const uint8_t* __restrict__ frow = a.fbins + ((int64_t)w.k * a.fny + (row_ok ? j : 0)) * a.fnx;
      const uint32_t* __restrict__ tmask = a.tile_mask + (int64_t)w.g * XT;
      row_tiles(w, tmask, XT, lane, dx, band_groups, every, frow, row_ok, a.fnx,
                [&](const int64_t q[3], int32_t fbv, int32_t) {
                  if (fbv >= 0) taken += ps.add<FQ, CLAMP>(q, fbv, sc, cells, copy, lds_tab);
                });
    }
  }
  if (taken) atomicAdd(&lds_count, taken);
  __syncthreads();
  if (!ok) return;
  flush_parzen<NT>(a, sc, cells, hot_cells, lds_tab, lds_count);
}

// Sampled forward: as parzen_fwd_kernel over the workgroup's share of the
// sample list (entries {x | y << 12 | slot << 24, z}), each sample's Q32
// coordinates formed straight from the matrix.
template <bool FQ, bool CLAMP, int NT>
__global__ __launch_bounds__(NT) void parzen_sampled_fwd_kernel(ParzenArgs a, const uint2* __restrict__ list,
                                                                const unsigned long long* __restrict__ n_list) {
  extern __shared__ __align__(16) unsigned long long lds_tab[];
  __shared__ uint32_t lds_count;
  const int B = a.bins;
  SweepCtx sc;
  block_work(a.chunks, a.n, a.bands, a.slab_major, sc.t, sc.chunk, sc.band);
  const int32_t n_slots = (int32_t)a.rows->n_slots;
  sc.r_lo = (int32_t)sc.band * a.band_rows;
  if (sc.r_lo >= n_slots) return;  // a band past the occupied rows (whole workgroup)
  sc.r_hi = min(n_slots, sc.r_lo + a.band_rows);
  const int cells = (sc.r_hi - sc.r_lo) * parzen_pitch(B);
  const int hot_cells = sc.r_lo == 0 ? parzen_hot_cells(B) : 0;
  for (int e = threadIdx.x; e < cells + hot_cells; e += NT) lds_tab[e] = 0ull;
  if (threadIdx.x == 0) lds_count = 0;
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)sc.t, Mq);
  __syncthreads();
  uint32_t taken = 0;
  const int copy = (threadIdx.x & (kHotCopies - 1));
  if (ok) {
    const ParzenFwdStep ps = ParzenFwdStep::template make<FQ>(a);
    const int64_t ns = (int64_t)*n_list;
    const int64_t s0 = ns * sc.chunk / a.chunks, s1 = ns * (sc.chunk + 1) / a.chunks;
    for (int64_t e = s0 + threadIdx.x; e < s1; e += NT) {
      const uint2 en = list[e];
      const int64_t x = en.x & 0xFFFu, y = (en.x >> 12) & 0xFFFu, z = en.y;
      const int32_t slot = (int32_t)(en.x >> 24);
      int64_t q[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) q[r] = Mq[4 * r] * x + Mq[4 * r + 1] * y + Mq[4 * r + 2] * z + Mq[4 * r + 3];
      // integer moving volumes come as 16-bit octs here: a sample's eight
      // corners in one cache line (the quads' two slices are two lines,
      // and the samples of a list share few lines with each other)
      taken += ps.add<FQ, CLAMP, !FQ>(q, slot, sc, cells, copy, lds_tab);
    }
  }
  if (taken) atomicAdd(&lds_count, taken);
  __syncthreads();
  if (!ok) return;
  flush_parzen<NT>(a, sc, cells, hot_cells, lds_tab, lds_count);
}

// ---------------------------------------------------------------------------
// d MI / d p tables
// ---------------------------------------------------------------------------

// One workgroup per transform:
//   Shannon           G = ln(p / p_m)
//   Tsallis additive  G = q/(q-1) * (p^(q-1) - p_m^(q-1))
//   Tsallis pseudo    G = q/(q-1) * (p^(q-1) - (1 + (1-q) S_q(F)) p_m^(q-1))
// and G = 0 where p = 0 (no voxel there has a non-zero B-spline slope).
// One workgroup per (transform, row slice), sliced like the MI reduction:
// the marginals come from the reduction (a.marg), so a slice reads only its
// own rows of the table.  Per entropy the column terms ln p_m (Shannon) or
// fac p_m^(q-1) (Tsallis) are formed once per workgroup.
__global__ __launch_bounds__(256) void dmi_dp_kernel(ParzenArgs a, QList ql, int32_t S) {
  const int B = a.bins;
  const size_t BB = (size_t)B * B;
  const int t = blockIdx.x / S, sl = blockIdx.x - t * S;
  int r0, r1;
  slice_rows(B, S, sl, r0, r1);
  __shared__ double pm[256], pf[256], cterm[256];
  __shared__ double red[256];
  const double* __restrict__ h = a.table + (size_t)t * BB;
  float* __restrict__ G = (float*)a.gtab + (size_t)t * ql.n * BB;
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)t, Mq);
  const double N = (double)a.count[t];
  if (!ok || !(N > 0)) {
    for (int iq = 0; iq < ql.n; ++iq)
      for (int e = r0 * B + threadIdx.x; e < r1 * B; e += 256) G[(size_t)iq * BB + e] = 0.0f;
    return;
  }
  const double invN = 1.0 / N;
  const double* __restrict__ mg = a.marg + (size_t)t * 2 * B;
  for (int i = threadIdx.x; i < B; i += 256) {
    pf[i] = mg[i] * invN;
    pm[i] = mg[B + i] * invN;
  }
  __syncthreads();
  for (int iq = 0; iq < ql.n; ++iq) {
    const double q = ql.q[iq], e1 = q - 1.0;
    double fac = 1.0;
    if (q != 1.0 && ql.pseudo) {
      // S_q(F) = -sum p expm1((q-1) ln p) / (q-1)
      double part = 0;
      for (int i = threadIdx.x; i < B; i += 256)
        if (pf[i] > 0) part += pf[i] * expm1(e1 * log(pf[i]));
      red[threadIdx.x] = part;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      fac = 1.0 + (1.0 - q) * (-red[0] / e1);
      __syncthreads();
    }
    for (int i = threadIdx.x; i < B; i += 256)
      cterm[i] = pm[i] > 0 ? (q == 1.0 ? log(pm[i]) : fac * pow(pm[i], e1)) : 0.0;
    __syncthreads();
    float* __restrict__ Gq = G + (size_t)iq * BB;
    for (int e = r0 * B + threadIdx.x; e < r1 * B; e += 256) {
      const double hv = h[e];
      double g = 0.0;
      if (hv > 0) {
        const double p = hv * invN, m = cterm[e % B];
        g = q == 1.0 ? log(p) - m : q / e1 * (pow(p, e1) - m);
      }
      Gq[e] = (float)g;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// backward: gradient sweep
// ---------------------------------------------------------------------------

template <bool FQ, bool CLAMP, int NQG, int NT>
__global__ __launch_bounds__(NT) void parzen_bwd_kernel(ParzenArgs a) {
  extern __shared__ float lds_g[];  // [NQG][band rows][B]
  constexpr int NW = NT / 64;
  __shared__ double part[NW][NQG * 12];
  const int B = a.bins;
  const size_t BB = (size_t)B * B;
  SweepCtx sc;
  block_work(a.chunks, a.n, a.bands, a.slab_major, sc.t, sc.chunk, sc.band);
  const int32_t n_slots = (int32_t)a.rows->n_slots;
  sc.r_lo = (int32_t)sc.band * a.band_rows;
  if (sc.r_lo >= n_slots) return;  // a band past the occupied rows (whole workgroup)
  sc.r_hi = min(n_slots, sc.r_lo + a.band_rows);
  const int cells = (sc.r_hi - sc.r_lo) * parzen_pitch(B);
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)sc.t, Mq);
  const int nqg = min(NQG, a.n_q - a.q0);
  {
    // a wave per band row: the row's pitch cells (B <= 256, so at most 5 per
    // lane), all loads issued before the first store
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, pitch = parzen_pitch(B);
    const int nrows = sc.r_hi - sc.r_lo;
    for (int g = 0; g < nqg; ++g) {
      const float* __restrict__ src = a.gtab + ((size_t)sc.t * a.n_q + a.q0 + g) * BB;
      for (int rr = wave; rr < nrows; rr += NW) {
        const float* __restrict__ srow = src + (size_t)a.rows->row_of_slot[sc.r_lo + rr] * B;
        float v[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int c = lane + 64 * k;
          v[k] = c < B ? srow[c] : 0.0f;
        }
        float* __restrict__ drow = lds_g + g * cells + rr * pitch;
#pragma unroll
        for (int k = 0; k < 5; ++k)
          if (lane + 64 * k < pitch) drow[lane + 64 * k] = v[k];
      }
    }
  }
  __syncthreads();
  float acc[NQG][12];
#pragma unroll
  for (int g = 0; g < NQG; ++g)
#pragma unroll
    for (int e = 0; e < 12; ++e) acc[g][e] = 0.0f;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (ok && a.count[sc.t] > 0) {
    const int dx = lane & (kTileX - 1), dy = lane / kTileX;
    GroupWalkFlex w;  // as in the forward
    w.init(Mq, a.fny, a.fnz, a.chunks, sc.chunk, wave, NW, dx, dy, sc.r_lo > 0);
    const int32_t nq[3] = {a.mnx, a.mny, a.mnz};
    const uint64_t top[3] = {(uint64_t)(a.mnx - 1) << 32, (uint64_t)(a.mny - 1) << 32,
                             (uint64_t)(a.mnz - 1) << 32};
    const uint32_t NY = (uint32_t)a.mny, MX = (uint32_t)a.mnx;
    const int32_t SZ = (FQ ? 16 : 8) * a.mnx * a.mny;  // quads: next slice
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.gvol, (short)0, (int)a.gvol_bytes, 0x00020000);
    const float smax = (float)(B - 3);
    const int32_t XT = (a.fnx + kTileX - 1) / kTileX;
    const uint32_t band_groups = slot_group_mask(sc.r_lo, sc.r_hi);
    const bool every = sc.r_lo == 0 && sc.r_hi >= n_slots;  // the band holds every slot
    for (; w.g < w.g1; w.next()) {
      if (!(a.row_mask[w.g] & band_groups)) continue;  // no slot of this band in the row group
      const int32_t j = w.j0 + dy;
      const bool row_ok = j < a.fny;
      const uint8_t* __restrict__ frow = a.fbins + ((int64_t)w.k * a.fny + (row_ok ? j : 0)) * a.fnx;
      const uint32_t* __restrict__ tmask = a.tile_mask + (int64_t)w.g * XT;
      const float fj = (float)j, fk = (float)w.k;
      // per-lane sums over the row group's x steps of gr and gr x
      float rs[NQG][3], rx[NQG][3];
#pragma unroll
      for (int g = 0; g < NQG; ++g)
#pragma unroll
        for (int r = 0; r < 3; ++r) rs[g][r] = rx[g][r] = 0.0f;
      // one voxel of slot fb in this band at Q32 coordinates q, x its column
      auto differentiate = [&](const int64_t q[3], int32_t fb, int32_t x) {
        uint32_t cell[3], frac[3];
        bool inside = true, moves[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          // a clamped coordinate does not move with the transform
          moves[r] = (uint64_t)q[r] <= top[r];
          if (CLAMP) {
            clamp_q32(q[r], nq[r], cell[r], frac[r]);
          } else {
            inside = inside && moves[r];
            cell[r] = (uint32_t)(q[r] >> 32);
            frac[r] = (uint32_t)q[r];
          }
        }
        if (!inside) return;
        const uint32_t idx = mad24(mad24(cell[2], NY, cell[1]), MX, cell[0]);
        float c[2][2][2];
        gather<FQ>(rsrc, idx, SZ, c);
        const float tx = (float)frac[0] * 2.3283064365386963e-10f;
        const float ty = (float)frac[1] * 2.3283064365386963e-10f;
        const float tz = (float)frac[2] * 2.3283064365386963e-10f;
        // x-lerps per (y, z) edge and their x-slopes
        const float e00 = lerpf(c[0][0][0], c[0][0][1], tx), e01 = lerpf(c[0][1][0], c[0][1][1], tx);
        const float e10 = lerpf(c[1][0][0], c[1][0][1], tx), e11 = lerpf(c[1][1][0], c[1][1][1], tx);
        const float d00 = c[0][0][1] - c[0][0][0], d01 = c[0][1][1] - c[0][1][0];
        const float d10 = c[1][0][1] - c[1][0][0], d11 = c[1][1][1] - c[1][1][0];
        const float v0 = lerpf(e00, e01, ty), v1 = lerpf(e10, e11, ty);
        const float v = lerpf(v0, v1, tz);
        float dv[3];
        dv[0] = lerpf(lerpf(d00, d01, ty), lerpf(d10, d11, ty), tz);
        dv[1] = lerpf(e01 - e00, e11 - e10, tz);
        dv[2] = v1 - v0;
#pragma unroll
        for (int r = 0; r < 3; ++r) dv[r] = moves[r] ? dv[r] : 0.0f;
        const float s = fminf(fmaxf(fmaf(v, a.sscale, 1.0f), 1.0f), smax);
        const float fl = floorf(s);
        float d[4];
        bspline_slopes(s - fl, d);
        const int col = (int)__umul24((uint32_t)(fb - sc.r_lo), (uint32_t)parzen_pitch(B)) + ((int32_t)fl - 1);
        const float fx = (float)x;
        // every group reads a table (groups past nqg repeat the last one and
        // are never written out), so no branch splits the groups' LDS reads
#pragma unroll
        for (int g = 0; g < NQG; ++g) {
          const float* Gr = lds_g + (g < nqg ? g : nqg - 1) * cells + col;
          // w(x) = -sum G beta3': subtracted below rather than negated
          const float w = Gr[0] * d[0] + Gr[1] * d[1] + Gr[2] * d[2] + Gr[3] * d[3];
          const float wx = w * fx;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            rs[g][r] = fmaf(-w, dv[r], rs[g][r]);
            rx[g][r] = fmaf(-wx, dv[r], rx[g][r]);
          }
        }
      };
      row_tiles(w, tmask, XT, lane, dx, band_groups, every, frow, row_ok, a.fnx,
                [&](const int64_t q[3], int32_t fbv, int32_t x) {
                  if (fbv >= sc.r_lo && fbv < sc.r_hi) differentiate(q, fbv, x);
                });
      // the row's sums into the gradient: along a lane's row only x varies,
      // so the j, k and constant columns take the plain sum times j, k, 1
#pragma unroll
      for (int g = 0; g < NQG; ++g)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          acc[g][4 * r] += rx[g][r];
          acc[g][4 * r + 1] = fmaf(rs[g][r], fj, acc[g][4 * r + 1]);
          acc[g][4 * r + 2] = fmaf(rs[g][r], fk, acc[g][4 * r + 2]);
          acc[g][4 * r + 3] += rs[g][r];
        }
    }
  }
  // workgroup sum in fp64: shuffle tree per wave, then waves in order
#pragma unroll
  for (int g = 0; g < NQG; ++g)
#pragma unroll
    for (int e = 0; e < 12; ++e) {
      double v = (double)acc[g][e];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) part[wave][g * 12 + e] = v;
    }
  __syncthreads();
  if (!ok || threadIdx.x >= nqg * 12) return;
  double sum = 0;
  for (int ww = 0; ww < NW; ++ww) sum += part[ww][threadIdx.x];
  const double N = (double)a.count[sc.t];
  if (N > 0 && sum != 0.0) {
    const int g = threadIdx.x / 12, e = threadIdx.x - g * 12;
    atomicAdd(&a.grad[((size_t)sc.t * a.n_q + a.q0 + g) * 12 + e], sum * a.dsdv / N);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <bool FQ, bool CLAMP, int NT>
static hipError_t fwd_variant(const ParzenArgs& a, size_t lds, hipStream_t s) {
  const hipError_t e = lds_guard((const void*)parzen_fwd_kernel<FQ, CLAMP, NT>, lds, kParzenLdsMax);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((parzen_fwd_kernel<FQ, CLAMP, NT>), dim3((unsigned)(a.n * a.chunks * a.bands)), dim3(NT),
                     lds, s, a);
  return hipGetLastError();
}

// The arguments of transforms [t0, t0 + n) of a batch: every per-transform
// array advanced to t0 (launches of whole transforms, transforms_per_launch).
static ParzenArgs sub_batch(const ParzenArgs& a, int32_t t0, int32_t n) {
  ParzenArgs b = a;
  const size_t BB = (size_t)a.bins * a.bins;
  b.n = n;
  b.transforms = a.transforms + 12 * (size_t)t0;
  if (a.table) b.table = a.table + (size_t)t0 * BB;
  if (a.count) b.count = a.count + t0;
  if (a.gtab) b.gtab = a.gtab + (size_t)t0 * a.n_q * BB;
  if (a.marg) b.marg = a.marg + (size_t)t0 * 2 * a.bins;
  if (a.grad) b.grad = a.grad + (size_t)t0 * a.n_q * 12;
  return b;
}

template <typename F>
static hipError_t in_launches(const ParzenArgs& a, int32_t block, F&& launch) {
  const int32_t step = transforms_per_launch((int64_t)a.chunks * a.bands, block);
  for (int32_t t0 = 0; t0 < a.n; t0 += step) {
    const hipError_t e = launch(sub_batch(a, t0, a.n - t0 < step ? a.n - t0 : step));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Calls f.template operator()<NT>() for the launch's workgroup size.
template <typename F>
static hipError_t by_block(int32_t block, F&& f) {
  switch (block) {
  case 256: return f.template operator()<256>();
  case 1024: return f.template operator()<1024>();
  default: return f.template operator()<512>();
  }
}

static int32_t block_of(const ParzenLaunch& L) {
  return (L.block == 256 || L.block == 1024) ? L.block : 512;
}

hipError_t launch_parzen_fwd(const ParzenLaunch& L, hipStream_t s) {
  const size_t lds = ((size_t)L.args.band_rows * parzen_pitch(L.args.bins) + parzen_hot_cells(L.args.bins)) * 8;
  return in_launches(L.args, block_of(L), [&](const ParzenArgs& a) {
    return by_block(L.block, [&]<int NT>() {
      if (L.float_quads)
        return L.clamp ? fwd_variant<true, true, NT>(a, lds, s) : fwd_variant<true, false, NT>(a, lds, s);
      return L.clamp ? fwd_variant<false, true, NT>(a, lds, s) : fwd_variant<false, false, NT>(a, lds, s);
    });
  });
}

template <bool FQ, bool CLAMP, int NT>
static hipError_t sampled_fwd_variant(const ParzenArgs& a, const uint2* list, const unsigned long long* n_list,
                                      size_t lds, hipStream_t s) {
  const hipError_t e = lds_guard((const void*)parzen_sampled_fwd_kernel<FQ, CLAMP, NT>, lds, kParzenLdsMax);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((parzen_sampled_fwd_kernel<FQ, CLAMP, NT>), dim3((unsigned)(a.n * a.chunks * a.bands)),
                     dim3(NT), lds, s, a, list, n_list);
  return hipGetLastError();
}

hipError_t launch_parzen_sampled_fwd(const ParzenLaunch& L, const uint2* list, const unsigned long long* n_list,
                                     hipStream_t s) {
  const size_t lds = ((size_t)L.args.band_rows * parzen_pitch(L.args.bins) + parzen_hot_cells(L.args.bins)) * 8;
  return in_launches(L.args, block_of(L), [&](const ParzenArgs& a) {
    return by_block(L.block, [&]<int NT>() {
      if (L.float_quads)
        return L.clamp ? sampled_fwd_variant<true, true, NT>(a, list, n_list, lds, s)
                       : sampled_fwd_variant<true, false, NT>(a, list, n_list, lds, s);
      return L.clamp ? sampled_fwd_variant<false, true, NT>(a, list, n_list, lds, s)
                     : sampled_fwd_variant<false, false, NT>(a, list, n_list, lds, s);
    });
  });
}

hipError_t launch_dmi_dp(const ParzenLaunch& L, const QList& q, hipStream_t s) {
  // sliced like the MI reduction of the whole batch, in launches of whole
  // transforms below 2^31 work-items each
  const int32_t S = reduce_splits(L.args.bins, L.args.n);
  const int32_t step = transforms_per_launch(S, 256);
  for (int32_t t0 = 0; t0 < L.args.n; t0 += step) {
    const ParzenArgs b = sub_batch(L.args, t0, L.args.n - t0 < step ? L.args.n - t0 : step);
    hipLaunchKernelGGL(dmi_dp_kernel, dim3((unsigned)((int64_t)b.n * S)), dim3(256), 0, s, b, q, S);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool FQ, bool CLAMP, int NT>
static hipError_t bwd_variant(const ParzenArgs& a, size_t lds, hipStream_t s) {
  const hipError_t e = lds_guard((const void*)parzen_bwd_kernel<FQ, CLAMP, 2, NT>, lds, kParzenLdsMax);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((parzen_bwd_kernel<FQ, CLAMP, 2, NT>), dim3((unsigned)(a.n * a.chunks * a.bands)), dim3(NT),
                     lds, s, a);
  return hipGetLastError();
}

hipError_t launch_parzen_bwd(const ParzenLaunch& L, hipStream_t s) {
  const size_t lds = (size_t)kParzenQGroup * L.args.band_rows * parzen_pitch(L.args.bins) * 4;
  return in_launches(L.args, block_of(L), [&](const ParzenArgs& a) {
    return by_block(L.block, [&]<int NT>() {
      if (L.float_quads)
        return L.clamp ? bwd_variant<true, true, NT>(a, lds, s) : bwd_variant<true, false, NT>(a, lds, s);
      return L.clamp ? bwd_variant<false, true, NT>(a, lds, s) : bwd_variant<false, false, NT>(a, lds, s);
    });
  });
}

// The bands are sized for at most kParzenLdsMax of dynamic LDS per
// workgroup.
template <bool FQ, bool CLAMP, int NT>
static hipError_t allow_lds_nt() {
  const int bytes = (int)kParzenLdsMax;
  const void* fns[3] = {(const void*)parzen_fwd_kernel<FQ, CLAMP, NT>,
                        (const void*)parzen_sampled_fwd_kernel<FQ, CLAMP, NT>,
                        (const void*)parzen_bwd_kernel<FQ, CLAMP, 2, NT>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess || (e = lds_register(f)) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool FQ, bool CLAMP>
static hipError_t allow_lds() {
  hipError_t e;
  if ((e = allow_lds_nt<FQ, CLAMP, 256>()) != hipSuccess) return e;
  if ((e = allow_lds_nt<FQ, CLAMP, 512>()) != hipSuccess) return e;
  return allow_lds_nt<FQ, CLAMP, 1024>();
}

hipError_t configure_parzen_kernels() {
  hipError_t e;
  if ((e = allow_lds<false, false>()) != hipSuccess) return e;
  if ((e = allow_lds<false, true>()) != hipSuccess) return e;
  if ((e = allow_lds<true, false>()) != hipSuccess) return e;
  return allow_lds<true, true>();
}

}  // namespace gemi
