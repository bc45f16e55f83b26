// Hard-binned joint histogram of fixed vs. transformed moving volume
// (Transform + Metric blocks of Fig. 1; "full histogram over all voxels",
// Discussion), for gfx950.
//
// Per call, the fixed volume is reduced to one bin byte per voxel and the
// moving volume to a "quad volume": each 8-byte element holds the clamped,
// offset intensities of a voxel and of its +x, +y and +x+y neighbours as
// 16-bit values, so the 2x2x2 trilinear neighbourhood is two aligned
// 64-bit loads; one zero slice makes the +z neighbours of the last slice
// addressable (their weight is 0).
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

#pragma clang fp contract(off)

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
// moving quad volume, once per call
// ---------------------------------------------------------------------------

// out[z][y][x] (z <= nz) holds four 16-bit clamped, offset intensities
// v' = clamp(v, lo, hi) - lo: (x, y), (x1, y) in .x and (x, y+1), (x1, y+1)
// in .y, with x1 = min(x+1, nx-1).  On the last row the y+1 values are 0
// and slice nz is all 0: those corners always carry weight 0.
template <typename T>
__global__ void pack_quads_kernel(const T* __restrict__ v, int32_t nx, int32_t ny, int32_t nz,
                                  int32_t lo, int32_t hi, uint2* __restrict__ out) {
  const int32_t y = blockIdx.y, z = blockIdx.z;
  uint2* __restrict__ orow = out + ((size_t)z * ny + y) * nx;
  if (z >= nz) {
    for (int32_t x = threadIdx.x; x < nx; x += blockDim.x) orow[x] = make_uint2(0u, 0u);
    return;
  }
  const T* __restrict__ r0 = v + ((size_t)z * ny + y) * nx;
  const bool has1 = y + 1 < ny;
  const T* __restrict__ r1 = r0 + (has1 ? nx : 0);
  auto c = [&](T raw) -> uint32_t {
    int32_t a = (int32_t)raw;
    a = a < lo ? lo : (a > hi ? hi : a);
    return (uint32_t)(a - lo);
  };
  for (int32_t x = threadIdx.x; x < nx; x += blockDim.x) {
    const int32_t x1 = x + 1 < nx ? x + 1 : nx - 1;
    const uint32_t lo_pair = c(r0[x]) | (c(r0[x1]) << 16);
    const uint32_t hi_pair = has1 ? (c(r1[x]) | (c(r1[x1]) << 16)) : 0u;
    orow[x] = make_uint2(lo_pair, hi_pair);
  }
}

hipError_t launch_pack_quads(const VolumeDesc& m, uint2* out, hipStream_t s) {
  const dim3 grid(1, (unsigned)m.ny, (unsigned)m.nz + 1);
  const int32_t lo = (int32_t)m.lo, hi = (int32_t)m.hi;
  if (m.dtype == 0)
    hipLaunchKernelGGL(pack_quads_kernel<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 1)
    hipLaunchKernelGGL(pack_quads_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 2)
    hipLaunchKernelGGL(pack_quads_kernel<int16_t>, grid, dim3(256), 0, s, (const int16_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the histogram sweep
// ---------------------------------------------------------------------------

struct HardArgs {
  const double* transforms;
  const uint8_t* fbins;
  const uint2* quads;
  uint32_t* hist;
  int32_t fnx, fny, fnz;
  int32_t mnx, mny, mnz;
  uint32_t quad_bytes;
  int32_t n, bins, chunks;
  int32_t slab_major;  // 1: consecutive workgroups of an XCD share a slab
  double scale;  // B / (R 2^48)
  Divider div;   // floor(X / R) for the exact fallback
};

typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));
typedef unsigned int uint2_t __attribute__((ext_vector_type(2)));

// Maps workgroup id -> (transform, slab).  Workgroups are dealt round-robin
// to the 8 XCDs, so XCD x receives ids x, x+8, ...; those all take slabs
// from the x-th eighth of the fixed volume.  Slab-major order then walks
// that eighth one thin slab at a time, all transforms per slab, so the
// workgroups resident on an XCD at once share one slab's moving footprint
// in that XCD's L2; transform-major order finishes a transform's slabs
// before the next transform.
__device__ __forceinline__ void block_work(int32_t chunks, int32_t n, int32_t slab_major,
                                           uint32_t& t, uint32_t& chunk) {
  const uint32_t bid = blockIdx.x;
  const uint32_t xcd = bid & 7u, slot = bid >> 3;
  const uint32_t c8 = (uint32_t)chunks >> 3;
  if (slab_major) {
    const uint32_t cl = slot / (uint32_t)n;
    t = slot - cl * (uint32_t)n;
    chunk = xcd * c8 + cl;
  } else {
    t = slot / c8;
    chunk = xcd * c8 + (slot - t * c8);
  }
}

// v0 (1 - w) + v1 w at 16-bit weight w = fx >> 16, exact: the pair's low
// half times (65535 - w), high half times w, plus the low half once more.
__device__ __forceinline__ uint32_t lerp_x(uint32_t pair, uint32_t wpack) {
  return __builtin_amdgcn_udot2(__builtin_bit_cast(ushort2_t, pair),
                                __builtin_bit_cast(ushort2_t, wpack), pair & 0xFFFFu, false);
}

// Exact bin of V = sum over corners, from the four exact x-lerps.
__device__ __noinline__ uint32_t exact_bin(uint32_t a00, uint32_t a10, uint32_t a01, uint32_t a11,
                                           uint32_t wy, uint32_t wz, uint32_t B, Divider div) {
  const uint64_t b0 = (uint64_t)a00 * (65536u - wy) + (uint64_t)a10 * wy;
  const uint64_t b1 = (uint64_t)a01 * (65536u - wy) + (uint64_t)a11 * wy;
  const uint64_t V = b0 * (65536u - wz) + b1 * wz;
  // floor(V B / (R 2^48)) = floor(X / R), X = floor(V B / 2^48) < 2^24
  const uint32_t X = (uint32_t)(V >> 48) * B + (uint32_t)(((V & 0xFFFFFFFFFFFFull) * B) >> 48);
  return div_small(X, div);
}

constexpr double kEdge = 1.0 / 536870912.0;  // 2^-29
constexpr int kTileX = 16, kTileY = 4;       // a wave64 sweeps 16 x 4 fixed voxels at a time

template <bool CLAMP, bool PACKED, int NT>
__global__ __launch_bounds__(NT) void hist_hard_kernel(HardArgs a) {
  extern __shared__ uint32_t lds_hist[];
  const int B = a.bins;
  const int words = PACKED ? (B * B + 1) / 2 : B * B;
  for (int e = threadIdx.x; e < words; e += NT) lds_hist[e] = 0;

  uint32_t t, chunk;
  block_work(a.chunks, a.n, a.slab_major, t, chunk);
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)t, Mq);
  __syncthreads();
  if (ok) {
    constexpr int NW = NT / 64;
    // the fixed volume as groups of kTileY consecutive rows of one slice
    const int32_t G = (a.fny + kTileY - 1) / kTileY;
    const int64_t groups = (int64_t)G * a.fnz;
    const int64_t g0 = groups * chunk / a.chunks, g1 = groups * (chunk + 1) / a.chunks;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int dx = lane & (kTileX - 1), dy = lane / kTileX;
    const int64_t w0 = g0 + (g1 - g0) * wave / NW, w1 = g0 + (g1 - g0) * (wave + 1) / NW;
    int32_t k = (int32_t)(w0 / G);
    int32_t j0 = (int32_t)(w0 - (int64_t)k * G) * kTileY;
    // Q32 coordinate of voxel (0, j0, k); per-group and slice-wrap deltas
    int64_t rx = Mq[1] * j0 + Mq[2] * k + Mq[3];
    int64_t ry = Mq[5] * j0 + Mq[6] * k + Mq[7];
    int64_t rz = Mq[9] * j0 + Mq[10] * k + Mq[11];
    const int64_t wrapx = Mq[2] - Mq[1] * ((int64_t)G * kTileY);
    const int64_t wrapy = Mq[6] - Mq[5] * ((int64_t)G * kTileY);
    const int64_t wrapz = Mq[10] - Mq[9] * ((int64_t)G * kTileY);
    const int64_t lx = Mq[0] * dx + Mq[1] * dy, ly = Mq[4] * dx + Mq[5] * dy,
                  lz = Mq[8] * dx + Mq[9] * dy;
    const int64_t sx = Mq[0] * kTileX, sy = Mq[4] * kTileX, sz = Mq[8] * kTileX;
    const uint64_t topx = (uint64_t)(a.mnx - 1) << 32;
    const uint64_t topy = (uint64_t)(a.mny - 1) << 32;
    const uint64_t topz = (uint64_t)(a.mnz - 1) << 32;
    const uint32_t NY = (uint32_t)a.mny, MX = (uint32_t)a.mnx;
    const int32_t SZ = 8 * a.mnx * a.mny;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.quads, (short)0, (int)a.quad_bytes, 0x00020000);
    const uint32_t Bu = (uint32_t)B;
    const double scale = a.scale;

    for (int64_t g = w0; g < w1; ++g) {
      const int32_t j = j0 + dy;
      if (j < a.fny) {
        const uint8_t* __restrict__ frow = a.fbins + ((int64_t)k * a.fny + j) * a.fnx;
        int64_t qx = rx + lx, qy = ry + ly, qz = rz + lz;
        for (int x = dx; x < a.fnx; x += kTileX, qx += sx, qy += sy, qz += sz) {
          uint64_t cx = (uint64_t)qx, cy = (uint64_t)qy, cz = (uint64_t)qz;
          if (CLAMP) {
            cx = qx < 0 ? 0 : (cx > topx ? topx : cx);
            cy = qy < 0 ? 0 : (cy > topy ? topy : cy);
            cz = qz < 0 ? 0 : (cz > topz ? topz : cz);
          } else {
            // 0 <= q <= top; a negative q wraps to a huge unsigned value
            if (cx > topx || cy > topy || cz > topz) continue;
          }
          const uint32_t ix = (uint32_t)(cx >> 32), iy = (uint32_t)(cy >> 32), iz = (uint32_t)(cz >> 32);
          const uint32_t fx = (uint32_t)cx, fy = (uint32_t)cy, fz = (uint32_t)cz;
          // (nz+1) * ny < 2^24 rows, so 24-bit multiplies are exact
          const uint32_t off = (__umul24(__umul24(iz, NY) + iy, MX) + ix) * 8u;
          const uint2_t q0 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0);
          const uint2_t q1 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, SZ, 0);
          const uint32_t fb = frow[x];
          // (65535 - wx) in the low half, wx in the high half
          const uint32_t wpack = (fx & 0xFFFF0000u) | ((fx >> 16) ^ 0xFFFFu);
          const uint32_t a00 = lerp_x(q0.x, wpack), a10 = lerp_x(q0.y, wpack);
          const uint32_t a01 = lerp_x(q1.x, wpack), a11 = lerp_x(q1.y, wpack);
          const uint32_t wy = fy >> 16, wz = fz >> 16;
          const double wyd = (double)wy, wzd = (double)wz;
          const double A00 = (double)a00, A10 = (double)a10, A01 = (double)a01, A11 = (double)a11;
          const double b0 = fma(A10 - A00, wyd, A00 * 65536.0);  // exact, < 2^48
          const double b1 = fma(A11 - A01, wyd, A01 * 65536.0);  // exact, < 2^48
          const double V = fma(b1 - b0, wzd, b0 * 65536.0);      // exact value rounded once
          const double tb = V * scale;
          uint32_t bm = (uint32_t)tb;
          const double fr = tb - (double)bm;
          if (fr < kEdge || fr > 1.0 - kEdge) bm = exact_bin(a00, a10, a01, a11, wy, wz, Bu, a.div);
          const uint32_t cell = __umul24(fb, Bu) + bm;
          if (PACKED)
            atomicAdd(&lds_hist[cell >> 1], 1u << ((cell & 1u) * 16u));
          else
            atomicAdd(&lds_hist[cell], 1u);
        }
      }
      // next group: rows j0+kTileY.., or the first group of the next slice
      j0 += kTileY;
      rx += Mq[1] * kTileY;
      ry += Mq[5] * kTileY;
      rz += Mq[9] * kTileY;
      if (j0 >= G * kTileY) {
        j0 = 0;
        ++k;
        rx += wrapx;
        ry += wrapy;
        rz += wrapz;
      }
    }
  }
  __syncthreads();
  if (!ok) return;
  uint32_t* __restrict__ out = a.hist + (size_t)t * B * B;
  for (int e = threadIdx.x; e < words; e += NT) {
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

template <bool CLAMP, bool PACKED, int NT>
static hipError_t launch_variant(const HardArgs& a, int n, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((hist_hard_kernel<CLAMP, PACKED, NT>), dim3((unsigned)(n * a.chunks)),
                     dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <int NT>
static hipError_t launch_nt(const HardArgs& a, int n, bool clamp, bool packed, size_t lds,
                            hipStream_t s) {
  if (clamp)
    return packed ? launch_variant<true, true, NT>(a, n, lds, s) : launch_variant<true, false, NT>(a, n, lds, s);
  return packed ? launch_variant<false, true, NT>(a, n, lds, s) : launch_variant<false, false, NT>(a, n, lds, s);
}

hipError_t launch_hist_hard(const HardLaunch& L, hipStream_t s) {
  if (L.n == 0) return hipSuccess;
  HardArgs a;
  a.transforms = L.transforms;
  a.fbins = L.fbins;
  a.quads = L.quads;
  a.hist = L.hist;
  a.fnx = L.fixed.nx;
  a.fny = L.fixed.ny;
  a.fnz = L.fixed.nz;
  a.mnx = L.moving.nx;
  a.mny = L.moving.ny;
  a.mnz = L.moving.nz;
  a.quad_bytes = (uint32_t)quad_volume_bytes(L.moving.nx, L.moving.ny, L.moving.nz);
  a.n = L.n;
  a.bins = L.bins;
  a.chunks = L.chunks;
  a.slab_major = L.slab_major;
  const uint32_t R = (uint32_t)((int32_t)L.moving.hi - (int32_t)L.moving.lo + 1);
  a.scale = ldexp((double)L.bins / (double)R, -48);
  a.div = make_divider(R);
  const size_t lds = L.packed ? (((size_t)L.bins * L.bins + 1) / 2) * 4 : (size_t)L.bins * L.bins * 4;
  switch (L.block) {
  case 256: return launch_nt<256>(a, L.n, L.clamp, L.packed, lds, s);
  case 512: return launch_nt<512>(a, L.n, L.clamp, L.packed, lds, s);
  case 1024: return launch_nt<1024>(a, L.n, L.clamp, L.packed, lds, s);
  default: return hipErrorInvalidValue;
  }
}

template <int NT>
static hipError_t allow_big_lds() {
  const int bytes = 160 * 1024;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)hist_hard_kernel<false, false, NT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)hist_hard_kernel<true, false, NT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)hist_hard_kernel<false, true, NT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)hist_hard_kernel<true, true, NT>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t configure_hard_kernels() {
  hipError_t e;
  if ((e = allow_big_lds<256>()) != hipSuccess) return e;
  if ((e = allow_big_lds<512>()) != hipSuccess) return e;
  return allow_big_lds<1024>();
}

}  // namespace gemi
