// Hard-binned joint histogram of fixed vs. transformed moving volume
// (Transform + Metric blocks of Fig. 1; "full histogram over all voxels",
// Discussion), for gfx950.
//
// Per call, the fixed volume is reduced to one bin byte per voxel and the
// moving volume to a padded "pair volume": each element holds the clamped,
// offset intensities of a voxel and of its +x neighbour as two 16-bit
// halves, so the 2x2x2 trilinear neighbourhood is four aligned 32-bit
// loads, and one zero row per slice plus one zero slice make the +y/+z
// neighbours of the last row/slice addressable (their weight is 0).
//
// One workgroup = one transform x one slab of fixed rows.  Each wave64
// walks its own run of rows with scalar row coordinates; its 64 lanes take
// consecutive x (coalesced fixed-bin reads) and step the exact Q32 moving
// coordinate by 64 * M[:,0] per iteration.  Each lane forms the exact
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
// moving pair volume, once per call
// ---------------------------------------------------------------------------

// out[z][y][x] (z <= nz, y <= ny) = v'(x,y,z) | v'(min(x+1, nx-1),y,z) << 16
// with v' = clamp(v, lo, hi) - lo; zero on the padding row and slice.
template <typename T>
__global__ void pack_pairs_kernel(const T* __restrict__ v, int32_t nx, int32_t ny, int32_t nz,
                                  int32_t lo, int32_t hi, uint32_t* __restrict__ out) {
  const int32_t y = blockIdx.y, z = blockIdx.z;
  uint32_t* __restrict__ orow = out + ((size_t)z * (ny + 1) + y) * nx;
  if (y >= ny || z >= nz) {
    for (int32_t x = threadIdx.x; x < nx; x += blockDim.x) orow[x] = 0u;
    return;
  }
  const T* __restrict__ row = v + ((size_t)z * ny + y) * nx;
  for (int32_t x = threadIdx.x; x < nx; x += blockDim.x) {
    int32_t a = (int32_t)row[x];
    int32_t b = (int32_t)row[x + 1 < nx ? x + 1 : nx - 1];
    a = a < lo ? lo : (a > hi ? hi : a);
    b = b < lo ? lo : (b > hi ? hi : b);
    orow[x] = (uint32_t)(a - lo) | ((uint32_t)(b - lo) << 16);
  }
}

hipError_t launch_pack_pairs(const VolumeDesc& m, uint32_t* out, hipStream_t s) {
  const dim3 grid(1, (unsigned)m.ny + 1, (unsigned)m.nz + 1);
  const int32_t lo = (int32_t)m.lo, hi = (int32_t)m.hi;
  if (m.dtype == 0)
    hipLaunchKernelGGL(pack_pairs_kernel<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 1)
    hipLaunchKernelGGL(pack_pairs_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)m.data,
                       m.nx, m.ny, m.nz, lo, hi, out);
  else if (m.dtype == 2)
    hipLaunchKernelGGL(pack_pairs_kernel<int16_t>, grid, dim3(256), 0, s, (const int16_t*)m.data,
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
  const uint32_t* pairs;
  uint32_t* hist;
  int32_t fnx, fny, fnz;
  int32_t mnx, mny, mnz;
  uint32_t pair_bytes;
  int32_t bins, chunks;
  double scale;  // B / (R 2^48)
  Divider div;   // floor(X / R) for the exact fallback
};

typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));

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

template <bool CLAMP, bool PACKED, int NT>
__global__ __launch_bounds__(NT) void hist_hard_kernel(HardArgs a) {
  extern __shared__ uint32_t lds_hist[];
  const int B = a.bins;
  const int words = PACKED ? (B * B + 1) / 2 : B * B;
  for (int e = threadIdx.x; e < words; e += NT) lds_hist[e] = 0;

  uint32_t t, chunk;
  block_work(a.chunks, t, chunk);
  int64_t Mq[12];
  const bool ok = quantize_transform(a.transforms + 12 * (size_t)t, Mq);
  __syncthreads();
  if (ok) {
    constexpr int NW = NT / 64;
    const int64_t rows = (int64_t)a.fny * a.fnz;
    const int64_t r0 = rows * chunk / a.chunks, r1 = rows * (chunk + 1) / a.chunks;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t w0 = r0 + (r1 - r0) * wave / NW, w1 = r0 + (r1 - r0) * (wave + 1) / NW;
    int32_t k = (int32_t)(w0 / a.fny), j = (int32_t)(w0 - (int64_t)k * a.fny);
    // Q32 coordinate of voxel (0, j, k); per-row and per-slice-wrap deltas
    int64_t rx = Mq[1] * j + Mq[2] * k + Mq[3];
    int64_t ry = Mq[5] * j + Mq[6] * k + Mq[7];
    int64_t rz = Mq[9] * j + Mq[10] * k + Mq[11];
    const int64_t wrapx = Mq[2] - Mq[1] * a.fny, wrapy = Mq[6] - Mq[5] * a.fny,
                  wrapz = Mq[10] - Mq[9] * a.fny;
    const int64_t lx = Mq[0] * lane, ly = Mq[4] * lane, lz = Mq[8] * lane;
    const int64_t sx = Mq[0] * 64, sy = Mq[4] * 64, sz = Mq[8] * 64;
    const uint64_t topx = (uint64_t)(a.mnx - 1) << 32;
    const uint64_t topy = (uint64_t)(a.mny - 1) << 32;
    const uint64_t topz = (uint64_t)(a.mnz - 1) << 32;
    const uint32_t PY = (uint32_t)a.mny + 1, MX = (uint32_t)a.mnx;
    const int32_t SY = 4 * a.mnx, SZ = 4 * a.mnx * (a.mny + 1);
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.pairs, (short)0, (int)a.pair_bytes, 0x00020000);
    const uint32_t Bu = (uint32_t)B;
    const double scale = a.scale;

    for (int64_t r = w0; r < w1; ++r) {
      const uint8_t* __restrict__ frow = a.fbins + r * a.fnx;
      int64_t qx = rx + lx, qy = ry + ly, qz = rz + lz;
      for (int x = lane; x < a.fnx; x += 64, qx += sx, qy += sy, qz += sz) {
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
        // padded row index < 4096 * 4097 < 2^24, so 24-bit multiplies are exact
        const uint32_t off = (__umul24(__umul24(iz, PY) + iy, MX) + ix) * 4u;
        const uint32_t p00 = __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0);
        const uint32_t p10 = __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, SY, 0);
        const uint32_t p01 = __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, SZ, 0);
        const uint32_t p11 = __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, SY + SZ, 0);
        const uint32_t fb = frow[x];
        // (65535 - wx) in the low half, wx in the high half
        const uint32_t wpack = (fx & 0xFFFF0000u) | ((fx >> 16) ^ 0xFFFFu);
        const uint32_t a00 = lerp_x(p00, wpack), a10 = lerp_x(p10, wpack);
        const uint32_t a01 = lerp_x(p01, wpack), a11 = lerp_x(p11, wpack);
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
      // next row: (j+1, k), or (0, k+1) after the last row of a slice
      rx += Mq[1];
      ry += Mq[5];
      rz += Mq[9];
      if (++j == a.fny) {
        j = 0;
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
  a.pairs = L.pairs;
  a.hist = L.hist;
  a.fnx = L.fixed.nx;
  a.fny = L.fixed.ny;
  a.fnz = L.fixed.nz;
  a.mnx = L.moving.nx;
  a.mny = L.moving.ny;
  a.mnz = L.moving.nz;
  a.pair_bytes = (uint32_t)((size_t)L.moving.nx * (L.moving.ny + 1) * (L.moving.nz + 1) * 4);
  a.bins = L.bins;
  a.chunks = L.chunks;
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
