// Hard-binned MI of many fixed/moving pairs of uneven sizes, each with its
// own transforms, in one persistent launch (the batched evaluation behind
// the exhaustive per-family sweeps of the Methodology, for many volumes).
//
// Work items are (pair, slab, transform) triples.  Each pair's slabs are
// split into 8 equal shares, one per XCD, and every XCD has its own work
// queue: a workgroup (resident for the whole launch) repeatedly takes the
// next item of its XCD's queue with one atomic, sweeps that slab for that
// transform into its LDS histogram, adds the histogram into the
// transform's HBM histogram and clears it.  Items are ordered pair-major,
// then slab-major, so the workgroups of an XCD work on one slab of one pair
// at a time and share its moving footprint in L2.  Every workgroup leaves
// the loop once its queue is empty, so the grid always drains.
//
// Per-pair fixed bins and moving oct volumes are prepared by two kernels
// over 256-voxel chunks of all pairs, and the transforms are gathered into
// one array for the MI reduction.
#include "common.h"
#include "sweep.h"

namespace gemi {

// Largest p with base[p] <= v, for base[0] = 0 <= v < base[P].
__device__ __forceinline__ int find_pair(const int64_t* __restrict__ base, int P, int64_t v) {
  int lo = 0, hi = P;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= v)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Device-memory views: the pairs' volume pointers are read from the pair
// table, so without the address space the compiler would use flat accesses.
typedef const __attribute__((address_space(1))) uint16_t global_u16;
typedef const __attribute__((address_space(1))) int16_t global_i16;
typedef const __attribute__((address_space(1))) uint32_t global_cu32;
typedef const __attribute__((address_space(1))) float global_f32;
typedef __attribute__((address_space(1))) uint8_t global_out8;
typedef __attribute__((address_space(1))) uint32_t global_out32;
typedef __attribute__((address_space(1))) uint2_t global_out2;
typedef __attribute__((address_space(1))) uint4_t global_out4;

__device__ __forceinline__ int32_t load_int(const void* p, int32_t dtype, size_t i) {
  switch (dtype) {
  case 0: return ((global_u8*)p)[i];
  case 1: return ((global_u16*)p)[i];
  default: return ((global_i16*)p)[i];
  }
}

__global__ void gather_transforms_kernel(PairsArgs a, int64_t total) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int p = find_pair(a.t_base, a.n_pairs, g);
    const double* src = a.pairs[p].transforms + 12 * (g - a.t_base[p]);
    for (int e = 0; e < 12; ++e) a.transforms[12 * g + e] = src[e];
  }
}

// A value every lane holds alike, moved to scalar registers.  The work item
// reaches the workgroup through LDS, so the compiler cannot tell that what is
// derived from it is uniform: without the broadcast the pair's geometry stays
// in vector registers, is reloaded inside the sweep, and each gather from the
// moving volume runs a loop over the distinct buffer descriptors of the wave.
template <typename T>
__device__ __forceinline__ T uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "32-bit words");
  uint32_t w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Calls f(p, item, lane) for the items of the concatenated item space
// [base[0], base[P]) that fall to this workgroup: a contiguous range per
// workgroup, one wave per item.  The pair is found once per wave and then
// advanced as the items ascend (a search per item would serialise dependent
// loads on every item of small volumes).
template <typename F>
__device__ __forceinline__ void for_each_item(const int64_t* __restrict__ base, int P, int64_t items,
                                              F&& f) {
  const int64_t per = (items + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < items ? r0 + per : items;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  if (r0 + wave >= r1) return;
  int p = uniform(find_pair(base, P, r0 + wave));
  for (int64_t r = r0 + wave; r < r1; r += nw) {
    while (r >= uniform(base[p + 1])) ++p;
    f(p, r - uniform(base[p]), lane);
  }
}

// Fixed bins of every pair, one wave per chunk of kPrepChunk consecutive
// voxels (four per lane) of a pair's fixed volume: every lane busy whatever
// the row length.
__global__ void prep_fixed_kernel(PairsArgs a, int64_t chunks) {
  for_each_item(a.fchunk_base, a.n_pairs, chunks, [&](int p, int64_t c, int lane) {
    const PairDesc d = uniform(a.pairs[p]);
    const int64_t nvox = (int64_t)d.geom.fnx * d.geom.fny * d.geom.fnz;
    const int64_t v0 = c * kPrepChunk + 4 * lane;
    if (v0 >= nvox) return;
    global_out8* __restrict__ out = (global_out8*)d.geom.fbins;
    if (d.fdtype == 0 && v0 + 4 <= nvox && ((uintptr_t)d.fixed & 3) == 0) {
      // u8, 4-byte aligned volume: one 32-bit load and store for four voxels
      // (the bins start 256-byte aligned and v0 is a multiple of 4)
      const uint32_t w = *(global_cu32*)((global_u8*)d.fixed + v0);
      uint32_t o = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        o |= fixed_bin_int((int32_t)((w >> (8 * k)) & 0xFFu), (int32_t)d.flo, (int32_t)d.fhi,
                           (uint32_t)d.geom.bins, d.fdiv) << (8 * k);
      *(global_out32*)(out + v0) = o;
      return;
    }
    for (int64_t v = v0; v < v0 + 4 && v < nvox; ++v) {
      uint32_t b;
      if (d.fdtype == 3)
        b = fixed_bin_real((double)((global_f32*)d.fixed)[v], d.flo, d.fhi, d.geom.bins);
      else
        b = fixed_bin_int(load_int(d.fixed, d.fdtype, v), (int32_t)d.flo, (int32_t)d.fhi,
                          (uint32_t)d.geom.bins, d.fdiv);
      out[v] = (uint8_t)b;
    }
  });
}

// Moving oct volumes of every pair, one wave per chunk of kPrepChunk
// consecutive voxels (four per lane), with the layout and clamping of the
// single-pair path.
__global__ void prep_moving_kernel(PairsArgs a, int64_t chunks) {
  for_each_item(a.mchunk_base, a.n_pairs, chunks, [&](int p, int64_t c, int lane) {
    const PairDesc d = uniform(a.pairs[p]);
    const int32_t nx = d.geom.mnx, ny = d.geom.mny, nz = d.geom.mnz;
    const uint32_t nvox = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;  // < 2^28
    const uint32_t v0 = (uint32_t)(c * kPrepChunk) + 4u * (uint32_t)lane;
    if (v0 >= nvox) return;
    auto v = [&](size_t i) -> uint32_t { return clamp_offset(load_int(d.moving, d.mdtype, i), d.mlo, d.mhi); };
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    if (d.geom.oct8 && d.mdtype == 0 && (nx & 3) == 0 && ((uintptr_t)d.moving & 3) == 0) {
      // u8 rows of a multiple of 4 voxels, 4-byte aligned volume: the lane's
      // four voxels share a row; each source row is read as one dword plus
      // its next (clamped) byte
      const uint32_t row = v0 / (uint32_t)nx, x0 = v0 - row * (uint32_t)nx;
      const uint32_t z = row / (uint32_t)ny, y = row - z * (uint32_t)ny;
      const size_t r00 = (size_t)row * nx;
      const size_t r10 = r00 + (y + 1 < (uint32_t)ny ? nx : 0);
      const size_t dz = z + 1 < (uint32_t)nz ? plane : 0;
      global_u8* __restrict__ mv = (global_u8*)d.moving;
      const size_t src[4] = {r00, r10, r00 + dz, r10 + dz};
      const uint32_t xn = x0 + 4 < (uint32_t)nx ? x0 + 4 : (uint32_t)nx - 1;
      uint32_t b[4][5];  // b[row][i] = clamped, offset value at x0 + i (i = 4: the neighbour)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t w = *(global_cu32*)(mv + src[r] + x0);
#pragma unroll
        for (int i = 0; i < 4; ++i) b[r][i] = clamp_offset((int32_t)((w >> (8 * i)) & 0xFFu), d.mlo, d.mhi);
        b[r][4] = clamp_offset((int32_t)mv[src[r] + xn], d.mlo, d.mhi);
      }
      uint32_t o[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        o[2 * i] = b[0][i] | (b[0][i + 1] << 8) | (b[1][i] << 16) | (b[1][i + 1] << 24);
        o[2 * i + 1] = b[2][i] | (b[2][i + 1] << 8) | (b[3][i] << 16) | (b[3][i + 1] << 24);
      }
      global_out4* __restrict__ out = (global_out4*)((global_out2*)d.geom.octs + v0);
      out[0] = uint4_t{o[0], o[1], o[2], o[3]};
      out[1] = uint4_t{o[4], o[5], o[6], o[7]};
      return;
    }
    for (uint32_t vx = v0; vx < v0 + 4 && vx < nvox; ++vx) {
      const uint32_t row = vx / (uint32_t)nx, x = vx - row * (uint32_t)nx;
      const uint32_t z = row / (uint32_t)ny, y = row - z * (uint32_t)ny;
      const size_t r00 = (size_t)row * nx;
      const size_t r10 = r00 + (y + 1 < (uint32_t)ny ? nx : 0);
      const size_t dz = z + 1 < (uint32_t)nz ? plane : 0;
      const uint32_t x1 = x + 1 < (uint32_t)nx ? x + 1 : (uint32_t)nx - 1;
      if (d.geom.oct8) {
        // 8-bit corners: byte 4 dz + 2 dy + dx' (layout of pack_oct8_kernel)
        ((global_out2*)d.geom.octs)[vx] =
            uint2_t{v(r00 + x) | (v(r00 + x1) << 8) | (v(r10 + x) << 16) | (v(r10 + x1) << 24),
                    v(r00 + dz + x) | (v(r00 + dz + x1) << 8) | (v(r10 + dz + x) << 16) |
                        (v(r10 + dz + x1) << 24)};
      } else {
        ((global_out4*)d.geom.octs)[vx] =
            uint4_t{v(r00 + x) | (v(r00 + x1) << 16), v(r10 + x) | (v(r10 + x1) << 16),
                    v(r00 + dz + x) | (v(r00 + dz + x1) << 16), v(r10 + dz + x) | (v(r10 + dz + x1) << 16)};
      }
    }
  });
}

template <bool CLAMP, bool PACKED, bool OCT8, int NT>
__global__ __launch_bounds__(NT) void hist_pairs_kernel(PairsArgs a) {
  extern __shared__ uint32_t lds_hist[];
  __shared__ int64_t item_sh;
  const int B = a.bins;
  const int words = PACKED ? (B * B + 1) / 2 : B * B;
  for (int e = threadIdx.x; e < words; e += NT) lds_hist[e] = 0;
  const uint32_t xcd = blockIdx.x & 7u;
  const int64_t* __restrict__ xbase = a.xcd_base + (int64_t)xcd * (a.n_pairs + 1);
  const int64_t total = xbase[a.n_pairs];
  for (;;) {
    if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(&a.counters[xcd], 1ull);
    __syncthreads();
    const int64_t item = uniform(item_sh);
    if (item >= total) break;  // the same for every thread of the workgroup
    const int p = find_pair(xbase, a.n_pairs, item);
    const HardGeom geom = uniform(a.pairs[p].geom);
    const int32_t n_t = uniform(a.pairs[p].n_t), chunks = uniform(a.pairs[p].chunks);
    const int64_t rem = item - xbase[p];
    const int64_t slab = rem / n_t, tl = rem - slab * n_t;
    const uint32_t chunk = xcd * (uint32_t)(chunks >> 3) + (uint32_t)slab;
    const int64_t t = uniform(a.t_base[p]) + tl;
    int64_t Mq[12];
    const bool ok = quantize_transform(a.transforms + 12 * t, Mq);
    if (ok) sweep_hard<CLAMP, PACKED, OCT8, NT / 64>(geom, Mq, chunks, chunk, lds_hist);
    __syncthreads();
    if (ok) flush_hist<PACKED, NT>(lds_hist, B, a.hist + (size_t)t * B * B, true);
    __syncthreads();
  }
}

// Workgroups (4 waves each) for a preparation kernel: a few per CU, fewer
// for small item counts.
static unsigned row_grid(int64_t rows) {
  const int64_t g = (rows + 3) / 4;
  return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

hipError_t launch_pairs_prep(const PairsLaunch& L, hipStream_t s) {
  if (L.total_t > 0) {
    const int64_t blocks = (L.total_t + 255) / 256;
    hipLaunchKernelGGL(gather_transforms_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)),
                       dim3(256), 0, s, L.args, L.total_t);
  }
  if (L.fixed_chunks > 0)
    hipLaunchKernelGGL(prep_fixed_kernel, dim3(row_grid(L.fixed_chunks)), dim3(256), 0, s, L.args,
                       L.fixed_chunks);
  if (L.moving_chunks > 0)
    hipLaunchKernelGGL(prep_moving_kernel, dim3(row_grid(L.moving_chunks)), dim3(256), 0, s, L.args,
                       L.moving_chunks);
  return hipGetLastError();
}

constexpr int kPairsBlock = 512;

template <bool CLAMP, bool PACKED, bool OCT8>
static hipError_t pairs_variant(const PairsLaunch& L, hipStream_t s) {
  const int B = L.args.bins;
  const size_t lds = PACKED ? (((size_t)B * B + 1) / 2) * 4 : (size_t)B * B * 4;
  if (lds > 150 * 1024) return hipErrorInvalidValue;  // the limit set below
  const void* fn = (const void*)hist_pairs_kernel<CLAMP, PACKED, OCT8, kPairsBlock>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPairsBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  // every queue needs workgroups: a multiple of 8 (one share per XCD)
  const unsigned grid = (unsigned)(((per_cu * L.cu_count + 7) / 8) * 8);
  hipLaunchKernelGGL((hist_pairs_kernel<CLAMP, PACKED, OCT8, kPairsBlock>), dim3(grid), dim3(kPairsBlock),
                     lds, s, L.args);
  return hipGetLastError();
}

template <bool OCT8>
static hipError_t pairs_layout(const PairsLaunch& L, hipStream_t s) {
  if (L.clamp)
    return L.packed ? pairs_variant<true, true, OCT8>(L, s) : pairs_variant<true, false, OCT8>(L, s);
  return L.packed ? pairs_variant<false, true, OCT8>(L, s) : pairs_variant<false, false, OCT8>(L, s);
}

hipError_t launch_pairs_hist(const PairsLaunch& L, hipStream_t s) {
  return L.oct8 ? pairs_layout<true>(L, s) : pairs_layout<false>(L, s);
}

}  // namespace gemi
