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
// at a time and share its moving footprint in L2.  A slab is a brick of
// whole x rows (GroupWalkBrick): the footprints of a pair's transforms on a
// compact brick overlap more than on a thin slab of whole slices, whose
// rotated images spread over many moving slices (16 rigid transforms of
// +-10 degrees: 23.1 -> 21.8 ms, the L2 misses being the sweep's limit).
// Every workgroup leaves the loop once its queue is empty, so the grid
// always drains.
//
// Per-pair fixed bins and moving oct volumes are prepared by two kernels
// over the items of all pairs (runs of 1024 consecutive fixed voxels; runs
// of 128 voxels of a moving xy plane through 8 slices), one wave per item,
// and the transforms are gathered into one array for the MI reduction.
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
typedef const __attribute__((address_space(1))) uint4_t global_cu4;
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
    double M[12];
    compose_index_matrix(src, a.pairs[p].geo, M);
    for (int e = 0; e < 12; ++e) a.transforms[12 * g + e] = M[e];
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

// Calls f(d, item, lane) for the items of the concatenated item space
// [base[0], base[P]) that fall to this workgroup, d being the descriptor of
// the item's pair and item its index within the pair: a contiguous range
// per workgroup, one wave per item.  The pair is found once per wave and
// then advanced as the items ascend; its bounds and descriptor are loaded
// again only when it changes (they come through vector loads, so a load
// per item would put two dependent round trips before every item's data).
template <typename F>
__device__ __forceinline__ void for_each_item(const PairDesc* __restrict__ pairs,
                                              const int64_t* __restrict__ base, int P, int64_t items,
                                              F&& f) {
  const int64_t per = (items + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < items ? r0 + per : items;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  if (r0 + wave >= r1) return;
  int p = uniform(find_pair(base, P, r0 + wave));
  int64_t lo = uniform(base[p]), hi = uniform(base[p + 1]);
  PairDesc d = uniform(pairs[p]);
  for (int64_t r = r0 + wave; r < r1; r += nw) {
    if (r >= hi) {
      do {
        ++p;
        lo = hi;
        hi = uniform(base[p + 1]);
      } while (r >= hi);
      d = uniform(pairs[p]);
    }
    f(d, r - lo, lane);
  }
}

// Fixed bins of every pair, one wave per chunk of kPrepFixedChunk
// consecutive voxels of a pair's fixed volume: every lane busy whatever the
// row length.  Full chunks of a u8 volume are read and their bins written in
// 16-byte accesses, 16 voxels per lane (with four bytes per lane the pass
// waited on one short load per wave at a time); otherwise lane l takes
// voxels l, l + 64, ..., so each access of the wave covers consecutive
// voxels.
__global__ void prep_fixed_kernel(PairsArgs a, int64_t chunks) {
  for_each_item(a.pairs, a.fchunk_base, a.n_pairs, chunks, [&](const PairDesc& d, int64_t c, int lane) {
    const int64_t nvox = (int64_t)d.geom.fnx * d.geom.fny * d.geom.fnz;
    const int64_t c0 = c * kPrepFixedChunk;
    global_out8* __restrict__ out = (global_out8*)d.geom.fbins;
    // the form is chosen for the whole chunk (a full chunk of an aligned u8
    // volume, or not), so every voxel of it is written once
    if (d.fdtype == 0 && c0 + kPrepFixedChunk <= nvox && (((uintptr_t)d.fixed | (uintptr_t)out) & 15) == 0) {
      const int64_t v0 = c0 + kPrepFixedLane * lane;  // a multiple of 16: 16-byte aligned accesses
      const uint4_t w = *(global_cu4*)((global_u8*)d.fixed + v0);
      uint4_t o;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t bj = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          bj |= fixed_bin_int((int32_t)((w[j] >> (8 * k)) & 0xFFu), (int32_t)d.flo, (int32_t)d.fhi,
                              (uint32_t)d.geom.bins, d.fdiv) << (8 * k);
        o[j] = bj;
      }
      *(global_out4*)(out + v0) = o;
      return;
    }
    for (int k = 0; k < kPrepFixedLane; ++k) {
      const int64_t v = c0 + lane + 64 * k;
      if (v >= nvox) break;
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

// Moving oct volumes of every pair, with the layout and clamping of the
// single-pair path.  An item is a run of kPrepPlaneRun voxels of an xy
// plane through a block of kPrepSlices consecutive slices: lane l takes
// plane voxels 2l and 2l + 1 of the run at every slice of the block.  The
// lane loads the source rows y and y + 1 of each slice of the block and of
// the one after it once, all before its first store, and the entries of
// slice z take slice z + 1's rows from registers; so a source row is
// fetched once per block instead of once for its own slice and again for
// the slice below (with flat chunks the moving preparation fetched 2.5x
// its source volume).  Each 16-byte store of the wave covers consecutive
// entries.
__global__ void prep_moving_kernel(PairsArgs a, int64_t items) {
  for_each_item(a.pairs, a.mchunk_base, a.n_pairs, items, [&](const PairDesc& d, int64_t c, int lane) {
    const uint32_t nx = (uint32_t)d.geom.mnx, ny = (uint32_t)d.geom.mny, nz = (uint32_t)d.geom.mnz;
    const uint32_t plane = nx * ny;  // nvox < 2^28
    const uint32_t runs = (plane + kPrepPlaneRun - 1) / kPrepPlaneRun;
    const uint32_t zb = (uint32_t)c / runs, run = (uint32_t)c - zb * runs;
    const uint32_t z0 = zb * kPrepSlices;
    const uint32_t nzb = nz - z0 < (uint32_t)kPrepSlices ? nz - z0 : (uint32_t)kPrepSlices;  // slices in the block
    const uint32_t vp = run * kPrepPlaneRun + 2u * (uint32_t)lane;  // plane index of the lane's first voxel
    if (vp >= plane) return;
    if (d.geom.oct8 && d.mdtype == 0 && (nx & 1) == 0 && ((uintptr_t)d.moving & 1) == 0) {
      // u8 rows of even length: the lane's two voxels (vp even) lie in one
      // row.  Per slice and source row (y, y + 1 clamped): a 2-byte load at
      // x and the byte at x + 2 (clamped to the last column).
      const uint32_t y = vp / nx, x = vp - y * nx;
      const size_t ry0 = vp, ry1 = y + 1 < ny ? (size_t)vp + nx : (size_t)vp;
      const uint32_t xn = x + 2 < nx ? 2u : nx - 1u - x;  // offset of the byte after the pair
      global_u8* __restrict__ mv = (global_u8*)d.moving;
      uint32_t w[kPrepSlices + 1][2], e[kPrepSlices + 1][2];
#pragma unroll
      for (int k = 0; k <= kPrepSlices; ++k) {
        uint32_t z = z0 + (uint32_t)k;
        z = z < nz ? z : nz - 1;  // slice z0 + nzb is the block's last slice + 1, clamped
        if ((uint32_t)k > nzb) z = z0;  // past the block: a valid slice, not used
        const size_t sz = (size_t)z * plane;
        w[k][0] = ((global_u16*)(mv + sz + ry0))[0];
        e[k][0] = mv[sz + ry0 + xn];
        w[k][1] = ((global_u16*)(mv + sz + ry1))[0];
        e[k][1] = mv[sz + ry1 + xn];
      }
      // with 8-bit corners R <= 256, so the clamp is the identity exactly
      // when the range is 0..255
      const bool ident = d.mlo == 0 && d.mhi == 255;
      uint32_t cw[kPrepSlices + 1][2], t[kPrepSlices + 1][2];  // (x, x+1) and (x+1, x+2) in bytes 0, 1
#pragma unroll
      for (int k = 0; k <= kPrepSlices; ++k)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          uint32_t b0 = w[k][r] & 0xFFu, b1 = w[k][r] >> 8, b2 = e[k][r];
          if (!ident) {
            b0 = clamp_offset((int32_t)b0, d.mlo, d.mhi);
            b1 = clamp_offset((int32_t)b1, d.mlo, d.mhi);
            b2 = clamp_offset((int32_t)b2, d.mlo, d.mhi);
          }
          cw[k][r] = b0 | (b1 << 8);
          t[k][r] = b1 | (b2 << 8);
        }
#pragma unroll
      for (int k = 0; k < kPrepSlices; ++k) {
        if ((uint32_t)k >= nzb) break;
        // entries: byte 4 dz + 2 dy + dx' (layout of pack_oct8_kernel)
        *(global_out4*)((global_out2*)d.geom.octs + (size_t)(z0 + k) * plane + vp) =
            uint4_t{cw[k][0] | (cw[k][1] << 16), cw[k + 1][0] | (cw[k + 1][1] << 16),
                    t[k][0] | (t[k][1] << 16), t[k + 1][0] | (t[k + 1][1] << 16)};
      }
      return;
    }
    auto val = [&](size_t i) -> uint32_t { return clamp_offset(load_int(d.moving, d.mdtype, i), d.mlo, d.mhi); };
    for (uint32_t j = 0; j < 2; ++j) {
      const uint32_t v = vp + j;
      if (v >= plane) break;
      const uint32_t y = v / nx, x = v - y * nx;
      const size_t row0 = (size_t)v - x, row1 = y + 1 < ny ? row0 + nx : row0;  // rows y, y + 1 (clamped)
      const uint32_t x1 = x + 1 < nx ? x + 1 : nx - 1;
      for (uint32_t k = 0; k < nzb; ++k) {
        const uint32_t z = z0 + k;
        const size_t s0 = (size_t)z * plane, s1 = z + 1 < nz ? s0 + plane : s0;  // slices z, z + 1 (clamped)
        const size_t a0 = s0 + row0, a1 = s0 + row1, b0 = s1 + row0, b1 = s1 + row1;
        const size_t out = s0 + v;
        if (d.geom.oct8) {
          // 8-bit corners: byte 4 dz + 2 dy + dx' (layout of pack_oct8_kernel)
          ((global_out2*)d.geom.octs)[out] =
              uint2_t{val(a0 + x) | (val(a0 + x1) << 8) | (val(a1 + x) << 16) | (val(a1 + x1) << 24),
                      val(b0 + x) | (val(b0 + x1) << 8) | (val(b1 + x) << 16) | (val(b1 + x1) << 24)};
        } else {
          ((global_out4*)d.geom.octs)[out] =
              uint4_t{val(a0 + x) | (val(a0 + x1) << 16), val(a1 + x) | (val(a1 + x1) << 16),
                      val(b0 + x) | (val(b0 + x1) << 16), val(b1 + x) | (val(b1 + x1) << 16)};
        }
      }
    }
  });
}

template <bool CLAMP, bool PACKED, bool OCT8, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void hist_pairs_kernel(PairsArgs a) {
  extern __shared__ uint32_t lds_hist[];
  const int B = a.bins;
  const int words = B * hist_row_words(B, PACKED);
  // the work-item slot follows the histogram in the dynamic LDS (the sweep
  // addresses the histogram from LDS address 0: no static LDS)
  int64_t& item_sh = *(int64_t*)(lds_hist + ((words + 1) & ~1));
  clear_hist<PACKED, NT>(lds_hist, B);
  const uint32_t xcd = blockIdx.x & 7u;
  const int64_t* __restrict__ xbase = a.xcd_base + (int64_t)xcd * (a.n_pairs + 1);
  const int64_t total = xbase[a.n_pairs];
  // The items a workgroup takes from its queue ascend, so its pair only
  // moves forward: the pair's bounds, geometry and counts are loaded again
  // only when an item falls past it (a search per item put about log2 P
  // dependent loads before every slab's sweep).
  int p = -1;
  int64_t p_lo = 0, p_hi = 0;  // xbase[p], xbase[p + 1]; xbase[0] = 0
  HardGeom geom;
  int32_t n_t = 0, chunks = 0;
  int64_t t0 = 0;
  for (;;) {
    if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(&a.counters[xcd], 1ull);
    __syncthreads();
    const int64_t item = uniform(item_sh);
    if (item >= total) break;  // the same for every thread of the workgroup
    if (item >= p_hi) {
      do {  // item < total = xbase[P] bounds p + 1 <= P
        ++p;
        p_lo = p_hi;
        p_hi = uniform(xbase[p + 1]);
      } while (item >= p_hi);
      geom = uniform(a.pairs[p].geom);
      n_t = uniform(a.pairs[p].n_t);
      chunks = uniform(a.pairs[p].chunks);
      t0 = uniform(a.t_base[p]);
    }
    const int64_t rem = item - p_lo;
    // slab-major items: one slab's transforms in a row (the slab's moving
    // footprint stays in L2); transform-major: a transform's slabs in a row
    int64_t slab, tl;
    if (a.transform_major) {
      const int64_t per = chunks >> 3;
      tl = rem / per;
      slab = rem - tl * per;
    } else {
      slab = rem / n_t;
      tl = rem - slab * n_t;
    }
    const uint32_t chunk = xcd * (uint32_t)(chunks >> 3) + (uint32_t)slab;
    const int64_t t = t0 + tl;
    const double* Md = a.transforms + 12 * t;
    int64_t Mq[12];
    const bool ok = quantize_transform(Md, Mq);  // (the wave-parallel form measured 0.8% slower here)
    if (ok) {
      int64_t Ms[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) Ms[e] = uniform64(Mq[e]);
      sweep_hard<CLAMP, PACKED, OCT8, NT / 64, GroupWalkBrick, false>(geom, Md, Ms, chunks, chunk, lds_hist);
    }
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

hipError_t launch_pairs_prep(const PairsLaunch& L, hipStream_t s, bool volumes) {
  if (L.total_t > 0) {
    const int64_t blocks = (L.total_t + 255) / 256;
    hipLaunchKernelGGL(gather_transforms_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)),
                       dim3(256), 0, s, L.args, L.total_t);
  }
  if (!volumes) return hipGetLastError();
  if (L.fixed_chunks > 0)
    hipLaunchKernelGGL(prep_fixed_kernel, dim3(row_grid(L.fixed_chunks)), dim3(256), 0, s, L.args,
                       L.fixed_chunks);
  if (L.moving_chunks > 0)
    hipLaunchKernelGGL(prep_moving_kernel, dim3(row_grid(L.moving_chunks)), dim3(256), 0, s, L.args,
                       L.moving_chunks);
  return hipGetLastError();
}

// Dynamic LDS limit of the pairs sweep (a u32 table up to 128 bins, 16-bit
// pairs above, and the work-item slot after it).
constexpr size_t kPairsLdsMax = 150 * 1024;

template <bool CLAMP, bool PACKED, bool OCT8, int NT>
static hipError_t pairs_variant(const PairsLaunch& L, hipStream_t s) {
  const int B = L.args.bins;
  const size_t words = (size_t)B * hist_row_words(B, PACKED);
  const size_t lds = ((words + 1) & ~(size_t)1) * 4 + 8;  // histogram, then the 8-byte item slot
  const void* fn = (const void*)hist_pairs_kernel<CLAMP, PACKED, OCT8, NT>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPairsLdsMax);
  if (e != hipSuccess || (e = lds_guard(fn, lds, kPairsLdsMax, true)) != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  // every queue needs workgroups: a multiple of 8 (one share per XCD)
  const unsigned grid = (unsigned)(((per_cu * L.cu_count + 7) / 8) * 8);
  hipLaunchKernelGGL((hist_pairs_kernel<CLAMP, PACKED, OCT8, NT>), dim3(grid), dim3(NT), lds, s, L.args);
  return hipGetLastError();
}

template <bool CLAMP, bool PACKED, bool OCT8>
static hipError_t pairs_block(const PairsLaunch& L, hipStream_t s) {
  switch (L.block) {
  case 256: return pairs_variant<CLAMP, PACKED, OCT8, 256>(L, s);
  case 1024: return pairs_variant<CLAMP, PACKED, OCT8, 1024>(L, s);
  default: return pairs_variant<CLAMP, PACKED, OCT8, 512>(L, s);
  }
}

template <bool OCT8>
static hipError_t pairs_layout(const PairsLaunch& L, hipStream_t s) {
  if (L.clamp) return L.packed ? pairs_block<true, true, OCT8>(L, s) : pairs_block<true, false, OCT8>(L, s);
  return L.packed ? pairs_block<false, true, OCT8>(L, s) : pairs_block<false, false, OCT8>(L, s);
}

hipError_t launch_pairs_hist(const PairsLaunch& L, hipStream_t s) {
  return L.oct8 ? pairs_layout<true>(L, s) : pairs_layout<false>(L, s);
}

}  // namespace gemi
