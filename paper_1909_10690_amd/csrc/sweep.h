// The hard-binned histogram sweep of one slab of the fixed volume for one
// transform, shared by the single-pair kernel (hard.hip) and the persistent
// multi-pair kernel (pairs.hip).  Internal to libgemi.so.
#pragma once

#include "common.h"

#pragma clang fp contract(off)

namespace gemi {

typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));
typedef unsigned int uint2_t __attribute__((ext_vector_type(2)));
typedef unsigned int uint4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) uint32_t lds_u32;
// Device-memory bytes: loads through such a pointer are global, not flat,
// also when the pointer itself was read from memory.
typedef const __attribute__((address_space(1))) uint8_t global_u8;

// Loads of one record of a buffer whose descriptor has a stride: the
// hardware forms base + index * stride, so the index needs no shift.
__device__ uint4_t struct_load_b128(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");
__device__ uint2_t struct_load_b64(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");

// v0 (1 - w) + v1 w at 16-bit weight w = fx >> 16, exact: the pair's low
// half times (65535 - w), high half times w, plus the low half once more.
__device__ __forceinline__ uint32_t lerp_x(uint32_t pair, uint32_t wpack) {
  return __builtin_amdgcn_udot2(__builtin_bit_cast(ushort2_t, pair),
                                __builtin_bit_cast(ushort2_t, wpack), pair & 0xFFFFu, false);
}

// Exact bin of V = sum over corners, from the four exact x-lerps.
static __device__ __noinline__ uint32_t exact_bin(uint32_t a00, uint32_t a10, uint32_t a01, uint32_t a11,
                                           uint32_t wy, uint32_t wz, uint32_t B, Divider div) {
  const uint64_t b0 = (uint64_t)a00 * (65536u - wy) + (uint64_t)a10 * wy;
  const uint64_t b1 = (uint64_t)a01 * (65536u - wy) + (uint64_t)a11 * wy;
  const uint64_t V = b0 * (65536u - wz) + b1 * wz;
  // floor(V B / (R 2^48)) = floor(X / R), X = floor(V B / 2^48) < 2^24
  const uint32_t X = (uint32_t)(V >> 48) * B + (uint32_t)(((V & 0xFFFFFFFFFFFFull) * B) >> 48);
  return div_small(X, div);
}

constexpr double kEdge = 1.0 / 536870912.0;  // 2^-29

// Per-launch constants of the hard-binned step of one fixed voxel: the
// moving gather volume, its upper coordinates, the bin scale and the LDS
// histogram's byte address.
struct HardStep {
  __amdgpu_buffer_rsrc_t rsrc;
  uint64_t topx, topy, topz;
  uint32_t NY, MX, Bu, row_bytes, row_cells;
  double scale;
  Divider div;

  // oct8: the gather volume's records are 8-bit corners (8 bytes), as the
  // kernel's OCT8 instance reads them; else 16-bit ones (16 bytes)
  __device__ __forceinline__ HardStep(const HardGeom& g, uint32_t* lds_hist, bool oct8) {
    topx = (uint64_t)(g.mnx - 1) << 32;
    topy = (uint64_t)(g.mny - 1) << 32;
    topz = (uint64_t)(g.mnz - 1) << 32;
    NY = (uint32_t)g.mny;
    MX = (uint32_t)g.mnx;
    // records of 8 (OCT8) or 16 bytes, indexed by voxel; the record bound is
    // given in bytes, which is no tighter than any record count
    rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)g.octs, (short)(oct8 ? 8 : 16), (int)g.oct_bytes,
                                             0x00020000);
    Bu = (uint32_t)g.bins;
    // LDS histogram row pitch: in bytes (u32 counters), in 16-bit cells
    // (packed counters)
    row_bytes = 4u * (uint32_t)hist_row_words(g.bins, false);
    row_cells = 2u * (uint32_t)hist_row_words(g.bins, true);
    scale = g.scale;
    div = g.div;
  }

  // Counts one fixed voxel whose exact Q32 moving coordinates (qx, qy, qz)
  // are given: clamped (CLAMP) or skipped when outside [0, n - 1] on any
  // axis; fixed_bin() supplies its fixed bin (read after the gather is
  // issued).  CHECK false: the caller has established that the voxel lies
  // inside on every axis, where clamping and skipping change nothing.
  template <bool CLAMP, bool PACKED, bool OCT8, bool CHECK = true, typename FB>
  __device__ __forceinline__ void count(int64_t qx, int64_t qy, int64_t qz, FB&& fixed_bin,
                                        uint32_t* lds_hist) const {
    uint64_t cx = (uint64_t)qx, cy = (uint64_t)qy, cz = (uint64_t)qz;
    if (!CHECK) {
    } else if (CLAMP) {
      cx = qx < 0 ? 0 : (cx > topx ? topx : cx);
      cy = qy < 0 ? 0 : (cy > topy ? topy : cy);
      cz = qz < 0 ? 0 : (cz > topz ? topz : cz);
    } else {
      // 0 <= q <= top; a negative q wraps to a huge unsigned value
      if (cx > topx || cy > topy || cz > topz) return;
    }
    const uint32_t ix = (uint32_t)(cx >> 32), iy = (uint32_t)(cy >> 32), iz = (uint32_t)(cz >> 32);
    // rows iz ny + iy < ny nz <= 2^24 and edges <= 4096: 24-bit operands
    const uint32_t vox = mad24(mad24(iz, NY, iy), MX, ix);
    uint4_t oc;
    if (OCT8) {
      // bytes (x,y), (x1,y), (x,y1), (x1,y1) of slice z in .x, of z1 in .y
      const uint2_t d = struct_load_b64(rsrc, (int)vox, 0, 0, 0);
      oc.x = __builtin_amdgcn_perm(0u, d.x, 0x0C010C00u);  // (b0, b1) as 16-bit halves
      oc.y = __builtin_amdgcn_perm(0u, d.x, 0x0C030C02u);  // (b2, b3)
      oc.z = __builtin_amdgcn_perm(0u, d.y, 0x0C010C00u);
      oc.w = __builtin_amdgcn_perm(0u, d.y, 0x0C030C02u);
    } else {
      oc = struct_load_b128(rsrc, (int)vox, 0, 0, 0);
    }
    bin_count<PACKED>(oc, fixed_bin(), (uint32_t)cx, (uint32_t)cy, (uint32_t)cz, lds_hist);
  }

  // The moving bin from the 16-bit corner pairs oc and the Q32 fractions,
  // exactly, and the count of cell [fb][bin].
  template <bool PACKED>
  __device__ __forceinline__ void bin_count(const uint4_t& oc, uint32_t fb, uint32_t fx, uint32_t fy,
                                            uint32_t fz, uint32_t* lds_hist) const {
    // (65535 - wx) in the low half, wx in the high half: the high halves of
    // ~fx and fx, one byte permute
    const uint32_t wpack = __builtin_amdgcn_perm(fx, ~fx, 0x07060302u);
    const uint32_t a00 = lerp_x(oc.x, wpack), a10 = lerp_x(oc.y, wpack);
    const uint32_t a01 = lerp_x(oc.z, wpack), a11 = lerp_x(oc.w, wpack);
    const uint32_t wy = fy >> 16, wz = fz >> 16;
    const double wyd = (double)wy, wzd = (double)wz;
    const double A00 = (double)a00, A10 = (double)a10, A01 = (double)a01, A11 = (double)a11;
    const double uyd = 65536.0 - wyd;
    const double b0 = fma(A10, wyd, A00 * uyd);         // exact, < 2^48
    const double b1 = fma(A11, wyd, A01 * uyd);         // exact, < 2^48
    const double V = fma(b1 - b0, wzd, b0 * 65536.0);  // exact value rounded once
    // the bin position shifted up by kEdge: its floor is the bin unless the
    // exact position lies within kEdge of a bin edge, which is when the
    // fraction falls below 2 kEdge (the rounding errors are far smaller)
    const double tb = fma(V, scale, kEdge);
    uint32_t bm = (uint32_t)tb;
    if (__builtin_amdgcn_fract(tb) < 2.0 * kEdge) bm = exact_bin(a00, a10, a01, a11, wy, wz, Bu, div);
    if (PACKED) {
      // 16-bit cell of counter [fb][bm]; the row pitch is even, so the
      // cell's word and half follow from it directly
      const uint32_t cell = __umul24(fb, row_cells) + bm;
      atomicAdd(&lds_hist[cell >> 1], 1u << ((cell & 1u) * 16u));
    } else {
      // LDS byte address of counter [fb][bm], formed directly: a mul24 and
      // a shift-add.  The kernels that sweep keep no static LDS, so their
      // dynamic histogram starts at address 0 (lds_guard checks this at
      // launch) and needs no base.
      const uint32_t addr = (bm << 2) + __umul24(fb, row_bytes);
      __hip_atomic_fetch_add((lds_u32*)(size_t)addr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
};

// The x ranges of a wave's row groups (range_lane, range_value, row_spans):
// lanes 0..15 hold the bound constants of the transform, and each row group
// takes the least v of each group of four lanes with two quad permutes.
struct RowRanges {
  RangeLane c;
  bool exact;  // uniform: every lane's constants exact

  // Md: the transform's 12 entries (index space, row-major 3 x 4) in device
  // memory; each lane reads its axis row and rounds it to Q32 as
  // quantize_transform does.
  __device__ __forceinline__ void init(const double* Md, const HardGeom& g, int lane) {
    const int a = (lane & 3) == 3 ? 0 : (lane & 3);
    const double* row = Md + 4 * a;
    const double q = 4294967296.0;
    const double m0 = __builtin_rint(row[0] * q), m1 = __builtin_rint(row[1] * q);
    const double m2 = __builtin_rint(row[2] * q), m3 = __builtin_rint(row[3] * q);
    const int32_t n = a == 0 ? g.mnx : (a == 1 ? g.mny : g.mnz);
    c = range_lane(lane, m0, m1, m2, m3, (double)(n - 1) * q);
    exact = __builtin_amdgcn_ballot_w64(!c.exact) == 0;
  }

  // Spans of the row group at (j0, k); the whole wave takes part.
  __device__ __forceinline__ RowSpans spans(int32_t j0, int32_t k, int32_t full, bool skip) const {
    if (!exact) return RowSpans{0, full, full, full};
    int32_t v = range_value(c, j0, k);
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false));  // quad_perm 2,3,0,1
    return row_spans(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 4),
                     __builtin_amdgcn_readlane(v, 8), __builtin_amdgcn_readlane(v, 12), full, skip);
  }
};

// Sweeps one slab of the fixed volume for one transform (Mq) into the
// workgroup's LDS histogram.  NW waves share the slab's 4-row groups, in
// the order of Walk (thin slabs, or bricks).
// OCT8: the oct volume holds 8-bit corners (one 64-bit gather), unpacked
// into the 16-bit pairs of the x-lerp with byte permutes.
// Md: the transform as stored; Mq: its Q32 rounding, in scalar registers
// (quantize_transform_wave).  RANGES false: every
// voxel is tested (the range lanes' registers would not fit a kernel already
// at its register budget).
template <bool CLAMP, bool PACKED, bool OCT8, int NW, typename Walk = GroupWalk, bool RANGES = true>
__device__ __forceinline__ void sweep_hard(const HardGeom& g, const double* Md, const int64_t* Mq,
                                           int32_t chunks, uint32_t chunk, uint32_t* lds_hist) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int dx = lane & (kTileX - 1), dy = lane / kTileX;
  // the matrix in scalar registers (quantize_transform_wave puts it there):
  // the walk's row coordinates and steps are then scalar values, and only
  // the lane offsets take vector registers
  const int64_t* M = Mq;
  Walk w;
  w.init(M, g.fny, g.fnz, chunks, chunk, wave, NW, dx, dy);
  const int64_t sx = w.step[0], sy = w.step[1], sz = w.step[2];
  const HardStep hs(g, lds_hist, OCT8);
  // fixed bins through a buffer descriptor: the lane's offset within the
  // tile in a vector register, the tile's in a scalar one (fixed voxels
  // < 2^28: 32-bit offsets)
  const uint32_t fnx = (uint32_t)g.fnx;
  const __amdgpu_buffer_rsrc_t frsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)g.fbins, (short)0, (int)(fnx * (uint32_t)g.fny * (uint32_t)g.fnz), 0x00020000);
  const int lane_f = (int)(dy * fnx + dx);
  const int32_t full = (int32_t)(fnx / kTileX);      // x steps every lane of the tile takes
  const bool tail = (uint32_t)dx < fnx % kTileX;  // the lane takes one more
  const bool has_tail = fnx % kTileX != 0;
  RowRanges ranges;
  if (RANGES) ranges.init(Md, g, lane);

  if constexpr (!RANGES) {
    for (; w.g < w.g1; w.next()) {
      if (w.j0 + dy >= g.fny) continue;
      uint32_t soff = ((uint32_t)w.k * (uint32_t)g.fny + (uint32_t)w.j0) * fnx;
      int64_t qx = w.r[0] + w.lane_off[0], qy = w.r[1] + w.lane_off[1], qz = w.r[2] + w.lane_off[2];
      auto fixed_bin = [&] { return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(frsrc, lane_f, (int)soff, 0); };
      for (int32_t it = 0; it < full; ++it, soff += kTileX, qx += sx, qy += sy, qz += sz)
        hs.count<CLAMP, PACKED, OCT8>(qx, qy, qz, fixed_bin, lds_hist);
      if (tail) hs.count<CLAMP, PACKED, OCT8>(qx, qy, qz, fixed_bin, lds_hist);
    }
    return;
  }
  for (; w.g < w.g1; w.next()) {
    // x steps [u0, c0) and [c1, u1) test each voxel, [c0, c1) has every
    // lane inside; with EXCLUDE no lane counts outside [u0, u1)
    const RowSpans sp = ranges.spans(w.j0, w.k, full, !CLAMP);
    const int32_t j = w.j0 + dy;
    if (j >= g.fny) continue;
    const uint32_t row = ((uint32_t)w.k * (uint32_t)g.fny + (uint32_t)w.j0) * fnx;
    uint32_t soff = row + (uint32_t)sp.u0 * kTileX;
    int64_t qx = w.r[0] + w.lane_off[0], qy = w.r[1] + w.lane_off[1], qz = w.r[2] + w.lane_off[2];
    if (sp.u0 > 0) {
      qx += sx * sp.u0;
      qy += sy * sp.u0;
      qz += sz * sp.u0;
    }
    auto fixed_bin = [&] { return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(frsrc, lane_f, (int)soff, 0); };
    int32_t it = sp.u0;
    for (; it < sp.c0; ++it, soff += kTileX, qx += sx, qy += sy, qz += sz)
      hs.count<CLAMP, PACKED, OCT8>(qx, qy, qz, fixed_bin, lds_hist);
    for (; it < sp.c1; ++it, soff += kTileX, qx += sx, qy += sy, qz += sz)
      hs.count<CLAMP, PACKED, OCT8, false>(qx, qy, qz, fixed_bin, lds_hist);
    for (; it < sp.u1; ++it, soff += kTileX, qx += sx, qy += sy, qz += sz)
      hs.count<CLAMP, PACKED, OCT8>(qx, qy, qz, fixed_bin, lds_hist);
    if (has_tail && tail) {
      soff = row + (uint32_t)full * kTileX;
      qx = w.r[0] + sx * full + w.lane_off[0];
      qy = w.r[1] + sy * full + w.lane_off[1];
      qz = w.r[2] + sz * full + w.lane_off[2];
      hs.count<CLAMP, PACKED, OCT8>(qx, qy, qz, fixed_bin, lds_hist);
    }
  }
}

// Clears a workgroup's LDS histogram, padding included (16-byte stores,
// then the last words).
template <bool PACKED, int NT>
__device__ __forceinline__ void clear_hist(uint32_t* lds_hist, int B) {
  const int words = B * hist_row_words(B, PACKED), quads = words >> 2;
  uint4_t* q = (uint4_t*)lds_hist;
  for (int e = threadIdx.x; e < quads; e += NT) q[e] = uint4_t{0u, 0u, 0u, 0u};
  for (int e = (quads << 2) + (int)threadIdx.x; e < words; e += NT) lds_hist[e] = 0;
}

// Adds the non-zero LDS bins into a transform's HBM histogram [B][B] (and
// clears them for the next use of the LDS histogram when `rezero`): a wave
// per fixed-bin row at a time, a lane per counter word.
// A row holds at most 256 counter words (B <= 256), four per lane, so each
// row is unrolled into four fixed chunks whose addresses differ from the
// first by immediate offsets.
template <bool PACKED, int NT>
__device__ __forceinline__ void flush_hist(uint32_t* lds_hist, int B, uint32_t* __restrict__ out,
                                           bool rezero) {
  const int pitch = hist_row_words(B, PACKED), used = PACKED ? (B + 1) / 2 : B;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int r = wave; r < B; r += NT / 64) {
    uint32_t* __restrict__ row = out + (size_t)r * B;
    uint32_t* src = lds_hist + r * pitch;
    uint32_t vs[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) vs[c] = lane + 64 * c < used ? src[lane + 64 * c] : 0u;  // reads issued together
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int w = lane + 64 * c;
      const uint32_t v = vs[c];
      if (v == 0) continue;
      if (rezero) src[w] = 0;
      if (PACKED) {
        if (v & 0xFFFFu) atomicAdd(&row[2 * w], v & 0xFFFFu);
        if (v >> 16) atomicAdd(&row[2 * w + 1], v >> 16);  // never set past the row's last bin
      } else {
        atomicAdd(&row[w], v);
      }
    }
  }
}

}  // namespace gemi
