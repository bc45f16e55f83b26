// Internal declarations shared by the HIP translation units of libgemi.so.
// Nothing here is part of the public ABI (include/gemi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "plan.h"

namespace gemi {

// a * b + c with 24-bit unsigned operands a, b and b uniform
// (v_mad_u32_u24, full rate; left to itself the compiler may pick the
// quarter-rate 64-bit multiply-add).
__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

constexpr int kMaxQ = 16;
constexpr int kBlock = 256;  // threads per workgroup of the reduction kernels (4 wave64)

// Entropic indices passed by value to the reduction kernels.
struct QList {
  double q[kMaxQ];
  int32_t n;
  int32_t pseudo;  // 1 = pseudo-additive Tsallis MI
};

// Exact floor(X / R) for 0 <= X < 2^24 as (X * m) >> s (Granlund and
// Montgomery, "Division by invariant integers using multiplication", PLDI
// 1994, Thm 4.2 with N = 24, l = ceil(log2 R), m = ceil(2^(N+l) / R)).
struct Divider {
  uint32_t m;
  uint32_t s;
};

inline Divider make_divider(uint32_t R) {
  uint32_t l = 0;
  while ((1u << l) < R) ++l;
  const uint64_t num = 1ull << (24 + l);
  Divider d;
  d.m = (uint32_t)((num + R - 1) / R);
  d.s = 24 + l;
  return d;
}

__device__ __forceinline__ uint32_t div_small(uint32_t x, Divider d) {
  return (uint32_t)(((uint64_t)x * d.m) >> d.s);
}

// Spacings and origins of a fixed/moving pair: voxel index i of a volume
// sits at origin + spacing * i (mm, per axis x, y, z).
struct Geometry {
  double fsp[3], forg[3];  // fixed
  double msp[3], morg[3];  // moving
};

// Index-space matrix M (fixed voxel index -> continuous moving index) of a
// physical fixed -> moving matrix P (Fig. 1 Transform block, mm):
//   M[r][c] = (P[r][c] * fsp[c]) / msp[r]                                        (c < 3)
//   M[r][3] = ((((P[r][0] forg[0] + P[r][1] forg[1]) + P[r][2] forg[2]) + P[r][3]) - morg[r]) / msp[r]
// one IEEE operation at a time in exactly this order, never fused, so that
// every implementation of the same definition quantises the same matrix.
__device__ __forceinline__ void compose_index_matrix(const double* __restrict__ P, const Geometry& g,
                                                     double* __restrict__ M) {
#pragma clang fp contract(off)
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a = P[4 * r + c] * g.fsp[c];
      M[4 * r + c] = a / g.msp[r];
    }
    double o = P[4 * r] * g.forg[0];
    const double o1 = P[4 * r + 1] * g.forg[1];
    o = o + o1;
    const double o2 = P[4 * r + 2] * g.forg[2];
    o = o + o2;
    o = o + P[4 * r + 3];
    o = o - g.morg[r];
    M[4 * r + 3] = o / g.msp[r];
  }
}

// Q32 quantisation of one index-space 3x4 transform: Mq = rne(M * 2^32).
// A transform is usable when every entry is finite, linear entries are
// within +-2^16 and translations within +-2^24 (so that every coordinate of
// a volume of at most 4096 voxels per axis fits in int64).
__device__ __forceinline__ bool quantize_transform(const double* __restrict__ M, int64_t* Mq) {
  bool ok = true;
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    const double m = M[e];
    const double lim = (e % 4 == 3) ? 16777216.0 : 65536.0;
    ok = ok && (fabs(m) <= lim);  // false for NaN and infinities
    Mq[e] = __double2ll_rn(m * 4294967296.0);
  }
  return ok;
}

// quantize_transform for a whole wave at once: lane e < 12 rounds entry e
// and the results are broadcast to scalar registers, with the same values
// and the same validity test.  Every lane of the wave takes part.
__device__ __forceinline__ bool quantize_transform_wave(const double* __restrict__ M, int64_t* Mq) {
  const int lane = threadIdx.x & 63;
  const int e = lane < 12 ? lane : 0;
  const double m = M[e];
  const double lim = (e % 4 == 3) ? 16777216.0 : 65536.0;
  const bool bad = lane < 12 && !(fabs(m) <= lim);  // true for NaN and infinities
  const int64_t v = __double2ll_rn(m * 4294967296.0);
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)((uint64_t)v >> 32);
#pragma unroll
  for (int i = 0; i < 12; ++i)
    Mq[i] = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, i) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane(lo, i));
  return __builtin_amdgcn_ballot_w64(bad) == 0;
}

// A value every lane holds alike, moved to scalar registers.  A value
// computed by vector instructions stays in vector registers otherwise, and
// the compiler drops a readfirstlane builtin of a value it knows is uniform,
// so the move is written out.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  uint32_t lo, hi;
  asm volatile("v_readfirstlane_b32 %0, %1" : "=s"(lo) : "v"((uint32_t)v));
  asm volatile("v_readfirstlane_b32 %0, %1" : "=s"(hi) : "v"((uint32_t)((uint64_t)v >> 32)));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// per-voxel input preparation shared by the single-pair and multi-pair paths
// ---------------------------------------------------------------------------

// Fixed bin of an integer intensity: floor((clamp(u) - lo) * B / R).
__device__ __forceinline__ uint32_t fixed_bin_int(int32_t u, int32_t lo, int32_t hi, uint32_t bins,
                                                  Divider d) {
  u = u < lo ? lo : (u > hi ? hi : u);
  return div_small((uint32_t)(u - lo) * bins, d);
}

// Fixed bin of a float intensity: min(B-1, floor(((u - lo)/(hi - lo)) * B))
// in fp64, each step one IEEE operation.
__device__ __forceinline__ uint32_t fixed_bin_real(double u, double lo, double hi, int32_t bins) {
  u = u < lo ? lo : (u > hi ? hi : u);
  const double r = __ddiv_rn(__dsub_rn(u, lo), __dsub_rn(hi, lo));
  const int32_t b = (int32_t)floor(__dmul_rn(r, (double)bins));
  return (uint32_t)(b > bins - 1 ? bins - 1 : (b < 0 ? 0 : b));
}

// Clamped, offset intensity v' = clamp(v, lo, hi) - lo.
__device__ __forceinline__ uint32_t clamp_offset(int32_t v, int32_t lo, int32_t hi) {
  v = v < lo ? lo : (v > hi ? hi : v);
  return (uint32_t)(v - lo);
}

// ---------------------------------------------------------------------------
// the fixed-volume sweep shared by the histogram kernels
// ---------------------------------------------------------------------------

// Maps workgroup id -> (transform, slab, band).  Workgroups are dealt
// round-robin to the 8 XCDs, so XCD x receives ids x, x+8, ...; those all
// take slabs from the x-th eighth of the fixed volume.  Slab-major order
// (within a band, when there are several) walks that eighth one thin slab
// at a time, all transforms per slab, so the workgroups resident on an XCD
// at once share one slab's moving footprint in that XCD's L2;
// transform-major order finishes a transform's slabs (all bands per slab)
// before the next transform.
__device__ __forceinline__ void block_work(int32_t chunks, int32_t n, int32_t bands,
                                           int32_t slab_major, uint32_t& t, uint32_t& chunk,
                                           uint32_t& band) {
  const uint32_t bid = blockIdx.x;
  const uint32_t xcd = bid & 7u, slot = bid >> 3;
  const uint32_t c8 = (uint32_t)chunks >> 3;
  const uint32_t nb = (uint32_t)bands;
  if (slab_major) {
    // bands slowest: every workgroup of band 0 is dispatched before any of
    // band 1, and so on.  A Parzen sweep's first band holds the background,
    // nearly every voxel of a CT, so its workgroups are the long ones:
    // dispatched first, they no longer trail the launch on a few CUs.
    const uint32_t per = c8 * (uint32_t)n;
    band = slot / per;
    const uint32_t rem = slot - band * per, cl = rem / (uint32_t)n;
    t = rem - cl * (uint32_t)n;
    chunk = xcd * c8 + cl;
  } else {
    const uint32_t per = c8 * nb;
    t = slot / per;
    const uint32_t rem = slot - t * per;
    band = rem / c8;
    chunk = xcd * c8 + (rem - band * c8);
  }
}

// The same walk in brick order: the row groups of a slice are cut along y
// into blocks of `yb` groups and a block is visited slice by slice before
// the next, so a slab -- a contiguous range of that numbering -- is a brick
// of whole x rows, about as many rows deep (4 yb) as slices long.  A thin
// slab of whole slices leaves its moving footprint under a small change of
// rotation; a brick keeps much of it, so the transforms a slab meets in turn
// reuse the XCD's L2 when they rotate widely (a rotation map).  Row
// coordinates stay exact: stepped by kTileY M[:,1] inside a block row and
// recomputed at each wrap.
struct GroupWalkBrick {
  int64_t g, g1;
  int32_t j0, k;
  int32_t G, nz, yb, b0, b1;  // y groups, slices, block width, current block [b0, b1)
  int64_t r[3], lane_off[3], step[3], adv[3], m1[3], m2[3], m3[3];

  __host__ __device__ __forceinline__ void init(const int64_t* Mq, int32_t fny, int32_t fnz,
                                                int32_t chunks, uint32_t chunk, int wave, int nwaves,
                                                int dx, int dy) {
    G = (fny + kTileY - 1) / kTileY;
    nz = fnz;
    const int64_t groups = (int64_t)G * fnz;
    const int64_t s0 = groups * chunk / chunks, s1 = groups * (chunk + 1) / chunks;
    g = s0 + (s1 - s0) * wave / nwaves;
    g1 = s0 + (s1 - s0) * (wave + 1) / nwaves;
    // bricks of 4 yb rows by per_slab / yb slices, twice as many rows as
    // slices (yb = sqrt(per_slab / 2)): on a 51^3 rotation map of a
    // 256x256x180 volume 4.61 s, against 5.53 s for square bricks and
    // 5.3-6.1 s for other widths
    const int64_t per_slab = (groups + chunks - 1) / chunks;
    const int32_t w = (int32_t)sqrt((double)per_slab * 0.5);
    yb = w < 1 ? 1 : (w > G ? G : w);
    const int64_t full = G / yb, per_full = (int64_t)yb * fnz;
    b0 = 0;
    b1 = G;
    k = 0;
    j0 = 0;
    if (g < g1) {
      if (g < full * per_full) {
        const int64_t blk = g / per_full, rem = g - blk * per_full;
        b0 = (int32_t)blk * yb;
        b1 = b0 + yb;
        k = (int32_t)(rem / yb);
        j0 = (b0 + (int32_t)(rem - (int64_t)k * yb)) * kTileY;
      } else {  // the last, narrower block (G not a multiple of yb)
        const int64_t rem = g - full * per_full;
        b0 = (int32_t)full * yb;
        const int32_t bw = G - b0;
        k = (int32_t)(rem / bw);
        j0 = (b0 + (int32_t)(rem - (int64_t)k * bw)) * kTileY;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t m0 = Mq[4 * a];
      m1[a] = Mq[4 * a + 1];
      m2[a] = Mq[4 * a + 2];
      m3[a] = Mq[4 * a + 3];
      r[a] = m1[a] * j0 + m2[a] * k + m3[a];
      lane_off[a] = m0 * dx + m1[a] * dy;
      step[a] = m0 * kTileX;
      adv[a] = m1[a] * kTileY;
    }
  }

  __host__ __device__ __forceinline__ void next() {
    ++g;
    j0 += kTileY;
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] += adv[a];
    if (j0 >= b1 * kTileY) {
      j0 = b0 * kTileY;
      if (++k >= nz) {
        k = 0;
        b0 = b1;
        b1 = b1 + yb < G ? b1 + yb : G;
        j0 = b0 * kTileY;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) r[a] = m1[a] * j0 + m2[a] * k + m3[a];
    }
  }
};

// Geometry of one fixed/moving pair for the hard-binned sweep.
struct HardGeom {
  const uint8_t* fbins;  // fixed bins, [fnz][fny][fnx]
  const void* octs;      // moving oct volume, [mnz][mny][mnx]: u16x8, or u8x8 when oct8
  int32_t fnx, fny, fnz;
  int32_t mnx, mny, mnz;
  uint32_t oct_bytes;
  int32_t oct8;          // 1: 8-bit corners (moving range R <= 256)
  int32_t bins;
  double scale;  // B / (R 2^48), R = moving hi - lo + 1
  Divider div;   // floor(X / R) for the exact fallback
};

// Host-side launch descriptions.
struct VolumeDesc {
  const void* data;
  int32_t nx, ny, nz, dtype;
  double lo, hi;
};

struct HardLaunch {
  const double* transforms;  // [n][12]
  const uint8_t* fbins;      // fixed-volume bins, [fnz][fny][fnx]
  const void* octs;          // moving oct volume, [mnz][mny][mnx] (u16x8 or u8x8)
  VolumeDesc fixed, moving;
  uint32_t* hist;  // [n][B][B]
  int32_t n, bins, clamp;
  int32_t chunks;  // workgroups per transform, multiple of 8
  int32_t packed;  // 1: two 16-bit counters per LDS word (bins > 128)
  int32_t block;   // threads per workgroup: 256, 512 or 1024
  int32_t slab_major;  // workgroup order: 1 slab-major, 0 transform-major
  int32_t brick;       // 1: slabs as bricks (GroupWalkBrick; 1024-thread launches)
  // processing order (launch_order_transforms), or NULL: the workgroups of
  // slot t sweep transform order[t] - order_t0; order_t0 is the batch index
  // of this launch's first transform
  const uint32_t* order;
  int64_t order_t0;
};

// Transforms per block of the processing order: the order is sorted within
// blocks of this many transforms, and launches that use it start at
// multiples of it.
constexpr int32_t kOrderBlock = 4096;

// The processing order of a batch of n index-space matrices for the hard
// sweep (order[i], absolute indices, a permutation of each block of
// kOrderBlock transforms): transforms whose images of the fixed volume lie
// at similar moving depths come together (see the kernel).
hipError_t launch_order_transforms(const double* M, int32_t n, int32_t fnx, int32_t fny, int32_t fnz, uint32_t* order,
                                   hipStream_t s);

// The gathers address their volume with 32-bit buffer offsets, so every
// gather volume stays below 4 GiB (the entry points check it).
constexpr size_t kMaxGatherBytes = 0xFFFFFFF0u;

// Bytes of the oct volume of an integer moving volume: per voxel the eight
// clamped, offset 16-bit corners of its 2x2x2 neighbourhood (16 bytes).
inline size_t oct_volume_bytes(int32_t nx, int32_t ny, int32_t nz) {
  return (size_t)nx * (size_t)ny * (size_t)nz * 16;
}

// The hard path packs 8-bit corners (8 bytes per voxel) when the moving
// range R = hi - lo + 1 is at most 256: the same single gather per voxel at
// half the bytes, which matters where the moving volumes stream from HBM.
inline bool oct8_range(double lo, double hi) { return hi - lo + 1.0 <= 256.0; }
inline size_t oct8_volume_bytes(int32_t nx, int32_t ny, int32_t nz) {
  return (size_t)nx * (size_t)ny * (size_t)nz * 8;
}

// Bytes of the 16-bit quad volume of an integer moving volume on the Parzen
// path: per voxel the four (x, y) corners of its neighbourhood in one slice
// (clamped, offset values), one extra slice; two 8-byte loads per voxel at
// half the footprint of the oct volume, which matters when one transform's
// gathers cover a moving volume larger than the caches.
inline size_t quad16_bytes(int32_t nx, int32_t ny, int32_t nz) {
  return (size_t)nx * (size_t)ny * (size_t)(nz + 1) * 8;
}

// Bytes of the fp32 quad volume of a float moving volume: per voxel the
// four (x, y) corners of its neighbourhood in one slice, one extra slice.
inline size_t quad_f32_bytes(int32_t nx, int32_t ny, int32_t nz) {
  return (size_t)nx * (size_t)ny * (size_t)(nz + 1) * 16;
}

// The MI reduction splits each transform's table into reduce_splits(B, n)
// row slices (with the same-numbered columns' marginals), one workgroup
// each: a few transforms then still keep many CUs busy (1024 / n slices,
// at most B / 8 of >= 8 rows), while a large batch uses one workgroup per
// transform, whose per-workgroup overheads small slices would multiply.
// The slices' compensated partial sums are merged in slice order, so a
// result does not depend on scheduling; batches with the same slice count
// give bit-identical results for the same transform.
__host__ __device__ inline int32_t reduce_splits(int32_t bins, int64_t n) {
  if (bins < 16 || n <= 0) return 1;
  const int64_t s = 1024 / n;
  return (int32_t)(s < 1 ? 1 : (s > bins / 8 ? bins / 8 : s));
}

// Bytes of the partial sums: per transform, slice and entropy, three
// compensated (sum, error) pairs.
inline size_t reduce_part_bytes(int64_t n, int32_t bins, int32_t n_q) {
  return (size_t)n * reduce_splits(bins, n) * n_q * 3 * 16;
}

// Rows [r0, r1) of slice s of a B-row table split into S slices.
__host__ __device__ inline void slice_rows(int B, int S, int s, int& r0, int& r1) {
  r0 = (int)(((int64_t)B * s) / S);
  r1 = (int)(((int64_t)B * (s + 1)) / S);
}

// Slices with at most this many cells and marginals keep p and ln p in LDS.
constexpr int kMaxSliceCells = 2304;

struct ReduceLaunch {
  const uint32_t* hist;  // [n][B][B] counts, or NULL when `table` is used
  const double* table;   // [n][B][B] Parzen masses, or NULL
  uint64_t* count;       // [n] N: given with a table; summed from hist otherwise
  double* part;          // reduce_part_bytes(n, B, n_q) of partial sums
  const double* transforms;
  int32_t n, bins;
  int32_t splits;        // reduce_splits(bins, n), set by launch_mi_reduce
  double* marg_out;      // [n][2B] row then column marginals (masses), or NULL
  QList q;
  double* mi_out;        // [n][n_q]
  uint64_t* overlap_out; // [n] or NULL
};

// Parzen sweeps (see parzen.hip).
// Occupied fixed-bin rows of a Parzen call.  The Parzen sweeps index the
// table's rows by "slot" (rank among the occupied rows), so that the LDS
// bands cover only rows that hold voxels: a CT-like fixed volume occupies a
// few clusters of its bins (air, soft tissue, bone) and empty bands would
// still cost a full walk of the fixed volume each.
struct RowMap {
  uint32_t used[256];         // 1 for every bin some fixed voxel falls in
  uint32_t row_of_slot[256];  // table row of each slot
  uint32_t slot_of_row[256];  // slot of each occupied row
  uint32_t n_slots;           // occupied rows
};

struct ParzenArgs {
  const double* transforms;
  const uint8_t* fbins;       // fixed-volume slots (see RowMap)
  const RowMap* rows;
  const uint32_t* tile_mask;  // [row groups][x tiles]: slot groups present in each 16 x 4 wave tile
  const uint32_t* row_mask;   // [row groups]: the OR of each row group's tile masks
  const void* gvol;    // integer moving: 16-bit quads (full sweeps) or octs (sampled); float: f32 quads
  double* table;       // [n][B][B] forward masses (fp64)
  uint64_t* count;     // [n] voxels that took part
  const float* gtab;   // [n][n_q][B][B] d MI / d p
  const double* marg;  // [n][2B] row then column marginals of the table (from the reduction)
  double* grad;        // [n][n_q][12]
  int32_t fnx, fny, fnz;
  int32_t mnx, mny, mnz;
  uint32_t gvol_bytes;
  int32_t n, bins, chunks, bands, band_rows, slab_major;
  int32_t n_q, q0;     // backward: entropies [q0, q0 + NQG) of n_q
  float sscale;        // (B - 4) / (hi - lo)
  double dsdv;         // (B - 4) / (hi - lo), fp64
};

constexpr int kParzenQGroup = 2;  // entropies per backward sweep

// Wave tiles of the Parzen walks (kTileX x kTileY fixed voxels, one wave
// step): bit g of a tile's mask is set when a voxel of the tile has a slot
// in [8 g, 8 g + 8).  A band's walk skips the tiles whose mask holds none
// of its slots, so every band but the background's skips the background.
constexpr int kSlotGroup = 8;
inline int64_t parzen_tiles(int32_t nx, int32_t ny, int32_t nz) {
  return (int64_t)((ny + kTileY - 1) / kTileY) * nz * ((nx + kTileX - 1) / kTileX);
}
// Row groups (kTileY rows of one slice): each also gets the OR of its
// tiles' masks, stored after the tile masks, so that a band's walk skips a
// row group without any of its slots in one test (in a CT nearly every
// voxel is background, so the other bands find their slots in a fifth of
// the row groups and a few percent of the tiles).
inline int64_t parzen_row_groups(int32_t ny, int32_t nz) { return (int64_t)((ny + kTileY - 1) / kTileY) * nz; }
__host__ __device__ inline uint32_t slot_group_mask(int32_t r_lo, int32_t r_hi) {
  const int32_t g0 = r_lo / kSlotGroup, g1 = (r_hi - 1) / kSlotGroup;  // r_hi > r_lo
  return (g1 >= 31 ? 0xFFFFFFFFu : ((2u << g1) - 1u)) & ~((1u << g0) - 1u);
}

// Forward sweeps: the background row (slot 0, the lowest occupied fixed
// bin: air in a CT) receives most voxels, all into a few cells.  Its first
// parzen_hot_cols(B) columns get kHotCopies private copies in LDS, lane l
// adding into copy l % kHotCopies; each copy is one cell longer than the
// columns it covers, so the same column of consecutive copies falls in
// different LDS banks.
constexpr int kHotCopies = 16;
// Row pitch (cells) of the Parzen sweeps' LDS tables: the band's B columns
// and a pad of 3, so that one column of consecutive rows falls 3 (fp32
// cells) or 6 (64-bit cells) banks apart, not in one bank as with a pitch
// of B (a multiple of 32 words for the usual bin counts).
__host__ __device__ inline int32_t parzen_pitch(int32_t bins) { return bins + 3; }
constexpr int kHotCols = 64;
__host__ __device__ inline int32_t parzen_hot_cols(int32_t bins) { return bins < kHotCols ? bins : kHotCols; }
__host__ __device__ inline int32_t parzen_hot_stride(int32_t bins) { return parzen_hot_cols(bins) + 1; }
__host__ __device__ inline int32_t parzen_hot_cells(int32_t bins) { return kHotCopies * parzen_hot_stride(bins); }


struct ParzenLaunch {
  ParzenArgs args;
  int32_t float_quads;  // 1: moving volume is fp32 (float4 quads, else uint4 octs)
  int32_t clamp;
  int32_t block;        // threads per workgroup of the sweeps: 256, 512 or 1024
};

// LDS guard of every launch with dynamic LDS: the kernel's static LDS (read
// once with hipFuncGetAttributes) plus `dynamic` must fit the device's
// per-workgroup maximum, and `dynamic` the maximum the kernel was
// configured for (hipErrorInvalidValue otherwise; nothing is launched).
// lds_register() records a kernel's static LDS and the device maximum at
// configuration; lds_guard() looks up kernels it has not seen.
hipError_t lds_register(const void* kernel);
// at_zero: the kernel addresses its dynamic LDS from address 0, so it must
// keep no static LDS.
hipError_t lds_guard(const void* kernel, size_t dynamic, size_t configured_max, bool at_zero = false);

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t value, hipStream_t s);
// Index-space matrices M[n][12] of the caller's physical matrices P[n][12].
hipError_t launch_compose(const double* P, int64_t n, const Geometry& g, double* M, hipStream_t s);
// d MI / d P from d MI / d M in place, rows of 12 (gradients of `rows`
// transform-entropy pairs): G_P[r][c] = (G_M[r][c] fsp[c] + G_M[r][3] forg[c]) / msp[r],
// G_P[r][3] = G_M[r][3] / msp[r].
hipError_t launch_grad_physical(double* grad, int64_t rows, const Geometry& g, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, hipStream_t s);
hipError_t launch_prebin_fixed(const VolumeDesc& f, int bins, uint8_t* out, hipStream_t s);
hipError_t launch_pack_octs(const VolumeDesc& m, uint4* out, hipStream_t s);
hipError_t launch_pack_oct8(const VolumeDesc& m, uint2* out, hipStream_t s);
hipError_t launch_hist_hard(const HardLaunch& L, hipStream_t s);
// Random subsampling (sample.hip): the kept fixed voxels as list entries
// {x | y << 12 | fixed bin << 24, z}; n_list must be zero beforehand.
hipError_t launch_sample_list(const uint8_t* fbins, int32_t nx, int32_t ny, int32_t nz, double fraction,
                              uint64_t seed, uint2* list, unsigned long long* n_list, hipStream_t s);
hipError_t launch_hist_sampled(const HardLaunch& L, const uint2* list, const unsigned long long* n_list,
                               hipStream_t s);

// Many fixed/moving pairs of uneven sizes (see pairs.hip).
struct PairDesc {
  const void* fixed;
  const void* moving;
  const double* transforms;  // caller's [n_t][12], physical
  Geometry geo;              // the pair's spacings and origins
  HardGeom geom;             // fbins / octs point into the workspace
  int32_t fdtype, mdtype;
  double flo, fhi;           // fixed range (fp64 rule for float fixed volumes)
  int32_t mlo, mhi;          // moving range
  Divider fdiv;              // floor(X / R_fixed)
  int32_t n_t, chunks;       // transforms, slabs (a multiple of 8)
};

// Pairs' preparation, one wave per item: fixed volumes in chunks of
// consecutive voxels (16 per lane); moving volumes in runs of kPrepPlaneRun
// voxels of an xy plane (two per lane) through blocks of kPrepSlices slices.
constexpr int kPrepFixedLane = 16, kPrepFixedChunk = 64 * kPrepFixedLane;
constexpr int kPrepPlaneRun = 128, kPrepSlices = 8;

struct PairsArgs {
  const PairDesc* pairs;
  int32_t n_pairs;
  const int64_t* fchunk_base;  // [P+1] prefix of kPrepFixedChunk-voxel chunks of the fixed volumes
  const int64_t* mchunk_base;  // [P+1] prefix of (plane run, slice block) items of the moving volumes
  const int64_t* t_base;     // [P+1] prefix of transforms
  const int64_t* xcd_base;   // [8][P+1] prefix of work items per XCD
  unsigned long long* counters;  // [8] work-queue heads
  double* transforms;        // [T][12], gathered and composed to index space
  uint32_t* hist;            // [T][B][B]
  int32_t bins;
  int32_t transform_major;   // work-item order within a pair: 0 slab-major, 1 transform-major
};

struct PairsLaunch {
  PairsArgs args;
  int64_t total_t, fixed_chunks, moving_chunks;
  int32_t clamp, packed, cu_count;
  int32_t block;  // threads per workgroup of the sweep: 256, 512 or 1024
  int32_t oct8;  // every pair's moving volume packed with 8-bit corners
};

// The transforms gathered and composed; with `volumes` also the pairs'
// fixed bins and oct volumes.
hipError_t launch_pairs_prep(const PairsLaunch& L, hipStream_t s, bool volumes = true);
hipError_t launch_pairs_hist(const PairsLaunch& L, hipStream_t s);
HardGeom make_hard_geom(const VolumeDesc& fixed, const VolumeDesc& moving, const uint8_t* fbins,
                        const void* octs, int32_t bins);
hipError_t launch_mi_reduce(const ReduceLaunch& L, hipStream_t s);
hipError_t launch_pack_quads_f32(const VolumeDesc& m, float4* out, hipStream_t s);
hipError_t launch_pack_quads16(const VolumeDesc& m, uint2* out, hipStream_t s);
hipError_t launch_row_map(uint8_t* fbins, size_t nvox, int32_t bins, RowMap* m, hipStream_t s);
// Tile masks of the slotted fixed volume (see kSlotGroup).
hipError_t launch_tile_mask(const uint8_t* slots, int32_t nx, int32_t ny, int32_t nz, uint32_t* mask, hipStream_t s);
hipError_t launch_parzen_fwd(const ParzenLaunch& L, hipStream_t s);
hipError_t launch_parzen_sampled_fwd(const ParzenLaunch& L, const uint2* list, const unsigned long long* n_list,
                                     hipStream_t s);
hipError_t launch_dmi_dp(const ParzenLaunch& L, const QList& q, hipStream_t s);
hipError_t launch_parzen_bwd(const ParzenLaunch& L, hipStream_t s);
hipError_t launch_lds_atomic_probe(uint32_t* out, int32_t blocks, int32_t iters, hipStream_t s);

}  // namespace gemi
