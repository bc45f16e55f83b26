// Host side of libgemi.so: argument validation, workspace layout, launch
// planning and dispatch for the C ABI declared in include/gemi.h.
#include "../../include/gemi.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "paths.h"

namespace gemi {
hipError_t configure_hard_kernels();
hipError_t configure_parzen_kernels();
hipError_t scratch_setup(int device);
void* scratch_device_ptr(int device);
}  // namespace gemi

using namespace gemi;

namespace {

constexpr int kTimers = 5;

struct EventPair {
  hipEvent_t start, stop;
};

thread_local std::string g_last_hip;

int hip_fail(hipError_t e, const char* where) {
  g_last_hip = std::string(where) + ": " + hipGetErrorString(e);
  return MI_ERR_HIP;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t voxels(const mi_volume* v) { return (size_t)v->nx * v->ny * v->nz; }

int check_volume(const mi_volume* v, bool need_integer) {
  if (!v || !v->data) return MI_ERR_NULL;
  if (v->dtype < MI_U8 || v->dtype > MI_F32) return MI_ERR_DTYPE;
  if (need_integer && v->dtype == MI_F32) return MI_ERR_DTYPE;
  const int32_t n[3] = {v->nx, v->ny, v->nz};
  for (int r = 0; r < 3; ++r)
    if (n[r] < 2 || n[r] > MI_MAX_EDGE) return MI_ERR_DIMS;
  if (voxels(v) > ((size_t)1 << 28)) return MI_ERR_DIMS;
  for (int r = 0; r < 3; ++r)
    if (!isfinite(v->spacing[r]) || !(v->spacing[r] > 0.0) || !isfinite(v->origin[r])) return MI_ERR_GEOMETRY;
  if (!isfinite(v->lo) || !isfinite(v->hi) || !(v->hi > v->lo)) return MI_ERR_RANGE;
  if (v->dtype != MI_F32) {
    if (v->lo != floor(v->lo) || v->hi != floor(v->hi)) return MI_ERR_RANGE;
    if (fabs(v->lo) > 2147483647.0 || fabs(v->hi) > 2147483647.0) return MI_ERR_RANGE;
    if (v->hi - v->lo + 1.0 > 65536.0) return MI_ERR_RANGE;
  }
  return MI_OK;
}

int check_q(const double* q, int32_t n_q) {
  if (n_q < 1 || n_q > MI_MAX_Q) return MI_ERR_Q;
  if (!q) return MI_ERR_NULL;
  for (int i = 0; i < n_q; ++i)
    if (!isfinite(q[i]) || !(q[i] > 0.0)) return MI_ERR_Q;
  return MI_OK;
}

// Bytes of the moving volume's gather layout on the Parzen path: fp32
// quads for float volumes; for integer ones 16-bit quads on full sweeps and
// 16-bit octs on sampled sweeps (one cache line per random sample).
size_t parzen_gather_bytes(const mi_volume* m, bool sampled = false) {
  if (m->dtype == MI_F32) return quad_f32_bytes(m->nx, m->ny, m->nz);
  return sampled ? oct_volume_bytes(m->nx, m->ny, m->nz) : quad16_bytes(m->nx, m->ny, m->nz);
}

// The largest gather layout any path uses for the volume (the hard path's
// 16-bit oct volume for integer volumes).
size_t gather_bytes(const mi_volume* m) {
  return m->dtype == MI_F32 ? quad_f32_bytes(m->nx, m->ny, m->nz)
                            : std::max(oct_volume_bytes(m->nx, m->ny, m->nz), quad16_bytes(m->nx, m->ny, m->nz));
}

// Bytes of the hard path's oct volume: 8-bit corners when the range allows.
size_t hard_gather_bytes(const mi_volume* m) {
  return oct8_range(m->lo, m->hi) ? oct8_volume_bytes(m->nx, m->ny, m->nz)
                                  : oct_volume_bytes(m->nx, m->ny, m->nz);
}

// A moving volume whose gather layout needs 32-bit buffer offsets beyond
// 4 GiB is refused (fewer than 2^28 voxels for integer volumes).
int check_moving(const mi_volume* m, bool need_integer) {
  const int st = check_volume(m, need_integer);
  if (st != MI_OK) return st;
  return gather_bytes(m) > kMaxGatherBytes ? MI_ERR_DIMS : MI_OK;
}

constexpr int32_t kKnownFlags = MI_BOUNDARY_CLAMP | MI_TSALLIS_PSEUDOADDITIVE | MI_HIST_PARZEN | MI_USE_GRAPH |
                                MI_VOLUMES_UNCHANGED | MI_SAMPLED | MI_COMPACT_SLABS | MI_GRADIENT;

// Random subsampling of the fixed volume (mi_eval_sampled).
struct SampleSpec {
  double fraction;  // share of fixed voxels kept (>= 1: all)
  uint64_t seed;
};

int check_fraction(double fraction) { return (isfinite(fraction) && fraction > 0.0) ? MI_OK : MI_ERR_SAMPLE; }

int check_common(const mi_volume* f, const mi_volume* m, int32_t n, int32_t bins, const double* q,
                 int32_t n_q, int32_t flags, bool parzen) {
  if (flags & ~kKnownFlags) return MI_ERR_FLAGS;
  int st;
  if ((st = check_volume(f, false)) != MI_OK) return st;
  if ((st = check_moving(m, !parzen)) != MI_OK) return st;
  if (n < 0 || n > (1 << 24)) return MI_ERR_COUNT;
  if (bins < (parzen ? 8 : 2) || bins > 256) return MI_ERR_BINS;
  if (q != nullptr || n_q != 0) {
    if ((st = check_q(q, n_q)) != MI_OK) return st;
  }
  return MI_OK;
}

// Workspace layout (each region 256-byte aligned):
//   index-space matrices f64[n][12] (the caller's physical ones composed)
//   fixed bins   u8[nvox_fixed]
//   hard:        moving oct volume u16x8[mnz][mny][mnx],
//                hist u32[n][B][B]          (only when the caller passes no hist_out)
//                count u64[n], MI partial sums (reduce_part_bytes)
//   Parzen:      moving oct volume (integer moving volume) or f32x4 quad
//                volume [mnz+1][mny][mnx] (float moving volume),
//                occupied-row map, wave-tile slot masks u32[tiles] and
//                their per-row-group ORs u32[row groups],
//                table f64[n][B][B], count u64[n]
//                MI partial sums (reduce_part_bytes)
//   Parzen grad: + table marginals f64[n][2B], dMI/dp tables f32[n][n_q][B][B]
//   sampled:     + sample list u32x2[nvox_fixed] and its length u64
struct Layout {
  size_t xf = 0, order = 0, fbins = 0, gvol = 0, hist = 0, rowmap = 0, tmask = 0, table = 0, count = 0, part = 0,
         marg = 0, gtab = 0, list = 0, nlist = 0, total = 0;
};


Layout layout(const mi_volume* f, const mi_volume* m, int32_t n, int32_t bins, int32_t n_q,
              bool parzen, bool grad, bool need_hist, bool sampled = false) {
  Layout L;
  size_t off = 0;
  L.xf = off;
  off += align256(96 * (size_t)n);
  L.order = off;  // the hard sweep's processing order
  off += align256(4 * (size_t)n);
  L.fbins = off;
  off += align256(voxels(f));
  const size_t bb = (size_t)bins * bins;
  if (!parzen) {
    L.gvol = off;
    off += align256(hard_gather_bytes(m));
    L.hist = off;
    if (need_hist) off += align256(bb * 4 * (size_t)n);
    L.count = off;
    off += align256(8 * (size_t)n);
    L.part = off;
    off += align256(reduce_part_bytes(n, bins, n_q));
  } else {
    L.gvol = off;
    off += align256(parzen_gather_bytes(m, sampled));
    L.rowmap = off;
    off += align256(sizeof(RowMap));
    L.tmask = off;
    off += align256(4 * (size_t)(parzen_tiles(f->nx, f->ny, f->nz) + parzen_row_groups(f->ny, f->nz)));
    L.table = off;
    off += align256(bb * 8 * (size_t)n);
    L.count = off;
    off += align256(8 * (size_t)n);
    L.part = off;
    off += align256(reduce_part_bytes(n, bins, n_q));
    if (grad) {
      L.marg = off;
      off += align256(16 * (size_t)bins * n);
      L.gtab = off;
      off += align256(bb * 4 * (size_t)n * n_q);
    }
  }
  if (sampled) {
    L.list = off;
    off += align256(8 * voxels(f));
    L.nlist = off;
    off += 256;
  }
  L.total = off;
  return L;
}

VolumeDesc desc(const mi_volume* v) {
  VolumeDesc d;
  d.data = v->data;
  d.nx = v->nx;
  d.ny = v->ny;
  d.nz = v->nz;
  d.dtype = v->dtype;
  d.lo = v->lo;
  d.hi = v->hi;
  return d;
}

Geometry geometry(const mi_volume* f, const mi_volume* m) {
  Geometry g;
  for (int r = 0; r < 3; ++r) {
    g.fsp[r] = f->spacing[r];
    g.forg[r] = f->origin[r];
    g.msp[r] = m->spacing[r];
    g.morg[r] = m->origin[r];
  }
  return g;
}

QList qlist(const double* q, int32_t n_q, int32_t flags) {
  QList L;
  memset(&L, 0, sizeof L);
  for (int i = 0; i < n_q; ++i) L.q[i] = q[i];
  L.n = n_q;
  L.pseudo = (flags & MI_TSALLIS_PSEUDOADDITIVE) ? 1 : 0;
  return L;
}

}  // namespace

constexpr size_t kStageBytes = 4u << 20;  // pinned staging for the pairs' tables

// Launch shape of the hard-binned sweep for one problem class.
struct HardTune {
  int32_t block = 1024;
  int32_t slab_major = 1;
  int32_t chunks = 0;   // 0 = planned per call
  int32_t packed = -1;  // LDS counters: -1 by bins (packed above 128), 0 u32, 1 two 16-bit per word
};

// LDS counter layout of a launch: packed is forced above 128 bins (a u32
// histogram would not fit), chosen by the tuning otherwise.
bool use_packed(const HardTune& t, int32_t bins) { return bins > 128 || t.packed == 1; }

// Launch shape of the persistent multi-pair sweep: workgroup size, voxels
// per slab (a work item sweeps one slab for one transform), LDS counter
// layout and the order of a pair's work items.  Results do not depend on it.
struct PairsTune {
  int32_t block = 512;
  int32_t slab_voxels = 131072;  // capped at 65535 with 16-bit counters
  int32_t packed = -1;           // -1 by bins (packed above 128), 0 u32, 1 two 16-bit per word
  int32_t transform_major = 0;
};

// Launch shape of the Parzen sweeps, forward and backward each: workgroup
// size and LDS budget per workgroup (the table's rows are split into bands
// that fit it; fewer, larger bands mean fewer walks over the fixed volume
// at one workgroup per CU); and workgroups per transform and band, as a
// power-of-two multiple of the planned count.  Results vary only by the
// merge order of workgroup partial sums (last bits).
struct ParzenTune {
  int32_t fwd_block = 512, fwd_lds_kib = 64;  // 256/512/1024; 16, 32, 64, 96 or 128
  int32_t bwd_block = 512, bwd_lds_kib = 64;
  int32_t chunk_shift = 0;  // -1, 0, 1, 2: half, as planned, twice, four times the workgroups
};

// The untuned shape.  Up to 64 bins a table fits one 64 KiB band, and
// 512-thread workgroups (two per CU) were fastest on the 128^3, 64-bin
// gradient (1.00 ms a call against 1.16 ms with 1024 threads and 128 KiB);
// above it, fewer, larger bands at one 1024-thread workgroup per CU were
// fastest on the 512x512x300 / 256^3, 256-bin CT/MR gradient: 128 KiB for
// both sweeps, 1.26 ms an iteration (forward 0.56, backward 0.62 ms)
// against 1.82 ms with 96 KiB and 1.88 ms with 64 KiB; and twice the
// planned workgroups, 1.17 ms (half: 1.44 ms).
ParzenTune parzen_shape_for_bins(int32_t bins) {
  ParzenTune t;
  if (bins > 64) {
    t.fwd_block = t.bwd_block = 1024;
    t.fwd_lds_kib = 128;
    t.bwd_lds_kib = 128;
    t.chunk_shift = 1;
  }
  return t;
}

// Problem class of the tuning cache.
struct TuneKey {
  int32_t v[11];
  bool operator==(const TuneKey& o) const { return memcmp(v, o.v, sizeof v) == 0; }
};

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraphExec_t exec;
};

constexpr size_t kMaxGraphs = 16;

struct mi_context {
  std::vector<uint64_t> last_prep;  // path, workspace, volumes and bins of the last preparation
  void* stage = nullptr;            // pinned host buffer, kStageBytes
  hipEvent_t stage_done = nullptr;  // recorded after the last copy out of `stage`
  bool stage_pending = false;
  int device = 0;
  int cu_count = 256;
  HardTune hard_default;  // launch shape when no tuned entry matches
  bool timing = false;
  std::mutex mu;
  std::vector<EventPair> events[kTimers];
  std::vector<std::pair<TuneKey, HardTune>> tuned;  // from mi_tune or the cache file
  std::vector<std::pair<TuneKey, PairsTune>> pairs_tuned;  // from mi_tune_pairs or the cache file
  std::vector<std::pair<TuneKey, ParzenTune>> parzen_tuned;  // from mi_tune (Parzen) or the cache file
  bool parzen_env = false;    // MI_TUNE_PARZEN_* set: parzen_default replaces the shape by bins
  ParzenTune parzen_default;  // launch shape when no tuned entry matches (with parzen_env)
  std::vector<uint64_t> last_pairs_prep;  // pairs, bins and workspace of the last pairs preparation
  std::string tune_file;                            // MI_TUNE_CACHE, if set
  std::vector<GraphEntry> graphs;                   // MI_USE_GRAPH replays, oldest first
};

namespace {

// Key of a per-call preparation (path, workspace, both volumes, bins).
std::vector<uint64_t> prep_key(int path, const void* ws, const mi_volume* f, const mi_volume* m, int32_t bins) {
  std::vector<uint64_t> k = {(uint64_t)path, (uint64_t)(uintptr_t)ws, (uint64_t)bins};
  for (const mi_volume* v : {f, m}) {
    uint64_t lo, hi;
    memcpy(&lo, &v->lo, 8);
    memcpy(&hi, &v->hi, 8);
    k.insert(k.end(), {(uint64_t)(uintptr_t)v->data, (uint64_t)v->nx, (uint64_t)v->ny, (uint64_t)v->nz,
                       (uint64_t)v->dtype, lo, hi});
  }
  return k;
}

// True when the caller allows reuse and the workspace already holds this
// preparation; otherwise records the preparation about to be made.
bool reuse_prep(mi_context* ctx, int32_t flags, std::vector<uint64_t> key) {
  if ((flags & MI_VOLUMES_UNCHANGED) && key == ctx->last_prep) return true;
  ctx->last_prep = std::move(key);
  return false;
}

// Brackets one kernel launch with timing events when timing is enabled.
struct TimedLaunch {
  mi_context* ctx;
  int which;
  hipStream_t stream;
  EventPair ev{nullptr, nullptr};
  TimedLaunch(mi_context* c, int w, hipStream_t s) : ctx(c), which(w), stream(s) {
    if (!ctx->timing) return;
    if (hipEventCreate(&ev.start) != hipSuccess || hipEventCreate(&ev.stop) != hipSuccess) {
      ev.start = ev.stop = nullptr;
      return;
    }
    (void)hipEventRecord(ev.start, stream);
  }
  void done() {
    if (!ev.start) return;
    (void)hipEventRecord(ev.stop, stream);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->events[which].push_back(ev);
    ev.start = ev.stop = nullptr;
  }
};

// Slabs per transform that keep one slab's share of the moving gather
// volume near 1.5 MiB: the workgroups of an XCD sweep one slab for many
// transforms at once, and their moving footprint must stay in the XCD's
// 4 MiB L2 (on the 1000-transform 256x256x180 sweep, 128 slabs instead of
// 32 cut the L2 miss traffic and the sweep time by 8%).
int64_t l2_slabs(size_t gather_volume_bytes) {
  const int64_t target = 3 << 19;  // 1.5 MiB
  const int64_t c = ((int64_t)gather_volume_bytes + target - 1) / target;
  return c < 32 ? 32 : c;
}

// Workgroups per transform for the histogram sweep.  The fixed volume is
// swept in groups of 4 rows; a transform's groups are split into `c`
// slabs: enough workgroups to fill the chip several times over, in
// slab-major order enough thin slabs that a slab's moving footprint fits
// an XCD's L2 (l2_slabs), a multiple of 8 (one share per XCD), and -- with
// 16-bit packed LDS counters -- few enough voxels per workgroup that no
// counter can exceed 65535.
int plan_chunks(const mi_context* ctx, const mi_volume* f, const mi_volume* m, int32_t n,
                bool packed, const HardTune& tune) {
  const int64_t groups = (int64_t)((f->ny + 3) / 4) * f->nz;
  int64_t c;
  if (tune.chunks) {
    c = tune.chunks;
  } else {
    c = ((int64_t)ctx->cu_count * 8 + n - 1) / n;
    const int64_t l2 = l2_slabs(hard_gather_bytes(m));
    if (tune.slab_major && c < l2) c = l2;
  }
  if (c > groups) c = groups;
  if (packed) {
    const int64_t per = 65535 / (4 * (int64_t)f->nx);  // groups per workgroup
    const int64_t need = (groups + per - 1) / per;
    if (c < need) c = need;
  }
  c = ((c + 7) / 8) * 8;
  return (int)c;
}


// Workgroups per transform and band for the Parzen sweeps (as plan_chunks).
int plan_parzen_chunks(const mi_context* ctx, const mi_volume* f, const mi_volume* m, int64_t units) {
  const int64_t groups = (int64_t)((f->ny + 3) / 4) * f->nz;
  int64_t c = ((int64_t)ctx->cu_count * 8 + units - 1) / units;
  const int64_t l2 = l2_slabs(parzen_gather_bytes(m));
  if (c < l2) c = l2;
  if (c > groups) c = groups;
  return (int)(((c + 7) / 8) * 8);
}

// Workgroups per transform (and band) for a sampled sweep over about
// `expected` samples: enough to fill the chip, but at least ~4096 samples
// per workgroup so that zeroing and flushing its LDS table stay small; a
// multiple of 8 (one share per XCD).
int plan_sampled_chunks(const mi_context* ctx, int64_t expected, int64_t units) {
  int64_t c = ((int64_t)ctx->cu_count * 8 + units - 1) / units;
  const int64_t cap = std::max<int64_t>(8, expected / 4096);
  if (c > cap) c = cap;
  if (c < 8) c = 8;
  c = ((c + 7) / 8) * 8;
  return (int)std::min<int64_t>(c, 1 << 20);
}

int64_t expected_samples(const mi_volume* f, const SampleSpec& smp) {
  const double nv = (double)voxels(f);
  return smp.fraction >= 1.0 ? (int64_t)nv : (int64_t)ceil(smp.fraction * nv);
}

// Rows of the table per band when `tables` fp32 tables of `bins` columns
// (rows padded to parzen_pitch) share an LDS budget of `budget` bytes.
int32_t band_rows_for(int32_t bins, int32_t tables, int32_t budget) {
  int32_t r = (int32_t)(budget / (4 * parzen_pitch(bins) * tables));
  return r < 1 ? 1 : (r < bins ? r : bins);
}

// Problem class of a Parzen call: volume shapes, moving dtype, bins,
// boundary, the power-of-two bucket of n and whether it is a gradient call.
TuneKey parzen_tune_key(const mi_volume* f, const mi_volume* m, int32_t n, int32_t bins, int32_t flags) {
  TuneKey k;
  int32_t nb = 0;
  while ((1 << nb) < n && nb < 30) ++nb;
  const int32_t v[11] = {-2, f->nx, f->ny, f->nz, m->nx, m->ny, m->nz, m->dtype, bins,
                         (flags & MI_BOUNDARY_CLAMP) ? 1 : 0, nb};
  memcpy(k.v, v, sizeof v);
  return k;
}

ParzenTune parzen_tune_for(const mi_context* ctx, const mi_volume* f, const mi_volume* m, int32_t n, int32_t bins,
                           int32_t flags) {
  const TuneKey k = parzen_tune_key(f, m, n, bins, flags);
  for (const auto& e : ctx->parzen_tuned)
    if (e.first == k) return e.second;
  return ctx->parzen_env ? ctx->parzen_default : parzen_shape_for_bins(bins);
}

// The Parzen path: forward table, MI, and (grad_out != NULL) the gradient.
int run_parzen(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
               const double* transforms, int32_t n, int32_t bins, const double* q, int32_t n_q,
               int32_t flags, double* mi_out, uint64_t* overlap_out, double* grad_out, char* ws,
               const Layout& L, hipStream_t s, const SampleSpec* smp = nullptr,
               const ParzenTune* tune_override = nullptr) {
  const ParzenTune tune = tune_override ? *tune_override : parzen_tune_for(ctx, fixed, moving, n, bins, flags);
  hipError_t e;
  // the caller's physical matrices -> index-space matrices in the workspace
  {
    double* M = (double*)(ws + L.xf);
    if ((e = launch_compose(transforms, n, geometry(fixed, moving), M, s)) != hipSuccess)
      return hip_fail(e, "compose");
    transforms = M;
  }
  uint8_t* fb = (uint8_t*)(ws + L.fbins);
  RowMap* rows = (RowMap*)(ws + L.rowmap);
  const bool fq = moving->dtype == MI_F32;
  void* gvol = ws + L.gvol;
  // a sampled call always prepares (its list is not part of the record)
  if (smp || !reuse_prep(ctx, flags, prep_key(2, ws, fixed, moving, bins))) {
    if ((e = launch_prebin_fixed(desc(fixed), bins, fb, s)) != hipSuccess) return hip_fail(e, "prebin");
    if ((e = launch_row_map(fb, voxels(fixed), bins, rows, s)) != hipSuccess) return hip_fail(e, "row map");
    if ((e = launch_tile_mask(fb, fixed->nx, fixed->ny, fixed->nz, (uint32_t*)(ws + L.tmask), s)) != hipSuccess)
      return hip_fail(e, "tile mask");
    e = fq  ? launch_pack_quads_f32(desc(moving), (float4*)gvol, s)
        : smp ? launch_pack_octs(desc(moving), (uint4*)gvol, s)
              : launch_pack_quads16(desc(moving), (uint2*)gvol, s);
    if (e != hipSuccess) return hip_fail(e, "pack");
  }
  uint2* list = (uint2*)(ws + L.list);
  unsigned long long* nlist = (unsigned long long*)(ws + L.nlist);
  if (smp) {
    ctx->last_prep.clear();
    if ((e = launch_fill_u32((uint32_t*)nlist, 2, 0u, s)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_sample_list(fb, fixed->nx, fixed->ny, fixed->nz, smp->fraction, smp->seed, list, nlist, s)) !=
        hipSuccess)
      return hip_fail(e, "sample list");
  }
  const size_t bb = (size_t)bins * bins;
  double* table = (double*)(ws + L.table);
  uint64_t* count = (uint64_t*)(ws + L.count);
  if ((e = launch_fill_f64(table, bb * n, s)) != hipSuccess) return hip_fail(e, "fill");
  if ((e = launch_fill_u32((uint32_t*)count, 2 * (size_t)n, 0u, s)) != hipSuccess) return hip_fail(e, "fill");
  if (grad_out && (e = launch_fill_f64(grad_out, (size_t)n * n_q * 12, s)) != hipSuccess)
    return hip_fail(e, "fill");

  ParzenLaunch P;
  memset(&P, 0, sizeof P);
  ParzenArgs& a = P.args;
  a.transforms = transforms;
  a.fbins = fb;
  a.rows = rows;
  a.tile_mask = (const uint32_t*)(ws + L.tmask);
  a.row_mask = a.tile_mask + parzen_tiles(fixed->nx, fixed->ny, fixed->nz);
  a.gvol = gvol;
  a.table = table;
  a.count = count;
  a.gtab = (const float*)(ws + L.gtab);
  a.grad = grad_out;
  a.fnx = fixed->nx;
  a.fny = fixed->ny;
  a.fnz = fixed->nz;
  a.mnx = moving->nx;
  a.mny = moving->ny;
  a.mnz = moving->nz;
  a.gvol_bytes = (uint32_t)parzen_gather_bytes(moving, smp != nullptr);
  a.n = n;
  a.bins = bins;
  a.slab_major = 1;
  a.n_q = n_q;
  a.sscale = (float)((double)(bins - 4) / (moving->hi - moving->lo));
  a.dsdv = (double)(bins - 4) / (moving->hi - moving->lo);
  P.float_quads = fq ? 1 : 0;
  P.clamp = (flags & MI_BOUNDARY_CLAMP) ? 1 : 0;

  // one launch covers at most 2^31 - 1 workgroups: split the transforms
  auto sweep = [&](bool backward, int which) -> int {
    ParzenLaunch part = P;
    ParzenArgs& pa = part.args;
    part.block = backward ? tune.bwd_block : tune.fwd_block;
    // backward: kParzenQGroup fp32 tables; forward: one table of 8-byte cells
    // plus the copies of the background row's hot columns
    const int32_t budget = (backward ? tune.bwd_lds_kib : tune.fwd_lds_kib) * 1024;
    pa.band_rows = backward ? band_rows_for(bins, kParzenQGroup, budget)
                            : std::min(bins, std::max(1, (budget / 8 - parzen_hot_cells(bins)) / parzen_pitch(bins)));
    pa.bands = (bins + pa.band_rows - 1) / pa.band_rows;
    int64_t chunks = smp ? plan_sampled_chunks(ctx, expected_samples(fixed, *smp), (int64_t)n * pa.bands)
                         : plan_parzen_chunks(ctx, fixed, moving, (int64_t)n * pa.bands);
    if (tune.chunk_shift > 0) chunks <<= tune.chunk_shift;
    if (tune.chunk_shift < 0) chunks = std::max<int64_t>(8, ((chunks / 2 + 7) / 8) * 8);
    pa.chunks = (int32_t)std::min<int64_t>(chunks, 1 << 24);
    const int64_t per_launch = 0x7FFFFFFFll / ((int64_t)pa.chunks * pa.bands);
    for (int64_t t0 = 0; t0 < n; t0 += per_launch) {
      pa.n = (int32_t)(n - t0 < per_launch ? n - t0 : per_launch);
      pa.transforms = transforms + 12 * t0;
      pa.table = table + bb * t0;
      pa.count = count + t0;
      pa.gtab = (const float*)(ws + L.gtab) + bb * n_q * t0;
      pa.grad = grad_out ? grad_out + (size_t)n_q * 12 * t0 : nullptr;
      TimedLaunch tl(ctx, which, s);
      hipError_t err = backward ? launch_parzen_bwd(part, s)
                       : smp      ? launch_parzen_sampled_fwd(part, list, nlist, s)
                                  : launch_parzen_fwd(part, s);
      if (err != hipSuccess) return hip_fail(err, backward ? "parzen_bwd" : "parzen_fwd");
      tl.done();
    }
    return MI_OK;
  };
  int st;
  if ((st = sweep(false, 1)) != MI_OK) return st;

  ReduceLaunch R;
  memset(&R, 0, sizeof R);
  R.table = table;
  R.count = count;
  R.part = (double*)(ws + L.part);
  R.marg_out = grad_out ? (double*)(ws + L.marg) : nullptr;
  P.args.marg = R.marg_out;
  R.transforms = transforms;
  R.n = n;
  R.bins = bins;
  R.q = qlist(q, n_q, flags);
  R.mi_out = mi_out;
  R.overlap_out = overlap_out;
  TimedLaunch tr(ctx, 4, s);
  if ((e = launch_mi_reduce(R, s)) != hipSuccess) return hip_fail(e, "mi_reduce");
  tr.done();
  if (!grad_out) return MI_OK;

  if ((e = launch_dmi_dp(P, R.q, s)) != hipSuccess) return hip_fail(e, "dmi_dp");
  for (int32_t q0 = 0; q0 < n_q; q0 += kParzenQGroup) {
    P.args.q0 = q0;
    if ((st = sweep(true, 2)) != MI_OK) return st;
  }
  // d MI / d M (index space) -> d MI / d P (the caller's physical entries)
  if ((e = launch_grad_physical(grad_out, (int64_t)n * n_q, geometry(fixed, moving), s)) != hipSuccess)
    return hip_fail(e, "grad chain rule");
  return MI_OK;
}


// Layout and work split of a multi-pair call (hard histograms).
struct PairsPlan {
  size_t tables = 0, table_bytes = 0, counters = 0, transforms = 0, hist = 0, count = 0, part = 0, total = 0;
  size_t off_desc = 0, off_frow = 0, off_mrow = 0, off_tbase = 0, off_xcd = 0;
  std::vector<size_t> fbins, octs;
  std::vector<int32_t> chunks;
  std::vector<int64_t> fchunk_base, mchunk_base, t_base, xcd_base;  // xcd_base: [8][P+1]
  int64_t total_t = 0;
  bool oct8 = true;    // every moving range <= 256: 8-bit corners for all pairs
  bool packed = false;  // 16-bit LDS counters
};

int plan_pairs(const mi_pair* pairs, int32_t n_pairs, int32_t bins, int32_t n_q, int32_t flags,
               PairsPlan& plan, const PairsTune& tune = PairsTune()) {
  if (flags & ~(MI_BOUNDARY_CLAMP | MI_TSALLIS_PSEUDOADDITIVE | MI_USE_GRAPH | MI_VOLUMES_UNCHANGED))
    return MI_ERR_FLAGS;
  if (n_pairs < 0 || n_pairs > (1 << 24)) return MI_ERR_COUNT;
  if (n_pairs > 0 && !pairs) return MI_ERR_NULL;
  if (bins < 2 || bins > 256) return MI_ERR_BINS;
  if (n_q < 1 || n_q > MI_MAX_Q) return MI_ERR_Q;
  const int P = n_pairs;
  plan.fbins.resize(P);
  plan.octs.resize(P);
  plan.chunks.resize(P);
  plan.fchunk_base.assign(P + 1, 0);
  plan.mchunk_base.assign(P + 1, 0);
  plan.t_base.assign(P + 1, 0);
  plan.xcd_base.assign(8 * (size_t)(P + 1), 0);
  const bool packed = bins > 128 || tune.packed == 1;
  plan.packed = packed;
  for (int p = 0; p < P; ++p) {
    const mi_pair& pr = pairs[p];
    int st;
    if ((st = check_volume(&pr.fixed, false)) != MI_OK) return st;
    if ((st = check_moving(&pr.moving, true)) != MI_OK) return st;
    if (pr.n_transforms < 0) return MI_ERR_COUNT;
    if (pr.n_transforms > 0 && !pr.transforms) return MI_ERR_NULL;
    // slabs of about tune.slab_voxels voxels (at most 65535 with 16-bit
    // counters), 8 or more, a multiple of 8
    const int64_t groups = (int64_t)((pr.fixed.ny + 3) / 4) * pr.fixed.nz;
    const int64_t gvox = 4 * (int64_t)pr.fixed.nx;
    const int64_t target = packed ? std::min<int64_t>(65535, tune.slab_voxels) : tune.slab_voxels;
    int64_t per = target / gvox;
    if (per < 1) per = 1;
    int64_t c = (groups + per - 1) / per;
    if (c < 8) c = 8;
    c = ((c + 7) / 8) * 8;
    plan.chunks[p] = (int32_t)c;
    plan.fchunk_base[p + 1] =
        plan.fchunk_base[p] + ((int64_t)voxels(&pr.fixed) + kPrepFixedChunk - 1) / kPrepFixedChunk;
    const int64_t mplane = (int64_t)pr.moving.nx * pr.moving.ny;
    plan.mchunk_base[p + 1] = plan.mchunk_base[p] + (mplane + kPrepPlaneRun - 1) / kPrepPlaneRun *
                                                        ((pr.moving.nz + kPrepSlices - 1) / kPrepSlices);
    plan.t_base[p + 1] = plan.t_base[p] + pr.n_transforms;
    for (int x = 0; x < 8; ++x)
      plan.xcd_base[(size_t)x * (P + 1) + p + 1] =
          plan.xcd_base[(size_t)x * (P + 1) + p] + (c / 8) * pr.n_transforms;
  }
  plan.total_t = plan.t_base[P];
  if (plan.total_t > (1 << 24)) return MI_ERR_COUNT;
  size_t off = 0;
  plan.off_desc = 0;
  off = align256(sizeof(PairDesc) * P);
  plan.off_frow = off;
  off += align256(8 * (size_t)(P + 1));
  plan.off_mrow = off;
  off += align256(8 * (size_t)(P + 1));
  plan.off_tbase = off;
  off += align256(8 * (size_t)(P + 1));
  plan.off_xcd = off;
  off += align256(64 * (size_t)(P + 1));
  plan.table_bytes = off;
  size_t w = 0;
  plan.tables = w;
  w += plan.table_bytes;
  plan.counters = w;
  w += align256(8 * 8);
  plan.transforms = w;
  w += align256(96 * (size_t)plan.total_t);
  plan.hist = w;
  w += align256(4 * (size_t)bins * bins * (size_t)plan.total_t);
  plan.count = w;
  w += align256(8 * (size_t)plan.total_t);
  plan.part = w;
  w += align256(reduce_part_bytes(plan.total_t, bins, n_q));
  plan.oct8 = true;
  for (int p = 0; p < P; ++p) plan.oct8 = plan.oct8 && oct8_range(pairs[p].moving.lo, pairs[p].moving.hi);
  for (int p = 0; p < P; ++p) {
    plan.fbins[p] = w;
    w += align256(voxels(&pairs[p].fixed));
    plan.octs[p] = w;
    const mi_volume& mv = pairs[p].moving;
    w += align256(plan.oct8 ? oct8_volume_bytes(mv.nx, mv.ny, mv.nz) : oct_volume_bytes(mv.nx, mv.ny, mv.nz));
  }
  plan.total = w;
  return MI_OK;
}

// ---- tuning cache ---------------------------------------------------------

TuneKey tune_key(const mi_volume* f, const mi_volume* m, int32_t n, int32_t bins, int32_t flags) {
  TuneKey k;
  int32_t nb = 0;
  while ((1 << nb) < n && nb < 30) ++nb;
  const int32_t v[11] = {f->nx, f->ny, f->nz, m->nx, m->ny, m->nz, m->dtype, bins,
                         (flags & MI_BOUNDARY_CLAMP) ? 1 : 0, nb, oct8_range(m->lo, m->hi) ? 1 : 0};
  memcpy(k.v, v, sizeof v);
  return k;
}

HardTune tune_for(const mi_context* ctx, const mi_volume* f, const mi_volume* m, int32_t n,
                  int32_t bins, int32_t flags) {
  const TuneKey k = tune_key(f, m, n, bins, flags);
  for (const auto& e : ctx->tuned)
    if (e.first == k) return e.second;
  return ctx->hard_default;
}

// Cache file: one problem class per line,
//   gemi-tune fnx fny fnz mnx mny mnz mdtype bins clamp nbucket oct8 block slab_major chunks packed
//   gemi-tune-pairs pairs voxels transforms bins clamp oct8 block slab_voxels packed transform_major
//   gemi-tune-parzen fnx fny fnz mnx mny mnz mdtype bins clamp nbucket fwd_block fwd_lds_kib bwd_block
//                    bwd_lds_kib chunk_shift
// (the pairs' counts are power-of-two buckets).
void load_tune_file(mi_context* c) {
  std::ifstream in(c->tune_file);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ss(line);
    std::string tag;
    TuneKey k;
    HardTune t;
    if (!(ss >> tag)) continue;
    if (tag == "gemi-tune-parzen") {
      k.v[0] = -2;
      ParzenTune pt;
      bool ok = true;
      for (int i = 1; i < 11 && ok; ++i) ok = static_cast<bool>(ss >> k.v[i]);
      ok = ok && (ss >> pt.fwd_block >> pt.fwd_lds_kib >> pt.bwd_block >> pt.bwd_lds_kib >> pt.chunk_shift);
      auto good_block = [](int32_t b) { return b == 256 || b == 512 || b == 1024; };
      auto good_kib = [](int32_t v) { return v == 16 || v == 32 || v == 64 || v == 96 || v == 128; };
      if (ok && good_block(pt.fwd_block) && good_block(pt.bwd_block) && good_kib(pt.fwd_lds_kib) &&
          good_kib(pt.bwd_lds_kib) && pt.chunk_shift >= -1 && pt.chunk_shift <= 2)
        c->parzen_tuned.emplace_back(k, pt);
      continue;
    }
    if (tag == "gemi-tune-pairs") {
      memset(k.v, 0, sizeof k.v);
      k.v[0] = -1;
      PairsTune pt;
      bool ok = true;
      for (int i = 1; i < 7 && ok; ++i) ok = static_cast<bool>(ss >> k.v[i]);
      ok = ok && (ss >> pt.block >> pt.slab_voxels >> pt.packed >> pt.transform_major);
      if (ok && (pt.block == 256 || pt.block == 512 || pt.block == 1024) && pt.slab_voxels >= 4096 &&
          pt.slab_voxels <= (1 << 22) && pt.packed >= -1 && pt.packed <= 1 &&
          (pt.transform_major == 0 || pt.transform_major == 1))
        c->pairs_tuned.emplace_back(k, pt);
      continue;
    }
    if (tag != "gemi-tune") continue;
    bool ok = true;
    for (int i = 0; i < 11 && ok; ++i) ok = static_cast<bool>(ss >> k.v[i]);
    ok = ok && (ss >> t.block >> t.slab_major >> t.chunks >> t.packed);
    if (!ok || (t.block != 256 && t.block != 512 && t.block != 1024) || t.chunks < 0 ||
        t.chunks % 8 != 0 || t.packed < -1 || t.packed > 1)
      continue;
    c->tuned.emplace_back(k, t);
  }
}

void save_tune_file(const mi_context* c) {
  if (c->tune_file.empty()) return;
  std::ofstream out(c->tune_file, std::ios::trunc);
  for (const auto& e : c->tuned) {
    out << "gemi-tune";
    for (int i = 0; i < 11; ++i) out << ' ' << e.first.v[i];
    out << ' ' << e.second.block << ' ' << e.second.slab_major << ' ' << e.second.chunks << ' '
        << e.second.packed << '\n';
  }
  for (const auto& e : c->parzen_tuned) {
    out << "gemi-tune-parzen";
    for (int i = 1; i < 11; ++i) out << ' ' << e.first.v[i];
    out << ' ' << e.second.fwd_block << ' ' << e.second.fwd_lds_kib << ' ' << e.second.bwd_block << ' '
        << e.second.bwd_lds_kib << ' ' << e.second.chunk_shift << '\n';
  }
  for (const auto& e : c->pairs_tuned) {
    out << "gemi-tune-pairs";
    for (int i = 1; i < 7; ++i) out << ' ' << e.first.v[i];
    out << ' ' << e.second.block << ' ' << e.second.slab_voxels << ' ' << e.second.packed << ' '
        << e.second.transform_major << '\n';
  }
}

// ---- graphs -----------------------------------------------------------------

bool use_graph(const mi_context* ctx, int32_t flags, hipStream_t s) {
  return (flags & MI_USE_GRAPH) && s != nullptr && !ctx->timing;
}

// A graph captures the composition with the volumes' spacings and origins
// as kernel arguments, so they are part of the key.
void key_volume(std::vector<uint64_t>& key, const mi_volume* v) {
  uint64_t lo, hi;
  memcpy(&lo, &v->lo, 8);
  memcpy(&hi, &v->hi, 8);
  key.insert(key.end(), {(uint64_t)(uintptr_t)v->data, (uint64_t)v->nx, (uint64_t)v->ny,
                         (uint64_t)v->nz, (uint64_t)v->dtype, lo, hi});
  for (int r = 0; r < 3; ++r) {
    uint64_t a, b;
    memcpy(&a, &v->spacing[r], 8);
    memcpy(&b, &v->origin[r], 8);
    key.push_back(a);
    key.push_back(b);
  }
}

void key_q(std::vector<uint64_t>& key, const double* q, int32_t n_q) {
  for (int i = 0; i < n_q; ++i) {
    uint64_t b;
    memcpy(&b, &q[i], 8);
    key.push_back(b);
  }
}

// Replays the graph recorded for `key`, or records `body`'s launches on `s`
// into a new graph and replays it.
template <class F>
int graph_run(mi_context* ctx, const std::vector<uint64_t>& key, hipStream_t s, F&& body) {
  hipError_t e;
  for (auto& g : ctx->graphs)
    if (g.key == key) {
      if ((e = hipGraphLaunch(g.exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      return MI_OK;
    }
  if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(e, "hipStreamBeginCapture");
  const int st = body();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (st != MI_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (ctx->graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  ctx->graphs.push_back(GraphEntry{key, exec});
  if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return MI_OK;
}

// ---- the hard-binned path ---------------------------------------------------

// Fixed bins, oct volume, zeroed histograms and the sweep (no reduction).
int launch_hard_hist(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
                     const double* transforms, int32_t n, int32_t bins, int32_t flags,
                     uint32_t* hist, char* ws, const Layout& L, hipStream_t s,
                     const HardTune& tune, bool prepare, const SampleSpec* smp = nullptr) {
  hipError_t e;
  uint8_t* fb = (uint8_t*)(ws + L.fbins);
  void* octs = ws + L.gvol;
  const size_t bb = (size_t)bins * bins;
  // a sampled call always prepares (its list is not part of the record)
  if (prepare && (smp || !reuse_prep(ctx, flags, prep_key(1, ws, fixed, moving, bins)))) {
    if ((e = launch_prebin_fixed(desc(fixed), bins, fb, s)) != hipSuccess) return hip_fail(e, "prebin");
    e = oct8_range(moving->lo, moving->hi) ? launch_pack_oct8(desc(moving), (uint2*)octs, s)
                                           : launch_pack_octs(desc(moving), (uint4*)octs, s);
    if (e != hipSuccess) return hip_fail(e, "pack");
  }
  if ((e = launch_fill_u32(hist, bb * n, 0u, s)) != hipSuccess) return hip_fail(e, "fill");
  HardLaunch H{};
  H.transforms = transforms;
  H.fbins = fb;
  H.octs = octs;
  H.fixed = desc(fixed);
  H.moving = desc(moving);
  H.hist = hist;
  H.n = n;
  H.bins = bins;
  H.clamp = (flags & MI_BOUNDARY_CLAMP) ? 1 : 0;
  H.packed = use_packed(tune, bins) ? 1 : 0;
  H.block = tune.block;
  H.slab_major = tune.slab_major;
  H.brick = (flags & MI_COMPACT_SLABS) ? 1 : 0;
  uint2* list = (uint2*)(ws + L.list);
  unsigned long long* nlist = (unsigned long long*)(ws + L.nlist);
  if (smp) {
    ctx->last_prep.clear();
    if ((e = launch_fill_u32((uint32_t*)nlist, 2, 0u, s)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_sample_list(fb, fixed->nx, fixed->ny, fixed->nz, smp->fraction, smp->seed, list, nlist, s)) !=
        hipSuccess)
      return hip_fail(e, "sample list");
    H.packed = bins > 128 ? 1 : 0;
    H.chunks = plan_sampled_chunks(ctx, expected_samples(fixed, *smp), n);
  } else {
    H.chunks = plan_chunks(ctx, fixed, moving, n, H.packed != 0, tune);
  }
  // one launch covers at most 2^31 - 1 workgroups: split the transforms
  int64_t per_launch = 0x7FFFFFFFll / H.chunks;
  // Thin slabs in slab-major order: the workgroups resident on an XCD sweep
  // one slab for consecutive transforms, so those are put in an order that
  // keeps their moving footprints together (launch_order_transforms; the
  // multi-modal sweep's 1000 transforms 16.8 -> 13.5 ms).  Launches then
  // start at multiples of the order's sorted blocks.
  uint32_t* order = (uint32_t*)(ws + L.order);
  const bool ordered = !smp && !H.brick && H.slab_major && n >= 64 && per_launch >= kOrderBlock;
  if (ordered) {
    per_launch -= per_launch % kOrderBlock;
    if ((e = launch_order_transforms(transforms, n, fixed->nx, fixed->ny, fixed->nz, order, s)) != hipSuccess)
      return hip_fail(e, "transform order");
  }
  for (int64_t t0 = 0; t0 < n; t0 += per_launch) {
    HardLaunch part = H;
    part.n = (int32_t)(n - t0 < per_launch ? n - t0 : per_launch);
    part.transforms = transforms + 12 * t0;
    part.hist = hist + bb * t0;
    if (ordered) {
      part.order = order + t0;
      part.order_t0 = t0;
    }
    TimedLaunch tl(ctx, 0, s);
    e = smp ? launch_hist_sampled(part, list, nlist, s) : launch_hist_hard(part, s);
    if (e != hipSuccess) return hip_fail(e, smp ? "hist_sampled" : "hist_hard");
    tl.done();
  }
  return MI_OK;
}

int run_hard(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
             const double* transforms, int32_t n, int32_t bins, const double* q, int32_t n_q,
             int32_t flags, double* mi_out, uint64_t* overlap_out, uint32_t* hist_out, char* ws,
             const Layout& L, hipStream_t s, const HardTune& tune, const SampleSpec* smp = nullptr) {
  uint32_t* hist = hist_out ? hist_out : (uint32_t*)(ws + L.hist);
  // the caller's physical matrices -> index-space matrices in the workspace
  double* M = (double*)(ws + L.xf);
  hipError_t ce = launch_compose(transforms, n, geometry(fixed, moving), M, s);
  if (ce != hipSuccess) return hip_fail(ce, "compose");
  transforms = M;
  int st = launch_hard_hist(ctx, fixed, moving, transforms, n, bins, flags, hist, ws, L, s, tune, true, smp);
  if (st != MI_OK) return st;
  ReduceLaunch R;
  memset(&R, 0, sizeof R);
  R.hist = hist;
  R.count = (uint64_t*)(ws + L.count);
  R.part = (double*)(ws + L.part);
  R.transforms = transforms;
  R.n = n;
  R.bins = bins;
  R.q = qlist(q, n_q, flags);
  R.mi_out = mi_out;
  R.overlap_out = overlap_out;
  TimedLaunch tr(ctx, 4, s);
  hipError_t e;
  if ((e = launch_mi_reduce(R, s)) != hipSuccess) return hip_fail(e, "mi_reduce");
  tr.done();
  return MI_OK;
}


// Autotuning of the Parzen sweeps (mi_tune with MI_HIST_PARZEN): the
// forward's shape first (forward + MI calls), then the backward's with the
// best forward (gradient calls), then the workgroup count, one entropy
// (Shannon).  The workspace is the gradient workspace for two entropies;
// the second entropy's dMI/dp tables hold the calls' MI and gradients.
int tune_parzen(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving, const double* transforms,
                int32_t n, int32_t bins, int32_t flags, char* ws, const Layout& L, hipStream_t s) {
  const size_t BB = (size_t)bins * bins;
  char* spare = ws + L.gtab + align256(BB * 4 * (size_t)n);
  double* mi = (double*)spare;
  double* grad = (double*)(spare + align256(8 * (size_t)n));
  const double one = 1.0;
  const int32_t fl = (flags & (MI_BOUNDARY_CLAMP | MI_TSALLIS_PSEUDOADDITIVE)) | MI_HIST_PARZEN;
  hipError_t e;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_fail(e, "tune events");
  }
  ParzenTune best = parzen_tune_for(ctx, fixed, moving, n, bins, flags);
  // the preparation once; the timed calls reuse it
  int st = run_parzen(ctx, fixed, moving, transforms, n, bins, &one, 1, fl, mi, nullptr, grad, ws, L, s, nullptr,
                      &best);
  auto timed = [&](const ParzenTune& c, bool with_grad, float& ms_out) -> int {
    float total = 0;
    for (int rep = 0; rep < 4; ++rep) {
      if ((e = hipEventRecord(t0, s)) != hipSuccess) return hip_fail(e, "tune");
      const int r = run_parzen(ctx, fixed, moving, transforms, n, bins, &one, 1, fl | MI_VOLUMES_UNCHANGED, mi,
                               nullptr, with_grad ? grad : nullptr, ws, L, s, nullptr, &c);
      if (r != MI_OK) return r;
      if ((e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess)
        return hip_fail(e, "tune");
      float ms = 0;
      (void)hipEventElapsedTime(&ms, t0, t1);
      if (rep > 0) total += ms;  // the first run warms caches
    }
    ms_out = total;
    return MI_OK;
  };
  const int32_t blocks[3] = {256, 512, 1024}, budgets[4] = {32, 64, 96, 128};
  for (int pass = 0; pass < 2 && st == MI_OK; ++pass) {  // 0: forward, 1: backward
    float best_ms = 3.4e38f;
    ParzenTune keep = best;
    for (int32_t b : blocks)
      for (int32_t kib : budgets) {
        ParzenTune c = best;
        if (pass == 0) {
          c.fwd_block = b;
          c.fwd_lds_kib = kib;
        } else {
          c.bwd_block = b;
          c.bwd_lds_kib = kib;
        }
        float ms = 0;
        if ((st = timed(c, pass == 1, ms)) != MI_OK) break;
        if (ms < best_ms) {
          best_ms = ms;
          keep = c;
        }
      }
    best = keep;
  }
  if (st == MI_OK) {
    float best_ms = 3.4e38f;
    ParzenTune keep = best;
    for (int32_t sh : {-1, 0, 1, 2}) {
      ParzenTune c = best;
      c.chunk_shift = sh;
      float ms = 0;
      if ((st = timed(c, true, ms)) != MI_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        keep = c;
      }
    }
    best = keep;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != MI_OK) return st;
  const TuneKey k = parzen_tune_key(fixed, moving, n, bins, flags);
  bool found = false;
  for (auto& entry : ctx->parzen_tuned)
    if (entry.first == k) {
      entry.second = best;
      found = true;
    }
  if (!found) ctx->parzen_tuned.emplace_back(k, best);
  save_tune_file(ctx);
  return MI_OK;
}

// ---- the multi-pair path -----------------------------------------------------

// Problem class of a pair set for the tuning cache: pair count, total fixed
// voxels and total transforms (power-of-two buckets), bins, boundary, corner
// layout.
TuneKey pairs_tune_key(const mi_pair* pairs, int32_t n_pairs, int32_t bins, int32_t flags) {
  int64_t vox = 0, nt = 0;
  bool oct8 = true;
  for (int p = 0; p < n_pairs; ++p) {
    vox += (int64_t)voxels(&pairs[p].fixed);
    nt += pairs[p].n_transforms;
    oct8 = oct8 && oct8_range(pairs[p].moving.lo, pairs[p].moving.hi);
  }
  auto bucket = [](int64_t v) {
    int32_t b = 0;
    while ((1ll << b) < v && b < 62) ++b;
    return b;
  };
  TuneKey k;
  memset(k.v, 0, sizeof k.v);
  const int32_t v[7] = {-1, bucket(n_pairs), bucket(vox), bucket(nt), bins, (flags & MI_BOUNDARY_CLAMP) ? 1 : 0,
                        oct8 ? 1 : 0};
  memcpy(k.v, v, sizeof v);
  return k;
}

PairsTune pairs_tune_for(const mi_context* ctx, const mi_pair* pairs, int32_t n_pairs, int32_t bins,
                         int32_t flags) {
  const TuneKey k = pairs_tune_key(pairs, n_pairs, bins, flags);
  for (const auto& e : ctx->pairs_tuned)
    if (e.first == k) return e.second;
  return PairsTune();
}

// Key of a pairs preparation: every pair's volumes, bins, workspace, layout.
std::vector<uint64_t> pairs_prep_key(const mi_pair* pairs, int32_t n_pairs, int32_t bins, const void* ws,
                                     bool oct8) {
  std::vector<uint64_t> k = {(uint64_t)n_pairs, (uint64_t)bins, (uint64_t)(uintptr_t)ws, oct8 ? 1u : 0u};
  for (int p = 0; p < n_pairs; ++p)
    for (const mi_volume* v : {&pairs[p].fixed, &pairs[p].moving}) {
      uint64_t lo, hi;
      memcpy(&lo, &v->lo, 8);
      memcpy(&hi, &v->hi, 8);
      k.insert(k.end(), {(uint64_t)(uintptr_t)v->data, (uint64_t)v->nx, (uint64_t)v->ny, (uint64_t)v->nz,
                         (uint64_t)v->dtype, lo, hi});
    }
  return k;
}

// One multi-pair evaluation: descriptor and prefix tables uploaded, the
// transforms gathered and composed, the pairs prepared (fixed bins, oct
// volumes) when `prepare`, the persistent sweep, and (unless `sweep_only`)
// the MI reduction.
int run_pairs(mi_context* ctx, const mi_pair* pairs, int32_t n_pairs, int32_t bins, const double* q,
              int32_t n_q, int32_t flags, double* mi_out, char* ws, hipStream_t s, const PairsPlan& plan,
              const PairsTune& tune, bool prepare, bool sweep_only = false) {
  hipError_t e;
  // device tables: descriptors, row / transform / per-XCD item prefixes
  const int P = n_pairs;
  std::vector<PairDesc> desc_v(P);
  for (int p = 0; p < P; ++p) {
    const mi_pair& pr = pairs[p];
    PairDesc& d = desc_v[p];
    memset(&d, 0, sizeof d);
    d.fixed = pr.fixed.data;
    d.moving = pr.moving.data;
    d.transforms = pr.transforms;
    d.geo = geometry(&pr.fixed, &pr.moving);
    d.geom = make_hard_geom(desc(&pr.fixed), desc(&pr.moving), (const uint8_t*)(ws + plan.fbins[p]),
                            (const void*)(ws + plan.octs[p]), bins);
    // one layout for every pair of the launch
    d.geom.oct8 = plan.oct8 ? 1 : 0;
    d.geom.oct_bytes = (uint32_t)(plan.oct8 ? oct8_volume_bytes(pr.moving.nx, pr.moving.ny, pr.moving.nz)
                                            : oct_volume_bytes(pr.moving.nx, pr.moving.ny, pr.moving.nz));
    d.fdtype = pr.fixed.dtype;
    d.mdtype = pr.moving.dtype;
    d.flo = pr.fixed.lo;
    d.fhi = pr.fixed.hi;
    d.mlo = (int32_t)pr.moving.lo;
    d.mhi = (int32_t)pr.moving.hi;
    if (pr.fixed.dtype != MI_F32) d.fdiv = make_divider((uint32_t)(pr.fixed.hi - pr.fixed.lo + 1.0));
    d.n_t = pr.n_transforms;
    d.chunks = plan.chunks[p];
  }
  std::vector<char> blob(plan.table_bytes, 0);
  char* b = blob.data();
  memcpy(b + plan.off_desc, desc_v.data(), sizeof(PairDesc) * P);
  memcpy(b + plan.off_frow, plan.fchunk_base.data(), 8 * (P + 1));
  memcpy(b + plan.off_mrow, plan.mchunk_base.data(), 8 * (P + 1));
  memcpy(b + plan.off_tbase, plan.t_base.data(), 8 * (P + 1));
  memcpy(b + plan.off_xcd, plan.xcd_base.data(), 8 * 8 * (P + 1));
  char* dtab = ws + plan.tables;
  if (plan.table_bytes <= kStageBytes) {
    if (ctx->stage_pending && (e = hipEventSynchronize(ctx->stage_done)) != hipSuccess)
      return hip_fail(e, "staging");
    memcpy(ctx->stage, b, plan.table_bytes);
    if ((e = hipMemcpyAsync(dtab, ctx->stage, plan.table_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(e, "table upload");
    if ((e = hipEventRecord(ctx->stage_done, s)) != hipSuccess) return hip_fail(e, "staging");
    ctx->stage_pending = true;
  } else {
    // tables beyond the staging buffer: wait for earlier users of the
    // workspace, then copy synchronously from pageable memory
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "table upload");
    if ((e = hipMemcpy(dtab, b, plan.table_bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "table upload");
  }

  PairsLaunch L;
  memset(&L, 0, sizeof L);
  PairsArgs& a = L.args;
  a.pairs = (const PairDesc*)(dtab + plan.off_desc);
  a.n_pairs = P;
  a.fchunk_base = (const int64_t*)(dtab + plan.off_frow);
  a.mchunk_base = (const int64_t*)(dtab + plan.off_mrow);
  a.t_base = (const int64_t*)(dtab + plan.off_tbase);
  a.xcd_base = (const int64_t*)(dtab + plan.off_xcd);
  a.counters = (unsigned long long*)(ws + plan.counters);
  a.transforms = (double*)(ws + plan.transforms);
  a.hist = (uint32_t*)(ws + plan.hist);
  a.bins = bins;
  a.transform_major = tune.transform_major;
  L.total_t = plan.total_t;
  L.fixed_chunks = plan.fchunk_base[P];
  L.moving_chunks = plan.mchunk_base[P];
  L.clamp = (flags & MI_BOUNDARY_CLAMP) ? 1 : 0;
  L.packed = plan.packed ? 1 : 0;
  L.oct8 = plan.oct8 ? 1 : 0;
  L.cu_count = ctx->cu_count;
  L.block = tune.block;
  const size_t bb = (size_t)bins * bins;
  auto body = [&]() -> int {
    hipError_t err;
    if ((err = launch_fill_u32((uint32_t*)a.counters, 16, 0u, s)) != hipSuccess) return hip_fail(err, "fill");
    if ((err = launch_fill_u32(a.hist, bb * plan.total_t, 0u, s)) != hipSuccess) return hip_fail(err, "fill");
    if ((err = launch_pairs_prep(L, s, prepare)) != hipSuccess) return hip_fail(err, "pairs prep");
    {
      TimedLaunch tl(ctx, 3, s);
      if ((err = launch_pairs_hist(L, s)) != hipSuccess) return hip_fail(err, "pairs hist");
      tl.done();
    }
    if (sweep_only) return MI_OK;
    ReduceLaunch R;
    memset(&R, 0, sizeof R);
    R.hist = a.hist;
    R.count = (uint64_t*)(ws + plan.count);
    R.part = (double*)(ws + plan.part);
    R.transforms = a.transforms;
    R.n = (int32_t)plan.total_t;
    R.bins = bins;
    R.q = qlist(q, n_q, flags);
    R.mi_out = mi_out;
    TimedLaunch tr(ctx, 4, s);
    if ((err = launch_mi_reduce(R, s)) != hipSuccess) return hip_fail(err, "mi_reduce");
    tr.done();
    return MI_OK;
  };
  if (sweep_only || !use_graph(ctx, flags, s)) return body();
  // the graph holds the launch shape and whether it prepares
  std::vector<uint64_t> key = {3,
                               (uint64_t)P,
                               (uint64_t)bins,
                               (uint64_t)flags,
                               (uint64_t)(uintptr_t)mi_out,
                               (uint64_t)(uintptr_t)ws,
                               (uint64_t)(uintptr_t)s,
                               prepare ? 1u : 0u,
                               (uint64_t)tune.block,
                               (uint64_t)tune.slab_voxels,
                               (uint64_t)(tune.packed + 1),
                               (uint64_t)tune.transform_major};
  key_q(key, q, n_q);
  for (int p = 0; p < P; ++p) {
    key_volume(key, &pairs[p].fixed);
    key_volume(key, &pairs[p].moving);
    key.push_back((uint64_t)(uintptr_t)pairs[p].transforms);
    key.push_back((uint64_t)pairs[p].n_transforms);
  }
  return graph_run(ctx, key, s, body);
}
}  // namespace

extern "C" {

const char* mi_status_string(int status) {
  switch (status) {
  case MI_OK: return "ok";
  case MI_ERR_NULL: return "a required pointer is NULL";
  case MI_ERR_DIMS: return "volume edge outside [2, 4096] or more than 2^28 voxels";
  case MI_ERR_DTYPE: return "unknown dtype, or float32 moving volume on the hard-binned path";
  case MI_ERR_BINS: return "bins outside [2, 256] (Parzen: [8, 256])";
  case MI_ERR_RANGE: return "intensity range lo/hi invalid";
  case MI_ERR_Q: return "q list invalid (1..16 entries, each finite and > 0)";
  case MI_ERR_WORKSPACE: return "workspace NULL or too small";
  case MI_ERR_UNSUPPORTED: return "request not supported";
  case MI_ERR_FLAGS: return "unknown flag bits";
  case MI_ERR_SAMPLE: return "sampling fraction not finite or not above 0";
  case MI_ERR_COUNT: return "transform or pair count out of range";
  case MI_ERR_TOO_LARGE: return "call needs more scratch than the library's fixed no-alloc buffer (MI_NOALLOC_SCRATCH_BYTES)";
  case MI_ERR_HIP: {
    static thread_local std::string s;
    s = "HIP error: " + g_last_hip;
    return s.c_str();
  }
  case MI_ERR_NO_DEVICE: return "no usable gfx950 device";
  default: return "unknown status";
  }
}

int mi_create(mi_context** out, int device) {
  if (!out) return MI_ERR_NULL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return MI_ERR_NO_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return MI_ERR_NO_DEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MI_ERR_NO_DEVICE;
  hipError_t e;
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = configure_hard_kernels()) != hipSuccess) return hip_fail(e, "configure kernels");
  if ((e = configure_parzen_kernels()) != hipSuccess) return hip_fail(e, "configure kernels");
  // the allocation-free entry point's scratch: this device's address of it
  if ((e = scratch_setup(device)) != hipSuccess) return hip_fail(e, "scratch address");
  mi_context* c = new mi_context();
  c->device = device;
  if ((e = hipHostMalloc(&c->stage, kStageBytes, hipHostMallocDefault)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming)) != hipSuccess) {
    if (c->stage) (void)hipHostFree(c->stage);
    delete c;
    return hip_fail(e, "staging buffer");
  }
  if (const char* b = getenv("MI_TUNE_HARD_BLOCK")) {
    const int v = atoi(b);
    if (v == 256 || v == 512 || v == 1024) c->hard_default.block = v;
  }
  if (const char* o = getenv("MI_TUNE_HARD_ORDER")) c->hard_default.slab_major = atoi(o) != 0;
  if (const char* k = getenv("MI_TUNE_HARD_CHUNKS")) {
    const int v = atoi(k);
    if (v >= 8 && v % 8 == 0) c->hard_default.chunks = v;
  }
  if (const char* b = getenv("MI_TUNE_PARZEN_BLOCK")) {
    const int v = atoi(b);
    if (v == 256 || v == 512 || v == 1024) {
      c->parzen_default.fwd_block = c->parzen_default.bwd_block = v;
      c->parzen_env = true;
    }
  }
  if (const char* l = getenv("MI_TUNE_PARZEN_LDS_KIB")) {
    const int v = atoi(l);
    if (v == 16 || v == 32 || v == 64 || v == 96 || v == 128) {
      c->parzen_default.fwd_lds_kib = c->parzen_default.bwd_lds_kib = v;
      c->parzen_env = true;
    }
  }
  if (const char* k = getenv("MI_TUNE_PARZEN_CHUNK_SHIFT")) {
    const int v = atoi(k);
    if (v >= -1 && v <= 2) {
      c->parzen_default.chunk_shift = v;
      c->parzen_env = true;
    }
  }
  if (const char* f = getenv("MI_TUNE_CACHE")) {
    c->tune_file = f;
    load_tune_file(c);
  }
  c->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  *out = c;
  return MI_OK;
}

int mi_destroy(mi_context* ctx) {
  if (!ctx) return MI_OK;
  for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  if (ctx->stage_pending) (void)hipEventSynchronize(ctx->stage_done);
  if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  for (int w = 0; w < kTimers; ++w)
    for (auto& ev : ctx->events[w]) {
      (void)hipEventDestroy(ev.start);
      (void)hipEventDestroy(ev.stop);
    }
  delete ctx;
  return MI_OK;
}

int mi_workspace_size(mi_context*, const mi_volume* fixed, const mi_volume* moving, int32_t n, int32_t bins,
                      int32_t n_q, int32_t flags, size_t* bytes) {
  if (!bytes) return MI_ERR_NULL;
  const bool for_grad = (flags & MI_GRADIENT) != 0;
  const bool parzen = for_grad || (flags & MI_HIST_PARZEN);
  int st = check_common(fixed, moving, n, bins, nullptr, 0, flags, parzen);
  if (st != MI_OK) return st;
  if (n_q < 1 || n_q > MI_MAX_Q) return MI_ERR_Q;
  if ((flags & MI_SAMPLED) && for_grad) return MI_ERR_UNSUPPORTED;
  *bytes = layout(fixed, moving, n, bins, n_q, parzen, for_grad, true, (flags & MI_SAMPLED) != 0).total;
  return MI_OK;
}

int mi_tune(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
            const double* transforms, int32_t n, int32_t bins, int32_t flags, void* workspace,
            size_t workspace_bytes, void* stream) {
  const bool parzen = (flags & MI_HIST_PARZEN) != 0;
  int st = check_common(fixed, moving, n, bins, nullptr, 0, flags & ~MI_USE_GRAPH, parzen);
  if (st != MI_OK) return st;
  if (flags & (MI_SAMPLED | MI_GRADIENT)) return MI_ERR_FLAGS;
  if (n > 0 && !transforms) return MI_ERR_NULL;
  if (parzen) {
    const Layout PL = layout(fixed, moving, n, bins, 2, true, true, false);
    if (!workspace || workspace_bytes < PL.total) return MI_ERR_WORKSPACE;
    if (!ctx) return MI_ERR_NULL;
    if (n == 0) return MI_OK;
    hipError_t pe;
    if ((pe = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(pe, "hipSetDevice");
    const bool was = ctx->timing;
    ctx->timing = false;
    const int r = tune_parzen(ctx, fixed, moving, transforms, n, bins, flags, (char*)workspace, PL,
                              (hipStream_t)stream);
    ctx->timing = was;
    ctx->last_prep.clear();
    return r;
  }
  const Layout L = layout(fixed, moving, n, bins, 1, false, false, true);
  if (!workspace || workspace_bytes < L.total) return MI_ERR_WORKSPACE;
  if (!ctx) return MI_ERR_NULL;
  if (n == 0) return MI_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  char* ws = (char*)workspace;
  uint32_t* hist = (uint32_t*)(ws + L.hist);
  // the caller's physical matrices -> index-space matrices, once
  {
    double* M = (double*)(ws + L.xf);
    if ((e = launch_compose(transforms, n, geometry(fixed, moving), M, s)) != hipSuccess)
      return hip_fail(e, "compose");
    transforms = M;
  }
  const bool was_timing = ctx->timing;
  ctx->timing = false;
  // fixed bins and octs once
  st = launch_hard_hist(ctx, fixed, moving, transforms, n, bins, flags, hist, ws, L, s,
                        ctx->hard_default, true);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (st == MI_OK && ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess))
    st = hip_fail(e, "tune events");
  HardTune best = ctx->hard_default;
  float best_ms = 3.4e38f;
  HardTune base = ctx->hard_default;
  base.chunks = plan_chunks(ctx, fixed, moving, n, use_packed(base, bins), base);
  const int32_t chunk_opts[3] = {base.chunks / 2, base.chunks, base.chunks * 2};
  // LDS counter layouts: u32 or packed 16-bit pairs (only packed fits above 128 bins)
  const int32_t n_layouts = bins > 128 ? 1 : 2;
  const int32_t layouts[2] = {bins > 128 ? 1 : 0, 1};
  for (int32_t li = 0; li < n_layouts; ++li)
  for (int32_t block : {256, 512, 1024}) {
    for (int32_t order : {1, 0}) {
      for (int32_t c : chunk_opts) {
        if (st != MI_OK) break;
        HardTune cand;
        cand.block = block;
        cand.slab_major = order;
        cand.chunks = ((c < 8 ? 8 : c) + 7) / 8 * 8;
        cand.packed = layouts[li];
        float total = 0;
        for (int rep = 0; rep < 3 && st == MI_OK; ++rep) {
          if ((e = hipEventRecord(t0, s)) != hipSuccess) { st = hip_fail(e, "tune"); break; }
          st = launch_hard_hist(ctx, fixed, moving, transforms, n, bins, flags, hist, ws, L, s, cand, false);
          if (st != MI_OK) break;
          if ((e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess) {
            st = hip_fail(e, "tune");
            break;
          }
          float ms = 0;
          (void)hipEventElapsedTime(&ms, t0, t1);
          if (rep > 0) total += ms;  // the first run warms caches
        }
        if (st == MI_OK && total < best_ms) {
          best_ms = total;
          best = cand;
        }
      }
    }
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  ctx->timing = was_timing;
  if (st != MI_OK) return st;
  const TuneKey k = tune_key(fixed, moving, n, bins, flags);
  bool found = false;
  for (auto& entry : ctx->tuned)
    if (entry.first == k) {
      entry.second = best;
      found = true;
    }
  if (!found) ctx->tuned.emplace_back(k, best);
  save_tune_file(ctx);
  return MI_OK;
}

int mi_timing_enable(mi_context* ctx, int enable) {
  if (!ctx) return MI_ERR_NULL;
  ctx->timing = enable != 0;
  return MI_OK;
}

int mi_timing_read(mi_context* ctx, int which, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return MI_ERR_NULL;
  if (which < 0 || which >= kTimers) return MI_ERR_UNSUPPORTED;
  std::vector<EventPair> evs;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    evs.swap(ctx->events[which]);
  }
  double sum = 0;
  int rc = MI_OK;
  for (auto& ev : evs) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(ev.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.start, ev.stop);
    if (e != hipSuccess && rc == MI_OK) rc = hip_fail(e, "timing");
    sum += ms;
    (void)hipEventDestroy(ev.start);
    (void)hipEventDestroy(ev.stop);
  }
  *total_ms = sum;
  *launches = (int64_t)evs.size();
  return rc;
}

int mi_eval(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
            const double* transforms, int32_t n, int32_t bins, const double* q, int32_t n_q,
            int32_t flags, double* mi_out, uint64_t* overlap_out, uint32_t* hist_out,
            void* workspace, size_t workspace_bytes, void* stream) {
  const bool parzen = (flags & MI_HIST_PARZEN) != 0;
  int st = check_common(fixed, moving, n, bins, q, n_q, flags, parzen);
  if (st != MI_OK) return st;
  if (flags & (MI_SAMPLED | MI_GRADIENT)) return MI_ERR_FLAGS;  // mi_eval_sampled, mi_grad
  if ((st = check_q(q, n_q)) != MI_OK) return st;
  if (n > 0 && (!transforms || !mi_out)) return MI_ERR_NULL;
  if (parzen && hist_out) return MI_ERR_UNSUPPORTED;
  const Layout L = layout(fixed, moving, n, bins, n_q, parzen, false, hist_out == nullptr);
  if (!workspace || workspace_bytes < L.total) return MI_ERR_WORKSPACE;
  if (!ctx) return MI_ERR_NULL;
  if (n == 0) return MI_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  char* ws = (char*)workspace;
  // a graph replays whatever it captured, so it always captures the
  // preparation: reuse is decided per call, graphs run later
  const bool graph = use_graph(ctx, flags, s);
  const int32_t run_flags = graph ? (flags & ~MI_VOLUMES_UNCHANGED) : flags;
  auto body = [&]() -> int {
    if (parzen)
      return run_parzen(ctx, fixed, moving, transforms, n, bins, q, n_q, run_flags, mi_out, overlap_out,
                        nullptr, ws, L, s);
    return run_hard(ctx, fixed, moving, transforms, n, bins, q, n_q, run_flags, mi_out, overlap_out,
                    hist_out, ws, L, s, tune_for(ctx, fixed, moving, n, bins, flags));
  };
  if (!graph) return body();
  std::vector<uint64_t> key = {1, (uint64_t)(uintptr_t)transforms, (uint64_t)n, (uint64_t)bins,
                               (uint64_t)flags, (uint64_t)(uintptr_t)mi_out,
                               (uint64_t)(uintptr_t)overlap_out, (uint64_t)(uintptr_t)hist_out,
                               (uint64_t)(uintptr_t)workspace, (uint64_t)(uintptr_t)s};
  key_volume(key, fixed);
  key_volume(key, moving);
  key_q(key, q, n_q);
  st = graph_run(ctx, key, s, body);
  ctx->last_prep = prep_key(parzen ? 2 : 1, ws, fixed, moving, bins);  // the graph prepared them
  return st;
}

int mi_eval_noalloc(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
                    const double* transforms, int32_t n, int32_t bins, const double* q, int32_t n_q,
                    int32_t flags, double* mi_out, uint64_t* overlap_out, uint32_t* hist_out,
                    void* stream) {
  const bool parzen = (flags & MI_HIST_PARZEN) != 0;
  if (flags & (MI_USE_GRAPH | MI_SAMPLED | MI_GRADIENT)) return MI_ERR_FLAGS;
  int st = check_common(fixed, moving, n, bins, q, n_q, flags, parzen);
  if (st != MI_OK) return st;
  if ((st = check_q(q, n_q)) != MI_OK) return st;
  if (n > 0 && (!transforms || !mi_out)) return MI_ERR_NULL;
  if (parzen && hist_out) return MI_ERR_UNSUPPORTED;
  const Layout L = layout(fixed, moving, n, bins, n_q, parzen, false, hist_out == nullptr);
  if (L.total > MI_NOALLOC_SCRATCH_BYTES) return MI_ERR_TOO_LARGE;
  if (!ctx) return MI_ERR_NULL;
  if (n == 0) return MI_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  // the device address looked up at mi_create (never the array's host-side name)
  char* ws = (char*)scratch_device_ptr(ctx->device);
  if (!ws) return hip_fail(hipErrorInvalidSymbol, "no-alloc scratch");
  // other contexts on this device share the array: always prepare, and keep
  // no record that a later call could take for a preparation still in place
  const int32_t run_flags = flags & ~MI_VOLUMES_UNCHANGED;
  const bool was_timing = ctx->timing;  // timing creates events: off for this call
  ctx->timing = false;
  if (parzen)
    st = run_parzen(ctx, fixed, moving, transforms, n, bins, q, n_q, run_flags, mi_out, overlap_out, nullptr,
                    ws, L, s);
  else
    st = run_hard(ctx, fixed, moving, transforms, n, bins, q, n_q, run_flags, mi_out, overlap_out, hist_out, ws,
                  L, s, tune_for(ctx, fixed, moving, n, bins, flags));
  ctx->timing = was_timing;
  ctx->last_prep.clear();
  return st;
}

int mi_eval_sampled(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
                    const double* transforms, int32_t n, int32_t bins, const double* q, int32_t n_q,
                    int32_t flags, double fraction, uint64_t seed, double* mi_out, uint64_t* overlap_out,
                    uint32_t* hist_out, void* workspace, size_t workspace_bytes, void* stream) {
  const bool parzen = (flags & MI_HIST_PARZEN) != 0;
  int st = check_common(fixed, moving, n, bins, q, n_q, flags, parzen);
  if (st != MI_OK) return st;
  if ((st = check_q(q, n_q)) != MI_OK) return st;
  if ((st = check_fraction(fraction)) != MI_OK) return st;
  if (flags & MI_GRADIENT) return MI_ERR_FLAGS;
  if (n > 0 && (!transforms || !mi_out)) return MI_ERR_NULL;
  if (parzen && hist_out) return MI_ERR_UNSUPPORTED;
  const Layout L = layout(fixed, moving, n, bins, n_q, parzen, false, hist_out == nullptr, true);
  if (!workspace || workspace_bytes < L.total) return MI_ERR_WORKSPACE;
  if (!ctx) return MI_ERR_NULL;
  if (n == 0) return MI_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  char* ws = (char*)workspace;
  const SampleSpec smp = {fraction, seed};
  const int32_t run_flags = flags & ~(MI_VOLUMES_UNCHANGED | MI_SAMPLED);
  auto body = [&]() -> int {
    if (parzen)
      return run_parzen(ctx, fixed, moving, transforms, n, bins, q, n_q, run_flags, mi_out, overlap_out,
                        nullptr, ws, L, s, &smp);
    return run_hard(ctx, fixed, moving, transforms, n, bins, q, n_q, run_flags, mi_out, overlap_out,
                    hist_out, ws, L, s, tune_for(ctx, fixed, moving, n, bins, flags), &smp);
  };
  if (!use_graph(ctx, flags, s)) return body();
  uint64_t fbits;
  memcpy(&fbits, &fraction, 8);
  std::vector<uint64_t> key = {4, (uint64_t)(uintptr_t)transforms, (uint64_t)n, (uint64_t)bins,
                               (uint64_t)flags, fbits, seed, (uint64_t)(uintptr_t)mi_out,
                               (uint64_t)(uintptr_t)overlap_out, (uint64_t)(uintptr_t)hist_out,
                               (uint64_t)(uintptr_t)workspace, (uint64_t)(uintptr_t)s};
  key_volume(key, fixed);
  key_volume(key, moving);
  key_q(key, q, n_q);
  st = graph_run(ctx, key, s, body);
  ctx->last_prep.clear();
  return st;
}

int mi_grad(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
            const double* transforms, int32_t n, int32_t bins, const double* q, int32_t n_q,
            int32_t flags, double* mi_out, double* grad_out, void* workspace,
            size_t workspace_bytes, void* stream) {
  int st = check_common(fixed, moving, n, bins, q, n_q, flags, true);
  if (st != MI_OK) return st;
  if (flags & MI_SAMPLED) return MI_ERR_FLAGS;
  if ((st = check_q(q, n_q)) != MI_OK) return st;
  if (n > 0 && (!transforms || !mi_out || !grad_out)) return MI_ERR_NULL;
  const Layout L = layout(fixed, moving, n, bins, n_q, true, true, false);
  if (!workspace || workspace_bytes < L.total) return MI_ERR_WORKSPACE;
  if (!ctx) return MI_ERR_NULL;
  if (n == 0) return MI_OK;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const bool graph = use_graph(ctx, flags, s);
  const int32_t run_flags = graph ? (flags & ~MI_VOLUMES_UNCHANGED) : flags;  // as in mi_eval
  auto body = [&]() -> int {
    return run_parzen(ctx, fixed, moving, transforms, n, bins, q, n_q, run_flags, mi_out, nullptr,
                      grad_out, (char*)workspace, L, s);
  };
  if (!graph) return body();
  std::vector<uint64_t> key = {2, (uint64_t)(uintptr_t)transforms, (uint64_t)n, (uint64_t)bins,
                               (uint64_t)flags, (uint64_t)(uintptr_t)mi_out,
                               (uint64_t)(uintptr_t)grad_out, (uint64_t)(uintptr_t)workspace,
                               (uint64_t)(uintptr_t)s};
  key_volume(key, fixed);
  key_volume(key, moving);
  key_q(key, q, n_q);
  st = graph_run(ctx, key, s, body);
  ctx->last_prep = prep_key(2, workspace, fixed, moving, bins);  // the graph prepared them
  return st;
}

int mi_map_paths(mi_context* ctx, const double* values, int32_t nx, int32_t ny, int32_t nz,
                 int32_t direction, int32_t cx, int32_t cy, int32_t cz, int32_t* next_out,
                 int32_t* sink_out, int64_t* stats_out, void* stream) {
  if (!values || !next_out || !sink_out || !stats_out) return MI_ERR_NULL;
  if (nx < 1 || ny < 1 || nz < 1 || nx > MI_MAX_EDGE || ny > MI_MAX_EDGE || nz > MI_MAX_EDGE)
    return MI_ERR_DIMS;
  if ((int64_t)nx * ny * nz > (int64_t)INT32_MAX) return MI_ERR_DIMS;
  if (cx < 0 || cx >= nx || cy < 0 || cy >= ny || cz < 0 || cz >= nz) return MI_ERR_DIMS;
  if (direction != 1 && direction != -1) return MI_ERR_FLAGS;
  if (!ctx) return MI_ERR_NULL;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  PathsLaunch L;
  L.values = values;
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.sign = (double)direction;
  L.cx = cx;
  L.cy = cy;
  L.cz = cz;
  L.next = next_out;
  L.sink = sink_out;
  L.stats = stats_out;
  if ((e = launch_map_paths(L, (hipStream_t)stream)) != hipSuccess) return hip_fail(e, "map paths");
  return MI_OK;
}

int mi_pairs_workspace_size(const mi_pair* pairs, int32_t n_pairs, int32_t bins, int32_t n_q,
                            int32_t flags, size_t* bytes) {
  if (!bytes) return MI_ERR_NULL;
  PairsPlan plan;
  int st = plan_pairs(pairs, n_pairs, bins, n_q, flags, plan);
  if (st != MI_OK) return st;
  *bytes = plan.total;
  return MI_OK;
}

int mi_eval_pairs(mi_context* ctx, const mi_pair* pairs, int32_t n_pairs, int32_t bins,
                  const double* q, int32_t n_q, int32_t flags, double* mi_out, void* workspace,
                  size_t workspace_bytes, void* stream) {
  int st = check_q(q, n_q);
  if (st != MI_OK) return st;
  PairsPlan plan;
  if ((st = plan_pairs(pairs, n_pairs, bins, n_q, flags, plan)) != MI_OK) return st;
  if (plan.total_t > 0 && !mi_out) return MI_ERR_NULL;
  if (!workspace || workspace_bytes < plan.total) return MI_ERR_WORKSPACE;
  if (!ctx) return MI_ERR_NULL;
  if (plan.total_t == 0) return MI_OK;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  const PairsTune tune = pairs_tune_for(ctx, pairs, n_pairs, bins, flags);
  if ((st = plan_pairs(pairs, n_pairs, bins, n_q, flags, plan, tune)) != MI_OK) return st;
  // the pairs' preparation (fixed bins, oct volumes) is kept in the
  // workspace and reused when the caller asserts unchanged volumes
  std::vector<uint64_t> pkey = pairs_prep_key(pairs, n_pairs, bins, workspace, plan.oct8);
  const bool prepare = !((flags & MI_VOLUMES_UNCHANGED) && pkey == ctx->last_pairs_prep);
  ctx->last_prep.clear();  // the pairs' layout overwrites any single-pair preparation
  st = run_pairs(ctx, pairs, n_pairs, bins, q, n_q, flags, mi_out, (char*)workspace, (hipStream_t)stream, plan,
                 tune, prepare);
  ctx->last_pairs_prep = st == MI_OK ? pkey : std::vector<uint64_t>();
  return st;
}

int mi_tune_pairs(mi_context* ctx, const mi_pair* pairs, int32_t n_pairs, int32_t bins, int32_t flags,
                  void* workspace, size_t workspace_bytes, void* stream) {
  if (flags & (MI_USE_GRAPH | MI_VOLUMES_UNCHANGED)) return MI_ERR_FLAGS;
  PairsPlan plan;
  int st = plan_pairs(pairs, n_pairs, bins, 1, flags, plan);
  if (st != MI_OK) return st;
  if (!workspace || workspace_bytes < plan.total) return MI_ERR_WORKSPACE;
  if (!ctx) return MI_ERR_NULL;
  if (plan.total_t == 0) return MI_OK;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const bool was_timing = ctx->timing;
  ctx->timing = false;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    ctx->timing = was_timing;
    return hip_fail(e, "tune events");
  }
  // the preparation once (it does not depend on the launch shape), then
  // each candidate's sweep timed over three runs after a warm-up run
  const double one = 1.0;
  PairsTune best;
  float best_ms = 3.4e38f;
  std::vector<PairsTune> cands;
  const int32_t layouts[2] = {bins > 128 ? 1 : 0, 1};
  for (int li = 0; li < (bins > 128 ? 1 : 2); ++li)
    for (int32_t block : {256, 512, 1024})
      for (int32_t vox : {65536, 131072, 262144})
        for (int32_t order : {0, 1}) {
          PairsTune c;
          c.block = block;
          c.slab_voxels = vox;
          c.packed = layouts[li];
          c.transform_major = order;
          if (c.packed == 1 && vox > 65536) continue;  // 16-bit counters: at most 65535 voxels per slab
          cands.push_back(c);
        }
  bool prepared = false;
  for (const PairsTune& c : cands) {
    if (st != MI_OK) break;
    PairsPlan cp;
    if ((st = plan_pairs(pairs, n_pairs, bins, 1, flags, cp, c)) != MI_OK) break;
    float total = 0;
    for (int rep = 0; rep < 4 && st == MI_OK; ++rep) {
      if ((e = hipEventRecord(t0, s)) != hipSuccess) { st = hip_fail(e, "tune"); break; }
      st = run_pairs(ctx, pairs, n_pairs, bins, &one, 1, flags, nullptr, ws, s, cp, c, !prepared, true);
      prepared = true;
      if (st != MI_OK) break;
      if ((e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess) {
        st = hip_fail(e, "tune");
        break;
      }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, t0, t1);
      if (rep > 0) total += ms;
    }
    if (st == MI_OK && total < best_ms) {
      best_ms = total;
      best = c;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  ctx->timing = was_timing;
  ctx->last_prep.clear();
  ctx->last_pairs_prep.clear();
  if (st != MI_OK) return st;
  const TuneKey k = pairs_tune_key(pairs, n_pairs, bins, flags);
  bool found = false;
  for (auto& entry : ctx->pairs_tuned)
    if (entry.first == k) {
      entry.second = best;
      found = true;
    }
  if (!found) ctx->pairs_tuned.emplace_back(k, best);
  save_tune_file(ctx);
  return MI_OK;
}

int mi_probe_lds_atomics(mi_context* ctx, void* scratch, size_t scratch_bytes, void* stream,
                         double* lane_atomics_per_s) {
  if (!ctx || !scratch || !lane_atomics_per_s) return MI_ERR_NULL;
  // one 1024-thread workgroup of 4 KiB output per CU slot, two per CU
  const int32_t blocks = 2 * ctx->cu_count;
  const size_t need = (size_t)blocks * 1024 * 4;
  if (scratch_bytes < need || scratch_bytes < ((size_t)4 << 20)) return MI_ERR_WORKSPACE;
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int32_t iters = 1 << 14;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_fail(e, "probe events");
  }
  float ms = 0.0f;
  int st = MI_OK;
  if ((e = launch_lds_atomic_probe((uint32_t*)scratch, blocks, iters, s)) != hipSuccess ||  // warm-up
      (e = hipEventRecord(t0, s)) != hipSuccess ||
      (e = launch_lds_atomic_probe((uint32_t*)scratch, blocks, iters, s)) != hipSuccess ||
      (e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess ||
      (e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess)
    st = hip_fail(e, "lds atomic probe");
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != MI_OK) return st;
  *lane_atomics_per_s = (double)blocks * 1024.0 * iters / (ms * 1e-3);
  return MI_OK;
}

}  // extern "C"
