// Host side of libgemi.so: argument validation, workspace layout, launch
// planning and dispatch for the C ABI declared in include/gemi.h.
#include "../../include/gemi.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace gemi {
hipError_t configure_hard_kernels();
hipError_t configure_parzen_kernels();
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

size_t dtype_size(int32_t d) { return d == MI_U8 ? 1 : (d == MI_F32 ? 4 : 2); }

size_t voxels(const mi_volume* v) { return (size_t)v->nx * v->ny * v->nz; }

int check_volume(const mi_volume* v, bool need_integer) {
  if (!v || !v->data) return MI_ERR_NULL;
  if (v->dtype < MI_U8 || v->dtype > MI_F32) return MI_ERR_DTYPE;
  if (need_integer && v->dtype == MI_F32) return MI_ERR_DTYPE;
  const int32_t n[3] = {v->nx, v->ny, v->nz};
  for (int r = 0; r < 3; ++r)
    if (n[r] < 2 || n[r] > MI_MAX_EDGE) return MI_ERR_DIMS;
  if (voxels(v) > ((size_t)1 << 28)) return MI_ERR_DIMS;
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

constexpr int32_t kKnownFlags = MI_BOUNDARY_CLAMP | MI_TSALLIS_PSEUDOADDITIVE | MI_HIST_PARZEN;

int check_common(const mi_volume* f, const mi_volume* m, int32_t n, int32_t bins, const double* q,
                 int32_t n_q, int32_t flags, bool parzen) {
  if (flags & ~kKnownFlags) return MI_ERR_FLAGS;
  int st;
  if ((st = check_volume(f, false)) != MI_OK) return st;
  if ((st = check_volume(m, !parzen)) != MI_OK) return st;
  if (n < 0 || n > (1 << 24)) return MI_ERR_COUNT;
  if (bins < (parzen ? 8 : 2) || bins > 256) return MI_ERR_BINS;
  if (q != nullptr || n_q != 0) {
    if ((st = check_q(q, n_q)) != MI_OK) return st;
  }
  return MI_OK;
}

// Workspace layout (each region 256-byte aligned):
//   fixed bins   u8[nvox_fixed]
//   hard:        moving quad volume u16x4[mnz+1][mny][mnx],
//                hist u32[n][B][B]          (only when the caller passes no hist_out)
//   Parzen:      table f64[n][B][B], count u64[n]
//   Parzen grad: + dMI/dp tables f32[n][n_q][B][B]
struct Layout {
  size_t fbins = 0, quads = 0, hist = 0, table = 0, count = 0, gtab = 0, total = 0;
};

Layout layout(const mi_volume* f, const mi_volume* m, int32_t n, int32_t bins, int32_t n_q,
              bool parzen, bool grad, bool need_hist) {
  Layout L;
  size_t off = 0;
  L.fbins = off;
  off += align256(voxels(f));
  const size_t bb = (size_t)bins * bins;
  if (!parzen) {
    L.quads = off;
    off += align256(quad_volume_bytes(m->nx, m->ny, m->nz));
    L.hist = off;
    if (need_hist) off += align256(bb * 4 * (size_t)n);
  } else {
    L.table = off;
    off += align256(bb * 8 * (size_t)n);
    L.count = off;
    off += align256(8 * (size_t)n);
    if (grad) {
      L.gtab = off;
      off += align256(bb * 4 * (size_t)n * n_q);
    }
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

QList qlist(const double* q, int32_t n_q, int32_t flags) {
  QList L;
  memset(&L, 0, sizeof L);
  for (int i = 0; i < n_q; ++i) L.q[i] = q[i];
  L.n = n_q;
  L.pseudo = (flags & MI_TSALLIS_PSEUDOADDITIVE) ? 1 : 0;
  return L;
}

}  // namespace

struct mi_context {
  int device = 0;
  int cu_count = 256;
  int hard_block = 512;   // threads per workgroup of the histogram sweep
  int hard_slab_major = 1;
  int hard_chunks = 0;    // workgroups per transform; 0 = planned per call
  bool timing = false;
  std::mutex mu;
  std::vector<EventPair> events[kTimers];
};

namespace {

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

// Workgroups per transform for the histogram sweep.  The fixed volume is
// swept in groups of 4 rows; a transform's groups are split into `c`
// slabs: enough workgroups to fill the chip several times over, at least
// 32 thin slabs in slab-major order (the moving footprint of one slab must
// fit an XCD's L2), a multiple of 8 (one share per XCD), and -- with 16-bit
// packed LDS counters -- few enough voxels per workgroup that no counter
// can exceed 65535.
int plan_chunks(const mi_context* ctx, const mi_volume* f, int32_t n, bool packed) {
  const int64_t groups = (int64_t)((f->ny + 3) / 4) * f->nz;
  int64_t c;
  if (ctx->hard_chunks) {
    c = ctx->hard_chunks;
  } else {
    c = ((int64_t)ctx->cu_count * 8 + n - 1) / n;
    if (ctx->hard_slab_major && c < 32) c = 32;
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
  case MI_ERR_COUNT: return "transform or pair count out of range";
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
  mi_context* c = new mi_context();
  c->device = device;
  if (const char* b = getenv("MI_TUNE_HARD_BLOCK")) {
    const int v = atoi(b);
    if (v == 256 || v == 512 || v == 1024) c->hard_block = v;
  }
  if (const char* o = getenv("MI_TUNE_HARD_ORDER")) c->hard_slab_major = atoi(o) != 0;
  if (const char* k = getenv("MI_TUNE_HARD_CHUNKS")) {
    const int v = atoi(k);
    if (v >= 8 && v % 8 == 0) c->hard_chunks = v;
  }
  c->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  *out = c;
  return MI_OK;
}

int mi_destroy(mi_context* ctx) {
  if (!ctx) return MI_OK;
  for (int w = 0; w < kTimers; ++w)
    for (auto& ev : ctx->events[w]) {
      (void)hipEventDestroy(ev.start);
      (void)hipEventDestroy(ev.stop);
    }
  delete ctx;
  return MI_OK;
}

int mi_workspace_size(const mi_volume* fixed, const mi_volume* moving, int32_t n, int32_t bins,
                      int32_t n_q, int32_t flags, int32_t for_grad, size_t* bytes) {
  if (!bytes) return MI_ERR_NULL;
  const bool parzen = for_grad || (flags & MI_HIST_PARZEN);
  int st = check_common(fixed, moving, n, bins, nullptr, 0, flags, parzen);
  if (st != MI_OK) return st;
  if (n_q < 1 || n_q > MI_MAX_Q) return MI_ERR_Q;
  *bytes = layout(fixed, moving, n, bins, n_q, parzen, for_grad != 0, true).total;
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
  uint8_t* fb = (uint8_t*)(ws + L.fbins);
  if ((e = launch_prebin_fixed(desc(fixed), bins, fb, s)) != hipSuccess) return hip_fail(e, "prebin");
  const size_t bb = (size_t)bins * bins;
  ReduceLaunch R;
  memset(&R, 0, sizeof R);
  R.transforms = transforms;
  R.n = n;
  R.bins = bins;
  R.q = qlist(q, n_q, flags);
  R.mi_out = mi_out;
  R.overlap_out = overlap_out;
  if (!parzen) {
    uint32_t* hist = hist_out ? hist_out : (uint32_t*)(ws + L.hist);
    uint2* quads = (uint2*)(ws + L.quads);
    if ((e = launch_pack_quads(desc(moving), quads, s)) != hipSuccess) return hip_fail(e, "pack");
    if ((e = launch_fill_u32(hist, bb * n, 0u, s)) != hipSuccess) return hip_fail(e, "fill");
    HardLaunch H;
    H.transforms = transforms;
    H.fbins = fb;
    H.quads = quads;
    H.fixed = desc(fixed);
    H.moving = desc(moving);
    H.hist = hist;
    H.n = n;
    H.bins = bins;
    H.clamp = (flags & MI_BOUNDARY_CLAMP) ? 1 : 0;
    H.packed = bins > 128 ? 1 : 0;
    H.block = ctx->hard_block;
    H.slab_major = ctx->hard_slab_major;
    H.chunks = plan_chunks(ctx, fixed, n, H.packed != 0);
    // one launch covers at most 2^31 - 1 workgroups: split the transforms
    const int64_t per_launch = 0x7FFFFFFFll / H.chunks;
    for (int64_t t0 = 0; t0 < n; t0 += per_launch) {
      HardLaunch part = H;
      part.n = (int32_t)(n - t0 < per_launch ? n - t0 : per_launch);
      part.transforms = transforms + 12 * t0;
      part.hist = hist + bb * t0;
      TimedLaunch tl(ctx, 0, s);
      if ((e = launch_hist_hard(part, s)) != hipSuccess) return hip_fail(e, "hist_hard");
      tl.done();
    }
    R.hist = hist;
  } else {
    return MI_ERR_UNSUPPORTED;  // Parzen forward: see mi_grad
  }
  TimedLaunch tr(ctx, 4, s);
  if ((e = launch_mi_reduce(R, s)) != hipSuccess) return hip_fail(e, "mi_reduce");
  tr.done();
  return MI_OK;
}

int mi_grad(mi_context* ctx, const mi_volume* fixed, const mi_volume* moving,
            const double* transforms, int32_t n, int32_t bins, const double* q, int32_t n_q,
            int32_t flags, double* mi_out, double* grad_out, void* workspace,
            size_t workspace_bytes, void* stream) {
  int st = check_common(fixed, moving, n, bins, q, n_q, flags | MI_HIST_PARZEN, true);
  if (st != MI_OK) return st;
  if ((st = check_q(q, n_q)) != MI_OK) return st;
  (void)ctx;
  (void)transforms;
  (void)mi_out;
  (void)grad_out;
  (void)workspace;
  (void)workspace_bytes;
  (void)stream;
  return MI_ERR_UNSUPPORTED;
}

int mi_pairs_workspace_size(const mi_pair* pairs, int32_t n_pairs, int32_t bins, int32_t n_q,
                            int32_t flags, size_t* bytes) {
  (void)pairs;
  (void)n_pairs;
  (void)bins;
  (void)n_q;
  (void)flags;
  if (!bytes) return MI_ERR_NULL;
  return MI_ERR_UNSUPPORTED;
}

int mi_eval_pairs(mi_context* ctx, const mi_pair* pairs, int32_t n_pairs, int32_t bins,
                  const double* q, int32_t n_q, int32_t flags, double* mi_out, void* workspace,
                  size_t workspace_bytes, void* stream) {
  (void)ctx;
  (void)pairs;
  (void)n_pairs;
  (void)bins;
  (void)q;
  (void)n_q;
  (void)flags;
  (void)mi_out;
  (void)workspace;
  (void)workspace_bytes;
  (void)stream;
  return MI_ERR_UNSUPPORTED;
}

}  // extern "C"
