/*
 * gemi.h -- C ABI of the MI355X (gfx950) generalised-entropy mutual
 * information library, libgemi.so.
 *
 * Computes, for many candidate affine transforms at once, the registration
 * metric of Vianna & Murta, "Analysis of Generalized Entropies in Mutual
 * Information Medical Image Registration" (arXiv 1909.10690): the moving
 * volume is resampled under each transform (Transform block of Fig. 1),
 * the joint intensity histogram of fixed vs. resampled moving voxels is
 * accumulated over the overlap, and that one histogram is reduced to
 * Shannon MI (Eq. (1), Eq. (2)) and Tsallis MI for any number of entropic
 * indices q (Discussion: the same histogram serves every entropy).  A
 * Parzen (cubic B-spline) variant adds the gradient with respect to the 12
 * transform entries, for gradient-based optimisation of Eq. (3).
 *
 * Conventions common to every entry point
 *  - Every data pointer (volumes, transforms, outputs, workspace) is a
 *    DEVICE pointer on the context's GPU, allocated and owned by the caller;
 *    the library never frees or retains them.  `q` arrays and `mi_pair`
 *    arrays are HOST pointers, read before the call returns.
 *  - Calls are asynchronous and ordered on `stream` (a hipStream_t; NULL =
 *    the default stream).  Outputs are valid once the stream reaches them.
 *  - No entry point allocates device memory: scratch space is the caller's
 *    `workspace`, sized by mi_workspace_size().  Calls that share one
 *    workspace must be ordered on one stream.
 *  - Arguments are validated before anything is launched; a negative
 *    status means nothing was enqueued.  No exception or abort crosses
 *    the ABI.
 *  - Per-transform degenerate cases are not errors: a transform with no
 *    overlap gives MI 0, overlap 0, gradient 0; a transform whose
 *    index-space matrix M has a non-finite entry, a linear entry beyond
 *    +-2^16 or a translation beyond +-2^24 gives MI NaN, overlap 0,
 *    gradient 0.
 *  - Every transform of a batch (up to 2^24) is evaluated: a sweep whose
 *    grid would pass the dispatch's 32-bit work-item count is issued as
 *    several launches of whole transforms on the same stream.
 *
 * Definitions (the paper prints only Eq. (1)-(3); these are the readings
 * the library implements, identical in the CPU oracle used to test it):
 *  - Geometry: voxel index i = (i, j, k) of a volume sits at the physical
 *    point origin + spacing * i (mm, per axis; voxel centres).
 *  - Transform: a physical 3x4 matrix P, row-major, mapping a point x of
 *    the fixed volume (mm) to the point P (x, 1) of the moving volume (mm)
 *    (Fig. 1 Transform block; the Methodology's transforms are in mm).  The
 *    library turns it into the index-space matrix M that maps fixed voxel
 *    index (i, j, k, 1) to a continuous moving voxel index,
 *    M = S_m^-1 (P (o_f + S_f i) - o_m), computed in fp64 one IEEE
 *    operation at a time, never fused, in exactly this order
 *    (sf, of: fixed spacing and origin; sm, om: moving):
 *      M[r][c] = (P[r][c] * sf[c]) / sm[r]                    for c < 3
 *      M[r][3] = ((((P[r][0] * of[0] + P[r][1] * of[1]) + P[r][2] * of[2])
 *                 + P[r][3]) - om[r]) / sm[r]
 *    With unit spacings and zero origins M equals P exactly.  M is
 *    quantised to signed Q32 fixed point, Mq = round-half-even(M * 2^32);
 *    coordinates are the exact int64 products Mq * (i, j, k, 1).
 *  - Overlap: MI_BOUNDARY_EXCLUDE keeps a fixed voxel iff every moving
 *    coordinate lies in [0, n - 1] (closed); MI_BOUNDARY_CLAMP clamps the
 *    coordinate to that interval and keeps every fixed voxel.
 *  - Intensities are clamped to the volume's [lo, hi] before use.
 *  - Hard histogram: trilinear interpolation with 16-bit truncated weights
 *    w = floor(frac * 2^16), exact integer sum V = sum v' * w_x w_y w_z over
 *    the 8 corners (v' = clamped value - lo); moving bin
 *    floor(V * B / (R * 2^48)), R = hi - lo + 1; fixed bin
 *    floor((u' * B) / R) for integer dtypes, min(B-1, floor(((u-lo)/(hi-lo))
 *    * B)) in fp64 for MI_F32.  Counts are exact; the histogram is unique.
 *  - Entropies in nats.  Shannon H = -sum p ln p.  Tsallis
 *    S_q = (1 - sum p^q)/(q - 1).  MI = H(F) + H(M) - H(F,M) (Eq. (2));
 *    Tsallis MI additive S_q(F) + S_q(M) - S_q(F,M), or with
 *    MI_TSALLIS_PSEUDOADDITIVE the extra term (1 - q) S_q(F) S_q(M).
 *    q == 1 means Shannon.  Reduced in fp64 with compensated sums.
 *  - Parzen histogram: fixed side hard-binned; moving side weighted by the
 *    centred cubic B-spline at s = 1 + (v - lo)/(hi - lo) * (B - 4), v the
 *    trilinear value with full-precision weights; p = table / N with N the
 *    number of fixed voxels that take part.
 */
#ifndef GEMI_H
#define GEMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MI_OK 0
#define MI_ERR_NULL (-1)        /* a required pointer is NULL             */
#define MI_ERR_DIMS (-2)        /* a volume edge outside [2, 4096], more than 2^28 voxels,
                                   or a moving volume of 2^28 voxels or more (integer) or
                                   of nx*ny*(nz+1) >= 2^28 (float, Parzen path): its
                                   gather layout must stay within 4 GiB */
#define MI_ERR_DTYPE (-3)       /* unknown dtype, or MI_F32 moving volume on the hard path */
#define MI_ERR_BINS (-4)        /* bins outside [2, 256] ([8, 256] for Parzen) */
#define MI_ERR_RANGE (-5)       /* lo/hi not finite, hi <= lo, or (integer dtypes) not
                                   integral, |lo|,|hi| > 2^31, or hi - lo + 1 > 65536 */
#define MI_ERR_Q (-6)           /* n_q outside [1, 16], or a q not finite or <= 0 */
#define MI_ERR_WORKSPACE (-7)   /* workspace NULL or smaller than mi_workspace_size() */
#define MI_ERR_UNSUPPORTED (-8) /* a valid request the library does not serve */
#define MI_ERR_FLAGS (-9)       /* unknown flag bits */
#define MI_ERR_COUNT (-10)      /* n_transforms (or n_pairs) negative or above 2^24 */
#define MI_ERR_SAMPLE (-11)     /* sampling fraction not finite or not above 0 */
#define MI_ERR_TOO_LARGE (-12)  /* mi_eval_noalloc: the call needs more scratch than
                                   MI_NOALLOC_SCRATCH_BYTES */
#define MI_ERR_GEOMETRY (-13)   /* a spacing not finite or not above 0, or an origin
                                   entry not finite */
#define MI_ERR_HIP (-20)        /* the HIP runtime reported an error (see mi_status_string) */
#define MI_ERR_NO_DEVICE (-21)  /* no usable GPU with the requested index */

/* ---- volume element types ---------------------------------------------- */
#define MI_U8 0
#define MI_U16 1
#define MI_I16 2
#define MI_F32 3

/* ---- flags (bitwise OR) ------------------------------------------------ */
#define MI_BOUNDARY_EXCLUDE 0x000
#define MI_BOUNDARY_CLAMP 0x001
#define MI_TSALLIS_ADDITIVE 0x000
#define MI_TSALLIS_PSEUDOADDITIVE 0x010
#define MI_HIST_HARD 0x000
#define MI_HIST_PARZEN 0x100
/* Capture the call's kernels into a HIP graph the first time a call with
 * exactly these arguments (pointers, sizes, q, flags, workspace, stream) is
 * seen, and replay the graph on later identical calls: one launch instead
 * of several.  Needs a non-NULL stream; ignored (eager launches) on the
 * NULL stream or while kernel timing is enabled.  Device data behind the
 * pointers may change between replays (e.g. transforms updated in place);
 * the context keeps the 16 most recent graphs. */
#define MI_USE_GRAPH 0x1000
/* The caller asserts that fixed, moving, bins, the boundary flag and the
 * workspace are those of the previous call on this context that prepared
 * them (same path: hard or Parzen), and that neither the volumes' contents
 * nor the workspace have changed since: the per-call preparation (fixed
 * binning, moving gather volume, occupied-row map) already in the workspace
 * is reused.  The library still compares the arguments with its record of
 * the last preparation and prepares again when they differ; it cannot see
 * changed contents.  Ignored by calls that use MI_USE_GRAPH (a captured
 * graph always prepares).  For loops over one volume pair (registration). */
#define MI_VOLUMES_UNCHANGED 0x2000
/* mi_workspace_size: size the workspace for mi_eval_sampled (adds the
 * sample list, 8 bytes per fixed voxel).  Accepted (and implied) by
 * mi_eval_sampled; rejected (MI_ERR_FLAGS) by the other calls. */
#define MI_SAMPLED 0x4000
/* Hint for hard-binned mi_eval (and mi_tune) calls whose transforms rotate
 * the moving volume widely, such as a rotation map: each workgroup sweeps a
 * compact brick of whole x rows instead of a thin slab of whole slices, so
 * that the moving footprints of the transforms running at once overlap in
 * L2.  Results are identical; applies to the 1024-thread launch shape (the
 * default); slower for translation-like batches.  Ignored by the Parzen
 * and sampled paths; mi_eval_pairs does not take it (MI_ERR_FLAGS). */
#define MI_COMPACT_SLABS 0x8000
/* mi_workspace_size: size the workspace for mi_grad (adds the dMI/dp
 * tables).  Accepted (and implied) by mi_grad; rejected (MI_ERR_FLAGS) by
 * the other calls. */
#define MI_GRADIENT 0x10000

#define MI_MAX_Q 16
#define MI_MAX_EDGE 4096

/* A volume: tightly packed C-order [nz][ny][nx] (x fastest) on the device,
 * placed in physical space by its spacing and origin. */
typedef struct mi_volume {
  const void *data; /* device pointer, nx*ny*nz elements of `dtype`        */
  int32_t nx, ny, nz; /* each in [2, 4096]; nx*ny*nz <= 2^28 */
  int32_t dtype;      /* MI_U8, MI_U16, MI_I16 or MI_F32                   */
  double spacing[3];  /* mm between voxel centres along x, y, z; finite, > 0 */
  double origin[3];   /* position (mm) of the centre of voxel (0, 0, 0); finite */
  double lo, hi;      /* intensity range mapped onto the bins              */
} mi_volume;

/* Opaque per-device state: device properties, tuning choices, timers. */
typedef struct mi_context mi_context;

/* Creates a context on HIP device `device` (made current for the call).
 * *out receives the context.  MI_ERR_NO_DEVICE if the device does not exist
 * or is not a gfx950 GPU. */
int mi_create(mi_context **out, int device);

/* Destroys a context (NULL is accepted).  Waits for nothing: the caller
 * must have synchronised any stream still using the context. */
int mi_destroy(mi_context *ctx);

/* Bytes of device workspace that mi_eval (hard or Parzen, per `flags`),
 * mi_eval_sampled (with MI_SAMPLED) or mi_grad (with MI_GRADIENT) needs for
 * these arguments.  Host-only; no GPU is touched; `ctx` may be NULL.
 * Validates like the call it sizes. */
int mi_workspace_size(mi_context *ctx, const mi_volume *fixed, const mi_volume *moving,
                      int32_t n_transforms, int32_t bins, int32_t n_q, int32_t flags, size_t *bytes);

/* MI of `n_transforms` candidate transforms (Fig. 1 Transform + Metric;
 * Eq. (1), Eq. (2); one histogram, every q).
 *   transforms  device double[n][12], row-major physical fixed -> moving
 *               3x4 matrices (mm; see Transform above)
 *   bins        histogram bins per axis, 2..256
 *   q, n_q      HOST double[n_q] entropic indices (1.0 = Shannon), n_q <= 16
 *   flags       boundary | tsallis form | MI_HIST_HARD or MI_HIST_PARZEN
 *   mi_out      device double[n][n_q]
 *   overlap_out device uint64[n] voxels that took part, or NULL
 *   hist_out    device uint32[n][bins][bins] joint counts (row = fixed bin),
 *               or NULL; hard histograms only (NULL required with Parzen)
 * The hard path needs an integer moving dtype (MI_U8, MI_U16, MI_I16). */
int mi_eval(mi_context *ctx, const mi_volume *fixed, const mi_volume *moving,
            const double *transforms, int32_t n_transforms, int32_t bins, const double *q,
            int32_t n_q, int32_t flags, double *mi_out, uint64_t *overlap_out,
            uint32_t *hist_out, void *workspace, size_t workspace_bytes, void *stream);

/* MI over a random subsample of the fixed voxels (Discussion: Mattes' MI
 * samples voxels at random where MI over all voxels does not, and the paper
 * leaves the effect of that sampling -- with binned histograms -- open).
 * Arguments and results as mi_eval (hard or Parzen per `flags`), computed
 * over the kept fixed voxels only; overlap_out counts the kept voxels that
 * took part (the MI normaliser).  Fixed voxel i (linear index
 * z*ny*nx + y*nx + x) is kept when the top 32 bits of the SplitMix64 output
 * for counter i of the stream seeded with `seed` -- i.e. of
 * mix(seed + (i + 1) * 0x9E3779B97F4A7C15) (Steele, Lea and Flood, OOPSLA
 * 2014) -- are below floor(fraction * 2^32); every voxel when fraction >= 1.
 * The sample depends only on (seed, fraction, fixed volume shape).
 *   fraction  in (0, 1]: expected share of fixed voxels kept
 *   seed      any 64-bit value
 * Workspace: mi_workspace_size() with MI_SAMPLED in `flags`.  Always
 * prepares the volumes (MI_VOLUMES_UNCHANGED is ignored).  MI_ERR_SAMPLE
 * for a fraction that is not finite or not above 0. */
int mi_eval_sampled(mi_context *ctx, const mi_volume *fixed, const mi_volume *moving,
                    const double *transforms, int32_t n_transforms, int32_t bins, const double *q,
                    int32_t n_q, int32_t flags, double fraction, uint64_t seed, double *mi_out,
                    uint64_t *overlap_out, uint32_t *hist_out, void *workspace,
                    size_t workspace_bytes, void *stream);

/* Parzen MI and its gradient with respect to the 12 entries of each
 * physical matrix (what a gradient optimiser of Eq. (3) consumes).
 *   mi_out    device double[n][n_q]
 *   grad_out  device double[n][n_q][12], d MI / d P[r][c] at index r*4+c,
 *             P the caller's physical matrix (the sweep differentiates with
 *             respect to the index-space entries; the library applies the
 *             chain rule of the composition above)
 * `flags` selects boundary and Tsallis form; the histogram is always the
 * Parzen one (MI_HIST_PARZEN may be given or not).  The gradient holds the
 * set of overlapping voxels fixed (exact for MI_BOUNDARY_CLAMP). */
int mi_grad(mi_context *ctx, const mi_volume *fixed, const mi_volume *moving,
            const double *transforms, int32_t n_transforms, int32_t bins, const double *q,
            int32_t n_q, int32_t flags, double *mi_out, double *grad_out, void *workspace,
            size_t workspace_bytes, void *stream);

/* One fixed/moving pair and its own physical transforms (device
 * double[n][12]), each volume with its own spacing and origin. */
typedef struct mi_pair {
  mi_volume fixed, moving;
  const double *transforms;
  int32_t n_transforms;
} mi_pair;

/* Hard-binned MI of many volume pairs of uneven sizes in one persistent
 * launch.  `pairs` is a HOST array; mi_out is device double[sum n][n_q],
 * pairs' rows concatenated in order.  Every pair uses `bins`, `q`, `flags`.
 * Workspace: mi_pairs_workspace_size().  Flags: boundary, Tsallis form,
 * MI_USE_GRAPH, and MI_VOLUMES_UNCHANGED (the caller asserts that every
 * pair's volumes, the bins and the workspace are those of the previous
 * mi_eval_pairs call on this context and that no contents changed: the
 * pairs' fixed bins and oct volumes in the workspace are reused; the
 * transforms are always read afresh).  The launch shape is the one
 * mi_tune_pairs chose for this class of pair set, if any. */
int mi_pairs_workspace_size(const mi_pair *pairs, int32_t n_pairs, int32_t bins, int32_t n_q,
                            int32_t flags, size_t *bytes);
int mi_eval_pairs(mi_context *ctx, const mi_pair *pairs, int32_t n_pairs, int32_t bins,
                  const double *q, int32_t n_q, int32_t flags, double *mi_out, void *workspace,
                  size_t workspace_bytes, void *stream);

/* Discrete gradient paths on a parameter-space map (Results: the metric of
 * one transform family -- translation, rotation or scale -- evaluated over
 * a 3D grid of its parameters, and the paths a gradient method follows on
 * that map; Discussion: the capture range of each entropy).  A path steps
 * from a grid point to the 26-connected neighbour of steepest rise of
 * direction * values, the rise scaled by the reciprocal step length (1, or
 * the fp64 values nearest 1/sqrt(2) and 1/sqrt(3)), ties to the first
 * neighbour in (dz, dy, dx) order, each running -1, 0, 1; it stops at a
 * point no neighbour rises from (a local extremum; NaN points are extrema
 * and never entered).
 *   values     device double[nz][ny][nx] (x fastest), e.g. one q's values
 *              of mi_eval over a grid of transforms
 *   direction  +1: paths climb to maxima; -1: they descend to minima
 *   cx, cy, cz grid index of the expected optimum (the map's centre)
 *   next_out   device int32[nz*ny*nx]: each point's successor (itself at an
 *              extremum), as a flat index z*ny*nx + y*nx + x
 *   sink_out   device int32[nz*ny*nx]: the extremum each point's path ends at
 *   stats_out  device int64[4]: number of extrema; the extremum the centre's
 *              path ends at; how many points end there; the capture radius,
 *              the largest r such that every point within Chebyshev
 *              distance r of the centre ends there (the largest such
 *              distance in the grid when every point does)
 * Errors, before any launch: MI_ERR_NULL (a pointer), MI_ERR_DIMS (an
 * extent outside [1, 4096], more than 2^31 - 1 points, or the centre
 * outside the grid), MI_ERR_FLAGS (direction not +1 or -1).  Asynchronous
 * on `stream`; allocates nothing; the buffers must not overlap. */
int mi_map_paths(mi_context *ctx, const double *values, int32_t nx, int32_t ny, int32_t nz,
                 int32_t direction, int32_t cx, int32_t cy, int32_t cz, int32_t *next_out,
                 int32_t *sink_out, int64_t *stats_out, void *stream);

/* Autotuner of the sweeps of mi_eval, mi_eval_sampled and mi_grad for this
 * problem class (volume shapes, moving dtype, bins, boundary, and the
 * power-of-two bucket of n_transforms): times the kernels on these
 * arguments for every candidate launch shape, keeps the fastest in the
 * context and, when the environment variable MI_TUNE_CACHE names a file,
 * records it there; later contexts read that file at mi_create.
 *  - Hard-binned (flags without MI_HIST_PARZEN): the histogram sweep, over
 *    workgroup sizes 256/512/1024, slab-major or transform-major workgroup
 *    order, three slab counts and (up to 128 bins) u32 or 16-bit LDS
 *    counters.  Results are unaffected (the sweep is exact whatever its
 *    shape).  The workspace is the one mi_eval would use with
 *    hist_out = NULL.
 *  - Parzen (MI_HIST_PARZEN): the forward sweep's, then the backward
 *    sweep's workgroup size (256/512/1024) and LDS band budget (32, 64, 96
 *    or 128 KiB: how many bands of table rows walk the fixed volume), then
 *    the workgroup count (half, as planned, twice, four times), timing
 *    forward and gradient calls with one entropy.  MI changes only in the
 *    last bits (the order in which workgroup partial sums merge), gradients
 *    at the level of the fp32 per-lane partial sums, whose grouping follows
 *    the shape (~1e-7 relative).  The workspace is mi_workspace_size() for
 *    these arguments with n_q = 2 and MI_GRADIENT; its contents are
 *    overwritten.
 * Synchronous: waits for `stream`.  MI_USE_GRAPH and MI_VOLUMES_UNCHANGED
 * are ignored; MI_SAMPLED and MI_GRADIENT give MI_ERR_FLAGS.
 * Environment defaults read at mi_create for untuned classes (measurement
 * aids): MI_TUNE_HARD_BLOCK, MI_TUNE_HARD_ORDER, MI_TUNE_HARD_CHUNKS,
 * MI_TUNE_PARZEN_BLOCK, MI_TUNE_PARZEN_LDS_KIB, MI_TUNE_PARZEN_CHUNK_SHIFT. */
int mi_tune(mi_context *ctx, const mi_volume *fixed, const mi_volume *moving,
            const double *transforms, int32_t n_transforms, int32_t bins, int32_t flags,
            void *workspace, size_t workspace_bytes, void *stream);

/* Autotuner of the persistent multi-pair sweep (mi_eval_pairs: the
 * batched evaluation behind the Methodology's exhaustive per-family
 * sweeps, over many volume pairs).
 * Prepares the pairs once, then times the sweep for every candidate launch
 * shape -- workgroup size 256/512/1024, about 64 K / 128 K / 256 K fixed
 * voxels per slab (a work item sweeps one slab for one transform), u32 or
 * packed 16-bit LDS counters (16-bit only with slabs of at most 65535
 * voxels; forced above 128 bins) and slab-major or transform-major work
 * items -- and keeps the fastest for this class of pair set (power-of-two
 * buckets of the pair count, total fixed voxels and total transforms; bins;
 * boundary; 8-bit corners) in the context, and in the MI_TUNE_CACHE file
 * when that is set.  Results are unaffected (the sweep is exact whatever
 * its shape).  Synchronous: waits for `stream`.  The workspace is the one
 * mi_eval_pairs uses (mi_pairs_workspace_size(), any n_q); its contents are
 * overwritten.  Flags: the boundary; MI_USE_GRAPH and MI_VOLUMES_UNCHANGED
 * are refused (MI_ERR_FLAGS). */
int mi_tune_pairs(mi_context *ctx, const mi_pair *pairs, int32_t n_pairs, int32_t bins, int32_t flags,
                  void *workspace, size_t workspace_bytes, void *stream);

/* Kernel timing.  While enabled, the library brackets every launch of its
 * histogram kernels with HIP events on the caller's stream.
 * mi_timing_read() synchronises on those events and returns the summed
 * duration (ms) and number of launches of kernel `which`
 * (0 = hard histogram, 1 = Parzen forward, 2 = Parzen backward,
 * 3 = pairs histogram, 4 = MI reduction), then clears that record. */
int mi_timing_enable(mi_context *ctx, int enable);
int mi_timing_read(mi_context *ctx, int which, double *total_ms, int64_t *launches);

/* Measurement probe (not part of the metric): the device's peak rate of
 * conflict-free 32-bit LDS atomic adds, in lane-atomics per second, the
 * ceiling for the LDS-atomic rate of the histogram sweeps.  Synchronous:
 * launches a short kernel on `stream`, waits for it and times it with HIP
 * events.  `scratch` is a device buffer of at least `scratch_bytes` >= 4 MiB
 * (overwritten).  Errors: MI_ERR_NULL, MI_ERR_WORKSPACE, MI_ERR_HIP. */
int mi_probe_lds_atomics(mi_context *ctx, void *scratch, size_t scratch_bytes, void *stream,
                         double *lane_atomics_per_s);

/* Allocation-free variant of mi_eval, for callers that cannot allocate
 * device memory or call allocating routines around their launches (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, results and errors as mi_eval (hard or Parzen per
 * `flags`), with no workspace: the scratch is a fixed device array of
 * MI_NOALLOC_SCRATCH_BYTES (64 MiB) built into the library, one per GPU,
 * held from the first mi_create on that GPU until the process ends.
 *  - MI_ERR_TOO_LARGE, before any launch, when the call needs more scratch
 *    than that.  It needs at most what mi_workspace_size() gives for the
 *    same arguments (less when hist_out is given: the histograms then go
 *    to the caller's buffer).
 *  - MI_ERR_FLAGS for MI_USE_GRAPH (instantiating a graph allocates; the
 *    caller may capture this call into its own graph instead) and
 *    MI_SAMPLED.  MI_VOLUMES_UNCHANGED is ignored: every call prepares
 *    its volumes.
 *  - Calls no hipMalloc, hipFree, event creation or other allocating
 *    routine; kernel timing (mi_timing_enable) does not record these calls.
 *  - Every call on one GPU, from any context or thread, shares that GPU's
 *    array, which keeps the last call's contents (each call clears what it
 *    needs zeroed).  Calls that overlap on one GPU -- on different streams,
 *    or from different threads without ordering -- race and give wrong
 *    results; order them on one stream. */
#define MI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mi_eval_noalloc(mi_context *ctx, const mi_volume *fixed, const mi_volume *moving,
                    const double *transforms, int32_t n_transforms, int32_t bins, const double *q,
                    int32_t n_q, int32_t flags, double *mi_out, uint64_t *overlap_out,
                    uint32_t *hist_out, void *stream);

/* Static description of a status code (never NULL).  For MI_ERR_HIP the
 * text of the last HIP error seen by this thread is appended. */
const char *mi_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* GEMI_H */
