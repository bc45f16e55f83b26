/*
 * CPU oracle for the generalised-entropy mutual-information metric of
 * Vianna & Murta, "Analysis of Generalized Entropies in Mutual Information
 * Medical Image Registration" (arXiv 1909.10690).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with
 * the GPU path.
 *
 * Every quantity is computed the plain way: one voxel at a time, coordinates
 * computed directly from the matrix (never incrementally), the eight
 * trilinear corners summed explicitly in 128-bit integers, bins found with a
 * 128-bit division, entropies in long double with compensated summation.
 *
 * What is computed (the paper prints only Eq. (1), Eq. (2) and Eq. (3); every
 * other rule below is a stated reading, listed with its reason in the design
 * notes of the repository):
 *
 *  - Transform block of Fig. 1: a physical 3x4 affine map P takes a point
 *    of the fixed volume (mm) to a point of the moving volume (mm).  Voxel
 *    index i of a volume sits at origin + spacing * i (voxel centres), so
 *    the map from fixed voxel index to continuous moving index is
 *    M = S_m^-1 (P (o_f + S_f i) - o_m), composed in fp64 in a fixed order
 *    of single IEEE operations (or_compose).  M is quantised once to signed
 *    Q32 fixed point, Mq = round-half-even(M * 2^32).
 *  - Overlap (EXCLUDE): a voxel counts iff every moving coordinate lies in
 *    the closed interval [0, n-1]; CLAMP clamps the coordinate instead and
 *    counts every fixed voxel.
 *  - Trilinear interpolation with 16-bit truncated weights
 *    w = floor(frac * 2^16), exact integer sum over the 8 corners.
 *  - Hard binning: bin = floor(value * B / R), R = hi - lo + 1, after the
 *    intensity is clamped to [lo, hi] and offset by lo.
 *  - Joint histogram of (fixed bin, moving bin) over the overlap, the "full
 *    histogram over all voxels" of the Discussion.
 *  - Shannon entropies, Eq. (1), natural log; MI, Eq. (2); Tsallis entropy
 *    S_q = (1 - sum p^q)/(q - 1) evaluated in the stable form
 *    -sum p * expm1((q-1) ln p)/(q-1); Tsallis MI additive by default
 *    (Eq. (2) with S_q), pseudo-additive on request.  One histogram serves
 *    every q (Discussion).
 *  - Parzen variant: fixed side hard-binned, moving side weighted by the
 *    cubic B-spline beta3 at s = 1 + (v - lo)/(hi - lo) * (B - 4); fp64
 *    trilinear value; gradient of every MI output with respect to the 12
 *    entries of P (the quantity a gradient optimiser for Eq. (3) needs).
 *  - Random subsampling (Discussion: Mattes' MI samples voxels at random,
 *    MI over all voxels does not, and the effect is left open): fixed voxel
 *    i (linear index, x fastest) takes part iff the top 32 bits of the
 *    SplitMix64 output for counter i under a seed are below
 *    floor(fraction * 2^32) (every voxel when fraction >= 1).  SplitMix64
 *    (Steele, Lea and Flood, OOPSLA 2014) is written here from its
 *    published definition: the i-th output (from 0) of the stream seeded
 *    with s mixes s + (i + 1) * 0x9E3779B97F4A7C15.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_U8 = 0, OR_U16 = 1, OR_I16 = 2, OR_F32 = 3 };
enum { OR_EXCLUDE = 0, OR_CLAMP = 1 };
enum { OR_ADDITIVE = 0, OR_PSEUDOADDITIVE = 1 };

typedef struct {
  const void *data; /* C order [nz][ny][nx], x fastest */
  int32_t nx, ny, nz;
  int32_t dtype;
  double lo, hi;
  double spacing[3]; /* mm per voxel along x, y, z */
  double origin[3];  /* position (mm) of the centre of voxel (0, 0, 0) */
} or_volume;

typedef __int128 i128;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* voxel access                                                        */
/* ------------------------------------------------------------------ */

static int64_t vox_int(const or_volume *v, int64_t ix, int64_t iy, int64_t iz) {
  int64_t idx = (iz * v->ny + iy) * v->nx + ix;
  switch (v->dtype) {
  case OR_U8: return ((const uint8_t *)v->data)[idx];
  case OR_U16: return ((const uint16_t *)v->data)[idx];
  case OR_I16: return ((const int16_t *)v->data)[idx];
  default: return 0;
  }
}

static double vox_real(const or_volume *v, int64_t ix, int64_t iy, int64_t iz) {
  int64_t idx = (iz * v->ny + iy) * v->nx + ix;
  switch (v->dtype) {
  case OR_U8: return ((const uint8_t *)v->data)[idx];
  case OR_U16: return ((const uint16_t *)v->data)[idx];
  case OR_I16: return ((const int16_t *)v->data)[idx];
  case OR_F32: return ((const float *)v->data)[idx];
  default: return 0.0;
  }
}

/* ------------------------------------------------------------------ */
/* transform quantisation                                              */
/* ------------------------------------------------------------------ */

/* Fixed voxel index -> continuous moving index of the physical map P:
 *   M[r][c] = (P[r][c] * sf[c]) / sm[r]                                (c < 3)
 *   M[r][3] = ((((P[r][0]*of[0] + P[r][1]*of[1]) + P[r][2]*of[2]) + P[r][3]) - om[r]) / sm[r]
 * each operation rounded once (the file is built without contraction), in
 * this order: the library documents the same order, so both sides quantise
 * the same fp64 matrix. */
void or_compose(const or_volume *f, const or_volume *m, const double P[12], double M[12]) {
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      double a = P[4 * r + c] * f->spacing[c];
      M[4 * r + c] = a / m->spacing[r];
    }
    double o = P[4 * r + 0] * f->origin[0];
    double o1 = P[4 * r + 1] * f->origin[1];
    o = o + o1;
    double o2 = P[4 * r + 2] * f->origin[2];
    o = o + o2;
    o = o + P[4 * r + 3];
    o = o - m->origin[r];
    M[4 * r + 3] = o / m->spacing[r];
  }
}

/* Linear entries are bounded by 2^16 and translations by 2^24 so that, for
 * volumes of at most 4096 voxels per axis, every coordinate fits in int64.
 * Returns 0 when the matrix is usable, 1 when it is not (non-finite or out
 * of range); an unusable matrix yields NaN MI and an empty histogram. */
int or_quantize(const double M[12], int64_t Mq[12]) {
  for (int e = 0; e < 12; ++e) {
    double m = M[e];
    double lim = (e % 4 == 3) ? 16777216.0 : 65536.0;
    if (!isfinite(m) || fabs(m) > lim) {
      for (int f = 0; f < 12; ++f) Mq[f] = 0;
      return 1;
    }
  }
  for (int e = 0; e < 12; ++e) Mq[e] = (int64_t)llrint(ldexp(M[e], 32));
  return 0;
}

/* Moving coordinate r (Q32) of fixed voxel (i,j,k), computed directly. */
static i128 coord_q32(const int64_t Mq[12], int r, int64_t i, int64_t j, int64_t k) {
  return (i128)Mq[4 * r + 0] * i + (i128)Mq[4 * r + 1] * j + (i128)Mq[4 * r + 2] * k +
         (i128)Mq[4 * r + 3];
}

/* Applies the overlap rule to the three coordinates.  Returns 1 if the voxel
 * takes part; clamped[r] tells whether axis r was clamped (CLAMP only). */
static int overlap_rule(const or_volume *m, int boundary, i128 q[3], int clamped[3]) {
  const int64_t n[3] = {m->nx, m->ny, m->nz};
  for (int r = 0; r < 3; ++r) {
    i128 top = (i128)(n[r] - 1) << 32;
    clamped[r] = 0;
    if (q[r] < 0 || q[r] > top) {
      if (boundary == OR_EXCLUDE) return 0;
      q[r] = q[r] < 0 ? 0 : top;
      clamped[r] = 1;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* hard-binned joint histogram                                         */
/* ------------------------------------------------------------------ */

static int64_t fixed_bin_int(const or_volume *f, int64_t u, int bins) {
  int64_t lo = (int64_t)f->lo, hi = (int64_t)f->hi;
  if (u < lo) u = lo;
  if (u > hi) u = hi;
  int64_t R = hi - lo + 1;
  return ((u - lo) * (int64_t)bins) / R;
}

static int64_t fixed_bin_real(const or_volume *f, double u, int bins) {
  if (u < f->lo) u = f->lo;
  if (u > f->hi) u = f->hi;
  double d = u - f->lo;
  double r = d / (f->hi - f->lo);
  double t = r * (double)bins;
  int64_t b = (int64_t)floor(t);
  if (b > bins - 1) b = bins - 1;
  if (b < 0) b = 0;
  return b;
}

/* Fixed bin of voxel (i,j,k), integer rule for integer dtypes and the fp64
 * rule floor(((u-lo)/(hi-lo)) * B), capped at B-1, for fp32. */
static int64_t fixed_bin(const or_volume *f, int64_t i, int64_t j, int64_t k, int bins) {
  if (f->dtype == OR_F32) return fixed_bin_real(f, vox_real(f, i, j, k), bins);
  return fixed_bin_int(f, vox_int(f, i, j, k), bins);
}

/* SplitMix64 output for counter i of the stream seeded with `seed`. */
uint64_t or_splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Whether fixed voxel `lin` takes part at this sampling fraction. */
static int keep_voxel(double fraction, uint64_t seed, int64_t lin) {
  if (fraction >= 1.0) return 1;
  const uint64_t thr = (uint64_t)floor(fraction * 4294967296.0);
  return (or_splitmix64(seed, (uint64_t)lin) >> 32) < thr;
}

/* Joint histogram of one transform over the fixed voxels kept by the
 * sampling rule; hist is bins*bins counts, row = fixed bin, column = moving
 * bin.  Returns the overlap count, or -1 when the transform is unusable
 * (hist left zero). */
int64_t or_hist_hard_sampled(const or_volume *f, const or_volume *m, const double P[12], int bins,
                             int boundary, double fraction, uint64_t seed, uint32_t *hist) {
  memset(hist, 0, sizeof(uint32_t) * (size_t)bins * (size_t)bins);
  double M[12];
  or_compose(f, m, P, M);
  int64_t Mq[12];
  if (or_quantize(M, Mq)) return -1;
  const int64_t mlo = (int64_t)m->lo, mhi = (int64_t)m->hi;
  const u128 R = (u128)(mhi - mlo + 1);
  const int64_t mn[3] = {m->nx, m->ny, m->nz};
  int64_t count = 0;
  for (int64_t k = 0; k < f->nz; ++k)
    for (int64_t j = 0; j < f->ny; ++j)
      for (int64_t i = 0; i < f->nx; ++i) {
        if (!keep_voxel(fraction, seed, (k * f->ny + j) * f->nx + i)) continue;
        i128 q[3];
        int clamped[3];
        for (int r = 0; r < 3; ++r) q[r] = coord_q32(Mq, r, i, j, k);
        if (!overlap_rule(m, boundary, q, clamped)) continue;
        int64_t ip[3];
        u128 w[3];
        for (int r = 0; r < 3; ++r) {
          ip[r] = (int64_t)(q[r] >> 32);
          w[r] = (u128)((q[r] >> 16) & 0xFFFF);
        }
        u128 V = 0;
        for (int c = 0; c < 8; ++c) {
          int64_t idx3[3];
          u128 wt = 1;
          for (int r = 0; r < 3; ++r) {
            int up = (c >> r) & 1;
            int64_t t = ip[r] + up;
            if (t > mn[r] - 1) t = mn[r] - 1;
            idx3[r] = t;
            wt *= up ? w[r] : ((u128)65536 - w[r]);
          }
          int64_t val = vox_int(m, idx3[0], idx3[1], idx3[2]);
          if (val < mlo) val = mlo;
          if (val > mhi) val = mhi;
          V += (u128)(val - mlo) * wt;
        }
        int64_t bm = (int64_t)((V * (u128)bins) / (R << 48));
        int64_t bf = fixed_bin(f, i, j, k, bins);
        hist[bf * bins + bm] += 1;
        ++count;
      }
  return count;
}

/* The histogram over every fixed voxel. */
int64_t or_hist_hard(const or_volume *f, const or_volume *m, const double P[12], int bins,
                     int boundary, uint32_t *hist) {
  return or_hist_hard_sampled(f, m, P, bins, boundary, 1.0, 0, hist);
}

/* ------------------------------------------------------------------ */
/* entropies                                                           */
/* ------------------------------------------------------------------ */

typedef struct {
  long double s, c;
} neu_t;

static void neu_add(neu_t *a, long double x) {
  long double t = a->s + x;
  if (fabsl(a->s) >= fabsl(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static long double neu_val(const neu_t *a) { return a->s + a->c; }

/* Shannon entropy, Eq. (1): H = -sum p ln p, p = h / N, zero cells skipped. */
static long double shannon(const long double *h, int64_t n, long double N) {
  neu_t acc = {0, 0};
  for (int64_t e = 0; e < n; ++e)
    if (h[e] > 0) {
      long double p = h[e] / N;
      neu_add(&acc, -p * logl(p));
    }
  return neu_val(&acc);
}

/* Tsallis entropy S_q = (1 - sum p^q)/(q-1), written as
 * -sum p * expm1((q-1) ln p) / (q-1) so that q near 1 does not cancel. */
static long double tsallis(const long double *h, int64_t n, long double N, long double q) {
  neu_t acc = {0, 0};
  for (int64_t e = 0; e < n; ++e)
    if (h[e] > 0) {
      long double p = h[e] / N;
      neu_add(&acc, -p * expm1l((q - 1) * logl(p)));
    }
  return neu_val(&acc) / (q - 1);
}

/* MI of a joint table h[bins][bins] (counts or Parzen masses) normalised by
 * N, for every q (q == 1 means Shannon).  out[iq].  N == 0 gives 0. */
static void mi_from_table(const long double *h, int bins, long double N, const double *qs,
                          int nq, int form, double *out) {
  if (!(N > 0)) {
    for (int a = 0; a < nq; ++a) out[a] = 0.0;
    return;
  }
  long double *hf = calloc((size_t)bins, sizeof(long double));
  long double *hm = calloc((size_t)bins, sizeof(long double));
  for (int a = 0; a < bins; ++a) {
    neu_t rs = {0, 0};
    for (int b = 0; b < bins; ++b) neu_add(&rs, h[(int64_t)a * bins + b]);
    hf[a] = neu_val(&rs);
  }
  for (int b = 0; b < bins; ++b) {
    neu_t cs = {0, 0};
    for (int a = 0; a < bins; ++a) neu_add(&cs, h[(int64_t)a * bins + b]);
    hm[b] = neu_val(&cs);
  }
  int64_t nn = (int64_t)bins * bins;
  for (int a = 0; a < nq; ++a) {
    long double q = qs[a];
    long double I;
    if (q == 1.0L) {
      I = shannon(hf, bins, N) + shannon(hm, bins, N) - shannon(h, nn, N);
    } else {
      long double Sf = tsallis(hf, bins, N, q), Sm = tsallis(hm, bins, N, q);
      long double Sj = tsallis(h, nn, N, q);
      I = Sf + Sm - Sj;
      if (form == OR_PSEUDOADDITIVE) I += (1 - q) * Sf * Sm;
    }
    out[a] = (double)I;
  }
  free(hf);
  free(hm);
}

/* MI (every q) of a count histogram with total N. */
void or_mi_from_counts(const uint32_t *hist, int bins, int64_t N, const double *qs, int nq,
                       int form, double *out) {
  int64_t nn = (int64_t)bins * bins;
  long double *h = malloc(sizeof(long double) * (size_t)nn);
  for (int64_t e = 0; e < nn; ++e) h[e] = hist[e];
  mi_from_table(h, bins, (long double)N, qs, nq, form, out);
  free(h);
}

/* MI (every q) of a real-valued table with normaliser N (Parzen masses). */
void or_mi_from_table(const double *table, int bins, double N, const double *qs, int nq,
                      int form, double *out) {
  int64_t nn = (int64_t)bins * bins;
  long double *h = malloc(sizeof(long double) * (size_t)nn);
  for (int64_t e = 0; e < nn; ++e) h[e] = table[e];
  mi_from_table(h, bins, (long double)N, qs, nq, form, out);
  free(h);
}

/* Hard-binned MI of n physical transforms (row-major [n][12]).  mi[n][nq] and
 * overlap[n]; an unusable transform gives NaN MI and overlap 0.  Transforms
 * are independent, so they are spread over OpenMP threads. */
void or_eval_hard_sampled(const or_volume *f, const or_volume *m, const double *P, int n, int bins,
                          const double *qs, int nq, int boundary, int form, double fraction,
                          uint64_t seed, double *mi, int64_t *overlap, uint32_t *hist_out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < n; ++t) {
    size_t nn = (size_t)bins * bins;
    uint32_t *h = hist_out ? hist_out + nn * (size_t)t : malloc(sizeof(uint32_t) * nn);
    int64_t N = or_hist_hard_sampled(f, m, P + 12 * t, bins, boundary, fraction, seed, h);
    if (N < 0) {
      for (int a = 0; a < nq; ++a) mi[(size_t)t * nq + a] = NAN;
      overlap[t] = 0;
    } else {
      or_mi_from_counts(h, bins, N, qs, nq, form, mi + (size_t)t * nq);
      overlap[t] = N;
    }
    if (!hist_out) free(h);
  }
}

void or_eval_hard(const or_volume *f, const or_volume *m, const double *P, int n, int bins,
                  const double *qs, int nq, int boundary, int form, double *mi,
                  int64_t *overlap, uint32_t *hist_out) {
  or_eval_hard_sampled(f, m, P, n, bins, qs, nq, boundary, form, 1.0, 0, mi, overlap, hist_out);
}

/* ------------------------------------------------------------------ */
/* Parzen (cubic B-spline) variant and its gradient                    */
/* ------------------------------------------------------------------ */

/* Centred cubic B-spline and its derivative. */
double or_beta3(double t) {
  double a = fabs(t);
  if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
  if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
  return 0.0;
}

double or_dbeta3(double t) {
  double a = fabs(t);
  double sg = t < 0 ? -1.0 : 1.0;
  if (a < 1.0) return -2.0 * t + 1.5 * t * a;
  if (a < 2.0) return -sg * (2.0 - a) * (2.0 - a) / 2.0;
  return 0.0;
}

/* Clamped moving intensity at a voxel, as a real number. */
static double mval(const or_volume *m, int64_t ix, int64_t iy, int64_t iz) {
  double v = vox_real(m, ix, iy, iz);
  if (v < m->lo) v = m->lo;
  if (v > m->hi) v = m->hi;
  return v;
}

/* Per-voxel sample of the Parzen path: interpolated value, its gradient
 * with respect to the moving coordinate, and the B-spline centre s. */
typedef struct {
  int take;
  int64_t bf;
  double v, s, dv[3];
} psample;

static psample parzen_sample(const or_volume *f, const or_volume *m, const int64_t Mq[12],
                             int bins, int boundary, int64_t i, int64_t j, int64_t k) {
  psample out;
  memset(&out, 0, sizeof out);
  i128 q[3];
  int clamped[3];
  for (int r = 0; r < 3; ++r) q[r] = coord_q32(Mq, r, i, j, k);
  if (!overlap_rule(m, boundary, q, clamped)) return out;
  const int64_t mn[3] = {m->nx, m->ny, m->nz};
  int64_t ip[3];
  double t[3];
  for (int r = 0; r < 3; ++r) {
    ip[r] = (int64_t)(q[r] >> 32);
    t[r] = (double)(uint32_t)(q[r] & 0xFFFFFFFF) / 4294967296.0;
  }
  /* corner values c[x][y][z] */
  double c[2][2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int d = 0; d < 2; ++d) {
        int64_t ix = ip[0] + a, iy = ip[1] + b, iz = ip[2] + d;
        if (ix > mn[0] - 1) ix = mn[0] - 1;
        if (iy > mn[1] - 1) iy = mn[1] - 1;
        if (iz > mn[2] - 1) iz = mn[2] - 1;
        c[a][b][d] = mval(m, ix, iy, iz);
      }
  double wx[2] = {1.0 - t[0], t[0]}, wy[2] = {1.0 - t[1], t[1]}, wz[2] = {1.0 - t[2], t[2]};
  double v = 0, gx = 0, gy = 0, gz = 0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int d = 0; d < 2; ++d) {
        double val = c[a][b][d];
        v += val * wx[a] * wy[b] * wz[d];
        gx += val * (a ? 1.0 : -1.0) * wy[b] * wz[d];
        gy += val * wx[a] * (b ? 1.0 : -1.0) * wz[d];
        gz += val * wx[a] * wy[b] * (d ? 1.0 : -1.0);
      }
  /* a coordinate that was clamped, or sits on the last sample (its upper
   * neighbour is the sample itself), does not move the value along r */
  double g[3] = {gx, gy, gz};
  for (int r = 0; r < 3; ++r)
    if (clamped[r] || ip[r] >= mn[r] - 1) g[r] = 0.0;
  double s = 1.0 + (v - m->lo) / (m->hi - m->lo) * (double)(bins - 4);
  if (s < 1.0) s = 1.0;
  if (s > (double)(bins - 3)) s = (double)(bins - 3);
  out.take = 1;
  out.bf = fixed_bin(f, i, j, k, bins);
  out.v = v;
  out.s = s;
  for (int r = 0; r < 3; ++r) out.dv[r] = g[r];
  return out;
}

/* Parzen joint table (unnormalised masses, fp64) of one transform.
 * Returns the number of voxels that took part (the normaliser N), or -1
 * when the transform is unusable. */
int64_t or_parzen_table_sampled(const or_volume *f, const or_volume *m, const double P[12], int bins,
                                int boundary, double fraction, uint64_t seed, double *table) {
  int64_t nn = (int64_t)bins * bins;
  for (int64_t e = 0; e < nn; ++e) table[e] = 0.0;
  double M[12];
  or_compose(f, m, P, M);
  int64_t Mq[12];
  if (or_quantize(M, Mq)) return -1;
  long double *acc = calloc((size_t)nn, sizeof(long double));
  int64_t N = 0;
  for (int64_t k = 0; k < f->nz; ++k)
    for (int64_t j = 0; j < f->ny; ++j)
      for (int64_t i = 0; i < f->nx; ++i) {
        if (!keep_voxel(fraction, seed, (k * f->ny + j) * f->nx + i)) continue;
        psample p = parzen_sample(f, m, Mq, bins, boundary, i, j, k);
        if (!p.take) continue;
        ++N;
        int64_t k0 = (int64_t)floor(p.s) - 1;
        for (int64_t kap = k0; kap < k0 + 4; ++kap) acc[p.bf * bins + kap] += or_beta3((double)kap - p.s);
      }
  for (int64_t e = 0; e < nn; ++e) table[e] = (double)acc[e];
  free(acc);
  return N;
}

int64_t or_parzen_table(const or_volume *f, const or_volume *m, const double P[12], int bins,
                        int boundary, double *table) {
  return or_parzen_table_sampled(f, m, P, bins, boundary, 1.0, 0, table);
}

/* dMI/dp table for one q on a Parzen table h with normaliser N:
 *   Shannon            G = ln(p / p_m)
 *   Tsallis additive   G = q/(q-1) * (p^(q-1) - p_m^(q-1))
 *   Tsallis pseudo     G = q/(q-1) * (p^(q-1) - (1 + (1-q) S_f) p_m^(q-1))
 * G = 0 where p = 0 (no voxel there has a non-zero B-spline slope). */
static void dmi_dp(const double *h, int bins, double N, double q, int form, double *G) {
  long double *hf = calloc((size_t)bins, sizeof(long double));
  long double *hm = calloc((size_t)bins, sizeof(long double));
  for (int a = 0; a < bins; ++a)
    for (int b = 0; b < bins; ++b) {
      hf[a] += h[(int64_t)a * bins + b];
      hm[b] += h[(int64_t)a * bins + b];
    }
  long double Sf = 0;
  if (q != 1.0 && form == OR_PSEUDOADDITIVE) Sf = tsallis(hf, bins, N, q);
  for (int a = 0; a < bins; ++a)
    for (int b = 0; b < bins; ++b) {
      long double hv = h[(int64_t)a * bins + b];
      long double g = 0;
      if (hv > 0) {
        long double p = hv / N, pm = hm[b] / N;
        if (q == 1.0) {
          g = logl(p / pm);
        } else {
          long double e = (long double)q - 1;
          long double fac = (form == OR_PSEUDOADDITIVE) ? 1 + (1 - (long double)q) * Sf : 1;
          g = (long double)q / e * (powl(p, e) - fac * powl(pm, e));
        }
      }
      G[(int64_t)a * bins + b] = (double)g;
    }
  free(hf);
  free(hm);
}

/* Parzen MI and its gradient for one transform.  mi[nq], grad[nq][12]
 * (d MI / d P[r][c] of the physical matrix, row-major r*4+c).  The moving
 * index is y_r = (sum_c P[r][c] x_c + P[r][3] - om[r]) / sm[r] with x the
 * voxel's physical position, so d y_r / d P[r][c] = x_c / sm[r] and
 * d y_r / d P[r][3] = 1 / sm[r].  Returns N, or -1 (unusable). */
int64_t or_parzen_grad(const or_volume *f, const or_volume *m, const double P[12], int bins,
                       const double *qs, int nq, int boundary, int form, double *mi,
                       double *grad) {
  int64_t nn = (int64_t)bins * bins;
  double *h = malloc(sizeof(double) * (size_t)nn);
  int64_t N = or_parzen_table(f, m, P, bins, boundary, h);
  for (int e = 0; e < 12 * nq; ++e) grad[e] = 0.0;
  if (N < 0) {
    for (int a = 0; a < nq; ++a) mi[a] = NAN;
    free(h);
    return -1;
  }
  or_mi_from_table(h, bins, (double)N, qs, nq, form, mi);
  if (N == 0) {
    free(h);
    return 0;
  }
  double M[12];
  or_compose(f, m, P, M);
  int64_t Mq[12];
  or_quantize(M, Mq);
  double *G = malloc(sizeof(double) * (size_t)nn * (size_t)nq);
  for (int a = 0; a < nq; ++a) dmi_dp(h, bins, (double)N, qs[a], form, G + nn * a);
  long double *acc = calloc((size_t)(12 * nq), sizeof(long double));
  for (int64_t k = 0; k < f->nz; ++k)
    for (int64_t j = 0; j < f->ny; ++j)
      for (int64_t i = 0; i < f->nx; ++i) {
        psample p = parzen_sample(f, m, Mq, bins, boundary, i, j, k);
        if (!p.take) continue;
        int64_t k0 = (int64_t)floor(p.s) - 1;
        /* the voxel's physical position, homogeneous */
        const long double xt[4] = {(long double)f->origin[0] + (long double)f->spacing[0] * i,
                                   (long double)f->origin[1] + (long double)f->spacing[1] * j,
                                   (long double)f->origin[2] + (long double)f->spacing[2] * k, 1.0L};
        for (int a = 0; a < nq; ++a) {
          long double w = 0;
          for (int64_t kap = k0; kap < k0 + 4; ++kap)
            w -= (long double)G[nn * a + p.bf * bins + kap] * or_dbeta3((double)kap - p.s);
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 4; ++c)
              acc[12 * a + 4 * r + c] += w * p.dv[r] * xt[c] / (long double)m->spacing[r];
        }
      }
  long double dsdv = (long double)(bins - 4) / ((long double)m->hi - (long double)m->lo);
  for (int e = 0; e < 12 * nq; ++e) grad[e] = (double)(acc[e] * dsdv / (long double)N);
  free(acc);
  free(G);
  free(h);
  return N;
}

/* Parzen MI and gradient of n transforms, OpenMP over transforms. */
void or_grad_batch(const or_volume *f, const or_volume *m, const double *P, int n, int bins,
                   const double *qs, int nq, int boundary, int form, double *mi, double *grad) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < n; ++t)
    or_parzen_grad(f, m, P + 12 * t, bins, qs, nq, boundary, form, mi + (size_t)t * nq,
                   grad + (size_t)t * nq * 12);
}

/* Parzen MI (no gradient) of n transforms. */
void or_eval_parzen_sampled(const or_volume *f, const or_volume *m, const double *P, int n, int bins,
                            const double *qs, int nq, int boundary, int form, double fraction,
                            uint64_t seed, double *mi, int64_t *overlap) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < n; ++t) {
    size_t nn = (size_t)bins * bins;
    double *h = malloc(sizeof(double) * nn);
    int64_t N = or_parzen_table_sampled(f, m, P + 12 * t, bins, boundary, fraction, seed, h);
    if (N < 0) {
      for (int a = 0; a < nq; ++a) mi[(size_t)t * nq + a] = NAN;
      overlap[t] = 0;
    } else {
      or_mi_from_table(h, bins, (double)N, qs, nq, form, mi + (size_t)t * nq);
      overlap[t] = N;
    }
    free(h);
  }
}

void or_eval_parzen(const or_volume *f, const or_volume *m, const double *P, int n, int bins,
                    const double *qs, int nq, int boundary, int form, double *mi,
                    int64_t *overlap) {
  or_eval_parzen_sampled(f, m, P, n, bins, qs, nq, boundary, form, 1.0, 0, mi, overlap);
}

int or_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of later parallel loops (timing at one thread and at all cores). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
