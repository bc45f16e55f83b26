/* Drives the CPU oracle's entry points on small seeded volumes, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer: out-of-bounds
 * voxel reads (clamped neighbours, ragged edges), histogram writes (bins
 * at both ends of the range), signed overflow in the Q32 coordinates and
 * the entropy loops.  Exit status 0 and no sanitizer report are the pass
 * condition.  Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  const void *data;
  int32_t nx, ny, nz;
  int32_t dtype;
  double lo, hi;
  double spacing[3];
  double origin[3];
} or_volume;

int64_t or_hist_hard(const or_volume *f, const or_volume *m, const double P[12], int bins, int boundary,
                     uint32_t *hist);
void or_eval_hard_sampled(const or_volume *f, const or_volume *m, const double *P, int n, int bins,
                          const double *qs, int nq, int boundary, int form, double fraction, uint64_t seed,
                          double *mi, int64_t *overlap, uint32_t *hist_out);
void or_grad_batch(const or_volume *f, const or_volume *m, const double *P, int n, int bins, const double *qs,
                   int nq, int boundary, int form, double *mi, double *grad);
void or_eval_parzen_sampled(const or_volume *f, const or_volume *m, const double *P, int n, int bins,
                            const double *qs, int nq, int boundary, int form, double fraction, uint64_t seed,
                            double *mi, int64_t *overlap);

static uint64_t state = 0x2545F4914F6CDD1Dull;
static double urand(void) {  /* xorshift64*, in [0, 1) */
  state ^= state >> 12;
  state ^= state << 25;
  state ^= state >> 27;
  return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) / 9007199254740992.0;
}

static void volume(or_volume *v, void *buf, int nx, int ny, int nz, int dtype, double lo, double hi) {
  size_t n = (size_t)nx * ny * nz;
  for (size_t i = 0; i < n; ++i) {
    double u = lo + urand() * (hi - lo + 1.0);
    switch (dtype) {
    case 0: ((uint8_t *)buf)[i] = (uint8_t)fmin(u, 255); break;
    case 1: ((uint16_t *)buf)[i] = (uint16_t)fmin(u, 65535); break;
    case 2: ((int16_t *)buf)[i] = (int16_t)fmax(fmin(u, 32767), -32768); break;
    default: ((float *)buf)[i] = (float)(lo + urand() * (hi - lo)); break;
    }
  }
  v->data = buf;
  v->nx = nx; v->ny = ny; v->nz = nz;
  v->dtype = dtype;
  v->lo = lo; v->hi = hi;
  for (int r = 0; r < 3; ++r) {
    v->spacing[r] = 0.5 + urand();
    v->origin[r] = -10.0 + 20.0 * urand();
  }
}

int main(void) {
  static uint8_t fb[7 * 5 * 3 * 4], mb[6 * 6 * 4 * 4];
  or_volume f, m;
  const double qs[4] = {1.0, 0.5, 2.0, 1.3};
  const int dtypes[4] = {0, 1, 2, 3};
  for (int trial = 0; trial < 24; ++trial) {
    int fd = dtypes[trial % 4], md = dtypes[(trial / 4) % 3];
    double flo = fd == 2 ? -1000 : 0, fhi = fd == 0 ? 255 : (fd == 3 ? 1.0 : 4095);
    double mlo = md == 2 ? -1000 : 0, mhi = md == 0 ? 255 : 4095;
    volume(&f, fb, 7, 5, 3, fd, flo, fhi);
    volume(&m, mb, 6, 6, 4, md, mlo, mhi);
    /* transforms: identity-like, rotated, far outside, non-finite, beyond the limits */
    double P[5][12];
    for (int t = 0; t < 5; ++t) {
      for (int e = 0; e < 12; ++e) P[t][e] = (e % 5 == 0 ? 1.0 : 0.0) + 0.3 * (urand() - 0.5);
      for (int r = 0; r < 3; ++r) P[t][4 * r + 3] = 4.0 * (urand() - 0.5);
    }
    P[2][3] = 1e6;
    P[3][7] = NAN;
    P[4][0] = 1e9;
    int bins = (trial % 3 == 0) ? 2 : ((trial % 3 == 1) ? 16 : 64);
    for (int boundary = 0; boundary < 2; ++boundary) {
      uint32_t *h = calloc((size_t)bins * bins * 5, sizeof(uint32_t));
      double mi[5 * 4];
      int64_t ov[5];
      if (md != 3) {
        or_hist_hard(&f, &m, P[0], bins, boundary, h);
        or_eval_hard_sampled(&f, &m, &P[0][0], 5, bins, qs, 4, boundary, trial & 1, trial % 2 ? 0.4 : 1.0,
                             (uint64_t)trial, mi, ov, h);
      }
      if (bins >= 8) {
        double g[5 * 4 * 12];
        or_grad_batch(&f, &m, &P[0][0], 5, bins, qs, 4, boundary, trial & 1, mi, g);
        or_eval_parzen_sampled(&f, &m, &P[0][0], 5, bins, qs, 4, boundary, 0, 0.5, 99, mi, ov);
      }
      free(h);
    }
  }
  puts("oracle driver ok");
  return 0;
}
