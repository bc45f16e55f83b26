// Reduction of one joint table per transform to Shannon MI (Eq. (1),
// Eq. (2)) and Tsallis MI for every requested q -- the same table serves
// every entropy (Discussion).  fp64 with compensated (Neumaier) partial
// sums per thread, wave64 shuffles and an ordered cross-wave combine, so
// the result does not depend on scheduling.
//
// With p = h / N over the cells of X (N = total count or, for Parzen
// tables, the number of voxels that took part):
//   Shannon  H(X) = -sum p ln p,                MI = H(F) + H(M) - H(F,M)
//   Tsallis  S_q(X) = -sum p expm1((q-1) ln p) / (q-1)
//            I_q = S_q(F) + S_q(M) - S_q(F,M)  [+ (1-q) S_q(F) S_q(M), pseudo-additive]
// The expm1 form of (1 - sum p^q)/(q-1) keeps q near 1 free of cancellation.
#include "common.h"

namespace gemi {

struct Comp {
  double s, c;
};

__device__ __forceinline__ void comp_add(Comp& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}

// (s1, c1) + (s2, c2) with the rounding error of s1 + s2 kept (TwoSum).
__device__ __forceinline__ Comp comp_merge(Comp a, Comp b) {
  const double s = a.s + b.s;
  const double bb = s - a.s;
  const double err = (a.s - (s - bb)) + (b.s - bb);
  Comp r;
  r.s = s;
  r.c = a.c + b.c + err;
  return r;
}

// Block-wide sum of three compensated accumulators; every thread gets the
// result.  Fixed combine order: xor-shuffle tree inside each wave, then
// waves in index order.
__device__ void block_sum3(Comp v[3], double out[3]) {
  __shared__ Comp part[kBlock / 64][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      Comp o;
      o.s = __shfl_xor(v[k].s, off, 64);
      o.c = __shfl_xor(v[k].c, off, 64);
      v[k] = comp_merge(v[k], o);
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int k = 0; k < 3; ++k) part[wave][k] = v[k];
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    Comp acc = part[0][k];
    for (int w = 1; w < kBlock / 64; ++w) acc = comp_merge(acc, part[w][k]);
    out[k] = acc.s + acc.c;
  }
  __syncthreads();
}

template <bool TABLE>
__global__ __launch_bounds__(kBlock) void mi_reduce_kernel(ReduceLaunch L) {
  const int B = L.bins;
  const size_t BB = (size_t)B * B;
  const int t = blockIdx.x;
  __shared__ double row[256], col[256];
  __shared__ double total_sh;

  int64_t Mq[12];
  const bool ok = quantize_transform(L.transforms + 12 * (size_t)t, Mq);
  if (!ok) {
    if (threadIdx.x < L.q.n) L.mi_out[(size_t)t * L.q.n + threadIdx.x] = __longlong_as_double(0x7FF8000000000000ll);
    if (threadIdx.x == 0 && L.overlap_out) L.overlap_out[t] = 0;
    return;
  }
  const uint32_t* __restrict__ h32 = TABLE ? nullptr : L.hist + t * BB;
  const double* __restrict__ hd = TABLE ? L.table + t * BB : nullptr;
  auto cell = [&](size_t e) -> double { return TABLE ? hd[e] : (double)h32[e]; };

  // marginals: exact for counts (integer sums < 2^53), compensated for masses
  for (int i = threadIdx.x; i < B; i += kBlock) {
    Comp r = {0, 0}, c = {0, 0};
    for (int k = 0; k < B; ++k) {
      comp_add(r, cell((size_t)i * B + k));
      comp_add(c, cell((size_t)k * B + i));
    }
    row[i] = r.s + r.c;
    col[i] = c.s + c.c;
  }
  __syncthreads();
  double N;
  uint64_t n_int = 0;
  if (TABLE) {
    n_int = L.count[t];
    N = (double)n_int;
  } else {
    if (threadIdx.x == 0) {
      double s = 0;
      for (int i = 0; i < B; ++i) s += row[i];  // integers: exact
      total_sh = s;
    }
    __syncthreads();
    N = total_sh;
    n_int = (uint64_t)N;
  }
  if (threadIdx.x == 0 && L.overlap_out) L.overlap_out[t] = n_int;
  if (!(N > 0)) {
    if (threadIdx.x < L.q.n) L.mi_out[(size_t)t * L.q.n + threadIdx.x] = 0.0;
    return;
  }
  const double invN = 1.0 / N;

  for (int iq = 0; iq < L.q.n; ++iq) {
    const double q = L.q.q[iq];
    const bool shannon = (q == 1.0);
    const double qm1 = q - 1.0;
    Comp acc[3] = {{0, 0}, {0, 0}, {0, 0}};  // joint, fixed, moving
    for (size_t e = threadIdx.x; e < BB; e += kBlock) {
      const double h = cell(e);
      if (h > 0) {
        const double p = h * invN, lp = log(p);
        comp_add(acc[0], shannon ? p * lp : p * expm1(qm1 * lp));
      }
    }
    for (int i = threadIdx.x; i < B; i += kBlock) {
      const double hr = row[i], hc = col[i];
      if (hr > 0) {
        const double p = hr * invN, lp = log(p);
        comp_add(acc[1], shannon ? p * lp : p * expm1(qm1 * lp));
      }
      if (hc > 0) {
        const double p = hc * invN, lp = log(p);
        comp_add(acc[2], shannon ? p * lp : p * expm1(qm1 * lp));
      }
    }
    double s[3];
    block_sum3(acc, s);
    if (threadIdx.x == 0) {
      double I;
      if (shannon) {
        I = (s[0] - s[1]) - s[2];
      } else {
        const double Sj = -s[0] / qm1, Sf = -s[1] / qm1, Sm = -s[2] / qm1;
        I = (Sf + Sm) - Sj;
        if (L.q.pseudo) I += (1.0 - q) * Sf * Sm;
      }
      L.mi_out[(size_t)t * L.q.n + iq] = I;
    }
  }
}

hipError_t launch_mi_reduce(const ReduceLaunch& L, hipStream_t s) {
  if (L.n == 0) return hipSuccess;
  if (L.table)
    hipLaunchKernelGGL(mi_reduce_kernel<true>, dim3(L.n), dim3(kBlock), 0, s, L);
  else
    hipLaunchKernelGGL(mi_reduce_kernel<false>, dim3(L.n), dim3(kBlock), 0, s, L);
  return hipGetLastError();
}

}  // namespace gemi
