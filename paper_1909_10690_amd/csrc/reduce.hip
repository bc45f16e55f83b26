// Reduction of one joint table per transform to Shannon MI (Eq. (1),
// Eq. (2)) and Tsallis MI for every requested q -- the same table serves
// every entropy (Discussion).  fp64 with compensated (Neumaier) partial
// sums per thread, wave64 shuffles and an ordered cross-wave combine, so
// the result does not depend on scheduling.
//
// Three launches: (hard histograms only) N = sum of the counts, exact in
// 64-bit integers; one workgroup per (transform, row slice) for the partial
// sums of its joint cells and of the marginals of its rows and of the
// same-numbered columns; one small workgroup per transform merging the
// slices in order.  Slicing spreads a single transform over up to B/8 CUs.
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

// N[t] += the counts of the slice's rows (count zeroed beforehand).
__global__ __launch_bounds__(kBlock) void hist_count_kernel(const uint32_t* __restrict__ hist, int B,
                                                            int S, uint64_t* __restrict__ count) {
  const int t = blockIdx.x / S, s = blockIdx.x - t * S;
  int r0, r1;
  slice_rows(B, S, s, r0, r1);
  const uint32_t* __restrict__ h = hist + (size_t)t * B * B;
  uint64_t sum = 0;
  for (int e = r0 * B + threadIdx.x; e < r1 * B; e += kBlock) sum += h[e];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  __shared__ uint64_t wsum[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) tot += wsum[w];
    if (tot) atomicAdd((unsigned long long*)&count[t], (unsigned long long)tot);
  }
}

// One workgroup per (transform, slice): per q, the compensated sums
//   joint  sum over the slice's cells of  f(p)
//   fixed  sum over the slice's rows of   f(row marginal)
//   moving sum over the slice's columns of f(column marginal)
// with f(p) = p ln p (Shannon) or p expm1((q-1) ln p) (Tsallis), p = h / N.
template <bool TABLE, bool CACHED>
__global__ __launch_bounds__(kBlock) void mi_partial_kernel(ReduceLaunch L) {
  const int B = L.bins, S = L.splits;
  const int t = blockIdx.x / S, s = blockIdx.x - t * S;
  int64_t Mq[12];
  if (!quantize_transform(L.transforms + 12 * (size_t)t, Mq)) return;
  const double N = (double)L.count[t];
  if (!(N > 0)) return;
  const double invN = 1.0 / N;
  int r0, r1;
  slice_rows(B, S, s, r0, r1);
  const int R = r1 - r0;
  const size_t BB = (size_t)B * B;
  const uint32_t* __restrict__ h32 = TABLE ? nullptr : L.hist + t * BB;
  const double* __restrict__ hd = TABLE ? L.table + t * BB : nullptr;
  auto cell = [&](size_t e) -> double { return TABLE ? hd[e] : (double)h32[e]; };

  // marginals of the slice's rows (lines 0..R-1) and columns (lines R..2R-1):
  // 8 lanes per line, exact for counts, compensated for masses
  __shared__ double marg[512];
  for (int l0 = 0; l0 < 2 * R; l0 += kBlock / 8) {
    const int line = l0 + (threadIdx.x >> 3), sub = threadIdx.x & 7;
    Comp a = {0, 0};
    if (line < 2 * R) {
      const bool is_row = line < R;
      const int i = r0 + (is_row ? line : line - R);
      for (int k = sub; k < B; k += 8) comp_add(a, cell(is_row ? (size_t)i * B + k : (size_t)k * B + i));
    }
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) {
      Comp o;
      o.s = __shfl_xor(a.s, off, 64);
      o.c = __shfl_xor(a.c, off, 64);
      a = comp_merge(a, o);
    }
    if (sub == 0 && line < 2 * R) {
      marg[line] = a.s + a.c;
      if (L.marg_out) {
        const int i = line < R ? r0 + line : B + r0 + (line - R);
        L.marg_out[(size_t)t * 2 * B + i] = a.s + a.c;
      }
    }
  }
  __syncthreads();

  // CACHED: p and ln p of the slice's cells (first R B entries) and
  // marginals (next 2R) once, so each entropy costs one expm1 per cell
  // (none for Shannon); otherwise ln p is recomputed per entropy
  constexpr int kCache = CACHED ? kMaxSliceCells : 1;  // host: R (B + 2) <= kMaxSliceCells
  __shared__ double pv[kCache], lpv[kCache];
  const int nc = R * B;
  if (CACHED) {
    for (int e = threadIdx.x; e < nc + 2 * R; e += kBlock) {
      const double h = e < nc ? cell((size_t)r0 * B + e) : marg[e - nc];
      const double p = h * invN;
      pv[e] = h > 0 ? p : 0.0;
      lpv[e] = h > 0 ? log(p) : 0.0;
    }
    __syncthreads();
  }
  // per entropy: compensated per-thread sums, a shuffle tree per wave into
  // LDS; after all entropies one barrier and the waves merged in order
  __shared__ Comp wpart[kMaxQ][3][kBlock / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int iq = 0; iq < L.q.n; ++iq) {
    const double q = L.q.q[iq];
    const bool shannon = (q == 1.0);
    const double qm1 = q - 1.0;
    Comp acc[3] = {{0, 0}, {0, 0}, {0, 0}};  // joint, fixed, moving
    for (int e = threadIdx.x; e < nc + 2 * R; e += kBlock) {
      double p, lp;
      if (CACHED) {
        p = pv[e];
        lp = lpv[e];
      } else {
        const double h = e < nc ? cell((size_t)r0 * B + e) : marg[e - nc];
        p = h > 0 ? h * invN : 0.0;
        lp = h > 0 ? log(p) : 0.0;
      }
      if (p > 0) {
        const int k = e < nc ? 0 : (e - nc < R ? 1 : 2);
        comp_add(acc[k], shannon ? p * lp : p * expm1(qm1 * lp));
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        Comp o;
        o.s = __shfl_xor(acc[k].s, off, 64);
        o.c = __shfl_xor(acc[k].c, off, 64);
        acc[k] = comp_merge(acc[k], o);
      }
      if (lane == 0) wpart[iq][k][wave] = acc[k];
    }
  }
  __syncthreads();
  Comp* __restrict__ out = (Comp*)L.part + (size_t)blockIdx.x * L.q.n * 3;
  if (threadIdx.x < L.q.n * 3) {
    const int iq = threadIdx.x / 3, k = threadIdx.x - iq * 3;
    Comp tot = wpart[iq][k][0];
    for (int w = 1; w < kBlock / 64; ++w) tot = comp_merge(tot, wpart[iq][k][w]);
    out[iq * 3 + k] = tot;
  }
}

// One wave per transform: merge the slices in order and form MI per q.
__global__ __launch_bounds__(64) void mi_final_kernel(ReduceLaunch L) {
  const int t = blockIdx.x, iq = threadIdx.x;
  const int S = L.splits;
  int64_t Mq[12];
  if (!quantize_transform(L.transforms + 12 * (size_t)t, Mq)) {
    if (iq < L.q.n) L.mi_out[(size_t)t * L.q.n + iq] = __longlong_as_double(0x7FF8000000000000ll);
    if (iq == 0 && L.overlap_out) L.overlap_out[t] = 0;
    return;
  }
  const uint64_t n_int = L.count[t];
  if (iq == 0 && L.overlap_out) L.overlap_out[t] = n_int;
  if (iq >= L.q.n) return;
  if (n_int == 0) {
    L.mi_out[(size_t)t * L.q.n + iq] = 0.0;
    return;
  }
  const Comp* __restrict__ part = (const Comp*)L.part + (size_t)t * S * L.q.n * 3;
  Comp acc[3] = {part[iq * 3], part[iq * 3 + 1], part[iq * 3 + 2]};
  for (int s = 1; s < S; ++s)
    for (int k = 0; k < 3; ++k) acc[k] = comp_merge(acc[k], part[((size_t)s * L.q.n + iq) * 3 + k]);
  const double q = L.q.q[iq], qm1 = q - 1.0;
  const double sj = acc[0].s + acc[0].c, sf = acc[1].s + acc[1].c, sm = acc[2].s + acc[2].c;
  double I;
  if (q == 1.0) {
    I = (sj - sf) - sm;
  } else {
    const double Sj = -sj / qm1, Sf = -sf / qm1, Sm = -sm / qm1;
    I = (Sf + Sm) - Sj;
    if (L.q.pseudo) I += (1.0 - q) * Sf * Sm;
  }
  L.mi_out[(size_t)t * L.q.n + iq] = I;
}

template <bool TABLE>
static void partial_variant(const ReduceLaunch& L, unsigned blocks, bool cached, hipStream_t s) {
  if (cached)
    hipLaunchKernelGGL((mi_partial_kernel<TABLE, true>), dim3(blocks), dim3(kBlock), 0, s, L);
  else
    hipLaunchKernelGGL((mi_partial_kernel<TABLE, false>), dim3(blocks), dim3(kBlock), 0, s, L);
}

hipError_t launch_mi_reduce(const ReduceLaunch& Lin, hipStream_t s) {
  if (Lin.n == 0) return hipSuccess;
  ReduceLaunch L = Lin;
  L.splits = reduce_splits(L.bins, L.n);
  hipError_t e;
  const int S = L.splits;
  const int max_rows = (L.bins + S - 1) / S;
  const bool cached = max_rows * (L.bins + 2) <= kMaxSliceCells;  // cells + 2 marginals per row
  if (!L.table && (e = launch_fill_u32((uint32_t*)L.count, 2 * (size_t)L.n, 0u, s)) != hipSuccess) return e;
  // launches of whole transforms, each below 2^31 work-items; the slice
  // count stays that of the whole batch
  const size_t BB = (size_t)L.bins * L.bins;
  const int32_t step = transforms_per_launch(S, kBlock);
  for (int32_t t0 = 0; t0 < L.n; t0 += step) {
    ReduceLaunch P = L;
    P.n = L.n - t0 < step ? L.n - t0 : step;
    if (L.hist) P.hist = L.hist + (size_t)t0 * BB;
    if (L.table) P.table = L.table + (size_t)t0 * BB;
    P.count = L.count + t0;
    P.part = L.part + (size_t)t0 * S * L.q.n * 3 * 2;  // (sum, error) pairs
    P.transforms = L.transforms + 12 * (size_t)t0;
    if (L.marg_out) P.marg_out = L.marg_out + (size_t)t0 * 2 * L.bins;
    P.mi_out = L.mi_out + (size_t)t0 * L.q.n;
    if (L.overlap_out) P.overlap_out = L.overlap_out + t0;
    const unsigned blocks = (unsigned)((int64_t)P.n * S);
    if (!P.table) {
      hipLaunchKernelGGL(hist_count_kernel, dim3(blocks), dim3(kBlock), 0, s, P.hist, P.bins, S, P.count);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      partial_variant<false>(P, blocks, cached, s);
    } else {
      partial_variant<true>(P, blocks, cached, s);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mi_final_kernel, dim3((unsigned)P.n), dim3(64), 0, s, P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace gemi
