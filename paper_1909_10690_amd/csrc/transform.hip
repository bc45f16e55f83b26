// Transform setup of every call (Fig. 1 Transform block): the caller's
// physical fixed -> moving matrices (mm) become index-space matrices, fixed
// voxel index -> continuous moving index, before any sweep; and the
// gradient with respect to the index-space entries, which the backward
// sweep accumulates, becomes the gradient with respect to the caller's
// physical entries.
#include "common.h"

namespace gemi {

__global__ void compose_kernel(const double* __restrict__ P, int64_t n, Geometry g, double* __restrict__ M) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double m[12];
    compose_index_matrix(P + 12 * t, g, m);
#pragma unroll
    for (int e = 0; e < 12; ++e) M[12 * t + e] = m[e];
  }
}

// With y_r = (sum_c P[r][c] x_c + P[r][3] - morg[r]) / msp[r] and the fixed
// voxel's position x_c = forg[c] + fsp[c] i_c, the moving index depends on
// P[r][c] through M[r][c] = P[r][c] fsp[c] / msp[r] and
// M[r][3] = (... + P[r][c] forg[c] ...) / msp[r]:
//   dMI/dP[r][c] = (dMI/dM[r][c] fsp[c] + dMI/dM[r][3] forg[c]) / msp[r],
//   dMI/dP[r][3] = dMI/dM[r][3] / msp[r].
__global__ void grad_physical_kernel(double* __restrict__ G, int64_t rows, Geometry g) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < rows;
       k += (int64_t)gridDim.x * blockDim.x) {
    double* row = G + 12 * k;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double gt = row[4 * r + 3];
#pragma unroll
      for (int c = 0; c < 3; ++c) row[4 * r + c] = (row[4 * r + c] * g.fsp[c] + gt * g.forg[c]) / g.msp[r];
      row[4 * r + 3] = gt / g.msp[r];
    }
  }
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_compose(const double* P, int64_t n, const Geometry& g, double* M, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(compose_kernel, dim3(grid_for(n)), dim3(256), 0, s, P, n, g, M);
  return hipGetLastError();
}

hipError_t launch_grad_physical(double* grad, int64_t rows, const Geometry& g, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(grad_physical_kernel, dim3(grid_for(rows)), dim3(256), 0, s, grad, rows, g);
  return hipGetLastError();
}

}  // namespace gemi
