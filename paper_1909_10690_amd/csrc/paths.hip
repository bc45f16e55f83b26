// Discrete gradient paths on a parameter-space map of the metric.
//
// Results: the metric of one transform family (translation, rotation or
// scale) is mapped over a 3D grid of its parameters, and the paths a
// gradient method follows on that map show which starting points reach the
// known optimum; Discussion: that capture range is what separates the
// entropies.  On the grid a path steps from a point to the 26-connected
// neighbour of steepest rise of sign * f,
//   slope = (sign f(q) - sign f(p)) * w,  w = 1, 1/sqrt 2 or 1/sqrt 3
// (the reciprocal of the step length, as the nearest fp64 value), and stops
// at a point no neighbour rises from (a local extremum).  Ties keep the
// first neighbour in (dz, dy, dx) order, each running -1, 0, 1.  NaN points
// are extrema and never entered.  Every point's successor rises strictly, so
// no path revisits a point and each ends within n steps.
#include "paths.h"

#include <stdint.h>

namespace gemi {

namespace {
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt3 = 0.57735026918962576451;
constexpr int kPathThreads = 256;

unsigned path_grid(int64_t n) {
  const int64_t g = (n + kPathThreads - 1) / kPathThreads;
  return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}
}  // namespace

__global__ __launch_bounds__(kPathThreads) void path_next_kernel(const double* __restrict__ f, int32_t nx,
                                                                 int32_t ny, int32_t nz, double sign,
                                                                 int32_t* __restrict__ next) {
  const int64_t n = (int64_t)nx * ny * nz;
  for (int64_t p = blockIdx.x * (int64_t)kPathThreads + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * kPathThreads) {
    const int32_t x = (int32_t)(p % nx);
    const int64_t r = p / nx;
    const int32_t y = (int32_t)(r % ny), z = (int32_t)(r / ny);
    const double fp = sign * f[p];
    double best = 0.0;
    int64_t arg = p;
    for (int dz = -1; dz <= 1; ++dz) {
      const int32_t zz = z + dz;
      if (zz < 0 || zz >= nz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int32_t yy = y + dy;
        if (yy < 0 || yy >= ny) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int32_t xx = x + dx;
          const int k = (dx != 0) + (dy != 0) + (dz != 0);
          if (xx < 0 || xx >= nx || k == 0) continue;
          const int64_t q = ((int64_t)zz * ny + yy) * nx + xx;
          const double w = k == 1 ? 1.0 : (k == 2 ? kInvSqrt2 : kInvSqrt3);
          const double s = (sign * f[q] - fp) * w;
          if (s > best) {
            best = s;
            arg = q;
          }
        }
      }
    }
    next[p] = (int32_t)arg;
  }
}

// Follows each point's successors to the extremum its path ends at.  The
// step bound n is never reached by a strictly rising path; it only makes
// the loop's end independent of the data.
__global__ __launch_bounds__(kPathThreads) void path_sink_kernel(const int32_t* __restrict__ next, int64_t n,
                                                                 int32_t* __restrict__ sink) {
  for (int64_t p = blockIdx.x * (int64_t)kPathThreads + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * kPathThreads) {
    int32_t q = (int32_t)p;
    for (int64_t step = 0; step < n; ++step) {
      const int32_t r = next[q];
      if (r == q) break;
      q = r;
    }
    sink[p] = q;
  }
}

// stats: [0] extrema, [1] sink of the centre, [2] points ending there,
// [3] (while counting) smallest Chebyshev distance from the centre of a
// point ending elsewhere.
__global__ void path_stats_init_kernel(int64_t* stats) {
  if (threadIdx.x == 0) {
    stats[0] = 0;
    stats[1] = 0;
    stats[2] = 0;
    stats[3] = INT64_MAX;
  }
}

__global__ __launch_bounds__(kPathThreads) void path_stats_kernel(const int32_t* __restrict__ next,
                                                                  const int32_t* __restrict__ sink,
                                                                  int32_t nx, int32_t ny, int32_t nz,
                                                                  int32_t cx, int32_t cy, int32_t cz,
                                                                  int64_t* __restrict__ stats) {
  const int64_t n = (int64_t)nx * ny * nz;
  const int32_t target = sink[((int64_t)cz * ny + cy) * nx + cx];
  uint64_t extrema = 0, basin = 0;
  int64_t dmin = INT64_MAX;
  for (int64_t p = blockIdx.x * (int64_t)kPathThreads + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * kPathThreads) {
    extrema += next[p] == (int32_t)p;
    if (sink[p] == target) {
      ++basin;
    } else {
      const int32_t x = (int32_t)(p % nx);
      const int64_t r = p / nx;
      const int32_t y = (int32_t)(r % ny), z = (int32_t)(r / ny);
      const int64_t d = max(abs(x - cx), max(abs(y - cy), abs(z - cz)));
      dmin = d < dmin ? d : dmin;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    extrema += __shfl_xor(extrema, off, 64);
    basin += __shfl_xor(basin, off, 64);
    const int64_t o = __shfl_xor(dmin, off, 64);
    dmin = o < dmin ? o : dmin;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd((unsigned long long*)&stats[0], (unsigned long long)extrema);
    atomicAdd((unsigned long long*)&stats[2], (unsigned long long)basin);
    atomicMin((unsigned long long*)&stats[3], (unsigned long long)dmin);
  }
}

// Capture radius: one less than the nearest point that ends elsewhere, or,
// when every point ends at the centre's extremum, the grid's largest
// Chebyshev distance from the centre.
__global__ void path_stats_final_kernel(const int32_t* __restrict__ sink, int32_t nx, int32_t ny, int32_t nz,
                                        int32_t cx, int32_t cy, int32_t cz, int64_t* stats) {
  if (threadIdx.x != 0) return;
  stats[1] = sink[((int64_t)cz * ny + cy) * nx + cx];
  if (stats[3] == INT64_MAX) {
    const int32_t ex = max(cx, nx - 1 - cx), ey = max(cy, ny - 1 - cy), ez = max(cz, nz - 1 - cz);
    stats[3] = max(ex, max(ey, ez));
  } else {
    stats[3] -= 1;
  }
}

hipError_t launch_map_paths(const PathsLaunch& L, hipStream_t s) {
  const int64_t n = (int64_t)L.nx * L.ny * L.nz;
  const unsigned g = path_grid(n);
  hipLaunchKernelGGL(path_next_kernel, dim3(g), dim3(kPathThreads), 0, s, L.values, L.nx, L.ny, L.nz,
                     L.sign, L.next);
  hipLaunchKernelGGL(path_sink_kernel, dim3(g), dim3(kPathThreads), 0, s, L.next, n, L.sink);
  hipLaunchKernelGGL(path_stats_init_kernel, dim3(1), dim3(64), 0, s, L.stats);
  hipLaunchKernelGGL(path_stats_kernel, dim3(g), dim3(kPathThreads), 0, s, L.next, L.sink, L.nx, L.ny, L.nz,
                     L.cx, L.cy, L.cz, L.stats);
  hipLaunchKernelGGL(path_stats_final_kernel, dim3(1), dim3(64), 0, s, L.sink, L.nx, L.ny, L.nz, L.cx, L.cy,
                     L.cz, L.stats);
  return hipGetLastError();
}

}  // namespace gemi
