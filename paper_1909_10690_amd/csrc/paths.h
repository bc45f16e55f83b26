// Launch description of the discrete gradient paths on a 3D parameter map
// (paths.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gemi {

struct PathsLaunch {
  const double* values;  // [nz][ny][nx]
  int32_t nx, ny, nz;
  double sign;           // +1 climb, -1 descend
  int32_t cx, cy, cz;    // centre of the map
  int32_t* next;         // [n]
  int32_t* sink;         // [n]
  int64_t* stats;        // [4]
};

hipError_t launch_map_paths(const PathsLaunch& L, hipStream_t s);

}  // namespace gemi
