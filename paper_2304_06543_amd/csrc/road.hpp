// road.hpp -- host launchers of the road-network cost-matrix construction
// (road.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbdd {

// centers searched per launch: the work buffer holds this many label arrays
constexpr int32_t ROAD_CHUNK = 256;

size_t road_work_bytes(int32_t V, int32_t k);
int road_cost_matrix(int32_t V, const int64_t *row_ptr, const int32_t *col, const int32_t *len, int32_t k,
                     const int32_t *centers, int64_t n, const int32_t *units, int32_t *cm, void *work,
                     hipStream_t st);

}  // namespace lbdd
