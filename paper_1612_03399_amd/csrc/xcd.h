// xcd.h -- block numbering for one-block-per-tile launches over element or
// marker arrays.  Workgroups are dealt to the eight XCDs in turn (workgroup i
// to XCD i mod 8), each XCD with its own L2.  xcd_block() gives XCD x one
// contiguous range of the n logical blocks (its k-th workgroup takes block
// start_x + k), so consecutive blocks, whose elements share nodes and grid
// points, are fetched into one L2 rather than into all eight.  A bijection of
// 0 .. n - 1 whatever the hardware's order.  (The work-unit kernels deal
// their units in chunks instead, xcd_unit in step_common.h.)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

__device__ __forceinline__ int64_t xcd_block() {
    const int64_t n = gridDim.x, i = blockIdx.x;
    const int64_t q = n / 8, r = n % 8, x = i % 8, k = i / 8;
    return x * q + (x < r ? x : r) + k;
}
