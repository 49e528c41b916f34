// Block-to-work mapping for a chip made of several accelerator dies (XCDs),
// each with its own L2: the dispatcher hands consecutive workgroups of a
// launch to the XCDs in turn.  xcd_order() turns the linear block index into
// a work index such that each XCD receives one contiguous 1/kXcds of the
// work range, so work items that share input lines (neighbouring tiles, one
// energy's image, one view group's rays) share an L2.  It is a permutation
// of [0, n) for any n: the first kXcds * floor(n / kXcds) blocks are grouped,
// the last n mod kXcds keep their index.
#pragma once

#include <hip/hip_runtime.h>

namespace dect {

constexpr unsigned kXcds = 8;

__device__ __forceinline__ unsigned xcd_order(unsigned linear, unsigned n)
{
    const unsigned q = n / kXcds;
    if (linear >= q * kXcds) return linear;
    return (linear % kXcds) * q + linear / kXcds;
}

// Linear index of this block in a 3-D grid (x fastest) and the grid's size.
__device__ __forceinline__ unsigned block_linear()
{
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ __forceinline__ unsigned grid_blocks() { return gridDim.x * gridDim.y * gridDim.z; }

}  // namespace dect
