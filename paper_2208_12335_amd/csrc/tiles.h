// Work distribution of the tiled MFMA kernels (shared by every kernel file that uses it).
#pragma once

#include <hip/hip_runtime.h>

namespace aims {

// XCD-aware work order: the dispatcher places workgroup g on XCD g % 8, so consecutive work
// items (tiles of the same batch, which share its slab) are given workgroup ids that differ by
// multiples of 8 and stay in one XCD's L2.
__device__ __forceinline__ int xcd_item(int g, int n) {
  const int per = (n + 7) / 8;
  return (g & 7) * per + (g >> 3);
}

// The same order as a bijection of [0, n) for a grid of exactly n workgroups: XCD x takes the
// contiguous run of n / 8 (+1 for the first n % 8 XCDs) items that starts at x (n / 8) + min(x, n % 8).
__device__ __forceinline__ int xcd_item_exact(int g, int n) {
  const int x = g & 7, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + (g >> 3);
}


// Work distribution.  Grid mode (queue == NULL): one workgroup per item, XCD-aware order.
// Persistent mode: a fixed grid of workgroups drains eight per-XCD queues of contiguous
// (spatially ordered) items; workgroup g starts on queue g % 8 -- the queue of its own XCD -- and
// steals from the other queues once that is empty.  queue[8] must be zero at launch.
template <typename F>
__device__ __forceinline__ void run_items(int n_items, int* __restrict__ queue, F&& tile) {
  if (!queue) {
    const int item = xcd_item(blockIdx.x, n_items);
    if (item < n_items) tile(item);
    return;
  }
  __shared__ int s_next;
  const int per = (n_items + 7) / 8;
  const int x0 = blockIdx.x & 7;
  for (int q = 0; q < 8;) {
    const int x = (x0 + q) & 7;
    if (threadIdx.x == 0) s_next = atomicAdd(queue + x, 1);
    __syncthreads();
    const int k = s_next;
    __syncthreads();
    const int item = x * per + k;
    if (k >= per || item >= n_items) {
      ++q;
      continue;
    }
    tile(item);
    __syncthreads();
  }
}

}  // namespace aims
