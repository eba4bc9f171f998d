// Device-wide exclusive scan (reduce-then-scan over 4096-element blocks,
// recursive over the block sums).  Included by each translation unit that
// needs it; everything lives in an unnamed namespace.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lod_device.hpp"
#include "lod_trace.hpp"

namespace {

constexpr int SCAN_TB = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_TB * SCAN_ITEMS;

template <typename T>
__global__ __launch_bounds__(SCAN_TB) void k_scan_block(T *data, uint64_t n, T *sums) {
  __shared__ T tmp[SCAN_TB / lodk::WAVE + 1];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const uint64_t e = base + i;
    v[i] = e < n ? data[e] : (T)0;
    run += v[i];
  }
  T total;
  T off = lodk::block_excl_scan<T>(run, tmp, total);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const uint64_t e = base + i;
    if (e < n) data[e] = off;
    off += v[i];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(SCAN_TB) void k_scan_add(T *data, uint64_t n, const T *sums) {
  const T add = sums[blockIdx.x];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
  for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_TB) {
    const uint64_t e = base + i;
    if (e < n) data[e] += add;
  }
}

// Elements of scratch the scan of n values needs.
template <typename T>
size_t scan_tmp_elems(uint64_t n) {
  size_t tot = 0;
  while (n > (uint64_t)SCAN_TILE) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    tot += n;
  }
  return tot + 1;
}

// Exclusive scan of data[0..n) in place; tmp holds scan_tmp_elems<T>(n).
template <typename T>
void device_scan(T *data, uint64_t n, T *tmp, hipStream_t s) {
  if (n == 0) return;
  const uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    LOD_LAUNCH(k_scan_block<T>, dim3(1), dim3(SCAN_TB), 0, s, data, n, (T *)nullptr);
    return;
  }
  T *sums = tmp;
  LOD_LAUNCH(k_scan_block<T>, dim3((unsigned)nb), dim3(SCAN_TB), 0, s, data, n, sums);
  device_scan<T>(sums, nb, tmp + nb, s);
  LOD_LAUNCH(k_scan_add<T>, dim3((unsigned)nb), dim3(SCAN_TB), 0, s, data, n, (const T *)sums);
}

}  // namespace
