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

// VEC: data is 16-byte aligned, and the blocks whose tile lies inside [0, n)
// move a thread's SCAN_ITEMS values with 16-byte loads and stores (one
// instruction per 16 bytes instead of one per value).
template <typename T, bool VEC>
__global__ __launch_bounds__(SCAN_TB) void k_scan_block(T *data, uint64_t n, T *sums) {
  static_assert((SCAN_ITEMS * sizeof(T)) % 16 == 0, "whole 16-byte words per thread");
  constexpr int NV = (int)(SCAN_ITEMS * sizeof(T) / 16);
  __shared__ T tmp[SCAN_TB / lodk::WAVE + 1];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  const bool whole = VEC && (uint64_t)(blockIdx.x + 1) * SCAN_TILE <= n;
  union Items {
    T v[SCAN_ITEMS];
    uint4 q[NV];
  } it;
  if (whole) {
    const uint4 *src = reinterpret_cast<const uint4 *>(data + base);
#pragma unroll
    for (int j = 0; j < NV; ++j) it.q[j] = src[j];
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      const uint64_t e = base + i;
      it.v[i] = e < n ? data[e] : (T)0;
    }
  }
  T run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) run += it.v[i];
  T total;
  T off = lodk::block_excl_scan<T>(run, tmp, total);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const T x = it.v[i];
    it.v[i] = off;
    off += x;
  }
  if (whole) {
    uint4 *dst = reinterpret_cast<uint4 *>(data + base);
#pragma unroll
    for (int j = 0; j < NV; ++j) dst[j] = it.q[j];
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      const uint64_t e = base + i;
      if (e < n) data[e] = it.v[i];
    }
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
    LOD_LAUNCH((k_scan_block<T, false>), dim3(1), dim3(SCAN_TB), 0, s, data, n, (T *)nullptr);
    return;
  }
  T *sums = tmp;
  if (reinterpret_cast<uintptr_t>(data) % 16 == 0)
    LOD_LAUNCH((k_scan_block<T, true>), dim3((unsigned)nb), dim3(SCAN_TB), 0, s, data, n, sums);
  else
    LOD_LAUNCH((k_scan_block<T, false>), dim3((unsigned)nb), dim3(SCAN_TB), 0, s, data, n, sums);
  device_scan<T>(sums, nb, tmp + nb, s);
  LOD_LAUNCH(k_scan_add<T>, dim3((unsigned)nb), dim3(SCAN_TB), 0, s, data, n, (const T *)sums);
}

// The scan without its add pass: data[0..n) gets each 4096-element block's
// own exclusive scan and tmp[0..nb) the exclusive scan of the block totals, so
// the scan of element i is data[i] + tmp[i / SCAN_TILE] (a consumer that
// reads each element once adds the two itself).  tmp holds
// scan_tmp_elems<T>(n) elements, as for device_scan.
template <typename T>
void device_scan_blocks(T *data, uint64_t n, T *tmp, hipStream_t s) {
  if (n == 0) return;
  const uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (reinterpret_cast<uintptr_t>(data) % 16 == 0)
    LOD_LAUNCH((k_scan_block<T, true>), dim3((unsigned)nb), dim3(SCAN_TB), 0, s, data, n, tmp);
  else
    LOD_LAUNCH((k_scan_block<T, false>), dim3((unsigned)nb), dim3(SCAN_TB), 0, s, data, n, tmp);
  device_scan<T>(tmp, nb, tmp + nb, s);
}

}  // namespace
