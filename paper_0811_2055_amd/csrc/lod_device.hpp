// Device-side building blocks for the gfx950 level-of-detail path.
// Wave64 throughout: ballots are 64-bit, lane masks are 64-bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lod.h"

namespace lodk {

constexpr int WAVE = 64;
constexpr uint32_t NONE = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0..c3), key
// (k0,k1); a round maps (c0,c1,c2,c3) to (hi(M1 c2)^c1^k0, lo(M1 c2),
// hi(M0 c0)^c3^k1, lo(M0 c0)); the key is bumped by the Weyl constants
// between rounds.  Only output word 0 is used by the method.
__device__ __forceinline__ uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    // one 32 x 32 -> 64-bit multiply gives both halves of each product
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
  }
  return c0;
}

// U = word0 + 1 in [1, 2^32] for particle `id` of snapshot `snap`.
__device__ __forceinline__ uint64_t particle_U(uint64_t id, uint32_t snap, uint64_t seed) {
  return (uint64_t)philox_word0((uint32_t)id, (uint32_t)(id >> 32), snap, 0u,
                                (uint32_t)seed, (uint32_t)(seed >> 32)) + 1ull;
}

// floor(U 2^31 / w) for U <= 2^32, 1 <= w < 2^31, without a 64-bit divide:
// 2^31 = a w + b, so the quotient is U a + floor(U b / w).  Both quotients
// come from one float64 reciprocal of w (relative error 2^-53 before the
// products): a is off by at most one and corrected both ways, U b / w < 2^32
// is off by far less than one unit and its remainder corrects it.
__device__ __forceinline__ uint64_t div_u2p31(uint64_t U, uint32_t w) {
  const double rw = 1.0 / (double)w;
  uint32_t a = (uint32_t)(2147483648.0 * rw);
  if ((uint64_t)a * w > 2147483648ull) --a;
  if ((uint64_t)(a + 1) * w <= 2147483648ull) ++a;
  const uint32_t b = (uint32_t)(2147483648ull - (uint64_t)a * w);
  const uint64_t x = U * (uint64_t)b;
  uint64_t q = (uint64_t)((double)x * rw);
  int64_t r = (int64_t)(x - q * (uint64_t)w);
  while (r < 0) { --q; r += w; }
  while (r >= (int64_t)w) { ++q; r -= w; }
  return U * (uint64_t)a + q;
}

// Integer selection key; smaller is kept first.
__device__ __forceinline__ uint64_t selection_key(uint64_t U, uint32_t w, int alpha) {
  if (alpha > 0) return div_u2p31(U, w);
  if (alpha == 0) return U << 31;
  return U * (uint64_t)w;
}

// Monotone 12-bit log-scale bin of a 64-bit key: K < 128 maps to itself,
// larger keys to 128 + 64 (e - 7) + the 6 bits after the leading one (e =
// index of the leading one).  K1 < K2 implies kbin(K1) <= kbin(K2).
__device__ __forceinline__ uint32_t kbin(uint64_t K) {
  if (K < 128) return (uint32_t)K;
  const int e = 63 - __clzll(K);
  return 128u + (uint32_t)(e - 7) * 64u + (uint32_t)((K >> (e - 6)) & 63u);
}

// kbin(floor(U 2^31 / w)) without the 64-bit quotient, when float64 decides
// it.  The bin edges are integers, so the quotient lies in the bin of the
// real x = U 2^31 / w.  In float64, x is found to within a relative 2^-50:
// U is exact, 1/w comes from the hardware reciprocal refined by three Newton
// steps (each squares the relative error and adds rounding: any start below
// 2^-8 ends near 2^-52), and the product is rounded once.  Its bin is that of x unless x
// lies within 64 float64 steps (2^-46 relative) of an edge (the 46 bits below
// the bin bits are nearly all zeros or all ones) or below 256.  Returns false
// in those (rare) cases: then the exact quotient decides.
__device__ __forceinline__ bool kbin_div_fast(uint64_t U, uint32_t w, uint32_t &bin) {
  const double wd = (double)w;
  double r = __builtin_amdgcn_rcp(wd);
  r = __builtin_fma(r, __builtin_fma(-wd, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-wd, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-wd, r, 1.0), r);
  const double x = ((double)(uint32_t)(U - 1ull) + 1.0) * r * 2147483648.0;
  const uint64_t bits = (uint64_t)__double_as_longlong(x);
  const int E = (int)(bits >> 52) - 1023;
  const uint64_t rest = bits & ((1ull << 46) - 1ull);
  bin = 128u + (uint32_t)(E - 7) * 64u + (uint32_t)((bits >> 46) & 63u);
  return E >= 8 && rest > 64ull && rest < (1ull << 46) - 64ull;
}

// w^alpha as float64 (alpha in {-1,0,1}).
__device__ __forceinline__ double weight_pow(uint32_t w, int alpha) {
  if (alpha > 0) return (double)w;
  if (alpha == 0) return 1.0;
  return 1.0 / (double)w;
}

// ---------------------------------------------------------------------------
// Workgroups go to the eight XCDs round-robin (block b to XCD b mod 8), and
// each XCD has its own L2.  Giving XCD x the x-th contiguous share of n work
// items (sort tiles) puts neighbouring items, whose outputs end and begin in
// the same cache lines, on one L2.  A bijection of [0, n).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t x = b & 7u, i = b >> 3;
  const uint32_t per = n >> 3, extra = n & 7u;   // XCD x takes per + (x < extra) items
  return x * per + min(x, extra) + i;
}

// ---------------------------------------------------------------------------
// Morton: spread the low 10 bits of v to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x3FFu;
  return v;
}

// Fixed point X = min(floor(a 2^(D+16)), 2^(D+16)-1) for a in [0,1]; the
// product is exact (power-of-two scaling) and floor of a float is a float.
// Returns false for NaN or a outside [0,1].
__device__ __forceinline__ bool fixed_coord(float a, int D, uint32_t &X) {
  if (!(a >= 0.0f && a <= 1.0f)) { X = 0; return false; }
  const float s = ldexpf(a, D + 16);
  uint32_t v = (uint32_t)floorf(s);
  const uint32_t top = (1u << (D + 16)) - 1u;
  X = v > top ? top : v;
  return true;
}

// q at depth d <= D from the depth-D cell coordinate and the 16 low bits.
__device__ __forceinline__ uint16_t quant_at(uint32_t cD, uint32_t lo16, int D, int d) {
  const uint32_t X = (cD << 16) | lo16;
  return (uint16_t)((X >> (D - d)) & 0xFFFFu);
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one value per thread (LDS, any blockDim that
// is a multiple of 64 and <= 1024).  `tmp` holds >= blockDim/64 + 1 entries.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T t = __shfl_up(v, o, WAVE);
    if (lane >= o) v += t;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *tmp, T &total) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
  T inc = wave_incl_scan(v);
  if (lane == WAVE - 1) tmp[wid] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int w = 0; w < nw; ++w) { T t = tmp[w]; tmp[w] = run; run += t; }
    tmp[nw] = run;
  }
  __syncthreads();
  T res = tmp[wid] + inc - v;
  total = tmp[nw];
  __syncthreads();
  return res;
}

template <typename T>
__device__ __forceinline__ T block_reduce_sum(T v, T *tmp) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  if (lane == 0) tmp[wid] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < nw; ++w) r += tmp[w];
    tmp[nw] = r;
  }
  __syncthreads();
  r = tmp[nw];
  __syncthreads();
  return r;
}

// lower_bound over a sorted uint32 array in [lo, hi) for the first element >= key.
__device__ __forceinline__ uint64_t lower_bound_u32(const uint32_t *a, uint64_t lo, uint64_t hi,
                                                    uint32_t key) {
  while (lo < hi) {
    uint64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace lodk
