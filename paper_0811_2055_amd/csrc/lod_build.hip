// Octree level-of-detail build for gfx950 (octree and quantisation
// paragraphs of arXiv:0811.2055; readings fixed in the oracle's docstrings).
//
// Data path (all device-resident, one stream, no host synchronisation):
//   keygen     domain check and digit-0 tile histograms of the sort key
//              (snapshot | 3D-bit Morton); the first scatter pass recomputes
//              the key and the 48-bit fraction from x, y, z
//   radix sort stable LSD, 8-bit digits, reduce-then-scan: per-tile digit
//              histograms, one device scan, scatter with wave-ballot ranks and
//              LDS-staged coalesced writes; payload (id, fraction, mass) rides
//              along so nothing is gathered at random afterwards
//   density    run lengths of equal depth-L cells (block max/min scans), then
//              Philox U and the 12-bit bin of the integer selection key K per
//              sorted position (on a second stream, beside the tree)
//   tree       level by level: octant boundaries by binary search, then the
//              next level emitted with one thread per (node, octant): counts,
//              one scan, writes
//   leaves     float64 leaf masses; the per-level schedule copies the leaves'
//              particles inside its selection launches
//   selection  bottom up, per node holding > n: the node's float64 mass from
//              its children, the (n+1)-th smallest (K, id) over the children's
//              top lists or own range (key-bin histogram, exact keys only in
//              the threshold bin), then an order-preserving compaction;
//              float64 renormalisation, 16-bit quantisation and output
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "lod.h"
#include "lod_device.hpp"
#include "lod_internal.hpp"
#include "lod_scan.hpp"

using namespace lodk;

namespace {

constexpr int TB = 256;          // threads per block for streaming kernels
constexpr int ITEMS = 16;        // elements per thread
constexpr int TILE = TB * ITEMS; // elements per density tile (4096)

// radix sort tiles: scatter blocks of STB threads x SITEMS elements; the
// histogram kernels (TB threads) cover the same STILE elements per block.
// 512-thread scatter blocks take 43 KB of LDS, so two run on a CU and one's
// ranking overlaps the other's stores (1024 threads and 84 KB: one block per
// CU, 2.5% slower build).
constexpr int STB = 512;                     // scatter threads per block
constexpr int SITEMS = 8;                    // elements per scatter thread
constexpr int STILE = STB * SITEMS;          // elements per sort tile
constexpr int HITEMS = STILE / TB;           // elements per histogram thread
constexpr int HCHUNK = 8;                    // loads issued together in keygen (twice that in upsweep)
static_assert(HITEMS % (2 * HCHUNK) == 0, "histogram chunks must divide the tile");
constexpr int RADIX = 256;
constexpr uint32_t STATUS_INTERNAL = 8u;

// ---------------------------------------------------------------------------
// parameters passed by value to kernels

struct BuildArgs {
  uint64_t N;
  uint32_t n;
  int D;
  int shift_rho;       // 3 (D - L)
  int alpha;
  uint64_t seed;
  uint32_t n_snap;
  const uint64_t *snap_off;   // device [n_snap+1] or null
  uint64_t node_cap, point_cap;
  uint64_t *counts;           // device [3]
};

__device__ __forceinline__ uint32_t snapshot_of(const BuildArgs &a, uint64_t e) {
  if (a.n_snap <= 1 || !a.snap_off) return 0;
  // largest s with snap_off[s] <= e
  uint32_t lo = 0, hi = a.n_snap;   // answer in [0, n_snap)
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (a.snap_off[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t local_id(const BuildArgs &a, uint32_t snap, uint32_t gidx) {
  return (a.n_snap <= 1 || !a.snap_off) ? (uint64_t)gidx : (uint64_t)gidx - a.snap_off[snap];
}

// ---------------------------------------------------------------------------
// snapshot offsets check (one block)

__global__ void k_check_offsets(BuildArgs a) {
  if (!a.snap_off || a.n_snap <= 1) return;
  bool bad = false;
  for (uint32_t s = threadIdx.x; s < a.n_snap; s += blockDim.x) {
    uint64_t lo = a.snap_off[s], hi = a.snap_off[s + 1];
    if (hi < lo || hi - lo >= (1ull << 31)) bad = true;
  }
  if (threadIdx.x == 0 && (a.snap_off[0] != 0 || a.snap_off[a.n_snap] != a.N)) bad = true;
  if (bad) atomicOr((unsigned long long *)&a.counts[2], (unsigned long long)LOD_STATUS_OFFSETS);
}

// ---------------------------------------------------------------------------
// sort key and 48-bit fraction of particle e.  Both the keygen histogram and
// the first scatter pass call this, so their digits agree bit for bit (NaN and
// out-of-range coordinates map to 0 and are reported by keygen's check).

struct PKey {
  uint32_t key;
  uint64_t lo;
  bool ok;
};

__device__ __forceinline__ PKey particle_key(const BuildArgs &a, float xe, float ye, float ze, float me,
                                             uint64_t e) {
  uint32_t X, Y, Z;
  bool ok = fixed_coord(xe, a.D, X);
  ok &= fixed_coord(ye, a.D, Y);
  ok &= fixed_coord(ze, a.D, Z);
  ok &= (me >= 0.0f) && (me <= 3.4028235e38f);
  const uint32_t cmask = (1u << a.D) - 1u;
  const uint32_t cx = (X >> 16) & cmask, cy = (Y >> 16) & cmask, cz = (Z >> 16) & cmask;
  uint32_t k = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
  if (a.n_snap > 1) k |= (uint32_t)(((uint64_t)snapshot_of(a, e) << (3 * a.D)) & 0xFFFFFFFFull);
  const uint64_t lo = (uint64_t)(X & 0xFFFFu) | ((uint64_t)(Y & 0xFFFFu) << 16) | ((uint64_t)(Z & 0xFFFFu) << 32);
  return PKey{k, lo, ok};
}

// keygen: domain check and digit-0 tile histograms (reads the input only; the
// first scatter pass recomputes the keys instead of reading them back)
__global__ __launch_bounds__(TB) void k_keygen(const float *__restrict__ x, const float *__restrict__ y,
                                               const float *__restrict__ z, BuildArgs a, uint32_t *__restrict__ thist,
                                               uint64_t n_tiles) {
  __shared__ uint32_t hist[RADIX];
  __shared__ int bad;
  for (int i = threadIdx.x; i < RADIX; i += TB) hist[i] = 0;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  bool my_bad = false;
  // all loads first (clamped indices: a predicated load is waited for alone)
  for (int c = 0; c < HITEMS; c += HCHUNK) {
    float xs[HCHUNK], ys[HCHUNK], zs[HCHUNK];
#pragma unroll
    for (int i = 0; i < HCHUNK; ++i) {
      const uint64_t e = min(tile * STILE + (uint64_t)(c + i) * TB + threadIdx.x, a.N - 1);
      xs[i] = x[e]; ys[i] = y[e]; zs[i] = z[e];
    }
#pragma unroll
    for (int i = 0; i < HCHUNK; ++i) {
      const uint64_t e = tile * STILE + (uint64_t)(c + i) * TB + threadIdx.x;
      if (e < a.N) {
        // positions only: the masses are checked by the first scatter pass
        const PKey pk = particle_key(a, xs[i], ys[i], zs[i], 0.0f, e);
        my_bad |= !pk.ok;
        atomicAdd(&hist[pk.key & 0xFFu], 1u);
      }
    }
  }
  if (my_bad) bad = 1;
  __syncthreads();
  for (int i = threadIdx.x; i < RADIX; i += TB) thist[(uint64_t)i * n_tiles + tile] = hist[i];
  if (threadIdx.x == 0 && bad)
    atomicOr((unsigned long long *)&a.counts[2], (unsigned long long)LOD_STATUS_DOMAIN);
}

// per-tile digit histogram for passes after the first
__global__ __launch_bounds__(TB) void k_upsweep(const uint32_t *__restrict__ key, uint64_t N, int shift,
                                                uint32_t *__restrict__ thist, uint64_t n_tiles) {
  __shared__ uint32_t hist[RADIX];
  for (int i = threadIdx.x; i < RADIX; i += TB) hist[i] = 0;
  __syncthreads();
  const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  for (int c = 0; c < HITEMS; c += 2 * HCHUNK) {
    uint32_t ks[2 * HCHUNK];
#pragma unroll
    for (int i = 0; i < 2 * HCHUNK; ++i)
      ks[i] = key[min(tile * STILE + (uint64_t)(c + i) * TB + threadIdx.x, N - 1)];
#pragma unroll
    for (int i = 0; i < 2 * HCHUNK; ++i)
      if (tile * STILE + (uint64_t)(c + i) * TB + threadIdx.x < N) atomicAdd(&hist[(ks[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < RADIX; i += TB) thist[(uint64_t)i * n_tiles + tile] = hist[i];
}

// Stable scatter of one LSD pass over STILE-element tiles, STB threads.  Wave
// w of the block owns tile elements [w*P, (w+1)*P) with P = STILE / waves; in
// round r lane l holds element w*P + r*64 + l, so element order is (w, r, l).
// All loads of a thread's SITEMS elements are issued first, so their latency
// overlaps the ranking.
// Ranks within a wave come from 8 ballots (the lanes sharing the digit) and a
// wave-private LDS counter per digit; the tile is staged in LDS in digit order
// so that the global writes of each digit run are contiguous.

// FIRST: the input is the particles themselves (x, y, z, m with ids implicit);
// keys and fractions come from particle_key.  Otherwise (key, id, fraction,
// mass) arrays of the previous pass.
// The fractions ride the sort as 6 bytes per particle: x and y's 16 bits in
// a 32-bit array, z's in a 16-bit one (18-byte records instead of 20).
struct ScatterIn {
  const uint32_t *key, *idx;
  const uint32_t *lo;
  const uint16_t *lz;
  const float *x, *y, *z, *m;
};

template <bool FIRST>
__global__ __launch_bounds__(STB) void k_scatter(BuildArgs a, int shift, const uint32_t *__restrict__ thist,
                                                 const uint32_t *__restrict__ tsum, uint64_t n_tiles, ScatterIn in,
                                                 uint32_t *__restrict__ key_out, uint32_t *__restrict__ idx_out,
                                                 uint32_t *__restrict__ lo_out, uint16_t *__restrict__ lz_out,
                                                 float *__restrict__ m_out) {
  const uint64_t N = a.N;
  constexpr int NW = STB / WAVE;              // waves per block
  constexpr int PER_WAVE = STILE / NW;
  constexpr int ROUNDS = PER_WAVE / WAVE;     // 8
  __shared__ uint32_t wcnt[NW][RADIX];
  __shared__ uint32_t bin_start[RADIX];       // tile-local start of each digit
  __shared__ uint32_t gofs[RADIX];            // global start of this tile's digit run
  __shared__ uint64_t stage[STILE];
  __shared__ uint32_t tmp[STB / WAVE + 1];

  const int lane = threadIdx.x & (WAVE - 1);
  const int w = threadIdx.x / WAVE;
  const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t tbase = tile * STILE;
  const uint64_t ebase = tbase + (uint64_t)w * PER_WAVE + lane;
  // this tile's global digit offsets (the scan of the digit-major counts: a
  // 4096-count block's own scan plus the scanned block totals), loaded first
  // (every thread, clamped index) so that waiting for them does not wait for
  // the element loads
  const uint64_t hi = (uint64_t)min((int)threadIdx.x, RADIX - 1) * n_tiles + tile;
  const uint32_t g0 = thist[hi] + tsum[hi / SCAN_TILE];
  uint32_t kk[ROUNDS], ii[ROUNDS];
  uint64_t ll[ROUNDS];
  float mm[ROUNDS];
  if (FIRST) {
    // every load of the thread first (the key computation branches on the
    // snapshot count, and a load issued after a branch waits for it)
    float xs[ROUNDS], ys[ROUNDS], zs[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      // clamped, unconditional loads; lanes past N are masked out below
      const uint64_t e = min(ebase + (uint64_t)r * WAVE, N - 1);
      xs[r] = in.x[e]; ys[r] = in.y[e]; zs[r] = in.z[e]; mm[r] = in.m[e];
    }
    bool bad_mass = false;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const uint64_t e = min(ebase + (uint64_t)r * WAVE, N - 1);
      const PKey pk = particle_key(a, xs[r], ys[r], zs[r], mm[r], e);
      kk[r] = pk.key;
      ll[r] = pk.lo;
      ii[r] = (uint32_t)(ebase + (uint64_t)r * WAVE);
      // keygen checked the positions; the masses are checked here
      bad_mass |= ebase + (uint64_t)r * WAVE < N && !(mm[r] >= 0.0f && mm[r] <= 3.4028235e38f);
    }
    if (bad_mass) atomicOr((unsigned long long *)&a.counts[2], (unsigned long long)LOD_STATUS_DOMAIN);
  } else {
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const uint64_t e = min(ebase + (uint64_t)r * WAVE, N - 1);
      kk[r] = in.key[e];
      ii[r] = in.idx[e];
      ll[r] = (uint64_t)in.lo[e] | ((uint64_t)in.lz[e] << 32);
      mm[r] = in.m[e];
    }
  }
  for (int i = threadIdx.x; i < NW * RADIX; i += STB) (&wcnt[0][0])[i] = 0;
  if (threadIdx.x < RADIX) gofs[threadIdx.x] = g0;
  __syncthreads();

  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
  uint32_t dig[ROUNDS];
  uint32_t rnk[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const bool valid = ebase + (uint64_t)r * WAVE < N;
    const uint32_t d = (kk[r] >> shift) & 0xFFu;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    const uint32_t old = valid ? wcnt[w][d] : 0u;
    if (valid && below == 0) wcnt[w][d] = old + cnt;
    dig[r] = d;
    rnk[r] = old + below;
  }
  // The payload loads have landed during the ranking: wait for them here,
  // before any store is issued.  Loads and stores share one counter, so a
  // wait placed where the values are first used would also wait for the
  // stores of the fields written before.  (Encoding: vmcnt 0, expcnt and
  // lgkmcnt left at their maxima.)
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  // per digit: wave prefix (in place) and tile total
  uint32_t tot = 0;
  if (threadIdx.x < RADIX) {
    const int d = threadIdx.x;
    for (int ww = 0; ww < NW; ++ww) {
      const uint32_t c = wcnt[ww][d];
      wcnt[ww][d] = tot;
      tot += c;
    }
  }
  uint32_t dummy;
  const uint32_t st = block_excl_scan<uint32_t>(threadIdx.x < RADIX ? tot : 0u, tmp, dummy);
  if (threadIdx.x < RADIX) bin_start[threadIdx.x] = st;
  __syncthreads();

  uint32_t slot[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) slot[r] = bin_start[dig[r]] + wcnt[w][dig[r]] + rnk[r];
  const uint32_t tile_n = (uint32_t)min((uint64_t)STILE, N - tbase);

  // keys (with their output positions), then ids, fractions, masses.  LDS
  // reads are unconditional (slots past the tile hold stale values) and
  // issued together; only the stores are predicated.
  uint64_t gpos[SITEMS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r)
    if (ebase + (uint64_t)r * WAVE < N) stage[slot[r]] = kk[r];
  __syncthreads();
  {
    uint32_t k[SITEMS], go[SITEMS], bs[SITEMS];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i) k[i] = (uint32_t)stage[i * STB + threadIdx.x];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i) {
      const uint32_t d = (k[i] >> shift) & 0xFFu;
      go[i] = gofs[d];
      bs[i] = bin_start[d];
    }
#pragma unroll
    for (int i = 0; i < SITEMS; ++i) {
      const uint32_t s = (uint32_t)i * STB + threadIdx.x;
      gpos[i] = (uint64_t)go[i] + (s - bs[i]);
      if (s < tile_n) key_out[gpos[i]] = k[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r)
    if (ebase + (uint64_t)r * WAVE < N) stage[slot[r]] = ii[r];
  __syncthreads();
  {
    uint32_t v[SITEMS];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i) v[i] = (uint32_t)stage[i * STB + threadIdx.x];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i)
      if ((uint32_t)i * STB + threadIdx.x < tile_n) idx_out[gpos[i]] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r)
    if (ebase + (uint64_t)r * WAVE < N) stage[slot[r]] = ll[r];
  __syncthreads();
  {
    uint64_t v[SITEMS];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i) v[i] = stage[i * STB + threadIdx.x];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i)
      if ((uint32_t)i * STB + threadIdx.x < tile_n) {
        lo_out[gpos[i]] = (uint32_t)v[i];
        lz_out[gpos[i]] = (uint16_t)(v[i] >> 32);
      }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r)
    if (ebase + (uint64_t)r * WAVE < N) stage[slot[r]] = (uint64_t)__float_as_uint(mm[r]);
  __syncthreads();
  {
    uint32_t v[SITEMS];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i) v[i] = (uint32_t)stage[i * STB + threadIdx.x];
#pragma unroll
    for (int i = 0; i < SITEMS; ++i)
      if ((uint32_t)i * STB + threadIdx.x < tile_n) m_out[gpos[i]] = __uint_as_float(v[i]);
  }
}

// ---------------------------------------------------------------------------
// density (run length of equal depth-L cells) and selection keys

template <bool MAXOP>
__device__ __forceinline__ uint64_t block_incl_scan_op(uint64_t v, uint64_t *tmp) {
  // inclusive max- or min-scan over threads in index order
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    uint64_t t = __shfl_up(v, o, WAVE);
    if (lane >= o) v = MAXOP ? max(v, t) : min(v, t);
  }
  if (lane == WAVE - 1) tmp[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = MAXOP ? 0ull : ~0ull;
    for (int ww = 0; ww < nw; ++ww) {
      uint64_t t = tmp[ww];
      tmp[ww] = run;
      run = MAXOP ? max(run, t) : min(run, t);
    }
  }
  __syncthreads();
  uint64_t pre = tmp[wid];
  __syncthreads();
  return MAXOP ? max(pre, v) : min(pre, v);
}

// Blocked layout: thread t owns tile elements [t*ITEMS, t*ITEMS+ITEMS).  A
// run's start is the largest run-start position at or before an element, its
// end the smallest run-end position after it; both come from a thread-local
// pass plus a block scan, and runs crossing the tile edge are closed by a
// binary search over the sorted keys.  The LDS arrays hold word i at
// i + i/16: blocked accesses (thread t at 16 t + k) would otherwise put a
// wave's lanes on four banks.
constexpr int DPAD = (TILE + 2) / 16 + 1;
__device__ __forceinline__ int dpad(int i) { return i + (i >> 4); }
__global__ __launch_bounds__(TB) void k_density(BuildArgs a, const uint32_t *__restrict__ skey,
                                                const uint32_t *__restrict__ sidx,
                                                uint32_t *__restrict__ w_out, uint16_t *__restrict__ kb_out) {
  __shared__ uint32_t cell[TILE + 2 + DPAD];   // cell[dpad(i+1)] = cell of element base+i
  __shared__ uint64_t tmp[TB / WAVE + 1];
  __shared__ uint64_t incl_max[TB];
  __shared__ uint64_t rev_min[TB];
  __shared__ uint64_t first_start, last_end;
  const uint64_t N = a.N;
  const uint64_t base = (uint64_t)blockIdx.x * TILE;
  const uint32_t tile_n = (uint32_t)min((uint64_t)TILE, N - base);
  const int sh = a.shift_rho;
  {
    // clamped, unconditional loads first, then the selects
    constexpr int CI = (TILE + 2 + TB - 1) / TB;
    uint32_t kc[CI];
#pragma unroll
    for (int j = 0; j < CI; ++j) {
      const int64_t e = (int64_t)base + j * TB + (int)threadIdx.x - 1;
      kc[j] = skey[(uint64_t)min(max(e, (int64_t)0), (int64_t)N - 1)];
    }
#pragma unroll
    for (int j = 0; j < CI; ++j) {
      const int i = j * TB + (int)threadIdx.x;
      const int64_t e = (int64_t)base + i - 1;
      if (i < TILE + 2)
        cell[dpad(i)] = (e >= 0 && (uint64_t)e < N && i <= (int)tile_n + 1) ? (kc[j] >> sh) : 0xFFFFFFFFu;
    }
  }
  __syncthreads();
  const bool has_prev = base > 0;
  const bool has_next = base + tile_n < N;
  if (threadIdx.x == 0) {
    // runs crossing the tile edges: galloping search outward from the edge
    uint64_t s0 = base;
    if (has_prev && cell[dpad(0)] == cell[dpad(1)]) {
      const uint32_t c = cell[dpad(1)];
      uint64_t right = base, step = 1, lo = 0;
      while (true) {
        if (right < step) { lo = 0; break; }
        const uint64_t probe = right - step;
        if ((skey[probe] >> sh) < c) { lo = probe + 1; break; }
        right = probe;
        step <<= 1;
      }
      uint64_t l = lo, h = right;
      while (l < h) {
        const uint64_t mid = l + ((h - l) >> 1);
        if ((skey[mid] >> sh) < c) l = mid + 1; else h = mid;
      }
      s0 = l;
    }
    first_start = s0;
    uint64_t e0 = base + tile_n;
    if (has_next && cell[dpad(tile_n)] == cell[dpad(tile_n + 1)]) {
      const uint32_t c = cell[dpad(tile_n)];
      uint64_t known = base + tile_n - 1, step = 1, hi = N;
      while (true) {
        const uint64_t probe = known + step;
        if (probe >= N) { hi = N; break; }
        if ((skey[probe] >> sh) > c) { hi = probe; break; }
        known = probe;
        step <<= 1;
      }
      uint64_t l = known + 1, h = hi;
      while (l < h) {
        const uint64_t mid = l + ((h - l) >> 1);
        if ((skey[mid] >> sh) <= c) l = mid + 1; else h = mid;
      }
      e0 = l;
    }
    last_end = e0;
  }
  __syncthreads();
  const int t0 = threadIdx.x * ITEMS;
  // Positions within the tile are kept as 32-bit local offsets: a run start
  // as li + 1 (0: the run began before the tile, at first_start); a run end
  // as li + 1 < tile_n, or tile_n for the tile's last run (which ends at
  // last_end).
  // run starts: thread-local running max
  uint32_t st[ITEMS];
  uint32_t runmax = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int li = t0 + i;
    const bool starts =
        (li == 0) ? (!has_prev || cell[dpad(0)] != cell[dpad(1)]) : (cell[dpad(li)] != cell[dpad(li + 1)]);
    if (li < (int)tile_n && starts) runmax = (uint32_t)li + 1;
    st[i] = runmax;
  }
  incl_max[threadIdx.x] = block_incl_scan_op<true>((uint64_t)runmax, tmp);
  // run ends: thread-local suffix min
  uint32_t en[ITEMS];
  uint32_t runmin = 0xFFFFFFFFu;
#pragma unroll
  for (int i = ITEMS - 1; i >= 0; --i) {
    const int li = t0 + i;
    if (li < (int)tile_n) {
      if (li == (int)tile_n - 1) runmin = tile_n;
      else if (cell[dpad(li + 1)] != cell[dpad(li + 2)]) runmin = min(runmin, (uint32_t)li + 1);
    }
    en[i] = runmin;
  }
  __syncthreads();
  // suffix over threads: thread t scans the value of thread TB-1-t
  rev_min[threadIdx.x] = runmin;
  __syncthreads();
  const uint64_t mirrored = rev_min[TB - 1 - threadIdx.x];
  __syncthreads();
  rev_min[threadIdx.x] = block_incl_scan_op<false>(mirrored, tmp);
  __syncthreads();
  const uint32_t prev_max = threadIdx.x ? (uint32_t)incl_max[threadIdx.x - 1] : 0u;
  // min over threads > t == reversed inclusive scan at position TB-2-t
  const uint32_t next_min = (threadIdx.x < TB - 1) ? (uint32_t)min(rev_min[TB - 2 - threadIdx.x], 0xFFFFFFFFull)
                                                   : 0xFFFFFFFFu;
  const uint64_t fs = first_start, le = last_end;
  // run lengths, blocked -> LDS, then striped (coalesced) keys, ids and outputs
  uint32_t *wl = (uint32_t *)cell;           // cell[] is no longer needed; reuse it
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int li = t0 + i;
    if (li < (int)tile_n) {
      const uint32_t sl = max(st[i], prev_max), el = min(en[i], next_min);
      const uint64_t sg = sl ? base + sl - 1 : fs;
      const uint64_t eg = (el == tile_n) ? le : base + el;
      wl[dpad(li)] = (uint32_t)(eg - sg);
    }
  }
  __syncthreads();
  const int sdb = 3 * a.D;
  constexpr int DCH = 8;                     // ids loaded together
#pragma unroll
  for (int c = 0; c < ITEMS; c += DCH) {
    uint32_t ids[DCH], snaps[DCH];
#pragma unroll
    for (int i = 0; i < DCH; ++i) {
      ids[i] = sidx[min(base + (uint64_t)((c + i) * TB + threadIdx.x), N - 1)];
      snaps[i] = 0u;
    }
    if (a.n_snap > 1) {
#pragma unroll
      for (int i = 0; i < DCH; ++i)
        snaps[i] = (uint32_t)((uint64_t)skey[min(base + (uint64_t)((c + i) * TB + threadIdx.x), N - 1)] >> sdb);
    }
    uint32_t exact = 0;                      // items whose bin needs the exact key (rare)
#pragma unroll
    for (int i = 0; i < DCH; ++i) {
      const int li = (c + i) * TB + threadIdx.x;
      if (li < (int)tile_n) {
        const uint64_t e = base + li;
        const uint32_t w = wl[dpad(li)];
        // one snapshot: the counter's words 1-3 are zero, which folds the
        // first round's second product
        const uint64_t U = a.n_snap > 1 ? particle_U(local_id(a, snaps[i], ids[i]), snaps[i], a.seed)
                                        : (uint64_t)philox_word0(ids[i], 0u, 0u, 0u, (uint32_t)a.seed,
                                                                 (uint32_t)(a.seed >> 32)) + 1ull;
        w_out[e] = w;
        uint32_t bin;
        if (a.alpha <= 0) bin = kbin(selection_key(U, w, a.alpha));
        else if (!kbin_div_fast(U, w, bin)) exact |= 1u << i;
        if (!((exact >> i) & 1u)) kb_out[e] = (uint16_t)bin;
      }
    }
    // one copy of the exact path, entered by few lanes
    while (exact) {
      const int i = __ffs(exact) - 1;
      exact &= exact - 1u;
      const int li = (c + i) * TB + threadIdx.x;
      const uint64_t e = base + li;
      const uint32_t snap = a.n_snap > 1 ? (uint32_t)((uint64_t)skey[e] >> sdb) : 0u;
      const uint64_t U = particle_U(local_id(a, snap, sidx[e]), snap, a.seed);
      kb_out[e] = (uint16_t)kbin(div_u2p31(U, wl[dpad(li)]));
    }
  }
}

// ---------------------------------------------------------------------------
// tree, level by level

struct TreeArgs {
  uint64_t *prefix;
  uint8_t *depth;
  uint32_t *parent;
  uint32_t *first_child;
  uint8_t *child_mask;
  uint64_t *part_begin;
  uint64_t *part_count;
  uint64_t *pt_begin;
  uint32_t *pt_count;
  double *node_mass;
  uint32_t *pt_id;
  uint16_t *qx, *qy, *qz;
  float *pt_mass;
  // workspace
  uint32_t *lvl;      // [D+3] level starts; lvl[d+1] = end of level d
  uint32_t *cs;       // [node_cap * 9] octant starts (sorted positions) of internal nodes
  uint32_t *sel_idx;  // [node_cap] rank among all selecting nodes (levels in order), or NONE
  uint32_t *sel_node; // [node_cap] node of each selecting rank (NONE if it was not emitted)
  uint32_t *wit;      // [node_cap] witness sorted position, or NONE
  uint32_t *pend;     // [node_cap] number of selecting children not yet reduced
  uint32_t *lsel;     // [D+3] selecting nodes at levels < d (cumulative)
};

__device__ __forceinline__ void set_status(const BuildArgs &a, uint32_t bits) {
  atomicOr((unsigned long long *)&a.counts[2], (unsigned long long)bits);
}

// Roots: one per non-empty snapshot (single block).
__global__ __launch_bounds__(1024) void k_roots(BuildArgs a, TreeArgs t, const uint32_t *__restrict__ skey) {
  __shared__ uint32_t tmp[1024 / WAVE + 1];
  __shared__ uint32_t base_nodes, base_sel;
  if (threadIdx.x == 0) { base_nodes = 0; base_sel = 0; t.lvl[0] = 0; t.lsel[0] = 0; }
  __syncthreads();
  const int D = a.D;
  for (uint32_t s0 = 0; s0 < a.n_snap; s0 += blockDim.x) {
    const uint32_t s = s0 + threadIdx.x;
    uint64_t lo = 0, hi = 0;
    if (s < a.n_snap) {
      if (a.n_snap == 1) { lo = 0; hi = a.N; }
      else {
        const uint64_t k0 = (uint64_t)s << (3 * D), k1 = (uint64_t)(s + 1) << (3 * D);
        uint64_t l = 0, h = a.N;
        while (l < h) { uint64_t mid = l + ((h - l) >> 1); if ((uint64_t)skey[mid] < k0) l = mid + 1; else h = mid; }
        lo = l; h = a.N;
        while (l < h) { uint64_t mid = l + ((h - l) >> 1); if ((uint64_t)skey[mid] < k1) l = mid + 1; else h = mid; }
        hi = l;
      }
    }
    const uint32_t ne = (s < a.n_snap && hi > lo) ? 1u : 0u;
    const uint32_t se = (ne && hi - lo > a.n) ? 1u : 0u;
    uint32_t tot_n, tot_s;
    uint32_t on = block_excl_scan<uint32_t>(ne, tmp, tot_n);
    uint32_t os = block_excl_scan<uint32_t>(se, tmp, tot_s);
    if (ne) {
      const uint32_t v = base_nodes + on;
      if (v < a.node_cap) {
        t.prefix[v] = s; t.depth[v] = 0; t.parent[v] = NONE; t.first_child[v] = NONE;
        t.child_mask[v] = 0; t.part_begin[v] = lo; t.part_count[v] = hi - lo;
        t.sel_idx[v] = se ? base_sel + os : NONE; t.wit[v] = NONE; t.pend[v] = 0;
        if (se && base_sel + os < a.node_cap) t.sel_node[base_sel + os] = v;
      } else {
        set_status(a, LOD_STATUS_CAPACITY);
        if (se && base_sel + os < a.node_cap) t.sel_node[base_sel + os] = NONE;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) { base_nodes += tot_n; base_sel += tot_s; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { t.lvl[1] = min((uint64_t)base_nodes, a.node_cap); t.lsel[1] = base_sel; }
}

// Octant boundaries of the internal nodes of level d: 8 lanes per node.
__global__ __launch_bounds__(TB) void k_octants(BuildArgs a, TreeArgs t, const uint32_t *__restrict__ skey, int d) {
  const uint32_t b = t.lvl[d], e = t.lvl[d + 1];
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const int sh = 3 * (a.D - d - 1);
  for (uint64_t g = gtid; g < (uint64_t)(e - b) * 8; g += stride) {
    const uint32_t v = b + (uint32_t)(g >> 3);
    const uint32_t o = (uint32_t)(g & 7);
    const uint64_t cnt = t.part_count[v];
    if (!(cnt > a.n && d < a.D)) continue;
    const uint64_t lo = t.part_begin[v], hi = lo + cnt;
    uint64_t start = lo;
    if (o) {
      const uint64_t target = ((t.prefix[v] << 3) | o) << sh;
      uint64_t l = lo, h = hi;
      while (l < h) { uint64_t mid = l + ((h - l) >> 1); if ((uint64_t)skey[mid] < target) l = mid + 1; else h = mid; }
      start = l;
    }
    t.cs[(uint64_t)v * 9 + o] = (uint32_t)start;
    if (o == 7) t.cs[(uint64_t)v * 9 + 8] = (uint32_t)hi;
  }
}

// Emit level d+1 from level d in three launches.  Thread (i, o) of a block
// of EMIT_BT handles octant o of node i (8 nodes per wave, 32 per block), so
// a child's index is the node-major, octant-minor count of non-empty octants
// before it: per-block totals (k_emit_count), one scan of them
// (k_emit_scan), and the writes (k_emit_write) with a block scan inside.
// The emission runs beside the density kernel, which fills the CUs: a
// 256-thread block finds room as soon as one density block ends, a
// 1024-thread block only when a whole CU drains (the eight levels' chain
// measured 0.52 against 0.67 ms with 1024-thread blocks).
constexpr int EMIT_BT = 256;
constexpr int EMIT_NODES = EMIT_BT / 8;   // nodes per block

struct EmitOct {
  uint32_t v, cnt, begin;
  bool valid, split;
};

__device__ __forceinline__ EmitOct emit_octant(const BuildArgs &a, const TreeArgs &t, int d) {
  const uint32_t b = t.lvl[d], e = t.lvl[d + 1];
  EmitOct r{};
  const uint64_t v = (uint64_t)b + (uint64_t)blockIdx.x * EMIT_NODES + threadIdx.x / 8;
  const uint32_t o = threadIdx.x & 7u;
  r.valid = v < e;
  r.v = (uint32_t)v;
  const uint32_t vc = r.valid ? r.v : b;   // in bounds when the level is not empty
  r.split = r.valid && t.part_count[vc] > a.n && d < a.D;
  const uint32_t s0 = t.cs[(uint64_t)vc * 9 + o], s1 = t.cs[(uint64_t)vc * 9 + o + 1];
  r.cnt = r.split ? s1 - s0 : 0u;
  r.begin = s0;
  return r;
}

__global__ __launch_bounds__(EMIT_BT) void k_emit_count(BuildArgs a, TreeArgs t, int d, uint32_t *__restrict__ tot) {
  __shared__ uint32_t tmp[EMIT_BT / WAVE + 1];
  if (t.lvl[d] + (uint64_t)blockIdx.x * EMIT_NODES >= t.lvl[d + 1]) {
    if (threadIdx.x == 0) { tot[2 * blockIdx.x] = 0; tot[2 * blockIdx.x + 1] = 0; }
    return;
  }
  const EmitOct x = emit_octant(a, t, d);
  uint32_t tk, ts;
  block_excl_scan<uint32_t>(x.cnt > 0 ? 1u : 0u, tmp, tk);
  block_excl_scan<uint32_t>(x.cnt > a.n ? 1u : 0u, tmp, ts);
  if (threadIdx.x == 0) { tot[2 * blockIdx.x] = tk; tot[2 * blockIdx.x + 1] = ts; }
}

// exclusive scan of the (children, selecting children) totals of nb blocks,
// and the extent of level d+1
__global__ __launch_bounds__(1024) void k_emit_scan(BuildArgs a, TreeArgs t, int d, uint32_t *__restrict__ tot,
                                                    uint32_t nb) {
  __shared__ uint32_t tmp[1024 / WAVE + 1];
  __shared__ uint32_t run_k, run_s;
  if (threadIdx.x == 0) { run_k = 0; run_s = 0; }
  __syncthreads();
  for (uint32_t j0 = 0; j0 < nb; j0 += blockDim.x) {
    const uint32_t j = j0 + threadIdx.x;
    const uint32_t ck = j < nb ? tot[2 * j] : 0u, cs = j < nb ? tot[2 * j + 1] : 0u;
    uint32_t tk, ts;
    const uint32_t ek = block_excl_scan<uint32_t>(ck, tmp, tk);
    const uint32_t es = block_excl_scan<uint32_t>(cs, tmp, ts);
    if (j < nb) { tot[2 * j] = run_k + ek; tot[2 * j + 1] = run_s + es; }
    __syncthreads();
    if (threadIdx.x == 0) { run_k += tk; run_s += ts; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint64_t end = (uint64_t)t.lvl[d + 1] + run_k;
    t.lvl[d + 2] = (uint32_t)min(end, a.node_cap);
    t.lsel[d + 2] = t.lsel[d + 1] + run_s;
  }
}

__global__ __launch_bounds__(EMIT_BT) void k_emit_write(BuildArgs a, TreeArgs t, int d,
                                                     const uint32_t *__restrict__ tot) {
  __shared__ uint32_t tmp[EMIT_BT / WAVE + 1];
  if (t.lvl[d] + (uint64_t)blockIdx.x * EMIT_NODES >= t.lvl[d + 1]) return;
  const EmitOct x = emit_octant(a, t, d);
  const uint32_t o = threadIdx.x & 7u;
  const bool ne = x.cnt > 0, se = x.cnt > a.n;
  uint32_t tk, ts;
  const uint32_t ok = block_excl_scan<uint32_t>(ne ? 1u : 0u, tmp, tk);
  const uint32_t os = block_excl_scan<uint32_t>(se ? 1u : 0u, tmp, ts);
  const uint64_t c = (uint64_t)t.lvl[d + 1] + tot[2 * blockIdx.x] + ok;   // this octant's child
  const uint32_t sidx = t.lsel[d + 1] + tot[2 * blockIdx.x + 1] + os;
  // the node's 8 octants are 8 consecutive lanes of one wave
  const int sh = (int)(threadIdx.x & (WAVE - 1) & ~7u);
  const uint32_t mask = (uint32_t)(__ballot(ne) >> sh) & 0xFFu;
  const uint32_t nsel = (uint32_t)__popc((uint32_t)(__ballot(se) >> sh) & 0xFFu);
  if (x.valid && o == 0) {
    t.child_mask[x.v] = (uint8_t)mask;
    t.pend[x.v] = nsel;
    t.first_child[x.v] = (mask && c + __popc(mask) <= a.node_cap) ? (uint32_t)c : NONE;
  }
  if (!ne) return;
  if (c >= a.node_cap) {
    set_status(a, LOD_STATUS_CAPACITY);
    if (se && sidx < a.node_cap) t.sel_node[sidx] = NONE;
    return;
  }
  t.prefix[c] = (t.prefix[x.v] << 3) | (uint64_t)o;
  t.depth[c] = (uint8_t)(d + 1);
  t.parent[c] = x.v;
  t.first_child[c] = NONE;
  t.child_mask[c] = 0;
  t.part_begin[c] = x.begin;
  t.part_count[c] = x.cnt;
  t.sel_idx[c] = se ? sidx : NONE;
  if (se && sidx < a.node_cap) t.sel_node[sidx] = (uint32_t)c;
  t.wit[c] = NONE;
  t.pend[c] = 0;
}

// pt_count for every slot < node_cap (0 beyond the node count) and n_nodes.
__global__ __launch_bounds__(TB) void k_ptcount(BuildArgs a, TreeArgs t, int D) {
  const uint32_t nn = t.lvl[D + 1];
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.node_cap;
       v += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t c = 0;
    if (v < nn) c = (uint32_t)min(t.part_count[v], (uint64_t)a.n);
    t.pt_count[v] = v < nn ? c : 0u;
    t.pt_begin[v] = c;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.counts[0] = nn;
}

__global__ void k_ptfinish(BuildArgs a, TreeArgs t) {
  // total = last exclusive offset + last count (both over node_cap slots)
  const uint64_t last = a.node_cap - 1;
  const uint64_t total = t.pt_begin[last] + t.pt_count[last];
  a.counts[1] = total;
  if (total > a.point_cap) set_status(a, LOD_STATUS_CAPACITY);
}

// ---------------------------------------------------------------------------
// leaves: float64 node mass; leaves holding <= n copy their particles

struct Sorted {
  const uint32_t *key;
  const uint32_t *idx;
  const uint32_t *lo;   // x and y fractions (16 bits each)
  const uint16_t *lz;   // z fraction
  const float *m;
  const uint32_t *w;
  const uint16_t *kb;   // log-scale bin of the selection key
};

// A stored point's fields read from the sorted arrays (loads are issued for
// every lane; the stores are predicated by the caller).
struct PointIn {
  uint32_t k, id;
  uint64_t l;
};

__device__ __forceinline__ PointIn read_point(const Sorted &s, uint64_t pos) {
  return PointIn{s.key[pos], s.idx[pos], (uint64_t)s.lo[pos] | ((uint64_t)s.lz[pos] << 32)};
}

__device__ __forceinline__ void store_point_pos(const BuildArgs &a, const TreeArgs &t, const PointIn &q,
                                                uint64_t out, int d) {
  const int D = a.D;
  const uint32_t kk = D ? (q.k & (uint32_t)((1ull << (3 * D)) - 1)) : 0u;
  const uint32_t cx = compact3(kk), cy = compact3(kk >> 1), cz = compact3(kk >> 2);
  const uint32_t snap = (a.n_snap > 1) ? (uint32_t)((uint64_t)q.k >> (3 * D)) : 0u;
  t.pt_id[out] = (uint32_t)local_id(a, snap, q.id);
  t.qx[out] = quant_at(cx, (uint32_t)(q.l & 0xFFFFu), D, d);
  t.qy[out] = quant_at(cy, (uint32_t)((q.l >> 16) & 0xFFFFu), D, d);
  t.qz[out] = quant_at(cz, (uint32_t)((q.l >> 32) & 0xFFFFu), D, d);
}

__device__ __forceinline__ void store_point(const BuildArgs &a, const TreeArgs &t, const PointIn &q, uint64_t out,
                                            int d, float mass) {
  store_point_pos(a, t, q, out, d);
  t.pt_mass[out] = mass;
}

// Exact selection key of the particle at sorted position p.
__device__ __forceinline__ uint64_t exact_K(const BuildArgs &a, const Sorted &s, uint32_t p) {
  const uint32_t snap = (a.n_snap > 1) ? (uint32_t)((uint64_t)s.key[p] >> (3 * a.D)) : 0u;
  const uint64_t U = particle_U(local_id(a, snap, s.idx[p]), snap, a.seed);
  return selection_key(U, s.w[p], a.alpha);
}

constexpr int LILP = 4;       // particles per thread per step when copying a leaf

// Copies leaf v's particles to its stored points (codes at the leaf's depth,
// float32 masses as given), whole block.
__device__ __forceinline__ void copy_leaf_points(const BuildArgs &a, const TreeArgs &t, const Sorted &s,
                                                 uint32_t v) {
  const uint64_t b = t.part_begin[v], c = t.part_count[v];
  const uint64_t ob = t.pt_begin[v];
  const int d = t.depth[v];
  const uint32_t BS = blockDim.x;
  for (uint64_t i0 = threadIdx.x; i0 < c; i0 += (uint64_t)BS * LILP) {
    float mm[LILP];
    PointIn q[LILP];
#pragma unroll
    for (int u = 0; u < LILP; ++u) {
      const uint64_t pos = b + min(i0 + (uint64_t)u * BS, c - 1);
      mm[u] = s.m[pos];
      q[u] = read_point(s, pos);
    }
#pragma unroll
    for (int u = 0; u < LILP; ++u) {
      const uint64_t i = i0 + (uint64_t)u * BS;
      if (i < c) store_point(a, t, q[u], ob + i, d, mm[u]);
    }
  }
}

// Leaves: float64 mass of every leaf and, with COPY, its stored points (the
// per-level schedule copies them inside the selection launches instead).
template <bool COPY>
__global__ __launch_bounds__(TB) void k_leaves(BuildArgs a, TreeArgs t, Sorted s) {
  __shared__ double red[TB / WAVE + 1];
  const uint32_t nn = t.lvl[a.D + 1];
  const bool cap_ok = a.counts[1] <= a.point_cap;
  for (uint32_t v = blockIdx.x; v < nn; v += gridDim.x) {
    if (t.first_child[v] != NONE) continue;
    const uint64_t b = t.part_begin[v], c = t.part_count[v];
    const bool copy = COPY && c <= a.n && cap_ok;
    const uint64_t ob = t.pt_begin[v];
    const int d = t.depth[v];
    double acc = 0.0;
    if (copy) {
      for (uint64_t i0 = threadIdx.x; i0 < c; i0 += TB * LILP) {
        float mm[LILP];
        PointIn q[LILP];
#pragma unroll
        for (int u = 0; u < LILP; ++u) {
          const uint64_t pos = b + min(i0 + (uint64_t)u * TB, c - 1);
          mm[u] = s.m[pos];
          q[u] = read_point(s, pos);
        }
#pragma unroll
        for (int u = 0; u < LILP; ++u) {
          const uint64_t i = i0 + (uint64_t)u * TB;
          if (i < c) {
            acc += (double)mm[u];
            store_point(a, t, q[u], ob + i, d, mm[u]);
          }
        }
      }
    } else {
      constexpr int MILP = 4 * LILP;
      for (uint64_t i0 = threadIdx.x; i0 < c; i0 += TB * MILP) {
        float mm[MILP];
#pragma unroll
        for (int u = 0; u < MILP; ++u) mm[u] = s.m[b + min(i0 + (uint64_t)u * TB, c - 1)];
#pragma unroll
        for (int u = 0; u < MILP; ++u)
          if (i0 + (uint64_t)u * TB < c) acc += (double)mm[u];
      }
    }
    const double M = block_reduce_sum<double>(acc, red);
    if (threadIdx.x == 0) t.node_mass[v] = M;
  }
}

// ---------------------------------------------------------------------------
// selection: per node holding > n particles, the n+1 smallest (K, id)

constexpr int SMALL = 512;
constexpr int KBINS = 4096;
constexpr int SILP = 8;       // candidates per lane per wave step
constexpr int CILP = 8;       // candidates per lane per step of the compaction pass of list nodes
constexpr int OILP = 4;       // list entries per thread per step of the output pass
constexpr int FILP = 2;       // candidates per lane per step of the fused pass of range-only nodes
constexpr int QCAP = 2048;    // bin-b0 candidates queued in LDS by the collect pass
constexpr int HT = 2 * SMALL; // slots of the table of ranked candidates (load <= 1/2)
static_assert(2 * HT <= KBINS, "the table lives in the histogram's storage");

__device__ __forceinline__ uint32_t ht_slot(uint32_t p) { return (p * 2654435761u) >> 22; }   // HT = 2^10
static_assert(HT == 1024, "ht_slot takes the top 10 bits");

// A list entry is a sorted position, its key bin and the candidate's density
// weight and mass (so that the parent's output pass reads them in list order
// instead of gathering them from the sorted arrays).
struct SelArgs {
  uint32_t *lpos;             // top-(n+1) lists by selecting rank: sorted positions
  uint16_t *lkb;              // and their key bins (a separate array: the counting passes read only these)
  uint2 *lwm;                 // and (w, mass bits)
  uint32_t n_minus_1;         // N - 1
  double *mhat;               // float64 mass scratch, one row of n per block
  uint32_t *src;              // source of each list entry, one row of n+1 per block
};

// sorted position of list entry i (clamped: the lists are workspace)
__device__ __forceinline__ uint32_t entry_pos(const SelArgs &sa, uint64_t i) { return min(sa.lpos[i], sa.n_minus_1); }

struct Segs {
  uint32_t nseg;
  uint64_t base[9];   // start sorted position (range) or list offset (list)
  uint32_t len[9];
  uint32_t is_list[9];
  // list segments: the child's witness position, its first stored point and
  // its octant (the bit each cell coordinate gains from parent to child)
  uint32_t cwit[9];
  uint64_t cob[9];
  uint32_t coct[9];
};

// A node's children's fields, loaded by one lane each so that the loads of
// all children are in flight together.
struct Children {
  uint64_t pc[8], pb[8], ptb[8];
  uint32_t sel[8], wit[8], oct[8];
  double m[8];
};

__device__ __forceinline__ void build_segments(const BuildArgs &a, const TreeArgs &t, uint32_t v, uint32_t fc,
                                               int nk, const Children &ch, Segs &g) {
  const uint32_t n = a.n;
  uint32_t ns = 0;
  if (fc == NONE) {
    g.base[0] = t.part_begin[v]; g.len[0] = (uint32_t)t.part_count[v]; g.is_list[0] = 0; ns = 1;
  } else {
    for (int k = 0; k < nk; ++k) {
      if (ch.pc[k] > n) {
        g.base[ns] = (uint64_t)ch.sel[k] * (n + 1); g.len[ns] = n + 1; g.is_list[ns] = 1;
        g.cwit[ns] = ch.wit[k]; g.cob[ns] = ch.ptb[k]; g.coct[ns] = ch.oct[k];
        ++ns;
      } else if (ns > 0 && !g.is_list[ns - 1]) {
        g.len[ns - 1] += (uint32_t)ch.pc[k];   // siblings are adjacent in sorted order
      } else {
        g.base[ns] = ch.pb[k]; g.len[ns] = (uint32_t)ch.pc[k]; g.is_list[ns] = 0;
        ++ns;
      }
    }
  }
  g.nseg = ns;
}

// The candidates of a node are the concatenation of its segments, in sorted
// position order (runs of leaf children form one range segment).  Wave w of the block owns the w-th of W equal contiguous
// parts of every segment, so (segment, wave) parts are in candidate order and
// a wave streams its part in steps of 64 x SILP without block barriers.
__device__ __forceinline__ void wave_part(uint32_t L, uint32_t w, uint32_t W, uint32_t &lo, uint32_t &hi) {
  const uint32_t P = (L + W - 1) / W;
  lo = min(L, w * P);
  hi = min(L, lo + P);
}

// Loads NL candidates (sorted position, key bin) of a wave step; indices
// are clamped into the part, so every load is issued unconditionally.
template <int NL>
__device__ __forceinline__ void load_step(const Segs &g, int k, const SelArgs &sa, const Sorted &s, uint32_t j0,
                                          uint32_t hi, uint32_t (&pos)[NL], uint32_t (&kb)[NL]) {
  const uint32_t lane = threadIdx.x & (WAVE - 1);
  const uint64_t base = g.base[k];
  if (g.is_list[k]) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const uint64_t i = base + min(j0 + u * WAVE + lane, hi - 1);
      pos[u] = entry_pos(sa, i);
      kb[u] = sa.lkb[i];
    }
  } else {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const uint64_t p = base + min(j0 + u * WAVE + lane, hi - 1);
      pos[u] = (uint32_t)p;
      kb[u] = s.kb[p];
    }
  }
}

// Calls f(k, p, kb) for every candidate of this wave's parts, in no
// particular order (f is inlined many times: keep it small), with 16-byte
// loads of 8 key bins per lane so that many bytes are in flight per wave.  p
// is the sorted position for a range segment and the index within the list
// for a list segment (entry_pos gives its position).  Reads may run up to 16
// bytes past a part; the key-bin arrays are padded for it.
constexpr int BU = 4;         // 16-byte loads in flight per lane
template <typename F>
__device__ __forceinline__ void for_parts_bulk(const Segs &g, const SelArgs &sa, const Sorted &s, F f) {
  const uint32_t W = blockDim.x / WAVE, w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  for (int k = 0; k < (int)g.nseg; ++k) {
    uint32_t lo, hi;
    wave_part(g.len[k], w, W, lo, hi);
    if (lo >= hi) continue;
    const uint64_t b = g.base[k] + lo, e = g.base[k] + hi;   // element range [b, e)
    const uint16_t *kbp = g.is_list[k] ? sa.lkb : s.kb;
    const uint64_t off = g.is_list[k] ? g.base[k] : 0;
    const uint64_t a0 = b & ~7ull, last = (e - 1) & ~7ull;
    for (uint64_t q0 = a0; q0 < e; q0 += 8ull * WAVE * BU) {
      uint4 v[BU];
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        const uint64_t i = min(q0 + 8ull * (u * WAVE + lane), last);
        v[u] = *reinterpret_cast<const uint4 *>(kbp + i);
      }
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        const uint64_t i = q0 + 8ull * (u * WAVE + lane);
        const uint32_t wd[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const uint64_t ih = i + h;
          if (ih >= b && ih < e) f(k, (uint32_t)(ih - off), (wd[h >> 1] >> (16 * (h & 1))) & 0xFFFFu);
        }
      }
    }
  }
}

// Calls f(k, pos, kb) for every candidate of this wave's parts.
template <typename F>
__device__ __forceinline__ void for_parts(const Segs &g, const SelArgs &sa, const Sorted &s, F f) {
  const uint32_t W = blockDim.x / WAVE, w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  for (int k = 0; k < (int)g.nseg; ++k) {
    uint32_t lo, hi;
    wave_part(g.len[k], w, W, lo, hi);
    for (uint32_t j0 = lo; j0 < hi; j0 += WAVE * SILP) {
      uint32_t pos[SILP], kb[SILP];
      load_step(g, k, sa, s, j0, hi, pos, kb);
#pragma unroll 1
      for (int u = 0; u < SILP; ++u)
        if (j0 + u * WAVE + lane < hi) f(k, pos[u], kb[u]);
    }
  }
}

// Whether the candidate at sorted position p lies at or below the witness
// (K_t, id_t) in (K, id) order, from its exact key.
__device__ __forceinline__ bool taken_exact(const BuildArgs &a, const Sorted &s, uint32_t p, uint64_t Kt, uint32_t It) {
  const uint64_t K = exact_K(a, s, p);
  return K < Kt || (K == Kt && s.idx[p] <= It);
}

// Sum of row[0..n) in an order fixed by n alone, so that every block size and
// schedule stores the same bits: 64-entry chunks summed by a wave's xor
// butterfly (lane i holds entry 64c + i, absent entries 0; lane 0's value),
// groups of 64 chunk sums by one more butterfly, and the group sums added in
// order by thread 0.  Rows of up to RS_CHUNKS chunks take one pass (the waves
// load their chunks together); longer rows go group by group.  cs: RS_CHUNKS
// doubles of LDS; the result is returned to every thread (barriers inside).
constexpr uint32_t RS_CHUNKS = 256;
__device__ double row_sum_fixed(const double *row, uint32_t n, double *cs, double *res) {
  const uint32_t W = blockDim.x / WAVE, w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  const uint32_t chunks = (n + WAVE - 1) / WAVE;
  double total = 0.0;   // thread 0's
  auto chunk_sum = [&](uint32_t c) {
    double x = c * WAVE + lane < n ? row[c * WAVE + lane] : 0.0;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
    return x;
  };
  auto group_sum = [&](uint32_t g, uint32_t count) {   // wave 0: chunk sums g*64.. of cs
    double x = g * WAVE + lane < count ? cs[g * WAVE + lane] : 0.0;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
    return x;
  };
  if (chunks <= RS_CHUNKS) {
    constexpr int CU = 4;   // chunks of a wave loaded together
    for (uint32_t c0 = w; c0 < chunks; c0 += W * CU) {
      double x[CU];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const uint32_t c = c0 + u * W;
        const uint32_t j = min(c * WAVE + lane, n - 1);
        x[u] = (c < chunks && c * WAVE + lane < n) ? row[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < CU; ++u) {
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) x[u] += __shfl_xor(x[u], o, WAVE);
        if (lane == 0 && c0 + u * W < chunks) cs[c0 + u * W] = x[u];
      }
    }
    __syncthreads();
    if (w == 0)
      for (uint32_t g = 0; g * WAVE < chunks; ++g) {
        const double x = group_sum(g, chunks);
        if (lane == 0) total += x;
      }
  } else {
    for (uint32_t c0 = 0; c0 < chunks; c0 += WAVE) {
      for (uint32_t c = c0 + w; c < min(chunks, c0 + WAVE); c += W) {
        const double x = chunk_sum(c);
        if (lane == 0) cs[c - c0] = x;
      }
      __syncthreads();
      if (w == 0) {
        const double x = group_sum(0, min(chunks - c0, (uint32_t)WAVE));
        if (lane == 0) total += x;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) *res = total;
  __syncthreads();
  return *res;
}

// One selecting node, whole block: the n+1 smallest (K, id) among its
// candidates (children's lists or its own range) form its list, ascending by
// sorted position; the (n+1)-th smallest is the witness.  The other n are
// its stored points, written with their float64-renormalised masses.
//
// Round 0 histograms the 12-bit log-scale bin of K (stored per particle); the
// exact K is recomputed only in the threshold bin (rare further rounds split
// it by 8-bit digits of K, then of the id).  The collect pass gathers the
// threshold bin's candidates and counts, per (segment, wave) part, the
// candidates below it; after ranking, one scan of those counts gives every
// part its output offset and the write pass compacts each part with wave
// ballots.
__device__ void select_node(const BuildArgs &a, const TreeArgs &t, const Sorted &s, const SelArgs &sa,
                            uint32_t v) {
  __shared__ Segs g;
  __shared__ Children ch;
  __shared__ uint32_t hist[KBINS];
  __shared__ uint64_t ck[SMALL];
  __shared__ uint32_t cidx[SMALL];
  __shared__ uint32_t cpos[SMALL];
  __shared__ uint16_t cpart[SMALL];
  __shared__ uint32_t pcnt[9 * (1024 / WAVE)];   // per (segment, wave) part: count, then offset
  __shared__ uint32_t ccount, sh_total, nq;
  __shared__ uint32_t qpos[QCAP];
  __shared__ uint16_t qpart[QCAP];
  __shared__ uint32_t red32[1024 / WAVE + 1];
  __shared__ double cs64[RS_CHUNKS];
  __shared__ double sh_mtot;
  __shared__ uint64_t sh_kt;
  __shared__ uint32_t sh_it, sh_pt;
  __shared__ uint32_t sh_b, sh_below, sh_cnt;
  __shared__ double sh_tau;
  const uint32_t n = a.n;
  const int BS = blockDim.x;
  const uint32_t W = BS / WAVE, w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  if (threadIdx.x < WAVE) {
    const uint32_t fc = t.first_child[v];
    const int nk = fc == NONE ? 0 : __popc((uint32_t)t.child_mask[v]);
    if ((int)threadIdx.x < nk) {
      const uint32_t u = fc + threadIdx.x;
      ch.pc[threadIdx.x] = t.part_count[u]; ch.pb[threadIdx.x] = t.part_begin[u];
      ch.ptb[threadIdx.x] = t.pt_begin[u]; ch.sel[threadIdx.x] = t.sel_idx[u];
      ch.wit[threadIdx.x] = t.wit[u]; ch.oct[threadIdx.x] = (uint32_t)(t.prefix[u] & 7u);
      ch.m[threadIdx.x] = t.node_mass[u];
    }
    // the lanes' LDS writes before lane 0's reads (one wave)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (threadIdx.x == 0) {
      build_segments(a, t, v, fc, nk, ch, g);
      // an internal node's float64 mass: its children's, summed in octant
      // order (read back by this block after the barriers below)
      if (fc != NONE) {
        double M = 0.0;
        for (int k = 0; k < nk; ++k) M += ch.m[k];
        t.node_mass[v] = M;
      }
    }
  }
  for (int i = threadIdx.x; i < KBINS; i += BS) hist[i] = 0;
  for (int i = threadIdx.x; i < 9 * (int)W; i += BS) pcnt[i] = 0;
  if (threadIdx.x == 0) { sh_b = 0; sh_below = 0; sh_cnt = 0; }
  __syncthreads();
  for_parts_bulk(g, sa, s, [&](int, uint32_t, uint32_t kb) { atomicAdd(&hist[kb], 1u); });
  __syncthreads();
  uint32_t r = n;                            // 0-based rank of the witness among in-play
  {
    const int per = KBINS / BS;
    uint32_t loc = 0;
    for (int i = 0; i < per; ++i) loc += hist[threadIdx.x * per + i];
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t>(loc, red32, tot);
    if (r >= ex && r < ex + loc) {
      uint32_t below = ex;
      for (int i = 0; i < per; ++i) {
        const uint32_t h = hist[threadIdx.x * per + i];
        if (r < below + h) { sh_b = threadIdx.x * per + i; sh_below = below; sh_cnt = h; break; }
        below += h;
      }
    }
    __syncthreads();
  }
  const uint32_t b0 = sh_b;
  r -= sh_below;
  uint32_t inplay = sh_cnt;
  const uint32_t sh_cnt0 = sh_cnt;           // candidates in bin b0
  int kshift;                                // K >> kshift == kp for the in-play candidates
  uint64_t kp;
  if (b0 < 128) { kp = b0; kshift = 0; }
  else {
    const int e = 7 + (int)((b0 - 128) / 64);
    kp = 64 + (b0 - 128) % 64;
    kshift = e - 6;
  }
  int phase = 0;                             // 0: K bits, 1: id bits
  int ishift = 32;
  uint32_t ip = 0;
  __syncthreads();
  // further rounds (rare): 8-bit digits of the exact K, then of the id
  while (inplay > SMALL && !(phase == 1 && ishift == 0)) {
    if (phase == 0 && kshift == 0) { phase = 1; continue; }
    const int wb = phase == 0 ? min(8, kshift) : min(8, ishift);
    const int sft = (phase == 0 ? kshift : ishift) - wb;
    for (int i = threadIdx.x; i < RADIX; i += BS) hist[i] = 0;
    __syncthreads();
    for_parts(g, sa, s, [&](int, uint32_t p, uint32_t kb) {
      if (kb != b0) return;
      const uint64_t K = exact_K(a, s, p);
      bool match;
      uint32_t dg;
      if (phase == 0) {
        match = (K >> kshift) == kp;
        dg = (uint32_t)((K >> sft) & ((1u << wb) - 1));
      } else {
        const uint32_t id = s.idx[p];
        match = (K == kp) && ((ishift >= 32) ? true : ((id >> ishift) == ip));
        dg = (id >> sft) & ((1u << wb) - 1);
      }
      if (match) atomicAdd(&hist[dg], 1u);
    });
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t below = 0, bsel = 0, cnt = 0;
      for (uint32_t bb = 0; bb < (1u << wb); ++bb) {
        const uint32_t h = hist[bb];
        if (r < below + h) { bsel = bb; cnt = h; break; }
        below += h;
      }
      sh_b = bsel; sh_below = below; sh_cnt = cnt;
    }
    __syncthreads();
    r -= sh_below;
    inplay = sh_cnt;
    if (phase == 0) { kp = (kp << wb) | sh_b; kshift = sft; }
    else { ip = (ip << wb) | sh_b; ishift = sft; }
    __syncthreads();
  }
  // collect the in-play candidates; count, per part, the candidates of lower
  // bins and (once ranked) the in-play ones at or below the witness
  if (threadIdx.x == 0) { ccount = 0; sh_pt = NONE; nq = 0; }
  __syncthreads();
  // a candidate of bin b0 with exact key K: in play (collected) or, if not,
  // counted when it lies below the in-play digits
  auto visit_b0 = [&](uint32_t part, uint32_t p) {
    const uint64_t K = exact_K(a, s, p);
    const uint32_t id = s.idx[p];
    bool inp, lower;
    if (phase == 0) {
      inp = (K >> kshift) == kp;
      lower = (K >> kshift) < kp;
    } else {
      inp = (K == kp) && ((ishift >= 32) ? true : ((id >> ishift) == ip));
      lower = (K < kp) || (K == kp && ishift < 32 && (id >> ishift) < ip);
    }
    if (inp) {
      const uint32_t slot = atomicAdd(&ccount, 1u);
      if (slot < SMALL) { ck[slot] = K; cidx[slot] = id; cpos[slot] = p; cpart[slot] = (uint16_t)part; }
    } else if (lower) {
      atomicAdd(&pcnt[part], 1u);
    }
  };
  {
    uint32_t below_cnt = 0;
    int cur = -1;
    if (sh_cnt0 <= QCAP) {
      // bin-b0 candidates are queued in LDS and keyed afterwards by the whole block
      for_parts_bulk(g, sa, s, [&](int k, uint32_t p, uint32_t kb) {
        if (k != cur) {
          if (cur >= 0 && below_cnt) atomicAdd(&pcnt[cur * W + w], below_cnt);
          cur = k; below_cnt = 0;
        }
        if (kb < b0) ++below_cnt;
        else if (kb == b0) {
          const uint32_t q = atomicAdd(&nq, 1u);
          qpos[q] = p; qpart[q] = (uint16_t)(k * W + w);
        }
      });
      if (cur >= 0 && below_cnt) atomicAdd(&pcnt[cur * W + w], below_cnt);
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < nq; q += BS) {
        // a queued list candidate is its index in the list: look up its position
        const uint32_t k = qpart[q] / W, p = qpos[q];
        visit_b0(qpart[q], g.is_list[k] ? entry_pos(sa, g.base[k] + p) : p);
      }
    } else {
      for_parts(g, sa, s, [&](int k, uint32_t p, uint32_t kb) {
        if (k != cur) {
          if (cur >= 0 && below_cnt) atomicAdd(&pcnt[cur * W + w], below_cnt);
          cur = k; below_cnt = 0;
        }
        if (kb < b0) ++below_cnt;
        else if (kb == b0) visit_b0(k * W + w, p);
      });
      if (cur >= 0 && below_cnt) atomicAdd(&pcnt[cur * W + w], below_cnt);
    }
  }
  __syncthreads();
  const uint32_t cc = min(ccount, (uint32_t)SMALL);
  // The ranked candidates go into a hash table (sorted position -> taken),
  // kept in the histogram's storage (no longer needed), so that the
  // compaction pass decides them without recomputing their keys.
  uint32_t *ht_key = hist, *ht_tk = hist + HT;
  for (int i = threadIdx.x; i < HT; i += BS) ht_key[i] = NONE;
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < cc; e += BS) {
    const uint64_t Ke = ck[e];
    const uint32_t Ie = cidx[e];
    uint32_t rank = 0;
    // eight entries per step, every read issued before any compare (clamped
    // indices, masked counts), and no branches: the loop is bound by LDS
    // throughput instead of one read's latency per entry
    for (uint32_t f0 = 0; f0 < cc; f0 += 8) {
      uint64_t Kf[8];
      uint32_t If[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t f = min(f0 + (uint32_t)u, cc - 1);
        Kf[u] = ck[f];
        If[u] = cidx[f];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool lt = (Kf[u] < Ke) | ((Kf[u] == Ke) & (If[u] < Ie));
        rank += (lt & (f0 + (uint32_t)u < cc)) ? 1u : 0u;
      }
    }
    if (rank == r) { sh_kt = Ke; sh_it = Ie; sh_pt = cpos[e]; }
    if (rank <= r) atomicAdd(&pcnt[cpart[e]], 1u);
    const uint32_t pe = cpos[e];
    uint32_t h = ht_slot(pe);
    while (atomicCAS(&ht_key[h], NONE, pe) != NONE) h = (h + 1) & (HT - 1);   // keys are distinct
    ht_tk[h] = rank <= r ? 1u : 0u;
  }
  __syncthreads();
  if (sh_pt == NONE || ccount > SMALL) {
    if (threadIdx.x == 0) set_status(a, STATUS_INTERNAL);
    __syncthreads();
    return;
  }
  const uint64_t Kt = sh_kt;
  const uint32_t It = sh_it;
  const uint32_t pt = sh_pt;
  {
    // part offsets (exclusive, candidate order; at most 9 x 16 parts)
    const uint32_t np = g.nseg * W;
    const uint32_t c = threadIdx.x < np ? pcnt[threadIdx.x] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t>(c, red32, tot);
    if (threadIdx.x < np) pcnt[threadIdx.x] = ex;
    if (threadIdx.x == 0) sh_total = tot;
  }
  if (threadIdx.x == 0) {
    // the witness's tau
    const uint32_t kt = s.key[pt];
    const uint32_t snap_t = (a.n_snap > 1) ? (uint32_t)((uint64_t)kt >> (3 * a.D)) : 0u;
    const uint64_t Ut = particle_U(local_id(a, snap_t, s.idx[pt]), snap_t, a.seed);
    sh_tau = weight_pow(s.w[pt], a.alpha) * 4294967296.0 / (double)Ut;
  }
  __syncthreads();
  if (sh_total != n + 1) {
    if (threadIdx.x == 0) set_status(a, STATUS_INTERNAL);
    __syncthreads();
    return;
  }
  // compaction pass: the n+1 list entries, in candidate (= sorted position) order
  const double tau = sh_tau;
  const bool out_ok = a.counts[1] <= a.point_cap;
  uint32_t *out_pos = sa.lpos + (uint64_t)t.sel_idx[v] * (n + 1);
  uint16_t *out_kb = sa.lkb + (uint64_t)t.sel_idx[v] * (n + 1);
  uint2 *out_wm = sa.lwm + (uint64_t)t.sel_idx[v] * (n + 1);
  double *mrow = sa.mhat + (uint64_t)blockIdx.x * n;
  uint32_t *srow = sa.src + (uint64_t)blockIdx.x * (n + 1);
  const uint64_t ob = t.pt_begin[v];
  const int d = t.depth[v];
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
  bool lists = false;
  for (int k = 0; k < (int)g.nseg; ++k) lists |= g.is_list[k] != 0;
  // whether a candidate of the threshold bin is taken: ranked above (the
  // usual case) or decided by its exact key
  auto taken_b0 = [&](uint32_t p) -> bool {
    uint32_t h = ht_slot(p), found = 2u;
    for (int pr = 0; pr < HT; ++pr) {
      const uint32_t kh = ht_key[h];
      if (kh == p) { found = ht_tk[h]; break; }
      if (kh == NONE) break;
      h = (h + 1) & (HT - 1);
    }
    if (found != 2u) return found != 0u;
    return taken_exact(a, s, p, Kt, It);
  };
  if (!lists) {
    // Only ranges: one pass writes the list and the stored points, the
    // candidates' data loaded alongside their key bins (contiguous reads).
    for (int k = 0; k < (int)g.nseg; ++k) {
      uint32_t lo, hi;
      wave_part(g.len[k], w, W, lo, hi);
      uint32_t run = pcnt[k * W + w];
      const uint64_t base = g.base[k];
      for (uint32_t j0 = lo; j0 < hi; j0 += WAVE * FILP) {
        uint32_t pp[FILP], kbv[FILP], wv[FILP];
        PointIn q[FILP];
        float mm[FILP];
#pragma unroll
        for (int u = 0; u < FILP; ++u) {
          const uint32_t pu = (uint32_t)(base + min(j0 + u * WAVE + lane, hi - 1));
          pp[u] = pu;
          kbv[u] = s.kb[pu];
          q[u] = read_point(s, pu);
          wv[u] = s.w[pu];
          mm[u] = s.m[pu];
        }
#pragma unroll
        for (int u = 0; u < FILP; ++u) {
          bool tk = j0 + u * WAVE + lane < hi && kbv[u] <= b0;
          if (tk && kbv[u] == b0) tk = taken_b0(pp[u]);
          const uint64_t bal = __ballot(tk);
          const uint32_t o = run + (uint32_t)__popcll(bal & lt_mask);
          run += (uint32_t)__popcll(bal);
          if (tk && o <= n) {
            out_pos[o] = pp[u];
            out_kb[o] = (uint16_t)kbv[u];
            out_wm[o] = make_uint2(wv[u], __float_as_uint(mm[u]));
            if (out_ok && pp[u] != pt) {
              const uint32_t j = o - (pp[u] > pt ? 1u : 0u);
              const double mhat = (double)mm[u] / fmin(1.0, weight_pow(wv[u], a.alpha) / tau);
              store_point_pos(a, t, q[u], ob + j, d);
              mrow[j] = mhat;
            }
          }
        }
      }
    }
  } else {
    for (int k = 0; k < (int)g.nseg; ++k) {
      uint32_t lo, hi;
      wave_part(g.len[k], w, W, lo, hi);
      uint32_t run = pcnt[k * W + w];
      for (uint32_t j0 = lo; j0 < hi; j0 += WAVE * CILP) {
        uint32_t pos[CILP], kb[CILP];
        load_step<CILP>(g, k, sa, s, j0, hi, pos, kb);
#pragma unroll
        for (int u = 0; u < CILP; ++u) {
          bool tk = j0 + u * WAVE + lane < hi && kb[u] <= b0;
          if (tk && kb[u] == b0) tk = taken_b0(pos[u]);
          const uint64_t bal = __ballot(tk);
          const uint32_t o = run + (uint32_t)__popcll(bal & lt_mask);
          run += (uint32_t)__popcll(bal);
          if (tk && o <= n) {
            out_pos[o] = pos[u];
            out_kb[o] = (uint16_t)kb[u];
            // an entry of a child's list: record where (segment, index in the
            // child's list), so that the output pass reads it in list order
            uint32_t src = NONE;
            if (g.is_list[k] && n < (1u << 24)) src = ((uint32_t)k << 24) | (j0 + u * WAVE + lane);
            srow[o] = src;
          }
        }
      }
    }
    __syncthreads();
    // output pass over the list (every lane busy): the list's (w, mass) and
    // the stored points with their unscaled float64 masses, kept in this
    // block's scratch row
    for (uint32_t j0 = threadIdx.x; j0 <= n; j0 += BS * OILP) {
      uint32_t pos[OILP], src[OILP];
#pragma unroll
      for (int u = 0; u < OILP; ++u) {
        const uint32_t jl = min(j0 + u * BS, n);
        pos[u] = min(out_pos[jl], sa.n_minus_1);
        src[u] = srow[jl];
      }
      // An entry of a child's list takes (w, mass) from that list and, unless
      // it is the child's witness, id and codes from the child's stored point
      // (contiguous reads; each code gains the child's octant bit on top).
      // The others are gathered from the sorted arrays.  Every lane issues
      // both sets of loads at clamped addresses (the unused set hits one
      // cached line).
      PointIn q[OILP];
      uint32_t cid[OILP], cq[OILP][3];
      uint2 wm[OILP], lw[OILP];
      bool cp[OILP];
#pragma unroll
      for (int u = 0; u < OILP; ++u) {
        const bool fl = src[u] != NONE;
        const uint32_t kk = fl ? src[u] >> 24 : 0u;
        const uint32_t ic = src[u] & 0xFFFFFFu;
        cp[u] = fl && pos[u] != g.cwit[kk];
        const uint64_t ci = cp[u] ? g.cob[kk] + ic - (pos[u] > g.cwit[kk] ? 1u : 0u) : 0u;
        q[u] = read_point(s, cp[u] ? pt : pos[u]);
        cid[u] = t.pt_id[ci];
        cq[u][0] = t.qx[ci]; cq[u][1] = t.qy[ci]; cq[u][2] = t.qz[ci];
        lw[u] = sa.lwm[fl ? g.base[kk] + ic : 0u];
        wm[u] = make_uint2(s.w[fl ? pt : pos[u]], __float_as_uint(s.m[fl ? pt : pos[u]]));
      }
#pragma unroll
      for (int u = 0; u < OILP; ++u) {
        const uint32_t jl = j0 + u * BS;
        if (jl > n) continue;
        const uint2 e = src[u] != NONE ? lw[u] : wm[u];
        out_wm[jl] = e;
        if (!out_ok || pos[u] == pt) continue;
        const uint32_t j = jl - (pos[u] > pt ? 1u : 0u);
        const double mhat = (double)__uint_as_float(e.y) / fmin(1.0, weight_pow(e.x, a.alpha) / tau);
        if (cp[u]) {
          const uint32_t oc = g.coct[src[u] >> 24];
          t.pt_id[ob + j] = cid[u];
          t.qx[ob + j] = (uint16_t)((cq[u][0] >> 1) | ((oc & 1u) << 15));
          t.qy[ob + j] = (uint16_t)((cq[u][1] >> 1) | (((oc >> 1) & 1u) << 15));
          t.qz[ob + j] = (uint16_t)((cq[u][2] >> 1) | (((oc >> 2) & 1u) << 15));
        } else {
          store_point_pos(a, t, q[u], ob + j, d);
        }
        mrow[j] = mhat;
      }
    }
  }
  __syncthreads();
  if (out_ok) {
    const double tot = row_sum_fixed(mrow, n, cs64, &sh_mtot);
    const double scale = t.node_mass[v] / tot;
    for (uint32_t j0 = threadIdx.x; j0 < n; j0 += BS * SILP) {
      double mv[SILP];
#pragma unroll
      for (int u = 0; u < SILP; ++u) mv[u] = mrow[min(j0 + u * BS, n - 1)];
#pragma unroll
      for (int u = 0; u < SILP; ++u)
        if (j0 + u * BS < n) t.pt_mass[ob + j0 + u * BS] = (float)(scale * mv[u]);
    }
  }
  if (threadIdx.x == 0) t.wit[v] = pt;
  __syncthreads();
}

// mode 1: one launch per level, one block per selecting node of that level.
// The stored points of the leaves (needed by nothing in the build) are copied
// by the same launches, so that the copy fills the chip while a level's last
// nodes are being selected.  Block j of every launch owns the nodes
// v = k G + j (G blocks per launch, k = 0, 1, ...) and resumes at its cursor
// leaf_ctl[j].  Above level 0 a block copies only while the level still has
// nodes being selected (done count in leaf_ctl[G + d]), and a block that
// selected a node only once every block with a node has started (count in
// leaf_ctl[G + D + 1 + d]), so that copying never holds back the dispatch of a
// selecting block.  Level 0, launched last, copies what is left.  No block
// waits for another.  leaf_ctl starts at zero.
__global__ __launch_bounds__(1024) void k_select_level(BuildArgs a, TreeArgs t, Sorted s, SelArgs sa, int d,
                                                       uint32_t *leaf_ctl) {
  __shared__ uint32_t sh_go;
  const uint32_t b = t.lvl[d], e = t.lvl[d + 1];
  const uint32_t G = gridDim.x;
  uint32_t *done = leaf_ctl ? leaf_ctl + G : nullptr;
  uint32_t *started = leaf_ctl ? leaf_ctl + G + a.D + 1 : nullptr;
  // the level's selecting nodes by rank, so that the blocks with a node come first
  const uint32_t r0 = t.lsel[d];
  const uint32_t r1 = (uint32_t)min((uint64_t)t.lsel[d + 1], a.node_cap);
  const uint32_t sel_blocks = r1 > r0 ? min(G, r1 - r0) : 0u;
  if (started && blockIdx.x < sel_blocks && threadIdx.x == 0) atomicAdd(&started[d], 1u);
  for (uint32_t r = r0 + blockIdx.x; r < r1; r += G) {
    const uint32_t v = t.sel_node[r];
    if (v == NONE || v < b || v >= e || t.part_count[v] <= a.n) continue;
    // the selecting waves ahead of the copying ones in each CU's instruction
    // arbitration (the level ends with its last node, not with the copy)
    __builtin_amdgcn_s_setprio(2);
    select_node(a, t, s, sa, v);
    __builtin_amdgcn_s_setprio(0);
    if (done && threadIdx.x == 0) atomicAdd(&done[d], 1u);
  }
  if (!leaf_ctl) return;
  const uint32_t total = t.lsel[d + 1] - t.lsel[d];   // selecting nodes of this level
  if (d > 0 && blockIdx.x < sel_blocks) {
    __syncthreads();
    if (threadIdx.x == 0)
      sh_go = __hip_atomic_load(&started[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= sel_blocks;
    __syncthreads();
    if (!sh_go) return;
  }
  const uint32_t nn = t.lvl[a.D + 1];
  const bool cap_ok = a.counts[1] <= a.point_cap;
  uint32_t k = leaf_ctl[blockIdx.x];
  while (true) {
    const uint64_t v = (uint64_t)k * G + blockIdx.x;
    if (v >= nn) break;
    if (d > 0) {
      __syncthreads();
      if (threadIdx.x == 0)
        sh_go = __hip_atomic_load(&done[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < total;
      __syncthreads();
      if (!sh_go) break;
    }
    if (t.first_child[v] == NONE && t.part_count[v] <= a.n && cap_ok) copy_leaf_points(a, t, s, (uint32_t)v);
    ++k;
  }
  if (threadIdx.x == 0) leaf_ctl[blockIdx.x] = k;
}

// mode 0: one launch per selecting node.
__global__ __launch_bounds__(1024) void k_select_one(BuildArgs a, TreeArgs t, Sorted s, SelArgs sa, uint32_t v) {
  if (v >= t.lvl[a.D + 1] || t.part_count[v] <= a.n) return;
  select_node(a, t, s, sa, v);
}

// Selecting nodes none of whose children select: the starting points of the
// persistent schedule (flags for a compaction).
__global__ void k_bottom_flags(BuildArgs a, TreeArgs t, uint32_t *__restrict__ flag) {
  const uint32_t nn = t.lvl[a.D + 1];
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= a.node_cap;
       v += (uint64_t)gridDim.x * blockDim.x)
    flag[v] = (v < nn && t.part_count[v] > a.n && t.pend[v] == 0) ? 1u : 0u;
}

__global__ void k_bottom_write(BuildArgs a, const uint32_t *__restrict__ flag, const uint32_t *__restrict__ scan,
                               uint32_t *__restrict__ bottom, uint32_t *__restrict__ ctl) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.node_cap;
       v += (uint64_t)gridDim.x * blockDim.x)
    if (flag[v]) bottom[scan[v]] = (uint32_t)v;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[0] = scan[a.node_cap];   // number of starting nodes
    ctl[1] = 0;                  // ticket
    ctl[2] = 0;                  // leaf-copy cursor
  }
}

// mode 2: one persistent launch over every selecting node of every level.
// A block takes a starting node by ticket (deepest first), reduces it (node
// mass, selection, output) and then, if it was the last of its parent's
// selecting children to finish, continues with the parent; otherwise it takes
// the next ticket.  Once the tickets are gone a block copies leaves, a chunk
// of nodes at a time from a shared cursor, until none are left.  No block
// ever waits for another, so the grid drains without spinning.  (Copying a
// chunk between tickets, or by only part of the grid, measured slower: it
// delays the starting nodes, and the climbs near the root gain little from
// the bandwidth left to them.)
//
// The eight XCDs do not share an L2, so a hand-off between blocks needs an
// agent-scope release by the writer (its lists, mass and witness written back
// to memory) and an agent-scope acquire by the climber.  A release writes the
// whole L2 of the XCD back, so a block issues one per node, from one wave,
// once every wave's stores have completed (a workgroup barrier alone does not
// wait for them); each wave of a climbing block acquires for itself.  A
// starting node's inputs come from earlier launches and need no acquire.
constexpr uint32_t LEAF_CHUNK = 8;   // nodes per leaf-copy grab

// Copies the leaves among the next LEAF_CHUNK nodes of the shared cursor;
// false once the cursor has passed every node (uniform over the block).
__device__ __forceinline__ bool copy_leaf_chunk(const BuildArgs &a, const TreeArgs &t, const Sorted &s,
                                                uint32_t *cursor, uint32_t &sh) {
  const uint32_t nn = t.lvl[a.D + 1];
  if (threadIdx.x == 0) sh = atomicAdd(cursor, LEAF_CHUNK);
  __syncthreads();
  const uint32_t v0 = sh;
  __syncthreads();
  if (v0 >= nn) return false;
  const bool cap_ok = a.counts[1] <= a.point_cap;
  const uint32_t v1 = min(nn, v0 + LEAF_CHUNK);
  for (uint32_t v = v0; v < v1; ++v)
    if (t.first_child[v] == NONE && t.part_count[v] <= a.n && cap_ok) copy_leaf_points(a, t, s, v);
  return true;
}

__global__ __launch_bounds__(1024) void k_select_persistent(BuildArgs a, TreeArgs t, Sorted s, SelArgs sa,
                                                            const uint32_t *__restrict__ bottom,
                                                            uint32_t *__restrict__ ctl) {
  __shared__ uint32_t sh_v;
  while (true) {
    if (threadIdx.x == 0) {
      // deepest starting nodes first, so that climbs overlap the remaining work
      const uint32_t tk = atomicAdd(&ctl[1], 1u);
      sh_v = tk < ctl[0] ? bottom[ctl[0] - 1 - tk] : NONE;
    }
    __syncthreads();
    uint32_t v = sh_v;
    __syncthreads();
    if (v == NONE) break;
    while (true) {
      select_node(a, t, s, sa, v);
      // publish this node's outputs before its parent can be claimed: every
      // wave waits for its own stores (vmcnt 0: stores count there on this
      // architecture), then one wave writes the L2 back
      __syncthreads();
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt 0; expcnt and lgkmcnt at their maxima
      __syncthreads();
      if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t par = t.parent[v];
        uint32_t nxt = NONE;
        if (par != NONE && atomicSub(&t.pend[par], 1u) == 1u) nxt = par;
        sh_v = nxt;
      }
      __syncthreads();
      v = sh_v;
      __syncthreads();
      if (v == NONE) break;
      // every child of v has released its outputs: see them (select_node
      // sums v's mass from its children and reads their lists)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  // leaves read only the sorted arrays and the node table, both written by
  // earlier launches
  while (copy_leaf_chunk(a, t, s, &ctl[2], sh_v)) {
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

namespace lodh {

namespace {
__global__ void k_copy32(const uint32_t *__restrict__ a, uint32_t *__restrict__ b, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

template <typename T>
__global__ void k_fill(T *p, uint64_t n, T v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
}  // namespace

void fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st) {
  if (!n) return;
  const unsigned g = (unsigned)std::min<uint64_t>(1024, (n + 255) / 256);
  LOD_LAUNCH(k_fill<uint64_t>, dim3(g), dim3(256), 0, st, p, n, v);
}

void fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) {
  if (!n) return;
  const unsigned g = (unsigned)std::min<uint64_t>(1024, (n + 255) / 256);
  LOD_LAUNCH(k_fill<uint32_t>, dim3(g), dim3(256), 0, st, p, n, v);
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Blocks of the emit kernels: enough for the largest level.  A level below
// the roots holds at most 8 children of each splitting node above it, and the
// splitting nodes of a level hold more than n particles each, disjointly.
static unsigned emit_blocks(uint64_t N, uint32_t n, uint32_t n_snap) {
  const uint64_t max_level = std::max<uint64_t>(8 * (N / ((uint64_t)n + 1)), n_snap);
  return (unsigned)std::max<uint64_t>(1, (max_level + EMIT_NODES - 1) / EMIT_NODES);
}

BuildLayout build_layout(uint64_t N, const lod_params &p, uint32_t n_snap) {
  BuildLayout L{};
  const uint64_t Np = N ? N : 1;
  const uint64_t tiles = (Np + STILE - 1) / STILE;
  L.tiles = tiles;
  uint64_t per_level = N / ((uint64_t)p.n + 1);
  L.node_cap = (uint64_t)n_snap + 8ull * p.max_depth * per_level;
  if (L.node_cap == 0) L.node_cap = 1;
  L.point_cap = N + (uint64_t)p.n * p.max_depth * per_level;
  if (L.point_cap == 0) L.point_cap = 1;
  // selecting nodes of one level are disjoint and hold > n particles each
  const uint64_t max_sel = (uint64_t)(p.max_depth + 1) * per_level + n_snap;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.keyA = take(4 * Np); L.keyB = take(4 * Np);
  L.idxA = take(4 * Np); L.idxB = take(4 * Np);
  L.loA = take(4 * Np); L.loB = take(4 * Np);
  L.lzA = take(2 * Np); L.lzB = take(2 * Np);
  L.mA = take(4 * Np); L.mB = take(4 * Np);
  L.thist = take(4 * (size_t)RADIX * tiles);
  L.scan32 = take(4 * std::max(scan_tmp_elems<uint32_t>((uint64_t)RADIX * tiles),
                               scan_tmp_elems<uint32_t>(L.node_cap + 1)));
  L.scan64 = take(8 * scan_tmp_elems<uint64_t>(L.node_cap));
  L.w = take(4 * Np);
  L.kb = take(2 * Np + 16);            // bulk selection reads may overrun by 16 bytes
  L.lvl = take(4 * (size_t)(p.max_depth + 4));
  L.lsel = take(4 * (size_t)(p.max_depth + 4));
  L.cs = take(4 * 9 * (size_t)L.node_cap);
  L.sel_idx = take(4 * (size_t)L.node_cap);
  L.sel_node = take(4 * (size_t)L.node_cap);
  L.wit = take(4 * (size_t)L.node_cap);
  L.pend = take(4 * (size_t)L.node_cap);
  L.bflag = take(4 * (size_t)(L.node_cap + 1));
  L.bscan = take(4 * (size_t)(L.node_cap + 1));
  L.bottom = take(4 * (size_t)L.node_cap);
  L.ctl = take(64);
  // lists: position and key bin of each entry (the key bins padded for the
  // 16-byte reads of the counting passes)
  L.lpos = take(4 * std::max<uint64_t>(1, max_sel * ((uint64_t)p.n + 1)));
  L.lkb = take(2 * std::max<uint64_t>(1, max_sel * ((uint64_t)p.n + 1)) + 16);
  L.lwm = take(8 * std::max<uint64_t>(1, max_sel * ((uint64_t)p.n + 1)));
  L.sel_rows = (uint32_t)std::min<uint64_t>(4096, N / ((uint64_t)p.n + 1) + n_snap + 1);
  L.mhat = take(8 * (size_t)L.sel_rows * p.n);
  L.src = take(4 * (size_t)L.sel_rows * ((uint64_t)p.n + 1));
  L.leafctl = take(4 * ((size_t)L.sel_rows + 2 * (p.max_depth + 1)));   // leaf-copy cursors, level counts
  L.emit_tot = take(8 * ((size_t)emit_blocks(N, p.n, n_snap) + 1));   // per-block child totals of the emit
  L.total = off;
  return L;
}

// A second stream of the device (default priority) and two events: the density
// kernel runs on it beside the tree construction, which does not read its
// output.  Created at the first build outside stream capture; a build captured
// before that runs on one stream.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // Held from the fork event's record on the caller's stream to the side
  // stream's wait on it: builds issued by several host threads then each
  // fork from their own stream.  The join needs no lock: a later record of
  // it lies later on the side stream, so waiting on it only waits longer.
  std::mutex mu;
};

static SideStream *side_stream(hipStream_t st) {
  static std::mutex mu;
  static SideStream per_dev[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  SideStream &r = per_dev[dev];
  if (!r.s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      (void)hipStreamDestroy(s);
      return nullptr;
    }
    r.s = s; r.fork = a; r.join = b;
  }
  return &r;
}

int key_bits(const lod_params &p, uint32_t n_snap) {
  int sb = 0;
  while ((1ull << sb) < n_snap) ++sb;
  return 3 * (int)p.max_depth + sb;
}

lod_status launch_build(const lod_input &in, const lod_params &p, void *ws, const BuildLayout &L,
                        lod_tree &out, hipStream_t st) {
  char *W = (char *)ws;
  const uint64_t N = in.n_particles;
  const uint32_t n_snap = in.snap_offsets ? in.n_snapshots : 1;
  BuildArgs a{};
  a.N = N; a.n = p.n; a.D = (int)p.max_depth; a.shift_rho = 3 * ((int)p.max_depth - (int)p.density_level);
  a.alpha = p.alpha; a.seed = p.seed; a.n_snap = n_snap; a.snap_off = in.snap_offsets;
  a.node_cap = L.node_cap; a.point_cap = out.point_capacity; a.counts = out.counts;

  // fills instead of memsets: the build may be captured into a graph
  fill_u64(out.counts, 3, 0, st);
  uint32_t *lvl = (uint32_t *)(W + L.lvl);
  fill_u32(lvl, p.max_depth + 4, 0, st);
  if (N == 0) return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;

  LOD_LAUNCH(k_check_offsets, dim3(1), dim3(256), 0, st, a);

  uint32_t *keyA = (uint32_t *)(W + L.keyA), *keyB = (uint32_t *)(W + L.keyB);
  uint32_t *idxA = (uint32_t *)(W + L.idxA), *idxB = (uint32_t *)(W + L.idxB);
  uint32_t *loA = (uint32_t *)(W + L.loA), *loB = (uint32_t *)(W + L.loB);
  uint16_t *lzA = (uint16_t *)(W + L.lzA), *lzB = (uint16_t *)(W + L.lzB);
  float *mA = (float *)(W + L.mA), *mB = (float *)(W + L.mB);
  uint32_t *thist = (uint32_t *)(W + L.thist);
  uint32_t *scan32 = (uint32_t *)(W + L.scan32);
  const uint64_t tiles = (N + STILE - 1) / STILE;
  const uint64_t hist_n = (uint64_t)RADIX * tiles;
  const uint64_t dtiles = (N + TILE - 1) / TILE;

  LOD_LAUNCH(k_keygen, dim3((unsigned)tiles), dim3(TB), 0, st, in.x, in.y, in.z, a, thist, tiles);
  const int kb = key_bits(p, n_snap);
  const int passes = std::max(1, (kb + 7) / 8);
  // pass 0 reads the particles (keys recomputed, ids implicit) and writes B
  device_scan_blocks<uint32_t>(thist, hist_n, scan32, st);
  LOD_LAUNCH(k_scatter<true>, dim3((unsigned)tiles), dim3(STB), 0, st, a, 0, thist, scan32, tiles,
             ScatterIn{nullptr, nullptr, nullptr, nullptr, in.x, in.y, in.z, in.mass}, keyB, idxB, loB, lzB, mB);
  uint32_t *ks = keyB, *is = idxB, *ls = loB; uint16_t *zs = lzB; float *ms = mB;
  uint32_t *kd = keyA, *id = idxA, *ld = loA; uint16_t *zd = lzA; float *md = mA;
  for (int ps = 1; ps < passes; ++ps) {
    LOD_LAUNCH(k_upsweep, dim3((unsigned)tiles), dim3(TB), 0, st, ks, N, 8 * ps, thist, tiles);
    device_scan_blocks<uint32_t>(thist, hist_n, scan32, st);
    LOD_LAUNCH(k_scatter<false>, dim3((unsigned)tiles), dim3(STB), 0, st, a, 8 * ps, thist, scan32, tiles,
               ScatterIn{ks, is, ls, zs, nullptr, nullptr, nullptr, ms}, kd, id, ld, zd, md);
    std::swap(ks, kd); std::swap(is, id); std::swap(ls, ld); std::swap(zs, zd); std::swap(ms, md);
  }
  Sorted s{ks, is, ls, zs, ms, (const uint32_t *)(W + L.w), (const uint16_t *)(W + L.kb)};

  // density weights and key bins on the side stream, beside the tree
  // construction; joined before the selection
  SideStream *side = side_stream(st);
  hipStream_t dst = st;
  if (side) {
    std::lock_guard<std::mutex> lk(side->mu);
    if (hipEventRecord(side->fork, st) != hipSuccess || hipStreamWaitEvent(side->s, side->fork, 0) != hipSuccess)
      return LOD_EDEVICE;
    dst = side->s;
  }
  LOD_LAUNCH(k_density, dim3((unsigned)dtiles), dim3(TB), 0, dst, a, ks, is,
             (uint32_t *)(W + L.w), (uint16_t *)(W + L.kb));
  if (side && hipEventRecord(side->join, side->s) != hipSuccess) return LOD_EDEVICE;

  TreeArgs t{};
  t.prefix = out.prefix; t.depth = out.depth; t.parent = out.parent; t.first_child = out.first_child;
  t.child_mask = out.child_mask; t.part_begin = out.part_begin; t.part_count = out.part_count;
  t.pt_begin = out.pt_begin; t.pt_count = out.pt_count; t.node_mass = out.node_mass;
  t.pt_id = out.pt_id; t.qx = out.qx; t.qy = out.qy; t.qz = out.qz; t.pt_mass = out.pt_mass;
  t.lvl = lvl; t.cs = (uint32_t *)(W + L.cs); t.sel_idx = (uint32_t *)(W + L.sel_idx);
  t.sel_node = (uint32_t *)(W + L.sel_node);
  t.wit = (uint32_t *)(W + L.wit); t.pend = (uint32_t *)(W + L.pend); t.lsel = (uint32_t *)(W + L.lsel);

  const int D = (int)p.max_depth;
  LOD_LAUNCH(k_roots, dim3(1), dim3(1024), 0, st, a, t, ks);
  const uint64_t per_level = N / ((uint64_t)p.n + 1) + n_snap;
  const unsigned oct_grid = (unsigned)std::min<uint64_t>(4096, (per_level * 8 + TB - 1) / TB + 1);
  // blocks of the emit kernels: enough for the largest level (every level but
  // the roots' holds at most 8 children per selecting node of the level above)
  const unsigned emit_grid = emit_blocks(N, p.n, n_snap);
  uint32_t *emit_tot = (uint32_t *)(W + L.emit_tot);
  for (int d = 0; d < D; ++d) {
    LOD_LAUNCH(k_octants, dim3(oct_grid), dim3(TB), 0, st, a, t, ks, d);
    LOD_LAUNCH(k_emit_count, dim3(emit_grid), dim3(EMIT_BT), 0, st, a, t, d, emit_tot);
    LOD_LAUNCH(k_emit_scan, dim3(1), dim3(1024), 0, st, a, t, d, emit_tot, emit_grid);
    LOD_LAUNCH(k_emit_write, dim3(emit_grid), dim3(EMIT_BT), 0, st, a, t, d, emit_tot);
  }
  const unsigned cap_grid = (unsigned)std::min<uint64_t>(4096, (L.node_cap + TB - 1) / TB);
  LOD_LAUNCH(k_ptcount, dim3(cap_grid), dim3(TB), 0, st, a, t, D);
  device_scan<uint64_t>(out.pt_begin, L.node_cap, (uint64_t *)(W + L.scan64), st);
  LOD_LAUNCH(k_ptfinish, dim3(1), dim3(1), 0, st, a, t);

  const unsigned node_grid = (unsigned)std::min<uint64_t>(8192, L.node_cap);
  // the per-level and persistent schedules copy the leaves' points inside
  // their selection launches
  uint32_t *leaf_ctl = p.mode == 1 ? (uint32_t *)(W + L.leafctl) : nullptr;
  if (leaf_ctl) fill_u32(leaf_ctl, (uint64_t)L.sel_rows + 2 * (p.max_depth + 1), 0, st);
  if (p.mode == 0) {
    LOD_LAUNCH(k_leaves<true>, dim3(node_grid), dim3(TB), 0, st, a, t, s);
  } else {
    LOD_LAUNCH(k_leaves<false>, dim3(node_grid), dim3(TB), 0, st, a, t, s);
  }
  if (side && hipStreamWaitEvent(st, side->join, 0) != hipSuccess) return LOD_EDEVICE;

  SelArgs sa{(uint32_t *)(W + L.lpos), (uint16_t *)(W + L.lkb), (uint2 *)(W + L.lwm), (uint32_t)(N - 1),
             (double *)(W + L.mhat),
             (uint32_t *)(W + L.src)};
  const unsigned sel_threads = p.select_threads ? p.select_threads : 1024;
  // one scratch row of float64 masses per block
  const unsigned sel_grid = (unsigned)std::min<uint64_t>(L.sel_rows, per_level + 1);
  if (p.mode == 2) {
    uint32_t *bflag = (uint32_t *)(W + L.bflag), *bscan = (uint32_t *)(W + L.bscan);
    uint32_t *ctl = (uint32_t *)(W + L.ctl);
    const unsigned fg = (unsigned)std::min<uint64_t>(4096, (L.node_cap + 256) / 256);
    LOD_LAUNCH(k_bottom_flags, dim3(fg), dim3(256), 0, st, a, t, bflag);
    LOD_LAUNCH(k_copy32, dim3(fg), dim3(256), 0, st, bflag, bscan, L.node_cap + 1);
    device_scan<uint32_t>(bscan, L.node_cap + 1, (uint32_t *)(W + L.scan32), st);
    LOD_LAUNCH(k_bottom_write, dim3(fg), dim3(256), 0, st, a, bflag, bscan, (uint32_t *)(W + L.bottom), ctl);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return LOD_EDEVICE;
    const unsigned pgrid = std::min<unsigned>(L.sel_rows, p.persistent_blocks ? p.persistent_blocks
                                                                              : (unsigned)(2 * cus));
    LOD_LAUNCH(k_select_persistent, dim3(pgrid), dim3(sel_threads), 0, st, a, t, s, sa,
               (const uint32_t *)(W + L.bottom), ctl);
    return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
  }
  // the per-node reference schedule needs the level sizes on the host
  std::vector<uint32_t> hl;
  std::vector<uint64_t> hcount;
  if (p.mode == 0) {
    hl.resize(D + 4);
    if (hipMemcpyAsync(hl.data(), lvl, 4 * (D + 4), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return LOD_EDEVICE;
    hcount.resize(hl[D + 1] + 1);
    if (hl[D + 1] &&
        (hipMemcpyAsync(hcount.data(), out.part_count, 8ull * hl[D + 1], hipMemcpyDeviceToHost, st) != hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
      return LOD_EDEVICE;
  }
  for (int d = D; d >= 0; --d) {
    if (p.mode == 0) {
      for (uint32_t v = hl[d]; v < hl[d + 1]; ++v) {
        if (hcount[v] <= p.n) continue;
        LOD_LAUNCH(k_select_one, dim3(1), dim3(sel_threads), 0, st, a, t, s, sa, v);
      }
    } else {
      // a level of at most 64 nodes cannot fill the chip: give each node 1024 threads
      const bool few = d <= 2 && ((uint64_t)n_snap << (3 * d)) <= 64;
      LOD_LAUNCH(k_select_level, dim3(sel_grid), dim3(few ? 1024u : sel_threads), 0, st, a, t, s, sa, d,
                 leaf_ctl);
    }
  }
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

void *workspace_view(void *ws, const BuildLayout &L, uint32_t which, uint64_t N, int passes, uint64_t *count) {
  char *W = (char *)ws;
  const bool inB = (passes % 2) == 1;
  switch (which) {
    case 0: *count = N; return W + (inB ? L.keyB : L.keyA);
    case 1: *count = N; return W + (inB ? L.idxB : L.idxA);
    case 2: *count = N; return W + L.w;
    case 3: *count = N; return W + L.kb;
    case 4: *count = L.node_cap; return W + L.wit;
    default: *count = 0; return nullptr;
  }
}

}  // namespace lodh
