// Additive Gaussian point splat, its adjoint, and the LOD point decode for
// gfx950 (rendering paragraph of arXiv:0811.2055: every point drawn as a
// blob evaluated for each pixel it covers).
//
// Forward: points are binned to 16x16 pixel tiles by a stable counting sort
// (per-wave units, a count pass and a fill pass, ballot ranks inside the
// wave), so a tile's pair list depends on the input alone.  Each list is cut
// into slices of at most 2048 points; one 256-thread block per slice adds the
// separable blobs to its 16x16 tile as rank-64 products on the matrix cores
// (MFMA 16x16x4, float32).  Each wave folds its products into compensated
// (Neumaier) float32 sums of its own, and the four wave sums of a pixel are
// folded in wave order at the end of the slice.  A final pass adds a tile's
// slice partials in slice order, again compensated.  No floating-point atomics:
// the image is bit-reproducible.  The LOD render feeds the binning straight
// from the tree's 16-bit node-relative points, decoding them in registers.
//
// The screen position and pixel offsets follow a fixed float32 sequence with
// no contraction (this file is compiled with -ffp-contract=off) so that the
// set of pixels a point covers is decided exactly as written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>

#include "lod.h"
#include "lod_device.hpp"
#include "lod_internal.hpp"
#include "lod_scan.hpp"

using namespace lodk;

namespace {

constexpr int TS = lodh::SPLAT_TS;
constexpr int PT = 256;            // threads per block

struct Cam {
  uint32_t proj, W, H;
  float px, py, pz, rx, ry, rz, ux, uy, uz, fx, fy, fz, F, near_z;
  float R;          // truncation half-width in pixels (float32)
  float inv2s2;     // 1 / (2 sigma^2)
  float norm;       // 1 / (2 pi sigma^2)
  float inv_s2;     // 1 / sigma^2
  int win;          // candidate half-window, ceil(R) + 2
  int narrow;       // 1 when a blob covers fewer than 8 pixels per axis (R < 3.98)
  float kexp2;      // -log2(e) / (2 sigma^2): Gaussian factor = exp2(o^2 kexp2)
  uint32_t tiles_x, tiles_y;
  uint32_t blob;    // LOD_BLOB_GAUSSIAN or LOD_BLOB_CUBIC
  float hpx;        // cubic: fixed pixel radius (when Fhw == 0)
  float Fhw;        // cubic, perspective world size: fl(F h_world), else 0
  float hmax;       // largest pixel radius a blob can take (binning window)
};

Cam make_cam(const lod_camera &c, const splat_params &sp, const lodh::SplatLayout *L) {
  Cam k{};
  k.proj = c.projection; k.W = c.W; k.H = c.H;
  k.px = c.pos[0]; k.py = c.pos[1]; k.pz = c.pos[2];
  k.rx = c.right[0]; k.ry = c.right[1]; k.rz = c.right[2];
  k.ux = c.up[0]; k.uy = c.up[1]; k.uz = c.up[2];
  k.fx = c.fwd[0]; k.fy = c.fwd[1]; k.fz = c.fwd[2];
  k.F = c.F; k.near_z = c.near_z;
  const float s = sp.sigma_px;
  k.R = sp.radius_sigmas * s;
  const double s64 = (double)s;
  k.inv2s2 = (float)(1.0 / (2.0 * s64 * s64));
  k.norm = (float)(1.0 / (2.0 * M_PI * s64 * s64));
  k.inv_s2 = (float)(1.0 / (s64 * s64));
  k.win = (int)std::ceil((double)k.R) + 2;
  k.narrow = (double)k.R < 3.98 ? 1 : 0;
  k.kexp2 = (float)(-1.4426950408889634 / (2.0 * s64 * s64));
  if (L) { k.tiles_x = L->tiles_x; k.tiles_y = L->tiles_y; }
  k.blob = sp.blob;
  k.hpx = sp.h_px;
  k.Fhw = (sp.blob == LOD_BLOB_CUBIC && sp.h_world > 0.0f) ? c.F * sp.h_world : 0.0f;
  k.hmax = lodh::blob_max_radius(sp);
  if (sp.blob == LOD_BLOB_CUBIC) k.win = (int)std::ceil((double)k.hmax) + 2;
  return k;
}

// Pinned float32 projection; returns false when culled.
__device__ __forceinline__ bool project(const Cam &c, float x, float y, float z, float &u, float &v,
                                        float &xc, float &yc, float &zc) {
  if (c.proj == 0) {
    u = x * (float)c.W;
    v = y * (float)c.H;
    xc = yc = zc = 0.0f;
    return true;
  }
  const float dx = x - c.px, dy = y - c.py, dz = z - c.pz;
  xc = ((dx * c.rx) + (dy * c.ry)) + (dz * c.rz);
  yc = ((dx * c.ux) + (dy * c.uy)) + (dz * c.uz);
  zc = ((dx * c.fx) + (dy * c.fy)) + (dz * c.fz);
  if (!(zc > c.near_z)) return false;
  u = (c.F * __fdiv_rn(xc, zc)) + (float)c.W * 0.5f;
  v = (c.F * __fdiv_rn(yc, zc)) + (float)c.H * 0.5f;
  return true;
}

// First and last index in [lo_clip, hi_clip] whose float32 offset
// fl(t - (i + 1/2)) lies in [-R, R].  The offset is non-increasing in i, so
// the set is an interval; a float estimate is corrected by exact tests.
__device__ __forceinline__ bool clip_range(float t, float R, int lo_clip, int hi_clip, int &lo, int &hi) {
  auto inside_hi = [&](int i) { return t - ((float)i + 0.5f) >= -R; };   // offset not below -R
  auto inside_lo = [&](int i) { return t - ((float)i + 0.5f) <= R; };    // offset not above R
  int a = (int)floorf(t - 0.5f - R);
  while (!inside_lo(a)) ++a;
  while (inside_lo(a - 1)) --a;
  int b = (int)floorf(t - 0.5f + R);
  while (!inside_hi(b)) --b;
  while (inside_hi(b + 1)) ++b;
  lo = max(a, lo_clip);
  hi = min(b, hi_clip);
  return lo <= hi;
}

// Inclusive range [lo, hi] of pixel indices along one axis whose float32
// offset fl(t - (i + 1/2)) lies within [-R, R], clipped to [0, size).
__device__ __forceinline__ bool axis_range(const Cam &c, float t, uint32_t size, int &lo, int &hi) {
  const float lim = c.R + 4.0f;
  if (!(t > -lim && t < (float)size + lim)) return false;
  return clip_range(t, c.R, 0, (int)size - 1, lo, hi);
}

// --- binning -----------------------------------------------------------------
//
// Points are binned to 16x16 pixel tiles by a stable counting sort, so that
// every tile's pair list -- and with it the image -- is a function of the
// input alone.  The points are cut into U = 64 C contiguous ranges ("units"),
// one wave each.  Pass 1 counts each unit's pairs per tile into row u of a
// [U][tiles] table; two column scans (within chunks of 64 units, then over the
// C chunks) and a scan over tiles give every (tile, unit) its slot range.
// Pass 2 re-derives the pairs in the same order (64-point rounds, then a
// point's tiles row by row, then lane) and ranks equal tiles inside the wave
// with ballots, so the list of a tile is ordered by (unit, round, tile index
// within the point, lane).

constexpr int BW = 64;              // binning block: one wave, one unit
constexpr int BR = 8;               // rounds of 64 points loaded together by the count pass
constexpr int BR_FILL = 16;         // and by the fill pass (measured: 1.67 vs 1.78 ms at 150 M points;
                                    // sixteen in the count pass cost it 0.3 ms)

// decoded float32 coordinate of a stored point (cell coordinate c at depth d,
// 16-bit offset q): centre of the quantisation cell, exact in float32
__device__ __forceinline__ float decode_coord(uint32_t c, uint32_t q, int d) {
  return (float)(2u * ((c << 16) + q) + 1u) * ldexpf(1.0f, -(d + 17));
}

// float32 nearest (2 (c 2^16 + q + 4 dq) + 1) 2^-(d+17): the position a motion
// code dq moves a stored point to (signed: a point may leave its cell)
__device__ __forceinline__ float decode_motion(uint32_t c, uint32_t q, int dq, int d) {
  const int64_t Q = ((int64_t)c << 16) + (int64_t)q + 4 * (int64_t)dq;
  return (float)(2 * Q + 1) * ldexpf(1.0f, -(d + 17));
}

// fl(a + fl(t fl(b - a))): the value at frame time t in [0, 1] between a and b
__device__ __forceinline__ float lerp_t(float a, float b, float t) { return a + t * (b - a); }

// Point sources.  A wave first resolves the addresses of its next BR rounds of
// points (resolve + end_round, in round order), then issues all their loads
// at once (fetch), so one memory latency covers BR rounds.

// raw float32 arrays
struct RawSrc {
  const float *x, *y, *z, *m;
  uint64_t n;
  struct Addr {
    uint64_t k;
  };
  struct Cursor {
    uint64_t last;      // a valid index: loads are unconditional (a predicated
                        // load would be waited for on its own)
    __device__ void begin(const RawSrc &, uint64_t b, uint64_t e) { last = e - 1; }
    __device__ __forceinline__ Addr resolve(const RawSrc &, uint64_t k, bool valid) {
      return Addr{valid ? k : last};
    }
    __device__ void end_round(const RawSrc &) {}
    __device__ __forceinline__ void fetch(const RawSrc &s, const Addr &a, bool, float &px, float &py,
                                          float &pz, float &pm) const {
      px = s.x[a.k]; py = s.y[a.k]; pz = s.z[a.k]; pm = s.m[a.k];
    }
    // the point's attribute (second image channel)
    __device__ __forceinline__ float attr(const RawSrc &s, const Addr &a) const { return s.aux[a.k]; }
    __device__ __forceinline__ float wradius(const RawSrc &, const Addr &) const { return 0.0f; }
  };
  __device__ uint64_t count() const { return n_dev ? min(*n_dev, n) : n; }
  const float *aux = nullptr;
  const uint64_t *n_dev = nullptr;   // device count (at most n), when set
};

// Two snapshots of the same particles and a frame time t: every quantity is
// fl(a + fl(t fl(b - a))); per-point world radii (cubic blob) and colours
// are optional.
struct InterpSrc {
  const float *xa, *ya, *za, *ma, *xb, *yb, *zb, *mb;
  const float *ha, *hb, *ca, *cb;   // may be null
  uint64_t n;
  float t;
  struct Addr {
    uint64_t k;
  };
  struct Cursor {
    uint64_t last;
    __device__ void begin(const InterpSrc &, uint64_t b, uint64_t e) { last = e - 1; }
    __device__ __forceinline__ Addr resolve(const InterpSrc &, uint64_t k, bool valid) {
      return Addr{valid ? k : last};
    }
    __device__ void end_round(const InterpSrc &) {}
    __device__ __forceinline__ void fetch(const InterpSrc &s, const Addr &a, bool, float &px, float &py,
                                          float &pz, float &pm) const {
      const float x0 = s.xa[a.k], y0 = s.ya[a.k], z0 = s.za[a.k], m0 = s.ma[a.k];
      const float x1 = s.xb[a.k], y1 = s.yb[a.k], z1 = s.zb[a.k], m1 = s.mb[a.k];
      px = lerp_t(x0, x1, s.t); py = lerp_t(y0, y1, s.t); pz = lerp_t(z0, z1, s.t); pm = lerp_t(m0, m1, s.t);
    }
    __device__ __forceinline__ float attr(const InterpSrc &s, const Addr &a) const {
      return lerp_t(s.ca[a.k], s.cb[a.k], s.t);
    }
    __device__ __forceinline__ float wradius(const InterpSrc &s, const Addr &a) const {
      return s.ha ? lerp_t(s.ha[a.k], s.hb[a.k], s.t) : 0.0f;
    }
  };
  __device__ uint64_t count() const { return n; }
};

// The stored points of a list of tree nodes, decoded on the fly.  offs is the
// exclusive scan of the nodes' point counts; the wave keeps the node holding
// its current point in registers and walks offs per lane when a round crosses
// into later nodes.
template <bool MOTION>
struct TreeSrcT {
  lod_tree t;
  const uint32_t *ids;
  const uint64_t *offs;
  const uint64_t *n_ids;
  uint64_t max_ids;
  const uint64_t *total;     // points to draw (device)
  struct Addr {
    uint64_t sidx;
    uint32_t cx, cy, cz;
    int d;
  };
  struct Cursor {
    uint64_t c, ob, oe, pb, far_c;
    uint32_t cx, cy, cz;
    int d;
    __device__ __forceinline__ void set(const TreeSrcT &s, uint64_t cc) {
      c = cc;
      const uint32_t v = s.ids[cc];
      ob = s.offs[cc]; oe = s.offs[cc + 1];
      d = s.t.depth[v];
      const uint64_t pfx = s.t.prefix[v];
      const uint32_t cell = d ? (uint32_t)(pfx & ((1ull << (3 * d)) - 1)) : 0u;
      cx = compact3(cell); cy = compact3(cell >> 1); cz = compact3(cell >> 2);
      pb = s.t.pt_begin[v];
      far_c = cc;
    }
    __device__ void begin(const TreeSrcT &s, uint64_t b, uint64_t) {
      // the last node whose offset is <= b; it holds point b (b < total)
      uint64_t lo = 0, hi = min(*s.n_ids, s.max_ids);
      while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (s.offs[mid] <= b) lo = mid; else hi = mid;
      }
      set(s, lo);
    }
    __device__ __forceinline__ Addr resolve(const TreeSrcT &s, uint64_t k, bool valid) {
      // invalid lanes load the cached node's first point (in bounds, unused)
      Addr a{pb, cx, cy, cz, d};
      if (!valid) return a;
      if (k < oe) {
        a.sidx = pb + (k - ob);
        return a;
      }
      uint64_t cl = c + 1;
      while (s.offs[cl + 1] <= k) ++cl;
      far_c = max(far_c, cl);
      const uint32_t v = s.ids[cl];
      a.d = s.t.depth[v];
      const uint64_t pfx = s.t.prefix[v];
      const uint32_t cell = a.d ? (uint32_t)(pfx & ((1ull << (3 * a.d)) - 1)) : 0u;
      a.cx = compact3(cell); a.cy = compact3(cell >> 1); a.cz = compact3(cell >> 2);
      a.sidx = s.t.pt_begin[v] + (k - s.offs[cl]);
      return a;
    }
    // move the cached node to the furthest node any lane reached
    __device__ void end_round(const TreeSrcT &s) {
      if (!__ballot(far_c != c)) return;      // every lane stayed in the cached node
      uint64_t f = far_c;
#pragma unroll
      for (int o = 1; o < WAVE; o <<= 1) f = max(f, (uint64_t)__shfl_xor(f, o, WAVE));
      if (f != c) set(s, f);
    }
    __device__ __forceinline__ void fetch(const TreeSrcT &s, const Addr &a, bool, float &px, float &py,
                                          float &pz, float &pm) const {
      const uint32_t qx = s.t.qx[a.sidx], qy = s.t.qy[a.sidx], qz = s.t.qz[a.sidx];
      pm = s.t.pt_mass[a.sidx];
      if constexpr (MOTION) {
        // the point at frame time t between its decoded position and the
        // position its motion code decodes to
        const int dx = s.dqx[a.sidx], dy = s.dqy[a.sidx], dz = s.dqz[a.sidx];
        px = lerp_t(decode_coord(a.cx, qx, a.d), decode_motion(a.cx, qx, dx, a.d), s.t_frame);
        py = lerp_t(decode_coord(a.cy, qy, a.d), decode_motion(a.cy, qy, dy, a.d), s.t_frame);
        pz = lerp_t(decode_coord(a.cz, qz, a.d), decode_motion(a.cz, qz, dz, a.d), s.t_frame);
      } else {
        px = decode_coord(a.cx, qx, a.d);
        py = decode_coord(a.cy, qy, a.d);
        pz = decode_coord(a.cz, qz, a.d);
      }
    }
    __device__ __forceinline__ float wradius(const TreeSrcT &, const Addr &) const { return 0.0f; }
    // 1 when the stored point's highlight flag is set, else 0
    __device__ __forceinline__ float attr(const TreeSrcT &s, const Addr &a) const {
      return s.hl_test(a.sidx, s.hl_word(a.sidx)) ? 1.0f : 0.0f;
    }
    __device__ __forceinline__ uint64_t point_index(const TreeSrcT &, const Addr &a) const { return a.sidx; }
  };
  __device__ uint64_t count() const { return *total; }
  const uint32_t *hl_flags = nullptr;  // highlight flags, one bit per stored point
  uint64_t hl_words = 1;
  const int16_t *dqx = nullptr, *dqy = nullptr, *dqz = nullptr;   // motion codes (MOTION)
  float t_frame = 0.0f;
  // the flag word of stored point s (in bounds for any s) and its flag
  __device__ __forceinline__ uint32_t hl_word(uint64_t sidx) const {
    return hl_flags[min(sidx >> 5, hl_words - 1)];
  }
  __device__ __forceinline__ bool hl_test(uint64_t sidx, uint32_t word) const {
    return (word >> (uint32_t)(sidx & 31u)) & 1u;
  }
};
using TreeSrc = TreeSrcT<false>;
using TreeMotionSrc = TreeSrcT<true>;
template <class S> struct IsTree { static constexpr bool value = false; };
template <bool M> struct IsTree<TreeSrcT<M>> { static constexpr bool value = true; };

// One point's screen position, pixel radius (cubic blob), attribute and tile
// rectangle (ntx = nty = 0: not drawn).
struct Blob {
  float u, v, m, h, a;
  int tx0, ty0, ntx, nty;
};

// Pair records of the binned (point, tile) pairs, one type per render form:
// Gaussian (u, v, m) is float3; the others carry the attribute and / or the
// cubic blob's pixel radius.
struct RecGA { float u, v, m, a; };        // Gaussian + attribute
struct RecC { float u, v, m, h; };         // cubic
struct RecCA { float u, v, m, h, a; };     // cubic + attribute
__device__ __forceinline__ void rec_put(float3 *r, uint64_t i, const Blob &b) { r[i] = make_float3(b.u, b.v, b.m); }
__device__ __forceinline__ void rec_put(RecGA *r, uint64_t i, const Blob &b) { r[i] = RecGA{b.u, b.v, b.m, b.a}; }
__device__ __forceinline__ void rec_put(RecC *r, uint64_t i, const Blob &b) { r[i] = RecC{b.u, b.v, b.m, b.h}; }
__device__ __forceinline__ void rec_put(RecCA *r, uint64_t i, const Blob &b) { r[i] = RecCA{b.u, b.v, b.m, b.h, b.a}; }
template <class R> struct RecInfo { static constexpr bool aux = false; static constexpr bool cubic = false; };
template <> struct RecInfo<RecGA> { static constexpr bool aux = true; static constexpr bool cubic = false; };
template <> struct RecInfo<RecC> { static constexpr bool aux = false; static constexpr bool cubic = true; };
template <> struct RecInfo<RecCA> { static constexpr bool aux = true; static constexpr bool cubic = true; };

// Pixels [lo, hi] (clipped to [0, size)) that contain every pixel a blob at
// screen coordinate t can cover: the float32 offset test |t - (i + 1/2)| <= R
// is decided to within 2^-8 for |t| < 2^15 (the camera limits), so a margin
// of 1/100 pixel makes the range conservative.  A tile this admits without a
// covered pixel only adds a pair whose rows are zero in the accumulation.
__device__ __forceinline__ bool cover_range(float R, float t, uint32_t size, int &lo, int &hi) {
  const float lim = R + 4.0f;
  if (!(t > -lim && t < (float)size + lim)) return false;
  lo = max((int)ceilf(t - 0.5f - R - 0.01f), 0);
  hi = min((int)floorf(t - 0.5f + R + 0.01f), (int)size - 1);
  return lo <= hi;
}

// Pixel radius of a cubic blob at camera depth zc: the fixed radius, or the
// projected world radius fl(fl(F h_world) / zc) clamped to [1, 16] pixels.
// A per-point world radius hw > 0 replaces the camera's.
__device__ __forceinline__ float cubic_radius(const Cam &c, float zc, float hw = 0.0f) {
  const float Fhw = hw > 0.0f ? c.F * hw : c.Fhw;
  if (Fhw > 0.0f) return fminf(fmaxf(__fdiv_rn(Fhw, zc), lodh::BLOB_H_MIN), lodh::BLOB_H_MAX);
  return c.hpx;
}

__device__ __forceinline__ Blob make_blob(const Cam &c, bool valid, float px, float py, float pz, float pm,
                                          float pa = 0.0f, float hw = 0.0f) {
  Blob b{0.0f, 0.0f, pm, 0.0f, pa, 0, 0, 0, 0};
  if (!valid) return b;
  float xc, yc, zc;
  if (!project(c, px, py, pz, b.u, b.v, xc, yc, zc)) return b;
  const float R = c.blob == LOD_BLOB_CUBIC ? cubic_radius(c, zc, hw) : c.R;
  b.h = R;
  int i0, i1, j0, j1;
  if (!cover_range(R, b.u, c.W, i0, i1) || !cover_range(R, b.v, c.H, j0, j1)) return b;
  b.tx0 = i0 / TS; b.ty0 = j0 / TS;
  b.ntx = i1 / TS - b.tx0 + 1;
  b.nty = j1 / TS - b.ty0 + 1;
  return b;
}

__device__ __forceinline__ void lds_count_add(uint32_t *lc, uint32_t t, uint32_t cnt) { atomicAdd(&lc[t], cnt); }
__device__ __forceinline__ void lds_count_add(uint16_t *lc, uint32_t t, uint32_t cnt) {
  atomicAdd(reinterpret_cast<uint32_t *>(lc) + (t >> 1), cnt << (16 * (t & 1u)));
}

// One tile of every lane with `has` (tile t): lanes holding the same tile form
// a group and rank by lane index inside it; a group adds its size to the
// tile's counter and, with FILL, writes its records at the counter's old
// value plus the rank.  Spatially coherent points share few tiles, so groups
// are peeled off by their lowest lane first, with the group mask in scalar
// registers; after four groups the rest is matched bit by bit.  The grouping,
// not the method, decides the ranks.  Counting adds to LDS without reading
// back (16-bit counters are added in their 32-bit word; a unit's counts stay
// below 2^16, so no carry crosses the halves).
template <bool FILL, class CT, class RecT>
__device__ __forceinline__ void emit_tile(uint32_t t, bool has, int nbits, CT *lc, RecT *__restrict__ rec,
                                          const Blob &bl) {
  const int lane = threadIdx.x & (WAVE - 1);
  uint64_t pending = __ballot(has);
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    if (!pending) return;
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t tl = __builtin_amdgcn_readlane(t, leader);
    const bool mine = has && t == tl;
    const uint64_t grp = __ballot(mine);
    const uint32_t cnt = (uint32_t)__popcll(grp);
    if (FILL) {
      const uint32_t old = (uint32_t)lc[tl];
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(grp >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)grp, 0u));
      if (mine) rec_put(rec, old + rank, bl);
      if (lane == leader) lc[tl] = (CT)(old + cnt);
    } else {
      if (lane == leader) lds_count_add(lc, t, cnt);   // the leader's own tile (t == tl)
    }
    pending &= ~grp;
  }
  if (!pending) return;
  const bool rest = ((pending >> lane) & 1ull) != 0;
  uint64_t peers = pending;
  for (int b = 0; b < nbits; ++b) {
    const uint64_t bal = __ballot((t >> b) & 1u);
    peers &= ((t >> b) & 1u) ? bal : ~bal;
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
  const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
  const uint32_t cnt = (uint32_t)__popcll(peers);
  if (FILL) {
    const uint32_t old = rest ? (uint32_t)lc[t] : 0u;
    if (rest && below == 0) lc[t] = (CT)(old + cnt);
    if (rest) rec_put(rec, old + below, bl);
  } else if (rest && below == 0) {
    lds_count_add(lc, t, cnt);
  }
}

// Highlight staging: the count pass writes the decoded points whose id is
// selected to x, y, z, m at [b, b + k) of its unit's point range [b, e)
// (sequence order), and k to count[unit].
struct HlStage {
  float *x, *y, *z, *m;
  uint64_t *count, *scan;   // per unit (scan: a copy, scanned afterwards)
};

// Points [u0 per, min(n, (u0 + g) per)) with per = ceil(n / units): g
// consecutive units of the partition.  Returns the points staged (HL).
template <class Src, bool FILL, class CT, class RecT, bool HL = false>
__device__ __forceinline__ uint32_t bin_unit(const Src &src, const Cam &c, uint32_t units, uint32_t u0, uint32_t g,
                                             int nbits, CT *lc, RecT *__restrict__ rec, HlStage hs = HlStage{}) {
  const int lane = threadIdx.x;
  const uint64_t n = src.count();
  const uint64_t per = (n + units - 1) / units;
  const uint64_t b = (uint64_t)u0 * per, e = min(n, b + (uint64_t)g * per);
  uint32_t staged = 0;
  if (b >= e) return 0;
  typename Src::Cursor cur;
  cur.begin(src, b, e);
  constexpr int R = FILL ? BR_FILL : BR;
  for (uint64_t k0 = b; k0 < e; k0 += (uint64_t)R * WAVE) {
    typename Src::Addr ad[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t k = k0 + (uint64_t)r * WAVE + lane;
      ad[r] = cur.resolve(src, k, k < e);
      cur.end_round(src);
    }
    float px[R], py[R], pz[R], pm[R], pa[R], ph[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t k = k0 + (uint64_t)r * WAVE + lane;
      cur.fetch(src, ad[r], k < e, px[r], py[r], pz[r], pm[r]);
      pa[r] = (FILL && RecInfo<RecT>::aux) ? cur.attr(src, ad[r]) : 0.0f;
      ph[r] = c.blob == LOD_BLOB_CUBIC ? cur.wradius(src, ad[r]) : 0.0f;
    }
    if constexpr (HL) {
      // ID highlighting: the flag test of every drawn point, and the
      // flagged ones staged in sequence order (wave ballot ranks).  A wave's
      // points are mostly consecutive stored points, so its flag loads fall
      // on one or two words.
      uint64_t pid[R];
      uint32_t word[R];
#pragma unroll
      for (int r = 0; r < R; ++r) pid[r] = cur.point_index(src, ad[r]);
#pragma unroll
      for (int r = 0; r < R; ++r) word[r] = src.hl_word(pid[r]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool in = k0 + (uint64_t)r * WAVE + lane < e && src.hl_test(pid[r], word[r]);
        const uint64_t mask = __ballot(in);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (in) {
          const uint64_t o = b + staged + rank;
          hs.x[o] = px[r]; hs.y[o] = py[r]; hs.z[o] = pz[r]; hs.m[o] = pm[r];
        }
        staged += (uint32_t)__popcll(mask);
      }
    }
    Blob blobs[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
      blobs[r] = make_blob(c, k0 + (uint64_t)r * WAVE + lane < e, px[r], py[r], pz[r], pm[r], pa[r], ph[r]);
    // pairs in the order (round, tile row, tile column, lane)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const Blob &bl = blobs[r];
      for (int dy = 0; __ballot(dy < bl.nty); ++dy) {
        for (int dx = 0; __ballot(dy < bl.nty && dx < bl.ntx); ++dx) {
          const bool has = dy < bl.nty && dx < bl.ntx;
          const uint32_t t = has ? (uint32_t)((bl.ty0 + dy) * (int)c.tiles_x + bl.tx0 + dx) : 0u;
          emit_tile<FILL, CT, RecT>(t, has, nbits, lc, rec, bl);
        }
      }
    }
  }
  return staged;
}

// Pass 1: row u of the [U][tiles] count table.  CT = uint16_t when a unit
// holds at most 65535 points (a point adds at most one pair per tile), which
// halves the LDS per wave and doubles the resident waves.
template <class Src, class CT, bool HL = false>
__global__ __launch_bounds__(BW) void k_bin_count(Src src, Cam c, uint32_t units, int nbits,
                                                  uint32_t *__restrict__ ucount, HlStage hs = HlStage{}) {
  extern __shared__ uint32_t lds_raw[];
  CT *lc = reinterpret_cast<CT *>(lds_raw);
  const uint32_t nt = c.tiles_x * c.tiles_y;
  for (uint32_t i = threadIdx.x; i < nt; i += BW) lc[i] = 0;
  __syncthreads();
  const uint32_t staged =
      bin_unit<Src, false, CT, float3, HL>(src, c, units, blockIdx.x, 1, nbits, lc, (float3 *)nullptr, hs);
  if (HL && threadIdx.x == 0) { hs.count[blockIdx.x] = staged; hs.scan[blockIdx.x] = staged; }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nt; i += BW) ucount[(uint64_t)blockIdx.x * nt + i] = lc[i];
}

// Gather the staged highlighted points into one array in unit order: unit u
// holds count[u] points at [u per, ...) of the staging arrays and goes to
// [off[u], ...) (off = exclusive scan of the counts, off[units] = total).
// At most cap points are kept; more sets the capacity status bit.
__global__ void k_hl_gather(HlStage hs, const uint64_t *__restrict__ off, const uint64_t *__restrict__ n_points,
                            uint64_t max_points, uint32_t units, float *__restrict__ x, float *__restrict__ y,
                            float *__restrict__ z, float *__restrict__ m, uint64_t cap,
                            uint64_t *__restrict__ total, uint64_t *status) {
  const uint64_t n = min(*n_points, max_points);
  const uint64_t per = (n + units - 1) / units;
  const uint32_t u = blockIdx.x;
  const uint64_t b = (uint64_t)u * per, o = off[u], k = hs.count[u];
  for (uint64_t j = threadIdx.x; j < k && o + j < cap; j += blockDim.x) {
    x[o + j] = hs.x[b + j]; y[o + j] = hs.y[b + j]; z[o + j] = hs.z[b + j]; m[o + j] = hs.m[b + j];
  }
  if (u == 0 && threadIdx.x == 0) {
    const uint64_t tot = off[units];
    *total = min(tot, cap);
    if (tot > cap) atomicOr((unsigned long long *)status, (unsigned long long)LOD_STATUS_CAPACITY);
  }
}

// Highlight flags of the stored points: bit s of flags (uint32 words) is set
// when the id of stored point s has its bit in the id bitset (ids >= n_bits
// are not selected).  One wave codes 64 consecutive points, two words.
__global__ void k_hl_flags(const lod_tree t, const uint32_t *__restrict__ bits, uint64_t n_bits,
                           uint64_t cap_points, uint32_t *__restrict__ flags) {
  const uint64_t np = min(t.counts[1], cap_points);
  const uint64_t nwords = (n_bits + 31) >> 5;
  const uint64_t nw = (cap_points + 63) >> 6;     // wave groups of 64 points
  const int lane = threadIdx.x & (WAVE - 1);
  for (uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; g < nw;
       g += ((uint64_t)gridDim.x * blockDim.x) >> 6) {
    const uint64_t sidx = g * 64 + lane;
    bool on = false;
    if (sidx < np) {
      const uint32_t id = t.pt_id[sidx];
      const uint32_t w = bits[min((uint64_t)(id >> 5), nwords - 1)];
      on = (uint64_t)id < n_bits && ((w >> (id & 31u)) & 1u);
    }
    const uint64_t mask = __ballot(on);
    if (lane == 0) reinterpret_cast<uint2 *>(flags)[g] = make_uint2((uint32_t)mask, (uint32_t)(mask >> 32));
  }
}

// Column scans of the count table: exclusive prefix over the 64 units of each
// chunk (in place) and the chunk totals.
__global__ void k_bin_colscan(uint32_t *__restrict__ ucount, uint32_t nt, uint32_t *__restrict__ pchunk) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t ch = blockIdx.y;
  if (t >= nt) return;
  uint32_t run = 0;
  for (uint32_t u = ch * 64; u < ch * 64 + 64; ++u) {
    const uint64_t i = (uint64_t)u * nt + t;
    const uint32_t v = ucount[i];
    ucount[i] = run;
    run += v;
  }
  pchunk[(uint64_t)ch * nt + t] = run;
}

// exclusive prefix over chunks (in place) and the tile totals
__global__ void k_bin_chunkscan(uint32_t *__restrict__ pchunk, uint32_t nt, uint32_t chunks,
                                uint32_t *__restrict__ tile_count) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  uint32_t run = 0;
  for (uint32_t ch = 0; ch < chunks; ++ch) {
    const uint64_t i = (uint64_t)ch * nt + t;
    const uint32_t v = pchunk[i];
    pchunk[i] = run;
    run += v;
  }
  tile_count[t] = run;
}

// Pass 2: write the (u, v, m) records.  Block f covers the g consecutive
// units f g .. f g + g - 1 (a tile's list holds their pairs in unit order, so
// one cursor per tile carries over from one unit to the next); its cursor for
// tile t starts at tile_off[t] + (pairs of earlier chunks) + (pairs of earlier
// units in its chunk).  The pair count (tile_off[nt]) is checked against the
// record capacity once: past it nothing is written and the status word says
// so.
template <class Src, class RecT>
__global__ __launch_bounds__(BW) void k_bin_fill(Src src, Cam c, uint32_t units, uint32_t g, int nbits,
                                                 const uint32_t *__restrict__ ucount,
                                                 const uint32_t *__restrict__ pchunk,
                                                 const uint32_t *__restrict__ tile_off,
                                                 RecT *__restrict__ rec, uint64_t max_pairs, uint64_t *status) {
  extern __shared__ uint32_t lc[];
  const uint32_t nt = c.tiles_x * c.tiles_y;
  if (tile_off[nt] > max_pairs) {
    if (threadIdx.x == 0) atomicOr((unsigned long long *)status, (unsigned long long)LOD_STATUS_CAPACITY);
    return;
  }
  const uint32_t u0 = blockIdx.x * g;
  const uint32_t ch = u0 / 64;
  for (uint32_t i = threadIdx.x; i < nt; i += BW)
    lc[i] = tile_off[i] + pchunk[(uint64_t)ch * nt + i] + ucount[(uint64_t)u0 * nt + i];
  __syncthreads();
  bin_unit<Src, true, uint32_t, RecT>(src, c, units, u0, g, nbits, lc, rec);
}

// slices per tile
__global__ void k_slice_count(const uint32_t *__restrict__ tile_count, uint32_t nt, uint32_t *__restrict__ ns) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x)
    ns[t] = (tile_count[t] + lodh::SPLAT_SLICE - 1) / lodh::SPLAT_SLICE;
}

// Slice descriptors: (first pair, tile | pairs << 16), one per slice.
__global__ void k_slice_table(const uint32_t *__restrict__ tile_off, const uint32_t *__restrict__ tile_count,
                              const uint32_t *__restrict__ slice_off, uint32_t nt, uint2 *__restrict__ table,
                              uint64_t max_slices) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
    const uint32_t b = slice_off[t], e = slice_off[t + 1], c = tile_count[t];
    for (uint32_t k = 0; b + k < e && b + k < max_slices; ++k) {
      const uint32_t n = min(c - k * lodh::SPLAT_SLICE, lodh::SPLAT_SLICE);
      table[b + k] = make_uint2(tile_off[t] + k * lodh::SPLAT_SLICE, t | (n << 16));
    }
  }
}

__device__ __forceinline__ void neumaier(float &s, float &c, float x) {
  const float t = s + x;
  if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// --- accumulation --------------------------------------------------------------

// One block per slice.  The blob is separable, so a chunk of 256 points adds
// Gy^T Gx to the 16x16 tile, with Gx[k][i] = exp(-ox^2/2s^2) and Gy[k][j] =
// m norm exp(-oy^2/2s^2) inside point k's truncation square and 0 outside.
// Phase A: thread k fills row k of Gx and Gy in LDS.  Phase B: wave g
// contracts its own points 64g..64g+63 on the matrix cores (MFMA 16x16x4,
// float32), each lane ending with 4 pixels of one column, and folds them
// (at most 64 products each) into its compensated (Neumaier) float32 sums.
// A wave reads only the rows its own lanes wrote, and LDS operations of one
// wave complete in order, so the waves of a block run the chunks without
// block barriers; at the end of the slice the four wave sums of each pixel
// are folded in wave order.  No atomics: the image is bit-reproducible.
// Pair record loads (the attribute of records that carry none is 0).
__device__ __forceinline__ void load_rec(const float3 *r, uint64_t q, float &u, float &v, float &m, float &a) {
  const float3 t = r[q];
  u = t.x; v = t.y; m = t.z; a = 0.0f;
}
__device__ __forceinline__ void load_rec(const RecGA *r, uint64_t q, float &u, float &v, float &m, float &a) {
  const float4 t = reinterpret_cast<const float4 *>(r)[q];
  u = t.x; v = t.y; m = t.z; a = t.w;
}

constexpr int GXS = TS + 1;          // padded row: conflict-free phase-A writes
typedef float float4v __attribute__((ext_vector_type(4)));
template <class RecT>
__global__ __launch_bounds__(PT) void k_accumulate(const uint2 *__restrict__ table,
                                                   const uint32_t *__restrict__ slice_off, uint32_t nt,
                                                   const RecT *__restrict__ rec, Cam c,
                                                   float *__restrict__ partial, float *__restrict__ partial_aux,
                                                   uint64_t max_slices, uint64_t max_pairs) {
  constexpr bool AUX = RecInfo<RecT>::aux;
  constexpr int PA = AUX ? PT : 1;
  __shared__ float gx[PT][GXS];
  __shared__ float gy[PT][GXS];
  __shared__ float gya[PA][GXS];        // attribute channel: rows weighted by m a
  __shared__ float part[4][TS * TS];   // the waves' slice sums
  __shared__ float parta[AUX ? 4 : 1][AUX ? TS * TS : 1];
  const uint32_t total_slices = (uint32_t)min((uint64_t)slice_off[nt], max_slices);
  const int grp = threadIdx.x / 64;                 // point group of phase B
  const int col = threadIdx.x % TS;                 // pixel column of phase B
  const int row0 = ((threadIdx.x % 64) / TS) * 4;   // first of 4 pixel rows of phase B
  if (blockIdx.x >= total_slices) return;
  // Each thread owns rows threadIdx.x of gx and gy for the whole launch.  In
  // the narrow case they start at zero and each chunk clears only the
  // previous chunk's 8-wide windows before writing its own.
  int pwx = 0, pwy = 0;
  if (c.narrow) {
#pragma unroll
    for (int e = 0; e < TS; ++e) {
      gx[threadIdx.x][e] = 0.0f; gy[threadIdx.x][e] = 0.0f;
      if (AUX) gya[threadIdx.x][e] = 0.0f;
    }
  }
  // pair records are loaded one chunk ahead, across slice boundaries too
  // (clamped indices: every load is issued unconditionally)
  const uint64_t last = max_pairs - 1;
  uint2 sd = table[blockIdx.x];
  float nu, nv, nm, na = 0.0f;
  {
    const uint64_t q = min((uint64_t)sd.x + threadIdx.x, last);
    load_rec(rec, q, nu, nv, nm, na);
  }
  for (uint32_t sl = blockIdx.x; sl < total_slices; sl += gridDim.x) {
    const uint32_t t = sd.y & 0xFFFFu;
    const uint64_t pb = sd.x;
    const uint64_t pe = min(pb + (sd.y >> 16), max_pairs);
    const uint32_t nsl = sl + gridDim.x;
    const uint2 nsd = table[min(nsl, total_slices - 1)];
    const int tx0 = (int)(t % c.tiles_x) * TS, ty0 = (int)(t / c.tiles_x) * TS;
    float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f}, c4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float s4a[4] = {0.0f, 0.0f, 0.0f, 0.0f}, c4a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint64_t c0 = pb; c0 < pe; c0 += PT) {
      const bool have = c0 + threadIdx.x < pe;
      // lanes past the slice hold whatever the clamped prefetch read: zero them
      // so that the 0/1 masking below multiplies finite values only
      const float u = have ? nu : 0.0f, v = have ? nv : 0.0f, m = have ? nm : 0.0f;
      const float pa = have ? na : 0.0f;
      {
        const uint64_t q = (c0 + PT < pe) ? c0 + PT + threadIdx.x : (uint64_t)nsd.x + threadIdx.x;
        const uint64_t qc = min(q, last);
        load_rec(rec, qc, nu, nv, nm, na);
      }
      // phase A: rows are zero outside the truncation square.  A pixel is
      // covered when its float32 offset fl(t - (i + 1/2)) lies in [-R, R],
      // tested pixel by pixel (the covered pixels of an axis form one run).
      // Pixels past the image edge are computed and dropped by the final sum.
      // The Gaussian factor is the hardware exp2 of o^2 (-log2 e / 2 sigma^2)
      // (relative error ~3e-7, ample for 1e-5); lanes past the slice carry
      // mass 0.
      const float R = c.R;
      const float w = m * c.norm;
      const float wa = (m * pa) * c.norm;
      if (c.narrow) {
        // fewer than 8 covered pixels per axis: clear the previous window,
        // then write an 8-wide window from a lower bound of the run's first
        // pixel (float32 offsets are within 1/100 pixel of the exact ones);
        // the rest of the row is still zero
        const int lx = (int)ceilf(u - 0.5f - R - 0.01f), ly = (int)ceilf(v - 0.5f - R - 0.01f);
        const int wx = min(max(lx - tx0, 0), TS - 8), wy = min(max(ly - ty0, 0), TS - 8);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          gx[threadIdx.x][pwx + e] = 0.0f; gy[threadIdx.x][pwy + e] = 0.0f;
          if (AUX) gya[threadIdx.x][pwy + e] = 0.0f;
        }
        pwx = wx; pwy = wy;
        // pixel centres i + 1/2 are small half-integers: adding q to the
        // first one is exact.  Away from the image's low edges (tile origin
        // >= 48, so t > 32) t - c0 and then each - q are exact too (all are
        // multiples of ulp(t) below 16 in magnitude), which saves an add per
        // pixel and gives the same bits.
        const float cx0 = (float)(tx0 + wx) + 0.5f, cy0 = (float)(ty0 + wy) + 0.5f;
        float oxs[8], oys[8];
        if (tx0 >= 48) {
          const float dx = u - cx0;
#pragma unroll
          for (int q = 0; q < 8; ++q) oxs[q] = dx - (float)q;
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) oxs[q] = u - (cx0 + (float)q);
        }
        if (ty0 >= 48) {
          const float dy = v - cy0;
#pragma unroll
          for (int q = 0; q < 8; ++q) oys[q] = dy - (float)q;
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) oys[q] = v - (cy0 + (float)q);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float ox = oxs[q], oy = oys[q];
          // exp2 of a non-positive finite argument lies in [0, 1]
          const float ex = __builtin_amdgcn_exp2f((ox * ox) * c.kexp2);
          const float ey = __builtin_amdgcn_exp2f((oy * oy) * c.kexp2);
          gx[threadIdx.x][wx + q] = fabsf(ox) <= R ? ex : 0.0f;
          gy[threadIdx.x][wy + q] = fabsf(oy) <= R ? w * ey : 0.0f;
          if (AUX) gya[threadIdx.x][wy + q] = fabsf(oy) <= R ? wa * ey : 0.0f;
        }
      } else {
        const float cx0 = (float)tx0 + 0.5f, cy0 = (float)ty0 + 0.5f;
#pragma unroll
        for (int e = 0; e < TS; ++e) {
          const float ox = u - (cx0 + (float)e);
          const float oy = v - (cy0 + (float)e);
          const float ex = __builtin_amdgcn_exp2f((ox * ox) * c.kexp2);
          const float ey = __builtin_amdgcn_exp2f((oy * oy) * c.kexp2);
          gx[threadIdx.x][e] = fabsf(ox) <= R ? ex : 0.0f;
          gy[threadIdx.x][e] = fabsf(oy) <= R ? w * ey : 0.0f;
          if (AUX) gya[threadIdx.x][e] = fabsf(oy) <= R ? wa * ey : 0.0f;
        }
      }
      // the rows of this wave's points were written by this wave
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // phase B: wave g accumulates points 64g..64g+63 with 16 MFMA steps of
      // 16x16x4 (float32); lane l feeds A[l%16][l/16] = Gy[k][row] and
      // B[l/16][l%16] = Gx[k][col] and receives rows 4(l/16)..+3 of column l%16
      const int kb = grp * 64;
      const int ln = threadIdx.x % 64;
      float4v acc4 = {0.0f, 0.0f, 0.0f, 0.0f};
      float av[16], bv[16];   // all LDS operands first: one wait, not sixteen
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const int kk = kb + st * 4 + ln / 16;
        av[st] = gy[kk][ln % 16];
        bv[st] = gx[kk][ln % 16];
      }
      __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
#pragma unroll
      for (int st = 0; st < 16; ++st) acc4 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[st], bv[st], acc4, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) neumaier(s4[i], c4[i], acc4[i]);
      if (AUX) {
        float4v acc4a = {0.0f, 0.0f, 0.0f, 0.0f};
        float aa[16];
#pragma unroll
        for (int st = 0; st < 16; ++st) aa[st] = gya[kb + st * 4 + ln / 16][ln % 16];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int st = 0; st < 16; ++st)
          acc4a = __builtin_amdgcn_mfma_f32_16x16x4f32(aa[st], bv[st], acc4a, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) neumaier(s4a[i], c4a[i], acc4a[i]);
      }
      // the next chunk rewrites this wave's rows after its reads above
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) part[grp][(row0 + i) * TS + col] = s4[i] + c4[i];
    if (AUX) {
#pragma unroll
      for (int i = 0; i < 4; ++i) parta[grp][(row0 + i) * TS + col] = s4a[i] + c4a[i];
    }
    __syncthreads();
    float s = 0.0f, cc = 0.0f;
#pragma unroll
    for (int g = 0; g < 4; ++g) neumaier(s, cc, part[g][threadIdx.x]);
    partial[(uint64_t)sl * (TS * TS) + threadIdx.x] = s + cc;
    if (AUX) {
      float sa = 0.0f, ca = 0.0f;
#pragma unroll
      for (int g = 0; g < 4; ++g) neumaier(sa, ca, parta[g][threadIdx.x]);
      partial_aux[(uint64_t)sl * (TS * TS) + threadIdx.x] = sa + ca;
    }
    sd = nsd;
    __syncthreads();
  }
}

// Sum each tile's slice partials in slice order and write the image.
__global__ __launch_bounds__(PT) void k_finalize(const uint32_t *__restrict__ slice_off, uint32_t nt,
                                                 const float *__restrict__ partial, Cam c,
                                                 float *__restrict__ image, uint64_t max_slices) {
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const uint32_t b = slice_off[t], e = slice_off[t + 1];
    float s = 0.0f, cc = 0.0f;
    for (uint32_t sl = b; sl < e && sl < max_slices; ++sl) neumaier(s, cc, partial[(uint64_t)sl * (TS * TS) + threadIdx.x]);
    const int i = (int)(t % c.tiles_x) * TS + (threadIdx.x % TS);
    const int j = (int)(t / c.tiles_x) * TS + (threadIdx.x / TS);
    if (i < (int)c.W && j < (int)c.H) image[(uint64_t)j * c.W + i] = s + cc;
  }
}

// --- radial cubic blob -------------------------------------------------------------
//
// The compact cubic spline of smoothed-particle hydrodynamics, normalised in
// two dimensions: W(r; h) = 40 / (7 pi h^2) w(r / h), w(q) = 1 - 6 q^2 + 6 q^3
// (q <= 1/2), 2 (1 - q)^3 (1/2 < q < 1), 0 beyond.  A pixel takes a point iff
// fl64(ox^2) + fl64(oy^2) < h^2 in float64 (both squares of the float32
// offsets are exact there).  The value is evaluated in float64: near the rim
// w ~ 2 (1 - q)^3 needs 1 - q to far better than float32's relative 6e-8 for
// the pixel's 1e-5 bound, so q = sqrt(r^2) / h is formed in float64 and the
// product m W is rounded once to float32 before the compensated sum.
constexpr double kCubicNorm = 40.0 / (7.0 * 3.14159265358979323846);

__device__ __forceinline__ double cubic_w(double q) {
  return q <= 0.5 ? (1.0 - 6.0 * q * q) + 6.0 * q * q * q : 2.0 * ((1.0 - q) * (1.0 - q)) * (1.0 - q);
}
// w'(q) / q, finite at q = 0
__device__ __forceinline__ double cubic_dw_over_q(double q) {
  return q <= 0.5 ? -12.0 + 18.0 * q : -6.0 * ((1.0 - q) * (1.0 - q)) / q;
}

__device__ __forceinline__ void load_rec(const RecC *r, uint64_t q, float &u, float &v, float &m, float &h,
                                         float &a) {
  const float4 t = reinterpret_cast<const float4 *>(r)[q];
  u = t.x; v = t.y; m = t.z; h = t.w; a = 0.0f;
}
__device__ __forceinline__ void load_rec(const RecCA *r, uint64_t q, float &u, float &v, float &m, float &h,
                                         float &a) {
  const RecCA t = r[q];
  u = t.u; v = t.v; m = t.m; h = t.h; a = t.a;
}

// One block per slice (as the Gaussian accumulation); the spline is not
// separable, so thread p owns pixel p of the 16x16 tile and gathers.  The
// slice's records are staged in LDS 256 at a time (u, v, h, m as one 16-byte
// entry, 1/h in float64 beside it); each wave runs through them in order and
// skips a record whose blob misses its four pixel rows (a wave-uniform test),
// so every pixel adds its contributions in record order: the image is
// bit-reproducible.  Covered pixels form q = r / h from a float64 reciprocal
// square root with one Newton step (relative error far below 1e-12).
template <class RecT>
__global__ __launch_bounds__(PT) void k_accumulate_cubic(const uint2 *__restrict__ table,
                                                         const uint32_t *__restrict__ slice_off, uint32_t nt,
                                                         const RecT *__restrict__ rec, Cam c,
                                                         float *__restrict__ partial,
                                                         float *__restrict__ partial_aux, uint64_t max_slices,
                                                         uint64_t max_pairs) {
  constexpr bool AUX = RecInfo<RecT>::aux;
  __shared__ float4 sr[PT];           // u, v, h, m
  __shared__ double sih[PT];          // 1 / h
  __shared__ float sa[AUX ? PT : 1];
  const uint32_t total_slices = (uint32_t)min((uint64_t)slice_off[nt], max_slices);
  if (blockIdx.x >= total_slices) return;
  const int px = threadIdx.x % TS, py = threadIdx.x / TS;
  const int wrow0 = (threadIdx.x / WAVE) * 4;      // a wave's first pixel row within the tile
  for (uint32_t sl = blockIdx.x; sl < total_slices; sl += gridDim.x) {
    const uint2 sd = table[sl];
    const uint32_t t = sd.y & 0xFFFFu;
    const uint64_t pb = sd.x;
    const uint64_t pe = min(pb + (sd.y >> 16), max_pairs);
    const int tx0 = (int)(t % c.tiles_x) * TS, ty0 = (int)(t / c.tiles_x) * TS;
    const float cx = (float)(tx0 + px) + 0.5f, cy = (float)(ty0 + py) + 0.5f;   // exact pixel centres
    const float rlo = (float)(ty0 + wrow0) + 0.5f, rhi = rlo + 3.0f;
    float s = 0.0f, cs = 0.0f, s_a = 0.0f, c_a = 0.0f;
    for (uint64_t c0 = pb; c0 < pe; c0 += PT) {
      __syncthreads();                               // the previous chunk has been read
      if (c0 + threadIdx.x < pe) {
        float u, v, m, h, a;
        load_rec(rec, c0 + threadIdx.x, u, v, m, h, a);
        sr[threadIdx.x] = make_float4(u, v, h, m);
        sih[threadIdx.x] = 1.0 / (double)h;
        if (AUX) sa[threadIdx.x] = a;
      }
      __syncthreads();
      const int nrec = (int)min((uint64_t)PT, pe - c0);
      for (int k = 0; k < nrec; ++k) {
        const float4 r = sr[k];
        const float u = r.x, v = r.y, h = r.z;
        // the blob covers |oy| < h: skip when it misses all four row centres
        if (v + h + 0.01f < rlo || v - h - 0.01f > rhi) continue;
        const float ox = u - cx, oy = v - cy;
        const float r2f = ox * ox + oy * oy;
        if (!(r2f < (h * h) * 1.001f)) continue;   // surely outside (float32 pre-test with margin)
        const double h64 = (double)h;
        const double hh = h64 * h64;
        const double r2 = (double)ox * (double)ox + (double)oy * (double)oy;
        if (!(r2 < hh)) continue;
        double q = 0.0;
        if (r2 > 0.0) {
          double y = __builtin_amdgcn_rsq(r2);
          y = y * (1.5 - (0.5 * r2) * (y * y));     // one Newton step
          q = (r2 * y) * sih[k];
        }
        const double val = (double)r.w * (kCubicNorm / hh) * cubic_w(q);
        neumaier(s, cs, (float)val);
        if (AUX) neumaier(s_a, c_a, (float)(val * (double)sa[k]));
      }
    }
    partial[(uint64_t)sl * (TS * TS) + threadIdx.x] = s + cs;
    if (AUX) partial_aux[(uint64_t)sl * (TS * TS) + threadIdx.x] = s_a + c_a;
  }
}

// The same sums for narrow blobs: every pixel radius below 1.9 (WIN = 4) or
// 3.9 (WIN = 8) pixels, so that a blob covers only pixels of the WIN x WIN
// window that starts at its first admitted pixel (the binning's conservative
// range: its first pixel, and at most WIN - 1 more, since 2 (h + 1/100)
// plus the float32 rounding of the range stays below WIN).  The gather form
// spends a wave's 64 lanes on one record, of which a handful are covered;
// here the work is split in two phases per chunk of CH records:
//   A: every lane evaluates one record at IPT window pixels (all lanes busy),
//      leaves the rounded contributions in LDS and, for each covered pixel
//      of the tile, sets the record's bit in that pixel's mask;
//   B: thread p owns pixel p of the tile as before and walks the set bits of
//      its mask in increasing record order, adding those contributions.
// The contributions are computed by the same float32 / float64 operations as
// in k_accumulate_cubic and every pixel adds the same ones in the same
// order: the image is bit-identical to the gather form's.
template <int WIN> struct CubicWin {
  static constexpr int WW = WIN * WIN;           // window pixels per record
  static constexpr int CH = WIN == 4 ? PT : 64;  // records per chunk
  static constexpr int IPT = WW * CH / PT;       // window pixels per thread in phase A
  static constexpr int VS = CH + 1;              // LDS stride of one window pixel's row
  static constexpr int MW = CH / 32;             // mask words per pixel
};

template <class RecT, int WIN>
__global__ __launch_bounds__(PT) void k_accumulate_cubic_win(const uint2 *__restrict__ table,
                                                             const uint32_t *__restrict__ slice_off, uint32_t nt,
                                                             const RecT *__restrict__ rec, Cam c,
                                                             float *__restrict__ partial,
                                                             float *__restrict__ partial_aux, uint64_t max_slices,
                                                             uint64_t max_pairs) {
  constexpr bool AUX = RecInfo<RecT>::aux;
  using CW = CubicWin<WIN>;
  constexpr int CH = CW::CH, IPT = CW::IPT, VS = CW::VS, MW = CW::MW;
  static_assert(IPT * PT == CW::WW * CH && CH % 32 == 0 && PT == TS * TS, "phase A covers every window pixel once");
  __shared__ float val[CW::WW * VS];             // [window pixel][record]
  __shared__ float vala[AUX ? CW::WW * VS : 1];
  __shared__ uint32_t org[CH];                   // window origin in the tile: x0 | y0 << 16 (int16 each)
  __shared__ uint32_t msk[MW * PT];              // [record / 32][pixel]: bit of each covering record
  const uint32_t total_slices = (uint32_t)min((uint64_t)slice_off[nt], max_slices);
  if (blockIdx.x >= total_slices) return;
  const int px = threadIdx.x % TS, py = threadIdx.x / TS;
  const int kA = threadIdx.x % CH;                 // phase A: this thread's record in the chunk
  const int iA = (threadIdx.x / CH) * IPT;         // and its first window pixel
  // phase B leaves each pixel's mask words cleared for the next chunk
#pragma unroll
  for (int wd = 0; wd < MW; ++wd) msk[wd * PT + threadIdx.x] = 0u;
  __syncthreads();
  for (uint32_t sl = blockIdx.x; sl < total_slices; sl += gridDim.x) {
    const uint2 sd = table[sl];
    const uint32_t t = sd.y & 0xFFFFu;
    const uint64_t pb = sd.x;
    const uint64_t pe = min(pb + (sd.y >> 16), max_pairs);
    const int tx0 = (int)(t % c.tiles_x) * TS, ty0 = (int)(t / c.tiles_x) * TS;
    float s = 0.0f, cs = 0.0f, s_a = 0.0f, c_a = 0.0f;
    for (uint64_t c0 = pb; c0 < pe; c0 += CH) {
      const int nrec = (int)min((uint64_t)CH, pe - c0);
      // phase A
      {
        const bool have = kA < nrec;
        float u, v, m, h, a;
        load_rec(rec, have ? c0 + kA : pb, u, v, m, h, a);
        const int lx = (int)ceilf(u - 0.5f - h - 0.01f), ly = (int)ceilf(v - 0.5f - h - 0.01f);
        const int x0 = lx - tx0, y0 = ly - ty0;
        if (iA == 0) org[kA] = ((uint32_t)x0 & 0xFFFFu) | ((uint32_t)y0 << 16);
        const double h64 = (double)h;
        const double hh = h64 * h64;
        const double ih = 1.0 / h64;
        const float hh32 = (h * h) * 1.001f;
        const uint32_t bit = 1u << (kA & 31);
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
          const int wi = iA + e;
          const int tpx = x0 + wi % WIN, tpy = y0 + wi / WIN;   // the pixel in the tile
          const float cx = (float)(lx + wi % WIN) + 0.5f, cy = (float)(ly + wi / WIN) + 0.5f;
          const float ox = u - cx, oy = v - cy;
          float vf = 0.0f, va = 0.0f;
          if (have && (ox * ox + oy * oy) < hh32) {
            const double r2 = (double)ox * (double)ox + (double)oy * (double)oy;
            if (r2 < hh) {
              double q = 0.0;
              if (r2 > 0.0) {
                double y = __builtin_amdgcn_rsq(r2);
                y = y * (1.5 - (0.5 * r2) * (y * y));
                q = (r2 * y) * ih;
              }
              const double w = (double)m * (kCubicNorm / hh) * cubic_w(q);
              vf = (float)w;
              if (AUX) va = (float)(w * (double)a);
              if ((unsigned)tpx < (unsigned)TS && (unsigned)tpy < (unsigned)TS)
                atomicOr(&msk[(kA >> 5) * PT + tpy * TS + tpx], bit);
            }
          }
          val[wi * VS + kA] = vf;
          if (AUX) vala[wi * VS + kA] = va;
        }
      }
      __syncthreads();
      // phase B: this pixel's covering records in increasing order
#pragma unroll
      for (int wd = 0; wd < MW; ++wd) {
        uint32_t bits = msk[wd * PT + threadIdx.x];
        msk[wd * PT + threadIdx.x] = 0u;
        while (bits) {
          const int k = wd * 32 + __builtin_ctz(bits);
          bits &= bits - 1u;
          const uint32_t o = org[k];
          const int dx = px - (int)(int16_t)(o & 0xFFFFu), dy = py - (int)(int16_t)(o >> 16);
          const int vi = (dy * WIN + dx) * VS + k;
          neumaier(s, cs, val[vi]);
          if (AUX) neumaier(s_a, c_a, vala[vi]);
        }
      }
      __syncthreads();
    }
    partial[(uint64_t)sl * (TS * TS) + threadIdx.x] = s + cs;
    if (AUX) partial_aux[(uint64_t)sl * (TS * TS) + threadIdx.x] = s_a + c_a;
  }
}

// Adjoint of the cubic blob, one thread per point over its own footprint
// (float64 sums): dI/dm = W, dI/dox = m 40/(7 pi h^4) (w'(q)/q) ox, and with a
// world-space size (radius not clamped) dI/dh = m 40/(7 pi h^3)
// (-2 w - q w'(q)) with dh/dp = -(h / zc) f.
__global__ __launch_bounds__(PT) void k_backward_cubic(const float *__restrict__ x, const float *__restrict__ y,
                                                       const float *__restrict__ z, const float *__restrict__ m,
                                                       uint64_t count, Cam c, const float *__restrict__ g,
                                                       float *__restrict__ gm, float *__restrict__ gx,
                                                       float *__restrict__ gy, float *__restrict__ gz) {
  for (uint64_t k = (uint64_t)blockIdx.x * PT + threadIdx.x; k < count; k += (uint64_t)gridDim.x * PT) {
    float u, v, xc, yc, zc;
    double am = 0.0, au = 0.0, av = 0.0, ah = 0.0;
    const bool vis = project(c, x[k], y[k], z[k], u, v, xc, yc, zc);
    const float h = vis ? cubic_radius(c, zc) : c.hpx;
    bool dh_live = false;
    if (vis && c.Fhw > 0.0f) {
      const float hp = __fdiv_rn(c.Fhw, zc);
      dh_live = hp >= lodh::BLOB_H_MIN && hp <= lodh::BLOB_H_MAX;
    }
    int i0, i1, j0, j1;
    const double mk = (double)m[k];
    if (vis && cover_range(h, u, c.W, i0, i1) && cover_range(h, v, c.H, j0, j1)) {
      const double h64 = (double)h, hh = h64 * h64;
      for (int j = j0; j <= j1; ++j) {
        const float oy = v - ((float)j + 0.5f);
        for (int i = i0; i <= i1; ++i) {
          const float ox = u - ((float)i + 0.5f);
          const double r2 = (double)ox * (double)ox + (double)oy * (double)oy;
          if (!(r2 < hh)) continue;
          const double q = sqrt(r2) / h64;
          const double w = cubic_w(q), dwq = cubic_dw_over_q(q);
          const double gp = (double)g[(uint64_t)j * c.W + i];
          am += (kCubicNorm / hh) * w * gp;
          const double tq = mk * kCubicNorm / (hh * hh) * dwq * gp;
          au += tq * (double)ox;
          av += tq * (double)oy;
          if (dh_live) ah += mk * kCubicNorm / (hh * h64) * (-2.0 * w - (q * q) * dwq) * gp;
        }
      }
    }
    double dx = 0.0, dy = 0.0, dz = 0.0;
    if (vis) {
      if (c.proj == 0) {
        dx = au * (double)c.W;
        dy = av * (double)c.H;
      } else {
        const double zz = (double)zc;
        const double a = (double)c.F / zz;
        const double bu = (double)c.F * (double)xc / (zz * zz);
        const double bv = (double)c.F * (double)yc / (zz * zz);
        const double dh = dh_live ? -(double)h / zz : 0.0;
        dx = au * (a * c.rx - bu * c.fx) + av * (a * c.ux - bv * c.fx) + ah * dh * c.fx;
        dy = au * (a * c.ry - bu * c.fy) + av * (a * c.uy - bv * c.fy) + ah * dh * c.fy;
        dz = au * (a * c.rz - bu * c.fz) + av * (a * c.uz - bv * c.fz) + ah * dh * c.fz;
      }
    }
    gm[k] = (float)am;
    if (gx) gx[k] = (float)dx;
    if (gy) gy[k] = (float)dy;
    if (gz) gz[k] = (float)dz;
  }
}

// --- adjoint -------------------------------------------------------------------

__global__ __launch_bounds__(PT) void k_backward(const float *__restrict__ x, const float *__restrict__ y,
                                                 const float *__restrict__ z, const float *__restrict__ m,
                                                 uint64_t count, Cam c, const float *__restrict__ g,
                                                 float *__restrict__ gm, float *__restrict__ gx,
                                                 float *__restrict__ gy, float *__restrict__ gz) {
  for (uint64_t k = (uint64_t)blockIdx.x * PT + threadIdx.x; k < count; k += (uint64_t)gridDim.x * PT) {
    float u, v, xc, yc, zc;
    float am = 0.0f, au = 0.0f, av = 0.0f;
    const bool vis = project(c, x[k], y[k], z[k], u, v, xc, yc, zc);
    int i0, i1, j0, j1;
    if (vis && axis_range(c, u, c.W, i0, i1) && axis_range(c, v, c.H, j0, j1)) {
      for (int j = j0; j <= j1; ++j) {
        const float oy = v - ((float)j + 0.5f);
        const float ey = c.norm * expf(-(oy * oy) * c.inv2s2);
        float rm = 0.0f, ru = 0.0f, rv = 0.0f;
        for (int i = i0; i <= i1; ++i) {
          const float ox = u - ((float)i + 0.5f);
          const float G = ey * expf(-(ox * ox) * c.inv2s2);
          const float gg = G * g[(uint64_t)j * c.W + i];
          rm += gg;
          ru -= gg * ox;
          rv -= gg * oy;
        }
        am += rm; au += ru; av += rv;
      }
    }
    const float mk = m[k];
    const float du = mk * au * c.inv_s2, dv = mk * av * c.inv_s2;
    float dx = 0.0f, dy = 0.0f, dz = 0.0f;
    if (vis) {
      if (c.proj == 0) {
        dx = du * (float)c.W;
        dy = dv * (float)c.H;
      } else {
        const float a = c.F / zc;
        const float bu = c.F * xc / (zc * zc);
        const float bv = c.F * yc / (zc * zc);
        dx = du * (a * c.rx - bu * c.fx) + dv * (a * c.ux - bv * c.fx);
        dy = du * (a * c.ry - bu * c.fy) + dv * (a * c.uy - bv * c.fy);
        dz = du * (a * c.rz - bu * c.fz) + dv * (a * c.uz - bv * c.fz);
      }
    }
    gm[k] = am;
    if (gx) gx[k] = dx;
    if (gy) gy[k] = dy;
    if (gz) gz[k] = dz;
  }
}

// --- motion codes ----------------------------------------------------------------

// Motion code of one coordinate: the particle's position a in the next
// snapshot against the stored code Q0 = (c << 16) + q at depth d,
// dq = floor((floor(a 2^(d+16)) - Q0 + 2) / 4) clamped to int16 (true when clamped).
__device__ __forceinline__ int16_t motion_code(float a, uint32_t c, uint32_t q, int d, bool &sat) {
  const int64_t Q1 = (int64_t)floorf(a * ldexpf(1.0f, d + 16));
  const int64_t Q0 = ((int64_t)c << 16) + (int64_t)q;
  const int64_t dq = (Q1 - Q0 + 2) >> 2;          // arithmetic shift: floor division by 4
  sat = dq < -32768 || dq > 32767;
  return (int16_t)max((int64_t)-32768, min((int64_t)32767, dq));
}

// One block per node (grid-stride over the node table); thread j codes the
// node's stored points j, j + blockDim, ...  The next snapshot's positions
// are indexed like the build input: snapshot offset + particle id.
__global__ void k_encode_motion(const lod_tree t, const float *__restrict__ xb, const float *__restrict__ yb,
                                const float *__restrict__ zb, const uint64_t *__restrict__ snap_off,
                                uint64_t cap_nodes, int16_t *__restrict__ dqx, int16_t *__restrict__ dqy,
                                int16_t *__restrict__ dqz, uint64_t *__restrict__ saturated) {
  const uint64_t nn = min(t.counts[0], cap_nodes);
  uint32_t sat_count = 0;
  for (uint64_t v = blockIdx.x; v < nn; v += gridDim.x) {
    const int d = t.depth[v];
    const uint64_t pfx = t.prefix[v];
    const uint32_t cell = d ? (uint32_t)(pfx & ((1ull << (3 * d)) - 1)) : 0u;
    const uint32_t cx = compact3(cell), cy = compact3(cell >> 1), cz = compact3(cell >> 2);
    const uint64_t base = snap_off ? snap_off[pfx >> (3 * d)] : 0ull;
    const uint64_t pb = t.pt_begin[v];
    const uint32_t pc = t.pt_count[v];
    for (uint32_t j = threadIdx.x; j < pc; j += blockDim.x) {
      const uint64_t sidx = pb + j;
      const uint64_t g = base + t.pt_id[sidx];
      bool s0, s1, s2;
      dqx[sidx] = motion_code(xb[g], cx, t.qx[sidx], d, s0);
      dqy[sidx] = motion_code(yb[g], cy, t.qy[sidx], d, s1);
      dqz[sidx] = motion_code(zb[g], cz, t.qz[sidx], d, s2);
      sat_count += (uint32_t)s0 + (uint32_t)s1 + (uint32_t)s2;
    }
  }
  if (sat_count) atomicAdd((unsigned long long *)saturated, (unsigned long long)sat_count);
}

// --- writing a node's points back (refinement) ---------------------------------

// Stored points of node v replaced by count positions and masses (count <=
// the node's pt_count): codes q = min(floor(a 2^(d+16)) - (c << 16), 65535)
// relative to the node's cell (positions outside the cell set the domain
// status bit and are clamped), masses as given.
__global__ void k_set_points(const lod_tree t, uint32_t v, const float *__restrict__ x, const float *__restrict__ y,
                             const float *__restrict__ z, const float *__restrict__ m, uint32_t count) {
  if ((uint64_t)v >= t.counts[0]) return;
  const int d = t.depth[v];
  const uint64_t pfx = t.prefix[v];
  const uint32_t cell = d ? (uint32_t)(pfx & ((1ull << (3 * d)) - 1)) : 0u;
  const uint32_t c3[3] = {compact3(cell), compact3(cell >> 1), compact3(cell >> 2)};
  const uint64_t pb = t.pt_begin[v];
  const uint32_t k = min(count, t.pt_count[v]);
  const float scale = ldexpf(1.0f, d + 16);
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x) {
    const float a[3] = {x[j], y[j], z[j]};
    uint16_t q[3];
    bool out = false;
    for (int ax = 0; ax < 3; ++ax) {
      const int64_t Q = (int64_t)floorf(a[ax] * scale) - ((int64_t)c3[ax] << 16);
      out |= !(Q >= 0 && Q <= 65535 + 1) || !(a[ax] >= 0.0f);
      q[ax] = (uint16_t)max((int64_t)0, min((int64_t)65535, Q));
    }
    if (out) atomicOr((unsigned long long *)&t.counts[2], (unsigned long long)LOD_STATUS_DOMAIN);
    t.qx[pb + j] = q[0]; t.qy[pb + j] = q[1]; t.qz[pb + j] = q[2];
    t.pt_mass[pb + j] = m[j];
  }
}

// --- LOD decode ----------------------------------------------------------------

__global__ void k_lod_counts(const lod_tree t, const uint32_t *__restrict__ ids, const uint64_t *__restrict__ n_ids,
                             uint64_t max_ids, uint64_t *__restrict__ offs) {
  const uint64_t nn = t.counts[0];
  const uint64_t ni = min(*n_ids, max_ids);
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= max_ids;
       k += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t c = 0;
    if (k < ni) {
      const uint32_t v = ids[k];
      if (v < nn) c = t.pt_count[v];
    }
    offs[k] = c;
  }
}

// offs[max_ids] holds the total after the scan.
__global__ void k_lod_total(const lod_tree t, const uint64_t *__restrict__ offs, uint64_t max_ids,
                            uint64_t max_points, uint64_t *__restrict__ total) {
  const uint64_t tot = offs[max_ids];
  *total = min(tot, max_points);
  if (tot > max_points) atomicOr((unsigned long long *)&t.counts[2], (unsigned long long)LOD_STATUS_CAPACITY);
}

__global__ __launch_bounds__(PT) void k_lod_decode(const lod_tree t, const uint32_t *__restrict__ ids,
                                                   const uint64_t *__restrict__ n_ids, uint64_t max_ids,
                                                   const uint64_t *__restrict__ offs, uint64_t max_points,
                                                   float *__restrict__ x, float *__restrict__ y,
                                                   float *__restrict__ z, float *__restrict__ m) {
  const uint64_t nn = t.counts[0];
  const uint64_t ni = min(*n_ids, max_ids);
  for (uint64_t k = blockIdx.x; k < ni; k += gridDim.x) {
    const uint32_t v = ids[k];
    if (v >= nn) continue;
    const int d = t.depth[v];
    const uint64_t pfx = t.prefix[v];
    const uint32_t cell = d ? (uint32_t)(pfx & ((1ull << (3 * d)) - 1)) : 0u;
    const uint32_t cx = compact3(cell), cy = compact3(cell >> 1), cz = compact3(cell >> 2);
    const uint64_t pb = t.pt_begin[v];
    const uint32_t pc = t.pt_count[v];
    const uint64_t ob = offs[k];
    for (uint32_t j = threadIdx.x; j < pc; j += PT) {
      const uint64_t o = ob + j;
      if (o >= max_points) break;
      const uint64_t s = pb + j;
      x[o] = decode_coord(cx, t.qx[s], d);
      y[o] = decode_coord(cy, t.qy[s], d);
      z[o] = decode_coord(cz, t.qz[s], d);
      m[o] = t.pt_mass[s];
    }
  }
}

// --- view-dependent cut ----------------------------------------------------------

struct CutArgs {
  uint32_t proj, W;
  double px, py, pz;
  double F, tau_cbrt;   // tau * n^(1/3)
};

__device__ __forceinline__ bool descends(const lod_tree &t, uint32_t v, const CutArgs &c) {
  if (t.first_child[v] == NONE) return false;
  const int d = t.depth[v];
  const double side = ldexp(1.0, -d);
  if (c.proj == 0) return (double)c.W * side > c.tau_cbrt;
  const uint32_t cell = d ? (uint32_t)(t.prefix[v] & ((1ull << (3 * d)) - 1)) : 0u;
  const double ox = (double)compact3(cell) * side;
  const double oy = (double)compact3(cell >> 1) * side;
  const double oz = (double)compact3(cell >> 2) * side;
  const bool inside = (ox <= c.px && c.px <= ox + side) && (oy <= c.py && c.py <= oy + side) &&
                      (oz <= c.pz && c.pz <= oz + side);
  if (inside) return true;
  const double h = side * 0.5;
  const double dx = (ox + h) - c.px;
  const double dy = (oy + h) - c.py;
  const double dz = (oz + h) - c.pz;
  const double dist = __dsqrt_rn((dx * dx + dy * dy) + dz * dz);
  return c.F * side > c.tau_cbrt * dist;
}

__global__ void k_cut_flags(const lod_tree t, CutArgs c, uint64_t cap_nodes, uint32_t *__restrict__ flag) {
  const uint64_t nn = min(t.counts[0], cap_nodes);
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= cap_nodes;
       v += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t f = 0;
    if (v < nn && !descends(t, (uint32_t)v, c)) {
      f = 1;
      uint32_t u = t.parent[v];
      while (u != NONE) {
        if (!descends(t, u, c)) { f = 0; break; }
        u = t.parent[u];
      }
    }
    flag[v] = f;
  }
}

__global__ void k_cut_write(const lod_tree t, uint64_t cap_nodes, const uint32_t *__restrict__ keep,
                            const uint32_t *__restrict__ scan, uint32_t *__restrict__ ids, uint64_t cap,
                            uint64_t *__restrict__ n_sel) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < cap_nodes;
       v += (uint64_t)gridDim.x * blockDim.x) {
    if (keep[v]) {
      const uint32_t o = scan[v];
      if (o < cap) ids[o] = (uint32_t)v;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint64_t tot = scan[cap_nodes];
    *n_sel = min(tot, cap);
    if (tot > cap) atomicOr((unsigned long long *)&t.counts[2], (unsigned long long)LOD_STATUS_CAPACITY);
  }
}

__global__ void k_copy_u32(const uint32_t *__restrict__ a, uint32_t *__restrict__ b, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

}  // namespace

// -----------------------------------------------------------------------------
// host side

namespace lodh {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Bytes of one binned (point, tile) record for a render form.
static size_t rec_bytes(const splat_params &sp, bool aux) {
  if (sp.blob == LOD_BLOB_CUBIC) return aux ? sizeof(RecCA) : sizeof(RecC);
  return aux ? sizeof(RecGA) : sizeof(float3);
}

lod_status splat_layout(uint64_t max_points, const lod_camera &cam, const splat_params &sp, SplatLayout &L,
                        bool aux) {
  L = SplatLayout{};
  L.tiles_x = (cam.W + TS - 1) / TS;
  L.tiles_y = (cam.H + TS - 1) / TS;
  const uint64_t nt = (uint64_t)L.tiles_x * L.tiles_y;
  if (nt == 0 || nt > SPLAT_MAX_TILES) return LOD_EUNSUPPORTED;
  L.n_tiles = (uint32_t)nt;
  const double R = (double)blob_max_radius(sp);
  const uint64_t width = 2 * (uint64_t)std::ceil(R) + 3;         // pixels a blob's tile range can span
  const uint64_t tpa = std::min<uint64_t>((width + TS - 1) / TS + 1, std::max(L.tiles_x, L.tiles_y));
  L.max_points = max_points;
  // pair counts are 32-bit, and a point adds at least one pair
  if (max_points >= (1ull << 32)) return LOD_EUNSUPPORTED;
  L.max_pairs = std::max<uint64_t>(1, max_points * tpa * tpa);
  if (L.max_pairs >= (1ull << 32)) return LOD_EUNSUPPORTED;
  L.max_slices = nt + L.max_pairs / SPLAT_SLICE + 1;
  L.aux = aux;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  // units: 64 per chunk, one chunk per 2^17 points (units of at most 2048
  // points until the 64-chunk cap: a million points are binned by 512
  // waves; 150 M by 4096 units of at most 36.6 k points)
  L.chunks = (uint32_t)std::min<uint64_t>(SPLAT_MAX_CHUNKS, std::max<uint64_t>(1, (max_points + (1u << 17) - 1) >> 17));
  L.units = 64 * L.chunks;
  L.tile_count = take(4 * (nt + 1));
  L.tile_off = take(4 * (nt + 1));
  L.ucount = take(4 * (size_t)L.units * nt);
  L.pchunk = take(4 * (size_t)L.chunks * nt);
  L.slice_off = take(4 * (nt + 1));
  L.scan_tmp = take(4 * scan_tmp_elems<uint32_t>(nt + 1));
  L.counters = take(64);
  L.rec = take(rec_bytes(sp, aux) * L.max_pairs);
  L.partial = take(4 * (size_t)TS * TS * L.max_slices);
  L.partial_aux = aux ? take(4 * (size_t)TS * TS * L.max_slices) : L.partial;
  L.slice_table = take(8 * (size_t)L.max_slices);
  L.total = off;
  return LOD_OK;
}

// Whether a source carries per-point world radii (the cubic blob's pixel
// radius then varies up to the clamp).
template <class Src> static bool has_point_radii(const Src &) { return false; }
static bool has_point_radii(const InterpSrc &s) { return s.ha != nullptr; }

// Binning, accumulation and the final slice sums for any point source and
// record form.  image_aux receives the attribute channel (RecT carrying one).
template <class Src, class RecT>
static lod_status launch_splat_src(const Src &src, bool any, const lod_camera &cam, const splat_params &sp,
                                   void *ws, const SplatLayout &L, float *image, float *image_aux,
                                   uint64_t *status_word, hipStream_t st, const HlStage *hs = nullptr) {
  char *W = (char *)ws;
  Cam c = make_cam(cam, sp, &L);
  const uint32_t nt = L.n_tiles;
  uint32_t *tcount = (uint32_t *)(W + L.tile_count);
  uint32_t *toff = (uint32_t *)(W + L.tile_off);
  uint32_t *ucount = (uint32_t *)(W + L.ucount);
  uint32_t *pchunk = (uint32_t *)(W + L.pchunk);
  uint32_t *soff = (uint32_t *)(W + L.slice_off);
  uint32_t *stmp = (uint32_t *)(W + L.scan_tmp);
  uint64_t *ctr = (uint64_t *)(W + L.counters);
  uint64_t *status = status_word ? status_word : ctr;
  RecT *rec = (RecT *)(W + L.rec);
  float *partial = (float *)(W + L.partial);
  float *partial_aux = (float *)(W + L.partial_aux);
  int nbits = 0;
  while ((1u << nbits) < nt) ++nbits;
  fill_u32(tcount, nt + 1, 0, st);
  if (!status_word) fill_u64(ctr, 1, 0, st);
  const size_t lds = 4 * (size_t)nt;
  if (any) {
    const bool narrow_counts = (L.max_points + L.units - 1) / L.units <= 65535;
    bool staged = false;
    if constexpr (IsTree<Src>::value) {
      if (hs) {
        staged = true;
        if (narrow_counts)
          LOD_LAUNCH((k_bin_count<Src, uint16_t, true>), dim3(L.units), dim3(BW), 2 * (size_t)nt, st, src, c,
                     L.units, nbits, ucount, *hs);
        else
          LOD_LAUNCH((k_bin_count<Src, uint32_t, true>), dim3(L.units), dim3(BW), lds, st, src, c, L.units, nbits,
                     ucount, *hs);
      }
    }
    if (!staged) {
      if (narrow_counts)
        LOD_LAUNCH((k_bin_count<Src, uint16_t>), dim3(L.units), dim3(BW), 2 * (size_t)nt, st, src, c, L.units,
                   nbits, ucount, HlStage{});
      else
        LOD_LAUNCH((k_bin_count<Src, uint32_t>), dim3(L.units), dim3(BW), lds, st, src, c, L.units, nbits, ucount,
                   HlStage{});
    }
    LOD_LAUNCH(k_bin_colscan, dim3((nt + 255) / 256, L.chunks), dim3(256), 0, st, ucount, nt, pchunk);
    LOD_LAUNCH(k_bin_chunkscan, dim3((nt + 255) / 256), dim3(256), 0, st, pchunk, nt, L.chunks, tcount);
  }
  // tile offsets (exclusive; toff[nt] = pairs), slices
  LOD_LAUNCH(k_copy_u32, dim3((nt + 256) / 256), dim3(256), 0, st, tcount, toff, (uint64_t)nt + 1);
  device_scan<uint32_t>(toff, nt + 1, stmp, st);
  if (any) {
    // fill blocks of two units when there are many (32-bit cursors take twice
    // the LDS of the 16-bit counts: fewer resident waves)
    const uint32_t g = L.units >= 4096 ? 2u : 1u;
    LOD_LAUNCH((k_bin_fill<Src, RecT>), dim3(L.units / g), dim3(BW), lds, st, src, c, L.units, g, nbits, ucount,
               pchunk, toff, rec, L.max_pairs, status);
  }
  LOD_LAUNCH(k_slice_count, dim3((nt + 255) / 256), dim3(256), 0, st, tcount, nt, soff);
  fill_u32(soff + nt, 1, 0, st);
  device_scan<uint32_t>(soff, nt + 1, stmp, st);
  uint2 *stab = (uint2 *)(W + L.slice_table);
  LOD_LAUNCH(k_slice_table, dim3((nt + 255) / 256), dim3(256), 0, st, toff, tcount, soff, nt, stab, L.max_slices);
  const unsigned agrid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(16384, L.max_slices));
  if (any) {
    if constexpr (RecInfo<RecT>::cubic) {
      // narrow blobs take the windowed form (same bits, fewer idle lanes)
      const float hmax = (c.Fhw > 0.0f || has_point_radii(src)) ? lodh::BLOB_H_MAX : c.hpx;
      if (hmax < 1.9f)
        LOD_LAUNCH((k_accumulate_cubic_win<RecT, 4>), dim3(agrid), dim3(PT), 0, st, stab, soff, nt, rec, c,
                   partial, partial_aux, L.max_slices, L.max_pairs);
      else if (hmax < 3.9f)
        LOD_LAUNCH((k_accumulate_cubic_win<RecT, 8>), dim3(agrid), dim3(PT), 0, st, stab, soff, nt, rec, c,
                   partial, partial_aux, L.max_slices, L.max_pairs);
      else
        LOD_LAUNCH(k_accumulate_cubic<RecT>, dim3(agrid), dim3(PT), 0, st, stab, soff, nt, rec, c, partial,
                   partial_aux, L.max_slices, L.max_pairs);
    } else
      LOD_LAUNCH(k_accumulate<RecT>, dim3(agrid), dim3(PT), 0, st, stab, soff, nt, rec, c, partial, partial_aux,
                 L.max_slices, L.max_pairs);
  }
  LOD_LAUNCH(k_finalize, dim3(std::min<uint32_t>(nt, 4096)), dim3(PT), 0, st, soff, nt, partial, c, image,
             L.max_slices);
  if constexpr (RecInfo<RecT>::aux)
    LOD_LAUNCH(k_finalize, dim3(std::min<uint32_t>(nt, 4096)), dim3(PT), 0, st, soff, nt, partial_aux, c,
               image_aux, L.max_slices);
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

// Dispatch on the blob kind and on whether an attribute channel is drawn.
template <class Src>
static lod_status splat_any(const Src &src, bool any, const lod_camera &cam, const splat_params &sp, void *ws,
                            const SplatLayout &L, float *image, float *image_aux, uint64_t *status_word,
                            hipStream_t st, const HlStage *hs = nullptr) {
  const bool cubic = sp.blob == LOD_BLOB_CUBIC;
  if constexpr (!IsTree<Src>::value) {   // the LOD render draws no attribute channel
    if (L.aux) {
      if (cubic) return launch_splat_src<Src, RecCA>(src, any, cam, sp, ws, L, image, image_aux, status_word, st, hs);
      return launch_splat_src<Src, RecGA>(src, any, cam, sp, ws, L, image, image_aux, status_word, st, hs);
    }
  }
  if (cubic) return launch_splat_src<Src, RecC>(src, any, cam, sp, ws, L, image, nullptr, status_word, st, hs);
  return launch_splat_src<Src, float3>(src, any, cam, sp, ws, L, image, nullptr, status_word, st, hs);
}

lod_status launch_splat(const float *x, const float *y, const float *z, const float *m, const float *aux,
                        uint64_t count, const lod_camera &cam, const splat_params &sp, void *ws, const SplatLayout &L,
                        float *image, float *image_aux, hipStream_t st) {
  RawSrc src{x, y, z, m, count};
  src.aux = aux;
  return splat_any(src, count > 0, cam, sp, ws, L, image, image_aux, nullptr, st);
}

lod_status launch_splat_interp(const InterpArgs &a, const lod_camera &cam, const splat_params &sp, void *ws,
                               const SplatLayout &L, float *image, float *image_color, hipStream_t st) {
  const InterpSrc src{a.xa, a.ya, a.za, a.ma, a.xb, a.yb, a.zb, a.mb, a.ha, a.hb, a.ca, a.cb, a.count, a.t};
  return splat_any(src, a.count > 0, cam, sp, ws, L, image, image_color, nullptr, st);
}

lod_status launch_encode_motion(const lod_tree &tree, const float *xb, const float *yb, const float *zb,
                                const uint64_t *snap_off, int16_t *dqx, int16_t *dqy, int16_t *dqz,
                                uint64_t *saturated, hipStream_t st) {
  fill_u64(saturated, 1, 0, st);
  const unsigned g = (unsigned)std::min<uint64_t>(16384, std::max<uint64_t>(1, tree.node_capacity));
  LOD_LAUNCH(k_encode_motion, dim3(g), dim3(256), 0, st, tree, xb, yb, zb, snap_off, tree.node_capacity, dqx, dqy,
             dqz, saturated);
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

lod_status launch_splat_lod_motion(const lod_tree &tree, const uint32_t *node_ids, const uint64_t *n_ids, void *ws,
                                   const LodDrawLayout &D, const int16_t *dqx, const int16_t *dqy,
                                   const int16_t *dqz, float t, const lod_camera &cam, const splat_params &sp,
                                   const SplatLayout &L, float *image, hipStream_t st) {
  char *W = (char *)ws;
  uint64_t *offs = (uint64_t *)(W + D.offs);
  uint64_t *cnt = (uint64_t *)(W + D.count);
  const unsigned g = (unsigned)std::min<uint64_t>(4096, (D.max_ids + 256) / 256);
  LOD_LAUNCH(k_lod_counts, dim3(g), dim3(256), 0, st, tree, node_ids, n_ids, D.max_ids, offs);
  device_scan<uint64_t>(offs, D.max_ids + 1, (uint64_t *)(W + D.scan_tmp), st);
  LOD_LAUNCH(k_lod_total, dim3(1), dim3(1), 0, st, tree, offs, D.max_ids, D.max_points, cnt);
  TreeMotionSrc src{tree, node_ids, offs, n_ids, D.max_ids, cnt};
  src.dqx = dqx; src.dqy = dqy; src.dqz = dqz;
  src.t_frame = t;
  return splat_any(src, true, cam, sp, W + D.total, L, image, nullptr, tree.counts + 2, st);
}

lod_status launch_set_points(const lod_tree &tree, uint32_t node, const float *x, const float *y, const float *z,
                             const float *m, uint32_t count, hipStream_t st) {
  if (!count) return LOD_OK;
  const unsigned g = (unsigned)std::min<uint64_t>(1024, (count + 255) / 256);
  LOD_LAUNCH(k_set_points, dim3(g), dim3(256), 0, st, tree, node, x, y, z, m, count);
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

lod_status launch_splat_backward(const float *x, const float *y, const float *z, const float *m, uint64_t count,
                                 const lod_camera &cam, const splat_params &sp, const float *grad, float *gm,
                                 float *gx, float *gy, float *gz, hipStream_t st) {
  if (!count) return LOD_OK;
  Cam c = make_cam(cam, sp, nullptr);
  const unsigned grid = (unsigned)std::min<uint64_t>(65535, (count + PT - 1) / PT);
  if (sp.blob == LOD_BLOB_CUBIC)
    LOD_LAUNCH(k_backward_cubic, dim3(grid), dim3(PT), 0, st, x, y, z, m, count, c, grad, gm, gx, gy, gz);
  else
    LOD_LAUNCH(k_backward, dim3(grid), dim3(PT), 0, st, x, y, z, m, count, c, grad, gm, gx, gy, gz);
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

LodDrawLayout lod_draw_layout(uint64_t node_capacity, uint64_t max_points) {
  LodDrawLayout L{};
  L.max_ids = std::max<uint64_t>(1, node_capacity);
  L.max_points = std::max<uint64_t>(1, max_points);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.offs = take(8 * (L.max_ids + 1));
  L.scan_tmp = take(8 * scan_tmp_elems<uint64_t>(L.max_ids + 1));
  L.count = take(64);
  L.total = off;
  return L;
}

HlLayout hl_layout(const SplatLayout &L, uint64_t max_highlighted, const lod_camera &cam, const splat_params &sp,
                   lod_status &s) {
  HlLayout H{};
  H.cap = std::max<uint64_t>(1, max_highlighted);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  for (int a = 0; a < 4; ++a) H.stage[a] = take(4 * L.max_points);
  H.count = take(8 * (size_t)L.units);
  H.scan = take(8 * ((size_t)L.units + 1));
  H.scan_tmp = take(8 * scan_tmp_elems<uint64_t>((uint64_t)L.units + 1));
  H.total_ctr = take(64);
  for (int a = 0; a < 4; ++a) H.pts[a] = take(4 * H.cap);
  s = splat_layout(H.cap, cam, sp, H.L2, false);
  H.splat = off;
  H.total = off + H.L2.total;
  return H;
}

lod_status launch_hl_flags(const lod_tree &tree, const uint32_t *bits, uint64_t n_bits, uint32_t *flags,
                           hipStream_t st) {
  const uint64_t groups = (tree.point_capacity + 63) / 64;
  const unsigned g = (unsigned)std::min<uint64_t>(65535, std::max<uint64_t>(1, (groups + 3) / 4));
  LOD_LAUNCH(k_hl_flags, dim3(g), dim3(256), 0, st, tree, bits, n_bits, tree.point_capacity, flags);
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

lod_status launch_splat_lod(const lod_tree &tree, const uint32_t *node_ids, const uint64_t *n_ids, void *ws,
                            const LodDrawLayout &D, const lod_camera &cam, const splat_params &sp,
                            const SplatLayout &L, const uint32_t *hl_flags, const HlLayout *H,
                            float *image, float *image_hl, hipStream_t st) {
  char *W = (char *)ws;
  uint64_t *offs = (uint64_t *)(W + D.offs);
  uint64_t *cnt = (uint64_t *)(W + D.count);
  const unsigned g = (unsigned)std::min<uint64_t>(4096, (D.max_ids + 256) / 256);
  LOD_LAUNCH(k_lod_counts, dim3(g), dim3(256), 0, st, tree, node_ids, n_ids, D.max_ids, offs);
  device_scan<uint64_t>(offs, D.max_ids + 1, (uint64_t *)(W + D.scan_tmp), st);
  LOD_LAUNCH(k_lod_total, dim3(1), dim3(1), 0, st, tree, offs, D.max_ids, D.max_points, cnt);
  TreeSrc src{tree, node_ids, offs, n_ids, D.max_ids, cnt};
  if (!H) return splat_any(src, true, cam, sp, W + D.total, L, image, nullptr, tree.counts + 2, st);
  // ID highlighting: the count pass of the main render tests every drawn
  // point's flag and stages the flagged ones; they are gathered in unit
  // order and drawn by a second, small render
  src.hl_flags = hl_flags;
  src.hl_words = (tree.point_capacity + 63) / 64 * 2;
  char *HW = W + D.total + L.total;
  HlStage hs{(float *)(HW + H->stage[0]), (float *)(HW + H->stage[1]), (float *)(HW + H->stage[2]),
             (float *)(HW + H->stage[3]), (uint64_t *)(HW + H->count), (uint64_t *)(HW + H->scan)};
  fill_u64(hs.scan + L.units, 1, 0, st);
  lod_status s = splat_any(src, true, cam, sp, W + D.total, L, image, nullptr, tree.counts + 2, st, &hs);
  if (s != LOD_OK) return s;
  device_scan<uint64_t>(hs.scan, (uint64_t)L.units + 1, (uint64_t *)(HW + H->scan_tmp), st);
  float *px = (float *)(HW + H->pts[0]), *py = (float *)(HW + H->pts[1]);
  float *pz = (float *)(HW + H->pts[2]), *pm = (float *)(HW + H->pts[3]);
  uint64_t *hl_total = (uint64_t *)(HW + H->total_ctr);
  LOD_LAUNCH(k_hl_gather, dim3(L.units), dim3(256), 0, st, hs, (const uint64_t *)hs.scan, (const uint64_t *)cnt,
             D.max_points, L.units, px, py, pz, pm, H->cap, hl_total, tree.counts + 2);
  RawSrc hsrc{px, py, pz, pm, H->cap};
  hsrc.n_dev = hl_total;
  return splat_any(hsrc, true, cam, sp, HW + H->splat, H->L2, image_hl, nullptr, tree.counts + 2, st);
}

size_t decode_workspace(uint64_t node_capacity) {
  const uint64_t n = std::max<uint64_t>(1, node_capacity);
  return align256(8 * (n + 1)) + align256(8 * scan_tmp_elems<uint64_t>(n + 1));
}

lod_status launch_decode(const lod_tree &tree, const uint32_t *node_ids, const uint64_t *n_ids, uint64_t max_points,
                         float *x, float *y, float *z, float *m, uint64_t *n_points, void *ws, hipStream_t st) {
  const uint64_t max_ids = std::max<uint64_t>(1, tree.node_capacity);
  char *W = (char *)ws;
  uint64_t *offs = (uint64_t *)W;
  uint64_t *tmp = (uint64_t *)(W + align256(8 * (max_ids + 1)));
  const unsigned g = (unsigned)std::min<uint64_t>(4096, (max_ids + 256) / 256);
  LOD_LAUNCH(k_lod_counts, dim3(g), dim3(256), 0, st, tree, node_ids, n_ids, max_ids, offs);
  device_scan<uint64_t>(offs, max_ids + 1, tmp, st);
  LOD_LAUNCH(k_lod_total, dim3(1), dim3(1), 0, st, tree, offs, max_ids, max_points, n_points);
  const unsigned dg = (unsigned)std::min<uint64_t>(16384, max_ids);
  LOD_LAUNCH(k_lod_decode, dim3(dg), dim3(PT), 0, st, tree, node_ids, n_ids, max_ids, offs, max_points, x, y, z, m);
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

size_t cut_workspace(uint64_t node_capacity) {
  const uint64_t n = std::max<uint64_t>(1, node_capacity) + 1;
  return align256(4 * n) * 2 + align256(4 * scan_tmp_elems<uint32_t>(n));
}

lod_status launch_cut(const lod_tree &tree, const lod_camera &cam, float tau_px, uint32_t n, uint32_t *node_ids,
                      uint64_t cap, uint64_t *n_selected, void *ws, hipStream_t st) {
  const uint64_t nc = std::max<uint64_t>(1, tree.node_capacity);
  char *W = (char *)ws;
  uint32_t *keep = (uint32_t *)W;
  uint32_t *scan = (uint32_t *)(W + align256(4 * (nc + 1)));
  uint32_t *tmp = (uint32_t *)(W + 2 * align256(4 * (nc + 1)));
  CutArgs c{};
  c.proj = cam.projection; c.W = cam.W;
  c.px = (double)cam.pos[0]; c.py = (double)cam.pos[1]; c.pz = (double)cam.pos[2];
  c.F = (double)cam.F;
  c.tau_cbrt = (double)tau_px * std::cbrt((double)n);
  const unsigned g = (unsigned)std::min<uint64_t>(4096, (nc + 256) / 256);
  LOD_LAUNCH(k_cut_flags, dim3(g), dim3(256), 0, st, tree, c, nc, keep);
  LOD_LAUNCH(k_copy_u32, dim3(g), dim3(256), 0, st, keep, scan, nc + 1);
  device_scan<uint32_t>(scan, nc + 1, tmp, st);
  LOD_LAUNCH(k_cut_write, dim3(g), dim3(256), 0, st, tree, nc, keep, scan, node_ids, cap, n_selected);
  return hipGetLastError() == hipSuccess ? LOD_OK : LOD_EDEVICE;
}

}  // namespace lodh
