// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lod.h"

namespace lodh {

// Byte offsets of the build workspace arrays (256-byte aligned).
struct BuildLayout {
  uint64_t tiles, node_cap, point_cap;
  size_t keyA, keyB, idxA, idxB, loA, loB, lzA, lzB, mA, mB;
  size_t thist, scan32, scan64;
  size_t w, kb;
  size_t lvl, lsel, cs, sel_idx, sel_node, wit, pend, bflag, bscan, bottom, ctl, leafctl, emit_tot;
  size_t lpos, lkb, lwm;
  uint32_t sel_rows;             // blocks of a selection launch (rows of mhat)
  size_t mhat, src;
  size_t total;
};

BuildLayout build_layout(uint64_t N, const lod_params &p, uint32_t n_snap);
int key_bits(const lod_params &p, uint32_t n_snap);
lod_status launch_build(const lod_input &in, const lod_params &p, void *ws, const BuildLayout &L,
                        lod_tree &out, hipStream_t st);
void *workspace_view(void *ws, const BuildLayout &L, uint32_t which, uint64_t N, int passes,
                     uint64_t *count);

// Splat workspace layout.
struct SplatLayout {
  uint32_t tiles_x, tiles_y, n_tiles;
  uint32_t units, chunks;            // binning units (waves), 64 per chunk
  uint64_t max_points, max_pairs, max_slices;
  bool aux;                          // an attribute channel is drawn
  size_t tile_count, tile_off, ucount, pchunk, slice_off, scan_tmp, counters;
  size_t rec, partial, partial_aux, slice_table;   // rec: float32 records of the (point, tile) pairs
  size_t total;
};

constexpr int SPLAT_TS = 16;           // tile edge in pixels
constexpr uint32_t SPLAT_MAX_TILES = 8192;
constexpr uint32_t SPLAT_SLICE = 4096; // points per accumulation slice (4096: LOD splat 5.05 vs 5.11 ms at 2048)
constexpr uint32_t SPLAT_MAX_CHUNKS = 64;
constexpr float BLOB_H_MIN = 1.0f;     // cubic blob: clamp of a projected world radius, pixels
constexpr float BLOB_H_MAX = 16.0f;

// The largest pixel radius a blob of these parameters can take.
inline float blob_max_radius(const splat_params &sp) {
  if (sp.blob == LOD_BLOB_CUBIC) return sp.h_world > 0.0f ? BLOB_H_MAX : sp.h_px;
  return sp.radius_sigmas * sp.sigma_px;
}

lod_status splat_layout(uint64_t max_points, const lod_camera &cam, const splat_params &sp,
                        SplatLayout &L, bool aux);
lod_status launch_splat(const float *x, const float *y, const float *z, const float *m, const float *aux,
                        uint64_t count, const lod_camera &cam, const splat_params &sp, void *ws, const SplatLayout &L,
                        float *image, float *image_aux, hipStream_t st);
// Two snapshots of the same particles and a frame time (time interpolation).
struct InterpArgs {
  const float *xa, *ya, *za, *ma, *xb, *yb, *zb, *mb;
  const float *ha, *hb, *ca, *cb;
  uint64_t count;
  float t;
};
lod_status launch_splat_interp(const InterpArgs &a, const lod_camera &cam, const splat_params &sp, void *ws,
                               const SplatLayout &L, float *image, float *image_color, hipStream_t st);
lod_status launch_splat_backward(const float *x, const float *y, const float *z, const float *m,
                                 uint64_t count, const lod_camera &cam, const splat_params &sp,
                                 const float *grad, float *gm, float *gx, float *gy, float *gz,
                                 hipStream_t st);

// LOD render: the chosen nodes' stored points, decoded inside the binning.
struct LodDrawLayout {
  uint64_t max_ids, max_points;
  size_t offs, scan_tmp, count;
  size_t total;
};
LodDrawLayout lod_draw_layout(uint64_t node_capacity, uint64_t max_points);
// ID highlighting: staging of the selected drawn points (4 float arrays of
// the main render's max_points), per-unit counts and their scan, the
// gathered points (4 float arrays of cap) and the small render's layout.
struct HlLayout {
  uint64_t cap;
  size_t stage[4], count, scan, scan_tmp, total_ctr, pts[4], splat;
  SplatLayout L2;
  size_t total;
};
HlLayout hl_layout(const SplatLayout &L, uint64_t max_highlighted, const lod_camera &cam, const splat_params &sp,
                   lod_status &s);
lod_status launch_hl_flags(const lod_tree &tree, const uint32_t *bits, uint64_t n_bits, uint32_t *flags,
                           hipStream_t st);
lod_status launch_splat_lod(const lod_tree &tree, const uint32_t *node_ids, const uint64_t *n_ids, void *ws,
                            const LodDrawLayout &D, const lod_camera &cam, const splat_params &sp,
                            const SplatLayout &L, const uint32_t *hl_flags, const HlLayout *H,
                            float *image, float *image_hl, hipStream_t st);
lod_status launch_encode_motion(const lod_tree &tree, const float *xb, const float *yb, const float *zb,
                                const uint64_t *snap_off, int16_t *dqx, int16_t *dqy, int16_t *dqz,
                                uint64_t *saturated, hipStream_t st);
lod_status launch_splat_lod_motion(const lod_tree &tree, const uint32_t *node_ids, const uint64_t *n_ids, void *ws,
                                   const LodDrawLayout &D, const int16_t *dqx, const int16_t *dqy,
                                   const int16_t *dqz, float t, const lod_camera &cam, const splat_params &sp,
                                   const SplatLayout &L, float *image, hipStream_t st);
lod_status launch_set_points(const lod_tree &tree, uint32_t node, const float *x, const float *y, const float *z,
                             const float *m, uint32_t count, hipStream_t st);
size_t decode_workspace(uint64_t node_capacity);
lod_status launch_decode(const lod_tree &tree, const uint32_t *node_ids, const uint64_t *n_ids, uint64_t max_points,
                         float *x, float *y, float *z, float *m, uint64_t *n_points, void *ws, hipStream_t st);

// View-dependent cut.
size_t cut_workspace(uint64_t node_capacity);
lod_status launch_cut(const lod_tree &tree, const lod_camera &cam, float tau_px, uint32_t n,
                      uint32_t *node_ids, uint64_t cap, uint64_t *n_selected, void *ws,
                      hipStream_t st);

// small utilities
void fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st);
void fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st);

}  // namespace lodh
