/*
 * lod.h -- C ABI of liblod.so: octree level-of-detail build and point splat
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Szalay, Springel, Lemson, "GPU-Based Interactive Visualization of
 * Billion Point Cosmological Simulations" (arXiv:0811.2055).  The octree
 * paragraph defines the structure: a spatial octree in which all data of a
 * node or leaf is represented by at most n points, surplus points being
 * thinned by a density-weighted random subselection, children holding the
 * parent's data at eight times the detail.  The quantisation paragraph
 * stores every coordinate in 2 bytes spanning the containing block.  The
 * rendering paragraph draws each point as a smeared blob; the block-choice
 * paragraph draws near regions from deep in the tree and far ones from
 * shallow nodes.
 *
 * Conventions shared by every entry point:
 *  - Every pointer named "device" is GPU memory owned by the caller; the
 *    library allocates no device memory and keeps no data between calls
 *    (its only state is one extra stream and two events per device, used by
 *    lod_build, and an open lod_trace_begin/lod_trace_end record).  Each call only enqueues work on `stream` (a hipStream_t;
 *    NULL = the null stream) and returns; results are valid once the stream
 *    has reached them.
 *  - Arguments are checked on the host before anything is enqueued; a bad
 *    argument returns LOD_EINVAL (or LOD_EUNSUPPORTED / LOD_ECAPACITY) and
 *    enqueues nothing.  Data-dependent errors found on the device (a
 *    position outside [0,1] or NaN, a negative or NaN mass, an output
 *    capacity exceeded) are reported through the tree's device status word
 *    (counts[2], LOD_STATUS_* bits); outputs are undefined when it is not 0.
 *  - Calls that share a workspace must not overlap in time.
 */
#ifndef LOD_H
#define LOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LOD_OK = 0,
  LOD_EINVAL = -1,        /* bad argument (null pointer, out-of-range parameter) */
  LOD_EDOMAIN = -2,       /* reserved: no entry point returns it; positions or masses
                             outside the domain are found on the device and reported
                             by the status bit LOD_STATUS_DOMAIN instead */
  LOD_ENOMEM = -3,        /* workspace smaller than the plan requires */
  LOD_EDEVICE = -4,       /* a HIP call failed (launch error, no device) */
  LOD_ECAPACITY = -5,     /* an output array is smaller than its bound */
  LOD_EUNSUPPORTED = -6   /* a valid request this build does not handle */
} lod_status;

/* device status word bits (lod_tree.counts[2]) */
#define LOD_STATUS_DOMAIN   1u   /* a position outside [0,1]/NaN or a mass < 0/NaN */
#define LOD_STATUS_CAPACITY 2u   /* node or point capacity exceeded */
#define LOD_STATUS_OFFSETS  4u   /* snapshot offsets not monotone / not ending at N */

#define LOD_NONE 0xFFFFFFFFu     /* "no node" in parent / first_child */

typedef void *lod_stream_t;      /* hipStream_t */

/* Build parameters.  n: maximum points stored per node (the paper uses
 * 16000).  max_depth D in [0,10]: leaves are at depth <= D, the root at 0.
 * density_level L in [0,D]: the density weight of a particle is the number
 * of particles in its depth-L cell.  alpha in {-1,0,+1}: the keep
 * probability grows with density^alpha.  seed: Philox4x32-10 key.
 * mode: 0 = one selection launch per node (reference schedule; reads the
 *           level sizes back to the host, so it synchronises the stream),
 *       1 = one selection launch per level over all of its nodes,
 *       2 = one persistent launch over every node of every level: a block
 *           reduces a node whose children are done and climbs to the parent
 *           when it finishes the parent's last selecting child.
 * All modes produce identical bytes.  select_threads (threads per node
 * block) and persistent_blocks (mode 2 grid) are schedule parameters, e.g.
 * from lod_autotune; 0 picks the defaults (1024 threads, 2 blocks per CU).
 * In mode 1, levels that hold at most 64 nodes (depth <= 2) always use
 * 1024-thread blocks; mode 2 grids are capped at the selection scratch rows
 * (min(4096, N/(n+1) + snapshots + 1)). */
typedef struct {
  uint32_t n;
  uint32_t max_depth;
  uint32_t density_level;
  int32_t alpha;
  uint64_t seed;
  uint32_t mode;
  uint32_t select_threads;     /* 0 or a power of two in 64..1024 */
  uint32_t persistent_blocks;  /* 0 or 1..65535 */
  uint32_t reserved;           /* must be 0 */
} lod_params;

/* Particle input, structure of arrays, all device float32 [n_particles].
 * Positions must lie in [0,1]; masses >= 0.  A batch of snapshots is
 * concatenated; snap_offsets (device, uint64 [n_snapshots+1], first 0,
 * non-decreasing, last n_particles) delimits them, or is NULL for a single
 * snapshot.  A particle's id is its index within its snapshot.  Each
 * snapshot gets its own tree; the snapshot index is prefixed to the keys,
 * enters the Philox counter, and the forest is stored breadth first over
 * all snapshots. */
typedef struct {
  const float *x, *y, *z, *mass;
  uint64_t n_particles;
  const uint64_t *snap_offsets;
  uint32_t n_snapshots;
} lod_input;

/* Output tree, all device arrays owned by the caller.
 * Node table (node_capacity entries, breadth-first order, Morton order
 * within a level): prefix = Morton key of the node's cell at its depth with
 * the snapshot index above it; depth; parent (LOD_NONE for roots);
 * first_child (LOD_NONE for leaves; children are contiguous, ascending
 * octant); child_mask (bit o set when octant o exists); part_begin /
 * part_count = the node's range in Morton-sorted particle order; pt_begin /
 * pt_count = its stored points; node_mass = float64 sum of its particles'
 * masses.
 * Stored points (point_capacity entries, grouped by node in node order,
 * ascending sorted position within a node): pt_id = particle id within its
 * snapshot; qx,qy,qz = min(floor(a 2^(d+16)) - (c_d << 16), 65535) relative
 * to the storing node's cell c_d at depth d; pt_mass = stored float32 mass.
 * counts: device uint64[3] = {n_nodes, n_points, status bits}. */
typedef struct {
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
  uint64_t node_capacity, point_capacity;
  uint64_t *counts;
} lod_tree;

/* Camera.  projection 0: orthographic along +z onto the xy face of the unit
 * cube, u = x W, v = y H.  projection 1: perspective from pos with the
 * orthonormal basis (right, up, fwd), focal length F in pixels, points with
 * camera depth <= near_z culled; u = F xc/zc + W/2, v = F yc/zc + H/2.
 * Image row j covers v in [j, j+1), column i covers u in [i, i+1). */
typedef struct {
  uint32_t projection;
  uint32_t W, H;
  float pos[3], right[3], up[3], fwd[3];
  float F, near_z;
} lod_camera;

/* Blob kinds (rendering paragraph: every point drawn as a smeared blob; the
 * paper names a radial cubic function). */
#define LOD_BLOB_GAUSSIAN 0u
#define LOD_BLOB_CUBIC 1u

/* blob = LOD_BLOB_GAUSSIAN: a Gaussian of standard deviation sigma_px
 * pixels, truncated to the square |ox|,|oy| <= radius_sigmas * sigma_px,
 * normalised by 1/(2 pi s^2); sigma_px in (0, 8], radius_sigmas in (0, 6].
 * blob = LOD_BLOB_CUBIC: the compact cubic spline W(r; h) = 40/(7 pi h^2)
 * w(r/h), w(q) = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (1/2 < q < 1), 0
 * beyond; a pixel takes a point iff ox^2 + oy^2 < h^2 (the squares of the
 * float32 offsets summed in float64).  Radius h: h_px pixels in (0, 16]
 * when h_world is 0; with a perspective camera and h_world > 0 the
 * projected world radius fl(fl(F h_world) / zc), clamped to [1, 16] pixels.
 * sigma_px and radius_sigmas are ignored for the cubic blob. */
typedef struct {
  float sigma_px;
  float radius_sigmas;
  uint32_t blob;
  float h_px;
  float h_world;
} splat_params;

/* ---- level-of-detail build ------------------------------------------- */

/* Host only; no device work.  Returns the workspace size lod_build needs and
 * upper bounds on the node and point counts:
 *   nodes  <= n_snapshots + 8 D floor(N / (n+1))
 *   points <= N + n D floor(N / (n+1)).
 * Errors: LOD_EINVAL for null pointers or parameters out of range,
 * LOD_EUNSUPPORTED when 3D key bits plus snapshot bits exceed 32 or a
 * snapshot could hold 2^31 particles or more. */
lod_status lod_build_plan(const lod_input *in, const lod_params *p,
                          size_t *workspace_bytes, uint64_t *node_cap_bound,
                          uint64_t *point_cap_bound);

/* Build the tree of `in` into `out` (octree paragraph; quantisation
 * paragraph).  Steps, all on the device: cell keys and 16-bit fractional
 * positions; stable LSD radix sort of (key, id, position, mass); node
 * table level by level; density weights; Philox draws and integer
 * selection keys; per node holding more than n particles, the n smallest
 * (key, id) taken bottom up from the children's n+1 smallest; float64
 * mass renormalisation; 16-bit quantisation; output.  No host
 * synchronisation; safe to capture in a HIP graph.  The density step runs on
 * a second stream of the device owned by the library (created by the first
 * call made outside stream capture), forked from and joined back into
 * `stream` (the fork is taken under a lock, so builds on several streams may
 * be issued from several host threads; they share that second stream, each
 * with its own workspace and tree).  workspace: device, >= the planned size,
 * 256-byte aligned.  LOD_ECAPACITY when out->node_capacity or point_capacity
 * is below the plan's bound. */
lod_status lod_build(const lod_input *in, const lod_params *p, void *workspace,
                     size_t workspace_bytes, lod_tree *out, lod_stream_t stream);

/* ---- view-dependent cut (block-choice paragraph) ---------------------- */

/* Workspace bytes lod_select needs for a tree of node_capacity nodes. */
lod_status lod_select_plan(uint64_t node_capacity, size_t *workspace_bytes);

/* Choose the nodes to draw for `cam`: from each root, descend while the node
 * has children and either the camera is inside its cube (perspective only)
 * or its projected point spacing exceeds tau_px pixels; spacing of a depth-d
 * node is W 2^-d / n^(1/3) (orthographic) or F 2^-d / (n^(1/3) dist),
 * dist = |node centre - cam.pos| (float64).  Writes the chosen node indices
 * in node order to node_ids (device, cap entries) and their count to
 * *n_selected (device uint64).  The tree is read on the device; its node
 * count comes from tree->counts.  Status bit LOD_STATUS_CAPACITY is set in
 * tree->counts[2] if more than cap nodes are chosen. */
lod_status lod_select(const lod_tree *tree, const lod_camera *cam, float tau_px,
                      uint32_t n, uint32_t *node_ids, uint64_t cap,
                      uint64_t *n_selected, void *workspace, size_t workspace_bytes,
                      lod_stream_t stream);

/* ---- additive point splat (rendering paragraph) ----------------------- */

/* Workspace bytes for splatting up to max_points points with cam/sp, by
 * splat_render or splat_render_aux. */
lod_status splat_plan(uint64_t max_points, const lod_camera *cam, const splat_params *sp,
                      size_t *workspace_bytes);

/* image[j*W + i] = sum_k m_k exp(-(ox^2+oy^2)/(2 s^2)) / (2 pi s^2) over
 * points whose truncated blob covers pixel (i,j); ox = fl(u - (i+1/2)),
 * oy = fl(v - (j+1/2)) in float32 from the pinned projection sequence
 * (no fused multiply-add); sums accumulated in float32 with compensation.
 * x,y,z,m: device float32 [count]; image: device float32 [H*W], overwritten. */
lod_status splat_render(const float *x, const float *y, const float *z, const float *m,
                        uint64_t count, const lod_camera *cam, const splat_params *sp,
                        void *workspace, size_t workspace_bytes, float *image,
                        lod_stream_t stream);

/* Second image channel: image_aux[j*W + i] = sum_k m_k a_k W_k(i, j) for a
 * per-point attribute a (device float32 [count]), e.g. a colour value or a
 * 0/1 selection; image as splat_render.  Same blobs, binning and sums as
 * splat_render (the rendering paragraph's per-point properties).  workspace
 * as sized by splat_plan. */
lod_status splat_render_aux(const float *x, const float *y, const float *z, const float *m, const float *aux,
                            uint64_t count, const lod_camera *cam, const splat_params *sp, void *workspace,
                            size_t workspace_bytes, float *image, float *image_aux, lod_stream_t stream);

/* Workspace bytes for splat_render_lod on a tree of node_capacity nodes
 * drawing at most max_points points. */
lod_status splat_lod_plan(uint64_t node_capacity, uint64_t max_points, const lod_camera *cam,
                          const splat_params *sp, size_t *workspace_bytes);

/* Render the stored points of the nodes node_ids[0 .. *n_ids) (device
 * arrays, count on the device) of `tree`, decoding each point from its
 * node: a = float32 nearest (c 2^16 + q + 1/2) 2^-(d+16).  max_points bounds
 * the points drawn (workspace sizing); more sets LOD_STATUS_CAPACITY. */
lod_status splat_render_lod(const lod_tree *tree, const uint32_t *node_ids,
                            const uint64_t *n_ids, uint64_t max_points,
                            const lod_camera *cam, const splat_params *sp,
                            void *workspace, size_t workspace_bytes, float *image,
                            lod_stream_t stream);

/* ID highlighting (highlighting paragraph: points whose id is in a list of
 * up to a million selected ids, tested as each point is drawn).  The list
 * is a bitset over ids (device uint32 [ceil(n_bits/32)], bit i of word i/32
 * = id i; ids >= n_bits are never selected).  lod_highlight_flags turns it,
 * once per list, into one flag bit per stored point of the tree: flags
 * (device uint32 [2 ceil(point_capacity / 64)]) bit s of word s/32 = stored
 * point s has a selected id (a list changes far less often than frames are
 * drawn, and the per-point flags are read in drawing order). */
lod_status lod_highlight_flags(const lod_tree *tree, const uint32_t *bits, uint64_t n_bits, uint32_t *flags,
                               lod_stream_t stream);

/* image as splat_render_lod; image_hl (device float32 [H*W]) = the same
 * blobs summed over the drawn points whose flag is set.  The flag test runs
 * inside the main render's binning pass, which stages the flagged points in
 * drawing order; they are then drawn by a second render of at most
 * max_highlighted points (a cut draws each particle at most once, so the
 * number of selected ids is a bound; more sets LOD_STATUS_CAPACITY in
 * tree->counts[2] and truncates).  Both images are bit-reproducible.
 * workspace: splat_lod_highlight_plan. */
lod_status splat_lod_highlight_plan(uint64_t node_capacity, uint64_t max_points, uint64_t max_highlighted,
                                    const lod_camera *cam, const splat_params *sp, size_t *workspace_bytes);
lod_status splat_render_lod_highlight(const lod_tree *tree, const uint32_t *node_ids, const uint64_t *n_ids,
                                      uint64_t max_points, const lod_camera *cam, const splat_params *sp,
                                      const uint32_t *flags, uint64_t max_highlighted, void *workspace,
                                      size_t workspace_bytes, float *image, float *image_hl, lod_stream_t stream);

/* ---- time interpolation between snapshots (rendering paragraph: points
 * carry time information; position, size and colour are interpolated for
 * every frame) ----------------------------------------------------------- */

/* One snapshot's per-particle arrays (device float32 [count]); the same
 * index is the same particle in both snapshots.  h: world radius of the
 * cubic blob (perspective only) or NULL; c: colour value or NULL. */
typedef struct {
  const float *x, *y, *z, *m, *h, *c;
} splat_frame;

/* The frame at time t in [0, 1] between snapshots a and b: every quantity
 * (position, mass, and the radius and colour when given) is
 * fl(q_a + fl(t fl(q_b - q_a))) in float32; image = splat_render of those
 * points; with colours, image_color = sum m(t) c(t) W (the attribute
 * channel of splat_render_aux).  Radii require blob = LOD_BLOB_CUBIC and a
 * perspective camera; they replace sp->h_world per point.  workspace as
 * sized by splat_plan. */
lod_status splat_render_interp(const splat_frame *a, const splat_frame *b, uint64_t count, float t,
                               const lod_camera *cam, const splat_params *sp, void *workspace,
                               size_t workspace_bytes, float *image, float *image_color, lod_stream_t stream);

/* Motion codes of a tree's stored points (quantisation paragraph: the other
 * properties of a point are encoded like its position): for a point stored
 * at depth d with position code Q0 = (c << 16) + q per axis and its
 * particle's position a in the next snapshot (x_next..z_next, device
 * float32, indexed like the build input: snapshot offset + id),
 * dq = floor((floor(a 2^(d+16)) - Q0 + 2) / 4) clamped to int16, i.e. the
 * motion in steps of four position quanta, two block sides either way.
 * dqx/dqy/dqz: device int16 [point capacity]; *saturated (device uint64)
 * receives the number of clamped components.  snap_offsets: as given to
 * lod_build, or NULL for a single snapshot. */
lod_status lod_encode_motion(const lod_tree *tree, const float *x_next, const float *y_next, const float *z_next,
                             const uint64_t *snap_offsets, int16_t *dqx, int16_t *dqy, int16_t *dqz,
                             uint64_t *saturated, lod_stream_t stream);

/* splat_render_lod at frame time t in [0, 1]: each stored point is drawn at
 * fl(p + fl(t fl(p' - p))) between its decoded position p and the position
 * p' = the float32 nearest (2 (c 2^16 + q + 4 dq) + 1) 2^-(d+17) of its
 * motion code.  Masses are the stored ones.  workspace: splat_lod_plan. */
lod_status splat_render_lod_motion(const lod_tree *tree, const uint32_t *node_ids, const uint64_t *n_ids,
                                   uint64_t max_points, const int16_t *dqx, const int16_t *dqy, const int16_t *dqz,
                                   float t, const lod_camera *cam, const splat_params *sp, void *workspace,
                                   size_t workspace_bytes, float *image, lod_stream_t stream);

/* Replace the first `count` stored points of node `node` (count at most its
 * pt_count; a refined node keeps its point count) with positions x, y, z and
 * masses m (device float32 [count]): each coordinate is coded as
 * min(floor(a 2^(d+16)) - (c << 16), 65535) relative to the node's cell, as
 * the build codes it (quantisation paragraph); a position outside the cell
 * sets LOD_STATUS_DOMAIN and is clamped to it.  For writing refined points
 * back into a tree. */
lod_status lod_set_node_points(const lod_tree *tree, uint32_t node, const float *x, const float *y, const float *z,
                               const float *m, uint32_t count, lod_stream_t stream);

/* Workspace bytes for lod_decode on a tree of node_capacity nodes. */
lod_status lod_decode_plan(uint64_t node_capacity, size_t *workspace_bytes);

/* Decode the stored points of nodes node_ids[0 .. *n_ids) (device arrays,
 * count on the device) into caller arrays x, y, z, m (device float32, at
 * least max_points each), node by node in the given order; each coordinate
 * is the float32 nearest (c 2^16 + q + 1/2) 2^-(d+16) for the storing node's
 * cell c at depth d (quantisation paragraph).  The number of points written
 * goes to *n_points (device uint64); more than max_points sets
 * LOD_STATUS_CAPACITY in tree->counts[2] and truncates. */
lod_status lod_decode(const lod_tree *tree, const uint32_t *node_ids, const uint64_t *n_ids,
                      uint64_t max_points, float *x, float *y, float *z, float *m,
                      uint64_t *n_points, void *workspace, size_t workspace_bytes,
                      lod_stream_t stream);

/* Adjoint of splat_render: given dL/dimage (device float32 [H*W]) write
 * dL/dm (device float32 [count]) and dL/dx, dL/dy, dL/dz (device float32
 * [count] each; any of them may be NULL to skip).  The derivative of the
 * truncation indicator is taken as zero.  Culled points get zero. */
lod_status splat_render_backward(const float *x, const float *y, const float *z,
                                 const float *m, uint64_t count, const lod_camera *cam,
                                 const splat_params *sp, const float *grad_image,
                                 float *grad_m, float *grad_x, float *grad_y,
                                 float *grad_z, lod_stream_t stream);

/* ---- allocation-free splat --------------------------------------------- */

/* Bytes of the device array that splat_render_noalloc uses as its workspace
 * (one array per device, held until the process ends). */
#define LOD_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): splat_render with
 * its workspace taken from a fixed 64 MiB device array inside the library
 * instead of a caller buffer.  Same arguments, image and bits as
 * splat_render.  Allocates nothing (no hipMalloc, no library allocation);
 * the first call on a device looks up that device's array address.
 * LOD_ECAPACITY, with nothing enqueued, when splat_plan(count, cam, sp)
 * exceeds LOD_NOALLOC_SCRATCH_BYTES (about 1.2 M points at 1024x1024 with
 * the default blob).  All calls on one device share its array: calls that
 * overlap in time on one device (several streams or host threads) race and
 * must be serialised by the caller. */
lod_status splat_render_noalloc(const float *x, const float *y, const float *z, const float *m,
                                uint64_t count, const lod_camera *cam, const splat_params *sp,
                                float *image, lod_stream_t stream);

/* ---- block store and view-dependent streaming (the IO paragraphs: only
 * the data a view needs is loaded, from a spatially indexed store, at the
 * rate of an ordinary link; the CPU decides which blocks to load and draw) */

/* Write a built tree to the file `path` (host call; synchronises `stream`).
 * Format (little endian): a 64-byte header (magic "LODSTOR1", version 1,
 * n, node and point counts, section offsets), the node table (prefix,
 * depth, parent, first_child, child_mask, part_begin, part_count, pt_count,
 * node_mass, block offset; each array 8-byte aligned), then one block per
 * node in node order: pt_id u32[k], qx, qy, qz u16[k], pt_mass f32[k]
 * (14 bytes per stored point).  n: the build's points per node.
 * LOD_EINVAL when the tree's status word is not 0 or the file cannot be
 * written. */
lod_status lod_store_save(const lod_tree *tree, uint32_t n, const char *path, lod_stream_t stream);

/* Node count, stored point count and n of a store file. */
lod_status lod_store_read_info(const char *path, uint64_t *n_nodes, uint64_t *n_points, uint32_t *n);

typedef struct lod_streamer lod_streamer;

/* Per-frame report of lod_streamer_frame. */
typedef struct {
  uint64_t bytes_loaded;    /* block bytes read and copied this frame */
  uint32_t nodes_loaded, nodes_evicted, nodes_drawn;
  uint32_t groups_waiting;  /* candidate groups left for later frames */
  uint64_t points_drawn;
  uint64_t resident_nodes;
  double decide_ms;         /* host: the choice of loads and evictions */
  double io_ms;             /* host: reading the loaded blocks from the store */
  double upload_ms;         /* copies to the device and the draw list, synchronised */
} lod_stream_stats;

/* Open a store for streaming into the caller's device arrays `view` (a
 * lod_tree: node arrays of at least the store's node count, point arrays of
 * at least pool_slots * n entries, counts[3]).  The node table is copied
 * once; the point arrays form a pool of pool_slots slots of n points; the
 * roots are loaded now and never evicted (LOD_ECAPACITY when they do not
 * fit).  After each frame, view->pt_begin holds the slot offsets of the
 * resident nodes, so splat_render_lod(view, draw list) draws the frame.
 * The streamer allocates pinned host staging, no device memory.  A file is
 * checked before anything reaches the device: LOD_EINVAL when it cannot be
 * read, has another magic or version, or its node table is not a tree
 * (indices out of range, a child that does not name its parent or follow
 * it in node order, more than n points in a node, a block past the end of the
 * file); LOD_EDEVICE when a copy or the pinned allocation fails. */
lod_status lod_streamer_open(const char *path, uint32_t pool_slots, lod_tree *view, lod_streamer **out);

/* One frame.  The link carries budget_bytes per frame: a credit grows by
 * that each frame and unused credit carries over, up to budget_bytes plus
 * one full group (8 n blocks).  From the roots, a visited node is descended
 * into when the camera wants more detail there (lod_select's test with
 * tau_px) and all its children are resident; the children of visited nodes
 * that want more detail form candidate groups, taken by priority (camera
 * inside the parent's cube, then larger projected spacing of the parent,
 * then smaller parent index); a group costs the blocks of its non-resident
 * children and loading stops at the first group that does not fit the
 * credit.  Slots are freed by evicting resident non-root nodes with no
 * resident children, not visited this frame and not children of a node
 * visited this frame that wants more detail, least recently visited first
 * (ties: larger index first); loading stops when none is left.  The frame
 * then draws the visit repeated over the new residency: the visited nodes
 * not descended into, ascending, written to draw_ids (device uint32, at
 * least the node count) and their number to *n_draw (device uint64).
 * Loaded and evicted node ids go to the optional host arrays (up to their
 * caps).  Synchronises `stream` (the staging buffers are reused). */
lod_status lod_streamer_frame(lod_streamer *s, const lod_camera *cam, float tau_px, uint64_t budget_bytes,
                              uint32_t *draw_ids, uint64_t *n_draw, lod_stream_stats *stats, uint32_t *loaded_ids,
                              uint32_t loaded_cap, uint32_t *evicted_ids, uint32_t evicted_cap,
                              lod_stream_t stream);

/* Close the store and release the streamer's host buffers. */
lod_status lod_streamer_close(lod_streamer *s);

/* ---- schedule autotuning ------------------------------------------------ */

/* Time lod_build on this input for each candidate schedule (mode 1 and 2,
 * select_threads in {256, 512, 1024}, mode 2 grids of 1, 2 and 4 blocks per
 * compute unit), two timed builds each with hipEvents on `stream`, and write
 * the fastest into p->mode, p->select_threads and p->persistent_blocks.
 * Every schedule produces identical bytes, so the choice affects speed only.
 * Candidates and their mean milliseconds are written to cand / ms (up to
 * cap entries; *n_cand gets the number tried).  Synchronises the stream.
 * Arguments as for lod_build. */
lod_status lod_autotune(const lod_input *in, lod_params *p, void *workspace, size_t workspace_bytes,
                        lod_tree *out, lod_params *cand, float *ms, uint32_t cap, uint32_t *n_cand,
                        lod_stream_t stream);

/* ---- introspection ----------------------------------------------------- */

/* Device pointers into a lod_build workspace, valid after a build with the
 * same input sizes and parameters.  which: 0 sorted keys (uint32 [N],
 * snapshot bits above 3D key bits), 1 sorted particle index (uint32 [N],
 * global), 2 density w (uint32 [N], sorted order), 3 the 12-bit key bin of
 * the selection key K (uint16 [N], sorted order: K itself for K < 128, else
 * 128 + 64 (e - 7) + the six bits of K after its leading one, e = the
 * leading one's position; the exact 64-bit K is not kept), 4 per-node
 * witness sorted position (uint32 [node capacity], LOD_NONE if none).
 * *count receives the number of elements.  For tests and diagnostics. */
lod_status lod_workspace_view(const lod_input *in, const lod_params *p, void *workspace,
                              uint32_t which, void **device_ptr, uint64_t *count);

/* Per-kernel timing for diagnostics and benchmarks.  Between
 * lod_trace_begin() and lod_trace_end() on one host thread, every kernel an
 * entry point enqueues is bracketed by two hipEvents recorded on its stream
 * (this adds a few microseconds per launch).  lod_trace_end() waits for
 * those events, writes up to `cap` records (static kernel name, elapsed
 * milliseconds) in launch order, stores the number of launches in
 * *n_records, and releases the events.  LOD_EINVAL if no trace is open. */
typedef struct {
  const char *name;
  float ms;
} lod_kernel_time;

lod_status lod_trace_begin(void);
lod_status lod_trace_end(lod_kernel_time *records, uint32_t cap, uint32_t *n_records);

/* Static description of an error code. */
const char *lod_status_string(lod_status s);

/* Library version string. */
const char *lod_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LOD_H */
