// C ABI of liblod.so: host-side argument checks, workspace plans and launch
// sequencing.  Every check runs before anything is enqueued.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "lod.h"
#include "lod_internal.hpp"
#include "lod_trace.hpp"

namespace {

lod_status check_params(const lod_input *in, const lod_params *p) {
  if (!in || !p) return LOD_EINVAL;
  if (p->n < 1) return LOD_EINVAL;
  if (p->max_depth > 10) return LOD_EINVAL;
  if (p->density_level > p->max_depth) return LOD_EINVAL;
  if (p->alpha < -1 || p->alpha > 1) return LOD_EINVAL;
  if (p->mode > 2 || p->reserved != 0 || p->persistent_blocks > 65535) return LOD_EINVAL;
  if (p->select_threads &&
      ((p->select_threads & (p->select_threads - 1)) || p->select_threads < 64 || p->select_threads > 1024))
    return LOD_EINVAL;
  const uint32_t ns = in->snap_offsets ? in->n_snapshots : 1;
  if (in->snap_offsets && in->n_snapshots < 1) return LOD_EINVAL;
  if (lodh::key_bits(*p, ns) > 32) return LOD_EUNSUPPORTED;
  // sorted positions are 32-bit; a single snapshot's ids must stay below 2^31
  if (in->n_particles >= 0xFFFFFFFFull) return LOD_EUNSUPPORTED;
  if (!in->snap_offsets && in->n_particles >= (1ull << 31)) return LOD_EUNSUPPORTED;
  return LOD_OK;
}

lod_status check_inputs(const lod_input *in, const lod_params *p) {
  lod_status s = check_params(in, p);
  if (s != LOD_OK) return s;
  if (in->n_particles && (!in->x || !in->y || !in->z || !in->mass)) return LOD_EINVAL;
  return LOD_OK;
}

bool check_camera(const lod_camera *c, const splat_params *sp) {
  if (!c || !sp) return false;
  if (c->projection > 1 || c->W == 0 || c->H == 0 || c->W > 16384 || c->H > 16384) return false;
  if (sp->blob == LOD_BLOB_GAUSSIAN) {
    if (!(sp->sigma_px > 0.0f && sp->sigma_px <= 8.0f)) return false;
    if (!(sp->radius_sigmas > 0.0f && sp->radius_sigmas <= 6.0f)) return false;
  } else if (sp->blob == LOD_BLOB_CUBIC) {
    if (sp->h_world != 0.0f) {
      if (!(sp->h_world > 0.0f) || !std::isfinite(sp->h_world) || c->projection != 1) return false;
      if (!std::isfinite(c->F * sp->h_world)) return false;
    } else if (!(sp->h_px > 0.0f && sp->h_px <= lodh::BLOB_H_MAX)) {
      return false;
    }
  } else {
    return false;
  }
  if (c->projection == 1) {
    if (!(c->near_z > 0.0f) || !std::isfinite(c->F) || !(c->F > 0.0f)) return false;
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(c->pos[i]) || !std::isfinite(c->right[i]) || !std::isfinite(c->up[i]) ||
          !std::isfinite(c->fwd[i]))
        return false;
  }
  return true;
}

bool tree_arrays_ok(const lod_tree *t) {
  return t && t->prefix && t->depth && t->parent && t->first_child && t->child_mask && t->part_begin &&
         t->part_count && t->pt_begin && t->pt_count && t->node_mass && t->pt_id && t->qx && t->qy && t->qz &&
         t->pt_mass && t->counts;
}

}  // namespace

namespace lodh {
Trace *&current_trace() {
  static thread_local Trace *t = nullptr;
  return t;
}
}  // namespace lodh

extern "C" {

lod_status lod_trace_begin(void) {
  lodh::Trace *&t = lodh::current_trace();
  if (t) return LOD_EINVAL;
  t = new lodh::Trace();
  return LOD_OK;
}

lod_status lod_trace_end(lod_kernel_time *records, uint32_t cap, uint32_t *n_records) {
  lodh::Trace *&t = lodh::current_trace();
  if (!t) return LOD_EINVAL;
  lod_status st = LOD_OK;
  uint32_t k = 0;
  for (auto &r : t->recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      st = LOD_EDEVICE;
    if (records && k < cap) records[k] = lod_kernel_time{r.name, ms};
    ++k;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (n_records) *n_records = k;
  delete t;
  t = nullptr;
  return st;
}


lod_status lod_build_plan(const lod_input *in, const lod_params *p, size_t *workspace_bytes,
                          uint64_t *node_cap_bound, uint64_t *point_cap_bound) {
  if (!workspace_bytes || !node_cap_bound || !point_cap_bound) return LOD_EINVAL;
  lod_status s = check_params(in, p);
  if (s != LOD_OK) return s;
  const uint32_t ns = in->snap_offsets ? in->n_snapshots : 1;
  lodh::BuildLayout L = lodh::build_layout(in->n_particles, *p, ns);
  *workspace_bytes = L.total;
  *node_cap_bound = L.node_cap;
  *point_cap_bound = L.point_cap;
  return LOD_OK;
}

lod_status lod_build(const lod_input *in, const lod_params *p, void *workspace, size_t workspace_bytes,
                     lod_tree *out, lod_stream_t stream) {
  lod_status s = check_inputs(in, p);
  if (s != LOD_OK) return s;
  if (!tree_arrays_ok(out) || !workspace) return LOD_EINVAL;
  if (((uintptr_t)workspace) & 255) return LOD_EINVAL;
  const uint32_t ns = in->snap_offsets ? in->n_snapshots : 1;
  lodh::BuildLayout L = lodh::build_layout(in->n_particles, *p, ns);
  if (workspace_bytes < L.total) return LOD_ENOMEM;
  if (out->node_capacity < L.node_cap || out->point_capacity < L.point_cap) return LOD_ECAPACITY;
  return lodh::launch_build(*in, *p, workspace, L, *out, (hipStream_t)stream);
}

lod_status lod_select_plan(uint64_t node_capacity, size_t *workspace_bytes) {
  if (!workspace_bytes) return LOD_EINVAL;
  *workspace_bytes = lodh::cut_workspace(node_capacity);
  return LOD_OK;
}

lod_status lod_select(const lod_tree *tree, const lod_camera *cam, float tau_px, uint32_t n, uint32_t *node_ids,
                      uint64_t cap, uint64_t *n_selected, void *workspace, size_t workspace_bytes,
                      lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || !cam || !node_ids || !n_selected || !workspace) return LOD_EINVAL;
  if (n < 1 || !(tau_px > 0.0f) || !std::isfinite(tau_px) || cap == 0) return LOD_EINVAL;
  splat_params dummy{1.0f, 3.0f, LOD_BLOB_GAUSSIAN, 0.0f, 0.0f};
  if (!check_camera(cam, &dummy)) return LOD_EINVAL;
  if (workspace_bytes < lodh::cut_workspace(tree->node_capacity)) return LOD_ENOMEM;
  return lodh::launch_cut(*tree, *cam, tau_px, n, node_ids, cap, n_selected, workspace, (hipStream_t)stream);
}

lod_status splat_plan(uint64_t max_points, const lod_camera *cam, const splat_params *sp, size_t *workspace_bytes) {
  if (!workspace_bytes || !check_camera(cam, sp)) return LOD_EINVAL;
  lodh::SplatLayout L;
  lod_status s = lodh::splat_layout(max_points, *cam, *sp, L, true);   // covers both forms
  if (s != LOD_OK) return s;
  *workspace_bytes = L.total;
  return LOD_OK;
}

static lod_status splat_common(const float *x, const float *y, const float *z, const float *m, const float *aux,
                               uint64_t count, const lod_camera *cam, const splat_params *sp, void *workspace,
                               size_t workspace_bytes, float *image, float *image_aux, lod_stream_t stream) {
  if (!check_camera(cam, sp) || !image || !workspace) return LOD_EINVAL;
  if (count && (!x || !y || !z || !m)) return LOD_EINVAL;
  if (((uintptr_t)workspace) & 255) return LOD_EINVAL;
  lodh::SplatLayout L;
  lod_status s = lodh::splat_layout(count, *cam, *sp, L, image_aux != nullptr);
  if (s != LOD_OK) return s;
  if (workspace_bytes < L.total) return LOD_ENOMEM;
  return lodh::launch_splat(x, y, z, m, aux, count, *cam, *sp, workspace, L, image, image_aux, (hipStream_t)stream);
}

lod_status splat_render(const float *x, const float *y, const float *z, const float *m, uint64_t count,
                        const lod_camera *cam, const splat_params *sp, void *workspace, size_t workspace_bytes,
                        float *image, lod_stream_t stream) {
  return splat_common(x, y, z, m, nullptr, count, cam, sp, workspace, workspace_bytes, image, nullptr, stream);
}

lod_status splat_render_aux(const float *x, const float *y, const float *z, const float *m, const float *aux,
                            uint64_t count, const lod_camera *cam, const splat_params *sp, void *workspace,
                            size_t workspace_bytes, float *image, float *image_aux, lod_stream_t stream) {
  if (!image_aux || (count && !aux)) return LOD_EINVAL;
  return splat_common(x, y, z, m, aux, count, cam, sp, workspace, workspace_bytes, image, image_aux, stream);
}

lod_status splat_render_lod(const lod_tree *tree, const uint32_t *node_ids, const uint64_t *n_ids,
                            uint64_t max_points, const lod_camera *cam, const splat_params *sp, void *workspace,
                            size_t workspace_bytes, float *image, lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || !node_ids || !n_ids || !check_camera(cam, sp) || !image || !workspace)
    return LOD_EINVAL;
  if (((uintptr_t)workspace) & 255) return LOD_EINVAL;
  lodh::LodDrawLayout D = lodh::lod_draw_layout(tree->node_capacity, max_points);
  lodh::SplatLayout L;
  lod_status s = lodh::splat_layout(D.max_points, *cam, *sp, L, false);
  if (s != LOD_OK) return s;
  if (workspace_bytes < D.total + L.total) return LOD_ENOMEM;
  return lodh::launch_splat_lod(*tree, node_ids, n_ids, workspace, D, *cam, *sp, L, nullptr, nullptr, image,
                                nullptr, (hipStream_t)stream);
}

lod_status splat_lod_plan(uint64_t node_capacity, uint64_t max_points, const lod_camera *cam,
                          const splat_params *sp, size_t *workspace_bytes) {
  if (!workspace_bytes || !check_camera(cam, sp)) return LOD_EINVAL;
  lodh::LodDrawLayout D = lodh::lod_draw_layout(node_capacity, max_points);
  lodh::SplatLayout L;
  lod_status s = lodh::splat_layout(D.max_points, *cam, *sp, L, false);
  if (s != LOD_OK) return s;
  *workspace_bytes = D.total + L.total;
  return LOD_OK;
}

// Layouts of the highlighted LOD render: the plain one, then the staging and
// the second render.
static lod_status highlight_layouts(uint64_t node_capacity, uint64_t max_points, uint64_t max_highlighted,
                                    const lod_camera *cam, const splat_params *sp, lodh::LodDrawLayout &D,
                                    lodh::SplatLayout &L, lodh::HlLayout &H) {
  D = lodh::lod_draw_layout(node_capacity, max_points);
  lod_status s = lodh::splat_layout(D.max_points, *cam, *sp, L, false);
  if (s != LOD_OK) return s;
  H = lodh::hl_layout(L, max_highlighted, *cam, *sp, s);
  return s;
}

lod_status splat_lod_highlight_plan(uint64_t node_capacity, uint64_t max_points, uint64_t max_highlighted,
                                    const lod_camera *cam, const splat_params *sp, size_t *workspace_bytes) {
  if (!workspace_bytes || !check_camera(cam, sp) || max_highlighted == 0) return LOD_EINVAL;
  lodh::LodDrawLayout D;
  lodh::SplatLayout L;
  lodh::HlLayout H;
  lod_status s = highlight_layouts(node_capacity, max_points, max_highlighted, cam, sp, D, L, H);
  if (s != LOD_OK) return s;
  *workspace_bytes = D.total + L.total + H.total;
  return LOD_OK;
}

lod_status lod_highlight_flags(const lod_tree *tree, const uint32_t *bits, uint64_t n_bits, uint32_t *flags,
                               lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || !bits || n_bits == 0 || !flags) return LOD_EINVAL;
  return lodh::launch_hl_flags(*tree, bits, n_bits, flags, (hipStream_t)stream);
}

lod_status splat_render_lod_highlight(const lod_tree *tree, const uint32_t *node_ids, const uint64_t *n_ids,
                                      uint64_t max_points, const lod_camera *cam, const splat_params *sp,
                                      const uint32_t *flags, uint64_t max_highlighted, void *workspace,
                                      size_t workspace_bytes, float *image, float *image_hl, lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || !node_ids || !n_ids || !check_camera(cam, sp) || !image || !workspace)
    return LOD_EINVAL;
  if (!flags || !image_hl || max_highlighted == 0) return LOD_EINVAL;
  if (((uintptr_t)workspace) & 255) return LOD_EINVAL;
  lodh::LodDrawLayout D;
  lodh::SplatLayout L;
  lodh::HlLayout H;
  lod_status s = highlight_layouts(tree->node_capacity, max_points, max_highlighted, cam, sp, D, L, H);
  if (s != LOD_OK) return s;
  if (workspace_bytes < D.total + L.total + H.total) return LOD_ENOMEM;
  return lodh::launch_splat_lod(*tree, node_ids, n_ids, workspace, D, *cam, *sp, L, flags, &H, image, image_hl,
                                (hipStream_t)stream);
}

lod_status splat_render_interp(const splat_frame *a, const splat_frame *b, uint64_t count, float t,
                               const lod_camera *cam, const splat_params *sp, void *workspace,
                               size_t workspace_bytes, float *image, float *image_color, lod_stream_t stream) {
  if (!a || !b || !check_camera(cam, sp) || !image || !workspace) return LOD_EINVAL;
  if (!(t >= 0.0f && t <= 1.0f)) return LOD_EINVAL;
  if (count && (!a->x || !a->y || !a->z || !a->m || !b->x || !b->y || !b->z || !b->m)) return LOD_EINVAL;
  const bool sizes = a->h || b->h, colours = a->c || b->c;
  if (sizes && (!a->h || !b->h || sp->blob != LOD_BLOB_CUBIC || cam->projection != 1)) return LOD_EINVAL;
  if (colours != (image_color != nullptr) || (colours && (!a->c || !b->c))) return LOD_EINVAL;
  if (((uintptr_t)workspace) & 255) return LOD_EINVAL;
  lodh::SplatLayout L;
  lod_status s = lodh::splat_layout(count, *cam, *sp, L, colours);
  if (s != LOD_OK) return s;
  if (workspace_bytes < L.total) return LOD_ENOMEM;
  lodh::InterpArgs ia{a->x, a->y, a->z, a->m, b->x, b->y, b->z, b->m, a->h, b->h, a->c, b->c, count, t};
  return lodh::launch_splat_interp(ia, *cam, *sp, workspace, L, image, image_color, (hipStream_t)stream);
}

lod_status lod_encode_motion(const lod_tree *tree, const float *x_next, const float *y_next, const float *z_next,
                             const uint64_t *snap_offsets, int16_t *dqx, int16_t *dqy, int16_t *dqz,
                             uint64_t *saturated, lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || !x_next || !y_next || !z_next || !dqx || !dqy || !dqz || !saturated)
    return LOD_EINVAL;
  return lodh::launch_encode_motion(*tree, x_next, y_next, z_next, snap_offsets, dqx, dqy, dqz, saturated,
                                    (hipStream_t)stream);
}

lod_status splat_render_lod_motion(const lod_tree *tree, const uint32_t *node_ids, const uint64_t *n_ids,
                                   uint64_t max_points, const int16_t *dqx, const int16_t *dqy, const int16_t *dqz,
                                   float t, const lod_camera *cam, const splat_params *sp, void *workspace,
                                   size_t workspace_bytes, float *image, lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || !node_ids || !n_ids || !dqx || !dqy || !dqz || !check_camera(cam, sp) || !image ||
      !workspace)
    return LOD_EINVAL;
  if (!(t >= 0.0f && t <= 1.0f)) return LOD_EINVAL;
  if (((uintptr_t)workspace) & 255) return LOD_EINVAL;
  lodh::LodDrawLayout D = lodh::lod_draw_layout(tree->node_capacity, max_points);
  lodh::SplatLayout L;
  lod_status s = lodh::splat_layout(D.max_points, *cam, *sp, L, false);
  if (s != LOD_OK) return s;
  if (workspace_bytes < D.total + L.total) return LOD_ENOMEM;
  return lodh::launch_splat_lod_motion(*tree, node_ids, n_ids, workspace, D, dqx, dqy, dqz, t, *cam, *sp, L, image,
                                       (hipStream_t)stream);
}

lod_status lod_set_node_points(const lod_tree *tree, uint32_t node, const float *x, const float *y, const float *z,
                               const float *m, uint32_t count, lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || (count && (!x || !y || !z || !m))) return LOD_EINVAL;
  if ((uint64_t)node >= tree->node_capacity) return LOD_EINVAL;
  return lodh::launch_set_points(*tree, node, x, y, z, m, count, (hipStream_t)stream);
}

lod_status lod_decode_plan(uint64_t node_capacity, size_t *workspace_bytes) {
  if (!workspace_bytes) return LOD_EINVAL;
  *workspace_bytes = lodh::decode_workspace(node_capacity);
  return LOD_OK;
}

lod_status lod_decode(const lod_tree *tree, const uint32_t *node_ids, const uint64_t *n_ids, uint64_t max_points,
                      float *x, float *y, float *z, float *m, uint64_t *n_points, void *workspace,
                      size_t workspace_bytes, lod_stream_t stream) {
  if (!tree_arrays_ok(tree) || !node_ids || !n_ids || !x || !y || !z || !m || !n_points || !workspace)
    return LOD_EINVAL;
  if (max_points == 0) return LOD_EINVAL;
  if (workspace_bytes < lodh::decode_workspace(tree->node_capacity)) return LOD_ENOMEM;
  return lodh::launch_decode(*tree, node_ids, n_ids, max_points, x, y, z, m, n_points, workspace,
                             (hipStream_t)stream);
}

lod_status splat_render_backward(const float *x, const float *y, const float *z, const float *m, uint64_t count,
                                 const lod_camera *cam, const splat_params *sp, const float *grad_image,
                                 float *grad_m, float *grad_x, float *grad_y, float *grad_z, lod_stream_t stream) {
  if (!check_camera(cam, sp) || !grad_image || !grad_m) return LOD_EINVAL;
  if (count && (!x || !y || !z || !m)) return LOD_EINVAL;
  return lodh::launch_splat_backward(x, y, z, m, count, *cam, *sp, grad_image, grad_m, grad_x, grad_y, grad_z,
                                     (hipStream_t)stream);
}

lod_status lod_workspace_view(const lod_input *in, const lod_params *p, void *workspace, uint32_t which,
                              void **device_ptr, uint64_t *count) {
  lod_status s = check_params(in, p);
  if (s != LOD_OK) return s;
  if (!workspace || !device_ptr || !count || which > 4) return LOD_EINVAL;
  const uint32_t ns = in->snap_offsets ? in->n_snapshots : 1;
  lodh::BuildLayout L = lodh::build_layout(in->n_particles, *p, ns);
  const int kb = lodh::key_bits(*p, ns);
  const int passes = kb > 8 ? (kb + 7) / 8 : 1;
  *device_ptr = lodh::workspace_view(workspace, L, which, in->n_particles, passes, count);
  return LOD_OK;
}

lod_status lod_autotune(const lod_input *in, lod_params *p, void *workspace, size_t workspace_bytes,
                        lod_tree *out, lod_params *cand, float *ms, uint32_t cap, uint32_t *n_cand,
                        lod_stream_t stream) {
  lod_status s = check_inputs(in, p);
  if (s != LOD_OK) return s;
  if (!tree_arrays_ok(out) || !workspace) return LOD_EINVAL;
  const uint32_t ns = in->snap_offsets ? in->n_snapshots : 1;
  lodh::BuildLayout L = lodh::build_layout(in->n_particles, *p, ns);
  if (workspace_bytes < L.total) return LOD_ENOMEM;
  if (out->node_capacity < L.node_cap || out->point_capacity < L.point_cap) return LOD_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return LOD_EDEVICE;
  std::vector<lod_params> cands;
  for (uint32_t thr : {256u, 512u, 1024u}) {
    lod_params c = *p; c.mode = 1; c.select_threads = thr; c.persistent_blocks = 0;
    cands.push_back(c);
    for (uint32_t per : {1u, 2u, 4u}) {
      lod_params c2 = *p; c2.mode = 2; c2.select_threads = thr; c2.persistent_blocks = per * (uint32_t)cus;
      cands.push_back(c2);
    }
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LOD_EDEVICE;
  float best = 1e30f;
  lod_params bestp = *p;
  uint32_t k = 0;
  lod_status rs = LOD_OK;
  for (const lod_params &c : cands) {
    if ((rs = lodh::launch_build(*in, c, workspace, L, *out, st)) != LOD_OK) break;   // warm-up
    if (hipEventRecord(e0, st) != hipSuccess) { rs = LOD_EDEVICE; break; }
    for (int r = 0; r < 2 && rs == LOD_OK; ++r) rs = lodh::launch_build(*in, c, workspace, L, *out, st);
    if (rs != LOD_OK) break;
    float t = 0.0f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      rs = LOD_EDEVICE;
      break;
    }
    t *= 0.5f;
    if (cand && ms && k < cap) { cand[k] = c; ms[k] = t; }
    ++k;
    if (t < best) { best = t; bestp = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (n_cand) *n_cand = k;
  if (rs != LOD_OK) return rs;
  p->mode = bestp.mode;
  p->select_threads = bestp.select_threads;
  p->persistent_blocks = bestp.persistent_blocks;
  return LOD_OK;
}

const char *lod_status_string(lod_status s) {
  switch (s) {
    case LOD_OK: return "ok";
    case LOD_EINVAL: return "invalid argument";
    case LOD_EDOMAIN: return "input outside the method's domain";
    case LOD_ENOMEM: return "workspace too small";
    case LOD_EDEVICE: return "HIP call failed";
    case LOD_ECAPACITY: return "output capacity below the bound";
    case LOD_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char *lod_version(void) { return "liblod 0.2 gfx950"; }

}  // extern "C"
