// Block store and view-dependent streaming: the paper's IO system (a
// spatially indexed store of octree-node blocks; only what a view needs is
// loaded, at the rate of an ordinary link; the CPU decides which blocks to
// load and draw, the GPU draws them).  Host code: the store is a file, the
// streamer keeps the node table on the host, a pool of node slots on the
// device (the caller's arrays) and draws the cut of the resident tree.
//
// Per frame f (credit, visit, groups, eviction as documented in lod.h):
// the visit from the roots descends into a node when the camera wants more
// detail there (the view-dependent cut's test) and all its children are
// resident; the children of visited nodes that want more detail form the
// candidate groups, loaded by priority while the link's credit lasts.
#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lod.h"
#include "lod_internal.hpp"

namespace {

constexpr char kMagic[8] = {'L', 'O', 'D', 'S', 'T', 'O', 'R', '1'};
constexpr uint32_t kVersion = 1;
constexpr uint64_t kBlockBytes = 14;   // per stored point: id 4, three codes 6, mass 4

struct StoreHeader {
  char magic[8];
  uint32_t version, n, reserved[2];
  uint64_t n_nodes, n_points, nodes_off, points_off;
  uint64_t pad;
};
static_assert(sizeof(StoreHeader) == 64, "store header is 64 bytes");

uint64_t align8(uint64_t v) { return (v + 7) & ~7ull; }

bool write_all(int fd, const void *p, size_t n, uint64_t off) {
  const char *c = (const char *)p;
  while (n) {
    const ssize_t w = pwrite(fd, c, n, (off_t)off);
    if (w <= 0) return false;
    c += w; n -= (size_t)w; off += (uint64_t)w;
  }
  return true;
}

bool read_all(int fd, void *p, size_t n, uint64_t off) {
  char *c = (char *)p;
  while (n) {
    const ssize_t r = pread(fd, c, n, (off_t)off);
    if (r <= 0) return false;
    c += r; n -= (size_t)r; off += (uint64_t)r;
  }
  return true;
}

template <class T>
bool d2h(std::vector<T> &v, const T *src, uint64_t n) {
  v.resize(n);
  return n == 0 || hipMemcpy(v.data(), src, n * sizeof(T), hipMemcpyDeviceToHost) == hipSuccess;
}

// cell coordinate of a Morton prefix (x in bit 0 of each triple)
uint32_t compact3_host(uint64_t v) {
  uint32_t c = 0;
  for (int k = 0; k < 21; ++k) c |= (uint32_t)((v >> (3 * k)) & 1u) << k;
  return c;
}

}  // namespace

struct lod_streamer {
  int fd = -1;
  uint32_t n = 0;
  uint64_t V = 0;
  std::vector<uint64_t> prefix, part_begin, part_count, block_off, pt_begin;
  std::vector<uint8_t> depth, child_mask;
  std::vector<uint32_t> parent, first_child, pt_count;
  std::vector<double> node_mass;
  std::vector<uint8_t> resident;
  std::vector<int64_t> used, wanted;
  std::vector<uint32_t> slot_of, free_slots, roots;
  uint32_t slots = 0;
  int64_t frame = -1;
  uint64_t credit = 0;
  lod_tree view{};
  char *staging = nullptr;        // pinned host: the frame's blocks
  size_t staging_bytes = 0;
  uint32_t *draw_host = nullptr;  // pinned host: the draw list

  lod_streamer() = default;
  lod_streamer(const lod_streamer &) = delete;
  lod_streamer &operator=(const lod_streamer &) = delete;
  ~lod_streamer() {
    if (fd >= 0) close(fd);
    if (staging) (void)hipHostFree(staging);
    if (draw_host) (void)hipHostFree(draw_host);
  }
};

namespace {

// The camera wants more detail in node v: the view-dependent cut's test
// (float64, in the same order as the device cut).
struct CutView {
  uint32_t proj, W;
  double px, py, pz, F, tau_cbrt, cbrt_n;
};

void node_box(const lod_streamer &s, uint64_t v, double &ox, double &oy, double &oz, double &side) {
  const int d = s.depth[v];
  side = std::ldexp(1.0, -d);
  const uint64_t cell = d ? (s.prefix[v] & ((1ull << (3 * d)) - 1)) : 0ull;
  ox = (double)compact3_host(cell) * side;
  oy = (double)compact3_host(cell >> 1) * side;
  oz = (double)compact3_host(cell >> 2) * side;
}

bool inside_box(const CutView &c, double ox, double oy, double oz, double side) {
  return (ox <= c.px && c.px <= ox + side) && (oy <= c.py && c.py <= oy + side) && (oz <= c.pz && c.pz <= oz + side);
}

double centre_dist(const CutView &c, double ox, double oy, double oz, double side) {
  const double h = side * 0.5;
  const double dx = (ox + h) - c.px, dy = (oy + h) - c.py, dz = (oz + h) - c.pz;
  return std::sqrt((dx * dx + dy * dy) + dz * dz);
}

bool wants_detail(const lod_streamer &s, uint64_t v, const CutView &c) {
  if (s.first_child[v] == LOD_NONE) return false;
  double ox, oy, oz, side;
  node_box(s, v, ox, oy, oz, side);
  if (c.proj == 0) return (double)c.W * side > c.tau_cbrt;
  if (inside_box(c, ox, oy, oz, side)) return true;
  return c.F * side > c.tau_cbrt * centre_dist(c, ox, oy, oz, side);
}

// Priority of a group (the children of v): camera inside v first, then v's
// projected point spacing, then smaller v.
struct Prio {
  int cls;
  double spacing;
  uint64_t v;
};
Prio group_priority(const lod_streamer &s, uint64_t v, const CutView &c) {
  double ox, oy, oz, side;
  node_box(s, v, ox, oy, oz, side);
  if (c.proj == 0) return Prio{1, (double)c.W * side / c.cbrt_n, v};
  if (inside_box(c, ox, oy, oz, side)) return Prio{2, 0.0, v};
  return Prio{1, c.F * side / (c.cbrt_n * centre_dist(c, ox, oy, oz, side)), v};
}

uint32_t n_children(const lod_streamer &s, uint64_t v) {
  return s.first_child[v] == LOD_NONE ? 0u : (uint32_t)__builtin_popcount(s.child_mask[v]);
}

bool all_children_resident(const lod_streamer &s, uint64_t v) {
  const uint32_t k = n_children(s, v);
  for (uint32_t i = 0; i < k; ++i)
    if (!s.resident[s.first_child[v] + i]) return false;
  return true;
}

// Visit from the roots; returns the draw list (sorted) and the visited nodes.
void visit(const lod_streamer &s, const std::vector<uint8_t> &desc, std::vector<uint32_t> &draw,
           std::vector<uint32_t> *visited) {
  draw.clear();
  if (visited) visited->clear();
  std::vector<uint32_t> stack(s.roots.rbegin(), s.roots.rend());
  while (!stack.empty()) {
    const uint32_t v = stack.back();
    stack.pop_back();
    if (visited) visited->push_back(v);
    const uint32_t k = n_children(s, v);
    if (desc[v] && k && all_children_resident(s, v)) {
      for (uint32_t i = k; i-- > 0;) stack.push_back(s.first_child[v] + i);
    } else {
      draw.push_back(v);
    }
  }
  std::sort(draw.begin(), draw.end());
}

int64_t pick_victim(const lod_streamer &s, int64_t f) {
  int64_t best = -1;
  for (uint64_t v = 0; v < s.V; ++v) {
    if (!s.resident[v] || s.parent[v] == LOD_NONE) continue;
    if (s.used[v] >= f || s.wanted[s.parent[v]] >= f) continue;
    bool kids = false;
    const uint32_t k = n_children(s, v);
    for (uint32_t i = 0; i < k && !kids; ++i) kids = s.resident[s.first_child[v] + i];
    if (kids) continue;
    // least recently used first; ties: larger node index first
    if (best < 0 || s.used[v] < s.used[best] || (s.used[v] == s.used[best] && (int64_t)v > best)) best = (int64_t)v;
  }
  return best;
}

uint64_t file_bytes(int fd) {
  struct stat st;
  return fstat(fd, &st) == 0 && st.st_size > 0 ? (uint64_t)st.st_size : 0;
}

// A node table read from a file is trusted only as far as this check goes:
// every index in range, each node the parent of exactly its children (which
// follow it: the visit terminates), at most n points per node, depths that fit
// the 64-bit prefix, and every block inside the file.
bool node_table_ok(const lod_streamer &s, uint64_t file_size) {
  const uint64_t V = s.V;
  if (s.n == 0 || V == 0 || V >= LOD_NONE) return false;
  for (uint64_t v = 0; v < V; ++v) {
    if (s.pt_count[v] > s.n || s.depth[v] > 21) return false;
    if (s.parent[v] != LOD_NONE && (s.parent[v] >= v || s.depth[v] != s.depth[s.parent[v]] + 1)) return false;
    if (s.parent[v] == LOD_NONE && s.depth[v] != 0) return false;
    const uint32_t k = (uint32_t)__builtin_popcount(s.child_mask[v]);
    if ((k == 0) != (s.first_child[v] == LOD_NONE)) return false;
    if (k) {
      const uint64_t c0 = s.first_child[v];
      if (c0 <= v || c0 + k > V) return false;
      for (uint32_t i = 0; i < k; ++i)
        if (s.parent[c0 + i] != v) return false;
    }
    const uint64_t b = s.block_off[v], bytes = kBlockBytes * s.pt_count[v];
    if (b > file_size || bytes > file_size - b) return false;
  }
  return true;
}

lod_status ensure_staging(lod_streamer &s, size_t bytes) {
  if (bytes <= s.staging_bytes) return LOD_OK;
  if (s.staging) (void)hipHostFree(s.staging);
  s.staging = nullptr;
  s.staging_bytes = 0;
  if (hipHostMalloc((void **)&s.staging, bytes) != hipSuccess) return LOD_EDEVICE;
  s.staging_bytes = bytes;
  return LOD_OK;
}

}  // namespace

extern "C" {

lod_status lod_store_save(const lod_tree *tree, uint32_t n, const char *path, lod_stream_t stream) {
  if (!tree || !tree->counts || !path || n == 0) return LOD_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return LOD_EDEVICE;
  uint64_t cnt[3];
  if (hipMemcpy(cnt, tree->counts, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess) return LOD_EDEVICE;
  if (cnt[2] != 0) return LOD_EINVAL;            // the build reported an error: its outputs are undefined
  const uint64_t V = cnt[0], S = cnt[1];
  std::vector<uint64_t> prefix, part_begin, part_count, pt_begin;
  std::vector<uint8_t> depth, child_mask;
  std::vector<uint32_t> parent, first_child, pt_count, pt_id;
  std::vector<double> node_mass;
  std::vector<uint16_t> qx, qy, qz;
  std::vector<float> pt_mass;
  if (!d2h(prefix, tree->prefix, V) || !d2h(depth, tree->depth, V) || !d2h(parent, tree->parent, V) ||
      !d2h(first_child, tree->first_child, V) || !d2h(child_mask, tree->child_mask, V) ||
      !d2h(part_begin, tree->part_begin, V) || !d2h(part_count, tree->part_count, V) ||
      !d2h(pt_begin, tree->pt_begin, V) || !d2h(pt_count, tree->pt_count, V) ||
      !d2h(node_mass, tree->node_mass, V) || !d2h(pt_id, tree->pt_id, S) || !d2h(qx, tree->qx, S) ||
      !d2h(qy, tree->qy, S) || !d2h(qz, tree->qz, S) || !d2h(pt_mass, tree->pt_mass, S))
    return LOD_EDEVICE;
  for (uint64_t v = 0; v < V; ++v)
    if (pt_count[v] > n) return LOD_EINVAL;
  StoreHeader h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = kVersion;
  h.n = n;
  h.n_nodes = V;
  h.n_points = S;
  h.nodes_off = sizeof(StoreHeader);
  // node section: prefix, depth, parent, first_child, child_mask, part_begin,
  // part_count, pt_count, node_mass, block_off (each array 8-byte aligned)
  const uint64_t sizes[10] = {8 * V, V, 4 * V, 4 * V, V, 8 * V, 8 * V, 4 * V, 8 * V, 8 * V};
  uint64_t off = h.nodes_off, offs[10];
  for (int i = 0; i < 10; ++i) { offs[i] = off; off = align8(off + sizes[i]); }
  h.points_off = off;
  std::vector<uint64_t> block_off(V);
  uint64_t b = h.points_off;
  for (uint64_t v = 0; v < V; ++v) { block_off[v] = b; b += kBlockBytes * pt_count[v]; }
  const int fd = open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (fd < 0) return LOD_EINVAL;
  bool ok = write_all(fd, &h, sizeof(h), 0);
  const void *arrs[10] = {prefix.data(), depth.data(), parent.data(), first_child.data(), child_mask.data(),
                          part_begin.data(), part_count.data(), pt_count.data(), node_mass.data(), block_off.data()};
  for (int i = 0; i < 10 && ok; ++i) ok = write_all(fd, arrs[i], sizes[i], offs[i]);
  std::vector<char> blk;
  for (uint64_t v = 0; v < V && ok; ++v) {
    const uint64_t k = pt_count[v], p0 = pt_begin[v];
    blk.resize(kBlockBytes * k);
    char *q = blk.data();
    std::memcpy(q, pt_id.data() + p0, 4 * k); q += 4 * k;
    std::memcpy(q, qx.data() + p0, 2 * k); q += 2 * k;
    std::memcpy(q, qy.data() + p0, 2 * k); q += 2 * k;
    std::memcpy(q, qz.data() + p0, 2 * k); q += 2 * k;
    std::memcpy(q, pt_mass.data() + p0, 4 * k);
    ok = write_all(fd, blk.data(), blk.size(), block_off[v]);
  }
  if (close(fd) != 0) ok = false;
  return ok ? LOD_OK : LOD_EINVAL;
}

lod_status lod_store_read_info(const char *path, uint64_t *n_nodes, uint64_t *n_points, uint32_t *n) {
  if (!path || !n_nodes || !n_points || !n) return LOD_EINVAL;
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return LOD_EINVAL;
  StoreHeader h{};
  const bool ok = read_all(fd, &h, sizeof(h), 0) && std::memcmp(h.magic, kMagic, 8) == 0 && h.version == kVersion;
  close(fd);
  if (!ok) return LOD_EINVAL;
  *n_nodes = h.n_nodes;
  *n_points = h.n_points;
  *n = h.n;
  return LOD_OK;
}

lod_status lod_streamer_open(const char *path, uint32_t pool_slots, lod_tree *view, lod_streamer **out) {
  if (!path || !view || !out || pool_slots == 0) return LOD_EINVAL;
  *out = nullptr;
  if (!view->prefix || !view->depth || !view->parent || !view->first_child || !view->child_mask ||
      !view->part_begin || !view->part_count || !view->pt_begin || !view->pt_count || !view->node_mass ||
      !view->pt_id || !view->qx || !view->qy || !view->qz || !view->pt_mass || !view->counts)
    return LOD_EINVAL;
  lod_streamer *s = new lod_streamer();
  auto fail = [&](lod_status st) {
    delete s;   // closes the file and frees the pinned buffers
    return st;
  };
  s->fd = open(path, O_RDONLY);
  if (s->fd < 0) return fail(LOD_EINVAL);
  StoreHeader h{};
  if (!read_all(s->fd, &h, sizeof(h), 0) || std::memcmp(h.magic, kMagic, 8) != 0 || h.version != kVersion)
    return fail(LOD_EINVAL);
  const uint64_t V = h.n_nodes;
  s->V = V;
  s->n = h.n;
  s->slots = pool_slots;
  if (view->node_capacity < V || view->point_capacity < (uint64_t)pool_slots * h.n) return fail(LOD_ECAPACITY);
  s->prefix.resize(V); s->depth.resize(V); s->parent.resize(V); s->first_child.resize(V); s->child_mask.resize(V);
  s->part_begin.resize(V); s->part_count.resize(V); s->pt_count.resize(V); s->node_mass.resize(V);
  s->block_off.resize(V);
  const uint64_t sizes[10] = {8 * V, V, 4 * V, 4 * V, V, 8 * V, 8 * V, 4 * V, 8 * V, 8 * V};
  void *arrs[10] = {s->prefix.data(), s->depth.data(), s->parent.data(), s->first_child.data(),
                    s->child_mask.data(), s->part_begin.data(), s->part_count.data(), s->pt_count.data(),
                    s->node_mass.data(), s->block_off.data()};
  uint64_t off = h.nodes_off;
  for (int i = 0; i < 10; ++i) {
    if (!read_all(s->fd, arrs[i], sizes[i], off)) return fail(LOD_EINVAL);
    off = align8(off + sizes[i]);
  }
  if (!node_table_ok(*s, file_bytes(s->fd))) return fail(LOD_EINVAL);
  s->resident.assign(V, 0);
  s->used.assign(V, -1);
  s->wanted.assign(V, -1);
  s->slot_of.assign(V, LOD_NONE);
  s->pt_begin.assign(V, 0);
  for (uint32_t i = pool_slots; i-- > 0;) s->free_slots.push_back(i);
  for (uint64_t v = 0; v < V; ++v)
    if (s->parent[v] == LOD_NONE) s->roots.push_back((uint32_t)v);
  if (s->roots.size() > pool_slots) return fail(LOD_ECAPACITY);
  s->view = *view;
  // the node table, once
  const lod_tree &t = s->view;
  bool ok = hipMemcpy(t.prefix, s->prefix.data(), 8 * V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.depth, s->depth.data(), V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.parent, s->parent.data(), 4 * V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.first_child, s->first_child.data(), 4 * V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.child_mask, s->child_mask.data(), V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.part_begin, s->part_begin.data(), 8 * V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.part_count, s->part_count.data(), 8 * V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.pt_count, s->pt_count.data(), 4 * V, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t.node_mass, s->node_mass.data(), 8 * V, hipMemcpyHostToDevice) == hipSuccess;
  const uint64_t counts[3] = {V, (uint64_t)pool_slots * s->n, 0};
  ok = ok && hipMemcpy(t.counts, counts, sizeof(counts), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) return fail(LOD_EDEVICE);
  if (hipHostMalloc((void **)&s->draw_host, 4 * std::max<uint64_t>(1, V)) != hipSuccess) return fail(LOD_EDEVICE);
  // the roots, once (never evicted)
  uint64_t root_bytes = 0;
  for (uint32_t r : s->roots) root_bytes += kBlockBytes * s->pt_count[r];
  if (ensure_staging(*s, std::max<uint64_t>(root_bytes, 1)) != LOD_OK) return fail(LOD_EDEVICE);
  uint64_t so = 0;
  for (uint32_t r : s->roots) {
    const uint64_t k = s->pt_count[r];
    const uint32_t slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->slot_of[r] = slot;
    s->resident[r] = 1;
    s->pt_begin[r] = (uint64_t)slot * s->n;
    if (!read_all(s->fd, s->staging + so, kBlockBytes * k, s->block_off[r])) return fail(LOD_EINVAL);
    const char *q = s->staging + so;
    const uint64_t d0 = s->pt_begin[r];
    ok = ok && hipMemcpy(t.pt_id + d0, q, 4 * k, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(t.qx + d0, q + 4 * k, 2 * k, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(t.qy + d0, q + 6 * k, 2 * k, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(t.qz + d0, q + 8 * k, 2 * k, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(t.pt_mass + d0, q + 10 * k, 4 * k, hipMemcpyHostToDevice) == hipSuccess;
    so += kBlockBytes * k;
  }
  ok = ok && hipMemcpy(t.pt_begin, s->pt_begin.data(), 8 * V, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) return fail(LOD_EDEVICE);
  *out = s;
  return LOD_OK;
}

lod_status lod_streamer_frame(lod_streamer *s, const lod_camera *cam, float tau_px, uint64_t budget_bytes,
                              uint32_t *draw_ids, uint64_t *n_draw, lod_stream_stats *stats, uint32_t *loaded_ids,
                              uint32_t loaded_cap, uint32_t *evicted_ids, uint32_t evicted_cap,
                              lod_stream_t stream) {
  if (!s || !cam || !draw_ids || !n_draw || !stats) return LOD_EINVAL;
  if (!(tau_px > 0.0f) || !std::isfinite(tau_px) || cam->projection > 1) return LOD_EINVAL;
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  hipStream_t st = (hipStream_t)stream;
  lod_stream_stats out{};
  const int64_t f = ++s->frame;
  const uint64_t cap = budget_bytes + 8ull * s->n * kBlockBytes;
  s->credit = std::min<uint64_t>(s->credit + budget_bytes, cap);
  CutView c{};
  c.proj = cam->projection; c.W = cam->W;
  c.px = (double)cam->pos[0]; c.py = (double)cam->pos[1]; c.pz = (double)cam->pos[2];
  c.F = (double)cam->F;
  c.cbrt_n = std::cbrt((double)s->n);
  c.tau_cbrt = (double)tau_px * c.cbrt_n;
  std::vector<uint8_t> desc(s->V);
  for (uint64_t v = 0; v < s->V; ++v) desc[v] = wants_detail(*s, v, c) ? 1 : 0;
  std::vector<uint32_t> draw, visited;
  visit(*s, desc, draw, &visited);
  std::vector<uint32_t> groups;
  for (uint32_t v : visited) {
    s->used[v] = f;
    if (desc[v]) {
      s->wanted[v] = f;
      if (n_children(*s, v) && !all_children_resident(*s, v)) groups.push_back(v);
    }
  }
  std::vector<Prio> pr;
  pr.reserve(groups.size());
  for (uint32_t g : groups) pr.push_back(group_priority(*s, g, c));
  std::sort(pr.begin(), pr.end(), [](const Prio &a, const Prio &b) {
    if (a.cls != b.cls) return a.cls > b.cls;
    if (a.spacing != b.spacing) return a.spacing > b.spacing;
    return a.v < b.v;
  });
  uint64_t left = s->credit;
  std::vector<uint32_t> loaded;
  uint32_t n_evicted = 0;
  bool stop = false;
  size_t gi = 0;
  for (; gi < pr.size() && !stop; ++gi) {
    const uint64_t g = pr[gi].v;
    std::vector<uint32_t> need;
    uint64_t cost = 0;
    for (uint32_t i = 0; i < n_children(*s, g); ++i) {
      const uint32_t ch = s->first_child[g] + i;
      if (!s->resident[ch]) { need.push_back(ch); cost += kBlockBytes * s->pt_count[ch]; }
    }
    if (cost > left) break;
    while (s->free_slots.size() < need.size()) {
      const int64_t vic = pick_victim(*s, f);
      if (vic < 0) break;
      s->resident[vic] = 0;
      s->free_slots.push_back(s->slot_of[vic]);
      s->slot_of[vic] = LOD_NONE;
      if (evicted_ids && n_evicted < evicted_cap) evicted_ids[n_evicted] = (uint32_t)vic;
      ++n_evicted;
    }
    if (s->free_slots.size() < need.size()) { stop = true; break; }
    for (uint32_t ch : need) {
      const uint32_t slot = s->free_slots.back();
      s->free_slots.pop_back();
      s->slot_of[ch] = slot;
      s->resident[ch] = 1;
      s->pt_begin[ch] = (uint64_t)slot * s->n;
      loaded.push_back(ch);
    }
    left -= cost;
  }
  out.groups_waiting = (uint32_t)(pr.size() - gi);
  const uint64_t spent = s->credit - left;
  s->credit = left;
  const auto t1 = clk::now();
  // read the loaded blocks into the pinned staging buffer, then copy them to
  // their slots and publish the new slot offsets
  lod_status rs = ensure_staging(*s, std::max<uint64_t>(spent, 1));
  if (rs != LOD_OK) return rs;
  uint64_t so = 0;
  const lod_tree &t = s->view;
  bool ok = true;
  for (uint32_t v : loaded) {
    const uint64_t k = s->pt_count[v];
    ok = ok && read_all(s->fd, s->staging + so, kBlockBytes * k, s->block_off[v]);
    so += kBlockBytes * k;
  }
  const auto t2 = clk::now();
  if (!ok) return LOD_EINVAL;
  so = 0;
  for (uint32_t v : loaded) {
    const uint64_t k = s->pt_count[v], d0 = s->pt_begin[v];
    const char *q = s->staging + so;
    ok = ok && hipMemcpyAsync(t.pt_id + d0, q, 4 * k, hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(t.qx + d0, q + 4 * k, 2 * k, hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(t.qy + d0, q + 6 * k, 2 * k, hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(t.qz + d0, q + 8 * k, 2 * k, hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(t.pt_mass + d0, q + 10 * k, 4 * k, hipMemcpyHostToDevice, st) == hipSuccess;
    so += kBlockBytes * k;
  }
  ok = ok && hipMemcpyAsync(t.pt_begin, s->pt_begin.data(), 8 * s->V, hipMemcpyHostToDevice, st) == hipSuccess;
  // the frame draws the cut of the new resident tree
  visit(*s, desc, draw, nullptr);
  uint64_t pts = 0;
  for (size_t i = 0; i < draw.size(); ++i) { s->draw_host[i] = draw[i]; pts += s->pt_count[draw[i]]; }
  const uint64_t nd = draw.size();
  ok = ok && hipMemcpyAsync(draw_ids, s->draw_host, 4 * std::max<uint64_t>(nd, 1), hipMemcpyHostToDevice, st) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(n_draw, &nd, sizeof(nd), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;   // staging and draw list are reused next frame
  if (!ok) return LOD_EDEVICE;
  const auto t3 = clk::now();
  for (size_t i = 0; i < loaded.size() && loaded_ids && i < loaded_cap; ++i) loaded_ids[i] = loaded[i];
  out.bytes_loaded = spent;
  out.nodes_loaded = (uint32_t)loaded.size();
  out.nodes_evicted = n_evicted;
  out.nodes_drawn = (uint32_t)nd;
  out.points_drawn = pts;
  uint64_t res = 0;
  for (uint64_t v = 0; v < s->V; ++v) res += s->resident[v];
  out.resident_nodes = res;
  out.decide_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  out.io_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
  out.upload_ms = std::chrono::duration<double, std::milli>(t3 - t2).count();
  *stats = out;
  return LOD_OK;
}

lod_status lod_streamer_close(lod_streamer *s) {
  if (!s) return LOD_EINVAL;
  delete s;
  return LOD_OK;
}

}  // extern "C"
