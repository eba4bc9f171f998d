// Host-side checks of the C-ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer against a build of the library whose host pass
// carries the same sanitizers: every entry point rejects bad arguments before it enqueues
// work, the plans stay in range at extreme sizes, and store files that are
// missing, truncated or corrupted are refused without reading or writing out
// of bounds.  Runs without a GPU; calls that would reach the device report an
// error instead.  Usage: abi_sanitize <scratch directory>.
#include <fcntl.h>
#include <unistd.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lod.h"

static int failures = 0;
#define EXPECT(cond)                                                        \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static lod_camera ortho(uint32_t W, uint32_t H) {
  lod_camera c{};
  c.projection = 0; c.W = W; c.H = H;
  c.right[0] = 1; c.up[1] = 1; c.fwd[2] = 1; c.F = 1; c.near_z = 0;
  return c;
}

static splat_params gaussian() {
  splat_params p{};
  p.sigma_px = 1.0f; p.radius_sigmas = 3.0f; p.blob = LOD_BLOB_GAUSSIAN;
  return p;
}

static lod_params params(uint32_t n, uint32_t D) {
  lod_params p{};
  p.n = n; p.max_depth = D; p.density_level = D; p.alpha = 1; p.mode = 1;
  return p;
}

// Every entry point with missing pointers or out-of-range values.
static void null_arguments() {
  lod_camera cam = ortho(64, 64);
  splat_params sp = gaussian();
  lod_params p = params(16, 4);
  lod_input in{};
  lod_tree tree{};
  size_t ws = 0;
  uint64_t a = 0, b = 0;
  uint32_t u = 0;
  EXPECT(lod_build_plan(nullptr, &p, &ws, &a, &b) == LOD_EINVAL);
  EXPECT(lod_build_plan(&in, nullptr, &ws, &a, &b) == LOD_EINVAL);
  EXPECT(lod_build_plan(&in, &p, nullptr, &a, &b) == LOD_EINVAL);
  EXPECT(lod_build(nullptr, &p, nullptr, 0, &tree, nullptr) == LOD_EINVAL);
  EXPECT(lod_build(&in, &p, nullptr, 0, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(lod_select_plan(16, nullptr) == LOD_EINVAL);
  EXPECT(lod_select(nullptr, &cam, 1.0f, 16, nullptr, 0, nullptr, nullptr, 0, nullptr) == LOD_EINVAL);
  EXPECT(lod_select(&tree, &cam, 1.0f, 16, nullptr, 0, nullptr, nullptr, 0, nullptr) == LOD_EINVAL);
  EXPECT(splat_plan(16, nullptr, &sp, &ws) == LOD_EINVAL);
  EXPECT(splat_plan(16, &cam, nullptr, &ws) == LOD_EINVAL);
  EXPECT(splat_plan(16, &cam, &sp, nullptr) == LOD_EINVAL);
  EXPECT(splat_render(nullptr, nullptr, nullptr, nullptr, 16, &cam, &sp, nullptr, 0, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(splat_render_aux(nullptr, nullptr, nullptr, nullptr, nullptr, 16, &cam, &sp, nullptr, 0, nullptr, nullptr,
                          nullptr) == LOD_EINVAL);
  EXPECT(splat_lod_plan(16, 16, nullptr, &sp, &ws) == LOD_EINVAL);
  EXPECT(splat_render_lod(nullptr, nullptr, nullptr, 16, &cam, &sp, nullptr, 0, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(lod_highlight_flags(nullptr, nullptr, 0, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(splat_lod_highlight_plan(16, 16, 0, &cam, &sp, &ws) == LOD_EINVAL);
  EXPECT(splat_render_lod_highlight(nullptr, nullptr, nullptr, 16, &cam, &sp, nullptr, 1, nullptr, 0, nullptr,
                                    nullptr, nullptr) == LOD_EINVAL);
  EXPECT(splat_render_interp(nullptr, nullptr, 16, 0.5f, &cam, &sp, nullptr, 0, nullptr, nullptr, nullptr) ==
         LOD_EINVAL);
  splat_frame fa{}, fb{};
  EXPECT(splat_render_interp(&fa, &fb, 16, 1.5f, &cam, &sp, nullptr, 0, nullptr, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(lod_encode_motion(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr) == LOD_EINVAL);
  EXPECT(splat_render_lod_motion(nullptr, nullptr, nullptr, 16, nullptr, nullptr, nullptr, 0.5f, &cam, &sp, nullptr,
                                 0, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(lod_set_node_points(nullptr, 0, nullptr, nullptr, nullptr, nullptr, 1, nullptr) == LOD_EINVAL);
  EXPECT(lod_decode_plan(16, nullptr) == LOD_EINVAL);
  EXPECT(lod_decode(nullptr, nullptr, nullptr, 16, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                    nullptr) == LOD_EINVAL);
  EXPECT(splat_render_backward(nullptr, nullptr, nullptr, nullptr, 16, &cam, &sp, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr) == LOD_EINVAL);
  EXPECT(splat_render_noalloc(nullptr, nullptr, nullptr, nullptr, 16, &cam, &sp, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(lod_store_save(nullptr, 16, "x", nullptr) == LOD_EINVAL);
  EXPECT(lod_store_read_info(nullptr, &a, &b, &u) == LOD_EINVAL);
  EXPECT(lod_streamer_open(nullptr, 4, &tree, nullptr) == LOD_EINVAL);
  lod_stream_stats st{};
  EXPECT(lod_streamer_frame(nullptr, &cam, 1.0f, 0, &u, &a, &st, nullptr, 0, nullptr, 0, nullptr) == LOD_EINVAL);
  EXPECT(lod_streamer_close(nullptr) == LOD_EINVAL);
  EXPECT(lod_autotune(nullptr, &p, nullptr, 0, &tree, nullptr, nullptr, 0, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(lod_workspace_view(nullptr, &p, nullptr, 0, nullptr, nullptr) == LOD_EINVAL);
  EXPECT(lod_trace_end(nullptr, 0, nullptr) == LOD_EINVAL);
  for (int s = 1; s >= -8; --s) EXPECT(lod_status_string((lod_status)s) != nullptr);
  EXPECT(lod_version() != nullptr && std::strlen(lod_version()) > 0);
}

// Plans at the edges of their ranges: no overflow, the documented codes.
static void plan_ranges() {
  lod_input in{};
  size_t ws = 0;
  uint64_t nc = 0, pc = 0;
  lod_params p = params(16, 4);
  in.n_particles = 0;
  EXPECT(lod_build_plan(&in, &p, &ws, &nc, &pc) == LOD_OK);
  in.n_particles = 1000;
  EXPECT(lod_build_plan(&in, &p, &ws, &nc, &pc) == LOD_OK && ws > 0 && nc >= 1 && pc >= 1000);
  lod_params q = p; q.n = 0;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EINVAL);
  q = p; q.max_depth = 11; q.density_level = 11;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EINVAL);
  q = p; q.density_level = 5;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EINVAL);
  q = p; q.alpha = 2;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EINVAL);
  q = p; q.select_threads = 100;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EINVAL);
  q = p; q.reserved = 1;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EINVAL);
  q = p; q.mode = 3;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EINVAL);
  // 10 levels (30 key bits) and 8 snapshot bits exceed the 32-bit key
  q = params(16, 10);
  in.n_snapshots = 256;
  uint64_t dummy_offsets = 0;
  in.snap_offsets = &dummy_offsets;
  EXPECT(lod_build_plan(&in, &q, &ws, &nc, &pc) == LOD_EUNSUPPORTED);
  in.snap_offsets = nullptr; in.n_snapshots = 0;
  // more particles than a 32-bit sorted position can name
  in.n_particles = 1ull << 40;
  EXPECT(lod_build_plan(&in, &p, &ws, &nc, &pc) != LOD_OK);
  in.n_particles = ~0ull;
  EXPECT(lod_build_plan(&in, &p, &ws, &nc, &pc) != LOD_OK);

  EXPECT(lod_select_plan(0, &ws) == LOD_OK);
  EXPECT(lod_select_plan(1u << 30, &ws) == LOD_OK);
  EXPECT(lod_decode_plan(1u << 30, &ws) == LOD_OK);

  lod_camera cam = ortho(1024, 1024);
  splat_params sp = gaussian();
  EXPECT(splat_plan(0, &cam, &sp, &ws) == LOD_OK);
  EXPECT(splat_plan(1000000, &cam, &sp, &ws) == LOD_OK && ws > 0);
  EXPECT(splat_plan(1ull << 40, &cam, &sp, &ws) == LOD_EUNSUPPORTED);   // pair counts past 32 bits
  EXPECT(splat_plan(~0ull, &cam, &sp, &ws) == LOD_EUNSUPPORTED);
  EXPECT(splat_plan(1ull << 62, &cam, &sp, &ws) == LOD_EUNSUPPORTED);   // points x 4 tiles wraps to 0
  lod_camera big = ortho(16384, 16384);                                  // more tiles than supported
  EXPECT(splat_plan(16, &big, &sp, &ws) == LOD_EUNSUPPORTED);
  lod_camera wide = ortho(16385, 64);                                    // past the camera's range
  EXPECT(splat_plan(16, &wide, &sp, &ws) == LOD_EINVAL);
  lod_camera zero = ortho(0, 64);
  EXPECT(splat_plan(16, &zero, &sp, &ws) == LOD_EINVAL);
  splat_params bad = sp; bad.sigma_px = 0.0f;
  EXPECT(splat_plan(16, &cam, &bad, &ws) == LOD_EINVAL);
  bad = sp; bad.sigma_px = 9.0f;
  EXPECT(splat_plan(16, &cam, &bad, &ws) == LOD_EINVAL);
  bad = sp; bad.radius_sigmas = 7.0f;
  EXPECT(splat_plan(16, &cam, &bad, &ws) == LOD_EINVAL);
  bad = sp; bad.blob = 7;
  EXPECT(splat_plan(16, &cam, &bad, &ws) == LOD_EINVAL);
  bad = sp; bad.blob = LOD_BLOB_CUBIC; bad.h_px = 0.0f;
  EXPECT(splat_plan(16, &cam, &bad, &ws) == LOD_EINVAL);
  bad.h_px = 17.0f;
  EXPECT(splat_plan(16, &cam, &bad, &ws) == LOD_EINVAL);
  bad.h_px = 1.5f;
  EXPECT(splat_plan(16, &cam, &bad, &ws) == LOD_OK);
  lod_camera persp = cam; persp.projection = 2;
  EXPECT(splat_plan(16, &persp, &sp, &ws) == LOD_EINVAL);
  EXPECT(splat_lod_plan(1u << 20, 1000000, &cam, &sp, &ws) == LOD_OK);
  EXPECT(splat_lod_plan(1u << 20, ~0ull, &cam, &sp, &ws) == LOD_EUNSUPPORTED);
  EXPECT(splat_lod_plan(1u << 20, 1ull << 62, &cam, &sp, &ws) == LOD_EUNSUPPORTED);
  EXPECT(splat_lod_highlight_plan(1u << 20, 1000000, 1000, &cam, &sp, &ws) == LOD_OK);
  EXPECT(splat_lod_highlight_plan(1u << 20, 1000000, ~0ull, &cam, &sp, &ws) != LOD_OK);
}

// ---- store files ---------------------------------------------------------

struct Store {
  uint32_t n = 4;
  std::vector<uint64_t> prefix, part_begin, part_count, block_off;
  std::vector<uint8_t> depth, child_mask;
  std::vector<uint32_t> parent, first_child, pt_count;
  std::vector<double> node_mass;
};

// A root holding n points and two leaf children holding two points each.
static Store small_store() {
  Store s;
  s.prefix = {0, 0, 7};
  s.depth = {0, 1, 1};
  s.parent = {LOD_NONE, 0, 0};
  s.first_child = {1, LOD_NONE, LOD_NONE};
  s.child_mask = {0x81, 0, 0};
  s.part_begin = {0, 0, 2};
  s.part_count = {s.n + 1ull, 2, 2};
  s.pt_count = {s.n, 2, 2};
  s.node_mass = {4.0, 2.0, 2.0};
  return s;
}

static uint64_t a8(uint64_t v) { return (v + 7) & ~7ull; }

// Writes the store; header fields can be overridden for corrupted files.
static bool write_store(const std::string &path, Store s, uint32_t version = 1, const char *magic = "LODSTOR1",
                        bool truncate_blocks = false, uint64_t nodes_off_override = 0) {
  const uint64_t V = s.parent.size();
  uint64_t npts = 0;
  for (uint32_t c : s.pt_count) npts += c;
  const uint64_t sizes[10] = {8 * V, V, 4 * V, 4 * V, V, 8 * V, 8 * V, 4 * V, 8 * V, 8 * V};
  uint64_t offs[10], off = 64;
  for (int i = 0; i < 10; ++i) { offs[i] = off; off = a8(off + sizes[i]); }
  const uint64_t points_off = off;
  if (s.block_off.empty()) {
    uint64_t b = points_off;
    for (uint64_t v = 0; v < V; ++v) { s.block_off.push_back(b); b += 14ull * s.pt_count[v]; }
  }
  std::vector<char> file(points_off + 14 * npts, 0);
  std::memcpy(file.data(), magic, 8);
  uint32_t h32[4] = {version, s.n, 0, 0};
  std::memcpy(file.data() + 8, h32, 16);
  uint64_t h64[5] = {V, npts, nodes_off_override ? nodes_off_override : 64, points_off, 0};
  std::memcpy(file.data() + 24, h64, 40);
  const void *arrs[10] = {s.prefix.data(), s.depth.data(), s.parent.data(), s.first_child.data(),
                          s.child_mask.data(), s.part_begin.data(), s.part_count.data(), s.pt_count.data(),
                          s.node_mass.data(), s.block_off.data()};
  for (int i = 0; i < 10; ++i) std::memcpy(file.data() + offs[i], arrs[i], sizes[i]);
  for (uint64_t k = 0; k < npts; ++k) file[points_off + 14 * k] = (char)k;
  if (truncate_blocks) file.resize(points_off + 3);
  const int fd = open(path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (fd < 0) return false;
  const bool ok = write(fd, file.data(), file.size()) == (ssize_t)file.size();
  return close(fd) == 0 && ok;
}

// Host buffers standing in for the view's device arrays: a file is checked
// before anything is copied to them.
struct HostView {
  std::vector<uint64_t> prefix, part_begin, part_count, pt_begin, counts;
  std::vector<uint8_t> depth, child_mask;
  std::vector<uint32_t> parent, first_child, pt_count, pt_id;
  std::vector<double> node_mass;
  std::vector<uint16_t> qx, qy, qz;
  std::vector<float> pt_mass;
  lod_tree t{};
  HostView(uint64_t nodes, uint64_t points) {
    prefix.resize(nodes); part_begin.resize(nodes); part_count.resize(nodes); pt_begin.resize(nodes);
    depth.resize(nodes); child_mask.resize(nodes); parent.resize(nodes); first_child.resize(nodes);
    pt_count.resize(nodes); node_mass.resize(nodes); counts.resize(3);
    pt_id.resize(points); qx.resize(points); qy.resize(points); qz.resize(points); pt_mass.resize(points);
    t = lod_tree{prefix.data(), depth.data(), parent.data(), first_child.data(), child_mask.data(),
                 part_begin.data(), part_count.data(), pt_begin.data(), pt_count.data(), node_mass.data(),
                 pt_id.data(), qx.data(), qy.data(), qz.data(), pt_mass.data(), nodes, points, counts.data()};
  }
};

static lod_status open_close(const std::string &path, uint32_t slots, HostView &hv) {
  lod_streamer *s = nullptr;
  const lod_status r = lod_streamer_open(path.c_str(), slots, &hv.t, &s);
  if (r == LOD_OK) {
    EXPECT(s != nullptr);
    EXPECT(lod_streamer_close(s) == LOD_OK);
  } else {
    EXPECT(s == nullptr);
  }
  return r;
}

static void store_files(const std::string &dir) {
  const std::string good = dir + "/good.lodstore";
  EXPECT(write_store(good, small_store()));
  uint64_t V = 0, S = 0;
  uint32_t n = 0;
  EXPECT(lod_store_read_info(good.c_str(), &V, &S, &n) == LOD_OK && V == 3 && S == 8 && n == 4);
  EXPECT(lod_store_read_info((dir + "/missing").c_str(), &V, &S, &n) == LOD_EINVAL);
  const std::string empty = dir + "/empty.lodstore";
  { const int fd = open(empty.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644); EXPECT(fd >= 0); close(fd); }
  EXPECT(lod_store_read_info(empty.c_str(), &V, &S, &n) == LOD_EINVAL);
  const std::string badmagic = dir + "/magic.lodstore";
  EXPECT(write_store(badmagic, small_store(), 1, "LODSTORX"));
  EXPECT(lod_store_read_info(badmagic.c_str(), &V, &S, &n) == LOD_EINVAL);
  const std::string badver = dir + "/version.lodstore";
  EXPECT(write_store(badver, small_store(), 2));
  EXPECT(lod_store_read_info(badver.c_str(), &V, &S, &n) == LOD_EINVAL);

  HostView hv(16, 64);
  // the well-formed file passes the checks; without a device the first copy fails
  const lod_status r = open_close(good, 8, hv);
  EXPECT(r == LOD_OK || r == LOD_EDEVICE);
  EXPECT(open_close(good, 0, hv) == LOD_EINVAL);
  HostView small(2, 64);
  EXPECT(open_close(good, 8, small) == LOD_ECAPACITY);   // fewer node slots than the store's nodes
  EXPECT(open_close(empty, 8, hv) == LOD_EINVAL);
  EXPECT(open_close(badmagic, 8, hv) == LOD_EINVAL);
  EXPECT(open_close(badver, 8, hv) == LOD_EINVAL);

  struct Case {
    const char *name;
    void (*corrupt)(Store &);
  };
  const Case cases[] = {
      {"points above n", [](Store &s) { s.pt_count[1] = s.n + 1; }},
      {"parent out of range", [](Store &s) { s.parent[2] = 9; }},
      {"parent after child", [](Store &s) { s.parent[1] = 2; }},
      {"child without parent link", [](Store &s) { s.parent[2] = LOD_NONE; s.depth[2] = 0; }},
      {"child list past the end", [](Store &s) { s.child_mask[0] = 0x83; }},
      {"mask without children", [](Store &s) { s.first_child[0] = LOD_NONE; }},
      {"children without mask", [](Store &s) { s.child_mask[0] = 0; }},
      {"child before its parent", [](Store &s) { s.first_child[1] = 0; s.child_mask[1] = 1; }},
      {"depth jump", [](Store &s) { s.depth[1] = 3; }},
      {"root below depth 0", [](Store &s) { s.depth[0] = 1; s.depth[1] = 2; s.depth[2] = 2; }},
      {"depth past the prefix", [](Store &s) { s.depth[0] = 30; s.depth[1] = 31; s.depth[2] = 31; }},
      {"block past the file", [](Store &s) { s.block_off = {64, 1ull << 40, 64}; }},
      {"block offset wraps", [](Store &s) { s.block_off = {64, ~0ull - 4, 64}; }},
      {"n zero", [](Store &s) { s.n = 0; s.pt_count = {0, 0, 0}; }},
  };
  for (const Case &c : cases) {
    Store s = small_store();
    c.corrupt(s);
    const std::string path = dir + "/corrupt.lodstore";
    EXPECT(write_store(path, s));
    const lod_status rc = open_close(path, 8, hv);
    if (rc != LOD_EINVAL) std::fprintf(stderr, "FAIL corrupted store '%s' gave %d\n", c.name, (int)rc);
    failures += rc != LOD_EINVAL;
  }
  const std::string trunc = dir + "/trunc.lodstore";
  EXPECT(write_store(trunc, small_store(), 1, "LODSTOR1", true));
  EXPECT(open_close(trunc, 8, hv) == LOD_EINVAL);
  const std::string badoff = dir + "/nodesoff.lodstore";
  EXPECT(write_store(badoff, small_store(), 1, "LODSTOR1", false, 1ull << 50));
  EXPECT(open_close(badoff, 8, hv) == LOD_EINVAL);
}

int main(int argc, char **argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s <scratch directory>\n", argv[0]);
    return 2;
  }
  null_arguments();
  plan_ranges();
  store_files(argv[1]);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("abi_sanitize: all checks passed\n");
  return 0;
}
