// Allocation-free variant of splat_render for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc): the splat's workspace is a fixed array in this
// library's device image instead of a caller buffer.
//
// The array exists once per device the library runs on and stays allocated
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device
// address is looked up once per device with hipGetSymbolAddress and kept.
// Every call on a device shares that device's array, so calls that overlap
// in time on one device race; each call rewrites every part of the array it
// reads before reading it (counters and tile tables are filled by kernels).
#include <hip/hip_runtime.h>

#include <mutex>

#include "lod.h"
#include "lod_internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[LOD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch array (looked up on first use).
lod_status scratch_for_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LOD_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LOD_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LOD_OK;
}

bool camera_ok(const lod_camera *c, const splat_params *sp) {
  size_t ws = 0;
  return splat_plan(0, c, sp, &ws) == LOD_OK;
}

}  // namespace

extern "C" {

lod_status splat_render_noalloc(const float *x, const float *y, const float *z, const float *m, uint64_t count,
                                const lod_camera *cam, const splat_params *sp, float *image, lod_stream_t stream) {
  if (!camera_ok(cam, sp) || !image) return LOD_EINVAL;
  if (count && (!x || !y || !z || !m)) return LOD_EINVAL;
  lodh::SplatLayout L;
  lod_status s = lodh::splat_layout(count, *cam, *sp, L, false);
  if (s != LOD_OK) return s;
  if (L.total > (size_t)LOD_NOALLOC_SCRATCH_BYTES) return LOD_ECAPACITY;
  void *ws = nullptr;
  if ((s = scratch_for_current_device(&ws)) != LOD_OK) return s;
  return lodh::launch_splat(x, y, z, m, nullptr, count, *cam, *sp, ws, L, image, nullptr, (hipStream_t)stream);
}

}  // extern "C"
