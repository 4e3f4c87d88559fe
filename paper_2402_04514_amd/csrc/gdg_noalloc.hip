// gdg_noalloc.hip -- gdg_solve_noalloc() of include/gdg.h: a whole solve
// (stencil set-up, state in, run to the final time, state out) for callers
// that cannot allocate device memory.  The workspace that gdg_create() takes
// from its caller is here a static device array of the library, one copy per
// GPU; nothing is allocated on the device, and no graph is captured (the
// device-driven steps are launched directly).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "gdg.h"
#include "gdg_internal.h"

namespace {

// The workspace of gdg_solve_noalloc(): GDG_NOALLOC_MAX_BYTES per GPU, held
// from the library's load until the process ends.  In host code its name is
// only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress() (see scratch_ptr).
static __device__ __align__(256) unsigned char scratch[GDG_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device, taken once

// Device address of the current device's copy of `scratch`, looked up at the
// first call on that device (with that device current).
gdg_status scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    gdg::set_create_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return GDG_E_DEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    gdg::set_create_error("device index out of the range the no-allocation workspace supports");
    return GDG_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      gdg::set_create_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return GDG_E_DEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GDG_OK;
}

}  // namespace

extern "C" {

gdg_status gdg_solve_noalloc(const gdg_mesh_desc *mesh, const gdg_params *prm, const double *U0, double *U,
                             double t_final, int64_t max_steps, void *hip_stream, gdg_stats *stats) {
  gdg::set_create_error("");
  if (!mesh || !prm || !U0 || !U) {
    gdg::set_create_error("null argument");
    return GDG_E_INVALID;
  }
  size_t need = 0;
  if (gdg_workspace_bytes(mesh, prm, &need) != GDG_OK) {
    gdg::set_create_error("invalid mesh description or scheme constants");
    return GDG_E_INVALID;
  }
  if (need > (size_t)GDG_NOALLOC_MAX_BYTES) {
    gdg::set_create_error("the mesh needs " + std::to_string(need) +
                          " bytes of workspace; gdg_solve_noalloc holds at most " +
                          std::to_string((size_t)GDG_NOALLOC_MAX_BYTES) + " (GDG_NOALLOC_MAX_BYTES)");
    return GDG_E_NOMEM;
  }
  void *ws = nullptr;
  if (gdg_status s = scratch_ptr(&ws)) return s;
  gdg_ctx *ctx = nullptr;
  if (gdg_status s = gdg_create(mesh, prm, ws, GDG_NOALLOC_MAX_BYTES, hip_stream, &ctx)) return s;
  gdg_status s = gdg_upload_state(ctx, U0, 0);
  if (s == GDG_OK) s = gdg::run_loop(ctx, t_final, max_steps, stats, false);
  if (s == GDG_OK) s = gdg_download_state(ctx, U, 0);
  if (s != GDG_OK) gdg::set_create_error(gdg_last_error(ctx));
  gdg_destroy(ctx);
  return s;
}

}  // extern "C"
