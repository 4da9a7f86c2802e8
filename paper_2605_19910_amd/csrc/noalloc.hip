// rgf_solve_noalloc: the sequential solve with its workspace in a static device
// array of the library instead of a caller-supplied buffer, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The array (NOALLOC_SCRATCH_BYTES per device, held until the process ends) is
// located once per device with hipGetSymbolAddress; host code uses only that
// address, never the array's name.  Every call on a device shares the array:
// calls that overlap on one device race.  Nothing in it needs to start at zero
// (the sweep writes every workspace block before reading it).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rgf.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Address of this device's copy of the array (located on first use per device).
rgf_status_t scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RGF_ERR_HIP;
  if (dev < 0 || dev >= MAX_DEVICES) return RGF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RGF_ERR_HIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return RGF_OK;
}

}  // namespace

extern "C" {

rgf_status_t rgf_solve_noalloc(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                               const double* energies, double eta_d, void* G, double* T, int32_t* info,
                               void* stream) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  size_t need = 0, ck = 0;
  if (rgf_plan_checkpoint_bytes(plan, &ck) != RGF_OK) return RGF_ERR_INVALID_ARG;
  if (ck != 0) return RGF_ERR_UNSUPPORTED;   // adjoint plans keep checkpoints for rgf_backward
  if (rgf_plan_workspace_bytes(plan, &need) != RGF_OK) return RGF_ERR_INVALID_ARG;
  if (need > NOALLOC_SCRATCH_BYTES) return RGF_ERR_WORKSPACE_TOO_SMALL;
  void* ws = nullptr;
  const rgf_status_t st = scratch_ptr(&ws);
  if (st != RGF_OK) return st;
  return rgf_solve(plan, H, sigma_L, sigma_R, energies, eta_d, G, T, info, ws, NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
