// Observables read off a solved band: the orbital-resolved density of states from
// the diagonal blocks of G^R, and the electron density from the diagonal blocks of
// G^< (the lesser stage), integrated over the energy grid with caller weights.
// Both are elementwise passes over the diagonal (HBM-bound, negligible beside the
// sweep); the density sums energies in a fixed order, so it is deterministic.
#include <hip/hip_runtime.h>

#include "epilogue.h"

namespace rgfk {

namespace {
constexpr double kPi = 3.141592653589793;

__global__ void dos_kernel(const double2* G, int l, int b, int w, int ne, double* dos) {
  const size_t lb = (size_t)l * b, bb = (size_t)b * b;
  const size_t total = lb * ne;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t e = idx / lb, r = idx % lb;
    const size_t i = r / b, s = r % b;
    const double2 x = G[(e * (2 * w + 1) + w) * l * bb + i * bb + s * b + s];
    dos[idx] = -x.y / kPi;
  }
}

__global__ void density_kernel(const double2* Gl, int l, int b, int w, int ne, const double* wts, double* n) {
  const size_t lb = (size_t)l * b, bb = (size_t)b * b;
  const double two_pi = 2.0 * kPi;
  for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < lb; r += (size_t)gridDim.x * blockDim.x) {
    const size_t i = r / b, s = r % b;
    double acc = 0.0;
    for (int e = 0; e < ne; ++e) {
      const double2 x = Gl[((size_t)e * (2 * w + 1) + w) * l * bb + i * bb + s * b + s];
      acc += wts[e] * x.y / two_pi;
    }
    n[r] = acc;
  }
}
}  // namespace

hipError_t launch_dos(const double2* G, int l, int b, int w, int ne, double* dos, hipStream_t s) {
  const size_t total = (size_t)l * b * ne;
  const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(dos_kernel, dim3(grid), dim3(256), 0, s, G, l, b, w, ne, dos);
  return hipGetLastError();
}

hipError_t launch_density(const double2* Gl, int l, int b, int w, int ne, const double* wts, double* n,
                          hipStream_t s) {
  const size_t total = (size_t)l * b;
  const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(density_kernel, dim3(grid), dim3(256), 0, s, Gl, l, b, w, ne, wts, n);
  return hipGetLastError();
}

}  // namespace rgfk
