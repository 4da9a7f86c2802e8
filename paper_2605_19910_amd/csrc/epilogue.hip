// Observables read off a solved band: the orbital-resolved density of states from
// the diagonal blocks of G^R, the electron density from the diagonal blocks of G^<
// (the lesser stage), integrated over the energy grid with caller weights, and the
// spectral particle current through every bond from the off-diagonal blocks of G^<.
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
// One workgroup (256 threads) per (energy, bond): Re Tr[H_{i,i+1} G^<_{i+1,i}] / pi
// as a strided dot product and a fixed-order tree reduction.
__global__ void bond_current_kernel(const double2* H, const double2* Gl, int l, int b, double* cur) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int i = blockIdx.x % (l - 1), e = blockIdx.x / (l - 1);
  const size_t bb = (size_t)b * b;
  const double2* Hu = H + ((size_t)2 * l + i) * bb;               // block (i, i+1) of the band of H
  const double2* Gd = Gl + ((size_t)e * 3 * l + (i + 1)) * bb;    // block (i+1, i) of G^<
  double acc = 0.0;
  for (size_t idx = t; idx < bb; idx += 256) {
    const size_t r = idx / b, c = idx % b;
    const double2 h = Hu[r * b + c], g = Gd[c * b + r];
    acc += h.x * g.x - h.y * g.y;
  }
  red[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) cur[(size_t)e * (l - 1) + i] = red[0] / kPi;
}
}  // namespace

hipError_t launch_bond_current(const double2* H, const double2* Gl, int l, int b, int ne, double* cur,
                               hipStream_t s) {
  hipLaunchKernelGGL(bond_current_kernel, dim3(ne * (l - 1)), dim3(256), 0, s, H, Gl, l, b, cur);
  return hipGetLastError();
}

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
