// Internal launch interface between the C ABI (plan/solve logic) and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rgfk {

// Sequential RGF sweep, block tridiagonal (w = 1), one workgroup per chain.
//
// A chain is one (system, energy) pair.  Chain c reads its blocks through
// per-chain strides so that the same kernel serves three callers:
//   * plain RGF on a full system:  H shared by all chains (stride 0), Sigma per energy;
//   * DDRGF reduced system:        "direct" mode, the band of M itself per chain;
//   * DDRGF interiors:             see ddrgf_extended_rgf (separate kernel).
struct SweepArgs {
  const double2* H;          // band [3][l][b][b]: H[1+k][i] = block (i, i+k)
  size_t h_stride;           // elements between the bands of consecutive chains (0 = shared)
  const double2* sigL;       // [chains][b][b] (may be null in direct mode)
  const double2* sigR;
  const double* E;           // [chains] energies (ignored in direct mode)
  double eta_d;
  int direct;                // 1: H holds the band of M itself (no E, no Sigma, no sign flip)
  double2* G;                // out band [chains][3][l][b][b]
  size_t g_stride;           // elements between the outputs of consecutive chains
  double2* first_row;        // optional out [chains][l][b][b]: G_{0,i} (null = not wanted)
  double* T;                 // optional out [chains]
  int* info;                 // [chains]
  double2* ws;               // workspace, ws_chain elements per chain
  size_t ws_chain;
  int l, b, chains;
};

size_t sweep_ws_chain_elems(int l, int bp);
int padded_block(int b);
hipError_t launch_rgf_sweep(const SweepArgs& a, hipStream_t s);

}  // namespace rgfk
