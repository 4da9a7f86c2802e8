// Launchers of the observables read off a solved band (epilogue.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace rgfk {
// dos[e][i b + s] = -(1/pi) Im G[e][w][i][s][s]   (band [ne][2w+1][l][b][b])
hipError_t launch_dos(const double2* G, int l, int b, int w, int ne, double* dos, hipStream_t s);
// n[i b + s] = sum_e wts[e] Im Gl[e][w][i][s][s] / (2 pi), energies in order
hipError_t launch_density(const double2* Gl, int l, int b, int w, int ne, const double* wts, double* n,
                          hipStream_t s);
// cur[e][i] = Re Tr[H_{i,i+1} G^<_{i+1,i}(E_e)] / pi, w = 1 bands (H [3][l][b][b],
// Gl [ne][3][l][b][b]), one workgroup per (energy, bond), fixed-order reduction
hipError_t launch_bond_current(const double2* H, const double2* Gl, int l, int b, int ne, double* cur,
                               hipStream_t s);
}  // namespace rgfk
