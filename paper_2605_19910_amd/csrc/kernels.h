// Internal launch interface between the C ABI (plan/solve logic) and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rgf.h"

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
  int* info;                 // status of chain c at info[c * info_stride + info_offset]
  int info_stride, info_offset;
  double2* ws;               // workspace, ws_chain elements per chain
  size_t ws_chain;
  int l, b, chains;
  int mixed;                 // 1: products on FP32 MFMA, FP64 pivots + one refinement step
  int nd, dlen;              // adjoint checkpoints: nd domains of dlen layers (nd = 0: none)
  double kappa_max;          // mixed: pivots with a larger kappa_1 send the chain back to FP64
  double2* ck;               // adjoint checkpoints (nd > 0): ck_chain elements per chain, layout
  size_t ck_chain;           // as AdjArgs::ck
  unsigned* sync;            // split sweep: one group counter per chain, 64 bytes apart
  long long spin_limit;      // split sweep: polls before a group barrier gives up
};

// Adjoint of T (one workgroup per (domain, energy chunk)); see adjoint.hip.
struct AdjArgs {
  const double2* H;          // band [3][l][b][b]
  const double2* sigL;       // [ne][b][b]
  const double2* sigR;
  const double* E;           // [ne]
  double eta_d;
  const double2* Gd;         // diagonal blocks of the forward's G: energy e at Gd + e gd_stride
  size_t gd_stride;
  const double* dLdT;        // [ne]
  const double2* ck;         // forward checkpoints, ck_chain elements per energy:
  size_t ck_chain;           //   S[nd], P(last layer)[nd], P(first layer)[nd], R(first layer)[nd], R_{l-1}
  double2* scratch;          // [nd * nch] workgroup slots of scratch_wg elements
  size_t scratch_wg;
  double* gradE;             // [ne][l][b] per-energy on-site gradients (null: not wanted)
  double2* hpart;            // [nch][3][l][b][b] per-chunk band gradients (null: not wanted)
  double* d_onsite;          // out [l][b]
  double2* dH;               // out band [3][l][b][b]
  int l, b, ne, nd, dlen, nch;
};

size_t adjoint_scratch_wg_elems(int dlen, int bp);
hipError_t launch_rgf_adjoint(const AdjArgs& a, hipStream_t s);

// Per-kernel timing: when the solve running on this host thread belongs to a plan
// with timing enabled, records an event on s after the named kernel's launch.
void ktime_mark(const char* kernel, hipStream_t s);
// g[l], U[l], L[l], R[2], Gamma_L, Gamma_R, X1, two blocks for the pivot refinement,
// one for G_{i-1,i} when the off-diagonal output is not wanted, two for P
__host__ __device__ inline size_t sweep_ws_chain_elems(int l, int bp) {
  return (size_t)(3 * (size_t)l + 10) * (size_t)bp * (size_t)bp;
}
int padded_block(int b);
hipError_t launch_rgf_sweep(const SweepArgs& a, hipStream_t s);

// Sequential sweep with K workgroups per chain (rgf_split.hip): FP64, plain solve
// (no checkpoints, no first row), padded block size 64 or 128.  split_workgroups
// returns the K (4, 2, or 1 = use launch_rgf_sweep) that fits the current device's
// co-resident capacity for ne chains (want: 0 = largest that fits, else only that
// K).  launch_rgf_split clears the counters and info, then launches cooperatively.
int split_workgroups(int b, int ne, int want);
hipError_t launch_rgf_split(const SweepArgs& a, int K, hipStream_t s);

// DDRGF (Algorithm 2), block tridiagonal, one level.
struct DDArgs {
  const double2* H;          // band [3][l][b][b], shared by all energies
  const double2* sigL;       // [ne][b][b]
  const double2* sigR;
  const double* E;           // [ne]
  double eta_d;
  double2* G;                // out band [ne][3][l][b][b]
  double* T;                 // out [ne] or null
  int* info;                 // out [ne]
  int l, b, m, ne;
  double2* ws_int;           // per (energy, interior) chain: ws_int_chain elements
  size_t ws_int_chain;
  double2* MS;               // reduced band [ne][3][m][b][b]
  double2* GS;               // its inverse band [ne][3][m][b][b]
  double2* GSrow;            // first block row of the reduced inverse [ne][m][b][b]
  double2* ws_red;           // sweep workspace of the reduced system
  size_t ws_red_chain;
  int* info_part;            // [ne][m + 1] per-stage status
  double2* ws_fin;           // [ne][4][bp][bp]
  int mixed;                 // 1: products on FP32 MFMA, FP64 pivots + one refinement step
  double kappa_max;          // as SweepArgs::kappa_max (reduced system)
  int* herm;                 // device flag: H exactly Hermitian (set by the check kernel)
  // multi-level DDRGF (the inner levels solve a reduced separator system):
  int direct;                // 1: the diagonal blocks of H hold M_ii itself (no E, eta_d, Sigma
                             //    added); the off-diagonal blocks hold -M_ij as those of H do
  size_t h_stride;           // elements between the bands of consecutive energies (0: H shared)
  double2* first_last;       // optional out: block (0, l-1) of the inverse of energy e at
  size_t first_last_stride;  //   first_last + e * first_last_stride (b x b)
  int info_stride, info_offset;   // status of energy e at info[e * stride + offset] (stride 0: 1)
};

size_t ddrgf_interior_ws_elems(int nmax, int bp);
void ddrgf_layout_host(int l, int m, int* base, int* rem);
// inner: the next level's arguments (its H is inner_band, filled here from a.MS), or
// null to solve the reduced system by the sequential sweep.
hipError_t launch_ddrgf(const DDArgs& a, const DDArgs* inner, double2* inner_band, hipStream_t s);

// Lesser Green's function on the band after a sequential w = 1 FP64 sweep
// (lesser.hip); reuses the sweep's per-energy workspace.
struct LesserArgs {
  const double2* sigL;       // [ne][b][b]
  const double2* sigR;
  const double* fL;          // [ne] occupation of the left lead
  const double* fR;          // [ne] occupation of the right lead
  const double2* G;          // band of G^R [ne][3][l][b][b] written by the sweep
  const int* info;           // [ne] the sweep's status
  double2* Gless;            // out band of G^< [ne][3][l][b][b]
  double2* ws;               // the sweep's workspace, ws_chain elements per energy
  size_t ws_chain;
  int l, b, ne;
};

hipError_t launch_rgf_lesser(const LesserArgs& a, hipStream_t s);

// Lead self-energies by decimation (leads.hip), one workgroup per energy.
struct LeadArgs {
  const double2* H00;        // [b][b] on-layer block of the lead
  const double2* H01;        // [b][b] coupling to the next layer away from the device
  const double2* Hc;         // [b][b] coupling from the device layer to the lead's surface
  const double* E;           // [ne]
  double eta;
  double tol;
  int max_steps;
  double2* sigma;            // out [ne][b][b]
  int* steps;                // out [ne]
  double2* ws;               // ws_chain elements per energy
  size_t ws_chain;
  int b, ne;
};

size_t lead_ws_chain_elems(int bp);
hipError_t launch_lead_decimation(const LeadArgs& a, hipStream_t s);

// Persistent batched launch (see rgf_batched_kernel).
struct BatchArgs {
  const rgf_batch_device_t* devs;   // device table [n_dev]
  const int* queue;                 // [n_items] instance ids in processing order
  const int* inst_dev;              // [n_items] device of each instance
  const int* inst_energy;           // [n_items] energy index of each instance
  const int* dev_shape;             // [n_dev][2]: the plan's (l, b) of each device
  int n_items;
  int* counter;                     // work-queue counter (reset by the launch)
  double2* ws_slots;                // one slot per persistent workgroup
  size_t ws_slot;                   // elements per slot
  double eta_d;
  int mixed;
  double kappa_max;                 // as SweepArgs::kappa_max
};

hipError_t launch_rgf_batched(const BatchArgs& a, int grid, int waves, hipStream_t s);

// Native n-diagonal sweep (w >= 1), one workgroup per energy.
struct NSweepArgs {
  const double2* H;          // band [2w+1][l][b][b]
  const double2* sigL;       // [ne][b][b]
  const double2* sigR;
  const double* E;
  double eta_d;
  double2* G;                // out band [ne][2w+1][l][b][b]
  double* T;                 // out [ne] or null
  int* info;                 // out [ne]
  double2* ws;
  size_t ws_chain;
  int l, b, w, ne;
  unsigned* sync;            // split sweep: one group counter per energy, 64 bytes apart
  long long spin_limit;      // split sweep: polls before a group barrier gives up
  // direct mode (the reduced separator system of the n-diagonal DDRGF): H holds the
  // band of M itself, every block as it is (no E, eta_d, Sigma), one band per energy
  int direct;
  size_t h_stride;           // elements between the bands of consecutive energies (direct)
  int nr;                    // first block rows propagated to the last column (>= 1)
  double2* rows_last;        // optional out: blocks (t, l-1), t < nr, at rows_last + (e nr + t) b b
};

// nr: first block rows carried to the last column (1 for a plain solve)
size_t nrgf_ws_chain_elems(int l, int w, int bp, int nr = 1);
// n-diagonal sweep with K workgroups per energy (nrgf_split.hip), FP64, padded block
// size 64 or 128; K from split_workgroups_n (as split_workgroups).
int split_workgroups_n(int b, int ne, int want);
hipError_t launch_nrgf_split(const NSweepArgs& a, int K, hipStream_t s);
hipError_t launch_nrgf_sweep(const NSweepArgs& a, hipStream_t s);

// DDRGF for block n-diagonal systems with separators of w layers (nddrgf.hip).
struct NDDArgs {
  const double2* H;          // band [2w+1][l][b][b], shared by all energies
  const double2* sigL;       // [ne][b][b]
  const double2* sigR;
  const double* E;           // [ne]
  double eta_d;
  double2* G;                // out band [ne][2w+1][l][b][b]
  double* T;                 // out [ne] or null
  int* info;                 // out [ne]
  int l, b, w, m, ne;
  double2* ws_int;           // per (energy, interior) chain: ws_int_chain elements
  size_t ws_int_chain;
  double2* MS;               // reduced band [ne][4w-1][m w][b][b] (half bandwidth 2w-1)
  double2* GS;               // its inverse band, same layout
  double2* GSlast;           // blocks (t, m w - 1), t < w, of the reduced inverse [ne][w][b][b]
  int* info_part;            // [ne][m]: first failing pivot of each interior (global layer + 1)
  int* info_red;             // [ne]: first failing pivot of the reduced system (reduced layer + 1)
  double2* ws_fin;           // [ne][4][bp][bp]
  int* herm;                 // device flag: H exactly Hermitian (set by the check kernel), or null
};

size_t nddrgf_interior_ws_elems(int nmax, int w, int bp);
void nddrgf_layout_host(int l, int m, int w, int* base, int* rem);
// red: the n-diagonal sweep arguments of the reduced system (direct mode, nr = w)
hipError_t launch_nddrgf(const NDDArgs& a, const NSweepArgs& red, hipStream_t s);

// Super-block view (w layers -> one layer of w*b orbitals) of a band and its leads.
struct FuseArgs {
  const double2* H;          // [2w+1][l][b][b]
  const double2* sigL;       // [ne][b][b]
  const double2* sigR;
  double2* Hf;               // [3][l/w][wb][wb]
  double2* sigLf;            // [ne][wb][wb]
  double2* sigRf;
  const double2* Gf;         // [ne][3][l/w][wb][wb]
  double2* G;                // [ne][2w+1][l][b][b]
  const int* info_f;         // [ne] status in super-layers
  int* info;                 // [ne] status in layers
  int l, b, w, ne;
};

hipError_t launch_fuse(const FuseArgs& a, hipStream_t s);
hipError_t launch_unfuse(const FuseArgs& a, hipStream_t s);

}  // namespace rgfk
