// Sequential RGF for block tridiagonal systems (paper Sec. 2.2, Algorithm 1) on gfx950.
//
// One workgroup per chain (one system at one energy); the chain's layer loop runs
// inside the kernel so the host boundary is crossed once.  Per layer:
//   upward   g_i = S_i^{-1}  (register-resident blocked Gauss-Jordan)
//            L_i = g_i M_{i,i-1},  U_i = M_{i-1,i} g_i,
//            S_{i-1} = M_{i-1,i-1} - M_{i-1,i} L_i   (assembled from H, E, Sigma on the fly)
//   downward G_{i-1,i} = -G_{i-1,i-1} U_i,  G_{i,i-1} = -L_i G_{i-1,i-1},
//            G_ii = g_i - L_i G_{i-1,i},  first block row R_i = -R_{i-1} U_i (R_0 = G_00)
// and finally T = Re Tr[Gamma_L R_{l-1} Gamma_R R_{l-1}^H], Gamma = i (Sigma - Sigma^H).
// g_i, U_i, L_i are kept in the workspace between the two passes.
//
// Two kernels share the per-chain body rgf_chain():
//   rgf_sweep_kernel    one workgroup per chain of a uniform batch (all outputs);
//   rgf_batched_kernel  persistent: workgroups pull chains of uneven size from a
//                       work queue (longest first) and write T and the diagonal blocks.
//
// Mixed precision (MIXED = 1): every block product on FP32 MFMA, each Schur pivot
// inverted in FP64 and refined once in FP64.  FP32 rounding (2^-24) of the products
// is amplified by the pivots' conditioning, so after each pivot's inversion the
// chain measures kappa_1(S_i) = ||S_i||_1 ||g_i||_1; as soon as one pivot exceeds
// kappa_max (tolerance / 2^-24) the chain is abandoned before any output is written
// and recomputed with FP64 products, and RGF_INFO_FP64_PRODUCTS is set in its status.
#include "block_engine.h"
#include "kernels.h"

namespace rgfk {

#if !defined(RGFK_INST_T) && !defined(RGFK_BATCHED_TU)
int padded_block(int b) { return ((b + 15) / 16) * 16; }
#endif


// Everything one chain needs.  Off-diagonal outputs Gl/Gu may be null (then not
// written; G_{i-1,i} goes to workspace scratch), first_row may be null, T may be null.
struct Chain {
  const double2* Hl;   // block (i, i-1) at Hl + i bb
  const double2* Hd;   // block (i, i)
  const double2* Hu;   // block (i, i+1)
  const double2* sL;   // null in direct mode
  const double2* sR;
  double2 z;           // E + i eta_d
  int direct;
  double2* Gl;
  double2* Gd;         // diagonal blocks (always written)
  double2* Gu;
  double2* first_row;
  double* T;
  int* info;
  double2* ws;
  int l, b;
  // adjoint checkpoints (null = none), for nd domains of dlen layers: the Schur pivot
  // S (before inversion) and the last-column propagator P at the last layer of each
  // domain, P and the first block row R = G_{0,i} at the first layer of each domain,
  // and R at the last layer
  double2* ckS;
  double2* ckP;
  double2* ckP0;
  double2* ckR;
  double2* Rlast;
  int nd, dlen;
  double kappa_max;    // mixed precision: largest pivot kappa_1 allowed with FP32 products
};

// Runs one chain.  Returns false (having written no output) when MIXED and a Schur
// pivot is too ill-conditioned for FP32 products; the caller reruns it in FP64.
template <int T, int NW, int MIXED>
__device__ __forceinline__ bool rgf_chain(const Chain& ch, GJShared& sh, double* red) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  const int t = threadIdx.x;
  const int l = ch.l, b = ch.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  double2* g = ch.ws;
  double2* U = g + (size_t)l * bpbp;
  double2* L = g + (size_t)2 * l * bpbp;
  double2* Rb = g + (size_t)3 * l * bpbp;
  double2* GamL = Rb + 2 * bpbp;
  double2* GamR = GamL + bpbp;
  double2* X1 = GamR + bpbp;
  double2* Ssave = X1 + bpbp;     // pivot before inversion (refinement)
  double2* Rres = Ssave + bpbp;   // I - S g (refinement)
  double2* Gup = Rres + bpbp;     // G_{i-1,i} when Gu is not an output
  double2* Pb = Gup + bpbp;       // 2 blocks: last-column propagator P (adjoint checkpoints)
  // off-diagonal blocks of M are -H (assembled) or the stored band (direct)
  const double ms = ch.direct ? 1.0 : -1.0;
  const double2* Hl = ch.Hl;
  const double2* Hd = ch.Hd;
  const double2* Hu = ch.Hu;

  int bad_layer = -1;
  Acc<T, NW> acc;

  // acc (+)= M_ii: assembled from H, E, Sigma, or read from the direct band
  auto diag = [&](int i) {
    if (ch.direct) {
      add_from<T, NW>(acc, opnd(Hd + (size_t)i * bb, b, b, b));
      // identity on the padding of a directly given block
      const int ln = lane_id();
      int tr0, tc0;
      tile_origin<T, NW>(tr0, tc0);
#pragma unroll
      for (int r = 0; r < Acc<T, NW>::RR; ++r)
#pragma unroll
        for (int c = 0; c < Acc<T, NW>::RC; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ii = 16 * (tr0 + r) + c_row(ln, v), jj = 16 * (tc0 + c) + c_col(ln);
            if (ii == jj && ii >= b && tr0 + r < T && tc0 + c < T) acc.re[r][c][v] += 1.0;
          }
    } else {
      assemble_diag<T, NW>(acc, Hd + (size_t)i * bb, b, ch.z, i == 0 ? ch.sL : nullptr,
                           i == l - 1 ? ch.sR : nullptr, true);
    }
  };
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pn = [&](const double2* p) { return opnd(p, b, b, b); };
  auto is_last_of_domain = [&](int i) { return i == l - 1 || (i + 1) % ch.dlen == 0; };

  // ---------------- upward pass ----------------
  if (ch.ckP) {
    // P_{l-1} = I
    acc_zero<T, NW>(acc);
    add_identity<T, NW>(acc);
    store<T, NW>(acc, Pb + (size_t)((l - 1) & 1) * bpbp, BP, BP, BP);
    store<T, NW>(acc, ch.ckP + (size_t)((l - 1) / ch.dlen) * bpbp, BP, BP, BP);
    if ((l - 1) % ch.dlen == 0) store<T, NW>(acc, ch.ckP0 + (size_t)((l - 1) / ch.dlen) * bpbp, BP, BP, BP);
  }
  acc_zero<T, NW>(acc);
  diag(l - 1);
  for (int i = l - 1; i >= 0; --i) {
    double2* gi = g + (size_t)i * bpbp;
    if (MIXED) store<T, NW>(acc, Ssave, BP, BP, BP);
    if (ch.ckS && is_last_of_domain(i)) store<T, NW>(acc, ch.ckS + (size_t)(i / ch.dlen) * bpbp, BP, BP, BP);
    gj_invert<T, NW>(acc, gi, sh);
    if (sh.bad && bad_layer < 0) bad_layer = i;
    __syncthreads();
    if (MIXED) {
      // one step of iterative refinement in FP64: g <- g + g (I - S g)
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(Ssave), P(gi), -1.0);
      add_identity<T, NW>(acc);
      store<T, NW>(acc, Rres, BP, BP, BP);
      __syncthreads();
      load<T, NW>(acc, P(gi));
      mma<T, NW>(acc, P(gi), P(Rres), 1.0);
      __syncthreads();
      store<T, NW>(acc, gi, BP, BP, BP);
      __syncthreads();
      // FP32 products only while every pivot so far is well enough conditioned
      const double kap = kappa1<T, NW>(Ssave, gi, reinterpret_cast<double*>(&sh.pn[0][0]), red);
      if (!(kap <= ch.kappa_max)) return false;
    }
    if (i == 0) break;
    gemm_to<MIXED, T, NW>(acc, P(gi), Pn(Hl + (size_t)i * bb), ms);
    store<T, NW>(acc, L + (size_t)i * bpbp, BP, BP, BP);
    gemm_to<MIXED, T, NW>(acc, Pn(Hu + (size_t)(i - 1) * bb), P(gi), ms);
    store<T, NW>(acc, U + (size_t)i * bpbp, BP, BP, BP);
    __syncthreads();
    if (ch.ckP) {
      // P_{i-1} = -U_i P_i; kept at the last layer of every domain
      gemm_to<MIXED, T, NW>(acc, P(U + (size_t)i * bpbp), P(Pb + (size_t)(i & 1) * bpbp), -1.0);
      store<T, NW>(acc, Pb + (size_t)((i - 1) & 1) * bpbp, BP, BP, BP);
      if (is_last_of_domain(i - 1))
        store<T, NW>(acc, ch.ckP + (size_t)((i - 1) / ch.dlen) * bpbp, BP, BP, BP);
      if ((i - 1) % ch.dlen == 0) store<T, NW>(acc, ch.ckP0 + (size_t)((i - 1) / ch.dlen) * bpbp, BP, BP, BP);
    }
    // S_{i-1} = M_{i-1,i-1} - M_{i-1,i} L_i
    gemm_to<MIXED, T, NW>(acc, Pn(Hu + (size_t)(i - 1) * bb), P(L + (size_t)i * bpbp), -ms);
    diag(i - 1);
  }

  // ---------------- downward pass ----------------
  load<T, NW>(acc, P(g));
  store<T, NW>(acc, ch.Gd, b, b, b);
  store<T, NW>(acc, Rb, BP, BP, BP);
  if (ch.first_row) store<T, NW>(acc, ch.first_row, b, b, b);
  if (ch.ckR) store<T, NW>(acc, ch.ckR, BP, BP, BP);
  if (ch.Rlast && l == 1) store<T, NW>(acc, ch.Rlast, BP, BP, BP);
  __syncthreads();
  for (int i = 1; i < l; ++i) {
    const double2* Gp = ch.Gd + (size_t)(i - 1) * bb;
    const double2* Ui = U + (size_t)i * bpbp;
    const double2* Li = L + (size_t)i * bpbp;
    // G_{i-1,i}: to the output band, or to scratch when only the diagonal is wanted
    double2* Gup_i = ch.Gu ? ch.Gu + (size_t)(i - 1) * bb : Gup;
    gemm_to<MIXED, T, NW>(acc, Pn(Gp), P(Ui), -1.0);
    store<T, NW>(acc, Gup_i, b, b, b);
    if (ch.Gl) {
      gemm_to<MIXED, T, NW>(acc, P(Li), Pn(Gp), -1.0);
      store<T, NW>(acc, ch.Gl + (size_t)i * bb, b, b, b);
    }
    if (ch.T || ch.first_row || ch.ckR) {
      gemm_to<MIXED, T, NW>(acc, P(Rb + (size_t)((i - 1) & 1) * bpbp), P(Ui), -1.0);
      store<T, NW>(acc, Rb + (size_t)(i & 1) * bpbp, BP, BP, BP);
      if (ch.first_row) store<T, NW>(acc, ch.first_row + (size_t)i * bb, b, b, b);
      if (ch.ckR && i % ch.dlen == 0) store<T, NW>(acc, ch.ckR + (size_t)(i / ch.dlen) * bpbp, BP, BP, BP);
      if (ch.Rlast && i == l - 1) store<T, NW>(acc, ch.Rlast, BP, BP, BP);
    }
    __syncthreads();
    gemm_to<MIXED, T, NW>(acc, P(Li), Pn(Gup_i), -1.0);
    add_from<T, NW>(acc, P(g + (size_t)i * bpbp));
    store<T, NW>(acc, ch.Gd + (size_t)i * bb, b, b, b);
    __syncthreads();
  }

  // ---------------- transmission ----------------
  double Tval = 0.0;
  if (ch.T && !ch.direct)
    Tval = transmission<T, NW>(acc, Rb + (size_t)((l - 1) & 1) * bpbp, ch.sL, ch.sR, b, GamL, GamR, X1, red);

  // ---------------- status ----------------
  if (bad_layer >= 0) {
    const double qnan = __builtin_nan("");
    for (size_t idx = t; idx < (size_t)l * bb; idx += NT) {
      ch.Gd[idx] = make_double2(qnan, qnan);
      if (ch.Gl) ch.Gl[idx] = make_double2(qnan, qnan);
      if (ch.Gu) ch.Gu[idx] = make_double2(qnan, qnan);
      if (ch.first_row) ch.first_row[idx] = make_double2(qnan, qnan);
    }
    Tval = qnan;
  }
  if (t == 0) {
    if (ch.T && !ch.direct) *ch.T = Tval;
    if (ch.info) *ch.info = bad_layer >= 0 ? bad_layer + 1 : 0;
  }
  __syncthreads();
  return true;
}

// Mixed chains fall back to FP64 products when a pivot is too ill-conditioned.
template <int T, int NW, int MIXED>
__device__ __forceinline__ void run_chain(const Chain& ch, GJShared& sh, double* red) {
  if (MIXED) {
    if (!rgf_chain<T, NW, 1>(ch, sh, red)) {
      rgf_chain<T, NW, 0>(ch, sh, red);
      if (threadIdx.x == 0 && ch.info) *ch.info |= RGF_INFO_FP64_PRODUCTS;
    }
  } else {
    rgf_chain<T, NW, 0>(ch, sh, red);
  }
}

template <int T, int NW, int MIXED>
__global__ __launch_bounds__(64 * NW, 1) void rgf_sweep_kernel(SweepArgs a) {
  __shared__ GJShared sh;
  __shared__ double red[NW];
  const int e = blockIdx.x;
  const int l = a.l, b = a.b;
  const size_t bb = (size_t)b * b;
  const double2* H = a.H + (size_t)e * a.h_stride;
  Chain ch;
  ch.Hl = H;
  ch.Hd = H + (size_t)l * bb;
  ch.Hu = H + (size_t)2 * l * bb;
  ch.direct = a.direct;
  ch.sL = a.direct ? nullptr : a.sigL + (size_t)e * bb;
  ch.sR = a.direct ? nullptr : a.sigR + (size_t)e * bb;
  ch.z = make_double2(a.direct ? 0.0 : a.E[e], a.direct ? 0.0 : a.eta_d);
  double2* Gout = a.G + (size_t)e * a.g_stride;
  ch.Gl = Gout;
  ch.Gd = Gout + (size_t)l * bb;
  ch.Gu = Gout + (size_t)2 * l * bb;
  ch.first_row = a.first_row ? a.first_row + (size_t)e * l * bb : nullptr;
  ch.T = (a.T && !a.direct) ? a.T + e : nullptr;
  ch.info = a.info ? a.info + (size_t)e * a.info_stride + a.info_offset : nullptr;
  ch.ws = a.ws + (size_t)e * a.ws_chain;
  ch.l = l;
  ch.b = b;
  ch.ckS = ch.ckP = ch.ckP0 = ch.ckR = ch.Rlast = nullptr;
  ch.nd = a.nd;
  ch.dlen = a.dlen > 0 ? a.dlen : 1;
  if (a.nd > 0) {
    const size_t bpbp = (size_t)16 * T * 16 * T;
    ch.ckS = a.ck + (size_t)e * a.ck_chain;
    ch.ckP = ch.ckS + (size_t)a.nd * bpbp;
    ch.ckP0 = ch.ckP + (size_t)a.nd * bpbp;
    ch.ckR = ch.ckP0 + (size_t)a.nd * bpbp;
    ch.Rlast = ch.ckR + (size_t)a.nd * bpbp;
  }
  ch.kappa_max = a.kappa_max;
  run_chain<T, NW, MIXED>(ch, sh, red);
}

#ifndef RGFK_BATCHED_TU
template <int T>
hipError_t launch_T(const SweepArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  if (a.mixed)
    hipLaunchKernelGGL((rgf_sweep_kernel<T, NW, 1>), dim3(a.chains), dim3(64 * NW), 0, s, a);
  else
    hipLaunchKernelGGL((rgf_sweep_kernel<T, NW, 0>), dim3(a.chains), dim3(64 * NW), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) ktime_mark("rgf_sweep_kernel", s);
  return err;
}

#ifdef RGFK_INST_T
template hipError_t launch_T<RGFK_INST_T>(const SweepArgs& a, hipStream_t s);
#else
extern template hipError_t launch_T<1>(const SweepArgs& a, hipStream_t s);
extern template hipError_t launch_T<2>(const SweepArgs& a, hipStream_t s);
extern template hipError_t launch_T<3>(const SweepArgs& a, hipStream_t s);
extern template hipError_t launch_T<4>(const SweepArgs& a, hipStream_t s);
extern template hipError_t launch_T<5>(const SweepArgs& a, hipStream_t s);
extern template hipError_t launch_T<6>(const SweepArgs& a, hipStream_t s);
extern template hipError_t launch_T<7>(const SweepArgs& a, hipStream_t s);
extern template hipError_t launch_T<8>(const SweepArgs& a, hipStream_t s);

hipError_t launch_rgf_sweep(const SweepArgs& a, hipStream_t s) {
  const int T = padded_block(a.b) / 16;
  switch (T) {
    case 1: return launch_T<1>(a, s);
    case 2: return launch_T<2>(a, s);
    case 3: return launch_T<3>(a, s);
    case 4: return launch_T<4>(a, s);
    case 5: return launch_T<5>(a, s);
    case 6: return launch_T<6>(a, s);
    case 7: return launch_T<7>(a, s);
    case 8: return launch_T<8>(a, s);
    default: return hipErrorInvalidValue;
  }
}
#endif  // RGFK_INST_T
#endif  // !RGFK_BATCHED_TU

#ifdef RGFK_BATCHED_TU
// ---------------------------------------------------------------------------
// Persistent batched launch over instances of uneven size.
//
// An instance is one (device, energy) pair; device d has its own band H_d (l_d layers
// of b_d orbitals, b_d a multiple of 16 up to 128) and its own energies.  The plan
// sorts the instances into queue[] (longest first by default); every workgroup takes
// the next queue entry with one atomic increment of a counter in the workspace, runs
// the whole chain with the code path of its block size, and stops when the queue is
// empty (every workgroup reaches that test, so the grid always drains).  Each
// workgroup owns one workspace slot sized for the largest chain.  NW (4 or 8 waves
// per workgroup, two or one workgroups per compute unit) is the plan's tile choice.
// ---------------------------------------------------------------------------
// One translation unit per (MIXED, NW) variant of the kernel (they build in
// parallel); the dispatch below is compiled in a unit of its own.
template <int MIXED, int NW>
hipError_t launch_batched_mn(const BatchArgs& a, int grid, hipStream_t s);

#if defined(RGFK_BMIXED)
template <int MIXED, int NW>
__global__ __launch_bounds__(64 * NW, 8 / NW) void rgf_batched_kernel(BatchArgs a) {
  __shared__ GJShared sh;
  __shared__ double red[NW];
  __shared__ int s_item;
  double2* ws = a.ws_slots + (size_t)blockIdx.x * a.ws_slot;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= a.n_items) break;
    const int inst = a.queue[item];
    const int d = a.inst_dev[inst], e = a.inst_energy[inst];
    const rgf_batch_device_t dv = a.devs[d];
    // the shapes come from the plan, for which the workspace slots are sized; the
    // table's shape fields are not read
    const int l = a.dev_shape[2 * d], b = a.dev_shape[2 * d + 1];
    const size_t bb = (size_t)b * b;
    const double2* H = static_cast<const double2*>(dv.H);
    Chain ch;
    ch.Hl = H;
    ch.Hd = H + (size_t)l * bb;
    ch.Hu = H + (size_t)2 * l * bb;
    ch.direct = 0;
    ch.sL = static_cast<const double2*>(dv.sigma_L) + (size_t)e * bb;
    ch.sR = static_cast<const double2*>(dv.sigma_R) + (size_t)e * bb;
    ch.z = make_double2(dv.energies[e], a.eta_d);
    ch.Gl = nullptr;
    ch.Gu = nullptr;
    ch.Gd = static_cast<double2*>(dv.G_diag) + (size_t)e * l * bb;
    ch.first_row = nullptr;
    ch.T = dv.T ? dv.T + e : nullptr;
    ch.info = dv.info + e;
    ch.ws = ws;
    ch.l = l;
    ch.b = b;
    ch.ckS = ch.ckP = ch.ckP0 = ch.ckR = ch.Rlast = nullptr;
    ch.nd = 0;
    ch.dlen = 1;
    ch.kappa_max = a.kappa_max;
    switch ((b + 15) >> 4) {
      case 1: run_chain<1, NW, MIXED>(ch, sh, red); break;
      case 2: run_chain<2, NW, MIXED>(ch, sh, red); break;
      case 3: run_chain<3, NW, MIXED>(ch, sh, red); break;
      case 4: run_chain<4, NW, MIXED>(ch, sh, red); break;
      case 5: run_chain<5, NW, MIXED>(ch, sh, red); break;
      case 6: run_chain<6, NW, MIXED>(ch, sh, red); break;
      case 7: run_chain<7, NW, MIXED>(ch, sh, red); break;
      case 8: run_chain<8, NW, MIXED>(ch, sh, red); break;
      default: break;   // rejected at plan creation
    }
  }
}

template <>
hipError_t launch_batched_mn<RGFK_BMIXED, RGFK_BNW>(const BatchArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((rgf_batched_kernel<RGFK_BMIXED, RGFK_BNW>), dim3(grid), dim3(64 * RGFK_BNW), 0, s, a);
  return hipGetLastError();
}
#else
template <>
hipError_t launch_batched_mn<0, 4>(const BatchArgs& a, int grid, hipStream_t s);
template <>
hipError_t launch_batched_mn<1, 4>(const BatchArgs& a, int grid, hipStream_t s);
template <>
hipError_t launch_batched_mn<0, 8>(const BatchArgs& a, int grid, hipStream_t s);
template <>
hipError_t launch_batched_mn<1, 8>(const BatchArgs& a, int grid, hipStream_t s);

__global__ void reset_counter_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0;
}

hipError_t launch_rgf_batched(const BatchArgs& a, int grid, int waves, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, a.counter);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (waves == 4) return a.mixed ? launch_batched_mn<1, 4>(a, grid, s) : launch_batched_mn<0, 4>(a, grid, s);
  return a.mixed ? launch_batched_mn<1, 8>(a, grid, s) : launch_batched_mn<0, 8>(a, grid, s);
}
#endif  // RGFK_BMIXED
#endif  // RGFK_BATCHED_TU

}  // namespace rgfk
