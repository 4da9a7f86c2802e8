// Sequential RGF for block tridiagonal systems (paper Sec. 2.2, Algorithm 1) on gfx950.
//
// One workgroup (4 wave64) per chain; the chain's layer loop runs inside the kernel
// so the host boundary is crossed once.  Per layer:
//   upward   g_i = S_i^{-1}  (register-resident blocked Gauss-Jordan)
//            L_i = g_i M_{i,i-1},  U_i = M_{i-1,i} g_i,
//            S_{i-1} = M_{i-1,i-1} - M_{i-1,i} L_i   (assembled from H, E, Sigma on the fly)
//   downward G_{i-1,i} = -G_{i-1,i-1} U_i,  G_{i,i-1} = -L_i G_{i-1,i-1},
//            G_ii = g_i - L_i G_{i-1,i},  first block row R_i = -R_{i-1} U_i (R_0 = G_00)
// and finally T = Re Tr[Gamma_L R_{l-1} Gamma_R R_{l-1}^H], Gamma = i (Sigma - Sigma^H).
// g_i, U_i, L_i are kept in the workspace between the two passes.
#include "block_engine.h"
#include "kernels.h"

namespace rgfk {

int padded_block(int b) { return ((b + 15) / 16) * 16; }

size_t sweep_ws_chain_elems(int l, int bp) {
  // g[l], U[l], L[l], R[2], Gamma_L, Gamma_R, X1, and two blocks for the pivot refinement
  return (size_t)(3 * (size_t)l + 7) * (size_t)bp * (size_t)bp;
}

template <int T, int NW, int MIXED>
__global__ __launch_bounds__(64 * NW, 1) void rgf_sweep_kernel(SweepArgs a) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  __shared__ GJShared sh;
  __shared__ double red[NW];

  const int e = blockIdx.x;
  const int t = threadIdx.x;
  const int l = a.l, b = a.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  double2* ws = a.ws + (size_t)e * a.ws_chain;
  double2* g = ws;
  double2* U = ws + (size_t)l * bpbp;
  double2* L = ws + (size_t)2 * l * bpbp;
  double2* Rb = ws + (size_t)3 * l * bpbp;
  double2* GamL = Rb + 2 * bpbp;
  double2* GamR = GamL + bpbp;
  double2* X1 = GamR + bpbp;
  double2* Ssave = X1 + bpbp;     // pivot before inversion (refinement)
  double2* Rres = Ssave + bpbp;   // I - S g (refinement)

  const double2* H = a.H + (size_t)e * a.h_stride;
  const double2* Hl = H;                          // block (i, i-1) at Hl + i*bb
  const double2* Hd = H + (size_t)l * bb;         // block (i, i)
  const double2* Hu = H + (size_t)2 * l * bb;     // block (i, i+1)
  const double2* sL = a.direct ? nullptr : a.sigL + (size_t)e * bb;
  const double2* sR = a.direct ? nullptr : a.sigR + (size_t)e * bb;
  const double2 z = make_double2(a.direct ? 0.0 : a.E[e], a.direct ? 0.0 : a.eta_d);
  // off-diagonal blocks of M are -H (assembled) or the stored band (direct)
  const double ms = a.direct ? 1.0 : -1.0;
  double2* Gout = a.G + (size_t)e * a.g_stride;
  double2* Gl = Gout;
  double2* Gd = Gout + (size_t)l * bb;
  double2* Gu = Gout + (size_t)2 * l * bb;

  int bad_layer = -1;
  Acc<T, NW> acc;

  // acc (+)= M_ii: assembled from H, E, Sigma, or read from the direct band
  auto diag = [&](int i, bool add) {
    if (a.direct) {
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
      assemble_diag<T, NW>(acc, Hd + (size_t)i * bb, b, z, i == 0 ? sL : nullptr,
                           i == l - 1 ? sR : nullptr, add);
    }
  };
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pb = [&](const double2* p) { return opnd(p, b, b, b); };

  // ---------------- upward pass ----------------
  acc_zero<T, NW>(acc);
  diag(l - 1, true);
  for (int i = l - 1; i >= 0; --i) {
    double2* gi = g + (size_t)i * bpbp;
    if (MIXED) store<T, NW>(acc, Ssave, BP, BP, BP);
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
    }
    if (i == 0) break;
    gemm_to<MIXED, T, NW>(acc, P(gi), Pb(Hl + (size_t)i * bb), ms);
    store<T, NW>(acc, L + (size_t)i * bpbp, BP, BP, BP);
    gemm_to<MIXED, T, NW>(acc, Pb(Hu + (size_t)(i - 1) * bb), P(gi), ms);
    store<T, NW>(acc, U + (size_t)i * bpbp, BP, BP, BP);
    __syncthreads();
    // S_{i-1} = M_{i-1,i-1} - M_{i-1,i} L_i
    gemm_to<MIXED, T, NW>(acc, Pb(Hu + (size_t)(i - 1) * bb), P(L + (size_t)i * bpbp), -ms);
    diag(i - 1, true);
  }

  // ---------------- downward pass ----------------
  load<T, NW>(acc, P(g));
  store<T, NW>(acc, Gd, b, b, b);
  store<T, NW>(acc, Rb, BP, BP, BP);
  if (a.first_row) store<T, NW>(acc, a.first_row + (size_t)e * l * bb, b, b, b);
  __syncthreads();
  for (int i = 1; i < l; ++i) {
    const double2* Gp = Gd + (size_t)(i - 1) * bb;
    const double2* Ui = U + (size_t)i * bpbp;
    const double2* Li = L + (size_t)i * bpbp;
    gemm_to<MIXED, T, NW>(acc, Pb(Gp), P(Ui), -1.0);
    store<T, NW>(acc, Gu + (size_t)(i - 1) * bb, b, b, b);
    gemm_to<MIXED, T, NW>(acc, P(Li), Pb(Gp), -1.0);
    store<T, NW>(acc, Gl + (size_t)i * bb, b, b, b);
    gemm_to<MIXED, T, NW>(acc, P(Rb + (size_t)((i - 1) & 1) * bpbp), P(Ui), -1.0);
    store<T, NW>(acc, Rb + (size_t)(i & 1) * bpbp, BP, BP, BP);
    if (a.first_row) store<T, NW>(acc, a.first_row + ((size_t)e * l + i) * bb, b, b, b);
    __syncthreads();
    gemm_to<MIXED, T, NW>(acc, P(Li), Pb(Gu + (size_t)(i - 1) * bb), -1.0);
    add_from<T, NW>(acc, P(g + (size_t)i * bpbp));
    store<T, NW>(acc, Gd + (size_t)i * bb, b, b, b);
    __syncthreads();
  }

  // ---------------- transmission ----------------
  double Tval = 0.0;
  if (a.T && !a.direct)
    Tval = transmission<T, NW>(acc, Rb + (size_t)((l - 1) & 1) * bpbp, sL, sR, b, GamL, GamR, X1, red);

  // ---------------- status ----------------
  if (bad_layer >= 0) {
    const double qnan = __builtin_nan("");
    for (size_t idx = t; idx < (size_t)3 * l * bb; idx += NT) Gout[idx] = make_double2(qnan, qnan);
    if (a.first_row)
      for (size_t idx = t; idx < (size_t)l * bb; idx += NT)
        a.first_row[(size_t)e * l * bb + idx] = make_double2(qnan, qnan);
    Tval = qnan;
  }
  if (t == 0) {
    if (a.T && !a.direct) a.T[e] = Tval;
    if (a.info) a.info[(size_t)e * a.info_stride + a.info_offset] = bad_layer >= 0 ? bad_layer + 1 : 0;
  }
}

template <int T>
static hipError_t launch_T(const SweepArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  if (a.mixed)
    hipLaunchKernelGGL((rgf_sweep_kernel<T, NW, 1>), dim3(a.chains), dim3(64 * NW), 0, s, a);
  else
    hipLaunchKernelGGL((rgf_sweep_kernel<T, NW, 0>), dim3(a.chains), dim3(64 * NW), 0, s, a);
  return hipGetLastError();
}

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

}  // namespace rgfk
