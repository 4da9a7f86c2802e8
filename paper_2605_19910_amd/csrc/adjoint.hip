// Adjoint of the transmission with respect to on-site energies, on gfx950.
//
// With H_ii,ss += eps_{i,s} (M_ss -= eps) the first-order change of G is dG = G dH G,
// so for T = Re Tr[Gamma_L G_{0,l-1} Gamma_R G_{0,l-1}^H]
//     dT/d eps_{i,s} = 2 Re[(G_{i,l-1} X G_{0,i})_{ss}],   X = Gamma_R G_{0,l-1}^H Gamma_L,
// where G_{0,i} = R_i is the first block row (R_i = -R_{i-1} U_i) and
// G_{i,l-1} = G_ii P_i the last block column (P_{l-1} = I, P_i = -U_{i+1} P_{i+1}).
// The forward sweep stored U_i for every layer and, at the boundaries of nd domains,
// R (first layer of each domain) and P (last layer of each domain).  One workgroup
// per (energy, domain) recomputes P and R inside its domain from those checkpoints
// (the domains are independent, so the adjoint has ne * nd parallel chains) and
// writes its energy's contribution dL/dT_E * dT_E/d eps; a second kernel sums the
// energies in a fixed order.
#include "block_engine.h"
#include "kernels.h"

namespace rgfk {

template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void rgf_adjoint_kernel(AdjArgs a) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  __shared__ double part[2][MAXBP];
  const int c = blockIdx.x;
  const int e = c / a.nd, k = c % a.nd;
  const int l = a.l, b = a.b;
  const int i0 = k * a.dlen;
  if (i0 >= l) return;   // uniform: the whole workgroup leaves
  const int i1 = (i0 + a.dlen < l ? i0 + a.dlen : l) - 1;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const double2* chain = a.ws + (size_t)e * a.ws_chain;
  const double2* U = chain + (size_t)l * bpbp;
  const double2* ckP = chain + sweep_ws_chain_elems(l, BP);
  const double2* ckR = ckP + (size_t)a.nd * bpbp;
  const double2* Rlast = ckR + (size_t)a.nd * bpbp;
  double2* scr = a.scratch + (size_t)c * a.scratch_chain;
  double2* Pd = scr;                               // dlen blocks: P_i, i in [i0, i1]
  double2* Rr = Pd + (size_t)a.dlen * bpbp;        // 2 blocks
  double2* X = Rr + 2 * bpbp;
  double2* Tmp = X + bpbp;
  double2* GamL = Tmp + bpbp;
  double2* GamR = GamL + bpbp;
  double2* Z = GamR + bpbp;
  const double2* sL = a.sigL + (size_t)e * bb;
  const double2* sR = a.sigR + (size_t)e * bb;
  const double2* Gd = a.G + ((size_t)e * 3 * l + l) * bb;
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  Acc<T, NW> acc;

  // Gamma blocks and X = Gamma_R R_{l-1}^H Gamma_L
  for (int idx = threadIdx.x; idx < BP * BP; idx += NT) {
    const int r = idx / BP, cc = idx % BP;
    double2 gl = make_double2(0.0, 0.0), gr = make_double2(0.0, 0.0);
    if (r < b && cc < b) {
      const double2 s1 = sL[(size_t)r * b + cc], s2 = sL[(size_t)cc * b + r];
      gl = make_double2(-(s1.y + s2.y), s1.x - s2.x);
      const double2 q1 = sR[(size_t)r * b + cc], q2 = sR[(size_t)cc * b + r];
      gr = make_double2(-(q1.y + q2.y), q1.x - q2.x);
    }
    GamL[idx] = gl;
    GamR[idx] = gr;
  }
  __syncthreads();
  acc_zero<T, NW>(acc);
  mma<T, NW>(acc, opnd(Rlast, BP, BP, BP, 1), P(GamL), 1.0);
  store<T, NW>(acc, Tmp, BP, BP, BP);
  __syncthreads();
  acc_zero<T, NW>(acc);
  mma<T, NW>(acc, P(GamR), P(Tmp), 1.0);
  store<T, NW>(acc, X, BP, BP, BP);

  // P_i for the domain, right to left from the checkpoint at its last layer
  load<T, NW>(acc, P(ckP + (size_t)k * bpbp));
  store<T, NW>(acc, Pd + (size_t)(i1 - i0) * bpbp, BP, BP, BP);
  __syncthreads();
  for (int i = i1 - 1; i >= i0; --i) {
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(U + (size_t)(i + 1) * bpbp), P(Pd + (size_t)(i + 1 - i0) * bpbp), -1.0);
    store<T, NW>(acc, Pd + (size_t)(i - i0) * bpbp, BP, BP, BP);
    __syncthreads();
  }

  // left to right: R_i, Z_i = X R_i, C_i = G_ii P_i, grad_s = 2 Re sum_k C_i[s,k] Z_i[k,s]
  load<T, NW>(acc, P(ckR + (size_t)k * bpbp));
  store<T, NW>(acc, Rr, BP, BP, BP);
  __syncthreads();
  const double w = 2.0 * a.dLdT[e];
  const int ln = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
  for (int i = i0; i <= i1; ++i) {
    const double2* Ri = Rr + (size_t)((i - i0) & 1) * bpbp;
    if (i > i0) {
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(Rr + (size_t)((i - 1 - i0) & 1) * bpbp), P(U + (size_t)i * bpbp), -1.0);
      store<T, NW>(acc, const_cast<double2*>(Ri), BP, BP, BP);
      __syncthreads();
    }
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(X), P(Ri), 1.0);
    store<T, NW>(acc, Z, BP, BP, BP);
    __syncthreads();
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, opnd(Gd + (size_t)i * bb, b, b, b), P(Pd + (size_t)(i - i0) * bpbp), 1.0);
    // per-row partial sums of Re(C[s][k] Z[k][s]) over this wave's columns
    for (int s = threadIdx.x; s < 2 * MAXBP; s += NT) (&part[0][0])[s] = 0.0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < Acc<T, NW>::RR; ++r) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int srow = 16 * (tr0 + r) + c_row(ln, v);
        double p = 0.0;
#pragma unroll
        for (int cc = 0; cc < Acc<T, NW>::RC; ++cc) {
          if (tr0 + r >= T || tc0 + cc >= T) continue;
          const int kcol = 16 * (tc0 + cc) + c_col(ln);
          const double2 zz = Z[(size_t)kcol * BP + srow];
          p += acc.re[r][cc][v] * zz.x - acc.im[r][cc][v] * zz.y;
        }
        // sum over the 16 lanes that hold the same row
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) p += __shfl_xor(p, off, 64);
        // exactly one lane of one wave per (column half, row): a plain store, deterministic
        if (c_col(ln) == 0 && tr0 + r < T) part[wave_id() & 1][srow] = p;
      }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < b; s += NT)
      a.gradE[((size_t)e * l + i) * b + s] = w * (part[0][s] + part[1][s]);
    __syncthreads();
  }
}

// d_onsite[j] = sum_e gradE[e][j], energies in increasing order
__global__ void adjoint_sum_kernel(AdjArgs a) {
  const size_t n = (size_t)a.l * a.b;
  for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int e = 0; e < a.ne; ++e) s += a.gradE[(size_t)e * n + j];
    a.d_onsite[j] = s;
  }
}

template <int T>
static hipError_t launch_adj_T(const AdjArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  hipLaunchKernelGGL((rgf_adjoint_kernel<T, NW>), dim3(a.ne * a.nd), dim3(64 * NW), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  ktime_mark("rgf_adjoint_kernel", s);
  hipLaunchKernelGGL(adjoint_sum_kernel, dim3(256), dim3(256), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("adjoint_sum_kernel", s);
  return hipSuccess;
}

hipError_t launch_rgf_adjoint(const AdjArgs& a, hipStream_t s) {
  switch (padded_block(a.b) / 16) {
    case 1: return launch_adj_T<1>(a, s);
    case 2: return launch_adj_T<2>(a, s);
    case 3: return launch_adj_T<3>(a, s);
    case 4: return launch_adj_T<4>(a, s);
    case 5: return launch_adj_T<5>(a, s);
    case 6: return launch_adj_T<6>(a, s);
    case 7: return launch_adj_T<7>(a, s);
    case 8: return launch_adj_T<8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rgfk
