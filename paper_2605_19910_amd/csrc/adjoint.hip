// Adjoint of the transmission on gfx950: gradients of L = sum_E w_E T(E) with
// respect to every entry of the band of H (dH) and to the on-site energies.
//
// M = (E + i eta_d) I - H - Sigma, so the first-order change of G is dG = G dH G and,
// Gamma being Hermitian, dT = 2 Re sum_{i,j} Tr[dH_ij Y_ij] with
//     Y_ij = G_{j,l-1} X G_{0,i},   X = Gamma_R G_{0,l-1}^H Gamma_L.
// For complex entries (PyTorch's convention d/dRe + i d/dIm) the gradient block is
// dT/dH_ij = 2 Y_ij^H; for a real on-site shift H_ii,ss += eps it is 2 Re (Y_ii)_ss.
// G_{0,i} = R_i is the first block row (R_i = -R_{i-1} U_i) and G_{j,l-1} = G_jj P_j
// the last block column (P_{l-1} = I, P_j = -U_{j+1} P_{j+1}); the U_i are the
// upward sweep's multipliers M_{i-1,i} g_i.
//
// Checkpointing.  The forward sweep keeps, per energy and per domain [i0, i1] of
// dlen layers, only the Schur pivot S_{i1} (before its inversion), P_{i1}, P_{i0}
// and R_{i0}, plus R_{l-1}.  One workgroup per (domain, energy chunk) rebuilds the
// domain's U_i by re-running the upward sweep from S_{i1} (the same Gauss-Jordan
// inversions and products as the forward, so the U_i are bitwise the forward's),
// then P right to left and R left to right.  On-site gradients are written per
// energy and summed over energies in increasing order; band gradients are
// accumulated over the chunk's energies in increasing order and the chunks summed in
// a fixed order.  Both results are deterministic and independent of the number of
// domains.
#include "block_engine.h"
#include "kernels.h"

namespace rgfk {

template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void rgf_adjoint_kernel(AdjArgs a) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  __shared__ GJShared sh;
  __shared__ double part[2][MAXBP];
  const int k = blockIdx.x % a.nd, c = blockIdx.x / a.nd;
  const int l = a.l, b = a.b;
  const int i0 = k * a.dlen;
  if (i0 >= l) return;   // uniform: the whole workgroup leaves
  const int i1 = (i0 + a.dlen < l ? i0 + a.dlen : l) - 1;
  const int n = i1 - i0 + 1;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const bool band = a.hpart != nullptr;
  double2* scr = a.scratch + (size_t)blockIdx.x * a.scratch_wg;
  double2* Ud = scr;                               // n blocks: U_i, i in [i0, i1]
  double2* Pd = Ud + (size_t)a.dlen * bpbp;        // dlen + 2 blocks: P_j, j in [i0 - 1, i1 + 1]
  double2* Cd = Pd + (size_t)(a.dlen + 2) * bpbp;  // dlen + 2 blocks: C_j = G_jj P_j
  double2* Rr = Cd + (size_t)(a.dlen + 2) * bpbp;  // 2 blocks
  double2* X = Rr + 2 * bpbp;
  double2* Tmp = X + bpbp;
  double2* GamL = Tmp + bpbp;
  double2* GamR = GamL + bpbp;
  double2* Z = GamR + bpbp;
  double2* gi = Z + bpbp;                          // inverse of the current pivot
  double2* Lt = gi + bpbp;                         // current left multiplier
  double2* hp = band ? a.hpart + (size_t)c * 3 * l * bb : nullptr;
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pn = [&](const double2* p) { return opnd(p, b, b, b); };
  const double2* Hl = a.H;
  const double2* Hd = a.H + (size_t)l * bb;
  const double2* Hu = a.H + (size_t)2 * l * bb;
  const int ln = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
  Acc<T, NW> acc;

  for (int e = c; e < a.ne; e += a.nch) {
    const double2* ck = a.ck + (size_t)e * a.ck_chain;
    const double2* ckS = ck;
    const double2* ckP1 = ck + (size_t)a.nd * bpbp;
    const double2* ckP0 = ckP1 + (size_t)a.nd * bpbp;
    const double2* ckR = ckP0 + (size_t)a.nd * bpbp;
    const double2* Rlast = ckR + (size_t)a.nd * bpbp;
    const double2* sL = a.sigL + (size_t)e * bb;
    const double2* sR = a.sigR + (size_t)e * bb;
    const double2* Gd = a.Gd + (size_t)e * a.gd_stride;
    const double2 z = make_double2(a.E[e], a.eta_d);
    const double w = 2.0 * a.dLdT[e];

    // ---- U_i of the domain: the upward sweep re-run from the checkpointed S_{i1} ----
    load<T, NW>(acc, P(ckS + (size_t)k * bpbp));
    for (int i = i1; i >= i0; --i) {
      __syncthreads();
      gj_invert<T, NW>(acc, gi, sh);
      __syncthreads();
      if (i >= 1) {
        // same operand order and signs as the forward: U_i = M_{i-1,i} g_i = -H_{i-1,i} g_i
        acc_zero<T, NW>(acc);
        mma<T, NW>(acc, Pn(Hu + (size_t)(i - 1) * bb), P(gi), -1.0);
        store<T, NW>(acc, Ud + (size_t)(i - i0) * bpbp, BP, BP, BP);
      }
      if (i > i0) {
        acc_zero<T, NW>(acc);
        mma<T, NW>(acc, P(gi), Pn(Hl + (size_t)i * bb), -1.0);
        store<T, NW>(acc, Lt, BP, BP, BP);
        __syncthreads();
        // S_{i-1} = M_{i-1,i-1} - M_{i-1,i} L_i = M_{i-1,i-1} + H_{i-1,i} L_i
        acc_zero<T, NW>(acc);
        mma<T, NW>(acc, Pn(Hu + (size_t)(i - 1) * bb), P(Lt), 1.0);
        assemble_diag<T, NW>(acc, Hd + (size_t)(i - 1) * bb, b, z, i - 1 == 0 ? sL : nullptr,
                             i - 1 == l - 1 ? sR : nullptr, true);
      }
    }
    __syncthreads();

    // ---- Gamma blocks and X = Gamma_R R_{l-1}^H Gamma_L ----
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

    // ---- P_j, j in [i0 - 1, i1 + 1] (slot j - i0 + 1), right to left ----
    load<T, NW>(acc, P(ckP1 + (size_t)k * bpbp));
    store<T, NW>(acc, Pd + (size_t)(n) * bpbp, BP, BP, BP);
    if (band && i1 + 1 < l) {
      load<T, NW>(acc, P(ckP0 + (size_t)(k + 1) * bpbp));
      store<T, NW>(acc, Pd + (size_t)(n + 1) * bpbp, BP, BP, BP);
    }
    __syncthreads();
    const int jlo = (band && i0 >= 1) ? i0 - 1 : i0;
    for (int j = i1 - 1; j >= jlo; --j) {
      // P_j = -U_{j+1} P_{j+1}, as in the forward
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(Ud + (size_t)(j + 1 - i0) * bpbp), P(Pd + (size_t)(j + 2 - i0) * bpbp), -1.0);
      store<T, NW>(acc, Pd + (size_t)(j + 1 - i0) * bpbp, BP, BP, BP);
      __syncthreads();
    }
    // C_j = G_jj P_j (last block column) for the rows and columns this domain needs
    if (band) {
      const int jhi = i1 + 1 < l ? i1 + 1 : i1;
      for (int j = jlo; j <= jhi; ++j) {
        acc_zero<T, NW>(acc);
        mma<T, NW>(acc, Pn(Gd + (size_t)j * bb), P(Pd + (size_t)(j + 1 - i0) * bpbp), 1.0);
        store<T, NW>(acc, Cd + (size_t)(j + 1 - i0) * bpbp, BP, BP, BP);
      }
      __syncthreads();
    }

    // ---- left to right: R_i, Z_i = X R_i, gradient rows of layer i ----
    load<T, NW>(acc, P(ckR + (size_t)k * bpbp));
    store<T, NW>(acc, Rr, BP, BP, BP);
    __syncthreads();
    for (int i = i0; i <= i1; ++i) {
      const double2* Ri = Rr + (size_t)((i - i0) & 1) * bpbp;
      if (i > i0) {
        acc_zero<T, NW>(acc);
        mma<T, NW>(acc, P(Rr + (size_t)((i - 1 - i0) & 1) * bpbp), P(Ud + (size_t)(i - i0) * bpbp), -1.0);
        store<T, NW>(acc, const_cast<double2*>(Ri), BP, BP, BP);
        __syncthreads();
      }
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(X), P(Ri), 1.0);
      store<T, NW>(acc, Z, BP, BP, BP);
      __syncthreads();
      if (a.gradE) {
        // on-site: 2 Re sum_k C_i[s,k] Z_i[k,s]
        acc_zero<T, NW>(acc);
        mma<T, NW>(acc, Pn(Gd + (size_t)i * bb), P(Pd + (size_t)(i + 1 - i0) * bpbp), 1.0);
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
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) p += __shfl_xor(p, off, 64);
            // exactly one lane of one wave per (column half, row): deterministic
            if (c_col(ln) == 0 && tr0 + r < T) part[wave_id() & 1][srow] = p;
          }
        }
        __syncthreads();
        for (int s = threadIdx.x; s < b; s += NT)
          a.gradE[((size_t)e * l + i) * b + s] = w * (part[0][s] + part[1][s]);
        __syncthreads();
      }
      if (band) {
        // dH_ij += 2 w (C_j Z_i)^H = 2 w Z_i^H C_j^H,  j = i-1, i, i+1
        for (int d = -1; d <= 1; ++d) {
          const int j = i + d;
          if (j < 0 || j >= l) continue;
          double2* dst = hp + ((size_t)(1 + d) * l + i) * bb;
          if (e == c)
            acc_zero<T, NW>(acc);
          else
            load<T, NW>(acc, Pn(dst));
          mma<T, NW>(acc, opnd(Z, BP, BP, BP, 1), opnd(Cd + (size_t)(j + 1 - i0) * bpbp, BP, BP, BP, 1), w);
          store<T, NW>(acc, dst, b, b, b);
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

#ifndef RGFK_INST_T
// d_onsite[j] = sum_e gradE[e][j] (energies in increasing order);
// dH[x] = sum_c hpart[c][x] for x inside the matrix (chunks in increasing order).
__global__ void adjoint_sum_kernel(AdjArgs a) {
  const size_t nl = (size_t)a.l * a.b;
  const size_t bb = (size_t)a.b * a.b;
  const size_t nh = a.hpart ? (size_t)3 * a.l * bb : 0;
  const size_t nn = (a.gradE ? nl : 0) + nh;
  for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < nn; j += (size_t)gridDim.x * blockDim.x) {
    if (a.gradE && j < nl) {
      double s = 0.0;
      for (int e = 0; e < a.ne; ++e) s += a.gradE[(size_t)e * nl + j];
      a.d_onsite[j] = s;
      continue;
    }
    const size_t x = a.gradE ? j - nl : j;
    const int k = (int)(x / ((size_t)a.l * bb)) - 1;        // band offset -1, 0, +1
    const int i = (int)((x / bb) % a.l);
    if (i + k < 0 || i + k >= a.l) continue;                // outside the matrix: not written
    double2 s = make_double2(0.0, 0.0);
    for (int c = 0; c < a.nch; ++c) {
      const double2 v = a.hpart[(size_t)c * nh + x];
      s.x += v.x;
      s.y += v.y;
    }
    a.dH[x] = s;
  }
}
#endif

template <int T>
hipError_t launch_adj_T(const AdjArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  hipLaunchKernelGGL((rgf_adjoint_kernel<T, NW>), dim3(a.nd * a.nch), dim3(64 * NW), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) ktime_mark("rgf_adjoint_kernel", s);
  return err;
}

#ifdef RGFK_INST_T
template hipError_t launch_adj_T<RGFK_INST_T>(const AdjArgs& a, hipStream_t s);
#else
extern template hipError_t launch_adj_T<1>(const AdjArgs& a, hipStream_t s);
extern template hipError_t launch_adj_T<2>(const AdjArgs& a, hipStream_t s);
extern template hipError_t launch_adj_T<3>(const AdjArgs& a, hipStream_t s);
extern template hipError_t launch_adj_T<4>(const AdjArgs& a, hipStream_t s);
extern template hipError_t launch_adj_T<5>(const AdjArgs& a, hipStream_t s);
extern template hipError_t launch_adj_T<6>(const AdjArgs& a, hipStream_t s);
extern template hipError_t launch_adj_T<7>(const AdjArgs& a, hipStream_t s);
extern template hipError_t launch_adj_T<8>(const AdjArgs& a, hipStream_t s);

hipError_t launch_rgf_adjoint(const AdjArgs& a, hipStream_t s) {
  hipError_t err = hipErrorInvalidValue;
  switch (padded_block(a.b) / 16) {
    case 1: err = launch_adj_T<1>(a, s); break;
    case 2: err = launch_adj_T<2>(a, s); break;
    case 3: err = launch_adj_T<3>(a, s); break;
    case 4: err = launch_adj_T<4>(a, s); break;
    case 5: err = launch_adj_T<5>(a, s); break;
    case 6: err = launch_adj_T<6>(a, s); break;
    case 7: err = launch_adj_T<7>(a, s); break;
    case 8: err = launch_adj_T<8>(a, s); break;
    default: break;
  }
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(adjoint_sum_kernel, dim3(1024), dim3(256), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("adjoint_sum_kernel", s);
  return hipSuccess;
}

size_t adjoint_scratch_wg_elems(int dlen, int bp) {
  // U (dlen), P (dlen + 2), C (dlen + 2), R (2), X, Tmp, Gamma_L, Gamma_R, Z, g, L
  return (size_t)(3 * (size_t)dlen + 13) * bp * bp;
}
#endif  // RGFK_INST_T

}  // namespace rgfk
