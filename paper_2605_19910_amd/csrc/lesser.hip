// Lesser Green's function on the band (the Keldysh equation G^< = G^R Sigma^< G^A,
// the step after the Dyson equation; the paper's introduction and outlook), after
// the sequential sweep of rgf_solve on the same workspace.
//
// With lead lesser self-energies Sigma^<_X = i f_X Gamma_X on the layer lead X
// attaches to (Gamma_X = i (Sigma_X - Sigma_X^H), f_X the lead's occupation),
//     G^<_ij = C_i A_L C_j^H + D_i A_R D_j^H,   A_X = Sigma^<_X,
// with the first block column C_i = G_{i,0} (C_0 = G_00, C_i = -L_i C_{i-1}) and the
// last block column D_i = G_{i,l-1} = G_ii P_i (P_{l-1} = I, P_{i-1} = -U_i P_i),
// L_i and U_i the multipliers the sweep leaves in the workspace.  G^< is
// anti-Hermitian, so G^<_{i-1,i} = -(G^<_{i,i-1})^H.  One workgroup per energy;
// per layer 9 complex products (P, C, D, C A_L, D A_R, two for G^<_ii, two for
// G^<_{i,i-1}).  The sweep's pivot inverses g_i are no longer needed: P_i takes
// their slots, and the other blocks reuse the sweep's per-chain scratch slots.
#include "kernels.h"
#include "block_engine.h"

namespace rgfk {

#ifdef RGFK_INST_T

template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void rgf_lesser_kernel(LesserArgs a) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  const int e = blockIdx.x;
  const int l = a.l, b = a.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  double2* g = a.ws + (size_t)e * a.ws_chain;
  const double2* U = g + (size_t)l * bpbp;
  const double2* L = g + (size_t)2 * l * bpbp;
  double2* Pd = g;                                  // P_i in the pivot-inverse slots
  double2* Cb = g + (size_t)3 * l * bpbp;           // 2 blocks: C_i, alternating
  double2* AL = Cb + 2 * bpbp;
  double2* AR = AL + bpbp;
  double2* CA = AR + bpbp;
  double2* DA = CA + bpbp;
  double2* Db = DA + 3 * bpbp;                      // 2 blocks: D_i, alternating
  const double2* sL = a.sigL + (size_t)e * bb;
  const double2* sR = a.sigR + (size_t)e * bb;
  const double2* Gd = a.G + ((size_t)e * 3 * l + l) * bb;
  double2* Gq = a.Gless + (size_t)e * 3 * l * bb;
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pc = [&](const double2* p) { return opnd(p, BP, BP, BP, 1); };
  auto Pn = [&](const double2* p) { return opnd(p, b, b, b); };

  if (a.info[e] != 0) {
    // the sweep failed for this energy: no lesser function either
    const double qnan = __builtin_nan("");
    for (size_t idx = threadIdx.x; idx < (size_t)3 * l * bb; idx += NT) Gq[idx] = make_double2(qnan, qnan);
    return;
  }
  // A_X = i f_X Gamma_X = -f_X (Sigma_X - Sigma_X^H), zero on the padding
  const double fl = a.fL[e], fr = a.fR[e];
  for (int idx = threadIdx.x; idx < BP * BP; idx += NT) {
    const int r = idx / BP, c = idx % BP;
    double2 al = make_double2(0.0, 0.0), ar = make_double2(0.0, 0.0);
    if (r < b && c < b) {
      const double2 s1 = sL[(size_t)r * b + c], s2 = sL[(size_t)c * b + r];
      al = make_double2(-fl * (s1.x - s2.x), -fl * (s1.y + s2.y));
      const double2 q1 = sR[(size_t)r * b + c], q2 = sR[(size_t)c * b + r];
      ar = make_double2(-fr * (q1.x - q2.x), -fr * (q1.y + q2.y));
    }
    AL[idx] = al;
    AR[idx] = ar;
  }
  Acc<T, NW> acc;
  // P_{l-1} = I, P_{i-1} = -U_i P_i
  acc_zero<T, NW>(acc);
  add_identity<T, NW>(acc);
  store<T, NW>(acc, Pd + (size_t)(l - 1) * bpbp, BP, BP, BP);
  __syncthreads();
  for (int i = l - 1; i >= 1; --i) {
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(U + (size_t)i * bpbp), P(Pd + (size_t)i * bpbp), -1.0);
    store<T, NW>(acc, Pd + (size_t)(i - 1) * bpbp, BP, BP, BP);
    __syncthreads();
  }
  for (int i = 0; i < l; ++i) {
    double2* Ci = Cb + (size_t)(i & 1) * bpbp;
    double2* Di = Db + (size_t)(i & 1) * bpbp;
    const double2* Cp = Cb + (size_t)((i + 1) & 1) * bpbp;
    const double2* Dp = Db + (size_t)((i + 1) & 1) * bpbp;
    if (i == 0) {
      load<T, NW>(acc, Pn(Gd));
    } else {
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(L + (size_t)i * bpbp), P(Cp), -1.0);
    }
    store<T, NW>(acc, Ci, BP, BP, BP);
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, Pn(Gd + (size_t)i * bb), P(Pd + (size_t)i * bpbp), 1.0);
    store<T, NW>(acc, Di, BP, BP, BP);
    __syncthreads();
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(Ci), P(AL), 1.0);
    store<T, NW>(acc, CA, BP, BP, BP);
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(Di), P(AR), 1.0);
    store<T, NW>(acc, DA, BP, BP, BP);
    __syncthreads();
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(CA), Pc(Ci), 1.0);
    mma<T, NW>(acc, P(DA), Pc(Di), 1.0);
    store<T, NW>(acc, Gq + ((size_t)l + i) * bb, b, b, b);
    if (i > 0) {
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(CA), Pc(Cp), 1.0);
      mma<T, NW>(acc, P(DA), Pc(Dp), 1.0);
      store<T, NW>(acc, Gq + (size_t)i * bb, b, b, b);
      store_conjT<T, NW>(acc, Gq + ((size_t)2 * l + i - 1) * bb, b, b, b, -1.0);
    }
    __syncthreads();
  }
}

template <int T>
hipError_t launch_lesser_T(const LesserArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  hipLaunchKernelGGL((rgf_lesser_kernel<T, NW>), dim3(a.ne), dim3(64 * NW), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) ktime_mark("rgf_lesser_kernel", s);
  return err;
}

template hipError_t launch_lesser_T<RGFK_INST_T>(const LesserArgs& a, hipStream_t s);

#elif !defined(RGFK_BATCHED_TU)

template <int T>
hipError_t launch_lesser_T(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<1>(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<2>(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<3>(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<4>(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<5>(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<6>(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<7>(const LesserArgs& a, hipStream_t s);
extern template hipError_t launch_lesser_T<8>(const LesserArgs& a, hipStream_t s);

hipError_t launch_rgf_lesser(const LesserArgs& a, hipStream_t s) {
  switch (padded_block(a.b) / 16) {
    case 1: return launch_lesser_T<1>(a, s);
    case 2: return launch_lesser_T<2>(a, s);
    case 3: return launch_lesser_T<3>(a, s);
    case 4: return launch_lesser_T<4>(a, s);
    case 5: return launch_lesser_T<5>(a, s);
    case 6: return launch_lesser_T<6>(a, s);
    case 7: return launch_lesser_T<7>(a, s);
    case 8: return launch_lesser_T<8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

#endif

}  // namespace rgfk
