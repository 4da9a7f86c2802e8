// Lesser Green's function on the band after the n-diagonal sweep (Sec. 2.3): the
// Keldysh equation G^< = G^R Sigma^< G^A with the leads' lesser self-energies
// Sigma^<_X = i f_X Gamma_X on the first and last layer, so that
//     G^<_ij = C_i A_L C_j^H + D_i A_R D_j^H,   |i - j| <= w,   A_X = Sigma^<_X,
// with the first block column C_i = G_{i,0} and the last D_i = G_{i,l-1}.
//   C: C_0 = G_00, C_i = -sum_c L_{i,c} C_c (c in [i-w, i-1]), the downward recursion
//      of the sweep for a column left of the diagonal;
//   D: on row i the last w entries up to column i, s_i = (G_{i,i-w+1}, ..., G_{i,i}),
//      continue to the right by s_j = s_{j-1} T_j (the recursion
//      G_{i,j} = -sum_c G_{i,c} U_{c,j}, j > i), so D_i = s_i P_i with P_{l-1} selecting
//      the last entry and P_{j-1}[t] = P_j[t-1] - U_{j-w+t,j} P_j[w-1] (P_j[-1] = 0),
//      formed from the last layer down.
// One workgroup per energy, on the sweep's workspace: the working band of S is no
// longer needed and holds C, D, A_L C^H and A_R D^H; P takes 2w extra blocks.
#include "nlesser.h"

#include "block_engine.h"

namespace rgfk {

template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void nrgf_lesser_kernel(LesserArgs a, int w) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  const int e = blockIdx.x;
  const int l = a.l, b = a.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  double2* ws = a.ws + (size_t)e * a.ws_chain;
  double2* Sw = ws;                                    // (2w+1) l blocks, free after the sweep
  double2* g = Sw + (size_t)(2 * w + 1) * l * bpbp;
  const double2* U = g + (size_t)l * bpbp;             // U_{c,i} at i w + (i - c - 1)
  const double2* L = U + (size_t)w * l * bpbp;         // L_{i,c} at i w + (i - c - 1)
  double2* R = const_cast<double2*>(L) + (size_t)w * l * bpbp;
  double2* AL = R + (size_t)l * bpbp;                  // the sweep's Gamma_L / Gamma_R slots
  double2* AR = AL + bpbp;
  double2* Pt = AR + 2 * bpbp;                         // 2 w blocks after the sweep's chain
  double2* C = Sw;
  double2* D = Sw + (size_t)l * bpbp;
  double2* X = Sw + (size_t)2 * l * bpbp;              // A_L C_j^H
  double2* Y = Sw + (size_t)3 * l * bpbp;              // A_R D_j^H
  const double2* sL = a.sigL + (size_t)e * bb;
  const double2* sR = a.sigR + (size_t)e * bb;
  const double2* Gout = a.G + (size_t)e * (2 * w + 1) * l * bb;
  double2* Gq = a.Gless + (size_t)e * (2 * w + 1) * l * bb;
  auto Gb = [&](int i, int j) { return Gout + ((size_t)(w + j - i) * l + i) * bb; };
  auto Qb = [&](int i, int j) { return Gq + ((size_t)(w + j - i) * l + i) * bb; };
  auto Ub = [&](int c, int i) { return U + ((size_t)i * w + (i - c - 1)) * bpbp; };
  auto Lb = [&](int i, int c) { return L + ((size_t)i * w + (i - c - 1)) * bpbp; };
  auto Pk = [&](int buf, int t) { return Pt + ((size_t)buf * w + t) * bpbp; };
  auto blk = [&](double2* base, int i) { return base + (size_t)i * bpbp; };
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pc = [&](const double2* p) { return opnd(p, BP, BP, BP, 1); };
  auto Pn = [&](const double2* p) { return opnd(p, b, b, b); };

  if (a.info[e] != 0) {
    // the sweep failed for this energy: no lesser function either
    const double qnan = __builtin_nan("");
    for (size_t idx = threadIdx.x; idx < (size_t)(2 * w + 1) * l * bb; idx += NT) Gq[idx] = make_double2(qnan, qnan);
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
  // first block column
  load<T, NW>(acc, Pn(Gb(0, 0)));
  store<T, NW>(acc, blk(C, 0), BP, BP, BP);
  __syncthreads();
  for (int i = 1; i < l; ++i) {
    const int c0 = i - w < 0 ? 0 : i - w;
    acc_zero<T, NW>(acc);
    for (int c = c0; c < i; ++c) mma<T, NW>(acc, P(Lb(i, c)), P(blk(C, c)), -1.0);
    store<T, NW>(acc, blk(C, i), BP, BP, BP);
    __syncthreads();
  }
  // last block column, from the last layer down
  for (int t = 0; t < w; ++t) {
    acc_zero<T, NW>(acc);
    if (t == w - 1) add_identity<T, NW>(acc);
    store<T, NW>(acc, Pk((l - 1) & 1, t), BP, BP, BP);
  }
  __syncthreads();
  for (int i = l - 1; i >= 0; --i) {
    const int cur = i & 1;
    acc_zero<T, NW>(acc);
    for (int t = 0; t < w; ++t) {
      const int cc = i - w + 1 + t;
      if (cc >= 0) mma<T, NW>(acc, Pn(Gb(i, cc)), P(Pk(cur, t)), 1.0);
    }
    store<T, NW>(acc, blk(D, i), BP, BP, BP);
    if (i >= 1) {
      for (int t = 0; t < w; ++t) {
        const int cc = i - w + t;
        if (t >= 1) load<T, NW>(acc, P(Pk(cur, t - 1))); else acc_zero<T, NW>(acc);
        if (cc >= 0) mma<T, NW>(acc, P(Ub(cc, i)), P(Pk(cur, w - 1)), -1.0);
        store<T, NW>(acc, Pk(cur ^ 1, t), BP, BP, BP);
      }
    }
    __syncthreads();
  }
  // A_L C_j^H and A_R D_j^H
  for (int j = 0; j < l; ++j) {
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(AL), Pc(blk(C, j)), 1.0);
    store<T, NW>(acc, blk(X, j), BP, BP, BP);
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(AR), Pc(blk(D, j)), 1.0);
    store<T, NW>(acc, blk(Y, j), BP, BP, BP);
  }
  __syncthreads();
  // G^<_ij = C_i A_L C_j^H + D_i A_R D_j^H inside the band
  for (int i = 0; i < l; ++i) {
    const int j0 = i - w < 0 ? 0 : i - w, j1 = i + w > l - 1 ? l - 1 : i + w;
    for (int j = j0; j <= j1; ++j) {
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(blk(C, i)), P(blk(X, j)), 1.0);
      mma<T, NW>(acc, P(blk(D, i)), P(blk(Y, j)), 1.0);
      store<T, NW>(acc, Qb(i, j), b, b, b);
    }
  }
}

template <int T>
static hipError_t launch_nl_T(const LesserArgs& a, int w, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  hipLaunchKernelGGL((nrgf_lesser_kernel<T, NW>), dim3(a.ne), dim3(64 * NW), 0, s, a, w);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) ktime_mark("nrgf_lesser_kernel", s);
  return err;
}

hipError_t launch_nrgf_lesser(const LesserArgs& a, int w, hipStream_t s) {
  switch (padded_block(a.b) / 16) {
    case 1: return launch_nl_T<1>(a, w, s);
    case 2: return launch_nl_T<2>(a, w, s);
    case 3: return launch_nl_T<3>(a, w, s);
    case 4: return launch_nl_T<4>(a, w, s);
    case 5: return launch_nl_T<5>(a, w, s);
    case 6: return launch_nl_T<6>(a, w, s);
    case 7: return launch_nl_T<7>(a, w, s);
    case 8: return launch_nl_T<8>(a, w, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rgfk
