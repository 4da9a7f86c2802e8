// Retarded self-energies of semi-infinite periodic leads, batched over energies
// (the inputs Sigma^r that the selected inversion takes as given).
//
// A lead repeats principal layers with on-layer block H00 and coupling H01 to the
// next layer away from the device.  Its surface Green's function solves
// g_s = (z - H00 - H01 g_s H10)^{-1}, z = E + i eta, H10 = H01^H; it is computed by
// the decimation of Lopez Sancho, Lopez Sancho and Rubio (J. Phys. F 15, 851
// (1985)): from eps_s = eps = H00, alpha = H01, beta = H10, each step
//     g = (z - eps)^{-1},
//     eps_s += alpha g beta,   eps += alpha g beta + beta g alpha,
//     alpha <- alpha g alpha,  beta <- beta g beta,
// halves the remaining chain, until max|alpha_ij| + max|beta_ij| < tolerance; then
// g_s = (z - eps_s)^{-1} and Sigma = Hc g_s Hc^H, Hc the coupling from the device
// layer to the lead's surface layer.  One workgroup per energy; per step one
// Gauss-Jordan inverse and six block products on the register-resident block
// engine.
#include "kernels.h"
#include "block_engine.h"

namespace rgfk {

#ifdef RGFK_INST_T

template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void lead_decimation_kernel(LeadArgs a) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  __shared__ GJShared sh;
  __shared__ double red[NW];
  const int e = blockIdx.x;
  const int b = a.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  double2* es = a.ws + (size_t)e * a.ws_chain;    // eps_s (b x b)
  double2* ep = es + bpbp;                        // eps (b x b)
  double2* al = ep + bpbp;                        // alpha (bp x bp, zero padding)
  double2* be = al + bpbp;                        // beta
  double2* ag = be + bpbp;                        // alpha g
  double2* bg = ag + bpbp;                        // beta g
  double2* g = bg + bpbp;                         // (z - eps)^{-1}
  double2* tmp = g + bpbp;
  const double2 z = make_double2(a.E[e], a.eta);
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pn = [&](const double2* p) { return opnd(p, b, b, b); };
  Acc<T, NW> acc;

  // element-wise maximum modulus of the accumulator (NaN wins)
  auto acc_absmax = [&]() {
    double m = 0.0;
#pragma unroll
    for (int r = 0; r < Acc<T, NW>::RR; ++r)
#pragma unroll
      for (int c = 0; c < Acc<T, NW>::RC; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double x = sqrt(acc.re[r][c][v] * acc.re[r][c][v] + acc.im[r][c][v] * acc.im[r][c][v]);
          m = (x > m || x != x) ? x : m;
        }
    return m;
  };

  load<T, NW>(acc, Pn(a.H00));
  store<T, NW>(acc, es, b, b, b);
  store<T, NW>(acc, ep, b, b, b);
  load<T, NW>(acc, Pn(a.H01));
  store<T, NW>(acc, al, BP, BP, BP);
  load<T, NW>(acc, opnd(a.H01, b, b, b, 1));
  store<T, NW>(acc, be, BP, BP, BP);
  __syncthreads();

  int steps = -1;
  for (int k = 1; k <= a.max_steps; ++k) {
    // g = (z - eps)^{-1} (identity on the padding)
    assemble_diag<T, NW>(acc, ep, b, z, nullptr, nullptr, false);
    gj_invert<T, NW>(acc, g, sh);
    __syncthreads();
    if (sh.bad) {
      steps = -2;
      break;
    }
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(al), P(g), 1.0);
    store<T, NW>(acc, ag, BP, BP, BP);
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(be), P(g), 1.0);
    store<T, NW>(acc, bg, BP, BP, BP);
    __syncthreads();
    // eps_s += alpha g beta;  eps += alpha g beta + beta g alpha
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(ag), P(be), 1.0);
    store<T, NW>(acc, tmp, BP, BP, BP);
    add_from<T, NW>(acc, Pn(es));
    store<T, NW>(acc, es, b, b, b);
    load<T, NW>(acc, P(tmp));
    add_from<T, NW>(acc, Pn(ep));
    mma<T, NW>(acc, P(bg), P(al), 1.0);
    store<T, NW>(acc, ep, b, b, b);
    // alpha <- alpha g alpha, beta <- beta g beta (every wave done reading the old
    // alpha / beta before they are overwritten)
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(ag), P(al), 1.0);
    const double amax = acc_absmax();
    __syncthreads();
    store<T, NW>(acc, al, BP, BP, BP);
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(bg), P(be), 1.0);
    const double bmax = acc_absmax();
    __syncthreads();
    store<T, NW>(acc, be, BP, BP, BP);
    __syncthreads();
    const double m = wg_max<NW>(amax, red) + wg_max<NW>(bmax, red);
    if (m < a.tol) {
      steps = k;
      break;
    }
  }
  double2* S = a.sigma + (size_t)e * bb;
  if (steps > 0) {
    // g_s = (z - eps_s)^{-1};  Sigma = Hc g_s Hc^H
    assemble_diag<T, NW>(acc, es, b, z, nullptr, nullptr, false);
    gj_invert<T, NW>(acc, g, sh);
    __syncthreads();
    if (sh.bad) steps = -2;
  }
  if (steps > 0) {
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, Pn(a.Hc), P(g), 1.0);
    store<T, NW>(acc, tmp, BP, BP, BP);
    __syncthreads();
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, P(tmp), opnd(a.Hc, b, b, b, 1), 1.0);
    store<T, NW>(acc, S, b, b, b);
  } else {
    const double qnan = __builtin_nan("");
    for (size_t idx = threadIdx.x; idx < bb; idx += NT) S[idx] = make_double2(qnan, qnan);
  }
  if (threadIdx.x == 0) a.steps[e] = steps;
}

template <int T>
hipError_t launch_leads_T(const LeadArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  hipLaunchKernelGGL((lead_decimation_kernel<T, NW>), dim3(a.ne), dim3(64 * NW), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_leads_T<RGFK_INST_T>(const LeadArgs& a, hipStream_t s);

#elif !defined(RGFK_BATCHED_TU)

template <int T>
hipError_t launch_leads_T(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<1>(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<2>(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<3>(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<4>(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<5>(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<6>(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<7>(const LeadArgs& a, hipStream_t s);
extern template hipError_t launch_leads_T<8>(const LeadArgs& a, hipStream_t s);

size_t lead_ws_chain_elems(int bp) { return (size_t)8 * bp * bp; }

hipError_t launch_lead_decimation(const LeadArgs& a, hipStream_t s) {
  switch (padded_block(a.b) / 16) {
    case 1: return launch_leads_T<1>(a, s);
    case 2: return launch_leads_T<2>(a, s);
    case 3: return launch_leads_T<3>(a, s);
    case 4: return launch_leads_T<4>(a, s);
    case 5: return launch_leads_T<5>(a, s);
    case 6: return launch_leads_T<6>(a, s);
    case 7: return launch_leads_T<7>(a, s);
    case 8: return launch_leads_T<8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

#endif

}  // namespace rgfk
