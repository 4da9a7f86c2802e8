// DDRGF for block tridiagonal systems (paper Sec. 3, Algorithm 2), one level, on gfx950.
//
// Layout (the figure of Sec. 3): m pairs (interior D2^k, separator D1^k), k = 0..m-1;
// interior k is layers [a_k, a_k + n_k - 1], separator k is the single layer
// p_k = a_k + n_k; the chain starts with an interior at layer 0 and ends with the
// separator p_{m-1} = l - 1.  The l - m interior layers are split as evenly as
// possible, the first (l - m) mod m interiors taking one extra layer.
//
// Kernels (all energies and domains batched in each launch):
//   1. ddrgf_interior_kernel  one workgroup per (energy, interior): RGF of the
//      closed interior (Algorithm 1) giving the band of X = (M_{D2^k})^{-1}, written
//      straight into G, plus the halo products needed later (the "internal halos"):
//        CL_i = X_{i,0} M_{a,qL},  RL_i = M_{qL,a} X_{0,i}     (first column / row)
//        CR_i = X_{i,n-1} M_{e,qR}, RR_i = M_{qR,e} X_{n-1,i}  (last column / row)
//      with qL = a - 1, qR = e + 1 the neighbouring separators.  First column/row
//      follow X_{i,0} = -L_i X_{i-1,0}, X_{0,i} = -X_{0,i-1} U_i; last column/row
//      X_{i,n-1} = X_ii P_i, X_{n-1,i} = Q_i X_ii with P_i = -U_{i+1} P_{i+1},
//      Q_i = -Q_{i+1} L_{i+1}; the couplings are folded into P, Q at the end layer.
//   2. ddrgf_schur_kernel  one workgroup per (energy, separator): the reduced
//      system T_S = T_11 - T_12 T_22^{-1} T_21 (eq. Schur complement in DDRGF),
//      block tridiagonal over the separators (Proposition 4) including the
//      couplings between neighbouring separators through one interior:
//        S_kk      = M_pp - M_{p,e_k} X^(k)_{ee} M_{e_k,p} - M_{p,a_{k+1}} X^(k+1)_{aa} M_{a_{k+1},p}
//        S_{k,k+1} = -M_{p_k,a_{k+1}} X^(k+1)_{a,e} M_{e_{k+1},p_{k+1}}
//        S_{k+1,k} = -M_{p_{k+1},e_{k+1}} X^(k+1)_{e,a} M_{a_{k+1},p_k}
//   3. the sequential sweep kernel on the reduced system ("direct" mode) gives the
//      band of G_S = T_S^{-1} and its first block row.
//   4. ddrgf_recover_kernel  one workgroup per (energy, interior): Algorithm 2 step 4,
//        G_{D2,D2} = X + X T_21 G_S T_12 X,  G_{D2,D1} = -X T_21 G_S,  G_{D1,D2} = -G_S T_12 X,
//      restricted to the band and added in place; step 5 (inverse reordering) is
//      the index map of the layout, nothing is permuted.
//   5. ddrgf_finalize_kernel  one workgroup per energy: T(E) from
//      G_{0,l-1} = -CR^(0)_0 G_S(0, m-1), status and NaN fill.
#include "block_engine.h"
#include "kernels.h"

namespace rgfk {

struct DDLayout {
  int base, rem;
  __host__ __device__ int n(int k) const { return base + (k < rem ? 1 : 0); }
  __host__ __device__ int a(int k) const { return k * (base + 1) + (k < rem ? k : rem); }
  __host__ __device__ int p(int k) const { return a(k) + n(k); }
};

__host__ __device__ inline DDLayout dd_layout(int l, int m) {
  DDLayout d;
  d.base = (l - m) / m;
  d.rem = (l - m) % m;
  return d;
}

#ifndef RGFK_INST_T
size_t ddrgf_interior_ws_elems(int nmax, int bp) { return (size_t)(9 * (size_t)nmax + 2) * bp * bp; }

__global__ void herm_flag_init_kernel(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 1;
}

// Clears *flag unless the band of H is exactly Hermitian: H_ii = H_ii^H and
// H_{i+1,i} = H_{i,i+1}^H entry by entry (NaN entries count as a mismatch).
__global__ void herm_check_kernel(const double2* H, int l, int b, int* flag) {
  const size_t bb = (size_t)b * b;
  const size_t total = (size_t)2 * l * bb;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx % b), r = (int)((idx / b) % b);
    const int i = (int)((idx / bb) % l);
    const bool diag = idx < (size_t)l * bb;
    double2 x, y;
    if (diag) {
      x = H[((size_t)l + i) * bb + (size_t)r * b + c];
      y = H[((size_t)l + i) * bb + (size_t)c * b + r];
    } else {
      if (i + 1 >= l) continue;
      x = H[(size_t)(i + 1) * bb + (size_t)r * b + c];              // block (i+1, i)
      y = H[((size_t)2 * l + i) * bb + (size_t)c * b + r];          // block (i, i+1), transposed
    }
    if (!(x.x == y.x && x.y == -y.y)) *flag = 0;
  }
}
#endif

// Diagonal block of M for global layer i: (E + i eta) I - H_ii - [i==0] Sigma_L - [i==l-1] Sigma_R.
// In direct mode (inner levels) the diagonal block is read as it is, with the
// identity on the padding.
template <int T, int NW>
__device__ __forceinline__ void diag_M(Acc<T, NW>& acc, const DDArgs& a, int e, int i, bool add = false) {
  const size_t bb = (size_t)a.b * a.b;
  if (a.direct) {
    if (!add) acc_zero<T, NW>(acc);
    add_from<T, NW>(acc, opnd(a.H + (size_t)(a.l + i) * bb, a.b, a.b, a.b));
    add_identity_beyond<T, NW>(acc, a.b);
    return;
  }
  const double2 z = make_double2(a.E[e], a.eta_d);
  assemble_diag<T, NW>(acc, a.H + (size_t)(a.l + i) * bb, a.b, z,
                       i == 0 ? a.sigL + (size_t)e * bb : nullptr,
                       i == a.l - 1 ? a.sigR + (size_t)e * bb : nullptr, add);
}

// H band accessors: block (i, i-1), (i, i+1)
__device__ __forceinline__ const double2* Hlo(const DDArgs& a, int i) {
  return a.H + (size_t)i * a.b * a.b;
}
__device__ __forceinline__ const double2* Hup(const DDArgs& a, int i) {
  return a.H + (size_t)(2 * a.l + i) * a.b * a.b;
}

// ---------------------------------------------------------------------------
// 1. interiors
// ---------------------------------------------------------------------------
template <int T, int NW, int MIXED>
__device__ __forceinline__ void interior_general(const DDArgs& a, int c, GJShared& sh) {
  constexpr int BP = 16 * T;
  const int e = c / a.m, k = c % a.m;
  const DDLayout lay = dd_layout(a.l, a.m);
  const int n = lay.n(k), a0 = lay.a(k), qR = lay.p(k), qL = a0 - 1;
  const int b = a.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const int nmax = lay.base + 1;
  double2* ws = a.ws_int + (size_t)c * a.ws_int_chain;
  double2* g = ws;
  double2* U = g + (size_t)nmax * bpbp;
  double2* L = U + (size_t)nmax * bpbp;
  double2* Pt = L + (size_t)nmax * bpbp;
  double2* Qt = Pt + (size_t)nmax * bpbp;
  double2* CL = Qt + (size_t)nmax * bpbp;
  double2* CR = CL + (size_t)nmax * bpbp;
  double2* RL = CR + (size_t)nmax * bpbp;
  double2* RR = RL + (size_t)nmax * bpbp;
  double2* Gout = a.G + (size_t)e * 3 * a.l * bb;
  double2* Gl = Gout;
  double2* Gd = Gout + (size_t)a.l * bb;
  double2* Gu = Gout + (size_t)2 * a.l * bb;
  const bool left = k > 0;

  int bad_layer = -1;
  Acc<T, NW> acc;

  // ---------------- upward pass over the closed interior ----------------
  double2* Ssave = ws + (size_t)9 * nmax * bpbp;     // refinement scratch (2 blocks)
  double2* Rres = Ssave + bpbp;
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pb = [&](const double2* p) { return opnd(p, b, b, b); };
  diag_M<T, NW>(acc, a, e, a0 + n - 1);
  for (int i = n - 1; i >= 0; --i) {
    double2* gi = g + (size_t)i * bpbp;
    if (MIXED) store<T, NW>(acc, Ssave, BP, BP, BP);
    gj_invert<T, NW>(acc, gi, sh);
    if (sh.bad && bad_layer < 0) bad_layer = a0 + i;
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
    if (i == n - 1) {
      // P_{n-1} folded with M_{e,qR} = -H_{e,e+1};  Q_{n-1} with M_{qR,e} = -H_{qR,qR-1}
      load<T, NW>(acc, Pb(Hup(a, a0 + n - 1)), -1.0);
      store<T, NW>(acc, Pt + (size_t)i * bpbp, BP, BP, BP);
      load<T, NW>(acc, Pb(Hlo(a, qR)), -1.0);
      store<T, NW>(acc, Qt + (size_t)i * bpbp, BP, BP, BP);
      __syncthreads();
    }
    if (i == 0) break;
    const int gl = a0 + i;
    gemm_to<MIXED, T, NW>(acc, P(gi), Pb(Hlo(a, gl)), -1.0);
    store<T, NW>(acc, L + (size_t)i * bpbp, BP, BP, BP);
    gemm_to<MIXED, T, NW>(acc, Pb(Hup(a, gl - 1)), P(gi), -1.0);
    store<T, NW>(acc, U + (size_t)i * bpbp, BP, BP, BP);
    __syncthreads();
    gemm_to<MIXED, T, NW>(acc, P(U + (size_t)i * bpbp), P(Pt + (size_t)i * bpbp), -1.0);
    store<T, NW>(acc, Pt + (size_t)(i - 1) * bpbp, BP, BP, BP);
    gemm_to<MIXED, T, NW>(acc, P(Qt + (size_t)i * bpbp), P(L + (size_t)i * bpbp), -1.0);
    store<T, NW>(acc, Qt + (size_t)(i - 1) * bpbp, BP, BP, BP);
    // S_{i-1} = M_{i-1,i-1} - M_{i-1,i} L_i = M_{i-1,i-1} + H_{i-1,i} L_i
    gemm_to<MIXED, T, NW>(acc, Pb(Hup(a, gl - 1)), P(L + (size_t)i * bpbp), 1.0);
    diag_M<T, NW>(acc, a, e, gl - 1, true);
    __syncthreads();
  }

  // ---------------- downward pass, band of X and halo products ----------------
  load<T, NW>(acc, P(g));
  store<T, NW>(acc, Gd + (size_t)a0 * bb, b, b, b);
  __syncthreads();
  const Opnd X00 = Pb(Gd + (size_t)a0 * bb);
  if (left) {
    gemm_to<MIXED, T, NW>(acc, X00, Pb(Hlo(a, a0)), -1.0);          // X_00 M_{a,qL}
    store<T, NW>(acc, CL, BP, BP, BP);
    gemm_to<MIXED, T, NW>(acc, Pb(Hup(a, qL)), X00, -1.0);          // M_{qL,a} X_00
    store<T, NW>(acc, RL, BP, BP, BP);
  }
  gemm_to<MIXED, T, NW>(acc, X00, P(Pt), 1.0);
  store<T, NW>(acc, CR, BP, BP, BP);
  gemm_to<MIXED, T, NW>(acc, P(Qt), X00, 1.0);
  store<T, NW>(acc, RR, BP, BP, BP);
  __syncthreads();
  for (int i = 1; i < n; ++i) {
    const int gl = a0 + i;
    const Opnd Xp = Pb(Gd + (size_t)(gl - 1) * bb);
    const Opnd Ui = P(U + (size_t)i * bpbp);
    const Opnd Li = P(L + (size_t)i * bpbp);
    gemm_to<MIXED, T, NW>(acc, Xp, Ui, -1.0);
    store<T, NW>(acc, Gu + (size_t)(gl - 1) * bb, b, b, b);
    gemm_to<MIXED, T, NW>(acc, Li, Xp, -1.0);
    store<T, NW>(acc, Gl + (size_t)gl * bb, b, b, b);
    if (left) {
      gemm_to<MIXED, T, NW>(acc, Li, P(CL + (size_t)(i - 1) * bpbp), -1.0);
      store<T, NW>(acc, CL + (size_t)i * bpbp, BP, BP, BP);
      gemm_to<MIXED, T, NW>(acc, P(RL + (size_t)(i - 1) * bpbp), Ui, -1.0);
      store<T, NW>(acc, RL + (size_t)i * bpbp, BP, BP, BP);
    }
    __syncthreads();
    gemm_to<MIXED, T, NW>(acc, Li, Pb(Gu + (size_t)(gl - 1) * bb), -1.0);
    add_from<T, NW>(acc, P(g + (size_t)i * bpbp));
    store<T, NW>(acc, Gd + (size_t)gl * bb, b, b, b);
    __syncthreads();
    const Opnd Xii = Pb(Gd + (size_t)gl * bb);
    gemm_to<MIXED, T, NW>(acc, Xii, P(Pt + (size_t)i * bpbp), 1.0);
    store<T, NW>(acc, CR + (size_t)i * bpbp, BP, BP, BP);
    gemm_to<MIXED, T, NW>(acc, P(Qt + (size_t)i * bpbp), Xii, 1.0);
    store<T, NW>(acc, RR + (size_t)i * bpbp, BP, BP, BP);
  }
  if (threadIdx.x == 0) a.info_part[(size_t)e * (a.m + 1) + k] = bad_layer >= 0 ? bad_layer + 1 : 0;
}

// Closed interior with a Hermitian matrix (H Hermitian, no lead in the interior,
// eta_d = 0, E real): X = M_D^{-1} is Hermitian, U_i = L_i^H, Q_i = P_i^H,
// X_{i-1,i} = X_{i,i-1}^H, and the halo products RL = CL^H, RR = CR^H, so per layer
// the upward pass forms L_i, P_{i-1} = -L_i^H P_i and the Schur update, and the
// downward pass X_{i,i-1}, X_ii, CL_i, CR_i: 7 products instead of 12.  RL and RR
// are not stored; the recovery reads CL^H and CR^H.
template <int T, int NW, int MIXED>
__device__ __forceinline__ void interior_herm(const DDArgs& a, int c, GJShared& sh) {
  constexpr int BP = 16 * T;
  const int e = c / a.m, k = c % a.m;
  const DDLayout lay = dd_layout(a.l, a.m);
  const int n = lay.n(k), a0 = lay.a(k);
  const int b = a.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const int nmax = lay.base + 1;
  double2* ws = a.ws_int + (size_t)c * a.ws_int_chain;
  // the general path's layout (g, U, L, P, Q, CL, CR, RL, RR); U, Q, RL, RR unused
  double2* g = ws;
  double2* L = g + (size_t)2 * nmax * bpbp;
  double2* Pt = L + (size_t)nmax * bpbp;
  double2* CL = Pt + (size_t)2 * nmax * bpbp;
  double2* CR = CL + (size_t)nmax * bpbp;
  double2* Gout = a.G + (size_t)e * 3 * a.l * bb;
  double2* Gl = Gout;
  double2* Gd = Gout + (size_t)a.l * bb;
  double2* Gu = Gout + (size_t)2 * a.l * bb;
  int bad_layer = -1;
  Acc<T, NW> acc;
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pb = [&](const double2* p) { return opnd(p, b, b, b); };

  // ---------------- upward pass ----------------
  diag_M<T, NW>(acc, a, e, a0 + n - 1);
  for (int i = n - 1; i >= 0; --i) {
    double2* gi = g + (size_t)i * bpbp;
    gj_invert<T, NW>(acc, gi, sh);
    if (sh.bad && bad_layer < 0) bad_layer = a0 + i;
    __syncthreads();
    if (i == n - 1) {
      // P_{n-1} folded with M_{e,qR} = -H_{e,e+1}
      load<T, NW>(acc, Pb(Hup(a, a0 + n - 1)), -1.0);
      store<T, NW>(acc, Pt + (size_t)i * bpbp, BP, BP, BP);
      __syncthreads();
    }
    if (i == 0) break;
    const int gl = a0 + i;
    gemm_to<MIXED, T, NW>(acc, P(gi), Pb(Hlo(a, gl)), -1.0);
    store<T, NW>(acc, L + (size_t)i * bpbp, BP, BP, BP);
    __syncthreads();
    // P_{i-1} = -U_i P_i = -L_i^H P_i
    gemm_to<MIXED, T, NW>(acc, opnd(L + (size_t)i * bpbp, BP, BP, BP, 1), P(Pt + (size_t)i * bpbp), -1.0);
    store<T, NW>(acc, Pt + (size_t)(i - 1) * bpbp, BP, BP, BP);
    // S_{i-1} = M_{i-1,i-1} + H_{i-1,i} L_i
    gemm_to<MIXED, T, NW>(acc, Pb(Hup(a, gl - 1)), P(L + (size_t)i * bpbp), 1.0);
    diag_M<T, NW>(acc, a, e, gl - 1, true);
    __syncthreads();
  }

  // ---------------- downward pass ----------------
  load<T, NW>(acc, P(g));
  store<T, NW>(acc, Gd + (size_t)a0 * bb, b, b, b);
  __syncthreads();
  const Opnd X00 = Pb(Gd + (size_t)a0 * bb);
  gemm_to<MIXED, T, NW>(acc, X00, Pb(Hlo(a, a0)), -1.0);            // CL_0 = X_00 M_{a,qL}
  store<T, NW>(acc, CL, BP, BP, BP);
  gemm_to<MIXED, T, NW>(acc, X00, P(Pt), 1.0);                      // CR_0 = X_00 P_0
  store<T, NW>(acc, CR, BP, BP, BP);
  __syncthreads();
  for (int i = 1; i < n; ++i) {
    const int gl = a0 + i;
    const Opnd Xp = Pb(Gd + (size_t)(gl - 1) * bb);
    const Opnd Li = P(L + (size_t)i * bpbp);
    // X_{i,i-1} = -L_i X_{i-1,i-1};  X_{i-1,i} = X_{i,i-1}^H
    gemm_to<MIXED, T, NW>(acc, Li, Xp, -1.0);
    store<T, NW>(acc, Gl + (size_t)gl * bb, b, b, b);
    store_conjT<T, NW>(acc, Gu + (size_t)(gl - 1) * bb, b, b, b);
    gemm_to<MIXED, T, NW>(acc, Li, P(CL + (size_t)(i - 1) * bpbp), -1.0);
    store<T, NW>(acc, CL + (size_t)i * bpbp, BP, BP, BP);
    __syncthreads();
    // X_ii = g_i - L_i X_{i-1,i}
    gemm_to<MIXED, T, NW>(acc, Li, Pb(Gu + (size_t)(gl - 1) * bb), -1.0);
    add_from<T, NW>(acc, P(g + (size_t)i * bpbp));
    store<T, NW>(acc, Gd + (size_t)gl * bb, b, b, b);
    __syncthreads();
    gemm_to<MIXED, T, NW>(acc, Pb(Gd + (size_t)gl * bb), P(Pt + (size_t)i * bpbp), 1.0);
    store<T, NW>(acc, CR + (size_t)i * bpbp, BP, BP, BP);
  }
  if (threadIdx.x == 0) a.info_part[(size_t)e * (a.m + 1) + k] = bad_layer >= 0 ? bad_layer + 1 : 0;
}

// Whether interior k of this solve takes the Hermitian path: H was found exactly
// Hermitian on the device, eta_d = 0, and the interior holds no lead (k > 0).
__device__ __forceinline__ bool herm_interior(const DDArgs& a, int k) {
  return a.herm != nullptr && *a.herm != 0 && a.eta_d == 0.0 && k > 0;
}

template <int T, int NW, int MIXED>
__global__ __launch_bounds__(64 * NW, 1) void ddrgf_interior_kernel(DDArgs a) {
  __shared__ GJShared sh;
  const int c = blockIdx.x;
  a.H += (size_t)(c / a.m) * a.h_stride;
  if (!MIXED && herm_interior(a, c % a.m))
    interior_herm<T, NW, MIXED>(a, c, sh);
  else
    interior_general<T, NW, MIXED>(a, c, sh);
}

// ---------------------------------------------------------------------------
// 2. reduced system on the separators
// ---------------------------------------------------------------------------
template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void ddrgf_schur_kernel(DDArgs a) {
  constexpr int BP = 16 * T;
  const int c = blockIdx.x;
  const int e = c / a.m, k = c % a.m;
  a.H += (size_t)e * a.h_stride;
  const DDLayout lay = dd_layout(a.l, a.m);
  const int b = a.b, m = a.m;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const int nmax = lay.base + 1;
  const int p = lay.p(k);
  auto halo = [&](int kk, int which, int i) -> const double2* {
    // which: 0 CL, 1 CR, 2 RL, 3 RR
    const double2* ws = a.ws_int + (size_t)(e * m + kk) * a.ws_int_chain;
    return ws + ((size_t)(5 + which) * nmax + i) * bpbp;
  };
  double2* MS = a.MS + (size_t)e * 3 * m * bb;    // direct band of T_S
  Acc<T, NW> acc;
  // S_kk = M_pp - M_{p,e_k} CR^(k)_{n-1} - M_{p,a_{k+1}} CL^(k+1)_0,  M_{p,e} = -H_{p,p-1}, M_{p,a} = -H_{p,p+1}
  diag_M<T, NW>(acc, a, e, p);
  mma<T, NW>(acc, opnd(Hlo(a, p), b, b, b), opnd(halo(k, 1, lay.n(k) - 1), BP, BP, BP), 1.0);
  if (k + 1 < m)
    mma<T, NW>(acc, opnd(Hup(a, p), b, b, b), opnd(halo(k + 1, 0, 0), BP, BP, BP), 1.0);
  store<T, NW>(acc, MS + (size_t)(m + k) * bb, b, b, b);
  if (k + 1 < m) {
    const int p1 = lay.p(k + 1);
    // S_{k,k+1} = -M_{p_k,a_{k+1}} CR^(k+1)_0 = H_{p,p+1} CR^(k+1)_0
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, opnd(Hup(a, p), b, b, b), opnd(halo(k + 1, 1, 0), BP, BP, BP), 1.0);
    store<T, NW>(acc, MS + (size_t)(2 * m + k) * bb, b, b, b);
    // S_{k+1,k} = -M_{p_{k+1},e_{k+1}} CL^(k+1)_{n-1} = H_{p1,p1-1} CL^(k+1)_{n-1}
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, opnd(Hlo(a, p1), b, b, b), opnd(halo(k + 1, 0, lay.n(k + 1) - 1), BP, BP, BP), 1.0);
    store<T, NW>(acc, MS + (size_t)(k + 1) * bb, b, b, b);
  }
}

// ---------------------------------------------------------------------------
// 4. recovery of the interior blocks and the separator couplings
// ---------------------------------------------------------------------------
template <int T, int NW, int MIXED>
__global__ __launch_bounds__(64 * NW, 1) void ddrgf_recover_kernel(DDArgs a) {
  constexpr int BP = 16 * T;
  const int c = blockIdx.x;
  const int e = c / a.m, k = c % a.m;
  a.H += (size_t)e * a.h_stride;
  const DDLayout lay = dd_layout(a.l, a.m);
  const int n = lay.n(k), a0 = lay.a(k), qR = lay.p(k), qL = a0 - 1;
  const int b = a.b, m = a.m;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const int nmax = lay.base + 1;
  const bool left = k > 0;
  double2* ws = a.ws_int + (size_t)c * a.ws_int_chain;
  const double2* CL = ws + (size_t)5 * nmax * bpbp;
  const double2* CR = ws + (size_t)6 * nmax * bpbp;
  const double2* RL = ws + (size_t)7 * nmax * bpbp;
  const double2* RR = ws + (size_t)8 * nmax * bpbp;
  // Hermitian interiors keep RL = CL^H and RR = CR^H implicit
  const bool herm = herm_interior(a, k);
  double2* VL = ws + (size_t)9 * nmax * bpbp;     // 1 block
  double2* VR = VL + bpbp;                         // 1 block (reuses the spare blocks)
  const double2* GS = a.GS + (size_t)e * 3 * m * bb;
  const Opnd ZRR = opnd(GS + (size_t)(m + k) * bb, b, b, b);
  const int km = left ? k - 1 : k;   // (unused when there is no left separator)
  const Opnd ZLL = opnd(GS + (size_t)(m + km) * bb, b, b, b);
  const Opnd ZLR = opnd(GS + (size_t)(2 * m + km) * bb, b, b, b);      // G_S(k-1, k)
  const Opnd ZRL = opnd(GS + (size_t)(k)*bb, b, b, b);                 // G_S(k, k-1)
  double2* Gout = a.G + (size_t)e * 3 * a.l * bb;
  double2* Gl = Gout;
  double2* Gd = Gout + (size_t)a.l * bb;
  double2* Gu = Gout + (size_t)2 * a.l * bb;
  auto blk = [&](const double2* base, int i) { return opnd(base + (size_t)i * bpbp, BP, BP, BP); };
  auto rblk = [&](const double2* base, const double2* cbase, int i) {
    return herm ? opnd(cbase + (size_t)i * bpbp, BP, BP, BP, 1) : blk(base, i);
  };

  Acc<T, NW> acc;
  // two-term products [X, Y] [Z1; Z2] as one product over a doubled k range when mixed
  auto gemm2 = [&](const Opnd& A1, const Opnd& B1, const Opnd& A2, const Opnd& B2, bool two) {
    gemm_to<MIXED, T, NW>(acc, A1, B1, 1.0);
    if (two) {
      if (MIXED) {
        Acc<T, NW> tmp;
        gemm_f32<T, NW>(tmp, A2, B2, 1.0);
        for (int r = 0; r < Acc<T, NW>::RR; ++r)
          for (int c = 0; c < Acc<T, NW>::RC; ++c) {
            acc.re[r][c] += tmp.re[r][c];
            acc.im[r][c] += tmp.im[r][c];
          }
      } else {
        mma<T, NW>(acc, A2, B2, 1.0);
      }
    }
  };
  for (int i = 0; i < n; ++i) {
    const int gi = a0 + i;
    // V_i = [CL_i, CR_i] Z
    if (left)
      gemm2(blk(CR, i), ZRR, blk(CL, i), ZLR, true);
    else
      gemm2(blk(CR, i), ZRR, blk(CR, i), ZRR, false);
    store<T, NW>(acc, VR, BP, BP, BP);
    if (i == n - 1) store<T, NW>(acc, Gu + (size_t)gi * bb, b, b, b, -1.0);   // G_{e,qR} = -V^R
    if (left) {
      gemm2(blk(CL, i), ZLL, blk(CR, i), ZRL, true);
      store<T, NW>(acc, VL, BP, BP, BP);
      if (i == 0) store<T, NW>(acc, Gl + (size_t)gi * bb, b, b, b, -1.0);     // G_{a,qL} = -V^L
    }
    __syncthreads();
    // G_ij += V^L_i RL_j + V^R_i RR_j for j = i-1, i, i+1 inside the interior
    for (int d = -1; d <= 1; ++d) {
      const int j = i + d;
      if (j < 0 || j >= n) continue;
      double2* dst = (d == 0 ? Gd : (d < 0 ? Gl : Gu)) + (size_t)gi * bb;
      gemm2(opnd(VR, BP, BP, BP), rblk(RR, CR, j), opnd(VL, BP, BP, BP), rblk(RL, CL, j), left);
      add_from<T, NW>(acc, opnd(dst, b, b, b));
      store<T, NW>(acc, dst, b, b, b);
    }
    __syncthreads();
  }
  // G_{qR,e} = -(G_S(k,k-1) RL_{n-1} + G_S(k,k) RR_{n-1});  G_{qL,a} = -(G_S(k-1,k-1) RL_0 + G_S(k-1,k) RR_0)
  acc_zero<T, NW>(acc);
  if (left) mma<T, NW>(acc, ZRL, rblk(RL, CL, n - 1), -1.0);
  mma<T, NW>(acc, ZRR, rblk(RR, CR, n - 1), -1.0);
  store<T, NW>(acc, Gl + (size_t)qR * bb, b, b, b);
  if (left) {
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, ZLL, rblk(RL, CL, 0), -1.0);
    mma<T, NW>(acc, ZLR, rblk(RR, CR, 0), -1.0);
    store<T, NW>(acc, Gu + (size_t)qL * bb, b, b, b);
  }
  // separator diagonal block
  load<T, NW>(acc, ZRR);
  store<T, NW>(acc, Gd + (size_t)qR * bb, b, b, b);
}

// ---------------------------------------------------------------------------
// 5. per-energy transmission, status and NaN fill
// ---------------------------------------------------------------------------
template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void ddrgf_finalize_kernel(DDArgs a) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  __shared__ double red[NW];
  __shared__ int s_info;
  const int e = blockIdx.x, t = threadIdx.x;
  const int b = a.b, m = a.m;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const DDLayout lay = dd_layout(a.l, m);
  const int nmax = lay.base + 1;
  if (t == 0) {
    int inf = 0;
    // first failing pivot in elimination order: interiors, then the reduced system
    for (int k = 0; k <= m && inf == 0; ++k) {
      const int v = a.info_part[(size_t)e * (m + 1) + k];
      if (v != 0) inf = (k < m) ? v : lay.p(v - 1) + 1;
    }
    s_info = inf;
  }
  __syncthreads();
  const int inf = s_info;
  double2* scr = a.ws_fin + (size_t)e * 4 * bpbp;
  double2* G0L = scr;
  double2* GamL = scr + bpbp;
  double2* GamR = scr + 2 * bpbp;
  double2* X1 = scr + 3 * bpbp;
  double Tval = 0.0;
  if (a.T || a.first_last) {
    // block (0, l-1) of the inverse: -(X^(0) T21)_{0, D1^0} G_S(0, m-1)
    const double2* CR0 = a.ws_int + (size_t)(e * m) * a.ws_int_chain + (size_t)6 * nmax * bpbp;
    const double2* GS = a.GS + (size_t)e * 3 * m * bb;
    const double2* GSrow = a.GSrow + (size_t)e * m * bb;
    const double2* Z = (m == 1) ? GS + (size_t)m * bb : GSrow + (size_t)(m - 1) * bb;
    Acc<T, NW> acc;
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, opnd(CR0, BP, BP, BP), opnd(Z, b, b, b), -1.0);
    store<T, NW>(acc, G0L, BP, BP, BP);
    if (a.first_last) store<T, NW>(acc, a.first_last + (size_t)e * a.first_last_stride, b, b, b);
    __syncthreads();
    if (a.T)
      Tval = transmission<T, NW>(acc, G0L, a.sigL + (size_t)e * bb, a.sigR + (size_t)e * bb, b, GamL, GamR,
                                 X1, red);
  }
  if (inf != 0) {
    const double qnan = __builtin_nan("");
    double2* Gout = a.G + (size_t)e * 3 * a.l * bb;
    for (size_t idx = t; idx < (size_t)3 * a.l * bb; idx += NT) Gout[idx] = make_double2(qnan, qnan);
    Tval = qnan;
  }
  if (t == 0) {
    if (a.T) a.T[e] = Tval;
    a.info[(size_t)e * (a.info_stride > 0 ? a.info_stride : 1) + a.info_offset] = inf;
  }
}

// Band of a reduced separator system (the band of M itself) to the form an inner
// DDRGF level reads: diagonal blocks as they are, off-diagonal blocks negated.
// (A template so that every block-size translation unit that launches it has it.)
template <int D = 0>
__global__ void reduced_to_inner_kernel(const double2* MS, double2* out, size_t n, size_t band_elems,
                                        size_t diag_lo, size_t diag_hi) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t r = idx % band_elems;
    const double2 x = MS[idx];
    out[idx] = (r >= diag_lo && r < diag_hi) ? x : make_double2(-x.x, -x.y);
  }
}

template <int T>
hipError_t launch_dd_T(const DDArgs& a, const DDArgs* inner, double2* inner_band, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  const int chains = a.ne * a.m;
  if (a.mixed)
    hipLaunchKernelGGL((ddrgf_interior_kernel<T, NW, 1>), dim3(chains), dim3(64 * NW), 0, s, a);
  else
    hipLaunchKernelGGL((ddrgf_interior_kernel<T, NW, 0>), dim3(chains), dim3(64 * NW), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  ktime_mark("ddrgf_interior_kernel", s);
  hipLaunchKernelGGL((ddrgf_schur_kernel<T, NW>), dim3(chains), dim3(64 * NW), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("ddrgf_schur_kernel", s);
  if (inner) {
    // multi-level: the reduced system by DDRGF again (its status, band and block
    // (first separator, last separator) land where the sweep would put them)
    const size_t bb = (size_t)a.b * a.b, band = (size_t)3 * a.m * bb;
    hipLaunchKernelGGL(reduced_to_inner_kernel<0>, dim3(1024), dim3(256), 0, s, a.MS, inner_band, band * a.ne, band,
                       (size_t)a.m * bb, (size_t)2 * a.m * bb);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = launch_dd_T<T>(*inner, nullptr, nullptr, s)) != hipSuccess) return err;
  } else {
  SweepArgs r{};
  r.H = a.MS;
  r.h_stride = (size_t)3 * a.m * a.b * a.b;
  r.direct = 1;
  r.G = a.GS;
  r.g_stride = (size_t)3 * a.m * a.b * a.b;
  r.first_row = a.GSrow;
  r.T = nullptr;
  r.info = a.info_part;   // strided below: reduced status goes to slot m of each energy
  r.ws = a.ws_red;
  r.ws_chain = a.ws_red_chain;
  r.l = a.m;
  r.b = a.b;
  r.chains = a.ne;
  r.info_stride = a.m + 1;
  r.info_offset = a.m;
  r.mixed = a.mixed;
  r.kappa_max = a.kappa_max;
  if ((err = launch_rgf_sweep(r, s)) != hipSuccess) return err;
  }
  if (a.mixed)
    hipLaunchKernelGGL((ddrgf_recover_kernel<T, NW, 1>), dim3(chains), dim3(64 * NW), 0, s, a);
  else
    hipLaunchKernelGGL((ddrgf_recover_kernel<T, NW, 0>), dim3(chains), dim3(64 * NW), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("ddrgf_recover_kernel", s);
  hipLaunchKernelGGL((ddrgf_finalize_kernel<T, NW>), dim3(a.ne), dim3(64 * NW), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("ddrgf_finalize_kernel", s);
  return hipSuccess;
}

#ifdef RGFK_INST_T
template hipError_t launch_dd_T<RGFK_INST_T>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                             hipStream_t s);
#else
extern template hipError_t launch_dd_T<1>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);
extern template hipError_t launch_dd_T<2>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);
extern template hipError_t launch_dd_T<3>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);
extern template hipError_t launch_dd_T<4>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);
extern template hipError_t launch_dd_T<5>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);
extern template hipError_t launch_dd_T<6>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);
extern template hipError_t launch_dd_T<7>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);
extern template hipError_t launch_dd_T<8>(const DDArgs& a, const DDArgs* inner, double2* inner_band,
                                                   hipStream_t s);

hipError_t launch_ddrgf(const DDArgs& a, const DDArgs* inner, double2* inner_band, hipStream_t s) {
  if (a.herm && !a.direct) {
    hipLaunchKernelGGL(herm_flag_init_kernel, dim3(1), dim3(64), 0, s, a.herm);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(herm_check_kernel, dim3(1024), dim3(256), 0, s, a.H, a.l, a.b, a.herm);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    ktime_mark("herm_check_kernel", s);
  }
  switch (padded_block(a.b) / 16) {
    case 1: return launch_dd_T<1>(a, inner, inner_band, s);
    case 2: return launch_dd_T<2>(a, inner, inner_band, s);
    case 3: return launch_dd_T<3>(a, inner, inner_band, s);
    case 4: return launch_dd_T<4>(a, inner, inner_band, s);
    case 5: return launch_dd_T<5>(a, inner, inner_band, s);
    case 6: return launch_dd_T<6>(a, inner, inner_band, s);
    case 7: return launch_dd_T<7>(a, inner, inner_band, s);
    case 8: return launch_dd_T<8>(a, inner, inner_band, s);
    default: return hipErrorInvalidValue;
  }
}

void ddrgf_layout_host(int l, int m, int* base, int* rem) {
  DDLayout d = dd_layout(l, m);
  *base = d.base;
  *rem = d.rem;
}
#endif  // RGFK_INST_T

}  // namespace rgfk
