// DDRGF for block n-diagonal systems (half bandwidth w >= 2) on gfx950: Algorithm 2
// of Sec. 3 with separators of w layers and the n-diagonal RGF of Sec. 2.3
// (Proposition 3) inside the closed interiors.
//
// Layout (the figure of Sec. 3 with separators of w layers): m pairs (interior D2^k,
// separator D1^k); interior k is layers [a_k, a_k + n_k - 1], separator k is layers
// [p_k, p_k + w - 1] with p_k = a_k + n_k; the chain starts with an interior and ends
// with a separator; the l - m w interior layers are split as evenly as possible, the
// first (l - m w) mod m interiors one layer longer; every n_k >= w.
//
// Local indices below run over an interior (0 .. n-1, layer a + i); pL = a - w and
// pR = a + n are the first layers of the left and right separators.
//
//   1. nddrgf_interior_kernel  one workgroup per (energy, interior): the n-diagonal
//      RGF of the closed interior writes the band of X = (M_{D2^k})^{-1} into G and
//      forms the halo products with the neighbouring separators, w blocks per layer:
//        CL_i[s] = sum_t X_{i,t} M_{a+t, pL+s},        RL_j[s] = sum_t M_{pL+s, a+t} X_{t,j}
//        CR_i[s] = sum_t X_{i,n-w+t} M_{a+n-w+t, pR+s}, RR_j[s] = sum_t M_{pR+s, a+n-w+t} X_{n-w+t,j}
//      CL, RL: direct sums over the band for the first w layers, then the downward
//      recursions of the sweep, CL_i = -sum_c L_{i,c} CL_c and RL_j = -sum_c RL_c U_{c,j}.
//      CR, RR: with s_i = (X_{a',i-w+1}, ..., X_{a',i}) the last w entries of row a' up to
//      column i, the recursion X_{a',i} = -sum_c X_{a',c} U_{c,i} (i > a') reads
//      s_i = s_{i-1} T_i, so CR_i = s_i P_i with P_{n-1} = M[last w of D2, right
//      separator] and P_{i-1}[t] = P_i[t-1] - U_{i-w+t,i} P_i[w-1] (P_i[-1] = 0), formed
//      in the upward pass; the rows mirror it: RR_j = Q_j sigma_j with
//      Q_{i-1}[.][t] = Q_i[.][t-1] - Q_i[.][w-1] L_{i,i-w+t}.
//      Hermitian interiors (H exactly Hermitian, checked on the device, eta_d = 0, no
//      lead in the interior): the transfer products of the rows are those of the
//      columns conjugated, Q_i = P_i^H, and are not formed.  The other Hermitian
//      identities (U_{c,i} = L_{i,c}^H, a Schur window updated in its lower triangle
//      only, the upper band or the row halos as conjugate transposes) are exact too,
//      but for w >= 2 they tie rounding errors of the two triangles together: on
//      interiors of tens of layers the lower-triangle Schur update alone diverges
//      (relative band error 1e-2 .. 1e-1 at 100 layers of 4 orbitals), and U = L^H or
//      conjugated halos cost one to two digits, so they are not used.
//   2. nddrgf_schur_kernel  one workgroup per (energy, separator): the reduced system
//      T_S = T_11 - T_12 T_22^{-1} T_21 (eq. Schur complement in DDRGF, Proposition 4)
//      on the m w separator layers, as a band of b x b blocks of half bandwidth 2w - 1:
//      the separator diagonal blocks, and the couplings between neighbouring
//      separators through one interior (the "orange" blocks).
//   3. the n-diagonal sweep in direct mode on the reduced system (several workgroups
//      per energy when they fit): band of G_S and its first w block rows at the last
//      column.
//   4. nddrgf_recover_kernel  one workgroup per (energy, interior): Algorithm 2 step 4,
//        G_{D2,D2} = X + X T_21 G_S T_12 X,  G_{D2,D1} = -X T_21 G_S,  G_{D1,D2} = -G_S T_12 X,
//      inside the band, added in place; step 5 (inverse reordering) is the index map.
//   5. nddrgf_finalize_kernel  one workgroup per energy: T(E) from
//      G_{0,l-1} = -sum_s CR^(0)_0[s] G_S(s, m w - 1), status and NaN fill.
#include "block_engine.h"
#include "kernels.h"

namespace rgfk {

struct NDLayout {
  int base, rem, w;
  __host__ __device__ int n(int k) const { return base + (k < rem ? 1 : 0); }
  __host__ __device__ int a(int k) const { return k * (base + w) + (k < rem ? k : rem); }
  __host__ __device__ int p(int k) const { return a(k) + n(k); }
};

__host__ __device__ inline NDLayout nd_layout(int l, int m, int w) {
  NDLayout d;
  d.base = (l - m * w) / m;
  d.rem = (l - m * w) % m;
  d.w = w;
  return d;
}

// Per (energy, interior) workspace, in bp x bp blocks, nmax = longest interior:
// S band (2w+1) nmax, g nmax, U w nmax, L w nmax, P w^2 nmax, Q w^2 nmax, CL, CR, RL,
// RR w nmax each, V 2w (recovery).
struct NDWs {
  double2 *S, *g, *U, *L, *P, *Q, *CL, *CR, *RL, *RR, *V;
};

__device__ __forceinline__ NDWs nd_ws(double2* base, int nmax, int w, size_t bpbp) {
  NDWs r;
  const size_t nb = (size_t)nmax * bpbp;
  r.S = base;
  r.g = r.S + (size_t)(2 * w + 1) * nb;
  r.U = r.g + nb;
  r.L = r.U + (size_t)w * nb;
  r.P = r.L + (size_t)w * nb;
  r.Q = r.P + (size_t)w * w * nb;
  r.CL = r.Q + (size_t)w * w * nb;
  r.CR = r.CL + (size_t)w * nb;
  r.RL = r.CR + (size_t)w * nb;
  r.RR = r.RL + (size_t)w * nb;
  r.V = r.RR + (size_t)w * nb;
  return r;
}

#if defined(RGFK_ND_T0)

// Clears *flag unless the band of H is exactly Hermitian: H_ij = H_ji^H entry by entry
// for |i - j| <= w (NaN entries count as a mismatch).  Templates, so that every
// instantiation unit that launches them has them.
template <int D>
__global__ void nd_herm_init_kernel(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 1;
}

template <int D>
__global__ void nd_herm_check_kernel(const double2* H, int l, int b, int w, int* flag) {
  const size_t bb = (size_t)b * b;
  const size_t total = (size_t)(2 * w + 1) * l * bb;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % b), row = (int)((idx / b) % b);
    const int i = (int)((idx / bb) % l);
    const int d = (int)(idx / (bb * l));       // block (i, i + d - w)
    const int j = i + d - w;
    if (j < 0 || j >= l) continue;
    const double2 x = H[idx];
    const double2 y = H[((size_t)(2 * w - d) * l + j) * bb + (size_t)col * b + row];   // block (j, i), transposed
    if (!(x.x == y.x && x.y == -y.y)) *flag = 0;
  }
}

// ---------------------------------------------------------------------------
// 1. interiors
// ---------------------------------------------------------------------------
template <int T, int NW, bool HERM>
__device__ __forceinline__ void nd_interior(const NDDArgs& a, GJShared& sh) {
  constexpr int BP = 16 * T;
  const int c = blockIdx.x;
  const int e = c / a.m, k = c % a.m;
  const int w = a.w, b = a.b, l = a.l;
  const NDLayout lay = nd_layout(l, a.m, w);
  const int n = lay.n(k), a0 = lay.a(k), pR = a0 + n, pL = a0 - w;
  const bool left = k > 0;
  const int nmax = lay.base + 1;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const NDWs W = nd_ws(a.ws_int + (size_t)c * a.ws_int_chain, nmax, w, bpbp);
  const double2 z = make_double2(a.E[e], a.eta_d);
  const double2* sL = a.sigL + (size_t)e * bb;
  const double2* sR = a.sigR + (size_t)e * bb;
  double2* Gout = a.G + (size_t)e * (2 * w + 1) * l * bb;
  auto Hb = [&](int i, int j) { return a.H + ((size_t)(w + j - i) * l + i) * bb; };     // global
  auto Gb = [&](int i, int j) { return Gout + ((size_t)(w + j - i) * l + i) * bb; };    // local
  auto Sb = [&](int i, int j) { return W.S + ((size_t)(w + j - i) * nmax + i) * bpbp; };
  auto gb = [&](int i) { return W.g + (size_t)i * bpbp; };
  auto Ub = [&](int cc, int i) { return W.U + ((size_t)i * w + (i - cc - 1)) * bpbp; };
  auto Lb = [&](int i, int cc) { return W.L + ((size_t)i * w + (i - cc - 1)) * bpbp; };
  auto Pk = [&](int i, int t, int s) { return W.P + (((size_t)i * w + t) * w + s) * bpbp; };
  auto Qk = [&](int i, int s, int t) { return W.Q + (((size_t)i * w + s) * w + t) * bpbp; };
  auto Hx = [&](double2* base, int i, int s) { return base + ((size_t)i * w + s) * bpbp; };
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pb = [&](const double2* p) { return opnd(p, b, b, b); };
  auto X = [&](int i, int j) { return Pb(Gb(a0 + i, a0 + j)); };
  // Q_i[s][t] (stored, or P_i[t][s]^H on the Hermitian path)
  auto Qop = [&](int i, int s, int t) { return HERM ? opnd(Pk(i, t, s), BP, BP, BP, 1) : P(Qk(i, s, t)); };
  Acc<T, NW> acc;
  int bad_layer = -1;

  // ---------------- S = band of M on the closed interior ----------------
  for (int i = 0; i < n; ++i) {
    const int j0 = i - w < 0 ? 0 : i - w, j1 = i + w > n - 1 ? n - 1 : i + w;
    for (int j = j0; j <= j1; ++j) {
      const int gi = a0 + i;
      if (i == j)
        assemble_diag<T, NW>(acc, Hb(gi, gi), b, z, gi == 0 ? sL : nullptr, gi == l - 1 ? sR : nullptr);
      else
        load<T, NW>(acc, Pb(Hb(gi, a0 + j)), -1.0);
      store<T, NW>(acc, Sb(i, j), BP, BP, BP);
    }
  }
  // P_{n-1}[t][s] = M_{a+n-w+t, pR+s},  Q_{n-1}[s][t] = M_{pR+s, a+n-w+t}: nonzero for s <= t
  for (int t = 0; t < w; ++t)
    for (int s = 0; s < w; ++s) {
      const int gi = a0 + n - w + t, gq = pR + s;
      if (s <= t) load<T, NW>(acc, Pb(Hb(gi, gq)), -1.0); else acc_zero<T, NW>(acc);
      store<T, NW>(acc, Pk(n - 1, t, s), BP, BP, BP);
      if (HERM) continue;
      if (s <= t) load<T, NW>(acc, Pb(Hb(gq, gi)), -1.0); else acc_zero<T, NW>(acc);
      store<T, NW>(acc, Qk(n - 1, s, t), BP, BP, BP);
    }
  __syncthreads();

  // ---------------- upward pass ----------------
  for (int i = n - 1; i >= 0; --i) {
    load<T, NW>(acc, P(Sb(i, i)));
    gj_invert<T, NW>(acc, gb(i), sh);
    if (sh.bad && bad_layer < 0) bad_layer = a0 + i;
    __syncthreads();
    const int c0 = i - w < 0 ? 0 : i - w;
    for (int cc = c0; cc < i; ++cc) {
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(gb(i)), P(Sb(i, cc)), 1.0);
      store<T, NW>(acc, Lb(i, cc), BP, BP, BP);
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(Sb(cc, i)), P(gb(i)), 1.0);
      store<T, NW>(acc, Ub(cc, i), BP, BP, BP);
    }
    __syncthreads();
    for (int ra = c0; ra < i; ++ra)
      for (int cc = c0; cc < i; ++cc) {
        load<T, NW>(acc, P(Sb(ra, cc)));
        mma<T, NW>(acc, P(Sb(ra, i)), P(Lb(i, cc)), -1.0);
        store<T, NW>(acc, Sb(ra, cc), BP, BP, BP);
      }
    if (i >= 1) {
      // transfer matrices of the last-column and last-row halos to layer i-1
      for (int t = 0; t < w; ++t) {
        const int cc = i - w + t;
        for (int s = 0; s < w; ++s) {
          if (t >= 1) load<T, NW>(acc, P(Pk(i, t - 1, s))); else acc_zero<T, NW>(acc);
          if (cc >= 0) mma<T, NW>(acc, P(Ub(cc, i)), P(Pk(i, w - 1, s)), -1.0);
          store<T, NW>(acc, Pk(i - 1, t, s), BP, BP, BP);
          if (HERM) continue;
          if (t >= 1) load<T, NW>(acc, P(Qk(i, s, t - 1))); else acc_zero<T, NW>(acc);
          if (cc >= 0) mma<T, NW>(acc, P(Qk(i, s, w - 1)), P(Lb(i, cc)), -1.0);
          store<T, NW>(acc, Qk(i - 1, s, t), BP, BP, BP);
        }
      }
    }
    __syncthreads();
  }

  // ---------------- downward pass: band of X and the halos ----------------
  // CR_i = s_i P_i and RR_i = Q_i sigma_i from row / column i of the band
  auto halos_right = [&](int i) {
    for (int s = 0; s < w; ++s) {
      acc_zero<T, NW>(acc);
      for (int t = 0; t < w; ++t) {
        const int cc = i - w + 1 + t;
        if (cc >= 0) mma<T, NW>(acc, X(i, cc), P(Pk(i, t, s)), 1.0);
      }
      store<T, NW>(acc, Hx(W.CR, i, s), BP, BP, BP);
      acc_zero<T, NW>(acc);
      for (int t = 0; t < w; ++t) {
        const int cc = i - w + 1 + t;
        if (cc >= 0) mma<T, NW>(acc, Qop(i, s, t), X(cc, i), 1.0);
      }
      store<T, NW>(acc, Hx(W.RR, i, s), BP, BP, BP);
    }
  };
  // CL_r, RL_r for r < w straight from the band (M_{a+t, pL+s} nonzero for t <= s)
  auto halos_left_first = [&]() {
    for (int r = 0; r < w && r < n; ++r)
      for (int s = 0; s < w; ++s) {
        acc_zero<T, NW>(acc);
        for (int t = 0; t <= s && t < n; ++t) mma<T, NW>(acc, X(r, t), Pb(Hb(a0 + t, pL + s)), -1.0);
        store<T, NW>(acc, Hx(W.CL, r, s), BP, BP, BP);
        acc_zero<T, NW>(acc);
        for (int t = 0; t <= s && t < n; ++t) mma<T, NW>(acc, Pb(Hb(pL + s, a0 + t)), X(t, r), -1.0);
        store<T, NW>(acc, Hx(W.RL, r, s), BP, BP, BP);
      }
  };

  load<T, NW>(acc, P(gb(0)));
  store<T, NW>(acc, Gb(a0, a0), b, b, b);
  __syncthreads();
  halos_right(0);
  if (left && w == 1) halos_left_first();
  __syncthreads();
  for (int i = 1; i < n; ++i) {
    const int c0 = i - w < 0 ? 0 : i - w;
    for (int ra = c0; ra < i; ++ra) {
      acc_zero<T, NW>(acc);
      for (int cc = c0; cc < i; ++cc) mma<T, NW>(acc, X(ra, cc), P(Ub(cc, i)), -1.0);
      store<T, NW>(acc, Gb(a0 + ra, a0 + i), b, b, b);
      acc_zero<T, NW>(acc);
      for (int cc = c0; cc < i; ++cc) mma<T, NW>(acc, P(Lb(i, cc)), X(cc, ra), -1.0);
      store<T, NW>(acc, Gb(a0 + i, a0 + ra), b, b, b);
    }
    __syncthreads();
    load<T, NW>(acc, P(gb(i)));
    for (int cc = c0; cc < i; ++cc) mma<T, NW>(acc, P(Lb(i, cc)), X(cc, i), -1.0);
    store<T, NW>(acc, Gb(a0 + i, a0 + i), b, b, b);
    __syncthreads();
    halos_right(i);
    if (left && i >= w) {
      for (int s = 0; s < w; ++s) {
        acc_zero<T, NW>(acc);
        for (int cc = i - w; cc < i; ++cc) mma<T, NW>(acc, P(Lb(i, cc)), P(Hx(W.CL, cc, s)), -1.0);
        store<T, NW>(acc, Hx(W.CL, i, s), BP, BP, BP);
        acc_zero<T, NW>(acc);
        for (int cc = i - w; cc < i; ++cc) mma<T, NW>(acc, P(Hx(W.RL, cc, s)), P(Ub(cc, i)), -1.0);
        store<T, NW>(acc, Hx(W.RL, i, s), BP, BP, BP);
      }
    }
    if (left && i == w - 1) halos_left_first();
    __syncthreads();
  }
  if (threadIdx.x == 0) a.info_part[(size_t)e * a.m + k] = bad_layer >= 0 ? bad_layer + 1 : 0;
}

// Whether interior k takes the Hermitian path: H found exactly Hermitian on the
// device, eta_d = 0, and no lead in the interior (k > 0).
__device__ __forceinline__ bool nd_herm_interior(const NDDArgs& a, int k) {
  return a.herm != nullptr && *a.herm != 0 && a.eta_d == 0.0 && k > 0;
}

template <int T, int NW>
__global__ __launch_bounds__(64 * NW, T == 4 ? 2 : 1) void nddrgf_interior_kernel(NDDArgs a) {
  __shared__ GJShared sh;
  if (nd_herm_interior(a, blockIdx.x % a.m))
    nd_interior<T, NW, true>(a, sh);
  else
    nd_interior<T, NW, false>(a, sh);
}

// ---------------------------------------------------------------------------
// 2. reduced system on the separator layers
// ---------------------------------------------------------------------------
template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void nddrgf_schur_kernel(NDDArgs a) {
  constexpr int BP = 16 * T;
  const int c = blockIdx.x;
  const int e = c / a.m, k = c % a.m;
  const int w = a.w, b = a.b, l = a.l, m = a.m;
  const int lr = m * w, wr = 2 * w - 1;
  const NDLayout lay = nd_layout(l, m, w);
  const int nmax = lay.base + 1;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const int p = lay.p(k), nk = lay.n(k);
  const double2 z = make_double2(a.E[e], a.eta_d);
  auto Hb = [&](int i, int j) { return a.H + ((size_t)(w + j - i) * l + i) * bb; };
  double2* MS = a.MS + (size_t)e * (2 * wr + 1) * lr * bb;
  auto halo = [&](int kk) { return nd_ws(a.ws_int + (size_t)(e * m + kk) * a.ws_int_chain, nmax, w, bpbp); };
  auto Hx = [&](double2* base, int i, int s) { return opnd(base + ((size_t)i * w + s) * bpbp, BP, BP, BP); };
  auto Pb = [&](const double2* q) { return opnd(q, b, b, b); };
  const NDWs Wk = halo(k);
  Acc<T, NW> acc;
  for (int s = 0; s < w; ++s) {
    const int r = k * w + s, gr = p + s;
    const int r0 = r - wr < 0 ? 0 : r - wr, r1 = r + wr > lr - 1 ? lr - 1 : r + wr;
    for (int r2 = r0; r2 <= r1; ++r2) {
      const int k2 = r2 / w, s2 = r2 % w;
      // -M_{sep, D} (X M_{D, sep'}) = H_{sep, D} (halo): every term enters with a plus sign
      if (k2 == k) {
        if (s2 == s)
          assemble_diag<T, NW>(acc, Hb(gr, gr), b, z, gr == 0 ? a.sigL + (size_t)e * bb : nullptr,
                               gr == l - 1 ? a.sigR + (size_t)e * bb : nullptr);
        else
          load<T, NW>(acc, Pb(Hb(gr, p + s2)), -1.0);
        for (int t = s; t < w; ++t) mma<T, NW>(acc, Pb(Hb(gr, p - w + t)), Hx(Wk.CR, nk - w + t, s2), 1.0);
        if (k + 1 < m) {
          const NDWs W1 = halo(k + 1);
          for (int t = 0; t <= s; ++t) mma<T, NW>(acc, Pb(Hb(gr, p + w + t)), Hx(W1.CL, t, s2), 1.0);
        }
      } else if (k2 == k + 1) {
        // orange coupling S_{k,k+1} through interior k+1
        const NDWs W1 = halo(k + 1);
        acc_zero<T, NW>(acc);
        for (int t = 0; t <= s; ++t) mma<T, NW>(acc, Pb(Hb(gr, p + w + t)), Hx(W1.CR, t, s2), 1.0);
      } else if (k2 == k - 1) {
        // orange coupling S_{k,k-1} through interior k
        acc_zero<T, NW>(acc);
        for (int t = s; t < w; ++t) mma<T, NW>(acc, Pb(Hb(gr, p - w + t)), Hx(Wk.CL, nk - w + t, s2), 1.0);
      } else {
        acc_zero<T, NW>(acc);
      }
      store<T, NW>(acc, MS + ((size_t)(wr + r2 - r) * lr + r) * bb, b, b, b);
    }
  }
}

// ---------------------------------------------------------------------------
// 4. recovery of the interior blocks and the separator couplings
// ---------------------------------------------------------------------------
template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void nddrgf_recover_kernel(NDDArgs a) {
  constexpr int BP = 16 * T;
  const int c = blockIdx.x;
  const int e = c / a.m, k = c % a.m;
  const int w = a.w, b = a.b, l = a.l, m = a.m;
  const int lr = m * w, wr = 2 * w - 1;
  const NDLayout lay = nd_layout(l, m, w);
  const int n = lay.n(k), a0 = lay.a(k);
  const int nmax = lay.base + 1;
  const bool left = k > 0;
  const int ng = left ? 2 : 1;             // separator groups next to the interior
  const int kg0 = left ? k - 1 : k;        // separator of group 0
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const NDWs W = nd_ws(a.ws_int + (size_t)c * a.ws_int_chain, nmax, w, bpbp);
  const double2* GS = a.GS + (size_t)e * (2 * wr + 1) * lr * bb;
  double2* Gout = a.G + (size_t)e * (2 * w + 1) * l * bb;
  auto Gb = [&](int i, int j) { return Gout + ((size_t)(w + j - i) * l + i) * bb; };
  auto Zb = [&](int g1, int s1, int g2, int s2) {
    const int r = (kg0 + g1) * w + s1, r2 = (kg0 + g2) * w + s2;
    return opnd(GS + ((size_t)(wr + r2 - r) * lr + r) * bb, b, b, b);
  };
  auto sepl = [&](int g, int s) { return lay.p(kg0 + g) + s; };   // global layer of separator row
  auto Ablk = [&](int i, int g, int s) {    // (X T_21)_{i, (g, s)}
    return opnd((left && g == 0 ? W.CL : W.CR) + ((size_t)i * w + s) * bpbp, BP, BP, BP);
  };
  auto Bblk = [&](int j, int g, int s) {    // (T_12 X)_{(g, s), j}
    return opnd((left && g == 0 ? W.RL : W.RR) + ((size_t)j * w + s) * bpbp, BP, BP, BP);
  };
  auto Vb = [&](int g, int s) { return W.V + ((size_t)g * w + s) * bpbp; };
  Acc<T, NW> acc;
  for (int i = 0; i < n; ++i) {
    const int gi = a0 + i;
    // V_i = (X T_21)_i G_S restricted to the neighbouring separators
    for (int g2 = 0; g2 < ng; ++g2)
      for (int s2 = 0; s2 < w; ++s2) {
        acc_zero<T, NW>(acc);
        for (int g1 = 0; g1 < ng; ++g1)
          for (int s1 = 0; s1 < w; ++s1) mma<T, NW>(acc, Ablk(i, g1, s1), Zb(g1, s1, g2, s2), 1.0);
        store<T, NW>(acc, Vb(g2, s2), BP, BP, BP);
        const int q = sepl(g2, s2);
        if (q - gi <= w && gi - q <= w) store<T, NW>(acc, Gb(gi, q), b, b, b, -1.0);   // G_{i,q} = -V
      }
    __syncthreads();
    // G_ij += V_i (T_12 X)_j inside the interior
    const int j0 = i - w < 0 ? 0 : i - w, j1 = i + w > n - 1 ? n - 1 : i + w;
    for (int j = j0; j <= j1; ++j) {
      double2* dst = Gb(gi, a0 + j);
      load<T, NW>(acc, opnd(dst, b, b, b));
      for (int g = 0; g < ng; ++g)
        for (int s = 0; s < w; ++s) mma<T, NW>(acc, opnd(Vb(g, s), BP, BP, BP), Bblk(j, g, s), 1.0);
      store<T, NW>(acc, dst, b, b, b);
    }
    __syncthreads();
  }
  // G_{q,j} = -(G_S T_12 X)_{q,j} for separator layers q inside the band of j
  for (int j = 0; j < n; ++j) {
    const int gj = a0 + j;
    for (int g1 = 0; g1 < ng; ++g1)
      for (int s1 = 0; s1 < w; ++s1) {
        const int q = sepl(g1, s1);
        if (q - gj > w || gj - q > w) continue;
        acc_zero<T, NW>(acc);
        for (int g2 = 0; g2 < ng; ++g2)
          for (int s2 = 0; s2 < w; ++s2) mma<T, NW>(acc, Zb(g1, s1, g2, s2), Bblk(j, g2, s2), -1.0);
        store<T, NW>(acc, Gb(q, gj), b, b, b);
      }
  }
  // the blocks of separator k itself
  const int gk = left ? 1 : 0;
  for (int s = 0; s < w; ++s)
    for (int s2 = 0; s2 < w; ++s2) {
      load<T, NW>(acc, Zb(gk, s, gk, s2));
      store<T, NW>(acc, Gb(sepl(gk, s), sepl(gk, s2)), b, b, b);
    }
}

// ---------------------------------------------------------------------------
// 5. per-energy transmission, status and NaN fill
// ---------------------------------------------------------------------------
template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void nddrgf_finalize_kernel(NDDArgs a) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  __shared__ double red[NW];
  __shared__ int s_info;
  const int e = blockIdx.x, t = threadIdx.x;
  const int w = a.w, b = a.b, l = a.l, m = a.m;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const NDLayout lay = nd_layout(l, m, w);
  const int nmax = lay.base + 1;
  if (t == 0) {
    // first failing pivot in elimination order: interiors, then the reduced system
    int inf = 0;
    for (int k = 0; k < m && inf == 0; ++k) inf = a.info_part[(size_t)e * m + k];
    const int ir = a.info_red[e];
    if (inf == 0 && (ir & RGF_INFO_SYNC_TIMEOUT)) {
      inf = RGF_INFO_SYNC_TIMEOUT;   // the split reduced sweep gave up waiting
    } else if (inf == 0 && ir != 0) {
      const int r = ir - 1;
      inf = lay.p(r / w) + r % w + 1;
    }
    s_info = inf;
  }
  __syncthreads();
  const int inf = s_info;
  double Tval = 0.0;
  if (a.T) {
    double2* scr = a.ws_fin + (size_t)e * 4 * bpbp;
    double2* G0L = scr;
    const NDWs W0 = nd_ws(a.ws_int + (size_t)(e * m) * a.ws_int_chain, nmax, w, bpbp);
    Acc<T, NW> acc;
    acc_zero<T, NW>(acc);
    for (int s = 0; s < w; ++s)
      mma<T, NW>(acc, opnd(W0.CR + (size_t)s * bpbp, BP, BP, BP),
                 opnd(a.GSlast + ((size_t)e * w + s) * bb, b, b, b), -1.0);
    store<T, NW>(acc, G0L, BP, BP, BP);
    __syncthreads();
    Tval = transmission<T, NW>(acc, G0L, a.sigL + (size_t)e * bb, a.sigR + (size_t)e * bb, b, scr + bpbp,
                               scr + 2 * bpbp, scr + 3 * bpbp, red);
  }
  if (inf != 0) {
    const double qnan = __builtin_nan("");
    double2* Gout = a.G + (size_t)e * (2 * w + 1) * l * bb;
    for (size_t idx = t; idx < (size_t)(2 * w + 1) * l * bb; idx += NT) Gout[idx] = make_double2(qnan, qnan);
    Tval = qnan;
  }
  if (t == 0) {
    if (a.T) a.T[e] = Tval;
    a.info[e] = inf;
  }
}

template <int T>
hipError_t launch_nd_T(const NDDArgs& a, const NSweepArgs& red, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  const int chains = a.ne * a.m;
  if (a.herm) {
    hipLaunchKernelGGL(nd_herm_init_kernel<0>, dim3(1), dim3(64), 0, s, a.herm);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(nd_herm_check_kernel<0>, dim3(1024), dim3(256), 0, s, a.H, a.l, a.b, a.w, a.herm);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    ktime_mark("nd_herm_check_kernel", s);
  }
  hipLaunchKernelGGL((nddrgf_interior_kernel<T, NW>), dim3(chains), dim3(64 * NW), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  ktime_mark("nddrgf_interior_kernel", s);
  hipLaunchKernelGGL((nddrgf_schur_kernel<T, NW>), dim3(chains), dim3(64 * NW), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("nddrgf_schur_kernel", s);
  // the reduced system with several workgroups per energy when they fit co-resident
  // (sync counters given: not under stream capture)
  const int K = red.sync ? split_workgroups_n(red.b, red.ne, 0) : 1;
  if ((err = K > 1 ? launch_nrgf_split(red, K, s) : launch_nrgf_sweep(red, s)) != hipSuccess) return err;
  hipLaunchKernelGGL((nddrgf_recover_kernel<T, NW>), dim3(chains), dim3(64 * NW), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("nddrgf_recover_kernel", s);
  hipLaunchKernelGGL((nddrgf_finalize_kernel<T, NW>), dim3(a.ne), dim3(64 * NW), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("nddrgf_finalize_kernel", s);
  return hipSuccess;
}

#define RGFK_ND_INST(TT)                                                                       \
  template hipError_t launch_nd_T<TT>(const NDDArgs& a, const NSweepArgs& red, hipStream_t s);
#if RGFK_ND_T0 <= 1 && 1 <= RGFK_ND_T1
RGFK_ND_INST(1)
#endif
#if RGFK_ND_T0 <= 2 && 2 <= RGFK_ND_T1
RGFK_ND_INST(2)
#endif
#if RGFK_ND_T0 <= 3 && 3 <= RGFK_ND_T1
RGFK_ND_INST(3)
#endif
#if RGFK_ND_T0 <= 4 && 4 <= RGFK_ND_T1
RGFK_ND_INST(4)
#endif
#if RGFK_ND_T0 <= 5 && 5 <= RGFK_ND_T1
RGFK_ND_INST(5)
#endif
#if RGFK_ND_T0 <= 6 && 6 <= RGFK_ND_T1
RGFK_ND_INST(6)
#endif
#if RGFK_ND_T0 <= 7 && 7 <= RGFK_ND_T1
RGFK_ND_INST(7)
#endif
#if RGFK_ND_T0 <= 8 && 8 <= RGFK_ND_T1
RGFK_ND_INST(8)
#endif

#else  // dispatch unit

template <int T>
hipError_t launch_nd_T(const NDDArgs& a, const NSweepArgs& red, hipStream_t s);

size_t nddrgf_interior_ws_elems(int nmax, int w, int bp) {
  return ((size_t)(2 * w * w + 8 * w + 2) * nmax + 2 * w) * (size_t)bp * bp;
}

void nddrgf_layout_host(int l, int m, int w, int* base, int* rem) {
  const NDLayout d = nd_layout(l, m, w);
  *base = d.base;
  *rem = d.rem;
}

hipError_t launch_nddrgf(const NDDArgs& a, const NSweepArgs& red, hipStream_t s) {
  switch (padded_block(a.b) / 16) {
    case 1: return launch_nd_T<1>(a, red, s);
    case 2: return launch_nd_T<2>(a, red, s);
    case 3: return launch_nd_T<3>(a, red, s);
    case 4: return launch_nd_T<4>(a, red, s);
    case 5: return launch_nd_T<5>(a, red, s);
    case 6: return launch_nd_T<6>(a, red, s);
    case 7: return launch_nd_T<7>(a, red, s);
    case 8: return launch_nd_T<8>(a, red, s);
    default: return hipErrorInvalidValue;
  }
}

#endif  // RGFK_ND_T0

}  // namespace rgfk
