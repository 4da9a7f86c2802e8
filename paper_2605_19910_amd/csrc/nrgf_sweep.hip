// Native RGF for block n-diagonal systems (paper Sec. 2.3), n = 2w + 1, on gfx950.
//
// One workgroup per energy.  A working copy S of the band of M(E) lives in the
// workspace (assembled in a prologue); the upward pass eliminates layers l-1 .. 0:
//   g_i = S_ii^{-1};  L_{i,c} = g_i S_{i,c},  U_{c,i} = S_{c,i} g_i   (c in C_i = [i-w, i-1]);
//   S_{a,c} -= S_{a,i} L_{i,c}                                       (a, c in C_i)
// which keeps the band (Proposition 3).  The downward pass uses that G U~ is block
// lower and L~ G block upper triangular (M = U~ D L~):
//   G_{a,i} = -sum_{c in C_i} G_{a,c} U_{c,i},  G_{i,a} = -sum_{c in C_i} L_{i,c} G_{c,a}  (a in C_i)
//   G_ii = g_i - sum_{c in C_i} L_{i,c} G_{c,i}
// and the first block row R_i = G_{0,i} = -sum_{c in C_i} R_c U_{c,i} feeds T(E).
// In direct mode (the reduced separator system of the n-diagonal DDRGF) the band of M
// is given per energy, and the first nr block rows are carried to the last column:
// G_{t,i} = -sum_c G_{t,c} U_{c,i} for i > t, with G_{t,c} from the band when c <= t.
#include "block_engine.h"
#include "kernels.h"

namespace rgfk {

#ifndef RGFK_INST_T
size_t nrgf_ws_chain_elems(int l, int w, int bp, int nr) {
  // S band (2w+1) l, g l, U w l, L w l, R l, Gamma_L, Gamma_R, X1, rows 1..nr-1 (l each)
  return ((size_t)(4 * w + 3) * l + 3 + (size_t)(nr - 1) * l) * (size_t)bp * bp;
}
#endif

template <int T, int NW>
__global__ __launch_bounds__(64 * NW, 1) void nrgf_sweep_kernel(NSweepArgs a) {
  constexpr int BP = 16 * T;
  __shared__ GJShared sh;
  __shared__ double red[NW];
  const int e = blockIdx.x, t = threadIdx.x;
  const int l = a.l, b = a.b, w = a.w;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  double2* ws = a.ws + (size_t)e * a.ws_chain;
  double2* Sw = ws;                                  // (2w+1) l blocks: S(i, i+k) at (w+k) l + i
  double2* g = Sw + (size_t)(2 * w + 1) * l * bpbp;  // l
  double2* U = g + (size_t)l * bpbp;                 // w l: U_{c,i} at i w + (i - c - 1)
  double2* L = U + (size_t)w * l * bpbp;             // w l: L_{i,c} at i w + (i - c - 1)
  double2* R = L + (size_t)w * l * bpbp;             // l: G_{0,i}
  double2* GamL = R + (size_t)l * bpbp;
  double2* GamR = GamL + bpbp;
  double2* X1 = GamR + bpbp;
  double2* Rx = X1 + bpbp;                           // rows t >= 1: G_{t,i} at (t-1) l + i
  const double2* sL = a.direct ? nullptr : a.sigL + (size_t)e * bb;
  const double2* sR = a.direct ? nullptr : a.sigR + (size_t)e * bb;
  const double2* Hband = a.H + (a.direct ? (size_t)e * a.h_stride : 0);
  const double2 z = make_double2(a.E[e], a.eta_d);
  double2* Gout = a.G + (size_t)e * (2 * w + 1) * l * bb;

  auto Sblk = [&](int i, int j) { return Sw + ((size_t)(w + j - i) * l + i) * bpbp; };
  auto Hblk = [&](int i, int j) { return Hband + ((size_t)(w + j - i) * l + i) * bb; };
  auto Gblk = [&](int i, int j) { return Gout + ((size_t)(w + j - i) * l + i) * bb; };
  auto Ublk = [&](int c, int i) { return U + ((size_t)i * w + (i - c - 1)) * bpbp; };
  auto Lblk = [&](int i, int c) { return L + ((size_t)i * w + (i - c - 1)) * bpbp; };
  auto Rrow = [&](int tr, int i) { return Rx + ((size_t)(tr - 1) * l + i) * bpbp; };
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pb = [&](const double2* p) { return opnd(p, b, b, b); };

  int bad_layer = -1;
  Acc<T, NW> acc;

  // ---------------- prologue: S = band of M(E) ----------------
  for (int i = 0; i < l; ++i) {
    for (int k = -w; k <= w; ++k) {
      const int j = i + k;
      if (j < 0 || j >= l) continue;
      if (a.direct) {
        load<T, NW>(acc, Pb(Hblk(i, j)));
        if (k == 0) add_identity_beyond<T, NW>(acc, b);
      } else if (k == 0) {
        assemble_diag<T, NW>(acc, Hblk(i, i), b, z, i == 0 ? sL : nullptr, i == l - 1 ? sR : nullptr);
      } else {
        load<T, NW>(acc, Pb(Hblk(i, j)), -1.0);
      }
      store<T, NW>(acc, Sblk(i, j), BP, BP, BP);
    }
  }
  __syncthreads();

  // ---------------- upward pass ----------------
  for (int i = l - 1; i >= 0; --i) {
    load<T, NW>(acc, P(Sblk(i, i)));
    gj_invert<T, NW>(acc, g + (size_t)i * bpbp, sh);
    if (sh.bad && bad_layer < 0) bad_layer = i;
    __syncthreads();
    const int c0 = i - w < 0 ? 0 : i - w;
    for (int c = c0; c < i; ++c) {
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(g + (size_t)i * bpbp), P(Sblk(i, c)), 1.0);
      store<T, NW>(acc, Lblk(i, c), BP, BP, BP);
      acc_zero<T, NW>(acc);
      mma<T, NW>(acc, P(Sblk(c, i)), P(g + (size_t)i * bpbp), 1.0);
      store<T, NW>(acc, Ublk(c, i), BP, BP, BP);
    }
    __syncthreads();
    for (int ra = c0; ra < i; ++ra)
      for (int c = c0; c < i; ++c) {
        load<T, NW>(acc, P(Sblk(ra, c)));
        mma<T, NW>(acc, P(Sblk(ra, i)), P(Lblk(i, c)), -1.0);
        store<T, NW>(acc, Sblk(ra, c), BP, BP, BP);
      }
    __syncthreads();
  }

  // ---------------- downward pass ----------------
  load<T, NW>(acc, P(g));
  store<T, NW>(acc, Gblk(0, 0), b, b, b);
  store<T, NW>(acc, R, BP, BP, BP);
  __syncthreads();
  for (int i = 1; i < l; ++i) {
    const int c0 = i - w < 0 ? 0 : i - w;
    for (int ra = c0; ra < i; ++ra) {
      acc_zero<T, NW>(acc);
      for (int c = c0; c < i; ++c) mma<T, NW>(acc, Pb(Gblk(ra, c)), P(Ublk(c, i)), -1.0);
      store<T, NW>(acc, Gblk(ra, i), b, b, b);
      acc_zero<T, NW>(acc);
      for (int c = c0; c < i; ++c) mma<T, NW>(acc, P(Lblk(i, c)), Pb(Gblk(c, ra)), -1.0);
      store<T, NW>(acc, Gblk(i, ra), b, b, b);
    }
    acc_zero<T, NW>(acc);
    for (int c = c0; c < i; ++c) mma<T, NW>(acc, P(R + (size_t)c * bpbp), P(Ublk(c, i)), -1.0);
    store<T, NW>(acc, R + (size_t)i * bpbp, BP, BP, BP);
    for (int tr = 1; tr < a.nr && tr < i; ++tr) {
      acc_zero<T, NW>(acc);
      for (int c = c0; c < i; ++c)
        mma<T, NW>(acc, c <= tr ? Pb(Gblk(tr, c)) : P(Rrow(tr, c)), P(Ublk(c, i)), -1.0);
      store<T, NW>(acc, Rrow(tr, i), BP, BP, BP);
    }
    __syncthreads();
    load<T, NW>(acc, P(g + (size_t)i * bpbp));
    for (int c = c0; c < i; ++c) mma<T, NW>(acc, P(Lblk(i, c)), Pb(Gblk(c, i)), -1.0);
    store<T, NW>(acc, Gblk(i, i), b, b, b);
    __syncthreads();
  }

  double Tval = 0.0;
  if (a.T) Tval = transmission<T, NW>(acc, R + (size_t)(l - 1) * bpbp, sL, sR, b, GamL, GamR, X1, red);
  if (a.rows_last) {
    // blocks (tr, l-1): from the band when tr = l-1, else from the propagated rows
    for (int tr = 0; tr < a.nr && tr < l; ++tr) {
      if (tr == l - 1)
        load<T, NW>(acc, Pb(Gblk(tr, l - 1)));
      else
        load<T, NW>(acc, P(tr == 0 ? R + (size_t)(l - 1) * bpbp : Rrow(tr, l - 1)));
      store<T, NW>(acc, a.rows_last + ((size_t)e * a.nr + tr) * bb, b, b, b);
    }
  }

  if (bad_layer >= 0) {
    const double qnan = __builtin_nan("");
    for (size_t idx = t; idx < (size_t)(2 * w + 1) * l * bb; idx += 64 * NW)
      Gout[idx] = make_double2(qnan, qnan);
    Tval = qnan;
  }
  if (t == 0) {
    if (a.T) a.T[e] = Tval;
    a.info[e] = bad_layer >= 0 ? bad_layer + 1 : 0;
  }
}

template <int T>
hipError_t launch_n_T(const NSweepArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  hipLaunchKernelGGL((nrgf_sweep_kernel<T, NW>), dim3(a.ne), dim3(64 * NW), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) ktime_mark("nrgf_sweep_kernel", s);
  return err;
}

#ifdef RGFK_INST_T
template hipError_t launch_n_T<RGFK_INST_T>(const NSweepArgs& a, hipStream_t s);
#else
extern template hipError_t launch_n_T<1>(const NSweepArgs& a, hipStream_t s);
extern template hipError_t launch_n_T<2>(const NSweepArgs& a, hipStream_t s);
extern template hipError_t launch_n_T<3>(const NSweepArgs& a, hipStream_t s);
extern template hipError_t launch_n_T<4>(const NSweepArgs& a, hipStream_t s);
extern template hipError_t launch_n_T<5>(const NSweepArgs& a, hipStream_t s);
extern template hipError_t launch_n_T<6>(const NSweepArgs& a, hipStream_t s);
extern template hipError_t launch_n_T<7>(const NSweepArgs& a, hipStream_t s);
extern template hipError_t launch_n_T<8>(const NSweepArgs& a, hipStream_t s);

hipError_t launch_nrgf_sweep(const NSweepArgs& a, hipStream_t s) {
  switch (padded_block(a.b) / 16) {
    case 1: return launch_n_T<1>(a, s);
    case 2: return launch_n_T<2>(a, s);
    case 3: return launch_n_T<3>(a, s);
    case 4: return launch_n_T<4>(a, s);
    case 5: return launch_n_T<5>(a, s);
    case 6: return launch_n_T<6>(a, s);
    case 7: return launch_n_T<7>(a, s);
    case 8: return launch_n_T<8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Super-block view of a block n-diagonal system: w consecutive layers of b
// orbitals become one layer of w*b orbitals and the band becomes tridiagonal.
// Used to run DDRGF with separators of w layers through the tridiagonal kernels;
// the wanted band of G is a sub-band of the super-block band.
// ---------------------------------------------------------------------------
__global__ void fuse_band_kernel(FuseArgs a) {
  // one thread per element of the super band [3][lf][B][B], B = w b
  const int w = a.w, b = a.b, B = w * b, lf = a.l / w;
  const size_t total = (size_t)3 * lf * B * B;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % B);
    const int row = (int)((idx / B) % B);
    const int I = (int)((idx / ((size_t)B * B)) % lf);
    const int kf = (int)(idx / ((size_t)B * B * lf)) - 1;        // -1, 0, +1
    const int i = I * w + row / b, j = (I + kf) * w + col / b;   // layer indices
    double2 v = make_double2(0.0, 0.0);
    const int k = j - i;
    if (I + kf >= 0 && I + kf < lf && k >= -w && k <= w)
      v = a.H[((size_t)(w + k) * a.l + i) * b * b + (size_t)(row % b) * b + (col % b)];
    a.Hf[idx] = v;
  }
}

__global__ void fuse_sigma_kernel(FuseArgs a) {
  // Sigma_L on the first sub-layer of super-layer 0, Sigma_R on the last sub-layer of the last
  const int w = a.w, b = a.b, B = w * b;
  const size_t total = (size_t)a.ne * B * B;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % B), row = (int)((idx / B) % B);
    const size_t e = idx / ((size_t)B * B);
    double2 vl = make_double2(0.0, 0.0), vr = make_double2(0.0, 0.0);
    if (row < b && col < b) vl = a.sigL[e * b * b + (size_t)row * b + col];
    const int r0 = (w - 1) * b;
    if (row >= r0 && col >= r0) vr = a.sigR[e * b * b + (size_t)(row - r0) * b + (col - r0)];
    a.sigLf[idx] = vl;
    a.sigRf[idx] = vr;
  }
}

__global__ void unfuse_band_kernel(FuseArgs a) {
  // G[e][w+k][i] (b x b) = sub-block of the super band Gf[e][1 + J - I][I]
  const int w = a.w, b = a.b, B = w * b, l = a.l, lf = l / w;
  const size_t per_e = (size_t)(2 * w + 1) * l * b * b;
  const size_t total = per_e * a.ne;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t e = idx / per_e;
    size_t r = idx % per_e;
    const int col = (int)(r % b), row = (int)((r / b) % b);
    const int i = (int)((r / ((size_t)b * b)) % l);
    const int k = (int)(r / ((size_t)b * b * l)) - w;
    const int j = i + k;
    if (j < 0 || j >= l) continue;   // outside the matrix: never written
    const int I = i / w, J = j / w;
    const size_t src = e * (size_t)3 * lf * B * B + ((size_t)(1 + J - I) * lf + I) * B * B +
                       (size_t)((i % w) * b + row) * B + (size_t)((j % w) * b + col);
    a.G[idx] = a.Gf[src];
  }
}

hipError_t launch_fuse(const FuseArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(fuse_band_kernel, dim3(2048), dim3(256), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  ktime_mark("fuse_band_kernel", s);
  hipLaunchKernelGGL(fuse_sigma_kernel, dim3(1024), dim3(256), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("fuse_sigma_kernel", s);
  return hipSuccess;
}

__global__ void unfuse_info_kernel(FuseArgs a) {
  // a failing super-layer J is reported as its first layer w J
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < a.ne) {
    const int v = a.info_f[e];
    a.info[e] = v == 0 ? 0 : a.w * (v - 1) + 1;
  }
}

hipError_t launch_unfuse(const FuseArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(unfuse_band_kernel, dim3(4096), dim3(256), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  ktime_mark("unfuse_band_kernel", s);
  hipLaunchKernelGGL(unfuse_info_kernel, dim3((a.ne + 255) / 256), dim3(256), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  ktime_mark("unfuse_info_kernel", s);
  return hipSuccess;
}
#endif  // RGFK_INST_T

}  // namespace rgfk
