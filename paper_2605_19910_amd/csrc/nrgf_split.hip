// Native n-diagonal sweep (Sec. 2.3) with K workgroups per energy, for grids with
// fewer energies than the device holds workgroups.
//
// As in the block tridiagonal split sweep (rgf_split.hip): workgroup k owns the row
// slab [k bp/K, (k+1) bp/K) of every block product, workgroup 0 also inverts the
// Schur pivots, and group barriers separate the steps that read a whole block
// another workgroup wrote.  Per layer of the upward pass: inverse | barrier |
// L_{i,c}, U_{c,i} slabs | barrier | window update S_{a,c} -= S_{a,i} L_{i,c} (each
// workgroup its own rows) | barrier; per layer of the downward pass: G_{a,i},
// G_{i,a}, R_i slabs | barrier | G_ii slab | barrier.  Every slab repeats the
// one-workgroup kernel's operations in the same order, so the results are bitwise
// those of nrgf_sweep_kernel, also in its direct mode (the reduced separator system
// of the n-diagonal DDRGF, with its first nr block rows carried to the last column).
#include "kernels.h"
#include "split_engine.h"

namespace rgfk {

#if defined(RGFK_INST_T) && (RGFK_INST_T == 4 || RGFK_INST_T == 8)

template <int T, int K, int NW>
__global__ __launch_bounds__(64 * NW, (T == 4 && K == 4) ? 2 : 1) void nrgf_split_kernel(NSweepArgs a) {
  constexpr int BP = 16 * T;
  constexpr int TR = T / K;
  __shared__ GJShared sh;
  __shared__ double red[NW];
  __shared__ int flag;
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int k = slot % K;
  const int e = (slot / K) * 8 + xcd;
  if (e >= a.ne) return;
  const bool leader = k == 0;
  const int row0 = 16 * TR * k;
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
  unsigned* ctr = a.sync + (size_t)e * 16;
  int* info = a.info + e;

  auto Sblk = [&](int i, int j) { return Sw + ((size_t)(w + j - i) * l + i) * bpbp; };
  auto Hblk = [&](int i, int j) { return Hband + ((size_t)(w + j - i) * l + i) * bb; };
  auto Rrow = [&](int tr, int i) { return Rx + ((size_t)(tr - 1) * l + i) * bpbp; };
  auto Gblk = [&](int i, int j) { return Gout + ((size_t)(w + j - i) * l + i) * bb; };
  auto Ublk = [&](int c, int i) { return U + ((size_t)i * w + (i - c - 1)) * bpbp; };
  auto Lblk = [&](int i, int c) { return L + ((size_t)i * w + (i - c - 1)) * bpbp; };
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pb = [&](const double2* p) { return opnd(p, b, b, b); };

  unsigned nbar = 0;
  auto bar = [&]() -> bool {
    ++nbar;
    return group_barrier(ctr, nbar * K, a.spin_limit, &flag);
  };
  SAcc<TR, T, NW> sa;
  int bad_layer = -1;

  auto body = [&]() -> bool {
    // ---------------- prologue: S = band of M(E) ----------------
    for (int i = 0; i < l; ++i) {
      for (int kk = -w; kk <= w; ++kk) {
        const int j = i + kk;
        if (j < 0 || j >= l) continue;
        if (a.direct) {
          sload<TR, T, NW>(sa, Pb(Hblk(i, j)), row0);
        } else if (kk == 0) {
          sacc_zero<TR, T, NW>(sa);
          sadd_diag<TR, T, NW>(sa, Hblk(i, i), b, z, i == 0 ? sL : nullptr, i == l - 1 ? sR : nullptr, row0);
        } else {
          sload<TR, T, NW>(sa, Pb(Hblk(i, j)), row0, -1.0);
        }
        sstore<TR, T, NW>(sa, Sblk(i, j), BP, BP, BP, row0);
        if (a.direct && kk == 0 && b < BP) {
          // identity on the padding of a directly given diagonal block (own rows)
          __syncthreads();
          for (int r = row0 + (int)threadIdx.x; r < row0 + 16 * TR; r += 64 * NW)
            if (r >= b) Sblk(i, i)[(size_t)r * BP + r] = make_double2(1.0, 0.0);
        }
      }
    }
    if (!bar()) return false;
    // ---------------- upward pass ----------------
    for (int i = l - 1; i >= 0; --i) {
      if (leader) {
        Acc<T, NW> acc;
        load<T, NW>(acc, P(Sblk(i, i)));
        gj_invert<T, NW>(acc, g + (size_t)i * bpbp, sh);
        if (sh.bad && bad_layer < 0) bad_layer = i;
      }
      if (!bar()) return false;
      const int c0 = i - w < 0 ? 0 : i - w;
      for (int c = c0; c < i; ++c) {
        sgemm<TR, T, NW>(sa, P(g + (size_t)i * bpbp), P(Sblk(i, c)), 1.0, row0);
        sstore<TR, T, NW>(sa, Lblk(i, c), BP, BP, BP, row0);
        sgemm<TR, T, NW>(sa, P(Sblk(c, i)), P(g + (size_t)i * bpbp), 1.0, row0);
        sstore<TR, T, NW>(sa, Ublk(c, i), BP, BP, BP, row0);
      }
      if (!bar()) return false;
      for (int ra = c0; ra < i; ++ra)
        for (int c = c0; c < i; ++c) {
          sload<TR, T, NW>(sa, P(Sblk(ra, c)), row0);
          smma<TR, T, NW>(sa, P(Sblk(ra, i)), P(Lblk(i, c)), -1.0, row0);
          sstore<TR, T, NW>(sa, Sblk(ra, c), BP, BP, BP, row0);
        }
      if (!bar()) return false;
    }
    // ---------------- downward pass ----------------
    sload<TR, T, NW>(sa, P(g), row0);
    sstore<TR, T, NW>(sa, Gblk(0, 0), b, b, b, row0);
    sstore<TR, T, NW>(sa, R, BP, BP, BP, row0);
    if (!bar()) return false;
    for (int i = 1; i < l; ++i) {
      const int c0 = i - w < 0 ? 0 : i - w;
      for (int ra = c0; ra < i; ++ra) {
        sacc_zero<TR, T, NW>(sa);
        for (int c = c0; c < i; ++c) smma<TR, T, NW>(sa, Pb(Gblk(ra, c)), P(Ublk(c, i)), -1.0, row0);
        sstore<TR, T, NW>(sa, Gblk(ra, i), b, b, b, row0);
        sacc_zero<TR, T, NW>(sa);
        for (int c = c0; c < i; ++c) smma<TR, T, NW>(sa, P(Lblk(i, c)), Pb(Gblk(c, ra)), -1.0, row0);
        sstore<TR, T, NW>(sa, Gblk(i, ra), b, b, b, row0);
      }
      sacc_zero<TR, T, NW>(sa);
      for (int c = c0; c < i; ++c) smma<TR, T, NW>(sa, P(R + (size_t)c * bpbp), P(Ublk(c, i)), -1.0, row0);
      sstore<TR, T, NW>(sa, R + (size_t)i * bpbp, BP, BP, BP, row0);
      for (int tr = 1; tr < a.nr && tr < i; ++tr) {
        sacc_zero<TR, T, NW>(sa);
        for (int c = c0; c < i; ++c)
          smma<TR, T, NW>(sa, c <= tr ? Pb(Gblk(tr, c)) : P(Rrow(tr, c)), P(Ublk(c, i)), -1.0, row0);
        sstore<TR, T, NW>(sa, Rrow(tr, i), BP, BP, BP, row0);
      }
      if (!bar()) return false;
      sload<TR, T, NW>(sa, P(g + (size_t)i * bpbp), row0);
      for (int c = c0; c < i; ++c) smma<TR, T, NW>(sa, P(Lblk(i, c)), Pb(Gblk(c, i)), -1.0, row0);
      sstore<TR, T, NW>(sa, Gblk(i, i), b, b, b, row0);
      if (!bar()) return false;
    }
    return true;
  };

  const bool ok = body();
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(info, RGF_INFO_SYNC_TIMEOUT);
    if (leader && threadIdx.x == 0 && a.T) a.T[e] = __builtin_nan("");
    return;
  }
  if (a.rows_last) {
    // blocks (tr, l-1), each workgroup its own rows: from the band when tr = l-1,
    // else from the propagated rows
    for (int tr = 0; tr < a.nr && tr < l; ++tr) {
      if (tr == l - 1)
        sload<TR, T, NW>(sa, Pb(Gblk(tr, l - 1)), row0);
      else
        sload<TR, T, NW>(sa, P(tr == 0 ? R + (size_t)(l - 1) * bpbp : Rrow(tr, l - 1)), row0);
      sstore<TR, T, NW>(sa, a.rows_last + ((size_t)e * a.nr + tr) * bb, b, b, b, row0);
    }
  }
  if (!leader) return;
  Acc<T, NW> acc;
  double Tval = 0.0;
  if (a.T) Tval = transmission<T, NW>(acc, R + (size_t)(l - 1) * bpbp, sL, sR, b, GamL, GamR, X1, red);
  if (bad_layer >= 0) {
    const double qnan = __builtin_nan("");
    for (size_t idx = threadIdx.x; idx < (size_t)(2 * w + 1) * l * bb; idx += 64 * NW)
      Gout[idx] = make_double2(qnan, qnan);
    Tval = qnan;
  }
  if (threadIdx.x == 0) {
    if (a.T) a.T[e] = Tval;
    if (bad_layer >= 0) atomicOr(info, bad_layer + 1);
  }
}

template <int T, int K>
hipError_t launch_nsplit_TK(const NSweepArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  const int groups = (a.ne + 7) / 8 * 8;
  NSweepArgs args = a;
  void* params[] = {&args};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&nrgf_split_kernel<T, K, NW>), dim3(groups * K),
                                    dim3(64 * NW), params, 0, s);
}

template <int T, int K>
int nsplit_capacity_TK() {
  constexpr int NW = T >= 7 ? 8 : 4;
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&nrgf_split_kernel<T, K, NW>),
                                                   64 * NW, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

static hipError_t launch_nsplit_T(const NSweepArgs& a, int K, hipStream_t s) {
  if (K == 2) return launch_nsplit_TK<RGFK_INST_T, 2>(a, s);
  if (K == 4) return launch_nsplit_TK<RGFK_INST_T, 4>(a, s);
  return hipErrorInvalidValue;
}

static int nsplit_capacity_T(int K) {
  if (K == 2) return nsplit_capacity_TK<RGFK_INST_T, 2>();
  if (K == 4) return nsplit_capacity_TK<RGFK_INST_T, 4>();
  return 0;
}

#if RGFK_INST_T == 4
hipError_t launch_nsplit_4(const NSweepArgs& a, int K, hipStream_t s) { return launch_nsplit_T(a, K, s); }
int nsplit_capacity_4(int K) { return nsplit_capacity_T(K); }
#else
hipError_t launch_nsplit_8(const NSweepArgs& a, int K, hipStream_t s) { return launch_nsplit_T(a, K, s); }
int nsplit_capacity_8(int K) { return nsplit_capacity_T(K); }
#endif

#endif  // RGFK_INST_T is 4 or 8

#if !defined(RGFK_INST_T) && !defined(RGFK_BATCHED_TU)
hipError_t launch_nsplit_4(const NSweepArgs& a, int K, hipStream_t s);
hipError_t launch_nsplit_8(const NSweepArgs& a, int K, hipStream_t s);
int nsplit_capacity_4(int K);
int nsplit_capacity_8(int K);

__global__ void nsplit_clear_kernel(unsigned* sync, int* info, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    sync[(size_t)e * 16] = 0u;
    info[e] = 0;
  }
}

int split_workgroups_n(int b, int ne, int want) {
  const int T = padded_block(b) / 16;
  if (T != 4 && T != 8) return 1;
  const int cands[2] = {4, 2};
  for (int K : cands) {
    if (want > 1 && K != want) continue;
    if (T % K != 0) continue;
    const int groups = (ne + 7) / 8 * 8;
    const int cap = T == 4 ? nsplit_capacity_4(K) : nsplit_capacity_8(K);
    if (cap > 0 && groups * K <= cap) return K;
  }
  return 1;
}

hipError_t launch_nrgf_split(const NSweepArgs& a, int K, hipStream_t s) {
  const int T = padded_block(a.b) / 16;
  hipLaunchKernelGGL(nsplit_clear_kernel, dim3((a.ne + 255) / 256), dim3(256), 0, s, a.sync, a.info, a.ne);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  err = T == 4 ? launch_nsplit_4(a, K, s) : T == 8 ? launch_nsplit_8(a, K, s) : hipErrorInvalidValue;
  if (err == hipSuccess) ktime_mark("nrgf_split_kernel", s);
  return err;
}
#endif

}  // namespace rgfk
