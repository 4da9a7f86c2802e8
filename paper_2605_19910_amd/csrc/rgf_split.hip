// Sequential RGF sweep (Algorithm 1, block tridiagonal) with K workgroups per
// energy, for grids with fewer energies than compute units.
//
// Workgroup k of a group owns the row slab [k bp/K, (k+1) bp/K) of every block
// product of the chain (split_engine.h); workgroup 0 also inverts each Schur pivot
// (the Gauss-Jordan inverse needs the whole block and stays on one compute unit).
// Per layer of the upward pass: inverse on workgroup 0 (the other workgroups compute
// the previous layer's U_{i+1} meanwhile) | barrier | L_i slabs | barrier | S_{i-1}
// slab | barrier; per layer of the downward pass: G_{i-1,i},
// G_{i,i-1}, R_i slabs | barrier | G_ii slab | barrier.  Blocks another workgroup
// reads go through the chain's workspace; the slabs of one block never overlap.
// The arithmetic of every output element is that of the one-workgroup sweep, so
// the results are bitwise the same.
//
// The members of a group must run at the same time: the launch is cooperative (all
// workgroups resident or no launch), and the group barriers are bounded waits.
// Group g's members are workgroups (g/8 K + k) * 8 + g%8, the same residue modulo 8,
// so that they share an XCD (and its L2) when workgroups are dealt to the XCDs in
// turn.
#include "kernels.h"
#include "split_engine.h"

namespace rgfk {

#if defined(RGFK_INST_T) && (RGFK_INST_T == 4 || RGFK_INST_T == 8)

template <int T, int K, int NW>
__global__ __launch_bounds__(64 * NW, (T == 4 && K == 4) ? 2 : 1) void rgf_split_kernel(SweepArgs a) {
  constexpr int BP = 16 * T;
  constexpr int TR = T / K;
  __shared__ GJShared sh;
  __shared__ double red[NW];
  __shared__ int flag;
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int k = slot % K;
  const int e = (slot / K) * 8 + xcd;
  if (e >= a.chains) return;
  const bool leader = k == 0;
  const int row0 = 16 * TR * k;
  const int l = a.l, b = a.b;
  const size_t bb = (size_t)b * b, bpbp = (size_t)BP * BP;
  const double2* Hl = a.H;
  const double2* Hd = a.H + (size_t)l * bb;
  const double2* Hu = a.H + (size_t)2 * l * bb;
  const double2* sL = a.sigL + (size_t)e * bb;
  const double2* sR = a.sigR + (size_t)e * bb;
  const double2 z = make_double2(a.E[e], a.eta_d);
  double2* Gout = a.G + (size_t)e * a.g_stride;
  double2* Gl = Gout;
  double2* Gd = Gout + (size_t)l * bb;
  double2* Gu = Gout + (size_t)2 * l * bb;
  // the sweep's workspace layout; the refinement slot holds the Schur pivot
  double2* g = a.ws + (size_t)e * a.ws_chain;
  double2* U = g + (size_t)l * bpbp;
  double2* L = g + (size_t)2 * l * bpbp;
  double2* Rb = g + (size_t)3 * l * bpbp;
  double2* GamL = Rb + 2 * bpbp;
  double2* GamR = GamL + bpbp;
  double2* X1 = GamR + bpbp;
  double2* Sbuf = X1 + bpbp;
  double2* Gup = Sbuf + 2 * bpbp;
  unsigned* ctr = a.sync + (size_t)e * 16;
  int* info = a.info + e;
  const double ms = -1.0;   // off-diagonal blocks of M are -H
  auto P = [&](const double2* p) { return opnd(p, BP, BP, BP); };
  auto Pn = [&](const double2* p) { return opnd(p, b, b, b); };

  unsigned nbar = 0;
  auto bar = [&]() -> bool {
    ++nbar;
    return group_barrier(ctr, nbar * K, a.spin_limit, &flag);
  };
  SAcc<TR, T, NW> sa;
  int bad_layer = -1;

  auto body = [&]() -> bool {
    // ---------------- upward pass ----------------
    sacc_zero<TR, T, NW>(sa);
    sadd_diag<TR, T, NW>(sa, Hd + (size_t)(l - 1) * bb, b, z, l == 1 ? sL : nullptr, sR, row0);
    sstore<TR, T, NW>(sa, Sbuf, BP, BP, BP, row0);
    if (!bar()) return false;
    // U_{i+1} = M_{i,i+1} g_{i+1} is needed only by the downward pass: its slabs are
    // computed by workgroups 1..K-1 while workgroup 0 inverts the next pivot
    // (workgroup 1 also takes workgroup 0's slab).
    auto u_slab = [&](int i1, int slab) {
      sgemm<TR, T, NW>(sa, Pn(Hu + (size_t)(i1 - 1) * bb), P(g + (size_t)i1 * bpbp), ms, 16 * TR * slab);
      sstore<TR, T, NW>(sa, U + (size_t)i1 * bpbp, BP, BP, BP, 16 * TR * slab);
    };
    for (int i = l - 1; i >= 0; --i) {
      double2* gi = g + (size_t)i * bpbp;
      if (leader) {
        Acc<T, NW> acc;
        load<T, NW>(acc, P(Sbuf));
        gj_invert<T, NW>(acc, gi, sh);
        if (sh.bad && bad_layer < 0) bad_layer = i;
      } else if (i + 1 < l) {
        u_slab(i + 1, k);
        if (k == 1) u_slab(i + 1, 0);
      }
      if (!bar()) return false;
      if (i == 0) break;
      sgemm<TR, T, NW>(sa, P(gi), Pn(Hl + (size_t)i * bb), ms, row0);
      sstore<TR, T, NW>(sa, L + (size_t)i * bpbp, BP, BP, BP, row0);
      if (!bar()) return false;
      // S_{i-1} = M_{i-1,i-1} - M_{i-1,i} L_i
      sgemm<TR, T, NW>(sa, Pn(Hu + (size_t)(i - 1) * bb), P(L + (size_t)i * bpbp), -ms, row0);
      sadd_diag<TR, T, NW>(sa, Hd + (size_t)(i - 1) * bb, b, z, i - 1 == 0 ? sL : nullptr, nullptr, row0);
      sstore<TR, T, NW>(sa, Sbuf, BP, BP, BP, row0);
      if (!bar()) return false;
    }
    // ---------------- downward pass ----------------
    sload<TR, T, NW>(sa, P(g), row0);
    sstore<TR, T, NW>(sa, Gd, b, b, b, row0);
    sstore<TR, T, NW>(sa, Rb, BP, BP, BP, row0);
    if (!bar()) return false;
    for (int i = 1; i < l; ++i) {
      const double2* Gp = Gd + (size_t)(i - 1) * bb;
      const double2* Ui = U + (size_t)i * bpbp;
      const double2* Li = L + (size_t)i * bpbp;
      double2* Gup_i = Gu + (size_t)(i - 1) * bb;
      sgemm<TR, T, NW>(sa, Pn(Gp), P(Ui), -1.0, row0);
      sstore<TR, T, NW>(sa, Gup_i, b, b, b, row0);
      sgemm<TR, T, NW>(sa, P(Li), Pn(Gp), -1.0, row0);
      sstore<TR, T, NW>(sa, Gl + (size_t)i * bb, b, b, b, row0);
      sgemm<TR, T, NW>(sa, P(Rb + (size_t)((i - 1) & 1) * bpbp), P(Ui), -1.0, row0);
      sstore<TR, T, NW>(sa, Rb + (size_t)(i & 1) * bpbp, BP, BP, BP, row0);
      if (!bar()) return false;
      sgemm<TR, T, NW>(sa, P(Li), Pn(Gup_i), -1.0, row0);
      sadd_from<TR, T, NW>(sa, P(g + (size_t)i * bpbp), row0);
      sstore<TR, T, NW>(sa, Gd + (size_t)i * bb, b, b, b, row0);
      if (!bar()) return false;
    }
    return true;
  };
  (void)Gup;

  const bool ok = body();
  if (!ok) {
    // a member of the group did not arrive in time: outputs undefined
    if (threadIdx.x == 0) atomicOr(info, RGF_INFO_SYNC_TIMEOUT);
    if (leader && threadIdx.x == 0 && a.T) a.T[e] = __builtin_nan("");
    return;
  }
  if (!leader) return;
  // ---------------- transmission and status (workgroup 0) ----------------
  Acc<T, NW> acc;
  double Tval = 0.0;
  if (a.T) Tval = transmission<T, NW>(acc, Rb + (size_t)((l - 1) & 1) * bpbp, sL, sR, b, GamL, GamR, X1, red);
  if (bad_layer >= 0) {
    const double qnan = __builtin_nan("");
    for (size_t idx = threadIdx.x; idx < (size_t)l * bb; idx += 64 * NW) {
      Gd[idx] = make_double2(qnan, qnan);
      Gl[idx] = make_double2(qnan, qnan);
      Gu[idx] = make_double2(qnan, qnan);
    }
    Tval = qnan;
  }
  if (threadIdx.x == 0) {
    if (a.T) a.T[e] = Tval;
    if (bad_layer >= 0) atomicOr(info, bad_layer + 1);
  }
}

template <int T, int K>
hipError_t launch_split_TK(const SweepArgs& a, hipStream_t s) {
  constexpr int NW = T >= 7 ? 8 : 4;
  const int groups = (a.chains + 7) / 8 * 8;
  SweepArgs args = a;
  void* params[] = {&args};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&rgf_split_kernel<T, K, NW>), dim3(groups * K),
                                    dim3(64 * NW), params, 0, s);
}

template <int T, int K>
int split_capacity_TK() {
  constexpr int NW = T >= 7 ? 8 : 4;
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&rgf_split_kernel<T, K, NW>),
                                                   64 * NW, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

static hipError_t launch_split_T(const SweepArgs& a, int K, hipStream_t s) {
  if (K == 2) return launch_split_TK<RGFK_INST_T, 2>(a, s);
  if (K == 4) return launch_split_TK<RGFK_INST_T, 4>(a, s);
  return hipErrorInvalidValue;
}

static int split_capacity_T(int K) {
  if (K == 2) return split_capacity_TK<RGFK_INST_T, 2>();
  if (K == 4) return split_capacity_TK<RGFK_INST_T, 4>();
  return 0;
}

#if RGFK_INST_T == 4
hipError_t launch_split_4(const SweepArgs& a, int K, hipStream_t s) { return launch_split_T(a, K, s); }
int split_capacity_4(int K) { return split_capacity_T(K); }
#else
hipError_t launch_split_8(const SweepArgs& a, int K, hipStream_t s) { return launch_split_T(a, K, s); }
int split_capacity_8(int K) { return split_capacity_T(K); }
#endif

#endif  // RGFK_INST_T is 4 or 8

#if !defined(RGFK_INST_T) && !defined(RGFK_BATCHED_TU)
hipError_t launch_split_4(const SweepArgs& a, int K, hipStream_t s);
hipError_t launch_split_8(const SweepArgs& a, int K, hipStream_t s);
int split_capacity_4(int K);
int split_capacity_8(int K);

__global__ void split_clear_kernel(unsigned* sync, int* info, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    sync[(size_t)e * 16] = 0u;
    info[e] = 0;
  }
}

int split_workgroups(int b, int ne, int want) {
  const int T = padded_block(b) / 16;
  if (T != 4 && T != 8) return 1;
  const int cands[2] = {4, 2};
  for (int K : cands) {
    if (want > 1 && K != want) continue;
    if (T % K != 0) continue;
    const int groups = (ne + 7) / 8 * 8;
    const int cap = T == 4 ? split_capacity_4(K) : split_capacity_8(K);
    if (cap > 0 && groups * K <= cap) return K;
  }
  return 1;
}

hipError_t launch_rgf_split(const SweepArgs& a, int K, hipStream_t s) {
  const int T = padded_block(a.b) / 16;
  hipLaunchKernelGGL(split_clear_kernel, dim3((a.chains + 255) / 256), dim3(256), 0, s, a.sync, a.info, a.chains);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  err = T == 4 ? launch_split_4(a, K, s) : T == 8 ? launch_split_8(a, K, s) : hipErrorInvalidValue;
  if (err == hipSuccess) ktime_mark("rgf_split_kernel", s);
  return err;
}
#endif

}  // namespace rgfk
