// Row-slab block operations for a chain shared by K workgroups (gfx950).
//
// The sequential sweep of one energy has little parallelism beyond one block
// product at a time.  When there are fewer energies than compute units, K
// workgroups share a chain: workgroup k owns the row slab [k*bp/K, (k+1)*bp/K) of
// every block product (TR = T/K tile rows, all T tile columns), the pivot inverse
// runs on workgroup 0, and the K workgroups meet at group barriers between the
// steps that read a whole block another one wrote.
//
// Every slab operation performs, for each output element, exactly the floating
// point operations of the whole-block routine of block_engine.h in the same
// order (same k order, same four real products per complex product, same sign
// handling), so a chain computed by K workgroups is bitwise the chain computed by
// one.
#pragma once
#include "block_engine.h"

namespace rgfk {

// Slab accumulator: TR x TC tiles of 16 x 16 over NW waves arranged WR x WC.
template <int TR, int TC, int NW>
struct SAcc {
  static constexpr int WR = TR < NW ? TR : NW;
  static constexpr int WC = NW / WR;
  static constexpr int RR = (TR + WR - 1) / WR;
  static constexpr int RC = (TC + WC - 1) / WC;
  dbl4 re[RR][RC];
  dbl4 im[RR][RC];
};

template <int TR, int TC, int NW>
__device__ __forceinline__ void slab_origin(int& tr0, int& tc0) {
  using S = SAcc<TR, TC, NW>;
  const int wv = wave_id();
  tr0 = (wv / S::WC) * S::RR;
  tc0 = (wv % S::WC) * S::RC;
}

template <int TR, int TC, int NW>
__device__ __forceinline__ void sacc_zero(SAcc<TR, TC, NW>& a) {
  using S = SAcc<TR, TC, NW>;
#pragma unroll
  for (int r = 0; r < S::RR; ++r)
#pragma unroll
    for (int c = 0; c < S::RC; ++c) {
      a.re[r][c] = dbl4{0.0, 0.0, 0.0, 0.0};
      a.im[r][c] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
}

// acc += sgn * A[row0 + (0..16TR), :] * B, k over 16 TC; A and B non-conjugated
// operand views of the whole blocks.  Mirrors mma(): fragments two k-steps ahead,
// sgn applied to B, first terms of every tile then the second ones.
template <int TR, int TC, int NW>
__device__ __forceinline__ void smma(SAcc<TR, TC, NW>& acc, const Opnd& A, const Opnd& B, double sgn,
                                     int row0) {
  using S = SAcc<TR, TC, NW>;
  constexpr int RR = S::RR, RC = S::RC;
  constexpr int NKS = 16 * TC / 4;
  const int l = lane_id();
  int tr0, tc0;
  slab_origin<TR, TC, NW>(tr0, tc0);
  const int li = l & 15, lk = l >> 4;
  double2 a[2][RR], b[2][RC];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int r = 0; r < RR; ++r)
      a[d][r] = (tr0 + r < TR) ? opnd_get_n(A, row0 + 16 * (tr0 + r) + li, 4 * d + lk) : make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < RC; ++c)
      b[d][c] = (tc0 + c < TC) ? opnd_get_n(B, 4 * d + lk, 16 * (tc0 + c) + li) : make_double2(0.0, 0.0);
  }
  for (int ks0 = 0; ks0 < NKS; ks0 += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int ks = ks0 + d;
      double2 ac[RR], bc[RC];
#pragma unroll
      for (int r = 0; r < RR; ++r) ac[r] = a[d][r];
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        bc[c] = b[d][c];
        bc[c].x *= sgn;
        bc[c].y *= sgn;
      }
      if (ks + 2 < NKS) {
        const int k = 4 * (ks + 2) + lk;
#pragma unroll
        for (int r = 0; r < RR; ++r)
          a[d][r] = (tr0 + r < TR) ? opnd_get_n(A, row0 + 16 * (tr0 + r) + li, k) : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < RC; ++c)
          b[d][c] = (tc0 + c < TC) ? opnd_get_n(B, k, 16 * (tc0 + c) + li) : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        if (tr0 + r >= TR) continue;
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          if (tc0 + c >= TC) continue;
          acc.re[r][c] = mfma(ac[r].x, bc[c].x, acc.re[r][c]);
          acc.im[r][c] = mfma(ac[r].x, bc[c].y, acc.im[r][c]);
        }
      }
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        if (tr0 + r >= TR) continue;
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          if (tc0 + c >= TC) continue;
          acc.re[r][c] = mfma(-ac[r].y, bc[c].y, acc.re[r][c]);
          acc.im[r][c] = mfma(ac[r].y, bc[c].x, acc.im[r][c]);
        }
      }
    }
  }
}

// acc = sgn * A[slab] * B
template <int TR, int TC, int NW>
__device__ __forceinline__ void sgemm(SAcc<TR, TC, NW>& acc, const Opnd& A, const Opnd& B, double sgn, int row0) {
  sacc_zero<TR, TC, NW>(acc);
  smma<TR, TC, NW>(acc, A, B, sgn, row0);
}

// Write the slab into rows row0.. of p (p[i*ld + j] for i < nr, j < nc).
template <int TR, int TC, int NW>
__device__ __forceinline__ void sstore(const SAcc<TR, TC, NW>& acc, double2* p, int ld, int nr, int nc, int row0) {
  using S = SAcc<TR, TC, NW>;
  const int l = lane_id();
  int tr0, tc0;
  slab_origin<TR, TC, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < S::RR; ++r) {
    if (tr0 + r >= TR) continue;
#pragma unroll
    for (int c = 0; c < S::RC; ++c) {
      if (tc0 + c >= TC) continue;
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + 16 * (tr0 + r) + c_row(l, v);
        if (i < nr && j < nc) p[(size_t)i * ld + j] = make_double2(acc.re[r][c][v], acc.im[r][c][v]);
      }
    }
  }
}

// acc = sgn * X[slab] (operand view of the whole block)
template <int TR, int TC, int NW>
__device__ __forceinline__ void sload(SAcc<TR, TC, NW>& acc, const Opnd& X, int row0, double sgn = 1.0) {
  using S = SAcc<TR, TC, NW>;
  const int l = lane_id();
  int tr0, tc0;
  slab_origin<TR, TC, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < S::RR; ++r)
#pragma unroll
    for (int c = 0; c < S::RC; ++c) {
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + 16 * (tr0 + r) + c_row(l, v);
        const double2 x = (tr0 + r < TR && tc0 + c < TC) ? opnd_get(X, i, j) : make_double2(0.0, 0.0);
        acc.re[r][c][v] = sgn * x.x;
        acc.im[r][c][v] = sgn * x.y;
      }
    }
}

// acc += X[slab]
template <int TR, int TC, int NW>
__device__ __forceinline__ void sadd_from(SAcc<TR, TC, NW>& acc, const Opnd& X, int row0) {
  using S = SAcc<TR, TC, NW>;
  const int l = lane_id();
  int tr0, tc0;
  slab_origin<TR, TC, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < S::RR; ++r)
#pragma unroll
    for (int c = 0; c < S::RC; ++c) {
      if (tr0 + r >= TR || tc0 + c >= TC) continue;
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double2 x = opnd_get(X, row0 + 16 * (tr0 + r) + c_row(l, v), j);
        acc.re[r][c][v] += x.x;
        acc.im[r][c][v] += x.y;
      }
    }
}

// acc += (z I - H_d - [first] Sigma_L - [last] Sigma_R) on the slab rows, identity on
// the padding (the arithmetic of assemble_diag(..., add = true)).
template <int TR, int TC, int NW>
__device__ __forceinline__ void sadd_diag(SAcc<TR, TC, NW>& acc, const double2* Hd, int b, double2 z,
                                          const double2* sL, const double2* sR, int row0) {
  using S = SAcc<TR, TC, NW>;
  const int l = lane_id();
  int tr0, tc0;
  slab_origin<TR, TC, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < S::RR; ++r)
#pragma unroll
    for (int c = 0; c < S::RC; ++c) {
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + 16 * (tr0 + r) + c_row(l, v);
        double2 x = make_double2(0.0, 0.0);
        if (tr0 + r < TR && tc0 + c < TC) {
          if (i < b && j < b) {
            const size_t o = (size_t)i * b + j;
            const double2 h = Hd[o];
            x.x = -h.x; x.y = -h.y;
            if (sL) { const double2 s = sL[o]; x.x -= s.x; x.y -= s.y; }
            if (sR) { const double2 s = sR[o]; x.x -= s.x; x.y -= s.y; }
            if (i == j) { x.x += z.x; x.y += z.y; }
          } else if (i == j) {
            x.x = 1.0;
          }
        }
        acc.re[r][c][v] += x.x;
        acc.im[r][c][v] += x.y;
      }
    }
}

// Group barrier of the K workgroups of one chain: every workgroup's global writes
// before the call are visible to every workgroup of the group after it.  Every wave
// first waits until its own stores have completed (reached the L2); after the
// workgroup barrier thread 0 releases at agent scope (the group may span XCDs,
// whose L2s are not coherent with each other: the L2's dirty lines are written
// back), increments the group's counter and waits until it reaches
// target = (barriers so far) * K, then acquires at agent scope (invalidating the
// compute unit's L1 for every wave of the workgroup).  One release per workgroup
// instead of one per wave: measured 20 us against 90-120 us per barrier for four
// workgroups with 256 KiB of stores each.  The wait is bounded: after spin_limit
// polls the workgroup gives up and the call returns false (the group's outputs are
// then undefined; the caller reports it).
__device__ __forceinline__ bool group_barrier(unsigned* ctr, unsigned target, long long spin_limit, int* flag) {
  // this wave's stores have completed; the memory clobber keeps the compiler from
  // moving any store of the phase below this point
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomicAdd(ctr, 1u);
    long long n = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++n > spin_limit) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = ok;
  }
  __syncthreads();
  const bool ok = *flag != 0;
  __syncthreads();
  return ok;
}

}  // namespace rgfk
