// Workgroup-level complex FP64 block engine for gfx950 (CDNA4).
//
// One workgroup of NW wave64 (NW = 4 or 8) owns one b x b complex block (b padded
// to bp = 16*T) held in registers as MFMA accumulator tiles of 16 x 16: wave
// (wr, wc), wr < NW/2, wc < 2, owns the RR x RC tiles starting at tile
// (wr*RR, wc*RC), RR = ceil(T / (NW/2)), RC = ceil(T/2).  Everything the
// recursive Green's function sweep needs is built from three operations on such a
// block:
//   * mma()        acc += sign * A * B with A, B streamed from global memory
//                  (complex product as four real MFMA products, "4M");
//   * gj_invert()  in-place inverse by blocked Gauss-Jordan with partial (row)
//                  pivoting, panel of 16 columns staged in LDS, rank-16 trailing
//                  updates on MFMA;
//   * store()/assemble_diag() to move a block between registers and memory.
//
// Complex numbers are interleaved (re, im) double pairs, blocks row-major.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgfk {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int MAXBP = 128;     // largest padded block size
constexpr int PNLD = 17;       // LDS row pitch of the panel (16 + 1 to spread banks)

// ---------------------------------------------------------------------------
// MFMA f64 16x16x4 register layout:
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element v (0..3) holds D[l / 16 + 4 * v][l % 16]
// ---------------------------------------------------------------------------
__device__ __forceinline__ int c_row(int l, int v) { return (l >> 4) + 4 * v; }
__device__ __forceinline__ int c_col(int l) { return l & 15; }

__device__ __forceinline__ dbl4 mfma(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cinv(double2 p) {
  double d = p.x * p.x + p.y * p.y;
  return make_double2(p.x / d, -p.y / d);
}
__device__ __forceinline__ double cabs1(double2 p) { return fabs(p.x) + fabs(p.y); }

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// An operand view of a complex matrix in global memory.  Entries outside
// [0, nr) x [0, nc) read as zero (this pads a b x b block to bp x bp).
// With conjT the logical operand is the conjugate transpose of the stored one.
struct Opnd {
  const double2* p;
  int ld;
  int nr, nc;
  int conjT;
};

__device__ __forceinline__ Opnd opnd(const double2* p, int ld, int nr, int nc, int conjT = 0) {
  Opnd o;
  o.p = p; o.ld = ld; o.nr = nr; o.nc = nc; o.conjT = conjT;
  return o;
}

__device__ __forceinline__ double2 opnd_get(const Opnd& o, int i, int j) {
  if (i >= o.nr || j >= o.nc) return make_double2(0.0, 0.0);
  if (!o.conjT) return o.p[(size_t)i * o.ld + j];
  double2 v = o.p[(size_t)j * o.ld + i];
  v.y = -v.y;
  return v;
}

// Accumulator: the part of a bp x bp complex block owned by this wave.
template <int T, int NW>
struct Acc {
  static constexpr int RR = (T + NW / 2 - 1) / (NW / 2);
  static constexpr int RC = (T + 1) / 2;
  static constexpr int NT = 64 * NW;
  dbl4 re[RR][RC];
  dbl4 im[RR][RC];
};

template <int T, int NW>
__device__ __forceinline__ void tile_origin(int& tr0, int& tc0) {
  const int wv = wave_id();
  tr0 = (wv >> 1) * Acc<T, NW>::RR;
  tc0 = (wv & 1) * Acc<T, NW>::RC;
}

template <int T, int NW>
__device__ __forceinline__ void acc_zero(Acc<T, NW>& a) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      a.re[r][c] = dbl4{0.0, 0.0, 0.0, 0.0};
      a.im[r][c] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
}

// acc += sgn * A * B for operands that may be conjugate-transposed: fragments
// read straight from global memory one k-step ahead.
template <int T, int NW>
__device__ __forceinline__ void mma_conj(Acc<T, NW>& acc, const Opnd& A, const Opnd& B, double sgn) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  constexpr int BP = 16 * T;
  constexpr int NKS = BP / 4;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
  const int li = l & 15, lk = l >> 4;

  double2 a[RR], b[RC], an[RR], bn[RC];
#pragma unroll
  for (int r = 0; r < RR; ++r) a[r] = opnd_get(A, 16 * (tr0 + r) + li, lk);
#pragma unroll
  for (int c = 0; c < RC; ++c) {
    b[c] = opnd_get(B, lk, 16 * (tc0 + c) + li);
    b[c].x *= sgn; b[c].y *= sgn;
  }
  for (int ks = 0; ks < NKS; ++ks) {
    if (ks + 1 < NKS) {
      const int k = 4 * (ks + 1) + lk;
#pragma unroll
      for (int r = 0; r < RR; ++r) an[r] = opnd_get(A, 16 * (tr0 + r) + li, k);
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        bn[c] = opnd_get(B, k, 16 * (tc0 + c) + li);
        bn[c].x *= sgn; bn[c].y *= sgn;
      }
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      if (tr0 + r >= T) continue;
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (tc0 + c >= T) continue;
        acc.re[r][c] = mfma(a[r].x, b[c].x, acc.re[r][c]);
        acc.re[r][c] = mfma(-a[r].y, b[c].y, acc.re[r][c]);
        acc.im[r][c] = mfma(a[r].x, b[c].y, acc.im[r][c]);
        acc.im[r][c] = mfma(a[r].y, b[c].x, acc.im[r][c]);
      }
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) a[r] = an[r];
#pragma unroll
    for (int c = 0; c < RC; ++c) b[c] = bn[c];
  }
}

__device__ __forceinline__ double2 opnd_get_n(const Opnd& o, int i, int j) {
  return (i < o.nr && j < o.nc) ? o.p[(size_t)i * o.ld + j] : make_double2(0.0, 0.0);
}

// acc += sgn * A * B, A and B logical bp x bp operands.  Non-conjugated operands
// stream from global memory two k-steps ahead of the MFMAs (the fragments of a
// k-step are in flight for two k-steps of MFMA work); each accumulator receives
// its four real products in the same order as in mma_conj, so both give
// bitwise the same result.
template <int T, int NW>
__device__ __forceinline__ void mma(Acc<T, NW>& acc, const Opnd& A, const Opnd& B, double sgn) {
  if (A.conjT || B.conjT) {
    mma_conj<T, NW>(acc, A, B, sgn);
    return;
  }
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  constexpr int BP = 16 * T;
  constexpr int NKS = BP / 4;       // k-steps, a multiple of 4
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
  const int li = l & 15, lk = l >> 4;
  double2 a[2][RR], b[2][RC];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int r = 0; r < RR; ++r)
      a[d][r] = (tr0 + r < T) ? opnd_get_n(A, 16 * (tr0 + r) + li, 4 * d + lk) : make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < RC; ++c)
      b[d][c] = (tc0 + c < T) ? opnd_get_n(B, 4 * d + lk, 16 * (tc0 + c) + li) : make_double2(0.0, 0.0);
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
          a[d][r] = (tr0 + r < T) ? opnd_get_n(A, 16 * (tr0 + r) + li, k) : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < RC; ++c)
          b[d][c] = (tc0 + c < T) ? opnd_get_n(B, k, 16 * (tc0 + c) + li) : make_double2(0.0, 0.0);
      }
      // first terms of every tile, then the second ones: consecutive MFMAs are independent
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        if (tr0 + r >= T) continue;
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          if (tc0 + c >= T) continue;
          acc.re[r][c] = mfma(ac[r].x, bc[c].x, acc.re[r][c]);
          acc.im[r][c] = mfma(ac[r].x, bc[c].y, acc.im[r][c]);
        }
      }
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        if (tr0 + r >= T) continue;
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          if (tc0 + c >= T) continue;
          acc.re[r][c] = mfma(-ac[r].y, bc[c].y, acc.re[r][c]);
          acc.im[r][c] = mfma(ac[r].y, bc[c].x, acc.im[r][c]);
        }
      }
    }
  }
}

// Write acc (times sgn) into p[i*ld + j] for i < nr, j < nc.
template <int T, int NW>
__device__ __forceinline__ void store(const Acc<T, NW>& acc, double2* p, int ld, int nr, int nc,
                                      double sgn = 1.0) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    if (tr0 + r >= T) continue;
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      if (tc0 + c >= T) continue;
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (tr0 + r) + c_row(l, v);
        if (i < nr && j < nc)
          p[(size_t)i * ld + j] = make_double2(sgn * acc.re[r][c][v], sgn * acc.im[r][c][v]);
      }
    }
  }
}

// Write (sgn * acc)^H into p: element (i, j) of acc goes to p[j*ld + i], conjugated,
// for j < nr, i < nc (nr x nc is the shape of the destination).
template <int T, int NW>
__device__ __forceinline__ void store_conjT(const Acc<T, NW>& acc, double2* p, int ld, int nr, int nc,
                                            double sgn = 1.0) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    if (tr0 + r >= T) continue;
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      if (tc0 + c >= T) continue;
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (tr0 + r) + c_row(l, v);
        if (j < nr && i < nc)
          p[(size_t)j * ld + i] = make_double2(sgn * acc.re[r][c][v], -sgn * acc.im[r][c][v]);
      }
    }
  }
}

// Load a block (read through an operand view) into acc.
template <int T, int NW>
__device__ __forceinline__ void load(Acc<T, NW>& acc, const Opnd& X, double sgn = 1.0) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (tr0 + r) + c_row(l, v);
        double2 x = (tr0 + r < T && tc0 + c < T) ? opnd_get(X, i, j) : make_double2(0.0, 0.0);
        acc.re[r][c][v] = sgn * x.x;
        acc.im[r][c][v] = sgn * x.y;
      }
    }
}

// acc = (z I - H_d - [first] Sigma_L - [last] Sigma_R) on the b x b part and the
// identity on the padding: a diagonal block of M(E) = (E + i eta) I - H - Sigma.
template <int T, int NW>
__device__ __forceinline__ void assemble_diag(Acc<T, NW>& acc, const double2* Hd, int b, double2 z,
                                              const double2* sL, const double2* sR, bool add = false) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (tr0 + r) + c_row(l, v);
        double2 x = make_double2(0.0, 0.0);
        if (tr0 + r < T && tc0 + c < T) {
          if (i < b && j < b) {
            const size_t o = (size_t)i * b + j;
            double2 h = Hd[o];
            x.x = -h.x; x.y = -h.y;
            if (sL) { double2 s = sL[o]; x.x -= s.x; x.y -= s.y; }
            if (sR) { double2 s = sR[o]; x.x -= s.x; x.y -= s.y; }
            if (i == j) { x.x += z.x; x.y += z.y; }
          } else if (i == j) {
            x.x = 1.0;
          }
        }
        if (add) {
          acc.re[r][c][v] += x.x;
          acc.im[r][c][v] += x.y;
        } else {
          acc.re[r][c][v] = x.x;
          acc.im[r][c][v] = x.y;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Mixed precision products: operands rounded to FP32 (round to nearest even),
// v_mfma_f32_16x16x4f32 with FP32 accumulation over the whole k range, the
// result widened to FP64 once.  F32_ROW(r) maps the row of an FP32 accumulator
// element onto the FP64 accumulator row of the same lane/element, by feeding the
// A operand with permuted rows.
// ---------------------------------------------------------------------------
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ flt4 mfma32(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP32 16x16x4 accumulator: lane l, element v holds row 4*(l/16) + v (FP64: l/16 + 4v).
// Feeding A'[r] = A[perm(r)] with perm(4q + v) = q + 4v puts row q + 4v there.
__device__ __forceinline__ int f32_row(int r) { return (r >> 2) + 4 * (r & 3); }

// acc = sgn * A * B with FP32 products and FP32 accumulation.
template <int T, int NW>
__device__ __forceinline__ void gemm_f32(Acc<T, NW>& acc, const Opnd& A, const Opnd& B, double sgn) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  constexpr int BP = 16 * T;
  constexpr int NKS = BP / 4;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
  const int li = f32_row(l & 15), lj = l & 15, lk = l >> 4;
  flt4 cre[RR][RC], cim[RR][RC];
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      cre[r][c] = flt4{0.f, 0.f, 0.f, 0.f};
      cim[r][c] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  float2 a[RR], b[RC], an[RR], bn[RC];
  auto ldA = [&](int r, int k) {
    const double2 x = opnd_get(A, 16 * (tr0 + r) + li, k);
    return make_float2((float)x.x, (float)x.y);
  };
  auto ldB = [&](int c, int k) {
    const double2 x = opnd_get(B, k, 16 * (tc0 + c) + lj);
    return make_float2((float)(sgn * x.x), (float)(sgn * x.y));
  };
#pragma unroll
  for (int r = 0; r < RR; ++r) a[r] = ldA(r, lk);
#pragma unroll
  for (int c = 0; c < RC; ++c) b[c] = ldB(c, lk);
  for (int ks = 0; ks < NKS; ++ks) {
    if (ks + 1 < NKS) {
      const int k = 4 * (ks + 1) + lk;
#pragma unroll
      for (int r = 0; r < RR; ++r) an[r] = ldA(r, k);
#pragma unroll
      for (int c = 0; c < RC; ++c) bn[c] = ldB(c, k);
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      if (tr0 + r >= T) continue;
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (tc0 + c >= T) continue;
        cre[r][c] = mfma32(a[r].x, b[c].x, cre[r][c]);
        cre[r][c] = mfma32(-a[r].y, b[c].y, cre[r][c]);
        cim[r][c] = mfma32(a[r].x, b[c].y, cim[r][c]);
        cim[r][c] = mfma32(a[r].y, b[c].x, cim[r][c]);
      }
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) a[r] = an[r];
#pragma unroll
    for (int c = 0; c < RC; ++c) b[c] = bn[c];
  }
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc.re[r][c][v] = (double)cre[r][c][v];
        acc.im[r][c][v] = (double)cim[r][c][v];
      }
}

// acc = sgn * A * B in the precision selected by MIXED (0: FP64 MFMA, 1: FP32 MFMA).
template <int MIXED, int T, int NW>
__device__ __forceinline__ void gemm_to(Acc<T, NW>& acc, const Opnd& A, const Opnd& B, double sgn) {
  if constexpr (MIXED) {
    gemm_f32<T, NW>(acc, A, B, sgn);
  } else {
    acc_zero<T, NW>(acc);
    mma<T, NW>(acc, A, B, sgn);
  }
}

// acc += sgn * X (X read through an operand view).
template <int T, int NW>
__device__ __forceinline__ void add_from(Acc<T, NW>& acc, const Opnd& X, double sgn = 1.0) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      if (tr0 + r >= T || tc0 + c >= T) continue;
      const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double2 x = opnd_get(X, 16 * (tr0 + r) + c_row(l, v), j);
        acc.re[r][c][v] += sgn * x.x;
        acc.im[r][c][v] += sgn * x.y;
      }
    }
}

// acc += I on the diagonal.
template <int T, int NW>
__device__ __forceinline__ void add_identity(Acc<T, NW>& acc) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      if (tr0 + r >= T || tc0 + c >= T) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (16 * (tr0 + r) + c_row(l, v) == 16 * (tc0 + c) + c_col(l)) acc.re[r][c][v] += 1.0;
    }
}

// acc += I on the diagonal entries with index >= b (the padding of a b x b block).
template <int T, int NW>
__device__ __forceinline__ void add_identity_beyond(Acc<T, NW>& acc, int b) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      if (tr0 + r >= T || tc0 + c >= T) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (tr0 + r) + c_row(l, v), j = 16 * (tc0 + c) + c_col(l);
        if (i == j && i >= b) acc.re[r][c][v] += 1.0;
      }
    }
}

// Pivot-search key of a row whose candidate has magnitude k (k < 0: non-finite):
// unpivoted rows rank above pivoted rows and lanes without a row (key 0),
// non-finite candidates below finite ones; finite ones by the top 57 bits of k,
// then by lowest row (the row, < 128, fills the low 7 bits).
__device__ __forceinline__ uint64_t pivot_key(double k, int row) {
  const uint64_t hi = k < 0.0 ? 1 : ((uint64_t)__double_as_longlong(k) >> 7) + 2;
  return (hi << 7) | (uint64_t)(127 - row);
}

// Wave-wide maximum of a 64-bit key (device library routine).
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);

// LDS scratch of the Gauss-Jordan inversion.
struct GJShared {
  double2 pn[MAXBP][PNLD];     // current 16-column panel (all rows)
  double2 rw[16][MAXBP];       // the panel's pivot rows, as they were before the panel
  int rowsel[MAXBP];           // rowsel[c] = row chosen as pivot for column c
  int slot[MAXBP];             // slot[row] = position of row among the panel pivots, or -1
  int rowdst[MAXBP];
  int bad;                     // nonzero: a pivot was zero or non-finite
};

// In-place inverse of the block held in acc, by blocked Gauss-Jordan with row
// pivoting (sweep operator on pivots (r_c, c), c = 0..bp-1, r_c chosen as the
// unpivoted row of largest |re|+|im| in column c).  The swept matrix B satisfies
// inverse[c_t][r_s] = B[r_t][c_s]; on exit the inverse is written to g (row-major,
// ld = bp) with that permutation applied, and acc is left holding B.
// Returns (in sh.bad) whether a zero or non-finite pivot was met.
template <int T, int NW>
__device__ __forceinline__ void gj_invert(Acc<T, NW>& acc, double2* g, GJShared& sh) {
  constexpr int RR = Acc<T, NW>::RR;
  constexpr int RC = Acc<T, NW>::RC;
  constexpr int BP = 16 * T;
  constexpr int NT = Acc<T, NW>::NT;
  constexpr int PSTEP = NT / 16;                   // row step of the panel mapping
  constexpr int PM = (BP + PSTEP - 1) / PSTEP;     // panel rows per thread
  const int t = threadIdx.x;
  const int l = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);

  for (int i = t; i < BP; i += NT) sh.slot[i] = -1;
  // pivoted flags of this lane's candidate rows l + 64 q (every wave tracks all pivots)
  constexpr int NQ = (BP + 63) / 64;
  unsigned pivmask = 0;
  if (t == 0) sh.bad = 0;
  __syncthreads();

  const int pj = t & 15;        // panel column handled by this thread
  const int pi0 = t >> 4;       // first panel row handled (rows pi0 + PSTEP m)

  for (int kt = 0; kt < T; ++kt) {
    // 1. panel columns [16 kt, 16 kt + 16) to LDS
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (tr0 + r >= T || tc0 + c != kt) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * (tr0 + r) + c_row(l, v);
          sh.pn[i][c_col(l)] = make_double2(acc.re[r][c][v], acc.im[r][c][v]);
        }
      }
    __syncthreads();

    // 2. sweep the 16 panel columns (restricted to the panel)
    for (int ci = 0; ci < 16; ++ci) {
      // pivot search, done redundantly by every wave: argmax of |re| + |im| over
      // the unpivoted rows (ties: lowest row) as one 64-bit maximum
      uint64_t u = 0;
      int nf = 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int row = l + 64 * q;
        if (row < BP && !((pivmask >> q) & 1)) {
          const double v = cabs1(sh.pn[row][ci]);
          const bool fin = (v == v && v <= 1.0e300);
          nf |= fin ? 0 : 1;
          const uint64_t kq = pivot_key(fin ? v : -1.0, row);
          u = kq > u ? kq : u;
        }
      }
      u = __ockl_wfred_max_u64(u);   // wave maximum through DPP row operations
      const bool col_bad = (u >> 7) <= 2 || __ballot(nf) != 0;   // zero or non-finite candidates
      const int pr = 127 - (int)(u & 127);
      if ((pr & 63) == l) pivmask |= 1u << (pr >> 6);
      const double2 p = sh.pn[pr][ci];
      const double2 prj = sh.pn[pr][pj];
      double2 pci[PM];
#pragma unroll
      for (int m = 0; m < PM; ++m) {
        const int i = pi0 + PSTEP * m;
        pci[m] = i < BP ? sh.pn[i][ci] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      const double2 pinv = cinv(p);
      const double2 rowv = cmul(prj, pinv);
#pragma unroll
      for (int m = 0; m < PM; ++m) {
        const int i = pi0 + PSTEP * m;
        if (i >= BP) continue;
        double2 nv;
        if (i == pr) {
          nv = (pj == ci) ? pinv : rowv;
        } else {
          const double2 f = pci[m];
          if (pj == ci) {
            const double2 q = cmul(f, pinv);
            nv = make_double2(-q.x, -q.y);
          } else {
            const double2 q = cmul(f, rowv);
            const double2 old = sh.pn[i][pj];
            nv = make_double2(old.x - q.x, old.y - q.y);
          }
        }
        sh.pn[i][pj] = nv;
      }
      if (t == 0) {
        sh.rowsel[16 * kt + ci] = pr;
        sh.slot[pr] = ci;
        if (col_bad) sh.bad = 1;
      }
      __syncthreads();
    }

    // 3. old pivot rows to LDS; zero them outside the panel columns
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (tr0 + r >= T || tc0 + c >= T) continue;
        const int j = 16 * (tc0 + c) + c_col(l);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * (tr0 + r) + c_row(l, v);
          const int s = sh.slot[i];
          if (s >= 0) {
            sh.rw[s][j] = make_double2(acc.re[r][c][v], acc.im[r][c][v]);
            acc.re[r][c][v] = 0.0;
            acc.im[r][c][v] = 0.0;
          }
        }
      }
    __syncthreads();

    // 4. trailing update  B[:, K'] = E_K B[:, K'] + P[:, K] * rows_K(B)[:, K'];  B[:, K] = P
    const int li = l & 15, lk = l >> 4;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      if (tr0 + r >= T) continue;
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (tc0 + c >= T) continue;
        if (tc0 + c == kt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double2 x = sh.pn[16 * (tr0 + r) + c_row(l, v)][c_col(l)];
            acc.re[r][c][v] = x.x;
            acc.im[r][c][v] = x.y;
          }
        } else {
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const double2 a = sh.pn[16 * (tr0 + r) + li][4 * ks + lk];
            const double2 b = sh.rw[4 * ks + lk][16 * (tc0 + c) + li];
            acc.re[r][c] = mfma(a.x, b.x, acc.re[r][c]);
            acc.re[r][c] = mfma(-a.y, b.y, acc.re[r][c]);
            acc.im[r][c] = mfma(a.x, b.y, acc.im[r][c]);
            acc.im[r][c] = mfma(a.y, b.x, acc.im[r][c]);
          }
        }
      }
    }
    __syncthreads();
    if (t < 16) sh.slot[sh.rowsel[16 * kt + t]] = -1;
    __syncthreads();
  }

  // 5. undo the pivoting while writing the inverse out
  for (int c = t; c < BP; c += NT) sh.rowdst[sh.rowsel[c]] = c;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    if (tr0 + r >= T) continue;
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      if (tc0 + c >= T) continue;
      const int j = 16 * (tc0 + c) + c_col(l);
      const int jd = sh.rowsel[j];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (tr0 + r) + c_row(l, v);
        g[(size_t)sh.rowdst[i] * BP + jd] = make_double2(acc.re[r][c][v], acc.im[r][c][v]);
      }
    }
  }
}

// Workgroup sum of one double per thread (deterministic order).
template <int NW>
__device__ __forceinline__ double wg_sum(double v, double* red /* LDS, >= NW */) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wv = wave_id();
  if (lane_id() == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) s += red[k];
  __syncthreads();
  return s;
}

// Workgroup maximum of one double per thread (every thread gets the result; NaN wins).
template <int NW>
__device__ __forceinline__ double wg_max(double v, double* red /* LDS, >= NW */) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = (o > v || o != o) ? o : v;
  }
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) m = (red[k] > m || red[k] != red[k]) ? red[k] : m;
  __syncthreads();
  return m;
}

// 1-norm condition number ||S||_1 ||g||_1 of a pivot S and its inverse g, both
// bp x bp row-major in global memory (the identity padding leaves both norms >= 1,
// so the value is never below the b x b block's).  Column sums of |s_rc| are split
// over all threads in row slices and combined through LDS scratch (at least
// 2 * NT doubles, free outside gj_invert).  Every thread gets the result.
template <int T, int NW>
__device__ __forceinline__ double kappa1(const double2* S, const double2* g, double* scr, double* red) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  constexpr int NS = NT / BP > 0 ? NT / BP : 1;        // row slices per column
  const int t = threadIdx.x;
  const int c = t % BP, s = t / BP;
  __syncthreads();
  if (s < NS) {
    double ps = 0.0, pg = 0.0;
    for (int r = s; r < BP; r += NS) {
      const double2 x = S[(size_t)r * BP + c];
      const double2 y = g[(size_t)r * BP + c];
      ps += sqrt(x.x * x.x + x.y * x.y);
      pg += sqrt(y.x * y.x + y.y * y.y);
    }
    scr[s * BP + c] = ps;
    scr[NS * BP + s * BP + c] = pg;
  }
  __syncthreads();
  double ns = 0.0, ng = 0.0;
  for (int cc = t; cc < BP; cc += NT) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < NS; ++k) {
      a += scr[k * BP + cc];
      b += scr[NS * BP + k * BP + cc];
    }
    ns = (a > ns || a != a) ? a : ns;
    ng = (b > ng || b != b) ? b : ng;
  }
  ns = wg_max<NW>(ns, red);
  ng = wg_max<NW>(ng, red);
  return ns * ng;
}

// T = Re Tr[Gamma_L R Gamma_R R^H] with Gamma = i (Sigma - Sigma^H), R = G_{0,l-1}
// (padded bp x bp, ld = bp, in global memory).  GamL, GamR, X1: bp x bp scratch.
// All threads call it; the result is returned to every thread.
template <int T, int NW>
__device__ __forceinline__ double transmission(Acc<T, NW>& acc, const double2* R, const double2* sL, const double2* sR,
                               int b, double2* GamL, double2* GamR, double2* X1, double* red) {
  constexpr int BP = 16 * T;
  constexpr int NT = 64 * NW;
  for (int idx = threadIdx.x; idx < BP * BP; idx += NT) {
    const int r = idx / BP, c = idx % BP;
    double2 gl = make_double2(0.0, 0.0), gr = make_double2(0.0, 0.0);
    if (r < b && c < b) {
      const double2 s1 = sL[(size_t)r * b + c], s2 = sL[(size_t)c * b + r];
      gl = make_double2(-(s1.y + s2.y), s1.x - s2.x);
      const double2 q1 = sR[(size_t)r * b + c], q2 = sR[(size_t)c * b + r];
      gr = make_double2(-(q1.y + q2.y), q1.x - q2.x);
    }
    GamL[idx] = gl;
    GamR[idx] = gr;
  }
  __syncthreads();
  acc_zero<T, NW>(acc);
  mma<T, NW>(acc, opnd(GamL, BP, BP, BP), opnd(R, BP, BP, BP), 1.0);
  store<T, NW>(acc, X1, BP, BP, BP);
  __syncthreads();
  acc_zero<T, NW>(acc);
  mma<T, NW>(acc, opnd(GamR, BP, BP, BP), opnd(R, BP, BP, BP, 1), 1.0);
  double part = 0.0;
  const int ln = lane_id();
  int tr0, tc0;
  tile_origin<T, NW>(tr0, tc0);
#pragma unroll
  for (int r = 0; r < Acc<T, NW>::RR; ++r)
#pragma unroll
    for (int c = 0; c < Acc<T, NW>::RC; ++c) {
      if (tr0 + r >= T || tc0 + c >= T) continue;
      const int jj = 16 * (tc0 + c) + c_col(ln);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int kk = 16 * (tr0 + r) + c_row(ln, v);
        const double2 x1 = X1[(size_t)jj * BP + kk];
        part += acc.re[r][c][v] * x1.x - acc.im[r][c][v] * x1.y;
      }
    }
  return wg_sum<NW>(part, red);
}

}  // namespace rgfk
