// FP64 inversion of the normal-equation matrix of one CP-ALS update, as a
// routine for one 256-thread workgroup: the matrix is gathered from the Gram
// partials of the two other factors and inverted by symmetric (LDL^T)
// elimination in Gauss-Jordan form.
#pragma once

#include "mtk_internal.h"

namespace mtk {

namespace fdev {

__device__ inline void tile_pair(int t, int& tr, int& ts) {
  int r = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  tr = r;
  ts = t - r * (r + 1) / 2;
}

}  // namespace fdev

// Lower triangle (with the diagonal) of V = G_a * G_b into A (row stride
// ld), padded to Rp x Rp with an identity block.  Entry (tile, k) of a
// 16 x 16 tile of G is the block-ordered sum of its partials.  Each round a
// thread loads every partial of U entries (NQ >= partial count, loads past
// it predicated off) before summing, so a round costs one memory latency.
// NQ <= kGramBlocksMax.
template <int NQ, int U>
__device__ inline void gather_v_nq(const FactorArgs& f, int Rp, double* A, int ld) {
  using fdev::tile_pair;
  const int R = f.R, na = f.na, nb = f.nb;
  const double* __restrict__ Pa = f.pa;
  const double* __restrict__ Pb = f.pb;
  const int nbk = Rp >> 4;
  const int tot = nbk * (nbk + 1) / 2 * 256;
  for (int e0 = threadIdx.x; e0 < tot; e0 += U * 256) {
    double va[U][NQ], vb[U][NQ];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 256;
      const size_t o = e < tot ? (size_t)(e >> 8) * kGramBlocksMax * 256 + (e & 255) : 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        va[u][q] = (e < tot && q < na) ? Pa[o + q * 256] : 0.0;
        vb[u][q] = (e < tot && q < nb) ? Pb[o + q * 256] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 256;
      if (e >= tot) continue;
      double ga = 0.0, gb = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) { ga += va[u][q]; gb += vb[u][q]; }
      int ti, tj;
      tile_pair(e >> 8, ti, tj);
      const int i = ti * 16 + ((e & 255) >> 4), j = tj * 16 + (e & 15);
      if (j <= i) A[i * ld + j] = (i < R && j < R) ? ga * gb : (i == j ? 1.0 : 0.0);
    }
  }
}

// All threads of the workgroup take part; the caller synchronises.  LEAN:
// one entry per round (fewer registers, for a workgroup that rides along in
// another kernel).
template <bool LEAN>
__device__ inline void gather_v(const FactorArgs& f, int Rp, double* A, int ld) {
  const int nq = f.na > f.nb ? f.na : f.nb;
  if constexpr (LEAN) {
    gather_v_nq<kGramBlocksMax, 1>(f, Rp, A, ld);
  } else {
    if (nq <= 4) gather_v_nq<4, 8>(f, Rp, A, ld);
    else if (nq <= 8) gather_v_nq<8, 4>(f, Rp, A, ld);
    else gather_v_nq<kGramBlocksMax, 2>(f, Rp, A, ld);
  }
}

// Inversion of V in place (any R <= 128; Rp = 16*B) by symmetric
// elimination: step k is the LDL^T (square-root-free Cholesky) step with
// pivot p = A(k,k) -- its Schur-complement update of the trailing block is
// the one of the factorisation -- done in Gauss-Jordan form, which also
// clears column k above the diagonal, so that after the last step A holds
// V^{-1}.  V is SPD, so there is no pivoting, and a pivot <= 0 (or NaN)
// means V is not SPD.  One workgroup of 256 threads as a 16 x 16 grid,
// thread (ti, tj) holding the B x B block of rows ti*B.., columns tj*B.. in
// registers.  Step k maps
//   A(k,k) <- 1/p,  A(k,j) <- A(k,j)/p,  A(i,k) <- -A(i,k)/p,
//   A(i,j) <- A(i,j) - A(i,k) A(k,j) / p          (i, j != k),
// after which A holds V^{-1}.  The owners of row k and column k publish
// them (start-of-step values) in a double-buffered LDS slot, so each step
// needs one barrier.  A slot holds element ti*B + u at u*16 + ti, so the 16
// column blocks of a wave read consecutive doubles (no bank conflicts).
// Padding rows/columns (identity) pass through.
template <int B, bool LEAN = false>
__device__ inline void factor_gj(const FactorArgs& f, double* lds) {
  constexpr int RP = 16 * B;
  constexpr int LD = RP + 1;
  const int R = f.R;
  const int tid = threadIdx.x;
  const int ti = tid >> 4, tj = tid & 15;
  const int i0 = ti * B, j0 = tj * B;
  double* A = lds;                                  // RP x LD, lower triangle of V
  double* bc = lds + RP * LD;                       // [buffer][column k | row k][RP]
  gather_v<LEAN>(f, RP, A, LD);
  __syncthreads();
  double a[B][B];
#pragma unroll
  for (int u = 0; u < B; ++u)
#pragma unroll
    for (int v = 0; v < B; ++v) {
      const int i = i0 + u, j = j0 + v;
      a[u][v] = i >= j ? A[i * LD + j] : A[j * LD + i];
    }
  bool bad = false;
  for (int kb = 0; kb < 16; ++kb) {
#pragma unroll
    for (int kk = 0; kk < B; ++kk) {
      const int k = kb * B + kk;
      const int buf = k & 1;
      if (tj == kb) {
#pragma unroll
        for (int u = 0; u < B; ++u) bc[(2 * buf) * RP + u * 16 + ti] = a[u][kk];
      }
      if (ti == kb) {
#pragma unroll
        for (int v = 0; v < B; ++v) bc[(2 * buf + 1) * RP + v * 16 + tj] = a[kk][v];
      }
      __syncthreads();
      const double p = bc[(2 * buf) * RP + kk * 16 + kb];
      bad |= !(p > 0.0);                           // uniform: every thread reads the same p
      const double r = 1.0 / p;
      double ci[B], rj[B];
#pragma unroll
      for (int u = 0; u < B; ++u) ci[u] = bc[(2 * buf) * RP + u * 16 + ti] * r;
#pragma unroll
      for (int v = 0; v < B; ++v) rj[v] = bc[(2 * buf + 1) * RP + v * 16 + tj];
#pragma unroll
      for (int u = 0; u < B; ++u)
#pragma unroll
        for (int v = 0; v < B; ++v) a[u][v] = fma(-ci[u], rj[v], a[u][v]);
      // Row k and column k (this thread's parts of them) take their own forms.
      if (ti == kb) {
#pragma unroll
        for (int v = 0; v < B; ++v) a[kk][v] = rj[v] * r;
      }
      if (tj == kb) {
#pragma unroll
        for (int u = 0; u < B; ++u) a[u][kk] = -ci[u];
        if (ti == kb) a[kk][kk] = r;
      }
    }
  }
  if (bad) {
    if (tid == 0) atomicOr(f.status, kStatusNotSPD);
    return;
  }
#pragma unroll
  for (int u = 0; u < B; ++u)
#pragma unroll
    for (int v = 0; v < B; ++v) {
      const int i = i0 + u, j = j0 + v;
      if (i < R && j < R) f.vinv[(int64_t)i * R + j] = a[u][v];
    }
}

// LDS of factor_gj (bytes): the gathered lower triangle and the two
// broadcast slots.
__host__ __device__ inline size_t factor_gj_lds_bytes(int R) {
  const size_t Rp = (size_t)((R + 15) & ~15);
  return (Rp * (Rp + 1) + 4 * Rp) * sizeof(double);
}

}  // namespace mtk
