// FP64 factorisation of the normal-equation matrix of one CP-ALS update, as
// routines for one 256-thread workgroup: the blocked form for any R <= 128
// and a register-resident form for R <= 32.
#pragma once

#include "mtk_internal.h"

namespace mtk {

// LDS the factorisation needs (bytes).
__host__ __device__ inline size_t factor_lds_bytes(int R) {
  const size_t Rp = (size_t)((R + 15) & ~15);
  return (Rp * (Rp + 1) + (Rp - 16) * 17 + Rp) * sizeof(double);
}

namespace fdev {

__device__ inline void tile_pair(int t, int& tr, int& ts) {
  int r = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  tr = r;
  ts = t - r * (r + 1) / 2;
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

}  // namespace fdev

// Lower triangle (with the diagonal) of V = G_a * G_b into A (row stride
// ld), padded to Rp x Rp with an identity block.  Entry (tile, k) of a
// 16 x 16 tile of G is the block-ordered sum of its partials.  All threads
// of the workgroup take part; the caller synchronises.
__device__ inline void gather_v(const FactorArgs& f, int Rp, double* A, int ld) {
  using fdev::tile_pair;
  const int R = f.R, na = f.na, nb = f.nb;
  const double* __restrict__ Pa = f.pa;
  const double* __restrict__ Pb = f.pb;
  const int tid = threadIdx.x;
  const int nbk = Rp >> 4;
  // With at most 8 partials per factor, the loads of 4 entries are all
  // issued before any sum.
  {
    const int tot = nbk * (nbk + 1) / 2 * 256;
    auto put = [&](int e, double v) {
      int ti, tj;
      tile_pair(e >> 8, ti, tj);
      const int i = ti * 16 + ((e & 255) >> 4), j = tj * 16 + (e & 15);
      if (j <= i) A[i * ld + j] = (i < R && j < R) ? v : (i == j ? 1.0 : 0.0);
    };
    if (na <= 8 && nb <= 8) {
      for (int e0 = tid; e0 < tot; e0 += 4 * 256) {
        double va[4][8], vb[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * 256;
          const size_t o = e < tot ? (size_t)(e >> 8) * kGramBlocksMax * 256 + (e & 255) : 0;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            va[u][q] = (e < tot && q < na) ? Pa[o + q * 256] : 0.0;
            vb[u][q] = (e < tot && q < nb) ? Pb[o + q * 256] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * 256;
          double ga = 0.0, gb = 0.0;
#pragma unroll
          for (int q = 0; q < 8; ++q) { ga += va[u][q]; gb += vb[u][q]; }
          if (e < tot) put(e, ga * gb);
        }
      }
    } else {
      for (int e = tid; e < tot; e += 256) {
        const size_t o = (size_t)(e >> 8) * kGramBlocksMax * 256 + (e & 255);
        double ga = 0.0, gb = 0.0;
        for (int q = 0; q < na; ++q) ga += Pa[o + q * 256];
        for (int q = 0; q < nb; ++q) gb += Pb[o + q * 256];
        put(e, ga * gb);
      }
    }
  }
}

// One workgroup (256 threads; `lds` holds factor_lds_bytes(R)):
// V = G_a * G_b (lower triangle, from the Gram partials of the two factors),
// V = L L^T, W = L^{-1}, and V^{-1} = W^T W, written as a full R x R
// row-major matrix.
//
// V is padded to Rp = 16*ceil(R/16) with an identity block.  Cholesky is
// right-looking in 16-column panels: wave 0 factors the diagonal block with
// its rows in lanes 0..15 and the pivots broadcast by readlane (no LDS
// round trips), all threads solve the panel rows against it, and the
// trailing lower triangle is updated in 4 x 4 register tiles.  The inverse
// is formed in place from the right: the diagonal blocks are inverted in
// parallel (16 lanes per block, one column per lane), then for each block
// column J from the last but one to the first, W(below, J) =
// -W(below, below) L(below, J) W(J, J).  V^{-1} = W^T W is summed in 4 x 4
// register tiles.  Every sum has a fixed order.
__device__ inline void factor_v_inv(const FactorArgs& f, double* lds) {
  using fdev::readlane_f64;
  using fdev::tile_pair;
  using fdev::wave_sync;
  const int R = f.R, na = f.na, nb = f.nb;
  const double* __restrict__ Pa = f.pa;
  const double* __restrict__ Pb = f.pb;
  double* __restrict__ Vinv = f.vinv;
  int* __restrict__ status = f.status;
  const int Rp = (R + 15) & ~15;
  const int nbk = Rp >> 4;
  const int ld = Rp + 1;
  double* A = lds;                                   // Rp x ld
  double* Xs = A + (size_t)Rp * ld;                  // (Rp - 16) x 17
  double* dinv = Xs + (size_t)(Rp - 16) * 17;        // Rp
  __shared__ int failed;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) failed = 0;
  gather_v(f, Rp, A, ld);
  __syncthreads();

  for (int pb = 0; pb < nbk; ++pb) {
    const int p0 = pb * 16;
    if (wave == 0) {
      // Rows p0..p0+15 in lanes 0..15 (repeated in the other lanes).  Step
      // jj updates with the unscaled column: L(i,jj) L(k,jj) = a(i) a(k) / piv,
      // so the next pivot depends on 1/piv only; sqrt(piv) and the column
      // scaling are off that chain.
      const int ri = lane & 15;
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = u <= ri ? A[(p0 + ri) * ld + p0 + u] : 0.0;
      bool bad = false;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        // A pivot <= 0 or NaN (uniform across the wave) marks the matrix
        // as not SPD; the steps still run (on NaNs) so the loop unrolls.
        const double piv = readlane_f64(a[jj], jj);
        double ck[16];
#pragma unroll
        for (int kk = jj + 1; kk < 16; ++kk) ck[kk] = readlane_f64(a[jj], kk);
        bad |= !(piv > 0.0);
        const double rp = 1.0 / piv;
        const double u = a[jj] * rp;
        // Entries above the diagonal (ri < kk) take the update too; they
        // are never read, which keeps the step free of lane masks.
#pragma unroll
        for (int kk = jj + 1; kk < 16; ++kk) a[kk] = fma(-u, ck[kk], a[kk]);
        const double sq = sqrt(piv);
        const double inv = 1.0 / sq;
        if (ri > jj) a[jj] *= inv;
        else if (ri == jj) a[jj] = sq;
        if (lane == 0) dinv[p0 + jj] = inv;
      }
      if (bad) {
        if (lane == 0) failed = 1;
      } else if (lane < 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (u <= ri) A[(p0 + ri) * ld + p0 + u] = a[u];
      }
    }
    __syncthreads();
    if (failed) {
      if (tid == 0) atomicOr(status, kStatusNotSPD);
      return;                                        // uniform after the barrier
    }
    const int base = p0 + 16;
    if (base >= Rp) break;
    // Panel rows: L21(i,:) = A21(i,:) L11^{-T} by substitution.
    for (int i = base + tid; i < Rp; i += 256) {
      double r[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) r[jj] = A[i * ld + p0 + jj];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        r[jj] *= dinv[p0 + jj];
#pragma unroll
        for (int kk = jj + 1; kk < 16; ++kk) r[kk] = fma(-r[jj], A[(p0 + kk) * ld + p0 + jj], r[kk]);
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) A[i * ld + p0 + jj] = r[jj];
    }
    __syncthreads();
    // Trailing lower triangle: A22(i,k) -= L21(i,:) . L21(k,:), 4 x 4 tiles.
    const int nt4 = (Rp - base) >> 2;
    const int ntile = nt4 * (nt4 + 1) / 2;
    for (int t = tid; t < ntile; t += 256) {
      int ti, tk;
      tile_pair(t, ti, tk);
      const int i0 = base + 4 * ti, k0 = base + 4 * tk;
      double c[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) c[u][v] = 0.0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { x[u] = A[(i0 + u) * ld + p0 + jj]; y[u] = A[(k0 + u) * ld + p0 + jj]; }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) c[u][v] = fma(x[u], y[v], c[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (k0 + v <= i0 + u) A[(i0 + u) * ld + k0 + v] -= c[u][v];
    }
    __syncthreads();
  }

  // Diagonal blocks: W(J,J) = L(J,J)^{-1}; lane k of a 16-lane group forms
  // column k by forward substitution, then the group overwrites the block.
  for (int J = tid >> 4; J < nbk; J += 16) {
    const int p0 = J * 16, k = tid & 15;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double s = i == k ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < i; ++m) s = fma(-A[(p0 + i) * ld + p0 + m], x[m], s);
      x[i] = i >= k ? s * dinv[p0 + i] : 0.0;
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i >= k) A[(p0 + i) * ld + p0 + k] = x[i];
  }
  __syncthreads();
  // Off-diagonal block columns from the right.
  for (int J = nbk - 2; J >= 0; --J) {
    const int p0 = J * 16, b0 = p0 + 16, nr = Rp - b0;
    // X(i, c) = sum_{k=b0..i} W(i,k) L(k, p0+c): 2 rows x 4 columns per thread.
    for (int t = tid; t < (nr >> 1) * 4; t += 256) {
      const int i0 = b0 + 2 * (t >> 2), c0 = 4 * (t & 3);
      double x0[4] = {0.0, 0.0, 0.0, 0.0}, x1[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int k = b0; k <= i0; ++k) {
        const double w0 = A[i0 * ld + k], w1 = A[(i0 + 1) * ld + k];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double l = A[k * ld + p0 + c0 + v];
          x0[v] = fma(w0, l, x0[v]);
          x1[v] = fma(w1, l, x1[v]);
        }
      }
      const double w11 = A[(i0 + 1) * ld + i0 + 1];
#pragma unroll
      for (int v = 0; v < 4; ++v) x1[v] = fma(w11, A[(i0 + 1) * ld + p0 + c0 + v], x1[v]);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Xs[(i0 - b0) * 17 + c0 + v] = x0[v];
        Xs[(i0 + 1 - b0) * 17 + c0 + v] = x1[v];
      }
    }
    __syncthreads();
    // W(i, p0+c) = -sum_{m=c..15} X(i,m) W(p0+m, p0+c).
    for (int e = tid; e < nr * 16; e += 256) {
      const int i = b0 + (e >> 4), c = e & 15;
      double s = 0.0;
#pragma unroll 4
      for (int m = c; m < 16; ++m) s = fma(Xs[(i - b0) * 17 + m], A[(p0 + m) * ld + p0 + c], s);
      A[i * ld + p0 + c] = -s;
    }
    __syncthreads();
  }
  // Zero the upper triangle, then V^{-1}(i,j) = sum_{k >= i} W(k,i) W(k,j)
  // for i >= j, 4 x 4 tiles of the lower triangle, written to both halves.
  for (int i = wave; i < Rp; i += 4)
    for (int j = i + 1 + lane; j < Rp; j += 64) A[i * ld + j] = 0.0;
  __syncthreads();
  {
    const int nt4 = Rp >> 2;
    const int ntile = nt4 * (nt4 + 1) / 2;
    for (int t = tid; t < ntile; t += 256) {
      int ti, tj;
      tile_pair(t, ti, tj);
      const int i0 = 4 * ti, j0 = 4 * tj;
      double c[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) c[u][v] = 0.0;
#pragma unroll 4
      for (int k = i0; k < Rp; ++k) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { x[u] = A[k * ld + i0 + u]; y[u] = A[k * ld + j0 + u]; }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) c[u][v] = fma(x[u], y[v], c[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + u, j = j0 + v;
          if (i < R && j <= i) {
            Vinv[(int64_t)i * R + j] = c[u][v];
            Vinv[(int64_t)j * R + i] = c[u][v];
          }
        }
    }
  }
}

// R <= RP (16 or 32), one workgroup: after the gather, wave 0 holds row r of
// V in lane r (registers) and factors it unblocked, each pivot broadcast by
// readlane; the update at pivot j uses the unscaled column (L(i,j) L(k,j) =
// a(i) a(k) / a(j,j)), so the chain from one pivot to the next is one
// reciprocal, one multiply and one fma.  Lane k then forms column k of
// W = L^{-1} by forward substitution on the broadcast rows of L, and all
// threads form V^{-1} = W^T W from W in LDS.
template <int RP>
__device__ inline void factor_v_inv_small(const FactorArgs& f) {
  using fdev::readlane_f64;
  constexpr int LD = RP + 1;
  __shared__ double A[RP * LD];
  __shared__ double Wl[RP * LD];
  __shared__ int failed;
  const int R = f.R;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) failed = 0;
  gather_v(f, RP, A, LD);
  __syncthreads();
  if (wave == 0) {
    const int ri = lane % RP;                      // lanes >= RP repeat rows
    double a[RP];
#pragma unroll
    for (int u = 0; u < RP; ++u) a[u] = u <= ri ? A[ri * LD + u] : 0.0;
    bool bad = false;
    double dl = 1.0;                               // 1 / L(ri, ri)
#pragma unroll
    for (int jj = 0; jj < RP; ++jj) {
      // A pivot <= 0 or NaN (uniform across the wave) marks V not SPD; the
      // steps still run so that the loop stays straight-line code.
      const double piv = readlane_f64(a[jj], jj);
      bad |= !(piv > 0.0);
      const double u = a[jj] * (1.0 / piv);
      // Entries above the diagonal take the update too; they are never read.
#pragma unroll
      for (int kk = jj + 1; kk < RP; ++kk) a[kk] = fma(-u, readlane_f64(a[jj], kk), a[kk]);
      const double sq = sqrt(piv);
      const double inv = 1.0 / sq;
      if (ri > jj) a[jj] *= inv;
      else if (ri == jj) { a[jj] = sq; dl = inv; }
    }
    double x[RP];                                  // x[i] = W(i, ri)
#pragma unroll
    for (int i = 0; i < RP; ++i) {
      double s = i == ri ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < i; ++m) s = fma(-readlane_f64(a[m], i), x[m], s);
      x[i] = i >= ri ? s * readlane_f64(dl, i) : 0.0;
    }
    if (bad) {
      if (lane == 0) failed = 1;
    } else if (lane < RP) {
#pragma unroll
      for (int i = 0; i < RP; ++i) Wl[i * LD + lane] = x[i];
    }
  }
  __syncthreads();
  if (failed) {
    if (tid == 0) atomicOr(f.status, kStatusNotSPD);
    return;
  }
  for (int e = tid; e < R * R; e += 256) {
    const int j = e / R, k = e - j * R;
    double s = 0.0;
    for (int i = j > k ? j : k; i < RP; ++i) s = fma(Wl[i * LD + j], Wl[i * LD + k], s);
    f.vinv[e] = s;
  }
}

}  // namespace mtk
