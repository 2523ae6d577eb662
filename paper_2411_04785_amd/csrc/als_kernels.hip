// FP64 normal-equation update of one CP factor, and the CP fit.
//
// Given the FP32 factors and the FP32 MTTKRP M (n x R) of mode `mode`:
//   V = G_a * G_b (Hadamard), G_m = A_m^T A_m over the two other modes (FP64)
//   V = L L^T (Cholesky, FP64; a pivot <= 0 sets the sticky NOT-SPD status)
//   F = M V^{-1} by two triangular solves per row, G L^T = M and F L = G (FP64)
//   lambda_r = ||F(:,r)||_2, factor = F(:,r) / lambda_r cast to FP32.
// Every reduction runs in a fixed order, so the update is deterministic.

#include "mtk_internal.h"

#include <algorithm>

namespace mtk {
namespace {

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Rows summed by one Gram partial: at least 128, and at most 64 partials.
__host__ __device__ inline int64_t gram_rows(int64_t n) { const int64_t r = cdiv(n, 64); return r > 128 ? r : 128; }
// Rows handled by one workgroup of the apply / normalise kernels (<= 256 groups).
__host__ __device__ inline int64_t apply_rows(int64_t n) { const int64_t r = cdiv(n, 256); return r > 64 ? r : 64; }

// part[f][rb][r][s] = sum over rows i of block rb of F_f(i,r) F_f(i,s), FP64,
// for the two factors f = 0, 1.  Block (16x16 tile, rb, f); 256 threads.
__global__ __launch_bounds__(256) void gram_partial_kernel(const float* __restrict__ F0, int64_t n0,
                                                           const float* __restrict__ F1, int64_t n1, int R,
                                                           int tiles_1d, int nrb_max, double* __restrict__ part) {
  const int f = blockIdx.z;
  const float* F = f ? F1 : F0;
  const int64_t n = f ? n1 : n0;
  const int64_t rows = gram_rows(n);
  const int rb = blockIdx.y;
  const int64_t i0 = (int64_t)rb * rows;
  if (i0 >= n) return;
  const int64_t i1 = min(n, i0 + rows);
  const int tile = blockIdx.x;
  const int tr = tile / tiles_1d, ts = tile % tiles_1d;
  const int r = tr * 16 + (threadIdx.x >> 4);
  const int s = ts * 16 + (threadIdx.x & 15);
  __shared__ float rows_r[64][17];
  __shared__ float rows_s[64][17];
  double acc = 0.0;
  for (int64_t c0 = i0; c0 < i1; c0 += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int ii = e >> 4, cc = e & 15;
      const int64_t i = c0 + ii;
      const int cr = tr * 16 + cc, cs = ts * 16 + cc;
      rows_r[ii][cc] = (i < i1 && cr < R) ? F[i * R + cr] : 0.f;
      rows_s[ii][cc] = (i < i1 && cs < R) ? F[i * R + cs] : 0.f;
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(64, i1 - c0);
    for (int ii = 0; ii < cnt; ++ii)
      acc = fma((double)rows_r[ii][threadIdx.x >> 4], (double)rows_s[ii][threadIdx.x & 15], acc);
    __syncthreads();
  }
  if (r < R && s < R) part[(((int64_t)f * nrb_max + rb) * R + r) * R + s] = acc;
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup: V = G_0 * G_1 (Hadamard of the summed Gram partials) and
// its Cholesky factor V = L L^T, FP64 in LDS.  Writes L (Rp x Rp, lower,
// zero above the diagonal) to Lg and 1 / L(r,r) to dinv.  A pivot <= 0 (or
// NaN) sets kStatusNotSPD and stops.
//
// V is padded to Rp = 16*ceil(R/16) with an identity block (whose factor is
// an identity block).  Blocked right-looking with 16 x 16 blocks: wave 0
// factors the diagonal block in registers (16 steps, lane shuffles), every thread then
// solves whole rows of the panel (L21 = A21 L11^{-T}), and the trailing lower
// triangle is updated (A22 -= L21 L21^T) in 2 x 2 register tiles.  Every sum
// runs in a fixed order: the factor is deterministic.
__global__ __launch_bounds__(256) void cholesky_kernel(const double* __restrict__ part, int nr0, int nr1,
                                                       int nrb_max, int R, double* __restrict__ Lg,
                                                       double* __restrict__ dinv, int* __restrict__ status) {
  extern __shared__ double lds[];
  const int Rp = (R + 15) & ~15;
  const int nb = Rp / 16;
  const int ld = Rp + 1;
  double* S = lds;                                   // Rp x ld
  __shared__ int failed;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t RR = (int64_t)R * R;
  if (tid == 0) failed = 0;
  // V = (sum of Gram partials of factor a) * (same for factor b), padded.
  // Entries are gathered 8 per thread at a time with all their loads in
  // flight together (the adds keep partial-index order).
  {
    const int total = Rp * Rp;
    for (int e0 = tid; e0 < total; e0 += 8 * 256) {
      double va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) { va[u] = 0.0; vb[u] = 0.0; }
      for (int q = 0; q < nr0; ++q) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * 256;
          const int i = e / Rp, j = e - i * Rp;
          if (e < total && i < R && j < R) va[u] += part[(int64_t)q * RR + (int64_t)i * R + j];
        }
      }
      for (int q = 0; q < nr1; ++q) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * 256;
          const int i = e / Rp, j = e - i * Rp;
          if (e < total && i < R && j < R) vb[u] += part[((int64_t)nrb_max + q) * RR + (int64_t)i * R + j];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        if (e < total) {
          const int i = e / Rp, j = e - i * Rp;
          S[i * ld + j] = (i < R && j < R) ? va[u] * vb[u] : (i == j ? 1.0 : 0.0);
        }
      }
    }
  }
  __syncthreads();

  for (int pb = 0; pb < nb; ++pb) {
    const int p0 = pb * 16;
    if (wave == 0) {
      // Diagonal block in registers: lane l holds row ri = l/4, columns
      // kq..kq+3 (kq = 4*(l%4)).  Step jj broadcasts the pivot with a
      // readlane, the row's L(ri,jj) within its quad, and L(k,jj) of the
      // lane's four columns with lane shuffles; no LDS round trips.
      const int ri = lane >> 2, kq = (lane & 3) * 4;
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = S[(p0 + ri) * ld + p0 + kq + u];
      bool bad = false;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int own = jj * 4 + (jj >> 2);              // lane holding (jj, jj)
        const double d = __shfl(a[jj & 3], own, 64);
        if (!(d > 0.0)) { bad = true; break; }           // uniform across the wave
        const double ljj = sqrt(d);
        const double inv = 1.0 / ljj;
        if ((lane & 3) == (jj >> 2)) {                    // lanes holding column jj
          if (ri == jj) a[jj & 3] = ljj;
          else if (ri > jj) a[jj & 3] *= inv;
        }
        const double lij = __shfl(a[jj & 3], (lane & ~3) | (jj >> 2), 64);
        double lkj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) lkj[u] = __shfl(a[jj & 3], (kq + u) * 4 + (jj >> 2), 64);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = kq + u;
          if (k > jj && k <= ri) a[u] -= lij * lkj[u];
        }
      }
      if (bad) {
        if (lane == 0) failed = 1;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) S[(p0 + ri) * ld + p0 + kq + u] = a[u];
      }
    }
    __syncthreads();
    if (failed) {
      if (tid == 0) atomicOr(status, kStatusNotSPD);
      return;                                        // uniform after the barrier
    }
    const int base = p0 + 16;
    if (base >= Rp) break;
    // Panel rows: L21(i,:) = A21(i,:) L11^{-T}.
    for (int i = base + tid; i < Rp; i += 256) {
      double* row = &S[i * ld + p0];
      double r[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) r[jj] = row[jj];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        double v = r[jj];
#pragma unroll
        for (int kk = 0; kk < jj; ++kk) v -= r[kk] * S[(p0 + jj) * ld + p0 + kk];
        r[jj] = v / S[(p0 + jj) * ld + p0 + jj];
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) row[jj] = r[jj];
    }
    __syncthreads();
    // Trailing lower triangle in 2 x 2 tiles: A22(i,k) -= L21(i,:) . L21(k,:).
    const int h = base >> 1, hp = Rp >> 1;
    for (int i2 = h + (tid >> 4); i2 < hp; i2 += 16) {
      for (int k2 = h + (tid & 15); k2 <= i2; k2 += 16) {
        const double* a0 = &S[(2 * i2) * ld + p0];
        const double* a1 = a0 + ld;
        const double* b0 = &S[(2 * k2) * ld + p0];
        const double* b1 = b0 + ld;
        double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const double x0 = a0[kk], x1 = a1[kk], y0 = b0[kk], y1 = b1[kk];
          c00 = fma(x0, y0, c00); c01 = fma(x0, y1, c01);
          c10 = fma(x1, y0, c10); c11 = fma(x1, y1, c11);
        }
        S[(2 * i2) * ld + 2 * k2] -= c00;
        if (k2 < i2) S[(2 * i2) * ld + 2 * k2 + 1] -= c01;
        S[(2 * i2 + 1) * ld + 2 * k2] -= c10;
        S[(2 * i2 + 1) * ld + 2 * k2 + 1] -= c11;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < Rp * Rp; e += 256) {
    const int i = e / Rp, j = e % Rp;
    Lg[e] = j <= i ? S[i * ld + j] : 0.0;
  }
  for (int i = tid; i < Rp; i += 256) dinv[i] = 1.0 / S[i * ld + i];
}

// F = M V^{-1} with V = L L^T for 16 rows per workgroup: forward solve
// G L^T = M, then back solve F L = G, FP64.  L (Rp x Rp) is staged in LDS.
// Each wave owns 4 rows and each row 16 lanes; rows never interact, so the
// waves only synchronise within themselves.  Blocked by 16 columns: a
// 16-step substitution inside the block, then one update of the remaining
// columns.  Also writes the workgroup's column sums of F^2 (fixed order).
__global__ __launch_bounds__(256) void trsm_rows_kernel(const float* __restrict__ M, int64_t n, int R,
                                                        const double* __restrict__ Lg,
                                                        const double* __restrict__ dinv,
                                                        const int* __restrict__ status, double* __restrict__ F,
                                                        double* __restrict__ colsq) {
  if (*status & kStatusNotSPD) return;
  extern __shared__ double lds[];
  const int Rp = (R + 15) & ~15;
  const int nb = Rp / 16;
  const int ldL = Rp + 1, ldY = Rp + 1;
  double* L = lds;                                   // Rp x ldL
  double* Y = L + (size_t)Rp * ldL;                  // 16 x ldY
  double* di = Y + 16 * ldY;                         // Rp
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < Rp * Rp; e += 256) L[(e / Rp) * ldL + (e % Rp)] = Lg[e];
  for (int e = tid; e < Rp; e += 256) di[e] = dinv[e];
  const int64_t q0 = (int64_t)blockIdx.x * 16;
  for (int e = tid; e < 16 * Rp; e += 256) {
    const int rr = e / Rp, c = e % Rp;
    const int64_t q = q0 + rr;
    Y[rr * ldY + c] = (q < n && c < R) ? (double)M[q * R + c] : 0.0;
  }
  __syncthreads();
  const int row = wave * 4 + (lane >> 4);            // row of this lane inside the block
  const int c = lane & 15;
  double* y = Y + row * ldY;
  // Forward: G(q,r) = (M(q,r) - sum_{s<r} L(r,s) G(q,s)) / L(r,r).
  for (int b = 0; b < nb; ++b) {
    const int p0 = b * 16;
    for (int jj = 0; jj < 16; ++jj) {
      if (c == jj) y[p0 + jj] *= di[p0 + jj];
      wave_sync();
      if (c > jj) y[p0 + c] -= y[p0 + jj] * L[(p0 + c) * ldL + p0 + jj];
      wave_sync();
    }
    for (int t = p0 + 16 + c; t < Rp; t += 16) {
      double acc = 0.0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) acc = fma(y[p0 + jj], L[t * ldL + p0 + jj], acc);
      y[t] -= acc;
    }
    wave_sync();
  }
  // Back: F(q,t) = (G(q,t) - sum_{r>t} F(q,r) L(r,t)) / L(t,t).
  for (int b = nb - 1; b >= 0; --b) {
    const int p0 = b * 16;
    for (int jj = 15; jj >= 0; --jj) {
      if (c == jj) y[p0 + jj] *= di[p0 + jj];
      wave_sync();
      if (c < jj) y[p0 + c] -= y[p0 + jj] * L[(p0 + jj) * ldL + p0 + c];
      wave_sync();
    }
    for (int t = c; t < p0; t += 16) {
      double acc = 0.0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) acc = fma(y[p0 + jj], L[(p0 + jj) * ldL + t], acc);
      y[t] -= acc;
    }
    wave_sync();
  }
  __syncthreads();
  for (int e = tid; e < 16 * R; e += 256) {
    const int rr = e / R, cc = e % R;
    const int64_t q = q0 + rr;
    if (q < n) F[q * R + cc] = Y[rr * ldY + cc];
  }
  for (int cc = tid; cc < R; cc += 256) {
    double sacc = 0.0;
    for (int rr = 0; rr < 16; ++rr) {
      const double v = (q0 + rr < n) ? Y[rr * ldY + cc] : 0.0;
      sacc = fma(v, v, sacc);
    }
    colsq[(int64_t)blockIdx.x * R + cc] = sacc;
  }
}

// lambda_c = sqrt(sum over blocks of colsq) (fixed order, recomputed by every
// workgroup), factor = F / lambda cast to FP32 (zero columns left unscaled).
__global__ __launch_bounds__(256) void normalize_kernel(const double* __restrict__ F, int64_t n, int R,
                                                        const double* __restrict__ colsq, int nblk,
                                                        const int* __restrict__ status, double* __restrict__ lam,
                                                        float* __restrict__ out) {
  if (*status & kStatusNotSPD) return;
  __shared__ double l[kMaxRank];
  if (threadIdx.x < R) {
    double t = 0.0;
#pragma unroll 8
    for (int b = 0; b < nblk; ++b) t += colsq[(int64_t)b * R + threadIdx.x];
    l[threadIdx.x] = sqrt(t);
    if (blockIdx.x == 0) lam[threadIdx.x] = l[threadIdx.x];
  }
  __syncthreads();
  const int64_t rows = apply_rows(n);
  const int64_t e0 = (int64_t)blockIdx.x * rows * R;
  const int64_t e1 = min(n * R, e0 + rows * R);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double lc = l[e % R];
    out[e] = (float)(lc > 0.0 ? F[e] / lc : F[e]);
  }
}

}  // namespace

size_t solve_ws_bytes(int64_t maxdim, int R) {
  const int64_t nrb = 64;
  const size_t Rp = (size_t)((R + 15) & ~15);
  const int64_t md = std::max<int64_t>(maxdim, 1);
  size_t b = 0;
  b += 2 * (size_t)nrb * R * R * sizeof(double);     // Gram partials of the two other factors
  b += Rp * Rp * sizeof(double);                      // L
  b += Rp * sizeof(double);                           // 1 / diag(L)
  b += (size_t)md * R * sizeof(double);               // F
  b += (size_t)cdiv(md, 16) * R * sizeof(double);     // column sums of squares per 16 rows
  return b + 6 * 256;
}

static inline char* take(char*& p, size_t bytes) {
  char* r = p;
  p += (bytes + 255) & ~(size_t)255;
  return r;
}

namespace {

// Workspace carve-up shared by the two halves of the update.
struct SolveWs {
  double* part;
  double* Lg;
  double* dinv;
  double* F;
  double* colsq;
  int nra, nrb, nrb_max, ntr, nblk;
};

SolveWs solve_ws(const int64_t dims[3], int R, int mode, void* ws) {
  const int oa = mode == 0 ? 1 : 0;
  const int ob = mode == 2 ? 1 : 2;
  const int64_t n = dims[mode];
  SolveWs w{};
  w.nra = (int)cdiv(dims[oa], gram_rows(dims[oa]));
  w.nrb = (int)cdiv(dims[ob], gram_rows(dims[ob]));
  w.nrb_max = std::max(w.nra, w.nrb);
  w.ntr = (int)cdiv(n, 16);
  w.nblk = (int)cdiv(n, apply_rows(n));
  const size_t Rp = (size_t)((R + 15) & ~15);
  char* p = static_cast<char*>(ws);
  w.part = reinterpret_cast<double*>(take(p, 2 * (size_t)w.nrb_max * R * R * sizeof(double)));
  w.Lg = reinterpret_cast<double*>(take(p, Rp * Rp * sizeof(double)));
  w.dinv = reinterpret_cast<double*>(take(p, Rp * sizeof(double)));
  w.F = reinterpret_cast<double*>(take(p, (size_t)n * R * sizeof(double)));
  w.colsq = reinterpret_cast<double*>(take(p, (size_t)w.ntr * R * sizeof(double)));
  return w;
}

}  // namespace

// First half: the Gram matrices of the two other factors and the Cholesky
// factor of their Hadamard product.  Reads only factors[m], m != mode, so it
// may run concurrently with the mode's MTTKRP.
hipError_t launch_gram_chol(const float* const factors[3], const int64_t dims[3], int R, int mode, void* ws,
                            int* status, hipStream_t st) {
  const int oa = mode == 0 ? 1 : 0;
  const int ob = mode == 2 ? 1 : 2;
  const int tiles_1d = (int)cdiv(R, 16);
  const size_t Rp = (size_t)((R + 15) & ~15);
  SolveWs w = solve_ws(dims, R, mode, ws);
  hipLaunchKernelGGL(gram_partial_kernel, dim3(tiles_1d * tiles_1d, w.nrb_max, 2), dim3(256), 0, st,
                     factors[oa], dims[oa], factors[ob], dims[ob], R, tiles_1d, w.nrb_max, w.part);
  const size_t lds_chol = Rp * (Rp + 1) * sizeof(double);
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(256), lds_chol, st, w.part, w.nra, w.nrb, w.nrb_max, R, w.Lg,
                     w.dinv, status);
  return hipGetLastError();
}

// Second half: F = M V^{-1} by the two triangular solves, lambda and the
// normalised FP32 factor.  Needs launch_gram_chol's results in the same ws.
hipError_t launch_solve_apply(const int64_t dims[3], int R, int mode, const float* M, float* factor_out,
                              double* lambda, void* ws, int* status, hipStream_t st) {
  const int64_t n = dims[mode];
  const size_t Rp = (size_t)((R + 15) & ~15);
  SolveWs w = solve_ws(dims, R, mode, ws);
  const size_t lds_trsm = (Rp * (Rp + 1) + 16 * (Rp + 1) + Rp) * sizeof(double);
  hipLaunchKernelGGL(trsm_rows_kernel, dim3(w.ntr), dim3(256), lds_trsm, st, M, n, R, w.Lg, w.dinv, status, w.F,
                     w.colsq);
  hipLaunchKernelGGL(normalize_kernel, dim3(w.nblk), dim3(256), 0, st, w.F, n, R, w.colsq, w.ntr, status, lambda,
                     factor_out);
  return hipGetLastError();
}

hipError_t launch_gram_solve(const float* const factors[3], const int64_t dims[3], int R, int mode,
                             const float* M, float* factor_out, double* lambda, void* ws, int* status,
                             hipStream_t st) {
  hipError_t e = launch_gram_chol(factors, dims, R, mode, ws, status, st);
  if (e != hipSuccess) return e;
  return launch_solve_apply(dims, R, mode, M, factor_out, lambda, ws, status, st);
}

// ---------------------------------------------------------------------------
// Fit: explicit residual.  Each workgroup takes one slice i and a block of
// 16 rows j; thread (jj, kk) loops over k = kk, kk+16, ...; the model value
// sum_r lambda_r A(i,r) B(j,r) C(k,r) is formed in FP64 from the FP32
// factors.  Partial sums (residual^2, ||X||^2) per workgroup, then a fixed-
// order final sum.
// ---------------------------------------------------------------------------
namespace {

__global__ __launch_bounds__(256) void fit_partial_kernel(const void* __restrict__ X, int fmt,
                                                          const int32_t* __restrict__ slice_exp,
                                                          int64_t I, int64_t J, int64_t K,
                                                          const float* __restrict__ A, const float* __restrict__ B,
                                                          const float* __restrict__ C,
                                                          const double* __restrict__ lam, int R,
                                                          double* __restrict__ part) {
  const int64_t i = blockIdx.y;
  const int64_t jb = blockIdx.x;
  const int jj = threadIdx.x >> 4, kk = threadIdx.x & 15;
  const int64_t j = jb * 16 + jj;
  __shared__ double w[16][kMaxRank];           // lambda_r A(i,r) B(j,r) for the 16 rows
  for (int e = threadIdx.x; e < 16 * R; e += 256) {
    const int q = e / R, r = e % R;
    const int64_t jq = jb * 16 + q;
    w[q][r] = jq < J ? lam[r] * (double)A[i * R + r] * (double)B[jq * R + r] : 0.0;
  }
  __syncthreads();
  double res = 0.0, nrm = 0.0;
  if (j < J) {
    const double sc = fmt == MTK_FP8_E4M3 ? ldexp(1.0, slice_exp[i]) : 1.0;
    for (int64_t k = kk; k < K; k += 16) {
      double model = 0.0;
      for (int r = 0; r < R; ++r) model = fma(w[jj][r], (double)C[k * R + r], model);
      double x;
      const int64_t off = (i * J + j) * K + k;
      if (fmt == MTK_FP8_E4M3) {
        const uint8_t c = static_cast<const uint8_t*>(X)[off];
        const int e = (c >> 3) & 15, mnt = c & 7;
        double v = e == 0 ? ldexp((double)mnt, -9) : ldexp(1.0 + mnt / 8.0, e - 7);
        if ((c & 0x7f) == 0x7f) v = __builtin_nan("");
        x = ((c & 0x80) ? -v : v) * sc;
      } else {
        x = (double)static_cast<const float*>(X)[off];
      }
      const double d = x - model;
      res = fma(d, d, res);
      nrm = fma(x, x, nrm);
    }
  }
  __shared__ double sr[256], sn[256];
  sr[threadIdx.x] = res;
  sn[threadIdx.x] = nrm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; sn[threadIdx.x] += sn[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t b = i * gridDim.x + jb;
    part[2 * b] = sr[0];
    part[2 * b + 1] = sn[0];
  }
}

__global__ __launch_bounds__(256) void fit_final_kernel(const double* __restrict__ part, int64_t nb,
                                                        double* __restrict__ acc2) {
  __shared__ double sr[256], sn[256];
  double r = 0.0, n = 0.0;
#pragma unroll 4
  for (int64_t b = threadIdx.x; b < nb; b += 256) { r += part[2 * b]; n += part[2 * b + 1]; }
  sr[threadIdx.x] = r;
  sn[threadIdx.x] = n;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; sn[threadIdx.x] += sn[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { acc2[0] = sr[0]; acc2[1] = sn[0]; }
}

}  // namespace

size_t fit_ws_bytes(const int64_t dims[3]) {
  return (size_t)dims[0] * cdiv(dims[1], 16) * 2 * sizeof(double) + 256;
}

hipError_t launch_fit(const void* X, int fmt, const int32_t* slice_exp, const int64_t dims[3],
                      const float* const factors[3], const double* lambda, int R, double* acc2, void* ws,
                      hipStream_t st) {
  double* part = static_cast<double*>(ws);
  const int64_t nb = dims[0] * cdiv(dims[1], 16);
  hipLaunchKernelGGL(fit_partial_kernel, dim3((unsigned)cdiv(dims[1], 16), (unsigned)dims[0]), dim3(256), 0,
                     st, X, fmt, slice_exp, dims[0], dims[1], dims[2], factors[0], factors[1], factors[2],
                     lambda, R, part);
  hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(256), 0, st, part, nb, acc2);
  return hipGetLastError();
}

}  // namespace mtk
