// FP64 normal-equation update of one CP factor, and the CP fit.
//
// Given the FP32 factors and the FP32 MTTKRP M (n x R) of mode `mode`:
//   V = G_a * G_b (Hadamard), G_m = A_m^T A_m over the two other modes (FP64)
//   V = L L^T (Cholesky, FP64; a pivot <= 0 sets the sticky NOT-SPD status)
//   F = M V^{-1}: per row, forward substitution with L then back
//       substitution with L^T (FP64)
//   lambda_r = ||F(:,r)||_2, factor = F(:,r) / lambda_r cast to FP32.
// Every reduction runs in a fixed order, so the update is deterministic.

#include "mtk_internal.h"

namespace mtk {
namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kRowsPerBlock = 2048;   // rows summed by one Gram / norm partial

// part[rb][r][s] = sum over rows i of block rb of F(i,r) F(i,s), FP64.
// Block (tile, rb), 256 threads = 16 x 16 entries of a 16 x 16 tile.
__global__ __launch_bounds__(256) void gram_partial_kernel(const float* __restrict__ F, int64_t n, int R,
                                                           int tiles_1d, double* __restrict__ part) {
  const int tile = blockIdx.x;
  const int rb = blockIdx.y;
  const int tr = tile / tiles_1d, ts = tile % tiles_1d;
  const int r = tr * 16 + (threadIdx.x >> 4);
  const int s = ts * 16 + (threadIdx.x & 15);
  __shared__ float rows_r[64][16];
  __shared__ float rows_s[64][16];
  const int64_t i0 = (int64_t)rb * kRowsPerBlock;
  const int64_t i1 = min(n, i0 + kRowsPerBlock);
  double acc = 0.0;
  for (int64_t c0 = i0; c0 < i1; c0 += 64) {
    // Stage 64 rows x 16 columns of both column groups.
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
  if (r < R && s < R) part[((int64_t)rb * R + r) * R + s] = acc;
}

// V[r][s] = (sum_rb pa[rb][r][s]) * (sum_rb pb[rb][r][s]), fixed order.
__global__ __launch_bounds__(256) void hadamard_kernel(const double* __restrict__ pa, int nra,
                                                       const double* __restrict__ pb, int nrb, int R,
                                                       double* __restrict__ V) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= R * R) return;
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nra; ++q) a += pa[(int64_t)q * R * R + e];
  for (int q = 0; q < nrb; ++q) b += pb[(int64_t)q * R * R + e];
  V[e] = a * b;
}

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Cholesky V = L L^T of one R x R matrix by a single workgroup, right-looking,
// packed lower triangle in LDS.  Writes L (packed) to Lg.  On a pivot <= 0
// (or NaN) sets kStatusNotSPD in *status and stops.
__global__ __launch_bounds__(256) void cholesky_kernel(const double* __restrict__ V, int R,
                                                       double* __restrict__ Lg, int* __restrict__ status) {
  extern __shared__ double P[];
  const int tid = threadIdx.x;
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, j = e % R;
    if (j <= i) P[tri(i, j)] = V[e];
  }
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    const double d = P[tri(j, j)];
    if (!(d > 0.0)) {
      if (tid == 0) atomicOr(status, kStatusNotSPD);
      return;                       // uniform: every thread read the same d
    }
    const double sd = sqrt(d);
    __syncthreads();
    for (int i = j + tid; i < R; i += 256) P[tri(i, j)] = (i == j) ? sd : P[tri(i, j)] / sd;
    __syncthreads();
    for (int i = j + 1 + (tid >> 4); i < R; i += 16) {
      const double lij = P[tri(i, j)];
      for (int k = j + 1 + (tid & 15); k <= i; k += 16) P[tri(i, k)] -= lij * P[tri(k, j)];
    }
    __syncthreads();
  }
  for (int e = tid; e < R * (R + 1) / 2; e += 256) Lg[e] = P[e];
}

// Sum over the 64 lanes of a wave, butterfly order fixed by lane index.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// F(q,:) = M(q,:) V^{-1} with V = L L^T: solve y L^T = m (forward with L),
// then f L = y (back with L^T).  One wave per row; lane owns columns lane and
// lane + 64.  Skips everything if the Cholesky failed.
__global__ __launch_bounds__(256) void trsolve_rows_kernel(const float* __restrict__ M, int64_t n, int R,
                                                           const double* __restrict__ L,
                                                           const int* __restrict__ status,
                                                           double* __restrict__ F) {
  if (*status & kStatusNotSPD) return;
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= n) return;
  double y0 = 0.0, y1 = 0.0;            // y / f of columns lane, lane + 64
  const float* m = M + q * R;
  // forward: y_r = (m_r - sum_{s<r} L[r][s] y_s) / L[r][r]
  for (int r = 0; r < R; ++r) {
    const double* Lr = L + tri(r, 0);
    double p = 0.0;
    if (lane < r) p = Lr[lane] * y0;
    if (lane + 64 < r) p = fma(Lr[lane + 64], y1, p);
    const double tot = wave_sum(p);
    const double yr = ((double)m[r] - tot) / Lr[r];
    if ((r & 63) == lane) { if (r < 64) y0 = yr; else y1 = yr; }
  }
  // back: f_r = (y_r - sum_{s>r} L[s][r] f_s) / L[r][r]
  double f0 = 0.0, f1 = 0.0;
  for (int r = R - 1; r >= 0; --r) {
    double p = 0.0;
    if (lane > r && lane < R) p = L[tri(lane, r)] * f0;
    if (lane + 64 > r && lane + 64 < R) p = fma(L[tri(lane + 64, r)], f1, p);
    const double tot = wave_sum(p);
    const double yr = __shfl(r < 64 ? y0 : y1, r & 63, 64);
    const double fr = (yr - tot) / L[tri(r, r)];
    if ((r & 63) == lane) { if (r < 64) f0 = fr; else f1 = fr; }
  }
  if (lane < R) F[q * R + lane] = f0;
  if (lane + 64 < R) F[q * R + lane + 64] = f1;
}

// part[rb][r] = sum over rows of block rb of F(i,r)^2.
__global__ __launch_bounds__(256) void colsq_partial_kernel(const double* __restrict__ F, int64_t n, int R,
                                                            const int* __restrict__ status,
                                                            double* __restrict__ part) {
  if (*status & kStatusNotSPD) return;
  const int c = blockIdx.x * 16 + (threadIdx.x & 15);
  const int g = threadIdx.x >> 4;       // 16 row groups
  const int64_t i0 = (int64_t)blockIdx.y * kRowsPerBlock;
  const int64_t i1 = min(n, i0 + kRowsPerBlock);
  double acc = 0.0;
  if (c < R)
    for (int64_t i = i0 + g; i < i1; i += 16) { const double v = F[i * R + c]; acc = fma(v, v, acc); }
  __shared__ double sh[16][16];
  sh[g][threadIdx.x & 15] = acc;
  __syncthreads();
  if (g == 0 && c < R) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += sh[q][threadIdx.x & 15];
    part[(int64_t)blockIdx.y * R + c] = s;
  }
}

__global__ __launch_bounds__(128) void lambda_kernel(const double* __restrict__ part, int nrb, int R,
                                                     const int* __restrict__ status, double* __restrict__ lam) {
  if (*status & kStatusNotSPD) return;
  const int c = threadIdx.x;
  if (c >= R) return;
  double s = 0.0;
  for (int q = 0; q < nrb; ++q) s += part[(int64_t)q * R + c];
  lam[c] = sqrt(s);
}

__global__ __launch_bounds__(256) void normalize_kernel(const double* __restrict__ F, int64_t n, int R,
                                                        const double* __restrict__ lam,
                                                        const int* __restrict__ status, float* __restrict__ out) {
  if (*status & kStatusNotSPD) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * R) return;
  const double l = lam[e % R];
  out[e] = (float)(l > 0.0 ? F[e] / l : F[e]);
}

}  // namespace

size_t solve_ws_bytes(int64_t maxdim, int R) {
  const int64_t nrb = cdiv(maxdim, kRowsPerBlock);
  size_t b = 0;
  b += 2 * (size_t)nrb * R * R * sizeof(double);     // Gram partials of the two other factors
  b += (size_t)R * R * sizeof(double);               // V
  b += (size_t)R * (R + 1) / 2 * sizeof(double);     // L
  b += (size_t)maxdim * R * sizeof(double);          // F
  b += (size_t)nrb * R * sizeof(double);             // column-norm partials
  return b + 6 * 256;
}

static inline char* take(char*& p, size_t bytes) {
  char* r = p;
  p += (bytes + 255) & ~(size_t)255;
  return r;
}

hipError_t launch_gram_solve(const float* const factors[3], const int64_t dims[3], int R, int mode,
                             const float* M, float* factor_out, double* lambda, void* ws, int* status,
                             hipStream_t st) {
  const int oa = mode == 0 ? 1 : 0;
  const int ob = mode == 2 ? 1 : 2;
  const int64_t n = dims[mode];
  const int tiles_1d = (int)cdiv(R, 16);
  const int nra = (int)cdiv(dims[oa], kRowsPerBlock);
  const int nrb = (int)cdiv(dims[ob], kRowsPerBlock);
  const int nrn = (int)cdiv(n, kRowsPerBlock);
  char* p = static_cast<char*>(ws);
  double* pa = reinterpret_cast<double*>(take(p, (size_t)nra * R * R * sizeof(double)));
  double* pb = reinterpret_cast<double*>(take(p, (size_t)nrb * R * R * sizeof(double)));
  double* V = reinterpret_cast<double*>(take(p, (size_t)R * R * sizeof(double)));
  double* L = reinterpret_cast<double*>(take(p, (size_t)R * (R + 1) / 2 * sizeof(double)));
  double* F = reinterpret_cast<double*>(take(p, (size_t)n * R * sizeof(double)));
  double* pn = reinterpret_cast<double*>(take(p, (size_t)nrn * R * sizeof(double)));

  hipLaunchKernelGGL(gram_partial_kernel, dim3(tiles_1d * tiles_1d, nra), dim3(256), 0, st,
                     factors[oa], dims[oa], R, tiles_1d, pa);
  hipLaunchKernelGGL(gram_partial_kernel, dim3(tiles_1d * tiles_1d, nrb), dim3(256), 0, st,
                     factors[ob], dims[ob], R, tiles_1d, pb);
  hipLaunchKernelGGL(hadamard_kernel, dim3((unsigned)cdiv((int64_t)R * R, 256)), dim3(256), 0, st,
                     pa, nra, pb, nrb, R, V);
  const size_t lds = (size_t)R * (R + 1) / 2 * sizeof(double);
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(256), lds, st, V, R, L, status);
  hipLaunchKernelGGL(trsolve_rows_kernel, dim3((unsigned)cdiv(n, 4)), dim3(256), 0, st, M, n, R, L,
                     status, F);
  hipLaunchKernelGGL(colsq_partial_kernel, dim3((unsigned)tiles_1d, nrn), dim3(256), 0, st, F, n, R,
                     status, pn);
  hipLaunchKernelGGL(lambda_kernel, dim3(1), dim3(128), 0, st, pn, nrn, R, status, lambda);
  hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)cdiv(n * R, 256)), dim3(256), 0, st, F, n, R,
                     lambda, status, factor_out);
  return hipGetLastError();
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
