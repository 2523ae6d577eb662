// FP64 normal-equation update of one CP factor, and the CP fit.
//
// Given the FP32 factors and the FP32 MTTKRP M (n x R) of mode `mode`:
//   G_m = A_m^T A_m, the Gram matrix of factor m (FP64 sums of FP32 products)
//   V = G_a * G_b (Hadamard) over the two other modes
//   V^{-1} by symmetric elimination: the LDL^T (square-root-free Cholesky)
//   factorisation in Gauss-Jordan form (FP64; a pivot <= 0 sets the sticky
//   NOT-SPD status)
//   F = M V^{-1} (FP64)
//   lambda_r = ||F(:,r)||_2, factor = F(:,r) / lambda_r cast to FP32.
// The Gram matrix of the factor just written is formed (as per-row-block
// partial sums) in the same pass that normalises it, so a sweep never
// recomputes one; the first mode of a sequence of sweeps takes them from
// launch_grams.  The consumer of a set of partials sums them, so no kernel
// needs a device-wide fence.
//
// Every reduction runs in a fixed order, so the update is deterministic.

#include "mtk_internal.h"
#include "srv_internal.h"
#include "factor_device.h"

#include <algorithm>

namespace mtk {
namespace {

using fdev::tile_pair;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// 16 x 16 tiles of the lower triangle of an R x R Gram matrix.
__host__ __device__ inline int gram_pairs(int R) { const int t = (R + 15) / 16; return t * (t + 1) / 2; }
// Row blocks of a Gram matrix (one partial each): about 128 workgroups in
// all (tile pairs x blocks), at most kGramBlocksMax blocks.  Their partials
// are summed where V is gathered (one workgroup), so fewer is cheaper there.
__host__ __device__ inline int gram_blocks(int64_t n, int R) {
  int64_t b = 128 / gram_pairs(R);
  b = b < 1 ? 1 : (b > kGramBlocksMax ? kGramBlocksMax : b);
  const int64_t bmax = cdiv(n, 64);
  return (int)(b < bmax ? b : bmax);
}
__host__ __device__ inline int64_t gram_rows(int64_t n, int R) { return cdiv(n, gram_blocks(n, R)); }
// Rows per workgroup of the apply kernel.
constexpr int kApplyRows = 16;
// Size of one factor's Gram partials: [tile pair][row block][16 x 16].
__host__ __device__ inline size_t gram_part_elems(int R) { return (size_t)gram_pairs(R) * kGramBlocksMax * 256; }


typedef __attribute__((ext_vector_type(4))) double gram_d4;

// Gram tile over rows [i0, i1) on FP64 MFMA (16x16x4): rows are taken in
// chunks of 64, wave w of the workgroup owning rows c0 + 16w + 4s + g of a
// chunk (step s = 0..3, g = lane / 16), lane (n, g) holding column tr*16 + n
// as the A operand and ts*16 + n as the B operand, so the 16 x 16 x 4 product
// adds four rows' outer products; step s accumulates into acc[s].  S chunks
// are loaded at once and the next S are in flight while these are summed.
// The accumulation order does not depend on S (acc[s] takes the chunks in
// increasing order).  Result layout (FP64 16x16x4, measured on the device):
// lane (n, g) receives tile rows g + 4v, column n.
template <int S, class Load, class Conv, class Emit>
__device__ void gram_tile_mfma(int64_t i0, int64_t i1, int R, int tr, int ts, Load load, Conv conv, Emit emit,
                               gram_d4 acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nn = lane & 15, g = lane >> 4;
  const int cr = tr * 16 + nn, cs = ts * 16 + nn;
  const int crl = min(cr, R - 1), csl = min(cs, R - 1);
  using Raw = decltype(load(int64_t(0), 0));
  Raw ra[S][4], rb[S][4];
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t i = min(c0 + 64 * q + 16 * w + 4 * s + g, i1 - 1);
        ra[q][s] = load(i, crl);
        rb[q][s] = load(i, csl);  // unused on a diagonal tile (a branch here would wait on the loads)
      }
  };
  if (i0 < i1) fetch(i0);
  for (int64_t c0 = i0; c0 < i1; c0 += 64 * S) {
    double a[S][4], b[S][4];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t i = c0 + 64 * q + 16 * w + 4 * s + g;
        float va = 0.f, vb = 0.f;
        if (i < i1 && cr < R) { va = conv(ra[q][s], cr); emit(i, cr, va); }
        if (i < i1 && cs < R) vb = tr == ts ? va : conv(rb[q][s], cs);
        a[q][s] = va;
        b[q][s] = vb;
      }
    if (c0 + 64 * S < i1) fetch(c0 + 64 * S);
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][s], b[q][s], acc[s], 0, 0, 0);
  }
}

// Accumulate the Gram tile (rows tr*16.., cols ts*16..) over rows [i0, i1) of
// a factor: load(i, col) reads the stored value and conv(raw, col) turns it
// into the FP32 factor value (emit(i, col, v) sees each value of a diagonal
// tile once).  Returns tile element (tid / 16, tid % 16) to thread tid: the
// four steps' sums added in order, then the four waves' in order.  Both Gram
// kernels use this one routine, so they agree bit for bit.  Row blocks of
// 1024 rows or more load four chunks at a time, shorter ones two (at most
// MAXS: the grouped serving kernel, whose factors are short, takes one and
// so keeps its registers low).
template <int MAXS = 4, class Load, class Conv, class Emit>
__device__ double gram_tile_rows(int64_t i0, int64_t i1, int R, int tr, int ts, Load load, Conv conv, Emit emit) {
  __shared__ double red[4][256];
  gram_d4 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = gram_d4{0.0, 0.0, 0.0, 0.0};
  if constexpr (MAXS >= 4) {
    if (i1 - i0 >= 1024) gram_tile_mfma<4>(i0, i1, R, tr, ts, load, conv, emit, acc);
    else gram_tile_mfma<2>(i0, i1, R, tr, ts, load, conv, emit, acc);
  } else {
    gram_tile_mfma<MAXS>(i0, i1, R, tr, ts, load, conv, emit, acc);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    red[w][((lane >> 4) + 4 * v) * 16 + (lane & 15)] = ((acc[0][v] + acc[1][v]) + acc[2][v]) + acc[3][v];
  __syncthreads();
  const int t = threadIdx.x;
  const double r = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
  __syncthreads();
  return r;
}

// Partial of tile `tile` over row block `rb`, stored as [tile][rb][16 x 16].
__device__ __forceinline__ void gram_store(double acc, double* __restrict__ part, int tile, int rb) {
  part[((size_t)tile * kGramBlocksMax + rb) * 256 + threadIdx.x] = acc;
}

// Gram partials of one or two FP32 factors.  Grid (tile pairs, row blocks, factors).
__global__ __launch_bounds__(256) void gram_kernel(const float* __restrict__ F0, int64_t n0, double* __restrict__ P0,
                                                   const float* __restrict__ F1, int64_t n1, double* __restrict__ P1,
                                                   int R) {
  const int f = blockIdx.z;
  const float* F = f ? F1 : F0;
  const int64_t n = f ? n1 : n0;
  const int nrb = gram_blocks(n, R);
  const int rb = blockIdx.y;
  if (rb >= nrb) return;
  int tr, ts;
  tile_pair(blockIdx.x, tr, ts);
  const int64_t rows = gram_rows(n, R);
  const int64_t i0 = (int64_t)rb * rows, i1 = min(n, i0 + rows);
  const double acc = gram_tile_rows(
      i0, i1, R, tr, ts, [&](int64_t i, int c) { return F[i * R + c]; }, [](float v, int) { return v; },
      [](int64_t, int, float) {});
  gram_store(acc, f ? P1 : P0, blockIdx.x, rb);
}


// Stand-alone factorisation (V^{-1}): one workgroup.
template <int B>
__global__ __launch_bounds__(256) void gj_inv_kernel(FactorArgs f) {
  extern __shared__ double lds[];
  factor_gj<B>(f, lds);
}

// F = M V^{-1}: workgroup (row block of 16, column block of 16); thread
// (g, c) owns row g, column c.  M arrives as S split-K slices, sstride floats
// apart, added here in the split-K reduction's order (slice k into partial
// k mod 8 in increasing k, then the 8 partials in order), so an update can
// take them without a separate reduction; S = 1 is a plain M.  Also writes
// the row block's sums of F^2 per column (rows in a fixed order).
// Workgroup (bx, by) of the apply launch (grid nblk x ceil(R/16)).
__device__ __forceinline__ void apply_body(const float* __restrict__ M, int S, int64_t sstride, int64_t n, int R,
                                           const double* __restrict__ Vinv, const int* __restrict__ status,
                                           double* __restrict__ F, double* __restrict__ colsq,
                                           double* __restrict__ ipsum, int64_t bx, int by) {
  if (*status & kStatusNotSPD) return;
  __shared__ double Vs[kMaxRank * 16];
  __shared__ float Ms[kApplyRows][kMaxRank + 1];
  __shared__ double red[16][16];
  const int tid = threadIdx.x, c = tid & 15, g = tid >> 4;
  const int cb = by * 16;
  const int64_t q0 = bx * kApplyRows;
  // Staging loads use clamped in-range indices and go out in batches before
  // any is stored.
  {
    constexpr int U = kMaxRank * 16 / 256;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + 256 * u;
      const int k = min(e >> 4, R - 1), cc = e & 15;
      v[u] = Vinv[(int64_t)k * R + min(cb + cc, R - 1)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + 256 * u;
      if (e < R * 16) Vs[e] = cb + (e & 15) < R ? v[u] : 0.0;
    }
  }
  const int64_t nrow = min<int64_t>(kApplyRows, n - q0);
  const int nm = (int)nrow * R;
  const float* Mb = M + q0 * R;
  if (S == 1) {
    for (int e0 = tid; e0 < kApplyRows * R; e0 += 256 * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = Mb[min(e0 + 256 * u, nm - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u;
        if (e < kApplyRows * R) {
          const int rr = e / R, k = e - rr * R;
          Ms[rr][k] = e < nm ? v[u] : 0.f;
        }
      }
    }
  } else {
    for (int e = tid; e < kApplyRows * R; e += 256) {
      const float* src = Mb + min(e, nm - 1);
      float p8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < S; k0 += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = src[(int64_t)min(k0 + u, S - 1) * sstride];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (k0 + u < S) p8[u & 7] += v[u];
      }
      float t = p8[0];
#pragma unroll
      for (int q = 1; q < 8; ++q) t += p8[q];
      const int rr = e / R, k = e - rr * R;
      Ms[rr][k] = e < nm ? t : 0.f;
    }
  }
  __syncthreads();
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < R; ++k) acc = fma((double)Ms[g][k], Vs[k * 16 + c], acc);
  double s = 0.0, ip = 0.0;
  const int col = cb + c;
  const int64_t q = q0 + g;
  if (q < n && col < R) {
    F[q * R + col] = acc;
    s = acc * acc;
    ip = acc * (double)Ms[g][col];
  }
  red[g][c] = s;
  __syncthreads();
  if (tid < 16 && cb + tid < R) {
    double t = 0.0;
#pragma unroll
    for (int gg = 0; gg < 16; ++gg) t += red[gg][tid];
    colsq[bx * R + cb + tid] = t;
  }
  if (ipsum) {                       // <F, M> of this block, per column (same order as colsq)
    __syncthreads();
    red[g][c] = ip;
    __syncthreads();
    if (tid < 16 && cb + tid < R) {
      double t = 0.0;
#pragma unroll
      for (int gg = 0; gg < 16; ++gg) t += red[gg][tid];
      ipsum[bx * R + cb + tid] = t;
    }
  }
}

__global__ __launch_bounds__(256) void apply_kernel(const float* __restrict__ M, int S, int64_t sstride, int64_t n,
                                                    int R, const double* __restrict__ Vinv,
                                                    const int* __restrict__ status, double* __restrict__ F,
                                                    double* __restrict__ colsq, double* __restrict__ ipsum) {
  apply_body(M, S, sstride, n, R, Vinv, status, F, colsq, ipsum, blockIdx.x, blockIdx.y);
}

// lambda_c = sqrt(sum over row blocks of colsq) (fixed order, recomputed by
// every workgroup), factor = F / lambda (FP32; zero columns left unscaled),
// and the Gram partials of that FP32 factor.  Grid (tile pairs, row blocks);
// the workgroups of diagonal tiles write the factor's columns of their tile,
// and those of row block 0 write lambda.
// Workgroup (bx = tile pair, by = row block) of the normalise launch.
template <int MAXS = 4>
__device__ __forceinline__ void normalize_gram_body(const double* __restrict__ F, int64_t n, int R,
                                                    const double* __restrict__ colsq, int nblk,
                                                    const int* __restrict__ status, double* __restrict__ lam,
                                                    float* __restrict__ out, double* __restrict__ part,
                                                    const double* __restrict__ ipsum, double* __restrict__ ip,
                                                    int bx, int by) {
  if (*status & kStatusNotSPD) return;
  __shared__ double lsum[8][32];
  __shared__ double lt[32];
  __shared__ double ired[256];
  int tr, ts;
  tile_pair(bx, tr, ts);
  const int tid = threadIdx.x;
  if (ipsum && bx == 0 && by == 0) {
    // <F, M> over the whole factor: strided per-thread sums (32 loads in
    // flight), then a tree, in fixed order.
    const int64_t ne = (int64_t)nblk * R;
    double t = 0.0;
    for (int64_t e0 = tid; e0 < ne; e0 += 256 * 32) {
      double v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = ipsum[min(e0 + 256 * u, ne - 1)];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (e0 + 256 * u < ne) t += v[u];
    }
    ired[tid] = t;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) ired[tid] += ired[tid + h];
      __syncthreads();
    }
    if (tid == 0) *ip = ired[0];
  }
  const bool diag = tr == ts;
  {
    // Column u of the tile pair (u < 16: tr, else ts): thread (q, u) sums
    // row blocks b = q, q + 8, ... in order, 32 loads in flight (a factor
    // of 65536 rows has 4096 row blocks).
    const int u = tid & 31, q = tid >> 5;
    const int col = (u < 16 ? tr : ts) * 16 + (u & 15);
    const int cl = min(col, R - 1);
    double t = 0.0;
    for (int b0 = q; b0 < nblk; b0 += 256) {
      double v[32];
#pragma unroll
      for (int w = 0; w < 32; ++w) v[w] = colsq[(int64_t)min(b0 + 8 * w, nblk - 1) * R + cl];
#pragma unroll
      for (int w = 0; w < 32; ++w)
        if (col < R && b0 + 8 * w < nblk) t += v[w];
    }
    lsum[q][u] = t;
  }
  __syncthreads();
  if (tid < 32) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t += lsum[q][tid];
    lt[tid] = sqrt(t);
    const int col = (tid < 16 ? tr : ts) * 16 + (tid & 15);
    if (diag && tid < 16 && by == 0 && col < R) lam[col] = lt[tid];
  }
  __syncthreads();
  const int rb = by;
  const int64_t rows = gram_rows(n, R);
  const int64_t i0 = (int64_t)rb * rows, i1 = min(n, i0 + rows);
  auto load = [&](int64_t i, int col) { return F[i * R + col]; };
  auto conv = [&](double f, int col) {
    const double l = lt[col / 16 == tr ? (col & 15) : 16 + (col & 15)];
    return (float)(l > 0.0 ? f / l : f);
  };
  auto emit = [&](int64_t i, int col, float v) {
    if (diag) out[i * R + col] = v;
  };
  const double acc = gram_tile_rows<MAXS>(i0, i1, R, tr, ts, load, conv, emit);
  gram_store(acc, part, bx, rb);
}

__global__ __launch_bounds__(256) void normalize_gram_kernel(const double* __restrict__ F, int64_t n, int R,
                                                             const double* __restrict__ colsq, int nblk,
                                                             const int* __restrict__ status, double* __restrict__ lam,
                                                             float* __restrict__ out, double* __restrict__ part,
                                                             const double* __restrict__ ipsum, double* __restrict__ ip) {
  normalize_gram_body(F, n, R, colsq, nblk, status, lam, out, part, ipsum, ip, blockIdx.x, blockIdx.y);
}

// Extrapolation candidate of one factor: E = P + d (Q - P) in FP64 into the
// solve region's F, with the per-16-row column sums of squares in the
// layout apply_kernel leaves them (normalize_gram_kernel then gives the
// unit-column FP32 factor, its norms and its Gram partials).  Workgroup
// (row block, 16-column tile); each column's 16 squares are added in row order.
__global__ __launch_bounds__(256) void extrapolate_kernel(const float* __restrict__ P, const float* __restrict__ Q,
                                                          int64_t n, int R, double d, double* __restrict__ F,
                                                          double* __restrict__ colsq) {
  __shared__ double sq[kApplyRows][17];
  const int rr = threadIdx.x >> 4, cc = threadIdx.x & 15;
  const int64_t i = (int64_t)blockIdx.x * kApplyRows + rr;
  const int c = blockIdx.y * 16 + cc;
  double e = 0.0;
  if (i < n && c < R) {
    const double p = P[i * R + c], q = Q[i * R + c];
    e = p + d * (q - p);
    F[i * R + c] = e;
  }
  sq[rr][cc] = e * e;
  __syncthreads();
  if (rr == 0 && c < R) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kApplyRows; ++k) t += sq[k][cc];
    colsq[(int64_t)blockIdx.x * R + c] = t;
  }
}

}  // namespace

namespace {

// Grouped update kernels of a serving step (see srv_internal.h).  Each
// workgroup strides over the step's work items, finds its request and runs
// the same body as the single-request launch; the barrier at the end of an
// item keeps the next item's LDS writes behind this item's reads.

// V^{-1} of every request: one workgroup per entry.
__global__ __launch_bounds__(256) void srv_factor_kernel(const SrvTable* __restrict__ t, int upd) {
  extern __shared__ double flds[];
  for (int q = blockIdx.x; q < t->nreq; q += gridDim.x) {
    const FactorArgs f = t->e[q][upd].u.fa;
    switch ((f.R + 15) / 16) {
      case 1: factor_gj<1>(f, flds); break;
      case 2: factor_gj<2>(f, flds); break;
      case 3: factor_gj<3>(f, flds); break;
      case 4: factor_gj<4>(f, flds); break;
      case 5: factor_gj<5>(f, flds); break;
      case 6: factor_gj<6>(f, flds); break;
      case 7: factor_gj<7>(f, flds); break;
      default: factor_gj<8>(f, flds); break;
    }
    __syncthreads();
  }
}

// F = M V^{-1} of every request: workgroup (row block, column block).
__global__ __launch_bounds__(256) void srv_apply_kernel(const SrvTable* __restrict__ t, int upd) {
  const int nreq = t->nreq;
  for (int64_t w = blockIdx.x; w < t->n_ab[upd]; w += gridDim.x) {
    const int q = srv_find(nreq, w, [&](int i) { return t->e[i][upd].ab0; });
    const SrvUpdate& u = t->e[q][upd].u;
    const int64_t local = w - t->e[q][upd].ab0;
    apply_body(u.M, u.S, u.sstride, u.n, u.R, u.fa.vinv, u.status, u.F, u.colsq, nullptr, local % u.nblk,
               (int)(local / u.nblk));
    __syncthreads();
  }
}

// lambda, the normalised factor and its Gram partials: workgroup (tile pair, row block).
__global__ __launch_bounds__(256) void srv_normalize_kernel(const SrvTable* __restrict__ t, int upd) {
  const int nreq = t->nreq;
  for (int64_t w = blockIdx.x; w < t->n_nb[upd]; w += gridDim.x) {
    const int q = srv_find(nreq, w, [&](int i) { return t->e[i][upd].nb0; });
    const SrvUpdate& u = t->e[q][upd].u;
    const int64_t local = w - t->e[q][upd].nb0;
    const int np = gram_pairs(u.R);
    normalize_gram_body<1>(u.F, u.n, u.R, u.colsq, u.nblk, u.status, u.lam, u.fout, u.gram_out, nullptr, nullptr,
                        (int)(local % np), (int)(local / np));
    __syncthreads();
  }
}

}  // namespace

// Workspace of the update: [Gram partials of factors 0, 1, 2][V^{-1} R^2]
// [F maxdim x R][column sums per row block].
static inline char* take(char*& p, size_t bytes) {
  char* r = p;
  p += (bytes + 255) & ~(size_t)255;
  return r;
}

namespace {
struct SolveWs {
  double* part[3];
  double* Vinv;
  double* F;
  double* colsq;
  double* ipsum;      // per row block and column: <F, M> (mode-3 update of a sweep)
  double* ip;         // their total
};

SolveWs solve_ws(int64_t maxdim, int R, void* ws) {
  SolveWs w{};
  const size_t md = (size_t)std::max<int64_t>(maxdim, 1);
  char* p = static_cast<char*>(ws);
  for (int m = 0; m < 3; ++m) w.part[m] = reinterpret_cast<double*>(take(p, gram_part_elems(R) * sizeof(double)));
  w.Vinv = reinterpret_cast<double*>(take(p, (size_t)R * R * sizeof(double)));
  w.F = reinterpret_cast<double*>(take(p, md * R * sizeof(double)));
  w.colsq = reinterpret_cast<double*>(take(p, (size_t)cdiv((int64_t)md, kApplyRows) * R * sizeof(double)));
  w.ipsum = reinterpret_cast<double*>(take(p, (size_t)cdiv((int64_t)md, kApplyRows) * R * sizeof(double)));
  w.ip = reinterpret_cast<double*>(take(p, sizeof(double)));
  return w;
}
}  // namespace

size_t solve_ws_bytes(int64_t maxdim, int R) {
  const size_t md = (size_t)std::max<int64_t>(maxdim, 1);
  auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t b = 3 * r256(gram_part_elems(R) * sizeof(double));
  b += r256((size_t)R * R * sizeof(double));
  b += r256(md * R * sizeof(double));
  b += 2 * r256((size_t)cdiv((int64_t)md, kApplyRows) * R * sizeof(double));
  b += 256;
  return b;
}

const double* solve_ip(int64_t maxdim, int R, void* ws) { return solve_ws(maxdim, R, ws).ip; }

hipError_t launch_grams(const float* const factors[3], const int64_t dims[3], int R, int ma, int mb, int64_t maxdim,
                        void* ws, int* status, hipStream_t st) {
  (void)status;
  SolveWs w = solve_ws(maxdim, R, ws);
  const int nrb = std::max(gram_blocks(dims[ma], R), mb >= 0 ? gram_blocks(dims[mb], R) : 0);
  const int nf = mb >= 0 ? 2 : 1;
  hipLaunchKernelGGL(gram_kernel, dim3(gram_pairs(R), nrb, nf), dim3(256), 0, st, factors[ma], dims[ma], w.part[ma],
                     mb >= 0 ? factors[mb] : nullptr, mb >= 0 ? dims[mb] : 0, mb >= 0 ? w.part[mb] : nullptr, R);
  return hipGetLastError();
}

FactorArgs factor_args(const int64_t dims[3], int R, int mode, int64_t maxdim, void* ws, int* status) {
  const int oa = mode == 0 ? 1 : 0;
  const int ob = mode == 2 ? 1 : 2;
  SolveWs w = solve_ws(maxdim, R, ws);
  FactorArgs f{};
  f.pa = w.part[oa];
  f.na = gram_blocks(dims[oa], R);
  f.pb = w.part[ob];
  f.nb = gram_blocks(dims[ob], R);
  f.R = R;
  f.vinv = w.Vinv;
  f.status = status;
  return f;
}

hipError_t launch_factor(const int64_t dims[3], int R, int mode, int64_t maxdim, void* ws, int* status,
                         hipStream_t st) {
  const FactorArgs f = factor_args(dims, R, mode, maxdim, ws, status);
  const size_t lds = factor_gj_lds_bytes(R);
  switch ((R + 15) / 16) {
    case 1: hipLaunchKernelGGL(gj_inv_kernel<1>, dim3(1), dim3(256), lds, st, f); break;
    case 2: hipLaunchKernelGGL(gj_inv_kernel<2>, dim3(1), dim3(256), lds, st, f); break;
    case 3: hipLaunchKernelGGL(gj_inv_kernel<3>, dim3(1), dim3(256), lds, st, f); break;
    case 4: hipLaunchKernelGGL(gj_inv_kernel<4>, dim3(1), dim3(256), lds, st, f); break;
    case 5: hipLaunchKernelGGL(gj_inv_kernel<5>, dim3(1), dim3(256), lds, st, f); break;
    case 6: hipLaunchKernelGGL(gj_inv_kernel<6>, dim3(1), dim3(256), lds, st, f); break;
    case 7: hipLaunchKernelGGL(gj_inv_kernel<7>, dim3(1), dim3(256), lds, st, f); break;
    default: hipLaunchKernelGGL(gj_inv_kernel<8>, dim3(1), dim3(256), lds, st, f); break;
  }
  return hipGetLastError();
}

hipError_t launch_apply(const int64_t dims[3], int R, int mode, const float* M, float* factor_out, double* lambda,
                        int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip) {
  return launch_apply(dims, R, mode, MSlices{M, 1, 0}, factor_out, lambda, maxdim, ws, status, st, with_ip);
}

hipError_t launch_apply(const int64_t dims[3], int R, int mode, const MSlices& m, float* factor_out, double* lambda,
                        int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip) {
  const int64_t n = dims[mode];
  if (m.slices < 1 || (m.slices > 1 && m.sstride < n * R)) return hipErrorInvalidValue;
  SolveWs w = solve_ws(maxdim, R, ws);
  const int nblk = (int)cdiv(n, kApplyRows);
  hipLaunchKernelGGL(apply_kernel, dim3(nblk, (R + 15) / 16), dim3(256), 0, st, m.p, m.slices, m.sstride, n, R,
                     w.Vinv, status, w.F, w.colsq, with_ip ? w.ipsum : nullptr);
  hipLaunchKernelGGL(normalize_gram_kernel, dim3(gram_pairs(R), gram_blocks(n, R)), dim3(256), 0, st, w.F, n, R, w.colsq,
                     nblk, status, lambda, factor_out, w.part[mode], with_ip ? w.ipsum : nullptr,
                     with_ip ? w.ip : nullptr);
  return hipGetLastError();
}

hipError_t launch_extrapolate(const int64_t dims[3], int R, int mode, const float* P, const float* Q, double d,
                              float* factor_out, double* lambda, int64_t maxdim, void* ws, int* status,
                              hipStream_t st) {
  const int64_t n = dims[mode];
  SolveWs w = solve_ws(maxdim, R, ws);
  const int nblk = (int)cdiv(n, kApplyRows);
  hipLaunchKernelGGL(extrapolate_kernel, dim3(nblk, (R + 15) / 16), dim3(256), 0, st, P, Q, n, R, d, w.F, w.colsq);
  hipLaunchKernelGGL(normalize_gram_kernel, dim3(gram_pairs(R), gram_blocks(n, R)), dim3(256), 0, st, w.F, n, R, w.colsq,
                     nblk, status, lambda, factor_out, w.part[mode], nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_update(const int64_t dims[3], int R, int mode, const float* M, float* factor_out, double* lambda,
                         int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip) {
  return launch_update(dims, R, mode, MSlices{M, 1, 0}, factor_out, lambda, maxdim, ws, status, st, with_ip);
}

hipError_t launch_update(const int64_t dims[3], int R, int mode, const MSlices& m, float* factor_out,
                         double* lambda, int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip) {
  hipError_t e = launch_factor(dims, R, mode, maxdim, ws, status, st);
  if (e != hipSuccess) return e;
  return launch_apply(dims, R, mode, m, factor_out, lambda, maxdim, ws, status, st, with_ip);
}

hipError_t launch_gram_solve(const float* const factors[3], const int64_t dims[3], int R, int mode,
                             const float* M, float* factor_out, double* lambda, void* ws, int* status,
                             hipStream_t st) {
  const int oa = mode == 0 ? 1 : 0;
  const int ob = mode == 2 ? 1 : 2;
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  hipError_t e = launch_grams(factors, dims, R, oa, ob, maxdim, ws, status, st);
  if (e != hipSuccess) return e;
  return launch_update(dims, R, mode, M, factor_out, lambda, maxdim, ws, status, st);
}

// ---------------------------------------------------------------------------
// Fit: explicit residual.  Each workgroup takes one slice i and a block of
// 16 rows j; thread (jj, kk) loops over k = kk, kk+16, ...; the model value
// sum_r lambda_r A(i,r) B(j,r) C(k,r) is formed in FP64 from the FP32
// factors.  Partial sums (residual^2, ||X||^2) per workgroup, then a fixed-
// order final sum.
// ---------------------------------------------------------------------------
namespace {

// Value of an e4m3 code (NaN for 0x7F / 0xFF).
__device__ inline double e4m3_to_double(uint8_t c) {
  const int e = (c >> 3) & 15, mnt = c & 7;
  double v = e == 0 ? ldexp((double)mnt, -9) : ldexp(1.0 + mnt / 8.0, e - 7);
  if ((c & 0x7f) == 0x7f) v = __builtin_nan("");
  return (c & 0x80) ? -v : v;
}

typedef __attribute__((ext_vector_type(4))) double d4;

// Squared residual and squared norm of X against the CP model, FP64.  For
// slice i the model block Xhat(j, k) = sum_r W(j, r) C(k, r), W(j, r) =
// lambda_r A(i, r) B(j, r), is a product of shape (16 j) x R x (16 k) per
// tile, done on FP64 MFMA (16x16x4): wave w of the workgroup owns JT tiles
// of 16 j and walks the k tiles; lane (n, g) holds W(j0 + n, 4s + g) as its
// A operand for step s (in registers for the whole walk) and reads
// C(k0 + n, 4s + g) as its B operand from LDS, and receives
// Xhat(j0 + g + 4v, k0 + n), v = 0..3 (the FP64 result layout, measured on
// the device; the FP32 16x16x4 one is rows 4g + v).  The four waves walk
// the same k tiles, so each 16-row tile of C (16 R contiguous floats) is
// loaded once per workgroup, widened to FP64 into one of two LDS buffers
// while the other feeds the MFMAs, with one barrier per tile.  Partial
// sums per workgroup in fixed order.
// Three waves per SIMD: the largest instances then keep a few registers in
// scratch, which costs less than the third wave gains (768^3 R=128:
// 2.44 -> 2.26 ms; 1024^3 R=64: 3.29 -> 3.14 ms).
#ifndef MTK_FIT_WAVES
#define MTK_FIT_WAVES 3
#endif
#if MTK_FIT_WAVES > 0
#define MTK_FIT_ATTR __attribute__((amdgpu_waves_per_eu(MTK_FIT_WAVES)))
#else
#define MTK_FIT_ATTR
#endif
template <int RQ, int JT>
__global__ __launch_bounds__(256) MTK_FIT_ATTR void fit_partial_kernel(const void* __restrict__ X, int fmt,
                                                          const int32_t* __restrict__ slice_exp,
                                                          int64_t I, int64_t J, int64_t K,
                                                          const float* __restrict__ A, const float* __restrict__ B,
                                                          const float* __restrict__ C,
                                                          const double* __restrict__ lam, int R, int64_t nbx,
                                                          double* __restrict__ part) {
  constexpr int RP = 4 * RQ + 1;                    // LDS row pitch (doubles)
  constexpr int CV = (16 * 4 * RQ + 1023) / 1024;   // float4 pieces of a C tile per thread (at most)
  __shared__ double cl[2][16][RP];
  __shared__ double sr[256], sn[256];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n = lane & 15, g = lane >> 4;
  // Columns R .. 4 RQ - 1 of both buffers stay zero.
  for (int e = tid; e < 2 * 16 * (4 * RQ - R); e += 256) {
    const int q = e / (4 * RQ - R), c = R + e % (4 * RQ - R);
    cl[q >> 4][q & 15][c] = 0.0;
  }
  const int64_t tile_elems = 16 * (int64_t)R, c_elems = K * (int64_t)R;
  float4 cn[CV];
  auto c_load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < CV; ++q) {
      const int64_t e = 4 * ((int64_t)tid + 256 * q);
      const int64_t ge = k0 * R + e;
      cn[q] = (e < tile_elems && ge < c_elems) ? *reinterpret_cast<const float4*>(C + ge) : float4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto c_store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < CV; ++q) {
      const int e = 4 * (tid + 256 * q);
      if (e < tile_elems) {
        const float v[4] = {cn[q].x, cn[q].y, cn[q].z, cn[q].w};
#pragma unroll
        for (int u = 0; u < 4; ++u) cl[buf][(e + u) / R][(e + u) % R] = (double)v[u];
      }
    }
  };
  // Work item b = (slice i, j block bx), i = b / nbx; the grid strides over
  // the I * nbx items, so no grid dimension grows with I.
  for (int64_t b = blockIdx.x; b < I * nbx; b += gridDim.x) {
  const int64_t i = b / nbx;
  const int64_t jw = ((b - i * nbx) * 4 + wave) * (16 * JT);   // first j of this wave
  double w[JT][RQ];
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int s = 0; s < RQ; ++s) {
      const int r = 4 * s + g;
      const int64_t j = jw + 16 * t + n;
      w[t][s] = (r < R && j < J) ? lam[r] * (double)A[i * R + r] * (double)B[j * R + r] : 0.0;
    }
  const double sc = fmt == MTK_FP8_E4M3 ? ldexp(1.0, slice_exp[i]) : 1.0;
  // This wave's X values of a k tile, loaded one tile ahead.
  float xq[JT][4];
  auto x_load = [&](int64_t k0) {
    const int64_t kc = k0 + n;
    const bool k_ok = kc < K;
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = jw + 16 * t + g + 4 * v;
        const bool ok = j < J && k_ok;
        const int64_t off = ok ? (i * J + j) * K + kc : 0;
        xq[t][v] = fmt == MTK_FP8_E4M3 ? (float)static_cast<const uint8_t*>(X)[off]
                                       : static_cast<const float*>(X)[off];
      }
  };
  double res = 0.0, nrm = 0.0;
  c_load(0);
  x_load(0);
  c_store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    const int64_t kc = k0 + n;
    const bool k_ok = kc < K;
    double xv[JT][4];
#pragma unroll
    for (int t = 0; t < JT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        xv[t][v] = fmt == MTK_FP8_E4M3 ? e4m3_to_double((uint8_t)xq[t][v]) * sc : (double)xq[t][v];
    const bool more = k0 + 16 < K;
    if (more) {
      c_load(k0 + 16);
      x_load(k0 + 16);
    }
#pragma unroll
    for (int t = 0; t < JT; ++t) {
      d4 m = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < RQ; ++s) m = __builtin_amdgcn_mfma_f64_16x16x4f64(w[t][s], cl[buf][n][4 * s + g], m, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = jw + 16 * t + g + 4 * v;
        if (j < J && k_ok) {
          const double x = xv[t][v];
          const double d = x - m[v];
          res = fma(d, d, res);
          nrm = fma(x, x, nrm);
        }
      }
    }
    if (more) c_store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  sr[tid] = res;
  sn[tid] = nrm;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) { sr[tid] += sr[tid + h]; sn[tid] += sn[tid + h]; }
    __syncthreads();
  }
  if (tid == 0) {
    part[2 * b] = sr[0];
    part[2 * b + 1] = sn[0];
  }
  __syncthreads();                    // sr / sn are reused by the next item
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

SrvUpdate srv_update(const int64_t dims[3], int R, int mode, int64_t maxdim, void* solve_ws_p, const float* M,
                     int S, int64_t sstride, float* fout, double* lam, int* status) {
  SolveWs w = solve_ws(maxdim, R, solve_ws_p);
  SrvUpdate u{};
  u.fa = factor_args(dims, R, mode, maxdim, solve_ws_p, status);
  u.M = M;
  u.S = S;
  u.sstride = sstride;
  u.n = dims[mode];
  u.R = R;
  u.nblk = (int)cdiv(u.n, kApplyRows);
  u.nrb = gram_blocks(u.n, R);
  u.F = w.F;
  u.colsq = w.colsq;
  u.lam = lam;
  u.fout = fout;
  u.gram_out = w.part[mode];
  u.status = status;
  return u;
}

int64_t srv_apply_blocks(const SrvUpdate& u) { return (int64_t)u.nblk * ((u.R + 15) / 16); }
int64_t srv_normalize_blocks(const SrvUpdate& u) { return (int64_t)gram_pairs(u.R) * u.nrb; }

size_t srv_factor_lds_bytes(int max_rank) { return factor_gj_lds_bytes(max_rank); }

hipError_t launch_srv_factor(const SrvTable* t, int u, int max_rank, hipStream_t st) {
  hipLaunchKernelGGL(srv_factor_kernel, dim3(kSrvMaxReq), dim3(256), srv_factor_lds_bytes(max_rank), st, t, u);
  return hipGetLastError();
}

hipError_t launch_srv_apply(const SrvTable* t, int u, hipStream_t st) {
  hipLaunchKernelGGL(srv_apply_kernel, dim3(kSrvApplyGrid), dim3(256), 0, st, t, u);
  return hipGetLastError();
}

hipError_t launch_srv_normalize(const SrvTable* t, int u, hipStream_t st) {
  hipLaunchKernelGGL(srv_normalize_kernel, dim3(kSrvNormalizeGrid), dim3(256), 0, st, t, u);
  return hipGetLastError();
}

size_t fit_ws_bytes(const int64_t dims[3]) {
  return (size_t)dims[0] * cdiv(dims[1], 16) * 2 * sizeof(double) + 256;
}

hipError_t launch_fit(const void* X, int fmt, const int32_t* slice_exp, const int64_t dims[3],
                      const float* const factors[3], const double* lambda, int R, double* acc2, void* ws,
                      hipStream_t st) {
  double* part = static_cast<double*>(ws);
  // MFMA steps RQ = R/4 rounded up to a power of two; two j tiles per wave
  // while the model operands fit in registers.
  const int rq = R <= 8 ? 2 : R <= 16 ? 4 : R <= 32 ? 8 : R <= 64 ? 16 : 32;
  const int jt = rq <= 16 ? 2 : 1;
  const int64_t nbx = cdiv(dims[1], 64 * jt);
  // One workgroup per (slice, j block) up to a grid of 2^20; beyond that the
  // workgroups stride over the items (same partials, same order).
  const int64_t items = dims[0] * nbx;
  const dim3 grid((unsigned)std::min<int64_t>(items, (int64_t)1 << 20));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, X, fmt, slice_exp, dims[0], dims[1], dims[2], factors[0],
                       factors[1], factors[2], lambda, R, nbx, part);
  };
  switch (rq) {
    case 2: go(fit_partial_kernel<2, 2>); break;
    case 4: go(fit_partial_kernel<4, 2>); break;
    case 8: go(fit_partial_kernel<8, 2>); break;
    case 16: go(fit_partial_kernel<16, 2>); break;
    default: go(fit_partial_kernel<32, 1>); break;
  }
  hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(256), 0, st, part, dims[0] * nbx, acc2);
  return hipGetLastError();
}

namespace {
// ||X||^2 partials (FP64): block b sums elements b, b + nb, ... of its
// grid-stride share in order and writes the pair (0, sum) for fit_final_kernel.
__global__ __launch_bounds__(256) void sumsq_kernel(const void* __restrict__ X, int fmt,
                                                    const int32_t* __restrict__ slice_exp, int64_t n, int64_t slice,
                                                    double* __restrict__ part) {
  double t = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double x;
    if (fmt == MTK_FP8_E4M3) x = e4m3_to_double(static_cast<const uint8_t*>(X)[e]) * ldexp(1.0, slice_exp[e / slice]);
    else x = (double)static_cast<const float*>(X)[e];
    t = fma(x, x, t);
  }
  __shared__ double red[256];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = 0.0;
    part[2 * blockIdx.x + 1] = red[0];
  }
}
}  // namespace

hipError_t launch_sumsq(const void* X, int fmt, const int32_t* slice_exp, const int64_t dims[3], double* acc2,
                        void* ws, hipStream_t st) {
  double* part = static_cast<double*>(ws);
  const int64_t n = dims[0] * dims[1] * dims[2];
  // fit_ws_bytes holds at least dims[0] pairs; 1024 blocks at most.
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>({1024, dims[0], cdiv(n, 256)}));
  hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)nb), dim3(256), 0, st, X, fmt, slice_exp, n, dims[1] * dims[2], part);
  hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(256), 0, st, part, nb, acc2);
  return hipGetLastError();
}

}  // namespace mtk
