// Dimension-tree MTTKRP for the first two updates of a CP-ALS sweep.
//
// The mode-1 and mode-2 MTTKRPs share the contraction with C:
//
//   Y(i, j, r) = sum_k X(i, j, k) C(k, r)                (one pass over X)
//   M1(i, r)   = sum_j Y(i, j, r) B(j, r)
//   M2(j, r)   = sum_i Y(i, j, r) A(i, r)
//
// and C does not change between the two updates (modes are updated in the
// order 1, 2, 3), so Y is formed once per sweep and the sweep reads X twice
// instead of three times.  Y is I*J x R FP32 (1/K of X's elements per rank
// column), kept in the sweep's workspace.
//
// ttm_kernel: X seen as the (I*J) x K row-major matrix, Y = X C.  A wave owns
// RT tiles of 16 consecutive rows for the whole reduction, so every Y entry
// is finished in one wave's accumulators and written once.  C passes through
// LDS in chunks of kw = 4*nv rows (double-buffered, one barrier per chunk);
// each wave reads its MFMA B-operand fragment of the chunk from there and
// uses it for all its row tiles.  The X tiles of the next chunk are loaded
// while the current chunk's MFMAs run.
//
// ysum_kernel: the two sums over Y with the weight factor, split over the
// summed index into partial slices that the slice reduction adds in fixed
// order.

#include "mtk_internal.h"
#include "factor_device.h"
#include "tile_device.h"

#include <algorithm>
#include <type_traits>

namespace mtk {
namespace {

// Reduction values per lane and row tiles per wave: fragment (nt*nv
// registers) and accumulators (rt*nt*4) sized like the contraction's.
#ifndef MTK_TTM_NV_A
#define MTK_TTM_NV_A 16
#endif
#ifndef MTK_TTM_RT_A
#define MTK_TTM_RT_A 4
#endif
#ifndef MTK_TTM_NV_B
#define MTK_TTM_NV_B 8
#endif
#ifndef MTK_TTM_RT_B
#define MTK_TTM_RT_B 4
#endif
template <int NT> struct TtmShape {
  static constexpr int nv = NT <= 2 ? MTK_TTM_NV_A : (NT <= 4 ? MTK_TTM_NV_B : 8);
  static constexpr int rt = NT <= 2 ? MTK_TTM_RT_A : (NT <= 4 ? MTK_TTM_RT_B : 2);
};

struct TtmArgs {
  const float* X;     // P x K row-major
  const float* C;     // K x R row-major
  float* Y;           // P x R row-major
  int64_t P;
  int K, R;
  int job_on;         // 1: workgroup 0 inverts job's V, the rest shift by one
  FactorArgs job;
  // Optional sum M1(i, r) = sum_j Y(i, j, r) B(j, r) while Y is formed, for
  // J a multiple of a workgroup's rows (each workgroup's rows share one i):
  // workgroup b writes the partial row m1part[s][i][:] of its J-block s.
  const float* B;     // J x R, or nullptr
  float* m1part;      // (J / rows per workgroup) x I x R
  int J;
  int64_t I;
};

__device__ __forceinline__ void run_factor_job(const FactorArgs& f, void* lds) {
  if (f.R <= 16) factor_gj<1, true>(f, static_cast<double*>(lds));
  else factor_gj<2, true>(f, static_cast<double*>(lds));
}

template <int PREC, int NT, int NV, bool VEC>
__global__ __launch_bounds__(256) void ttm_kernel(TtmArgs a) {
  extern __shared__ float lds[];
  if constexpr (NT <= 2) {
    if (a.job_on && blockIdx.x == 0) {
      run_factor_job(a.job, lds);
      return;
    }
  }
  constexpr int KW = 4 * NV;
  constexpr int RT = TtmShape<NT>::rt;
  constexpr int SC = (KW * NT * 16 + 255) / 256;     // staged C values per thread per chunk
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n = lane & 15;          // A-operand row / B-operand column of this lane
  const int g = lane >> 4;          // reduction group of this lane
  const int R = a.R, K = a.K;
  const int64_t blk = (int64_t)blockIdx.x - a.job_on;
  const int64_t p0 = (blk * 4 + wave) * (16 * RT);
  const int chunk = KW * R;                           // C floats per chunk (rows k contiguous)
  const int nch = (K + KW - 1) / KW;
  // Workgroup b takes the chunks in the order b, b+1, ... (mod nch), so that
  // concurrent workgroups read different column ranges of their rows and
  // spread over the HBM channels.
#ifndef MTK_TTM_ROT
#define MTK_TTM_ROT 1
#endif
  const int rot = MTK_TTM_ROT ? (int)(blk % nch) : 0;
  auto chunk_of = [&](int c) { const int cc = c + rot; return cc >= nch ? cc - nch : cc; };
  const int64_t ctot = (int64_t)K * R;
  // A chunk sits in LDS transposed, CT[col][kk] with row stride LDK (the
  // 4-float pad puts the 8 lanes of a 16-byte read on distinct banks), so a
  // lane reads its nv fragment values of a column as 16-byte vectors.
  constexpr int LDK = KW + 4;
  constexpr int kBuf = NT * 16 * LDK;                 // floats per chunk buffer
  const float inv_r = 1.f / (float)R;

  // Staging is branch-free: out-of-range values load C[0] and are zeroed.
  // Element e of the chunk is C row kk = e / R (exact in FP32 for e < 2^12),
  // column e - kk R.  The zeroing happens at the store, so nothing between
  // the loads (issued at a chunk's start) and the store (at its end) waits
  // for them.
  auto stage_ok = [&](int c, int q) {
    const int e = tid + 256 * q;
    return e < chunk && (int64_t)c * chunk + e < ctot;
  };
  auto stage_load = [&](float (&s)[SC], int c) {
#pragma unroll
    for (int q = 0; q < SC; ++q)
      s[q] = a.C[stage_ok(c, q) ? (int64_t)c * chunk + tid + 256 * q : 0];
  };
  auto stage_store = [&](const float (&s)[SC], int c, float* b) {
#pragma unroll
    for (int q = 0; q < SC; ++q) {
      const int e = tid + 256 * q;
      const int kk = (int)(((float)e + 0.5f) * inv_r);
      // Values past the chunk (zeros) go to the unread pad of row 0.
      b[e < chunk ? (e - kk * R) * LDK + kk : KW] = stage_ok(c, q) ? s[q] : 0.f;
    }
  };
  auto frag_load = [&](Frag<PREC, NT, NV>& fr, const float* b) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 16 + n;
      const bool ok = col < R;
      const float4* bc = reinterpret_cast<const float4*>(b + col * LDK + g * NV);
      if constexpr (PREC == MTK_FP32) {
#pragma unroll
        for (int e4 = 0; e4 < NV / 4; ++e4) {
          const float4 v = bc[e4];
          fr.f[t][4 * e4 + 0] = ok ? v.x : 0.f;
          fr.f[t][4 * e4 + 1] = ok ? v.y : 0.f;
          fr.f[t][4 * e4 + 2] = ok ? v.z : 0.f;
          fr.f[t][4 * e4 + 3] = ok ? v.w : 0.f;
        }
      } else {
#pragma unroll
        for (int s = 0; s < NV / 8; ++s)
#pragma unroll
          for (int h4 = 0; h4 < 2; ++h4) {
            const float4 v = bc[2 * s + h4];
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) frag_put(fr, t, s, 4 * h4 + e, ok ? vv[e] : 0.f);
          }
      }
    }
  };

  f4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rt][t] = zero4();

  auto run = [&](auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    XRegs<PREC, NV> x[RT];
    auto load_tile = [&](XRegs<PREC, NV>& xr, int c, int rt) {
      const int64_t row = p0 + rt * 16 + n;
      const bool row_ok = row < a.P;
      const int red0 = c * KW + g * NV;
      load_x<PREC, NV, true, VEC, FULL>(xr, a.X, (row_ok ? row : 0) * (int64_t)K + red0, 1, row_ok, red0, K);
    };
    {
      float s[SC];
      stage_load(s, chunk_of(0));
      stage_store(s, chunk_of(0), lds);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      load_tile(x[rt], chunk_of(0), rt);
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // Every chunk but the last also stages and prefetches the next one; the
    // last is peeled so that neither needs a branch.
    auto step = [&](int c, auto last_tag) {
      constexpr bool LAST = decltype(last_tag)::value;
      float s[SC];
      const int cn = chunk_of(c + 1);
      if constexpr (!LAST) stage_load(s, cn);
      __builtin_amdgcn_sched_barrier(0);             // the staging loads stay ahead, unconsumed
      Frag<PREC, NT, NV> fr;
      frag_load(fr, lds + (c & 1) * kBuf);
      __builtin_amdgcn_sched_barrier(0);             // all fragment reads before the MFMAs
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        tile_mfma<PREC, NT, NV, true>(acc[rt], x[rt], fr);
        if constexpr (!LAST) {
          __builtin_amdgcn_sched_barrier(0);
          load_tile(x[rt], cn, rt);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if constexpr (!LAST) {
        stage_store(s, cn, lds + ((c + 1) & 1) * kBuf);
        __syncthreads();
      }
    };
    for (int c = 0; c + 1 < nch; ++c) step(c, std::false_type{});
    step(nch - 1, std::true_type{});
  };
  if (p0 + 16 * RT <= a.P && K % KW == 0) run(std::true_type{});
  else run(std::false_type{});

  // Y itself (not stored when only its row sums are asked for: a.Y null).
  if (a.Y) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = t * 16 + n;
        if (col >= R) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = p0 + rt * 16 + g * 4 + v;
          if (row < a.P) a.Y[row * R + col] = acc[rt][t][v];
        }
      }
  }

  if (a.B) {
    // All rows of the workgroup have the same i (the launcher checks J).
    // Lane sums over its rows (rt, then v), then lane groups g and waves
    // in order through LDS: one fixed summation order.
    const int64_t pw = blk * (int64_t)(64 * RT);
    const int64_t i = pw / a.J;
    const int jb = (int)(pw - i * a.J);
    const int sl = jb / (64 * RT);
    float bv[RT][4][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int j = (int)(p0 - i * a.J) + rt * 16 + g * 4 + v;
          bv[rt][v][t] = a.B[(int64_t)j * R + min(t * 16 + n, R - 1)];
        }
    float sv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      sv[t] = 0.f;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) sv[t] = fmaf(acc[rt][t][v], bv[rt][v][t], sv[t]);
    }
    __syncthreads();                                  // LDS chunk buffers are free from here
    float* red = lds;                                 // [wave][g][NT * 16]
#pragma unroll
    for (int t = 0; t < NT; ++t) red[(wave * 4 + g) * (NT * 16) + t * 16 + n] = sv[t];
    __syncthreads();
    if (tid < R) {
      float m = 0.f;
      for (int q = 0; q < 16; ++q) m += red[q * (NT * 16) + tid];
      a.m1part[((int64_t)sl * a.I + i) * R + tid] = m;
    }
  }
}

struct YsumArgs {
  const float* Y;
  int64_t so, sq;     // element strides of Y along the output and the summed index
  int nO, nQ, R;
  const float* W;     // weight factor, nQ x R
  int qper;           // summed indices per slice
  float* part;        // slices x nO x R
  int job_on;
  FactorArgs job;
};

// part[s][o][r] = sum over q in slice s of Y(o, q, r) W(q, r), in q order.
// Thread (sub, r) of a workgroup owns output (ob*nsub + sub, r), nsub =
// 256 / R, so a workgroup's loads of one q cover nsub rows of R values.
__global__ __launch_bounds__(256) void ysum_kernel(YsumArgs a) {
  extern __shared__ double jlds[];
  if (a.job_on && blockIdx.x == 0) {
    run_factor_job(a.job, jlds);
    return;
  }
  const int R = a.R;
  const int nsub = 256 / R;
  const int nob = (a.nO + nsub - 1) / nsub;
  const int b = (int)blockIdx.x - a.job_on;
  const int ob = b % nob, s = b / nob;
  const int r = threadIdx.x % R, sub = threadIdx.x / R;
  const int o = ob * nsub + sub;
  if (sub >= nsub || o >= a.nO) return;
  const int q0 = s * a.qper;
  const int q1 = min(a.nQ, q0 + a.qper);
  const float* y = a.Y + o * a.so + r;
  const float* w = a.W + r;
  float acc = 0.f;
#pragma unroll 8
  for (int q = q0; q < q1; ++q) acc = fmaf(y[q * a.sq], w[(int64_t)q * R], acc);
  a.part[((int64_t)s * a.nO + o) * R + r] = acc;
}

template <int PREC, int NT>
hipError_t launch_ttm_nt(const TtmArgs& a, bool vec, hipStream_t st) {
  constexpr int NV = TtmShape<NT>::nv;
  constexpr int RT = TtmShape<NT>::rt;
  const int64_t rows_per_wg = 64 * RT;
  const int64_t grid = (a.P + rows_per_wg - 1) / rows_per_wg + a.job_on;
  size_t lds = 2 * (size_t)NT * 16 * (4 * NV + 4) * sizeof(float);
  if (a.job_on) lds = std::max(lds, factor_gj_lds_bytes(a.job.R));
  if (vec)
    hipLaunchKernelGGL((ttm_kernel<PREC, NT, NV, true>), dim3((unsigned)grid), dim3(256), lds, st, a);
  else
    hipLaunchKernelGGL((ttm_kernel<PREC, NT, NV, false>), dim3((unsigned)grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_ttm_prec(const TtmArgs& a, bool vec, hipStream_t st) {
  switch ((a.R + 15) / 16) {
    case 1: return launch_ttm_nt<PREC, 1>(a, vec, st);
    case 2: return launch_ttm_nt<PREC, 2>(a, vec, st);
    case 3: return launch_ttm_nt<PREC, 3>(a, vec, st);
    case 4: return launch_ttm_nt<PREC, 4>(a, vec, st);
    case 5: return launch_ttm_nt<PREC, 5>(a, vec, st);
    case 6: return launch_ttm_nt<PREC, 6>(a, vec, st);
    case 7: return launch_ttm_nt<PREC, 7>(a, vec, st);
    case 8: return launch_ttm_nt<PREC, 8>(a, vec, st);
  }
  return hipErrorInvalidValue;
}

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Slices of a Y sum: about 1024 workgroups in all, at least 8 summed indices each.
void ysum_split(int nO, int nQ, int R, int& slices, int& qper) {
  const int nob = (int)cdiv64(nO, 256 / R);
  int s = (int)std::min<int64_t>(std::max<int64_t>(1, cdiv64(1024, nob)), std::max(1, nQ / 8));
  qper = (int)cdiv64(nQ, s);
  slices = (int)cdiv64(nQ, qper);
}

size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

// Rows of Y per workgroup of the Y kernel (64 per row tile).
int ttm_rows_per_wg(int R) {
  const int nt = (R + 15) / 16;
  return 64 * (nt <= 2 ? MTK_TTM_RT_A : (nt <= 4 ? MTK_TTM_RT_B : 2));
}

// Partial slices of M1 summed inside the Y kernel, or 0 where J is not a
// multiple of its rows per workgroup (then the Y-sum kernel runs).
int64_t ttm_fused_slices(const int64_t dims[3], int R) {
  const int rw = ttm_rows_per_wg(R);
  return dims[1] % rw == 0 ? dims[1] / rw : 0;
}

}  // namespace

// Mode-1 MTTKRP from the Y kernel's row sums with Y itself not stored:
// M1(i, r) = sum_j B(j, r) sum_k X(i, j, k) C(k, r), each workgroup's rows
// (one i, a block of j) summed inside it in fixed order, then the J blocks'
// partial rows added in order.  X is read row by row (rows of K elements),
// where the contraction's 16-row tiles would take rows J*K apart.  For J a
// multiple of the kernel's rows per workgroup (m1_slices > 0); `ws` holds
// m1_ws_bytes.
int64_t ttm_m1_slices(const int64_t dims[3], int R) { return ttm_fused_slices(dims, R); }

size_t ttm_m1_ws_bytes(const int64_t dims[3], int R) {
  const int64_t s = ttm_fused_slices(dims, R);
  return s > 1 ? r256((size_t)s * dims[0] * R * sizeof(float)) : 0;
}

hipError_t launch_ttm_m1(const float* X, bool x_aligned16, const int64_t dims[3], const float* const factors[3],
                         int R, int prec, float* out, void* ws, hipStream_t st, const FactorArgs* job) {
  const int64_t fused = ttm_fused_slices(dims, R);
  if (fused < 1 || (prec != MTK_FP32 && prec != MTK_BF16X3 && prec != MTK_BF16X6) || R < 1 || R > kMaxRank ||
      dims[0] * dims[1] > kDimtreeMaxRows || (job && (job->R > kJobMaxRank || R > 32)))
    return hipErrorInvalidValue;
  TtmArgs t{};
  t.X = X;
  t.C = factors[2];
  t.Y = nullptr;
  t.P = dims[0] * dims[1];
  t.K = (int)dims[2];
  t.R = R;
  t.job_on = job ? 1 : 0;
  if (job) t.job = *job;
  t.B = factors[1];
  t.m1part = fused > 1 ? static_cast<float*>(ws) : out;
  t.J = (int)dims[1];
  t.I = dims[0];
  const bool vec = x_aligned16 && dims[2] % 4 == 0;
  hipError_t e = prec == MTK_FP32     ? launch_ttm_prec<MTK_FP32>(t, vec, st)
                 : prec == MTK_BF16X3 ? launch_ttm_prec<MTK_BF16X3>(t, vec, st)
                                      : launch_ttm_prec<MTK_BF16X6>(t, vec, st);
  if (e != hipSuccess) return e;
  if (fused > 1) return launch_slice_reduce(static_cast<float*>(ws), (int)fused, dims[0] * R, out, st);
  return hipSuccess;
}

bool dimtree_used(const int64_t dims[3], int R, int prec) {
  // Y costs one write and two reads of I*J*R floats against the saved pass
  // over I*J*K elements: worth it from K >= 8 R.
  return prec != MTK_FP8_E4M3 && dims[2] >= 8 * (int64_t)R && dims[0] * dims[1] <= kDimtreeMaxRows;
}

size_t dimtree_ws_bytes(const int64_t dims[3], int R) {
  int s0, q0, s1, q1;
  ysum_split((int)dims[0], (int)dims[1], R, s0, q0);
  ysum_split((int)dims[1], (int)dims[0], R, s1, q1);
  const size_t fs = (size_t)ttm_fused_slices(dims, R);
  const size_t part = std::max({(size_t)s0 * dims[0], (size_t)s1 * dims[1], fs * dims[0]}) * R * sizeof(float);
  return r256((size_t)dims[0] * dims[1] * R * sizeof(float)) + r256(part);
}

hipError_t launch_dimtree_mttkrp(int mode, bool form_y, const float* X, bool x_aligned16, const int64_t dims[3],
                                 const float* const factors[3], int R, int prec, float* out, void* ws,
                                 hipStream_t st, const FactorArgs* job, MSlices* defer) {
  if ((mode != 0 && mode != 1) || (prec != MTK_FP32 && prec != MTK_BF16X3 && prec != MTK_BF16X6) || R < 1 ||
      R > kMaxRank)
    return hipErrorInvalidValue;
  if (job && job->R > kJobMaxRank) return hipErrorInvalidValue;
  const int64_t I = dims[0], J = dims[1], K = dims[2];
  if (I * J > kDimtreeMaxRows) return hipErrorInvalidValue;
  float* Y = static_cast<float*>(ws);
  float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + r256((size_t)I * J * R * sizeof(float)));
  hipError_t e;
  // Mode 0 with Y formed here: M1 comes out of the Y kernel when J allows.
  const int64_t fused = (mode == 0 && form_y) ? ttm_fused_slices(dims, R) : 0;
  if (form_y) {
    TtmArgs t{};
    t.X = X;
    t.C = factors[2];
    t.Y = Y;
    t.P = I * J;
    t.K = (int)K;
    t.R = R;
    t.job_on = (job && mode == 0) ? 1 : 0;
    if (t.job_on) t.job = *job;
    if (fused) {
      t.B = factors[1];
      t.m1part = fused > 1 ? part : out;
      t.J = (int)J;
      t.I = I;
    }
    const bool vec = x_aligned16 && K % 4 == 0;
    e = prec == MTK_FP32     ? launch_ttm_prec<MTK_FP32>(t, vec, st)
        : prec == MTK_BF16X3 ? launch_ttm_prec<MTK_BF16X3>(t, vec, st)
                             : launch_ttm_prec<MTK_BF16X6>(t, vec, st);
    if (e != hipSuccess) return e;
    if (fused) {
      if (defer) {
        *defer = MSlices{fused > 1 ? part : out, (int)fused, I * R};
        return hipSuccess;
      }
      if (fused > 1) return launch_slice_reduce(part, (int)fused, I * R, out, st);
      return hipSuccess;
    }
  }
  YsumArgs y{};
  y.Y = Y;
  y.R = R;
  if (mode == 0) {            // M1(i, r) = sum_j Y(i, j, r) B(j, r)
    y.so = J * R; y.sq = R; y.nO = (int)I; y.nQ = (int)J; y.W = factors[1];
  } else {                    // M2(j, r) = sum_i Y(i, j, r) A(i, r)
    y.so = R; y.sq = J * R; y.nO = (int)J; y.nQ = (int)I; y.W = factors[0];
  }
  int slices;
  ysum_split(y.nO, y.nQ, R, slices, y.qper);
  y.part = slices > 1 ? part : out;
  size_t lds = 0;
  if (mode == 1 && job) {
    y.job_on = 1;
    y.job = *job;
    lds = factor_gj_lds_bytes(job->R);
  }
  const int64_t grid = cdiv64(y.nO, 256 / R) * slices + y.job_on;
  hipLaunchKernelGGL(ysum_kernel, dim3((unsigned)grid), dim3(256), lds, st, y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (defer) {
    *defer = MSlices{slices > 1 ? part : out, slices, (int64_t)y.nO * R};
    return hipSuccess;
  }
  if (slices > 1) return launch_slice_reduce(part, slices, (int64_t)y.nO * R, out, st);
  return hipSuccess;
}

}  // namespace mtk
