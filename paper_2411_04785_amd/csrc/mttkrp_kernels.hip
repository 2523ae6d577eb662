// Dense 3-way MTTKRP on CDNA4 matrix cores.
//
// All three modes are one contraction pattern.  Write the tensor element as
// X(m, red, loop) with element offset m*sM + red*sRed + loop*sLoop:
//
//   mode 0: m = i, red = k, loop = j   M(i,r) = sum_j B(j,r) sum_k X C(k,r)
//   mode 1: m = j, red = k, loop = i   M(j,r) = sum_i A(i,r) sum_k X C(k,r)
//   mode 2: m = k, red = j, loop = i   M(k,r) = sum_i A(i,r) sum_j X B(j,r)
//
// The Khatri-Rao row of the definition, W((loop, red), r) = F(loop,r) G(red,r),
// factors into a "fragment" factor G (applied inside the MFMA along the
// reduction) and a "weight" factor F (applied once per (loop, m, r) in the
// epilogue).  Each W entry is thus generated implicitly and never stored:
// the fragment of G a wave needs stays in registers as MFMA B-operands for
// the whole kernel, and F is a per-column scale of each finished tile.
//
// Work decomposition.  A wave owns a reduction window of kw = 4*nv values,
// an M-tile of 16 output rows and a block of loop iterations.  Per loop
// iteration it streams the 16 x kw tile of X (A-operand, lane (m, g) holds
// row m and the nv contiguous reduction values g*nv .. g*nv+nv-1 -- any
// consistent pairing of A and B lane elements is a valid MFMA reduction
// order), runs nt MFMA chains (one per 16 columns of R) into a fresh tile T,
// and adds F(loop, r) * T into its accumulator.  Workgroups are 4 waves:
// for modes 0/1 (contiguous reduction) up to 4 waves cover adjacent
// reduction windows of the same rows and are summed through LDS in fixed
// order; for mode 2 the 4 waves cover 4 adjacent M-tiles (64 consecutive k).
// Each workgroup writes one partial slice; a second kernel sums the slices
// in fixed order.  Every sum therefore has an order fixed by
// (dims, R, mode, precision) alone, so results are bitwise reproducible.

#include "mtk_internal.h"
#include "srv_internal.h"
#include "factor_device.h"
#include "fp8_codec.h"
#include "tile_device.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

namespace mtk {
namespace {

struct KArgs {
  const void* X;
  const int32_t* slice_exp;   // FP8 tensor: per mode-1 slice exponent
  const float* frag_src;      // fragment factor G, nRed x R (FP32 / BF16X3 / BF16X6)
  const uint8_t* frag_q;      // FP8: e4m3 codes of G, column-major R x red_pad, hi then lo plane
  int red_pad;                // FP8: padded column length of frag_q (covers every window)
  const int32_t* frag_exp;    // FP8: per-column exponent of G
  const float* weight;        // weight factor F, nLoop x R
  float* part;                // slices x nM x R (or the output when slices == 1)
  int64_t sM, sRed, sLoop;
  int nM, nRed, nLoop, R;
  int wr, mt_per_wg, n_rg, n_mg, loop_block, n_lb;
  int ncg;                    // column groups: waves splitting R over the same tile
  int cb0;                    // first column of the workgroup (grouped launches: column tile * 16)
  int mode;
  int job_on;                 // 1: workgroup 0 inverts job's V, the rest shift by one
  FactorArgs job;
};

// The inversion of an update's V (R <= kJobMaxRank) run by one extra
// workgroup of a contraction launch, so that it overlaps the contraction
// with no launch or stream dependency of its own.  It is workgroup 0, the
// first dispatched, so it starts with the contraction rather than in its
// last wave.  Only the instantiations with at most 2 column tiles (R <= 32)
// carry it.
__device__ __forceinline__ bool run_job(const KArgs& a, float* lds) {
  if (!a.job_on || blockIdx.x != 0) return false;
  if (a.job.R <= 16) factor_gj<1, true>(a.job, reinterpret_cast<double*>(lds));
  else factor_gj<2, true>(a.job, reinterpret_cast<double*>(lds));
  return true;
}

// Copy a workgroup's epilogue weights into LDS: the rows F(l0..l1-1, :) are
// contiguous (n floats from w).  Each thread sends kStageBatch loads before it
// stores any, so the copy costs a few memory round trips instead of one per
// element.  SCALE (FP8 modes 1, 2) multiplies row il by 2^sexp[il]; the row
// of element e is floor((e + 1/2) / R), exact in FP32 for e < 2^22 (n is at
// most MTK_STAGE_FLOATS).
constexpr int kStageBatch = 8;
template <bool SCALE>
__device__ __forceinline__ void stage_weights(float* wl, const float* w, int n, int R, const int32_t* sexp) {
  const float inv_r = 1.f / (float)R;
  for (int base = threadIdx.x; base < n; base += 256 * kStageBatch) {
    float v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) v[u] = w[min(base + 256 * u, n - 1)];
    if constexpr (SCALE) {
      int ex[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int e = min(base + 256 * u, n - 1);
        ex[u] = sexp[(int)(((float)e + 0.5f) * inv_r)];
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) v[u] = ldexpf(v[u], ex[u]);
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (base + 256 * u < n) wl[base + 256 * u] = v[u];
  }
}

// Most 16-column MFMA tiles one FP8 wave holds (its two-term fragment takes
// 16 VGPRs per tile at nv = 32); waves of a workgroup split wider ranks.
// Eight: up to R = 128 one wave holds every column tile (128 fragment
// VGPRs), because two waves sharing an X tile each load it, and those
// duplicate loads cost more than the lost occupancy (768^3: 16-row x
// 128-byte tiles stream at 3.7 TB/s loaded twice, 5.3-5.7 TB/s once, the
// latter also at one workgroup per CU).
#ifndef MTK_FP8_NTW
#define MTK_FP8_NTW 8
#endif
// FP8 waves of more than four column tiles, held to two waves per SIMD so
// that one wave's epilogue issues while the other's MFMAs run (1: one wave
// per SIMD, with the epilogue interleaved into the MFMAs instead).
#ifndef MTK_FP8_WIDE_WAVES
#define MTK_FP8_WIDE_WAVES 2
#endif
// Most fragment VGPRs per lane an FP8 plan gives a wave (sets its nv; nv
// does not go below 32).
#ifndef MTK_FP8_FRAG_REGS
#define MTK_FP8_FRAG_REGS 64
#endif

// Tiles kept in flight per wave: deeper for small tiles so that every CU has
// enough bytes outstanding to cover the HBM latency.
#ifndef MTK_PIPE_FP8
#define MTK_PIPE_FP8 4
#endif
// Tiles in flight of an FP8 wave holding more than four column tiles: at
// two waves per SIMD its fragment leaves room for two (a third spills).
#ifndef MTK_PIPE_FP8_WIDE
#define MTK_PIPE_FP8_WIDE 2
#endif
#ifndef MTK_PIPE_SMALL
#define MTK_PIPE_SMALL 3
#endif
template <int PREC, int NV> struct PipeDepth {
  static constexpr int tile_vgprs = (PREC == MTK_FP8_E4M3) ? NV / 4 : NV;
  static constexpr int value = PREC == MTK_FP8_E4M3 ? MTK_PIPE_FP8
                               : (tile_vgprs <= 8 ? 4 : (tile_vgprs <= 16 ? MTK_PIPE_SMALL : 2));
};

template <int PREC, int NT, int NV>
__device__ __forceinline__ void load_frag(Frag<PREC, NT, NV>& fr, const KArgs& a, int red0, int n, int cb) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = cb + t * 16 + n;
    const bool col_ok = col < a.R;
    if constexpr (PREC == MTK_FP32) {
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        const int red = red0 + e;
        fr.f[t][e] = (col_ok && red < a.nRed) ? a.frag_src[(int64_t)red * a.R + col] : 0.f;
      }
    } else if constexpr (PREC == MTK_BF16X3 || PREC == MTK_BF16X6) {
#pragma unroll
      for (int s = 0; s < NV / 8; ++s) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int red = red0 + s * 8 + e;
          const float v = (col_ok && red < a.nRed) ? a.frag_src[(int64_t)red * a.R + col] : 0.f;
          frag_put(fr, t, s, e, v);
        }
      }
    } else {
      // Codes are column-major, zero-padded to red_pad >= every window end.
      const int64_t plane = (int64_t)a.R * a.red_pad;
      const uint8_t* ph = a.frag_q + (int64_t)(col_ok ? col : 0) * a.red_pad + red0;
#pragma unroll
      for (int s = 0; s < NV / 32; ++s) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // Past R the lane holds column 0's codes: its MFMA output column is
          // never stored and its epilogue weight is zero.  With no select,
          // all fragment loads go out together.
          const int o = fp8_piece_off(s * 32 + h * 16);
          const uint4 u = *reinterpret_cast<const uint4*>(ph + o);
          const uint4 ul = *reinterpret_cast<const uint4*>(ph + plane + o);
          fr.q[t][s][4 * h + 0] = (int)u.x; fr.q[t][s][4 * h + 1] = (int)u.y;
          fr.q[t][s][4 * h + 2] = (int)u.z; fr.q[t][s][4 * h + 3] = (int)u.w;
          fr.ql[t][s][4 * h + 0] = (int)ul.x; fr.ql[t][s][4 * h + 1] = (int)ul.y;
          fr.ql[t][s][4 * h + 2] = (int)ul.z; fr.ql[t][s][4 * h + 3] = (int)ul.w;
        }
      }
      fr.sh[t] = 127 + a.frag_exp[col_ok ? col : 0];
      fr.sl[t] = 127 + a.frag_exp[a.R + (col_ok ? col : 0)];
    }
  }
}

// One workgroup's share of a contraction launch: workgroup `bid` of the
// plan in `a` (dyn_lds: the launch's dynamic LDS).  The waves that added
// their partial tiles into another wave's return early.
template <int PREC, int NT, int NV, bool CONTIG, bool VEC, bool GROUPED = false>
__device__ __forceinline__ void contract_body(const KArgs& a, int bid, float* dyn_lds) {
  constexpr int KW = 4 * NV;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m_l = lane & 15;      // A-operand row / B-operand column of this lane
  const int g = lane >> 4;        // reduction element group of this lane

  // Workgroup -> (reduction group, M group, loop block); the reduction group
  // varies fastest so neighbouring workgroups read neighbouring windows.
  const int rg = bid % a.n_rg; bid /= a.n_rg;
  const int mg = bid % a.n_mg; bid /= a.n_mg;
  const int lb = bid;

  // Wave -> (column group, reduction window, M-tile) inside the workgroup.
  const int cg = wave % a.ncg;
  const int wred = (wave / a.ncg) % a.wr;
  const int wm = wave / (a.ncg * a.wr);
  const int cb = (GROUPED ? a.cb0 : 0) + cg * NT * 16;   // first column of this wave
  const int win = rg * a.wr + wred;                   // reduction window of this wave
  const int red_base = win * KW;
  // This lane's first reduction value (FP8: its first 16-byte piece).
  const int red0 = red_base + g * (PREC == MTK_FP8_E4M3 ? 16 : NV);
  const int mt = mg * a.mt_per_wg + wm;               // M-tile of this wave
  const int m0 = mt * 16;
  const int row = m0 + m_l;
  const bool row_ok = row < a.nM;
  const bool tile_full = (m0 + 16 <= a.nM) && (red_base + KW <= a.nRed);

  Frag<PREC, NT, NV> fr;
  load_frag<PREC, NT, NV>(fr, a, red0, m_l, cb);

  f4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = zero4();

  const int l0 = lb * a.loop_block;
  const int l1 = min(a.nLoop, l0 + a.loop_block);
  const int64_t off0 = (int64_t)(row_ok ? row : 0) * a.sM + (int64_t)red0 * a.sRed;

  // The block's weight rows F(l0..l1-1, :) in LDS (FP8 modes 1, 2: times the
  // slice scale 2^e_i of the loop index), read back with LDS loads so that
  // the only outstanding global loads in the loop are the X prefetches.
  float* wl = dyn_lds;
  {
    const float* w = a.weight + (int64_t)l0 * a.R;
    const int nw = (l1 - l0) * a.R;
    if (PREC == MTK_FP8_E4M3 && a.mode != 0) stage_weights<true>(wl, w, nw, a.R, a.slice_exp + l0);
    else stage_weights<false>(wl, w, nw, a.R, nullptr);
  }
  __syncthreads();

  auto step = [&](const XRegs<PREC, NV>& x, int it) {
    f4 T[NT];
    tile_mfma<PREC, NT, NV>(T, x, fr);
    const float* wr = wl + (it - l0) * a.R;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = cb + t * 16 + m_l;
      const float wv = wr[min(col, a.R - 1)];
      const float w = col < a.R ? wv : 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][v] = fmaf(w, T[t][v], acc[t][v]);
    }
  };

  // Stream over the loop block with DEPTH tiles in flight (registers).  Full
  // tiles and ragged tiles get separate straight-line loops, so the only
  // wait before a tile's MFMAs is for that tile's own loads.  Prefetches past
  // the block re-read its last tile instead of branching.
  auto run = [&](auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    constexpr int D = (PREC == MTK_FP8_E4M3 && NT > 4) ? MTK_PIPE_FP8_WIDE : PipeDepth<PREC, NV>::value;
    if (l0 >= l1) return;
    XRegs<PREC, NV> x[D];
    // The prologue loads stay in tile order: the loop head's wait is shared
    // by this path and the back edge, and must only need the oldest tile.
#pragma unroll
    for (int d = 0; d < D - 1; ++d) {
      load_x<PREC, NV, CONTIG, VEC, FULL>(x[d], a.X, off0 + (int64_t)min(l0 + d, l1 - 1) * a.sLoop, a.sRed,
                                          row_ok, red0, a.nRed);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int it = l0; it < l1; it += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int nx = min(it + d + D - 1, l1 - 1);
        load_x<PREC, NV, CONTIG, VEC, FULL>(x[(d + D - 1) % D], a.X, off0 + (int64_t)nx * a.sLoop, a.sRed,
                                            row_ok, red0, a.nRed);
        __builtin_amdgcn_sched_barrier(0);      // keep the prefetch ahead of this tile's MFMAs
        if (it + d < l1) step(x[d], it + d);
      }
    }
  };
  // Built for one wave per SIMD (MTK_FP8_WIDE_WAVES = 1), FP8 with more than
  // four column tiles per wave has nothing else to cover its epilogue: the
  // MFMAs of step s are issued between the FMAs of step s - 1 (its products
  // in Tp, its weights in wp, read from LDS at the end of step s - 1 and
  // first used in step s, so that no LDS wait falls among the MFMAs).  Same
  // products, same order of the FMAs into acc as `run`.
  auto run_pipe = [&](auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    constexpr int D = MTK_PIPE_FP8_WIDE;
    if (l0 >= l1) return;
    XRegs<PREC, NV> x[D];
#pragma unroll
    for (int d = 0; d < D - 1; ++d) {
      load_x<PREC, NV, CONTIG, VEC, FULL>(x[d], a.X, off0 + (int64_t)min(l0 + d, l1 - 1) * a.sLoop, a.sRed,
                                          row_ok, red0, a.nRed);
      __builtin_amdgcn_sched_barrier(0);
    }
    int colc[NT];
    bool colv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = cb + t * 16 + m_l;
      colc[t] = min(col, a.R - 1);
      colv[t] = col < a.R;
    }
    f4 Tp[NT];
    float wp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) { Tp[t] = zero4(); wp[t] = 0.f; }
    for (int it = l0; it < l1; it += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int nx = min(it + d + D - 1, l1 - 1);
        load_x<PREC, NV, CONTIG, VEC, FULL>(x[(d + D - 1) % D], a.X, off0 + (int64_t)nx * a.sLoop, a.sRed,
                                            row_ok, red0, a.nRed);
        __builtin_amdgcn_sched_barrier(0);
        if (it + d < l1) {
          f4 Tc[NT];
          tile_mfma<PREC, NT, NV>(Tc, x[d], fr);
          // Step l0 has no predecessor: Tp and wp are zero, and acc + 0 * 0 is acc.
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] = fmaf(colv[t] ? wp[t] : 0.f, Tp[t][v], acc[t][v]);
#pragma unroll
          for (int i = 0; i < 2 * NT * (NV / 32); ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);   // two VALU
          }
          __builtin_amdgcn_sched_barrier(0);
          const float* wr = wl + (it + d - l0) * a.R;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            Tp[t] = Tc[t];
            wp[t] = wr[colc[t]];   // its select waits for the next step
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][v] = fmaf(colv[t] ? wp[t] : 0.f, Tp[t][v], acc[t][v]);
  };
  if constexpr (PREC == MTK_FP8_E4M3 && NT > 4 && MTK_FP8_WIDE_WAVES == 1) {
    if (tile_full) run_pipe(std::true_type{});
    else run_pipe(std::false_type{});
  } else {
    if (tile_full) run(std::true_type{});
    else run(std::false_type{});
  }

  // FP8 mode 0: each output row is a slice i; apply its power-of-two scale.
  if constexpr (PREC == MTK_FP8_E4M3) {
    if (a.mode == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int orow = m0 + g * 4 + v;
        const float s = orow < a.nM ? ldexpf(1.f, a.slice_exp[orow]) : 0.f;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t][v] *= s;
      }
    }
  }

  // Sum the waves that share an M-tile (adjacent reduction windows) in LDS,
  // in fixed wave order, then write this workgroup's partial slice.
  if (a.wr > 1) {
    float* red_lds = dyn_lds + a.loop_block * a.R;   // [4 waves][NT*4][64]
    auto at = [&](int w, int k) -> float& { return red_lds[(w * NT * 4 + k) * 64 + lane]; };
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) at(wave, t * 4 + v) = acc[t][v];
    __syncthreads();
    if (wred != 0) return;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float s = at(wave, t * 4 + v);
        for (int q = 1; q < a.wr; ++q) s += at(wave + q * a.ncg, t * 4 + v);
        acc[t][v] = s;
      }
  }

  const int slice = rg * a.n_lb + lb;
  float* outp = a.part + (int64_t)slice * a.nM * a.R;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = cb + t * 16 + m_l;
    if (col >= a.R) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int orow = m0 + g * 4 + v;
      if (orow < a.nM) outp[(int64_t)orow * a.R + col] = acc[t][v];
    }
  }
}

template <int PREC, int NT, int NV, bool CONTIG, bool VEC>
__global__ __launch_bounds__(256) void contract_kernel(KArgs a) {
  extern __shared__ float dyn_lds[];
  if constexpr (NT <= 2) {
    if (run_job(a, dyn_lds)) return;
  }
  contract_body<PREC, NT, NV, CONTIG, VEC>(a, (int)blockIdx.x - a.job_on, dyn_lds);
}

// (The byte-wise load forms, for unaligned or strided X, do not fit two
// waves without spilling and keep one.)
template <int PREC, int NT, int NV, bool CONTIG, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(VEC ? MTK_FP8_WIDE_WAVES : 1)))
void contract_wide_kernel(KArgs a) {
  extern __shared__ float dyn_lds[];
  contract_body<PREC, NT, NV, CONTIG, VEC>(a, (int)blockIdx.x - a.job_on, dyn_lds);
}
template <int PREC, int NT, int NV, bool CONTIG, bool VEC>
constexpr const void* contract_entry() {
  if constexpr (PREC == MTK_FP8_E4M3 && NT > 4)
    return reinterpret_cast<const void*>(&contract_wide_kernel<PREC, NT, NV, CONTIG, VEC>);
  else
    return reinterpret_cast<const void*>(&contract_kernel<PREC, NT, NV, CONTIG, VEC>);
}

// ---------------------------------------------------------------------------
// Mode 2 with a strided reduction (X(m, red, loop), m contiguous): row-
// interleaved tiles.  A wave covers 64 consecutive rows m0 .. m0+63 as four
// MFMA row tiles; tile c holds rows m0 + 4*rho + c (rho = 0..15).  Lane
// (rho, g) reads, for each of its nv reduction values, one 16-byte vector
// X(m0+4rho .. m0+4rho+3, red, loop): component c is its A-operand element
// of tile c.  A load instruction thus reads four 256-byte contiguous runs,
// and each fragment register feeds four MFMAs.
// ---------------------------------------------------------------------------
template <int NV> struct XRegsCM { f4 v[NV]; };

template <int PREC, int NT> struct PipeDepthCM { static constexpr int value = NT == 1 ? 3 : 2; };

template <int NV, bool full>
__device__ __forceinline__ void load_x_cm(XRegsCM<NV>& x, const float* X, int64_t off, int64_t sRed,
                                          bool row_ok, int red0, int nRed) {
  const float* p = X + off;
#pragma unroll
  for (int e = 0; e < NV; ++e) {
    // Rows come in aligned groups of four (nM % 4 == 0), so a vector is all
    // in range or all out; out-of-range vectors read X[0..3] and are zeroed.
    const bool ok = full || (row_ok && red0 + e < nRed);
    const f4 u = *reinterpret_cast<const f4*>(ok ? p + (int64_t)e * sRed : X);
    x.v[e] = ok ? u : zero4();
  }
}

template <int PREC, int NT, int NV>
__device__ __forceinline__ void tile_mfma_cm(f4 (&T)[4][NT], const XRegsCM<NV>& x,
                                             const Frag<PREC, NT, NV>& fr) {
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int t = 0; t < NT; ++t) T[c][t] = zero4();
  if constexpr (PREC == MTK_FP32) {
#pragma unroll
    for (int s = 0; s < NV; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          T[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.v[s][c], fr.f[t][s], T[c][t], 0, 0, 0);
  } else {
#pragma unroll
    for (int s = 0; s < NV / 8; ++s) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float xs[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) xs[e] = x.v[s * 8 + e][c];
        split_step<PREC, NT, NV>(T[c], xs, fr, s);
      }
    }
  }

}

template <int PREC, int NT, int NV>
__global__ __launch_bounds__(256) void contract_cm_kernel(KArgs a) {
  extern __shared__ float dyn_lds[];
  if constexpr (NT <= 2) {
    if (run_job(a, dyn_lds)) return;
  }
  constexpr int KW = 4 * NV;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rho = lane & 15;      // row of each interleaved tile / B-operand column
  const int g = lane >> 4;        // reduction element group

  int bid = (int)blockIdx.x - a.job_on;
  const int rg = bid % a.n_rg; bid /= a.n_rg;
  const int mg = bid % a.n_mg; bid /= a.n_mg;
  const int lb = bid;

  const int cg = wave % a.ncg;
  const int wred = (wave / a.ncg) % a.wr;
  const int wm = wave / (a.ncg * a.wr);
  const int cb = cg * NT * 16;
  const int red_base = (rg * a.wr + wred) * KW;
  const int red0 = red_base + g * NV;
  const int m0 = (mg * a.mt_per_wg + wm) * 64;         // 64-row block of this wave
  const int row4 = m0 + 4 * rho;                        // first of this lane's 4 rows
  const bool row_ok = row4 < a.nM;
  const bool tile_full = (m0 + 64 <= a.nM) && (red_base + KW <= a.nRed);

  Frag<PREC, NT, NV> fr;
  load_frag<PREC, NT, NV>(fr, a, red0, rho, cb);

  f4 acc[4][NT];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[c][t] = zero4();

  const int l0 = lb * a.loop_block;
  const int l1 = min(a.nLoop, l0 + a.loop_block);
  const float* X = static_cast<const float*>(a.X);
  const int64_t off0 = (int64_t)(row_ok ? row4 : 0) + (int64_t)red0 * a.sRed;

  float* wl = dyn_lds;
  stage_weights<false>(wl, a.weight + (int64_t)l0 * a.R, (l1 - l0) * a.R, a.R, nullptr);
  __syncthreads();

  auto step = [&](const XRegsCM<NV>& x, int it) {
    f4 T[4][NT];
    tile_mfma_cm<PREC, NT, NV>(T, x, fr);
    const float* wr = wl + (it - l0) * a.R;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = cb + t * 16 + rho;
      const float wv = wr[min(col, a.R - 1)];
      const float w = col < a.R ? wv : 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[c][t][v] = fmaf(w, T[c][t][v], acc[c][t][v]);
    }
  };

  auto run = [&](auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    constexpr int D = PipeDepthCM<PREC, NT>::value;
    if (l0 >= l1) return;
    XRegsCM<NV> x[D];
#pragma unroll
    for (int d = 0; d < D - 1; ++d) {
      load_x_cm<NV, FULL>(x[d], X, off0 + (int64_t)min(l0 + d, l1 - 1) * a.sLoop, a.sRed, row_ok, red0, a.nRed);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int it = l0; it < l1; it += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int nx = min(it + d + D - 1, l1 - 1);
        load_x_cm<NV, FULL>(x[(d + D - 1) % D], X, off0 + (int64_t)nx * a.sLoop, a.sRed, row_ok, red0, a.nRed);
        __builtin_amdgcn_sched_barrier(0);
        if (it + d < l1) step(x[d], it + d);
      }
    }
  };
  if (tile_full) run(std::true_type{});
  else run(std::false_type{});

  if (a.wr > 1) {
    float* red_lds = dyn_lds + a.loop_block * a.R;   // [4 waves][4*NT*4][64]
    auto at = [&](int w, int k) -> float& { return red_lds[(w * 16 * NT + k) * 64 + lane]; };
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) at(wave, (c * NT + t) * 4 + v) = acc[c][t][v];
    __syncthreads();
    if (wred != 0) return;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = (c * NT + t) * 4 + v;
          float s = at(wave, k);
          for (int q = 1; q < a.wr; ++q) s += at(wave + q * a.ncg, k);
          acc[c][t][v] = s;
        }
  }

  const int slice = rg * a.n_lb + lb;
  float* outp = a.part + (int64_t)slice * a.nM * a.R;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = cb + t * 16 + rho;
    if (col >= a.R) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // MFMA output row g*4+v of tile c is tensor row m0 + 4*(g*4+v) + c.
        const int orow = m0 + 4 * (g * 4 + v) + c;
        if (orow < a.nM) outp[(int64_t)orow * a.R + col] = acc[c][t][v];
      }
  }
}

// out[e] = sum over the S partial slices of part[s][e].  A block covers 32
// consecutive elements with 8 slice groups: group q sums slices q, q+8, ...
// in increasing order, then the 8 group sums are added in group order.  The
// order depends only on S, so the result is deterministic.
__device__ __forceinline__ void splitk_reduce_body(const float* __restrict__ part, int S, int64_t n,
                                                   float* __restrict__ out, int64_t blk) {
  __shared__ float red[8][33];
  const int eo = threadIdx.x & 31;
  const int q = threadIdx.x >> 5;
  const int64_t e = blk * 32 + eo;
  // Slices q, q + 8, ... in order; their loads go out 8 at a time (clamped
  // to the last slice) ahead of the adds.
  float s = 0.f;
  if (e < n) {
    for (int k0 = q; k0 < S; k0 += 64) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)min(k0 + 8 * u, S - 1) * n + e];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + 8 * u < S) s += v[u];
    }
  }
  red[q][eo] = s;
  __syncthreads();
  if (q == 0 && e < n) {
    float t = red[0][eo];
#pragma unroll
    for (int k = 1; k < 8; ++k) t += red[k][eo];
    out[e] = t;
  }
}

__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* __restrict__ part, int S,
                                                            int64_t n, float* __restrict__ out) {
  splitk_reduce_body(part, S, n, out, blockIdx.x);
}

__device__ __forceinline__ float e4m3_decode_dev(uint32_t c) {
  const uint32_t e = (c >> 3) & 15u, m = c & 7u;
  const float v = e == 0 ? ldexpf((float)m, -9) : ldexpf(1.f + (float)m * 0.125f, (int)e - 7);
  return (c & 0x80u) ? -v : v;
}

__device__ float block_max(float m, float* smax) {
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
    __syncthreads();
  }
  const float r = smax[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void frag_quant_kernel(const float* __restrict__ G, int nRed, int R, int red_pad,
                                                         uint8_t* __restrict__ q, int32_t* __restrict__ ex) {
  const int r = blockIdx.x;
  __shared__ float smax[256];
  const int64_t plane = (int64_t)R * red_pad;
  uint8_t* qh = q + (int64_t)r * red_pad;
  uint8_t* ql = qh + plane;
  // Each pass reads the column 4 values per thread at a time (clamped to the
  // last row, loads ahead of their use); values at i >= nRed are unused.
  constexpr int U = 4;
  auto col4 = [&](int i0, float (&g)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = G[(int64_t)min(i0 + 256 * u, nRed - 1) * R + r];
  };
  float m = 0.f;
  for (int i0 = threadIdx.x; i0 < nRed; i0 += 256 * U) {
    float g[U];
    col4(i0, g);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + 256 * u < nRed) m = fmaxf(m, fabsf(g[u]));
  }
  const int eh = scale_exponent_dev(block_max(m, smax));
  const float ih = ldexpf(1.f, -eh), sh = ldexpf(1.f, eh);
  float mr = 0.f;
  for (int i0 = threadIdx.x; i0 < red_pad; i0 += 256 * U) {
    float g[U];
    col4(i0, g);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 256 * u;
      uint32_t c = 0;
      if (i < nRed) {
        c = e4m3_encode_dev(g[u] * ih);
        mr = fmaxf(mr, fabsf(g[u] - e4m3_decode_dev(c) * sh));
      }
      if (i < red_pad) qh[i] = static_cast<uint8_t>(c);
    }
  }
  const int el = scale_exponent_dev(block_max(mr, smax));
  const float il = ldexpf(1.f, -el);
  for (int i0 = threadIdx.x; i0 < red_pad; i0 += 256 * U) {
    float g[U];
    col4(i0, g);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 256 * u;
      uint32_t c = 0;
      if (i < nRed) c = e4m3_encode_dev((g[u] - e4m3_decode_dev(qh[i]) * sh) * il);
      if (i < red_pad) ql[i] = static_cast<uint8_t>(c);
    }
  }
  if (threadIdx.x == 0) {
    ex[r] = eh;
    ex[R + r] = el;
  }
}

// Grouped contraction of a serving step: work item w belongs to the entry
// whose first item is the largest one <= w; its local index splits into the
// 16-column tile (fastest) and the workgroup of that request's plan.  A
// request's items compute exactly what its own launch would, so the
// result does not depend on the other entries.  The barrier at the end of
// an item keeps the next item's LDS staging behind this item's reads.
// With `with_factor`, the first nreq items each invert one request's V
// (factor_gj, LDS within the launch's for R <= kSrvFusedMaxRank), so the
// inversion overlaps the contraction with no launch of its own.
__global__ __launch_bounds__(256) void srv_contract_kernel(const SrvTable* __restrict__ t, int upd, int with_factor) {
  extern __shared__ float dyn_lds[];
  const int nreq = t->nreq;
  const int64_t jobs = with_factor ? nreq : 0;
  const int64_t nwi = t->n_wi[upd] + jobs;
  for (int64_t w = blockIdx.x; w < nwi; w += gridDim.x) {
    if (w < jobs) {
      const FactorArgs f = t->e[w][upd].u.fa;
      double* dl = reinterpret_cast<double*>(dyn_lds);
      switch ((f.R + 15) / 16) {
        case 1: factor_gj<1>(f, dl); break;
        case 2: factor_gj<2>(f, dl); break;
        case 3: factor_gj<3>(f, dl); break;
        default: factor_gj<4>(f, dl); break;
      }
      __syncthreads();
      continue;
    }
    const int64_t wc = w - jobs;
    const int q = srv_find(nreq, wc, [&](int i) { return t->e[i][upd].wi0; });
    const SrvContract& c = t->e[q][upd].c;
    int local = (int)(wc - t->e[q][upd].wi0);
    const int ct = local % c.nct;
    local /= c.nct;
    KArgs a{};
    a.X = c.X;
    a.frag_src = c.frag;
    a.weight = c.weight;
    a.part = c.part;
    a.sM = c.sM; a.sRed = c.sRed; a.sLoop = c.sLoop;
    a.nM = c.nM; a.nRed = c.nRed; a.nLoop = c.nLoop; a.R = c.R;
    a.wr = c.wr; a.mt_per_wg = c.mt_per_wg; a.n_rg = c.n_rg; a.n_mg = c.n_mg;
    a.loop_block = c.loop_block; a.n_lb = c.n_lb;
    a.ncg = 1;
    a.cb0 = ct * 16;
    a.mode = c.mode;
    switch (c.prec * 3 + c.form) {
      case 0: contract_body<MTK_FP32, 1, 8, true, true, true>(a, local, dyn_lds); break;
      case 1: contract_body<MTK_FP32, 1, 8, true, false, true>(a, local, dyn_lds); break;
      case 2: contract_body<MTK_FP32, 1, 8, false, false, true>(a, local, dyn_lds); break;
      case 3: contract_body<MTK_BF16X3, 1, 8, true, true, true>(a, local, dyn_lds); break;
      case 4: contract_body<MTK_BF16X3, 1, 8, true, false, true>(a, local, dyn_lds); break;
      default: contract_body<MTK_BF16X3, 1, 8, false, false, true>(a, local, dyn_lds); break;
    }
    __syncthreads();
  }
}

// Grid and LDS of a launch: the contraction's, plus the job's workgroup (and
// at least its LDS) when one rides along.
inline void with_job(const KArgs& a, int64_t& grid, size_t& lds) {
  if (a.job_on) {
    grid += 1;
    lds = std::max(lds, factor_gj_lds_bytes(a.job.R));
  }
}

template <int PREC, int NT, int NV, bool CONTIG, bool VEC>
hipError_t launch_one(const KArgs& a, int64_t grid, hipStream_t st) {
  size_t lds = ((size_t)a.loop_block * a.R + (a.wr > 1 ? 4 * NT * 4 * 64 : 0)) * sizeof(float);
  with_job(a, grid, lds);
  if constexpr (PREC == MTK_FP8_E4M3 && NT > 4)
    hipLaunchKernelGGL((contract_wide_kernel<PREC, NT, NV, CONTIG, VEC>), dim3((unsigned)grid), dim3(256), lds, st, a);
  else
    hipLaunchKernelGGL((contract_kernel<PREC, NT, NV, CONTIG, VEC>), dim3((unsigned)grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int NT, int NV>
hipError_t dispatch_cv(const KArgs& a, const ContractPlan& p, hipStream_t st) {
  if (p.sRed == 1) {
    if (p.vec) return launch_one<PREC, NT, NV, true, true>(a, p.grid(), st);
    return launch_one<PREC, NT, NV, true, false>(a, p.grid(), st);
  }
  return launch_one<PREC, NT, NV, false, false>(a, p.grid(), st);
}

// nv choices: FP32 / BF16X3 {8,16,32,64}; FP8 {32,64,128}.
template <int PREC, int NT>
hipError_t dispatch_nv(const KArgs& a, const ContractPlan& p, hipStream_t st) {
  if constexpr (PREC == MTK_FP8_E4M3) {
    switch (p.nv) {
      case 32: return dispatch_cv<PREC, NT, 32>(a, p, st);
      case 64: if constexpr (NT <= 2) return dispatch_cv<PREC, NT, 64>(a, p, st); break;
      case 128: if constexpr (NT <= 1) return dispatch_cv<PREC, NT, 128>(a, p, st); break;
    }
  } else {
    switch (p.nv) {
      case 8: return dispatch_cv<PREC, NT, 8>(a, p, st);
      case 16: if constexpr (NT <= 4) return dispatch_cv<PREC, NT, 16>(a, p, st); break;
      case 32: if constexpr (NT <= 2) return dispatch_cv<PREC, NT, 32>(a, p, st); break;
      case 64: if constexpr (NT <= 1) return dispatch_cv<PREC, NT, 64>(a, p, st); break;
    }
  }
  return hipErrorInvalidValue;
}

template <int PREC, int NT>
hipError_t launch_cm(const KArgs& a, const ContractPlan& p, hipStream_t st) {
  constexpr int NV = 8;
  if (p.nv != NV) return hipErrorInvalidValue;
  size_t lds = ((size_t)a.loop_block * a.R + (a.wr > 1 ? 4 * 16 * NT * 64 : 0)) * sizeof(float);
  int64_t grid = p.grid();
  with_job(a, grid, lds);
  hipLaunchKernelGGL((contract_cm_kernel<PREC, NT, NV>), dim3((unsigned)grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

template <int PREC>
hipError_t dispatch_nt(const KArgs& a, const ContractPlan& p, hipStream_t st) {
  if constexpr (PREC != MTK_FP8_E4M3) {
    if (p.cm) {
      if (p.ntw == 1) return launch_cm<PREC, 1>(a, p, st);
      if (p.ntw == 2) return launch_cm<PREC, 2>(a, p, st);
      if (p.ntw == 3) return launch_cm<PREC, 3>(a, p, st);
      if (p.ntw == 4) return launch_cm<PREC, 4>(a, p, st);
      return hipErrorInvalidValue;
    }
  }
  if constexpr (PREC == MTK_FP8_E4M3) {
    switch (p.ntw) {
      case 1: return dispatch_nv<PREC, 1>(a, p, st);
      case 2: return dispatch_nv<PREC, 2>(a, p, st);
      case 3: return dispatch_nv<PREC, 3>(a, p, st);
      case 4: return dispatch_nv<PREC, 4>(a, p, st);
#if MTK_FP8_NTW > 4
      case 5: return dispatch_nv<PREC, 5>(a, p, st);
      case 6: return dispatch_nv<PREC, 6>(a, p, st);
      case 7: return dispatch_nv<PREC, 7>(a, p, st);
      case 8: return dispatch_nv<PREC, 8>(a, p, st);
#endif
    }
    return hipErrorInvalidValue;
  } else {
  switch (p.ntw) {
    case 1: return dispatch_nv<PREC, 1>(a, p, st);
    case 2: return dispatch_nv<PREC, 2>(a, p, st);
    case 3: return dispatch_nv<PREC, 3>(a, p, st);
    case 4: return dispatch_nv<PREC, 4>(a, p, st);
    case 5: return dispatch_nv<PREC, 5>(a, p, st);
    case 6: return dispatch_nv<PREC, 6>(a, p, st);
    case 7: return dispatch_nv<PREC, 7>(a, p, st);
    case 8: return dispatch_nv<PREC, 8>(a, p, st);
  }
  return hipErrorInvalidValue;
  }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
constexpr int64_t kMaxGridX = 0x7fffffff;

// Plan limits (compile-time so a build can be tuned without code changes):
// widest per-lane reduction run for FP32 / bf16x3.
#ifndef MTK_NV_MAX
#define MTK_NV_MAX 16
#endif
// Largest staged weight block (floats) of a workgroup.
#ifndef MTK_STAGE_FLOATS
#define MTK_STAGE_FLOATS 8192
#endif

// Most fragment VGPRs per lane a bf16x6 plan gives a wave (sets its nv).
#ifndef MTK_X6_FRAG_REGS
#define MTK_X6_FRAG_REGS 96
#endif
// Most 16-column tiles one wave of the mode-3 (row-interleaved) kernel
// holds; wider ranks split their columns over the fewest waves of a
// workgroup (each such wave streams the same X rows).
#ifndef MTK_CM_NTW
#define MTK_CM_NTW 4
#endif

// Column length of the padded FP8 fragment codes: every window of the plan.
inline int frag_red_pad(const ContractPlan& p) { return p.n_rg * p.wr * p.kw; }

}  // namespace

// The kernel a plan launches, for its occupancy.  A contiguous plan stands
// for its 16-byte-load form and a strided one for the strided form, so the
// plan -- and with it the summation order -- does not depend on the
// tensor's alignment.
template <int PREC, int NT>
const void* kernel_of_nt(const ContractPlan& p) {
  if constexpr (PREC != MTK_FP8_E4M3) {
    if (p.cm) return reinterpret_cast<const void*>(&contract_cm_kernel<PREC, NT, 8>);
  }
  const bool c = p.sRed == 1;
  auto pick = [&](auto nv_tag) -> const void* {
    constexpr int NV = decltype(nv_tag)::value;
    if (c) return contract_entry<PREC, NT, NV, true, true>();
    return contract_entry<PREC, NT, NV, false, false>();
  };
  if constexpr (PREC == MTK_FP8_E4M3) {
    if (p.nv == 32) return pick(std::integral_constant<int, 32>{});
    if constexpr (NT <= 2) if (p.nv == 64) return pick(std::integral_constant<int, 64>{});
    if constexpr (NT <= 1) if (p.nv == 128) return pick(std::integral_constant<int, 128>{});
  } else {
    if (p.nv == 8) return pick(std::integral_constant<int, 8>{});
    if constexpr (NT <= 4) if (p.nv == 16) return pick(std::integral_constant<int, 16>{});
    if constexpr (NT <= 2) if (p.nv == 32) return pick(std::integral_constant<int, 32>{});
    if constexpr (NT <= 1) if (p.nv == 64) return pick(std::integral_constant<int, 64>{});
  }
  return nullptr;
}

template <int PREC>
const void* kernel_of_prec(const ContractPlan& p) {
  switch (p.ntw) {
    case 1: return kernel_of_nt<PREC, 1>(p);
    case 2: return kernel_of_nt<PREC, 2>(p);
    case 3: return kernel_of_nt<PREC, 3>(p);
    case 4: return kernel_of_nt<PREC, 4>(p);
  }
  if (PREC != MTK_FP8_E4M3 || MTK_FP8_NTW > 4) {
    switch (p.ntw) {
      case 5: return kernel_of_nt<PREC, 5>(p);
      case 6: return kernel_of_nt<PREC, 6>(p);
      case 7: return kernel_of_nt<PREC, 7>(p);
      case 8: return kernel_of_nt<PREC, 8>(p);
    }
  }
  return nullptr;
}

// Resident workgroups per CU of a plan's kernel (its registers and the
// largest LDS a plan gives it) and the device's CU count, looked up once per
// kernel.  Two per CU on 256 CUs if the runtime cannot tell (no device).
struct Slots {
  int64_t cus, per_cu;
};
Slots plan_slots(const ContractPlan& p, int prec) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, Slots> cache;
  const void* k = prec == MTK_FP32     ? kernel_of_prec<MTK_FP32>(p)
                  : prec == MTK_BF16X3 ? kernel_of_prec<MTK_BF16X3>(p)
                  : prec == MTK_BF16X6 ? kernel_of_prec<MTK_BF16X6>(p)
                                       : kernel_of_prec<MTK_FP8_E4M3>(p);
  // LDS at the largest loop block: staged weights plus the wave-sum area.
  const size_t red = p.cm ? (size_t)4 * 16 * p.ntw * 64 : (p.wr > 1 ? (size_t)4 * p.ntw * 4 * 64 : 0);
  const size_t lds = ((size_t)std::max(1, MTK_STAGE_FLOATS / p.R) * p.R + red) * sizeof(float);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({k, lds});
  if (it != cache.end()) return it->second;
  Slots sl{256, 2};
  int dev = 0, cus = 0, per_cu = 0;
  if (k && hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds) == hipSuccess && cus > 0 && per_cu > 0) {
    sl = Slots{cus, per_cu};
  } else {
    (void)hipGetLastError();
  }
  cache[{k, lds}] = sl;
  return sl;
}

// Split the outer loop into blocks, by a cost model in units of one
// workgroup loop iteration.  Workgroups spread evenly over the CUs; a CU
// runs up to per_cu of them at once, in rounds, and its stream saturates at
// about two resident workgroups (eight waves).  So a CU with c workgroups
// at once takes rounds x (loop block + ~4 iterations of prologue: fragment
// load, weight staging, epilogue) x c / min(c, 2), and the split-K partial
// slices (written, then read by the reduction) add their bytes at the
// saturated rate.  The cheapest block count wins, fewer slices on ties;
// the staged weights must fit their LDS budget.
static void set_loop_blocks(ContractPlan& p, int prec, Slots sl) {
  const int64_t base = (int64_t)p.n_rg * p.n_mg;
  const int64_t lb_cap = std::max(1, MTK_STAGE_FLOATS / p.R);
  const double elem = prec == MTK_FP8_E4M3 ? 1.0 : 4.0;
  // Bytes of X a workgroup reads per loop iteration.
  const double it_bytes = (p.cm ? 64.0 : 16.0) * p.mt_per_wg * p.wr * p.kw * elem;
  const double slice_bytes = 2.0 * p.nM * p.R * 4.0;
  constexpr double kSat = 2.0, kPrologue = 4.0;
  const int64_t max_blocks = std::min<int64_t>(p.nLoop, std::max<int64_t>(1, 16 * sl.cus * sl.per_cu / base + 1));
  int64_t best_n = 0;
  double best_cost = 0.0;
  for (int64_t n = 1; n <= max_blocks; ++n) {
    const int64_t lb = cdiv(p.nLoop, n);
    if (lb > lb_cap) continue;
    const int64_t nb = cdiv(p.nLoop, lb);
    if (nb != n) continue;                                   // same split as a smaller n
    const int64_t grid = base * nb;
    if (grid + 1 > kMaxGridX) break;
    const int64_t per_cu = cdiv(grid, sl.cus);
    const int64_t conc = std::min(per_cu, sl.per_cu);
    const int64_t rounds = cdiv(per_cu, sl.per_cu);
    double cost = rounds * (lb + kPrologue) * conc / std::min<double>(conc, kSat);
    if (p.n_rg * nb > 1) cost += p.n_rg * nb * slice_bytes / (sl.cus * kSat * it_bytes);
    if (best_n == 0 || cost < best_cost) { best_n = nb; best_cost = cost; }
  }
  if (best_n == 0) best_n = cdiv(p.nLoop, lb_cap);          // the weight budget forces the split
  p.loop_block = (int)cdiv(p.nLoop, best_n);
  p.n_lb = (int)cdiv(p.nLoop, p.loop_block);
  p.slices = p.n_rg * p.n_lb;
}

// Waves of a workgroup along a contiguous reduction of `windows` windows:
// the largest of 4, 2, 1 (at most wmax) that leaves the fewest windows past
// the end idle.
static int pick_wr(int64_t windows, int wmax) {
  int best = 1;
  int64_t best_idle = -1;
  for (int wr = std::min(4, wmax); wr >= 1; wr /= 2) {
    const int64_t idle = cdiv(windows, wr) * wr - windows;
    if (best_idle < 0 || idle < best_idle) { best = wr; best_idle = idle; }
  }
  return best;
}

ContractPlan make_plan(const int64_t dims[3], int R, int mode, int prec, bool x_aligned16, bool transposed) {
  ContractPlan p{};
  const int64_t I = dims[0], J = dims[1], K = dims[2];
  p.R = R;
  p.nt = (int)cdiv(R, 16);
  // FP8 needs 32 reduction values per lane per MFMA; above 64 columns two
  // waves split R over the same X tile so the fragments stay in registers.
  p.ncg = (prec == MTK_FP8_E4M3 && p.nt > MTK_FP8_NTW) ? (int)cdiv(p.nt, MTK_FP8_NTW) : 1;
  p.ntw = (int)cdiv(p.nt, p.ncg);
  if (mode == 0) { p.nM = (int)I; p.nRed = (int)K; p.nLoop = (int)J; p.sM = J * K; p.sRed = 1; p.sLoop = K; }
  else if (mode == 1) { p.nM = (int)J; p.nRed = (int)K; p.nLoop = (int)I; p.sM = K; p.sRed = 1; p.sLoop = J * K; }
  else if (transposed) { p.nM = (int)K; p.nRed = (int)J; p.nLoop = (int)I; p.sM = J; p.sRed = 1; p.sLoop = J * K; }
  else { p.nM = (int)K; p.nRed = (int)J; p.nLoop = (int)I; p.sM = 1; p.sRed = K; p.sLoop = J * K; }

  // Mode 2 of an FP32 tensor with k contiguous: row-interleaved tiles of 64
  // rows read with 16-byte vectors (needs 16-byte aligned rows: K % 4 == 0).
  if (mode == 2 && !transposed && prec != MTK_FP8_E4M3 && x_aligned16 && K % 4 == 0) {
    p.cm = true;
    // bf16x6's third fragment term leaves a four-tile wave one wave per SIMD.
    p.ncg = (int)cdiv(p.nt, prec == MTK_BF16X6 ? 2 : MTK_CM_NTW);
    p.ntw = (int)cdiv(p.nt, p.ncg);
    p.nv = 8;
    p.kw = 32;
    const int64_t windows = cdiv(p.nRed, p.kw);
    p.wr = pick_wr(windows, 4 / p.ncg);
    p.mt_per_wg = 4 / (p.ncg * p.wr);
    p.n_rg = (int)cdiv(p.nRed, (int64_t)p.wr * p.kw);
    p.n_mg = (int)cdiv(cdiv(p.nM, 64), p.mt_per_wg);
    p.vec = true;
    set_loop_blocks(p, prec, plan_slots(p, prec));
    return p;
  }

  // Fragment registers per lane: nt*nv (FP32; BF16X3 hi+lo), 3 nt*nv/2
  // (BF16X6 hi+mid+lo) or nt*nv/4 (FP8); keep <= 64 (BF16X6: MTK_X6_FRAG_REGS).
  int nv;
  if (prec == MTK_FP8_E4M3) {
    nv = 128;
    while (nv > 32 && p.ntw * nv / 2 > MTK_FP8_FRAG_REGS) nv /= 2;      // hi + lo terms
    while (nv > 32 && 4 * (nv / 2) >= p.nRed) nv /= 2;
  } else {
    nv = MTK_NV_MAX;
    if (prec == MTK_BF16X6) {
      while (nv > 8 && 3 * p.ntw * nv / 2 > MTK_X6_FRAG_REGS) nv /= 2;
    } else {
      while (nv > 8 && p.ntw * nv > 64) nv /= 2;
    }
    while (nv > 8 && 4 * (nv / 2) >= p.nRed) nv /= 2;
  }
  p.nv = nv;
  p.kw = 4 * nv;
  const int64_t windows = cdiv(p.nRed, p.kw);
  const int wmax = 4 / p.ncg;
  p.wr = p.sRed == 1 ? pick_wr(windows, wmax) : 1;
  p.mt_per_wg = 4 / (p.ncg * p.wr);
  p.n_rg = (int)cdiv(p.nRed, (int64_t)p.wr * p.kw);
  p.n_mg = (int)cdiv(cdiv(p.nM, 16), p.mt_per_wg);

  set_loop_blocks(p, prec, plan_slots(p, prec));
  const int elem = prec == MTK_FP8_E4M3 ? 1 : 4;
  p.vec = (p.sRed == 1) && x_aligned16 && ((int64_t)p.nRed * elem % 16 == 0);
  return p;
}

size_t contract_ws_bytes(const ContractPlan& p, int prec) {
  size_t b = 0;
  if (p.slices > 1) b += (size_t)p.slices * p.nM * p.R * sizeof(float);
  b = (b + 255) & ~(size_t)255;
  if (prec == MTK_FP8_E4M3) {
    b += (2 * (size_t)frag_red_pad(p) * p.R + 255) & ~(size_t)255;
    b += 256 + 2 * (size_t)p.R * sizeof(int32_t);
  }
  return b;
}

hipError_t launch_contract(const ContractPlan& p, int prec, int mode, const void* X,
                           const int32_t* slice_exp, const float* frag_src, const float* weight,
                           float* out, void* ws, hipStream_t st, const FactorArgs* job) {
  if (job && (job->R > kJobMaxRank || p.ntw > 2)) return hipErrorInvalidValue;
  // One-dimensional grids (contraction, reduction) must fit gridDim.x.
  if (p.grid() + 1 > kMaxGridX || cdiv((int64_t)p.nM * p.R, 32) > kMaxGridX) return hipErrorInvalidConfiguration;
  KArgs a{};
  a.job_on = job ? 1 : 0;
  if (job) a.job = *job;
  a.X = X;
  a.slice_exp = slice_exp;
  a.frag_src = frag_src;
  a.weight = weight;
  a.sM = p.sM; a.sRed = p.sRed; a.sLoop = p.sLoop;
  a.nM = p.nM; a.nRed = p.nRed; a.nLoop = p.nLoop; a.R = p.R;
  a.wr = p.wr; a.mt_per_wg = p.mt_per_wg; a.n_rg = p.n_rg; a.n_mg = p.n_mg;
  a.loop_block = p.loop_block; a.n_lb = p.n_lb;
  a.ncg = p.ncg;
  a.mode = mode;
  char* w = static_cast<char*>(ws);
  size_t partial_bytes = 0;
  if (p.slices > 1) {
    a.part = reinterpret_cast<float*>(w);
    partial_bytes = ((size_t)p.slices * p.nM * p.R * sizeof(float) + 255) & ~(size_t)255;
  } else {
    a.part = out;
  }
  if (prec == MTK_FP8_E4M3) {
    const int red_pad = frag_red_pad(p);
    uint8_t* q = reinterpret_cast<uint8_t*>(w + partial_bytes);
    int32_t* ex = reinterpret_cast<int32_t*>(w + partial_bytes + ((2 * (size_t)red_pad * p.R + 255) & ~(size_t)255));
    hipLaunchKernelGGL(frag_quant_kernel, dim3(p.R), dim3(256), 0, st, frag_src, p.nRed, p.R, red_pad, q, ex);
    a.red_pad = red_pad;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.frag_q = q;
    a.frag_exp = ex;
  }
  hipError_t e;
  switch (prec) {
    case MTK_FP32: e = dispatch_nt<MTK_FP32>(a, p, st); break;
    case MTK_BF16X3: e = dispatch_nt<MTK_BF16X3>(a, p, st); break;
    case MTK_BF16X6: e = dispatch_nt<MTK_BF16X6>(a, p, st); break;
    case MTK_FP8_E4M3: e = dispatch_nt<MTK_FP8_E4M3>(a, p, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (p.slices > 1) e = launch_slice_reduce(a.part, p.slices, (int64_t)p.nM * p.R, out, st);
  return e;
}

hipError_t launch_slice_reduce(const float* part, int slices, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(n, 32)), dim3(256), 0, st, part, slices, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Serving: plan of one request's contraction in a grouped step.  nv = 8
// (kw = 32 values per wave window), one 16-column tile per workgroup; modes
// 0 and 1 reduce over contiguous k (up to 4 waves on adjacent windows),
// mode 2 over strided j (4 waves on adjacent 16-row tiles).  The outer loop
// is split so that a workgroup covers about 32K tensor elements, with at
// most 128 partial slices.  Everything depends on (dims, R, mode, prec)
// only.
// ---------------------------------------------------------------------------
SrvContract srv_contract_plan(const int64_t dims[3], int R, int mode, int prec, bool x_aligned16) {
  SrvContract c{};
  const int64_t I = dims[0], J = dims[1], K = dims[2];
  c.R = R;
  c.mode = mode;
  c.prec = prec;
  if (mode == 0) { c.nM = (int)I; c.nRed = (int)K; c.nLoop = (int)J; c.sM = J * K; c.sRed = 1; c.sLoop = K; }
  else if (mode == 1) { c.nM = (int)J; c.nRed = (int)K; c.nLoop = (int)I; c.sM = K; c.sRed = 1; c.sLoop = J * K; }
  else { c.nM = (int)K; c.nRed = (int)J; c.nLoop = (int)I; c.sM = 1; c.sRed = K; c.sLoop = J * K; }
  constexpr int kw = 32;
  if (mode != 2) {
    c.form = (x_aligned16 && c.nRed % 4 == 0) ? 0 : 1;
    const int64_t windows = cdiv(c.nRed, kw);
    c.wr = windows >= 4 ? 4 : (windows >= 2 ? 2 : 1);
  } else {
    c.form = 2;
    c.wr = 1;
  }
  c.mt_per_wg = 4 / c.wr;
  c.n_rg = (int)cdiv(c.nRed, (int64_t)c.wr * kw);
  c.n_mg = (int)cdiv(cdiv(c.nM, 16), c.mt_per_wg);
  c.nct = (int)cdiv(R, 16);
  const int64_t base = (int64_t)c.n_rg * c.n_mg * c.nct;
  const int64_t want = std::max<int64_t>(1, cdiv(I * J * K, 32768));
  int64_t n_lb = std::max<int64_t>(1, std::min<int64_t>(c.nLoop, cdiv(want, base)));
  while (n_lb > 1 && (int64_t)c.n_rg * n_lb > 128) n_lb = cdiv(n_lb, 2);
  c.loop_block = (int)cdiv(c.nLoop, n_lb);
  c.loop_block = std::min(c.loop_block, std::max(1, MTK_STAGE_FLOATS / R));
  c.n_lb = (int)cdiv(c.nLoop, c.loop_block);
  c.slices = c.n_rg * c.n_lb;
  return c;
}

int64_t srv_contract_items(const SrvContract& c) { return (int64_t)c.n_rg * c.n_mg * c.n_lb * c.nct; }

size_t srv_contract_lds_bytes() {
  return std::max(((size_t)MTK_STAGE_FLOATS + 4 * 4 * 64) * sizeof(float), factor_gj_lds_bytes(kSrvFusedMaxRank));
}

hipError_t launch_srv_contract(const SrvTable* t, int u, bool with_factor, hipStream_t st) {
  hipLaunchKernelGGL(srv_contract_kernel, dim3(kSrvContractGrid), dim3(256), srv_contract_lds_bytes(), st, t, u,
                     with_factor ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mtk
