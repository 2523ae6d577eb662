// Register tiles of the MFMA contraction shared by the MTTKRP kernels and
// the tensor-times-matrix kernel of the dimension-tree sweep: the lane's
// slice of an X tile, the factor fragment held as MFMA B-operands, and one
// tile step.  Lane (m, g) of a wave holds row m (0..15) of the tile and nv
// contiguous reduction values g*nv .. g*nv+nv-1; any consistent pairing of
// A and B lane elements is a valid MFMA reduction order.
#pragma once

#include "mtk_internal.h"
#include "fp8_codec.h"

namespace mtk {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(8))) int i32x8;

__device__ __forceinline__ f4 zero4() { return f4{0.f, 0.f, 0.f, 0.f}; }

// ---------------------------------------------------------------------------
// Per-precision element type of X and MFMA step shape.
// ---------------------------------------------------------------------------
template <int PREC> struct PrecT;
template <> struct PrecT<MTK_FP32> { using XT = float; static constexpr int kStep = 1; };
template <> struct PrecT<MTK_BF16X3> { using XT = float; static constexpr int kStep = 8; };
template <> struct PrecT<MTK_BF16X6> { using XT = float; static constexpr int kStep = 8; };
template <> struct PrecT<MTK_FP8_E4M3> { using XT = uint8_t; static constexpr int kStep = 32; };

// X tile registers of one lane: nv reduction values of one row.
template <int PREC, int NV> struct XRegs;
template <int NV> struct XRegs<MTK_FP32, NV> { float v[NV]; };
template <int NV> struct XRegs<MTK_BF16X3, NV> { float v[NV]; };
template <int NV> struct XRegs<MTK_BF16X6, NV> { float v[NV]; };
template <int NV> struct XRegs<MTK_FP8_E4M3, NV> { uint32_t w[NV / 4]; };

// Load this lane's nv reduction values of tile row `m` (global offset `off`
// of its first value).  `full` means the whole window and row are in range.
// FP8 lanes hold their nv values as 16-byte pieces: lane group g's element e
// is at offset 64 (e / 16) + 16 g + e % 16 of the window, so one 16-byte load
// instruction of a wave reads 64 contiguous bytes of each row.  `red0` and
// `off` of an FP8 lane point at window offset 16 g; fp8_piece_off(e) is the
// rest.  The factor fragment uses the same offsets, so A and B elements of a
// lane pair up on the same reduction index.
__device__ __forceinline__ constexpr int fp8_piece_off(int e) { return (e >> 4) * 64 + (e & 15); }

template <int PREC, int NV, bool CONTIG, bool VEC, bool full>
__device__ __forceinline__ void load_x(XRegs<PREC, NV>& x, const void* X, int64_t off,
                                       int64_t sRed, bool row_ok, int red0, int nRed) {
  if constexpr (PREC == MTK_FP8_E4M3) {
    const uint8_t* p = static_cast<const uint8_t*>(X) + off;
    if constexpr (CONTIG && VEC && full) {
#pragma unroll
      for (int q = 0; q < NV / 16; ++q) {
        const uint4 u = *reinterpret_cast<const uint4*>(p + q * 64);
        x.w[4 * q + 0] = u.x; x.w[4 * q + 1] = u.y; x.w[4 * q + 2] = u.z; x.w[4 * q + 3] = u.w;
      }
    } else if constexpr (CONTIG && VEC) {
      // nRed is a multiple of 16 here, so each 16-byte piece is all in or all out.
#pragma unroll
      for (int q = 0; q < NV / 16; ++q) {
        uint4 u = make_uint4(0, 0, 0, 0);
        if (row_ok && red0 + 64 * q < nRed) u = *reinterpret_cast<const uint4*>(p + q * 64);
        x.w[4 * q + 0] = u.x; x.w[4 * q + 1] = u.y; x.w[4 * q + 2] = u.z; x.w[4 * q + 3] = u.w;
      }
    } else {
      // Ragged or strided bytes: outside the row or the reduction range the
      // load reads the tensor's first byte instead and the value is zeroed.
#pragma unroll
      for (int q = 0; q < NV / 4; ++q) {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int k = fp8_piece_off(4 * q + b);
          const bool ok = full || (row_ok && red0 + k < nRed);
          const uint32_t v = *(ok ? p + (int64_t)k * sRed : static_cast<const uint8_t*>(X));
          w |= (ok ? v : 0u) << (8 * b);
        }
        x.w[q] = w;
      }
    }
  } else {
    const float* p = static_cast<const float*>(X) + off;
    if constexpr (CONTIG && VEC && full) {
#pragma unroll
      for (int q = 0; q < NV / 4; ++q) {
        const float4 u = *reinterpret_cast<const float4*>(p + q * 4);
        x.v[4 * q + 0] = u.x; x.v[4 * q + 1] = u.y; x.v[4 * q + 2] = u.z; x.v[4 * q + 3] = u.w;
      }
    } else if constexpr (CONTIG && VEC) {
      // nRed is a multiple of 4 here, so each 16-byte chunk is all in or all out.
#pragma unroll
      for (int q = 0; q < NV / 4; ++q) {
        float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row_ok && red0 + 4 * q < nRed) u = *reinterpret_cast<const float4*>(p + q * 4);
        x.v[4 * q + 0] = u.x; x.v[4 * q + 1] = u.y; x.v[4 * q + 2] = u.z; x.v[4 * q + 3] = u.w;
      }
    } else {
      // Strided or unaligned rows: the address of element e is the lane's
      // pointer p plus the wave-uniform step e*sRed; outside the row or the
      // reduction range the load reads the tensor's first element instead
      // and the value is replaced by zero.
      const float* X0 = static_cast<const float*>(X);
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        const bool ok = full || (row_ok && red0 + e < nRed);
        const float v = *(ok ? p + (int64_t)e * sRed : X0);
        x.v[e] = ok ? v : 0.f;
      }
    }
  }
}

// bf16 round-to-nearest-even split of a binary32 value: hi = bf16(x),
// lo = bf16(x - hi); x - hi is exact.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  lo = static_cast<__bf16>(x - static_cast<float>(hi));
}

// Three-term split: hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi -
// mid); both differences are exact, and the three 8-bit significands cover
// the 24 of a binary32 value (x = hi + mid + lo for normal values).
__device__ __forceinline__ void split3_bf16(float x, __bf16& hi, __bf16& mid, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  const float r = x - static_cast<float>(hi);
  mid = static_cast<__bf16>(r);
  lo = static_cast<__bf16>(r - static_cast<float>(mid));
}

// Fragment of the factor G held by one lane for the whole kernel: for N-tile
// t and MFMA step s, the values G(red0 + s*kStep + e, t*16 + n) for the
// lane's element slots e (n = lane & 15, red0 = window start + g*nv).
template <int PREC, int NT, int NV> struct Frag;
template <int NT, int NV> struct Frag<MTK_FP32, NT, NV> { float f[NT][NV]; };
template <int NT, int NV> struct Frag<MTK_BF16X3, NT, NV> { bf16x8 hi[NT][NV / 8]; bf16x8 lo[NT][NV / 8]; };
template <int NT, int NV> struct Frag<MTK_BF16X6, NT, NV> {
  bf16x8 hi[NT][NV / 8];
  bf16x8 mid[NT][NV / 8];
  bf16x8 lo[NT][NV / 8];
};
// FP8: the factor is held as two e4m3 terms, hi = e4m3(G 2^-eh) and
// lo = e4m3((G - hi 2^eh) 2^-el), with per-column exponents eh, el.  The
// exponents of the lane's column travel as E8M0 B-operand scales (127 + e),
// which the MFMA applies per column, so both terms accumulate into one tile.
template <int NT, int NV> struct Frag<MTK_FP8_E4M3, NT, NV> {
  i32x8 q[NT][NV / 32];
  i32x8 ql[NT][NV / 32];
  int sh[NT], sl[NT];
};

// Factor value v into slot (t, s, e) of a split (bf16x3 / bf16x6) fragment.
template <int PREC, int NT, int NV>
__device__ __forceinline__ void frag_put(Frag<PREC, NT, NV>& fr, int t, int s, int e, float v) {
  if constexpr (PREC == MTK_BF16X3) {
    __bf16 h, l;
    split_bf16(v, h, l);
    fr.hi[t][s][e] = h;
    fr.lo[t][s][e] = l;
  } else if constexpr (PREC == MTK_BF16X6) {
    __bf16 h, m, l;
    split3_bf16(v, h, m, l);
    fr.hi[t][s][e] = h;
    fr.mid[t][s][e] = m;
    fr.lo[t][s][e] = l;
  }
}

// One bf16 MFMA step of a split path for every N-tile t: the 8 X values xs
// of the lane (reduction slots of step s) split like the fragment, and the
// products accumulated smallest first.  bf16x3: x_lo G_hi, x_hi G_lo,
// x_hi G_hi (x_lo G_lo, below 2^-16 relative, dropped).  bf16x6: the six
// products down to 2^-16 relative (x_lo G_hi, x_hi G_lo, x_mid G_mid, x_mid
// G_hi, x_hi G_mid, x_hi G_hi); the dropped ones are below 2^-24.
template <int PREC, int NT, int NV>
__device__ __forceinline__ void split_step(f4 (&T)[NT], const float (&xs)[8], const Frag<PREC, NT, NV>& fr,
                                           int s) {
  if constexpr (PREC == MTK_BF16X3) {
    bf16x8 ah, al;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h, l;
      split_bf16(xs[e], h, l);
      ah[e] = h;
      al[e] = l;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, fr.hi[t][s], T[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, fr.lo[t][s], T[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, fr.hi[t][s], T[t], 0, 0, 0);
  } else {
    bf16x8 ah, am, al;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h, m, l;
      split3_bf16(xs[e], h, m, l);
      ah[e] = h;
      am[e] = m;
      al[e] = l;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, fr.hi[t][s], T[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, fr.lo[t][s], T[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, fr.mid[t][s], T[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, fr.hi[t][s], T[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, fr.mid[t][s], T[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, fr.hi[t][s], T[t], 0, 0, 0);
  }
}

// T[t] = X-tile (16 x kw) times fragment (kw x 16) for every N-tile t
// (ACC: added to T[t] instead).
template <int PREC, int NT, int NV, bool ACC = false>
__device__ __forceinline__ void tile_mfma(f4 (&T)[NT], const XRegs<PREC, NV>& x,
                                          const Frag<PREC, NT, NV>& fr) {
  if constexpr (!ACC) {
#pragma unroll
    for (int t = 0; t < NT; ++t) T[t] = zero4();
  }
  if constexpr (PREC == MTK_FP32) {
#pragma unroll
    for (int s = 0; s < NV; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        T[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.v[s], fr.f[t][s], T[t], 0, 0, 0);
  } else if constexpr (PREC == MTK_BF16X3 || PREC == MTK_BF16X6) {
#pragma unroll
    for (int s = 0; s < NV / 8; ++s) {
      float xs[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xs[e] = x.v[s * 8 + e];
      split_step<PREC, NT, NV>(T, xs, fr, s);
    }
  } else {
#pragma unroll
    for (int s = 0; s < NV / 32; ++s) {
      i32x8 xq;
#pragma unroll
      for (int w = 0; w < 8; ++w) xq[w] = static_cast<int>(x.w[s * 8 + w]);
      // e4m3 x e4m3 (format code 0 for both); A scale 2^0 (127), B scale
      // 2^eh / 2^el of the lane's column.  Small term first.
#pragma unroll
      for (int t = 0; t < NT; ++t)
        T[t] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(xq, fr.ql[t][s], T[t], 0, 0, 0, 127, 0, fr.sl[t]);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        T[t] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(xq, fr.q[t][s], T[t], 0, 0, 0, 127, 0, fr.sh[t]);
    }
  }
}

}  // namespace
}  // namespace mtk
