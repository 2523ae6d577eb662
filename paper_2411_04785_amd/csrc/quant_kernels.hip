// FP8 tensor preparation: per mode-1 slice power-of-two scaled OCP e4m3.
//
// Slice i (the I-th block of J*K contiguous values) gets
// e_i = min{ e : amax_i <= 448 * 2^e } and codes e4m3(x * 2^-e_i).  The
// maximum is exact and the scaling by a power of two is exact, so the codes
// are a deterministic function of the FP32 input, bit for bit.  Optionally a
// second copy holds every slice transposed ((i, k, j) order), so that the
// mode-3 contraction (over j) reads contiguous bytes.

#include "mtk_internal.h"
#include "fp8_codec.h"

#include <algorithm>

namespace mtk {
namespace {

// One workgroup per slice: amax over the slice, then its exponent.
__global__ __launch_bounds__(256) void slice_amax_kernel(const float* __restrict__ x, int64_t JK,
                                                         int32_t* __restrict__ exps) {
  const int64_t i = blockIdx.x;
  const float* p = x + i * JK;
  float m = 0.f;
  const bool vec = (JK % 4 == 0) && ((reinterpret_cast<uintptr_t>(x) & 15) == 0);
  if (vec) {
    const float4* p4 = reinterpret_cast<const float4*>(p);
    for (int64_t e = threadIdx.x; e < JK / 4; e += 256) {
      const float4 v = p4[e];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
  } else {
    for (int64_t e = threadIdx.x; e < JK; e += 256) m = fmaxf(m, fabsf(p[e]));
  }
  __shared__ float sh[256];
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) exps[i] = scale_exponent_dev(sh[0]);
}

// Encode 4 consecutive values per thread.
__global__ __launch_bounds__(256) void slice_encode_kernel(const float* __restrict__ x, int64_t JK, int64_t n,
                                                           const int32_t* __restrict__ exps,
                                                           uint8_t* __restrict__ q) {
  const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (e0 >= n) return;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t e = e0 + b;
    if (e < n) {
      const float inv = ldexpf(1.f, -exps[e / JK]);
      q[e] = static_cast<uint8_t>(e4m3_encode_dev(x[e] * inv));
    }
  }
}

// qt[(i*K + k)*J + j] = q[(i*J + j)*K + k]: each mode-1 slice transposed,
// through a 64 x 64 byte tile in LDS.  Tile t = (slice i, j tile, k tile),
// k tile fastest; the workgroups stride over the I * nj * nk tiles, so no
// grid dimension grows with I.
__global__ __launch_bounds__(256) void slice_transpose_kernel(const uint8_t* __restrict__ q, int64_t I, int64_t J,
                                                              int64_t K, uint8_t* __restrict__ qt) {
  __shared__ uint8_t tile[64][65];
  const int64_t nj = (J + 63) / 64, nk = (K + 63) / 64;
  const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
  for (int64_t t = blockIdx.x; t < I * nj * nk; t += gridDim.x) {
    const int64_t i = t / (nj * nk);
    const int64_t jt = (t - i * nj * nk) / nk;
    const int64_t j0 = jt * 64, k0 = (t - i * nj * nk - jt * nk) * 64;
    {
      const int64_t j = j0 + r;
      const uint8_t* src = q + (i * J + j) * K + k0 + c0;
      const bool full = j < J && k0 + c0 + 16 <= K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0);
      if (full) {
        const uint4 u = *reinterpret_cast<const uint4*>(src);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int b = 0; b < 16; ++b) tile[r][c0 + b] = (uint8_t)(w[b >> 2] >> (8 * (b & 3)));
      } else {
        for (int b = 0; b < 16; ++b) tile[r][c0 + b] = (j < J && k0 + c0 + b < K) ? src[b] : 0;
      }
    }
    __syncthreads();
    const int64_t k = k0 + r;
    if (k < K) {
      uint8_t* dst = qt + (i * K + k) * J + j0 + c0;
      const bool full = j0 + c0 + 16 <= J && ((reinterpret_cast<uintptr_t>(dst) & 15) == 0);
      if (full) {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 16; ++b) w[b >> 2] |= (uint32_t)tile[c0 + b][r] << (8 * (b & 3));
        *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
      } else {
        for (int b = 0; b < 16; ++b)
          if (j0 + c0 + b < J) dst[b] = tile[c0 + b][r];
      }
    }
    __syncthreads();                  // the tile is refilled by the next item
  }
}

}  // namespace

hipError_t launch_quantize_slices(const float* x, int64_t I, int64_t J, int64_t K, uint8_t* q, uint8_t* qt,
                                  int32_t* exps, hipStream_t st) {
  const int64_t JK = J * K;
  hipLaunchKernelGGL(slice_amax_kernel, dim3((unsigned)I), dim3(256), 0, st, x, JK, exps);
  const int64_t n = I * JK;
  const int64_t blocks = (n / 4 + 255) / 256 + 1;
  hipLaunchKernelGGL(slice_encode_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, JK, n, exps, q);
  if (qt) {
    const int64_t tiles = I * ((J + 63) / 64) * ((K + 63) / 64);
    hipLaunchKernelGGL(slice_transpose_kernel, dim3((unsigned)std::min<int64_t>(tiles, (int64_t)1 << 20)), dim3(256), 0,
                       st, q, I, J, K, qt);
  }
  return hipGetLastError();
}

}  // namespace mtk
