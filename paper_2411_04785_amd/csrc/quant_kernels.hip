// FP8 tensor preparation: per mode-1 slice power-of-two scaled OCP e4m3.
//
// Slice i (the I-th block of J*K contiguous values) gets
// e_i = min{ e : amax_i <= 448 * 2^e } and codes e4m3(x * 2^-e_i).  The
// maximum is exact and the scaling by a power of two is exact, so the codes
// are a deterministic function of the FP32 input, bit for bit.

#include "mtk_internal.h"
#include "fp8_codec.h"

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

}  // namespace

hipError_t launch_quantize_slices(const float* x, int64_t I, int64_t JK, uint8_t* q, int32_t* exps,
                                  hipStream_t st) {
  hipLaunchKernelGGL(slice_amax_kernel, dim3((unsigned)I), dim3(256), 0, st, x, JK, exps);
  const int64_t n = I * JK;
  const int64_t blocks = (n / 4 + 255) / 256 + 1;
  hipLaunchKernelGGL(slice_encode_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, JK, n, exps, q);
  return hipGetLastError();
}

}  // namespace mtk
