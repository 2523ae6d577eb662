// Khatri-Rao rows for the N-way MTTKRP (mttkrp_nway in api.hip).
//
// A mode-n MTTKRP of an N-way row-major tensor is a three-way MTTKRP of the
// same bytes viewed as (P, d_n, Q) (or (d_0, P, Q), (P, Q, d_{N-1}) for the
// first and last modes), where P and Q are products of consecutive
// dimensions: the factor of a merged group of modes is the Khatri-Rao
// product of its factors, row (i_a, ..., i_b) = A_a(i_a, :) * ... * A_b(i_b, :)
// with the first mode's index slowest -- the order in which those indices
// run through the row-major tensor.  This kernel writes such a product.

#include "mtk_internal.h"

#include <algorithm>

namespace mtk {
namespace {

struct KrArgs {
  const float* f[kMaxNwayModes];
  int64_t d[kMaxNwayModes];
  int n;              // modes in the group
  int R;
  int64_t rows;       // product of d[0..n-1]
  float* out;         // rows x R
};

// out(row, r) = prod over the group's modes in increasing order of
// f[m](i_m, r), where row runs over (i_0, ..., i_{n-1}) with i_{n-1} fastest.
__global__ __launch_bounds__(256) void kr_rows_kernel(KrArgs a) {
  const int64_t total = a.rows * a.R;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / a.R;
    const int r = (int)(e - row * a.R);
    int64_t idx[kMaxNwayModes];
    int64_t rest = row;
    for (int m = a.n - 1; m >= 0; --m) {
      idx[m] = rest % a.d[m];
      rest /= a.d[m];
    }
    float p = a.f[0][idx[0] * a.R + r];
    for (int m = 1; m < a.n; ++m) p *= a.f[m][idx[m] * a.R + r];
    a.out[e] = p;
  }
}

}  // namespace

hipError_t launch_kr_rows(const float* const* factors, const int64_t* dims, int n, int R, float* out,
                          hipStream_t st) {
  if (n < 1 || n > kMaxNwayModes) return hipErrorInvalidValue;
  KrArgs a{};
  a.rows = 1;
  for (int m = 0; m < n; ++m) {
    a.f[m] = factors[m];
    a.d[m] = dims[m];
    a.rows *= dims[m];
  }
  a.n = n;
  a.R = R;
  a.out = out;
  const int64_t blocks = std::min<int64_t>((a.rows * R + 255) / 256, (int64_t)1 << 20);
  hipLaunchKernelGGL(kr_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace mtk
