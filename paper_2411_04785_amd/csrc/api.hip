// C-ABI entry points of libmttkrp (declared in include/mttkrp.h).

#include "mtk_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

namespace mtk {
// Extrapolation candidate of factor `mode` (als_kernels.hip): normalise(P +
// d (Q - P)) into factor_out (FP32, unit columns; the norms into lambda) and
// its Gram partials into the mode's slot of the solve region `ws`.
hipError_t launch_extrapolate(const int64_t dims[3], int R, int mode, const float* P, const float* Q, double d,
                              float* factor_out, double* lambda, int64_t maxdim, void* ws, int* status,
                              hipStream_t st);
// Mode-1 MTTKRP from the Y kernel's row sums, Y not stored (dimtree.hip):
// its J-block partial slices (0: J does not fit the kernel's row blocks),
// their scratch, and the launch (plus the slice reduction).
int64_t ttm_m1_slices(const int64_t dims[3], int R);
size_t ttm_m1_ws_bytes(const int64_t dims[3], int R);
hipError_t launch_ttm_m1(const float* X, bool x_aligned16, const int64_t dims[3], const float* const factors[3],
                         int R, int prec, float* out, void* ws, hipStream_t st, const FactorArgs* job);
}  // namespace mtk

namespace {

using mtk::ContractPlan;

struct GraphKey {
  const void* X;
  const void* Xt;
  int64_t dims[3];
  int fmt;
  const void* slice_exp;
  const void* f[3];
  const void* lambda;
  int R, prec, with_fit;
  bool operator<(const GraphKey& o) const {
    return std::tie(X, Xt, dims[0], dims[1], dims[2], fmt, slice_exp, f[0], f[1], f[2], lambda, R, prec, with_fit) <
           std::tie(o.X, o.Xt, o.dims[0], o.dims[1], o.dims[2], o.fmt, o.slice_exp, o.f[0], o.f[1], o.f[2], o.lambda,
                    o.R, o.prec, o.with_fit);
  }
};

struct GraphCache {
  hipStream_t capture_stream = nullptr;
  std::map<GraphKey, hipGraphExec_t> execs;
  std::vector<hipGraphExec_t> retired;   // no longer looked up; may still be in flight
  std::vector<hipGraph_t> graphs;
};

mtk_status fail(mtk_ctx* c, mtk_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

mtk_status hip_fail(mtk_ctx* c, hipError_t e, const char* where) {
  return fail(c, MTK_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(ctx, call)                          \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// Move every cached sweep graph out of the lookup (they reference the old
// workspace); they are destroyed by mtk_graph_reset / mtk_destroy.
void retire_graphs(mtk_ctx* c) {
  GraphCache* gc = static_cast<GraphCache*>(c->graph_cache);
  if (!gc) return;
  for (auto& kv : gc->execs) gc->retired.push_back(kv.second);
  gc->execs.clear();
}

bool factor_dims_ok(const int64_t d[3]) {
  return d[0] >= 1 && d[1] >= 1 && d[2] >= 1 && d[0] <= (1 << 30) && d[1] <= (1 << 30) && d[2] <= (1 << 30);
}

bool dims_ok(const int64_t d[3]) {
  if (!factor_dims_ok(d)) return false;
  const double n = (double)d[0] * d[1] * d[2];
  return n < 1099511627776.0;   // 2^40
}

// Grow the workspace to at least `bytes`.  The old block may still be read
// by work queued on any stream, and the cached sweep graphs hold its
// address, so neither is released here: both are retired (kept alive) and
// freed by mtk_graph_reset or mtk_destroy, which synchronise the device.
// Growth therefore never waits for the device.  Sizes grow at least 1.5x,
// so the retired blocks add up to less than twice the live one.
mtk_status ensure_ws(mtk_ctx* c, size_t bytes, hipStream_t st) {
  (void)st;
  if (bytes <= c->ws_bytes) return MTK_OK;
  size_t want = std::max<size_t>(bytes, 1 << 20);
  if (c->ws) want = std::max(want, c->ws_bytes + c->ws_bytes / 2);
  void* nw = nullptr;
  if (hipMalloc(&nw, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, MTK_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  if (c->ws) {
    c->retired_ws.push_back(c->ws);
    retire_graphs(c);
  }
  c->ws = nw;
  c->ws_bytes = want;
  return MTK_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

mtk_status check_tensor(mtk_ctx* c, const mtk_tensor* X) {
  if (!X) return fail(c, MTK_EINVAL, "X is NULL");
  if (!X->data) return fail(c, MTK_EINVAL, "X->data is NULL");
  if (!dims_ok(X->dims)) return fail(c, MTK_EINVAL, "X->dims out of range (each >= 1, product < 2^40)");
  if (X->fmt != MTK_FP32 && X->fmt != MTK_FP8_E4M3) return fail(c, MTK_EINVAL, "X->fmt must be MTK_FP32 or MTK_FP8_E4M3");
  if (X->fmt == MTK_FP8_E4M3 && !X->slice_exp) return fail(c, MTK_EINVAL, "FP8 tensor needs slice_exp");
  if (X->fmt == MTK_FP32 && (reinterpret_cast<uintptr_t>(X->data) & 3)) return fail(c, MTK_EINVAL, "FP32 X->data not 4-byte aligned");
  return MTK_OK;
}

mtk_status check_prec(mtk_ctx* c, const mtk_tensor* X, int prec) {
  if (prec != MTK_FP32 && prec != MTK_BF16X3 && prec != MTK_BF16X6 && prec != MTK_FP8_E4M3)
    return fail(c, MTK_EINVAL, "unknown precision");
  if (X->fmt == MTK_FP8_E4M3 && prec != MTK_FP8_E4M3) return fail(c, MTK_EINVAL, "FP8 tensor requires prec MTK_FP8_E4M3");
  if (X->fmt == MTK_FP32 && prec == MTK_FP8_E4M3) return fail(c, MTK_EINVAL, "prec MTK_FP8_E4M3 requires an FP8 tensor (mtk_quantize_fp8)");
  return MTK_OK;
}

// Mode 1 of an FP32 tensor in bf16x3 whose mode-1 slices are far apart
// (J*K >= 65536 elements): the contraction's 16-row tiles would read 16
// rows J*K apart (1024^3: 5.2 TB/s for such a pattern against 6.0 TB/s for
// rows K apart), so the Y kernel's row sums serve it instead, with Y not
// stored, reading X row by row (1024^3 R=64, same device: 932 -> 776 us;
// MTK_M1_ROUTE=0 builds without it).  Rows must be long (K >= 512): on
// rows of 128 elements the Y kernel's per-row work outweighs the gain
// (128 x 16384 x 128, R=32: 207 against 188 us).  FP32 is MFMA-bound
// there, and bf16x6 came out slower and, summing a workgroup's rows in
// FP32, at twice its error; both keep the contraction.
#ifndef MTK_M1_ROUTE
#define MTK_M1_ROUTE 1
#endif
static bool m1_route(const int64_t dims[3], int R, int mode, int fmt, int prec) {
  return MTK_M1_ROUTE && mode == 0 && fmt == MTK_FP32 && prec == MTK_BF16X3 &&
         mtk::ttm_m1_slices(dims, R) > 0 && dims[0] * dims[1] <= mtk::kDimtreeMaxRows &&
         dims[1] * dims[2] >= 65536 && dims[2] >= 512;
}

size_t mttkrp_ws(const int64_t dims[3], int R, int mode, int prec) {
  if (m1_route(dims, R, mode, MTK_FP32, prec)) return mtk::ttm_m1_ws_bytes(dims, R);
  size_t b = 0;
  for (int tr = 0; tr < 2; ++tr)
    for (int al = 0; al < 2; ++al)
      b = std::max(b, mtk::contract_ws_bytes(mtk::make_plan(dims, R, mode, prec, al != 0, tr != 0), prec));
  return b;
}

// Scratch of a sweep: [contraction / fit region][solve region]; the two
// regions are disjoint because the Gram matrices kept in the solve region
// live across the MTTKRPs.
size_t sweep_contract_bytes(const int64_t dims[3], int R, int prec) {
  size_t b = 0;
  for (int m = 0; m < 3; ++m) b = std::max(b, mttkrp_ws(dims, R, m, prec));
  return round256(std::max(b, mtk::fit_ws_bytes(dims)));
}

// ... followed by the dimension-tree region (Y and its partial sums) when
// the sweep uses one.
size_t sweep_scratch_bytes(const int64_t dims[3], int R, int prec) {
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  const size_t dt = mtk::dimtree_used(dims, R, prec) ? mtk::dimtree_ws_bytes(dims, R) : 0;
  return sweep_contract_bytes(dims, R, prec) + mtk::solve_ws_bytes(maxdim, R) + dt;
}

// Scratch of mttkrp_noalloc: device memory that no call allocates.  Each
// device the library runs on holds its own copy of this array from the
// moment the code object is loaded until the process ends.  Host code must
// not pass the array's name to a kernel (on the host it names a stand-in,
// not device memory): mtk_create looks up the device address of the copy
// on its device once and keeps it in g_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `device` (looked up on
// first use per device).
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

mtk_status mtk_create(mtk_ctx** ctx, int device) {
  if (!ctx) return MTK_EINVAL;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MTK_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return MTK_EHIP;
  void* scratch_ptr = nullptr;
  if (scratch_address(device, &scratch_ptr) != hipSuccess) return MTK_EHIP;
  mtk_ctx* c = new (std::nothrow) mtk_ctx();
  if (!c) return MTK_ENOMEM;
  c->device = device;
  c->scratch = scratch_ptr;
  const size_t status_bytes = mtk::kStatusWords * sizeof(int);
  if (hipMalloc(&c->d_status, status_bytes) != hipSuccess || hipMemset(c->d_status, 0, status_bytes) != hipSuccess) {
    delete c;
    return MTK_ENOMEM;
  }
  if (hipMalloc(&c->d_fit, 2 * sizeof(double)) != hipSuccess) {
    (void)hipFree(c->d_status);
    delete c;
    return MTK_ENOMEM;
  }
  GraphCache* gc = new (std::nothrow) GraphCache();
  if (!gc || hipStreamCreateWithFlags(&gc->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    delete gc;
    (void)hipFree(c->d_status);
    (void)hipFree(c->d_fit);
    delete c;
    return MTK_EHIP;
  }
  c->graph_cache = gc;
  bool ok = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess;
  for (int m = 0; m < 3 && ok; ++m)
    ok = hipEventCreateWithFlags(&c->fork_ev[m], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->join_ev[m], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    mtk_destroy(c);
    return MTK_EHIP;
  }
  *ctx = c;
  return MTK_OK;
}

mtk_status mtk_graph_reset(mtk_ctx* c) {
  if (!c) return MTK_EINVAL;
  GraphCache* gc = static_cast<GraphCache*>(c->graph_cache);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (gc) {
    for (auto& kv : gc->execs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraphExec_t e : gc->retired) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : gc->graphs) (void)hipGraphDestroy(g);
    gc->execs.clear();
    gc->retired.clear();
    gc->graphs.clear();
  }
  for (void* p : c->retired_ws) (void)hipFree(p);
  c->retired_ws.clear();
  return MTK_OK;
}

mtk_status mtk_destroy(mtk_ctx* c) {
  if (!c) return MTK_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  mtk_graph_reset(c);
  GraphCache* gc = static_cast<GraphCache*>(c->graph_cache);
  if (gc) {
    if (gc->capture_stream) (void)hipStreamDestroy(gc->capture_stream);
    delete gc;
  }
  for (int m = 0; m < 3; ++m) {
    if (c->fork_ev[m]) (void)hipEventDestroy(c->fork_ev[m]);
    if (c->join_ev[m]) (void)hipEventDestroy(c->join_ev[m]);
  }
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->ws) (void)hipFree(c->ws);
  if (c->d_status) (void)hipFree(c->d_status);
  if (c->d_fit) (void)hipFree(c->d_fit);
  delete c;
  return MTK_OK;
}

const char* mtk_last_error(const mtk_ctx* c) { return c ? c->last_error.c_str() : "NULL context"; }

mtk_status mtk_check(mtk_ctx* c, void* stream) {
  if (!c) return MTK_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_OR_FAIL(c, hipStreamSynchronize(st));
  int s = 0;
  HIP_OR_FAIL(c, hipMemcpy(&s, c->d_status, sizeof(int), hipMemcpyDeviceToHost));
  if (s != 0) {
    HIP_OR_FAIL(c, hipMemset(c->d_status, 0, sizeof(int)));
    if (s & mtk::kStatusNotSPD) return fail(c, MTK_ENOTSPD, "normal-equation matrix not positive definite");
  }
  return MTK_OK;
}

mtk_status mtk_reserve(mtk_ctx* c, const int64_t dims[3], int64_t R, int prec) {
  if (!c || !dims) return fail(c, MTK_EINVAL, "NULL argument");
  if (!dims_ok(dims)) return fail(c, MTK_EINVAL, "dims out of range");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  size_t b = round256((size_t)maxdim * R * sizeof(float)) + sweep_scratch_bytes(dims, (int)R, prec);
  return ensure_ws(c, b, nullptr);
}

mtk_status mtk_quantize_fp8(mtk_ctx* c, const float* x, const int64_t dims[3], uint8_t* q_out, uint8_t* qt_out,
                            int32_t* exp_out, void* stream) {
  if (!c) return MTK_EINVAL;
  if (!x || !dims || !q_out || !exp_out) return fail(c, MTK_EINVAL, "NULL argument");
  if (!dims_ok(dims)) return fail(c, MTK_EINVAL, "dims out of range");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipError_t e = mtk::launch_quantize_slices(x, dims[0], dims[1], dims[2], q_out, qt_out, exp_out,
                                             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "quantize");
  return MTK_OK;
}

static mtk_status mttkrp_impl(mtk_ctx* c, const mtk_tensor* X, const float* const factors[3], int R, int mode,
                              int prec, float* out, void* ws, hipStream_t st,
                              const mtk::FactorArgs* job = nullptr) {
  if (m1_route(X->dims, R, mode, X->fmt, prec)) {
    hipError_t e = mtk::launch_ttm_m1(static_cast<const float*>(X->data), aligned16(X->data), X->dims, factors, R,
                                      prec, out, ws, st, job);
    if (e != hipSuccess) return hip_fail(c, e, "mttkrp launch");
    return MTK_OK;
  }
  const float* fr;     // fragment factor (inside the MFMA)
  const float* wt;     // weight factor (epilogue)
  if (mode == 0) { fr = factors[2]; wt = factors[1]; }
  else if (mode == 1) { fr = factors[2]; wt = factors[0]; }
  else { fr = factors[1]; wt = factors[0]; }
  const bool tr = mode == 2 && X->fmt == MTK_FP8_E4M3 && X->data_t != nullptr;
  const void* data = tr ? X->data_t : X->data;
  ContractPlan p = mtk::make_plan(X->dims, R, mode, prec, aligned16(data), tr);
  hipError_t e = mtk::launch_contract(p, prec, mode, data, X->slice_exp, fr, wt, out, ws, st, job);
  if (e != hipSuccess) return hip_fail(c, e, "mttkrp launch");
  return MTK_OK;
}

mtk_status mttkrp(mtk_ctx* c, const mtk_tensor* X, const float* const factors[3], int64_t R, int mode, int prec,
                  float* out, void* stream) {
  if (!c) return MTK_EINVAL;
  mtk_status s = check_tensor(c, X);
  if (s != MTK_OK) return s;
  if ((s = check_prec(c, X, prec)) != MTK_OK) return s;
  if (mode < 0 || mode > 2) return fail(c, MTK_EINVAL, "mode must be 0, 1 or 2");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  if (!factors || !out) return fail(c, MTK_EINVAL, "NULL factors or out");
  for (int m = 0; m < 3; ++m)
    if (m != mode && !factors[m]) return fail(c, MTK_EINVAL, "NULL factor pointer");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = ensure_ws(c, mttkrp_ws(X->dims, (int)R, mode, prec), st)) != MTK_OK) return s;
  return mttkrp_impl(c, X, factors, (int)R, mode, prec, out, c->ws, st);
}

mtk_status mttkrp_noalloc(mtk_ctx* c, const mtk_tensor* X, const float* const factors[3], int64_t R, int mode,
                          int prec, float* out, void* stream) {
  if (!c) return MTK_EINVAL;
  mtk_status s = check_tensor(c, X);
  if (s != MTK_OK) return s;
  if ((s = check_prec(c, X, prec)) != MTK_OK) return s;
  if (mode < 0 || mode > 2) return fail(c, MTK_EINVAL, "mode must be 0, 1 or 2");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  if (!factors || !out) return fail(c, MTK_EINVAL, "NULL factors or out");
  for (int m = 0; m < 3; ++m)
    if (m != mode && !factors[m]) return fail(c, MTK_EINVAL, "NULL factor pointer");
  if (!c->scratch) return fail(c, MTK_EHIP, "no device address for the static scratch");
  // The same plan as mttkrp (so the same result, bit for bit); its
  // partial slices and FP8 fragment codes must fit the static scratch.
  const bool tr = mode == 2 && X->fmt == MTK_FP8_E4M3 && X->data_t != nullptr;
  const ContractPlan p = mtk::make_plan(X->dims, (int)R, mode, prec, aligned16(tr ? X->data_t : X->data), tr);
  const size_t need = m1_route(X->dims, (int)R, mode, X->fmt, prec) ? mtk::ttm_m1_ws_bytes(X->dims, (int)R)
                                                                     : mtk::contract_ws_bytes(p, prec);
  if (need > kNoAllocScratchBytes)
    return fail(c, MTK_EUNSUPPORTED, "mttkrp_noalloc: this shape needs " + std::to_string(need) +
                                         " bytes of scratch, above the " + std::to_string(kNoAllocScratchBytes) +
                                         "-byte static buffer (use mttkrp)");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  return mttkrp_impl(c, X, factors, (int)R, mode, prec, out, c->scratch, static_cast<hipStream_t>(stream));
}

// The three-way view of an N-way mode-n MTTKRP: dimensions (v[0], v[1],
// v[2]), the output's position vm in it, and for the two other positions
// the range of original modes [lo, hi) merged into them (one mode: its own
// factor; several: their Khatri-Rao product).  A first or last mode splits
// the other modes into two groups of balanced size.
struct NwayView {
  int64_t v[3];
  int vm;
  int lo[3], hi[3];
};

static NwayView nway_view(int n, const int64_t* d, int mode) {
  NwayView w{};
  auto prod = [&](int a, int b) { int64_t p = 1; for (int m = a; m < b; ++m) p *= d[m]; return p; };
  auto split = [&](int a, int b) {           // cut [a, b) at s, a < s < b, balancing the products
    int best = a + 1;
    double bd = 1e300;
    for (int s = a + 1; s < b; ++s) {
      const double x = std::fabs(std::log((double)prod(a, s)) - std::log((double)prod(s, b)));
      if (x < bd) { bd = x; best = s; }
    }
    return best;
  };
  if (mode == 0) {
    const int s = split(1, n);
    w.vm = 0; w.lo[0] = 0; w.hi[0] = 1; w.lo[1] = 1; w.hi[1] = s; w.lo[2] = s; w.hi[2] = n;
  } else if (mode == n - 1) {
    const int s = split(0, n - 1);
    w.vm = 2; w.lo[0] = 0; w.hi[0] = s; w.lo[1] = s; w.hi[1] = n - 1; w.lo[2] = n - 1; w.hi[2] = n;
  } else {
    w.vm = 1; w.lo[0] = 0; w.hi[0] = mode; w.lo[1] = mode; w.hi[1] = mode + 1; w.lo[2] = mode + 1; w.hi[2] = n;
  }
  for (int p = 0; p < 3; ++p) w.v[p] = prod(w.lo[p], w.hi[p]);
  return w;
}

mtk_status mttkrp_nway(mtk_ctx* c, const float* X, int nmodes, const int64_t* dims, const float* const* factors,
                       int64_t R, int mode, int prec, float* out, void* stream) {
  if (!c) return MTK_EINVAL;
  if (!X || !dims || !factors || !out) return fail(c, MTK_EINVAL, "NULL argument");
  if (nmodes < 3 || nmodes > mtk::kMaxNwayModes) return fail(c, MTK_EINVAL, "nmodes must be in [3, 8]");
  if (mode < 0 || mode >= nmodes) return fail(c, MTK_EINVAL, "mode out of range");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  if (prec != MTK_FP32 && prec != MTK_BF16X3 && prec != MTK_BF16X6)
    return fail(c, MTK_EINVAL, "mttkrp_nway: prec must be MTK_FP32, MTK_BF16X3 or MTK_BF16X6");
  if (reinterpret_cast<uintptr_t>(X) & 3) return fail(c, MTK_EINVAL, "X not 4-byte aligned");
  double total = 1.0;
  for (int m = 0; m < nmodes; ++m) {
    if (dims[m] < 1 || dims[m] > (1 << 30)) return fail(c, MTK_EINVAL, "dims out of range");
    total *= (double)dims[m];
    if (m != mode && !factors[m]) return fail(c, MTK_EINVAL, "NULL factor pointer");
  }
  if (total >= 1099511627776.0) return fail(c, MTK_EINVAL, "tensor has 2^40 elements or more");
  const NwayView w = nway_view(nmodes, dims, mode);
  for (int p = 0; p < 3; ++p)
    if (w.v[p] > (1 << 30)) return fail(c, MTK_EUNSUPPORTED, "mttkrp_nway: a merged dimension exceeds 2^30");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // Workspace: the merged groups' Khatri-Rao products, then the contraction's.
  size_t kr_bytes[3] = {0, 0, 0};
  for (int p = 0; p < 3; ++p)
    if (p != w.vm && w.hi[p] - w.lo[p] > 1) kr_bytes[p] = round256((size_t)w.v[p] * R * sizeof(float));
  mtk_tensor t3{X, nullptr, {w.v[0], w.v[1], w.v[2]}, MTK_FP32, nullptr};
  const size_t need = kr_bytes[0] + kr_bytes[1] + kr_bytes[2] + mttkrp_ws(t3.dims, (int)R, w.vm, prec);
  mtk_status s = ensure_ws(c, need, st);
  if (s != MTK_OK) return s;
  char* wp = static_cast<char*>(c->ws);
  const float* f3[3] = {nullptr, nullptr, nullptr};
  for (int p = 0; p < 3; ++p) {
    if (p == w.vm) continue;
    if (w.hi[p] - w.lo[p] == 1) {
      f3[p] = factors[w.lo[p]];
      continue;
    }
    float* kr = reinterpret_cast<float*>(wp);
    wp += kr_bytes[p];
    hipError_t e = mtk::launch_kr_rows(factors + w.lo[p], dims + w.lo[p], w.hi[p] - w.lo[p], (int)R, kr, st);
    if (e != hipSuccess) return hip_fail(c, e, "Khatri-Rao launch");
    f3[p] = kr;
  }
  return mttkrp_impl(c, &t3, f3, (int)R, w.vm, prec, out, wp, st);
}

mtk_status als_sweep_nway(mtk_ctx* c, const float* X, int nmodes, const int64_t* dims, float* const* factors,
                          double* lambda, int64_t R, int prec, int nsweeps, void* stream) {
  if (!c) return MTK_EINVAL;
  if (!X || !dims || !factors || !lambda) return fail(c, MTK_EINVAL, "NULL argument");
  if (nmodes < 3 || nmodes > mtk::kMaxNwayModes) return fail(c, MTK_EINVAL, "nmodes must be in [3, 8]");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  if (nsweeps < 0) return fail(c, MTK_EINVAL, "nsweeps must be >= 0");
  if (prec != MTK_FP32 && prec != MTK_BF16X3 && prec != MTK_BF16X6)
    return fail(c, MTK_EINVAL, "als_sweep_nway: prec must be MTK_FP32, MTK_BF16X3 or MTK_BF16X6");
  if (reinterpret_cast<uintptr_t>(X) & 3) return fail(c, MTK_EINVAL, "X not 4-byte aligned");
  double total = 1.0;
  for (int m = 0; m < nmodes; ++m) {
    if (dims[m] < 1 || dims[m] > (1 << 30)) return fail(c, MTK_EINVAL, "dims out of range");
    if (!factors[m]) return fail(c, MTK_EINVAL, "NULL factor pointer");
    total *= (double)dims[m];
  }
  if (total >= 1099511627776.0) return fail(c, MTK_EINVAL, "tensor has 2^40 elements or more");
  // Workspace: [solve region][M][Khatri-Rao matrices of the two merged
  // groups][contraction], each part sized for the largest over the modes.
  size_t solve_b = 0, m_b = 0, kr_b = 0, con_b = 0;
  for (int n = 0; n < nmodes; ++n) {
    const NwayView w = nway_view(nmodes, dims, n);
    for (int p = 0; p < 3; ++p)
      if (w.v[p] > (1 << 30)) return fail(c, MTK_EUNSUPPORTED, "als_sweep_nway: a merged dimension exceeds 2^30");
    const int64_t d3[3] = {w.v[0], w.v[1], w.v[2]};
    solve_b = std::max(solve_b, mtk::solve_ws_bytes(std::max(d3[0], std::max(d3[1], d3[2])), (int)R));
    m_b = std::max(m_b, round256((size_t)dims[n] * R * sizeof(float)));
    size_t k = 0;
    for (int p = 0; p < 3; ++p)
      if (p != w.vm && w.hi[p] - w.lo[p] > 1) k += round256((size_t)w.v[p] * R * sizeof(float));
    kr_b = std::max(kr_b, k);
    con_b = std::max(con_b, mttkrp_ws(d3, (int)R, w.vm, prec));
  }
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  mtk_status s = ensure_ws(c, round256(solve_b) + m_b + kr_b + con_b, st);
  if (s != MTK_OK) return s;
  char* solve_ws = static_cast<char*>(c->ws);
  float* M = reinterpret_cast<float*>(solve_ws + round256(solve_b));
  char* kr_ws = reinterpret_cast<char*>(M) + m_b;
  void* cws = kr_ws + kr_b;
  for (int sw = 0; sw < nsweeps; ++sw)
    for (int n = 0; n < nmodes; ++n) {
      // Mode n in the three-way view (P, d_n, Q): the merged groups' factors
      // are their Khatri-Rao products, whose Gram matrices are the Hadamard
      // products of their factors' Grams, so the three-way update is the
      // N-way one.
      const NwayView w = nway_view(nmodes, dims, n);
      const int64_t d3[3] = {w.v[0], w.v[1], w.v[2]};
      const mtk_tensor t3{X, nullptr, {d3[0], d3[1], d3[2]}, MTK_FP32, nullptr};
      const float* f3[3] = {nullptr, nullptr, nullptr};
      char* wp = kr_ws;
      for (int p = 0; p < 3; ++p) {
        if (p == w.vm) {
          f3[p] = factors[n];
          continue;
        }
        if (w.hi[p] - w.lo[p] == 1) {
          f3[p] = factors[w.lo[p]];
          continue;
        }
        float* kr = reinterpret_cast<float*>(wp);
        wp += round256((size_t)w.v[p] * R * sizeof(float));
        hipError_t e = mtk::launch_kr_rows(factors + w.lo[p], dims + w.lo[p], w.hi[p] - w.lo[p], (int)R, kr, st);
        if (e != hipSuccess) return hip_fail(c, e, "Khatri-Rao launch");
        f3[p] = kr;
      }
      if ((s = mttkrp_impl(c, &t3, f3, (int)R, w.vm, prec, M, cws, st)) != MTK_OK) return s;
      hipError_t e = mtk::launch_gram_solve(f3, d3, (int)R, w.vm, M, factors[n], lambda, solve_ws, c->d_status, st);
      if (e != hipSuccess) return hip_fail(c, e, "N-way update launch");
    }
  return mtk_check(c, stream);
}

mtk_status mttkrp_dimtree(mtk_ctx* c, const mtk_tensor* X, const float* const factors[3], int64_t R, int mode,
                          int prec, float* out, void* stream) {
  if (!c) return MTK_EINVAL;
  mtk_status s = check_tensor(c, X);
  if (s != MTK_OK) return s;
  if ((s = check_prec(c, X, prec)) != MTK_OK) return s;
  if (X->fmt != MTK_FP32) return fail(c, MTK_EINVAL, "mttkrp_dimtree takes an FP32 tensor (prec MTK_FP32, MTK_BF16X3 or MTK_BF16X6)");
  if (mode != 0 && mode != 1) return fail(c, MTK_EINVAL, "mttkrp_dimtree: mode must be 0 or 1");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  if (!factors || !out || !factors[2] || !factors[1 - mode]) return fail(c, MTK_EINVAL, "NULL factors or out");
  if (X->dims[0] * X->dims[1] > mtk::kDimtreeMaxRows)
    return fail(c, MTK_EUNSUPPORTED, "mttkrp_dimtree: dims[0]*dims[1] above 2^36");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = ensure_ws(c, mtk::dimtree_ws_bytes(X->dims, (int)R), st)) != MTK_OK) return s;
  hipError_t e = mtk::launch_dimtree_mttkrp(mode, true, static_cast<const float*>(X->data), aligned16(X->data),
                                            X->dims, factors, (int)R, prec, out, c->ws, st, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "dimension-tree launch");
  return MTK_OK;
}

int mtk_sweep_uses_dimtree(const int64_t dims[3], int64_t R, int prec) {
  if (!dims || !dims_ok(dims) || R < 1 || R > mtk::kMaxRank) return 0;
  return mtk::dimtree_used(dims, (int)R, prec) ? 1 : 0;
}

mtk_status gram_solve(mtk_ctx* c, const float* const factors[3], const int64_t dims[3], int64_t R, int mode,
                      const float* M, float* factor_out, double* lambda_out, void* stream) {
  if (!c) return MTK_EINVAL;
  if (!factors || !dims || !M || !factor_out || !lambda_out) return fail(c, MTK_EINVAL, "NULL argument");
  if (!factor_dims_ok(dims)) return fail(c, MTK_EINVAL, "dims out of range (each in [1, 2^30])");
  if (mode < 0 || mode > 2) return fail(c, MTK_EINVAL, "mode must be 0, 1 or 2");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  for (int m = 0; m < 3; ++m)
    if (m != mode && !factors[m]) return fail(c, MTK_EINVAL, "NULL factor pointer");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  mtk_status s = ensure_ws(c, mtk::solve_ws_bytes(maxdim, (int)R), st);
  if (s != MTK_OK) return s;
  hipError_t e = mtk::launch_gram_solve(factors, dims, (int)R, mode, M, factor_out, lambda_out, c->ws,
                                        c->d_status, st);
  if (e != hipSuccess) return hip_fail(c, e, "gram_solve launch");
  return MTK_OK;
}

mtk_status mtk_fit(mtk_ctx* c, const mtk_tensor* X, const float* const factors[3], const double* lambda,
                   int64_t R, double* fit_host, void* stream) {
  if (!c) return MTK_EINVAL;
  mtk_status s = check_tensor(c, X);
  if (s != MTK_OK) return s;
  if (!factors || !factors[0] || !factors[1] || !factors[2] || !lambda || !fit_host)
    return fail(c, MTK_EINVAL, "NULL argument");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = ensure_ws(c, mtk::fit_ws_bytes(X->dims), st)) != MTK_OK) return s;
  hipError_t e = mtk::launch_fit(X->data, X->fmt, X->slice_exp, X->dims, factors, lambda, (int)R, c->d_fit, c->ws, st);
  if (e != hipSuccess) return hip_fail(c, e, "fit launch");
  double acc[2];
  HIP_OR_FAIL(c, hipMemcpyAsync(acc, c->d_fit, sizeof(acc), hipMemcpyDeviceToHost, st));
  HIP_OR_FAIL(c, hipStreamSynchronize(st));
  *fit_host = 1.0 - std::sqrt(acc[0]) / std::sqrt(acc[1]);
  return MTK_OK;
}

// One CP-ALS sweep (modes 0, 1, 2) enqueued on `st`, optionally followed by
// the fit partial sums into c->d_fit.  M buffer and contraction scratch (cws)
// come from ws.
// Per mode: MTTKRP, then the update (LDL^T / Gauss-Jordan inverse of V from the Gram
// matrices kept in the solve region, F = M V^{-1}, normalise, and the Gram
// matrix of the new factor); for large R the factorisation runs on the
// side stream concurrently with the MTTKRP.  The Gram matrices of factors 1 and 2 must be
// in the solve region before the first sweep (enqueue_initial_grams).
static void* sweep_solve_ws(mtk_ctx* c, const int64_t dims[3], int R, int prec) {
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  char* cws = static_cast<char*>(c->ws) + round256((size_t)maxdim * R * sizeof(float));
  return cws + sweep_contract_bytes(dims, R, prec);
}

static void* sweep_dimtree_ws(mtk_ctx* c, const int64_t dims[3], int R, int prec) {
  if (!mtk::dimtree_used(dims, R, prec)) return nullptr;
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  return static_cast<char*>(sweep_solve_ws(c, dims, R, prec)) + mtk::solve_ws_bytes(maxdim, R);
}

// The mode-n MTTKRP of a sweep, into *ms: modes 0 and 1 from the dimension
// tree when the sweep uses one (dt_ws != nullptr; its split-K slices go to
// the update unreduced), otherwise the direct contraction into M.
static mtk_status sweep_mttkrp(mtk_ctx* c, const mtk_tensor* X, const float* const cf[3], int R, int n, int prec,
                               float* M, void* cws, void* dt_ws, hipStream_t st, mtk::MSlices* ms,
                               const mtk::FactorArgs* job = nullptr) {
  *ms = mtk::MSlices{M, 1, 0};
  if (dt_ws && n < 2) {
    hipError_t e = mtk::launch_dimtree_mttkrp(n, n == 0, static_cast<const float*>(X->data), aligned16(X->data),
                                              X->dims, cf, R, prec, M, dt_ws, st, job, ms);
    if (e != hipSuccess) return hip_fail(c, e, "dimension-tree launch");
    return MTK_OK;
  }
  return mttkrp_impl(c, X, cf, R, n, prec, M, cws, st, job);
}

static mtk_status enqueue_initial_grams(mtk_ctx* c, const mtk_tensor* X, float* const factors[3], int R, int prec,
                                        hipStream_t st) {
  const int64_t maxdim = std::max(X->dims[0], std::max(X->dims[1], X->dims[2]));
  const float* cf[3] = {factors[0], factors[1], factors[2]};
  hipError_t e = mtk::launch_grams(cf, X->dims, R, 1, 2, maxdim, sweep_solve_ws(c, X->dims, R, prec), c->d_status, st);
  if (e != hipSuccess) return hip_fail(c, e, "Gram launch");
  return MTK_OK;
}

// How an update's factorisation (V^{-1}) is placed against the MTTKRP it
// does not depend on.  R <= kJobMaxRank: as one extra workgroup of the
// contraction launch.  R >= kOverlapMinRank: on the side stream (a
// cross-stream dependency costs about 10 us, hidden from R = 64 on).  In
// between: its own launch after the MTTKRP.
constexpr int kOverlapMinRank = 41;

static mtk_status enqueue_sweep(mtk_ctx* c, const mtk_tensor* X, float* const factors[3], double* lambda, int R,
                                int prec, bool with_fit, hipStream_t st) {
  const int64_t maxdim = std::max(X->dims[0], std::max(X->dims[1], X->dims[2]));
  float* M = static_cast<float*>(c->ws);
  void* cws = static_cast<char*>(c->ws) + round256((size_t)maxdim * R * sizeof(float));
  void* solve_ws = sweep_solve_ws(c, X->dims, R, prec);
  void* dt_ws = sweep_dimtree_ws(c, X->dims, R, prec);
  const float* cf[3] = {factors[0], factors[1], factors[2]};
  const bool overlap = R >= kOverlapMinRank;
  const bool tree = mtk::dimtree_used(X->dims, R, prec);
  for (int n = 0; n < 3; ++n) {
    if (R <= mtk::kJobMaxRank) {
      const mtk::FactorArgs f = mtk::factor_args(X->dims, R, n, maxdim, solve_ws, c->d_status);
      mtk::MSlices ms;
      mtk_status s = sweep_mttkrp(c, X, cf, R, n, prec, M, cws, dt_ws, st, &ms, &f);
      if (s != MTK_OK) return s;
      hipError_t e = mtk::launch_apply(X->dims, R, n, ms, factors[n], lambda, maxdim, solve_ws, c->d_status, st,
                                       n == 2);
      if (e != hipSuccess) return hip_fail(c, e, "update launch");
      continue;
    }
    if (!overlap) {
      mtk::MSlices ms;
      mtk_status s = sweep_mttkrp(c, X, cf, R, n, prec, M, cws, dt_ws, st, &ms);
      if (s != MTK_OK) return s;
      hipError_t e = mtk::launch_update(X->dims, R, n, ms, factors[n], lambda, maxdim, solve_ws, c->d_status, st,
                                        n == 2);
      if (e != hipSuccess) return hip_fail(c, e, "update launch");
      continue;
    }
    // In a captured graph the runtime keeps a node's first-captured child
    // on its queue.  With the dimension tree the MTTKRPs (the Y kernel, the
    // mode-3 contraction) run far longer than the factorisation: the MTTKRP
    // is enqueued first (the fork still recorded before it), so it and the
    // update stay on one queue and only the factorisation crosses over.
    // With three contractions (FP8; short K) an MTTKRP takes about as long
    // as the factorisation, which then needs a free CU at the start (on a
    // full GPU it runs twice as long): the factorisation is enqueued first.
    const bool mttkrp_first = tree;
    HIP_OR_FAIL(c, hipEventRecord(c->fork_ev[n], st));
    mtk::MSlices ms;
    if (mttkrp_first) {
      mtk_status s = sweep_mttkrp(c, X, cf, R, n, prec, M, cws, dt_ws, st, &ms);
      if (s != MTK_OK) return s;
    }
    HIP_OR_FAIL(c, hipStreamWaitEvent(c->side, c->fork_ev[n], 0));
    hipError_t e = mtk::launch_factor(X->dims, R, n, maxdim, solve_ws, c->d_status, c->side);
    if (e != hipSuccess) return hip_fail(c, e, "factorisation launch");
    HIP_OR_FAIL(c, hipEventRecord(c->join_ev[n], c->side));
    if (!mttkrp_first) {
      mtk_status s = sweep_mttkrp(c, X, cf, R, n, prec, M, cws, dt_ws, st, &ms);
      if (s != MTK_OK) return s;
    }
    HIP_OR_FAIL(c, hipStreamWaitEvent(st, c->join_ev[n], 0));
    e = mtk::launch_apply(X->dims, R, n, ms, factors[n], lambda, maxdim, solve_ws, c->d_status, st, n == 2);
    if (e != hipSuccess) return hip_fail(c, e, "update launch");
  }
  if (with_fit) {
    hipError_t e = mtk::launch_fit(X->data, X->fmt, X->slice_exp, X->dims, cf, lambda, R, c->d_fit, cws, st);
    if (e != hipSuccess) return hip_fail(c, e, "fit launch");
  }
  return MTK_OK;
}

// The captured sweep for these buffers (created and cached on first use).
static mtk_status sweep_graph(mtk_ctx* c, const mtk_tensor* X, float* const factors[3], double* lambda, int R,
                              int prec, bool with_fit, hipGraphExec_t* out) {
  GraphCache* gc = static_cast<GraphCache*>(c->graph_cache);
  GraphKey key{};
  key.X = X->data;
  key.Xt = X->data_t;
  for (int m = 0; m < 3; ++m) { key.dims[m] = X->dims[m]; key.f[m] = factors[m]; }
  key.fmt = X->fmt;
  key.slice_exp = X->slice_exp;
  key.lambda = lambda;
  key.R = R;
  key.prec = prec;
  key.with_fit = with_fit;
  auto it = gc->execs.find(key);
  if (it != gc->execs.end()) {
    *out = it->second;
    return MTK_OK;
  }
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_OR_FAIL(c, hipStreamBeginCapture(gc->capture_stream, hipStreamCaptureModeThreadLocal));
  mtk_status s = enqueue_sweep(c, X, factors, lambda, R, prec, with_fit, gc->capture_stream);
  hipError_t ee = hipStreamEndCapture(gc->capture_stream, &g);
  if (s != MTK_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (ee != hipSuccess) return hip_fail(c, ee, "hipStreamEndCapture");
  ee = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  if (ee != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(c, ee, "hipGraphInstantiate");
  }
  gc->graphs.push_back(g);
  gc->execs[key] = exec;
  *out = exec;
  return MTK_OK;
}

mtk_status als_sweep(mtk_ctx* c, const mtk_tensor* X, float* const factors[3], double* lambda, int64_t R, int prec,
                     int nsweeps, double* fit_host, void* stream) {
  if (!c) return MTK_EINVAL;
  mtk_status s = check_tensor(c, X);
  if (s != MTK_OK) return s;
  if ((s = check_prec(c, X, prec)) != MTK_OK) return s;
  if (!factors || !factors[0] || !factors[1] || !factors[2] || !lambda) return fail(c, MTK_EINVAL, "NULL argument");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  if (nsweeps < 0) return fail(c, MTK_EINVAL, "nsweeps < 0");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t maxdim = std::max(X->dims[0], std::max(X->dims[1], X->dims[2]));
  const size_t need = round256((size_t)maxdim * R * sizeof(float)) + sweep_scratch_bytes(X->dims, (int)R, prec);
  if ((s = ensure_ws(c, need, st)) != MTK_OK) return s;   // growing it drops the cached graphs
  if (nsweeps == 0) return mtk_check(c, stream);

  const bool with_fit = fit_host != nullptr;
  hipGraphExec_t exec = nullptr;
  if ((s = sweep_graph(c, X, factors, lambda, (int)R, prec, with_fit, &exec)) != MTK_OK) return s;
  // The Gram matrices the first mode needs; every later one is formed by the
  // update that writes its factor.
  if ((s = enqueue_initial_grams(c, X, factors, (int)R, prec, st)) != MTK_OK) return s;
  std::vector<double> acc(with_fit ? 2 * (size_t)nsweeps : 0);
  for (int sw = 0; sw < nsweeps; ++sw) {
    HIP_OR_FAIL(c, hipGraphLaunch(exec, st));
    if (with_fit)
      HIP_OR_FAIL(c, hipMemcpyAsync(&acc[2 * (size_t)sw], c->d_fit, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  s = mtk_check(c, stream);
  if (with_fit)
    for (int sw = 0; sw < nsweeps; ++sw) fit_host[sw] = 1.0 - std::sqrt(acc[2 * sw]) / std::sqrt(acc[2 * sw + 1]);
  return s;
}

// Region of the extrapolation candidate, after the sweep's scratch: the
// first two factors as a sweep found them, the candidate's three factors,
// its lambda (and a discarded one), and a solve region of its own.
struct LsRegion {
  float* prev[2];
  float* cand[3];
  double* lam;
  double* lam_discard;
  void* solve;
};

static size_t ls_region_bytes(const int64_t dims[3], int R) {
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  size_t b = 0;
  for (int m = 0; m < 2; ++m) b += 2 * round256((size_t)dims[m] * R * sizeof(float));
  b += round256((size_t)dims[2] * R * sizeof(float)) + 2 * round256((size_t)R * sizeof(double));
  return b + mtk::solve_ws_bytes(maxdim, R);
}

static LsRegion ls_region(char* p, const int64_t dims[3], int R) {
  LsRegion r{};
  auto take = [&](size_t bytes) {
    char* q = p;
    p += round256(bytes);
    return q;
  };
  for (int m = 0; m < 2; ++m) r.prev[m] = reinterpret_cast<float*>(take((size_t)dims[m] * R * sizeof(float)));
  for (int m = 0; m < 3; ++m) r.cand[m] = reinterpret_cast<float*>(take((size_t)dims[m] * R * sizeof(float)));
  r.lam = reinterpret_cast<double*>(take((size_t)R * sizeof(double)));
  r.lam_discard = reinterpret_cast<double*>(take((size_t)R * sizeof(double)));
  r.solve = p;
  return r;
}

// CP-ALS until the fit settles, optionally with an extrapolation candidate
// after every sweep s >= ls_start (ls_start <= 0: none).
static mtk_status als_run_impl(mtk_ctx* c, const mtk_tensor* X, float* const factors[3], double* lambda, int64_t R,
                               int prec, int max_sweeps, double tol, int ls_start, double* fits_host,
                               int* accepted_host, int* sweeps_done, double* fit_final, void* stream) {
  if (!c) return MTK_EINVAL;
  mtk_status s = check_tensor(c, X);
  if (s != MTK_OK) return s;
  if ((s = check_prec(c, X, prec)) != MTK_OK) return s;
  if (!factors || !factors[0] || !factors[1] || !factors[2] || !lambda || !sweeps_done)
    return fail(c, MTK_EINVAL, "NULL argument");
  if (R < 1 || R > mtk::kMaxRank) return fail(c, MTK_EINVAL, "R must be in [1, 128]");
  if (max_sweeps < 0) return fail(c, MTK_EINVAL, "max_sweeps < 0");
  if (!(tol >= 0.0)) return fail(c, MTK_EINVAL, "tol must be >= 0");
  *sweeps_done = 0;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t* dims = X->dims;
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  const size_t m_bytes = round256((size_t)maxdim * R * sizeof(float));
  const size_t sweep_b = sweep_scratch_bytes(dims, (int)R, prec);
  const bool ls = ls_start > 0 && max_sweeps >= ls_start;
  const size_t need = m_bytes + sweep_b + (ls ? ls_region_bytes(dims, (int)R) : 0);
  if ((s = ensure_ws(c, need, st)) != MTK_OK) return s;
  float* M = static_cast<float*>(c->ws);
  void* cws = static_cast<char*>(c->ws) + m_bytes;
  const float* cf[3] = {factors[0], factors[1], factors[2]};
  if (max_sweeps > 0) {
    hipGraphExec_t exec = nullptr;
    if ((s = sweep_graph(c, X, factors, lambda, (int)R, prec, false, &exec)) != MTK_OK) return s;
    double acc[2] = {0.0, 0.0};
    hipError_t e = mtk::launch_sumsq(X->data, X->fmt, X->slice_exp, dims, c->d_fit, cws, st);
    if (e != hipSuccess) return hip_fail(c, e, "norm launch");
    HIP_OR_FAIL(c, hipMemcpyAsync(acc, c->d_fit, sizeof(acc), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(c, hipStreamSynchronize(st));   // acc is host memory written by the copy
    if ((s = enqueue_initial_grams(c, X, factors, (int)R, prec, st)) != MTK_OK) return s;
    void* live_solve = sweep_solve_ws(c, dims, (int)R, prec);
    const double* ip_dev = mtk::solve_ip(maxdim, (int)R, live_solve);
    const LsRegion lr = ls ? ls_region(static_cast<char*>(cws) + sweep_b, dims, (int)R) : LsRegion{};
    const double* cand_ip_dev = ls ? mtk::solve_ip(maxdim, (int)R, lr.solve) : nullptr;
    const double nx2 = acc[1];
    auto fit_of = [&](double ip) { return 1.0 - std::sqrt(std::max(0.0, nx2 - ip)) / std::sqrt(nx2); };
    double prev = 0.0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
      const int sweep_no = sw + 1;
      const bool try_ls = ls && sweep_no >= ls_start;
      if (try_ls)
        for (int m = 0; m < 2; ++m)
          HIP_OR_FAIL(c, hipMemcpyAsync(lr.prev[m], factors[m], (size_t)dims[m] * R * sizeof(float),
                                        hipMemcpyDeviceToDevice, st));
      HIP_OR_FAIL(c, hipGraphLaunch(exec, st));
      double ip = 0.0;
      int status = 0;
      HIP_OR_FAIL(c, hipMemcpyAsync(&ip, ip_dev, sizeof(ip), hipMemcpyDeviceToHost, st));
      HIP_OR_FAIL(c, hipMemcpyAsync(&status, c->d_status, sizeof(status), hipMemcpyDeviceToHost, st));
      HIP_OR_FAIL(c, hipStreamSynchronize(st));
      *sweeps_done = sweep_no;
      if (status != 0) break;                    // reported by mtk_check below
      // At the least-squares solution of the last update, ||Xhat||^2 = <X, Xhat> = <F, M>.
      double fit = fit_of(ip);
      int took = 0;
      if (try_ls) {
        // Candidate: the first two factors moved further along their change
        // over this sweep, the third solved exactly from them.
        const double d = std::cbrt((double)sweep_no);
        for (int m = 0; m < 2; ++m) {
          e = mtk::launch_extrapolate(dims, (int)R, m, lr.prev[m], factors[m], d, lr.cand[m], lr.lam_discard, maxdim,
                                      lr.solve, c->d_status, st);
          if (e != hipSuccess) return hip_fail(c, e, "extrapolation launch");
        }
        const float* ef[3] = {lr.cand[0], lr.cand[1], factors[2]};
        if ((s = mttkrp_impl(c, X, ef, (int)R, 2, prec, M, cws, st)) != MTK_OK) return s;
        e = mtk::launch_update(dims, (int)R, 2, M, lr.cand[2], lr.lam, maxdim, lr.solve, c->d_status, st, true);
        if (e != hipSuccess) return hip_fail(c, e, "extrapolation update launch");
        double cip = 0.0;
        HIP_OR_FAIL(c, hipMemcpyAsync(&cip, cand_ip_dev, sizeof(cip), hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(c, hipMemcpyAsync(&status, c->d_status, sizeof(status), hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(c, hipStreamSynchronize(st));
        if (status != 0) break;
        const double cfit = fit_of(cip);
        if (cfit > fit) {
          for (int m = 0; m < 3; ++m)
            HIP_OR_FAIL(c, hipMemcpyAsync(factors[m], lr.cand[m], (size_t)dims[m] * R * sizeof(float),
                                          hipMemcpyDeviceToDevice, st));
          HIP_OR_FAIL(c, hipMemcpyAsync(lambda, lr.lam, (size_t)R * sizeof(double), hipMemcpyDeviceToDevice, st));
          // The next sweep's first update reads the Gram matrices of the
          // second and third factors from the live solve region.
          if ((s = enqueue_initial_grams(c, X, factors, (int)R, prec, st)) != MTK_OK) return s;
          fit = cfit;
          took = 1;
        }
      }
      if (fits_host) fits_host[sw] = fit;
      if (accepted_host) accepted_host[sw] = took;
      if (sw > 0 && std::fabs(fit - prev) < tol) break;
      prev = fit;
    }
  }
  if (fit_final) {
    double acc[2] = {0.0, 0.0};
    hipError_t e = mtk::launch_fit(X->data, X->fmt, X->slice_exp, dims, cf, lambda, (int)R, c->d_fit, cws, st);
    if (e != hipSuccess) return hip_fail(c, e, "fit launch");
    HIP_OR_FAIL(c, hipMemcpyAsync(acc, c->d_fit, sizeof(acc), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(c, hipStreamSynchronize(st));
    *fit_final = 1.0 - std::sqrt(acc[0]) / std::sqrt(acc[1]);
  }
  return mtk_check(c, stream);
}

mtk_status als_run(mtk_ctx* c, const mtk_tensor* X, float* const factors[3], double* lambda, int64_t R, int prec,
                   int max_sweeps, double tol, double* fits_host, int* sweeps_done, double* fit_final, void* stream) {
  return als_run_impl(c, X, factors, lambda, R, prec, max_sweeps, tol, 0, fits_host, nullptr, sweeps_done, fit_final,
                      stream);
}

mtk_status als_run_extrapolated(mtk_ctx* c, const mtk_tensor* X, float* const factors[3], double* lambda, int64_t R,
                                int prec, int max_sweeps, double tol, int ls_start, double* fits_host,
                                int* accepted_host, int* sweeps_done, double* fit_final, void* stream) {
  if (c && ls_start < 1) return fail(c, MTK_EINVAL, "ls_start must be >= 1");
  return als_run_impl(c, X, factors, lambda, R, prec, max_sweeps, tol, ls_start, fits_host, accepted_host,
                      sweeps_done, fit_final, stream);
}

}  // extern "C"
