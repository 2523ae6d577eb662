// Internal declarations shared by the HIP sources of libmttkrp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mttkrp.h"

namespace mtk {

// Largest factor rank the kernels are instantiated for (8 MFMA N-tiles of 16).
constexpr int kMaxRank = 128;
// Lanes per wavefront on CDNA.
constexpr int kWave = 64;

// Device-side sticky status bits (OR-ed into the context's status word).
constexpr int kStatusNotSPD = 1;

// Gram partials are stored per factor as [tile pair][row block][16 x 16],
// with room for this many row blocks.
constexpr int kGramBlocksMax = 16;

// Inputs / outputs of the FP64 inversion of one update's V (see
// factor_device.h): V^{-1} from the Gram partials of the two other factors.
struct FactorArgs {
  const double* pa;   // Gram partials of the first other factor
  int na;             // its row blocks
  const double* pb;   // Gram partials of the second other factor
  int nb;
  int R;
  double* vinv;       // out: V^{-1}, R x R row-major (FP64)
  int* status;        // sticky status word (kStatusNotSPD)
};

// Work decomposition of one contraction launch (see mttkrp_kernels.hip).
struct ContractPlan {
  int nM, nRed, nLoop, R;        // extents: output rows, reduction length, outer loop length
  int64_t sM, sRed, sLoop;       // element strides of X along the three roles
  int nt;                        // MFMA N-tiles (16 columns each) covering R
  int ncg;                       // column groups: waves of a workgroup splitting R (1 or 2)
  int ntw;                       // N-tiles per wave = ceil(nt / ncg)
  int nv;                        // reduction values per lane per tile
  int kw;                        // reduction values per wave = 4 * nv
  int wr;                        // waves of a workgroup along the reduction (1, 2 or 4)
  int mt_per_wg;                 // M-tiles per workgroup = 4 / (ncg * wr)
  int n_rg;                      // reduction groups = ceil(nRed / (wr * kw))
  int n_mg;                      // M groups = ceil(ceil(nM / 16) / mt_per_wg)
  int loop_block;                // outer-loop iterations per workgroup
  int n_lb;                      // outer-loop blocks
  int slices;                    // partial slices = n_rg * n_lb
  bool vec;                      // 16-byte vector loads along a contiguous reduction
  bool cm;                       // mode 2, m contiguous: row-interleaved 64-row tiles
  int64_t grid() const { return (int64_t)n_rg * n_mg * n_lb; }
};

// Launch the mode-n contraction.  prec: MTK_FP32 / MTK_BF16X3 / MTK_FP8_E4M3.
// X_fmt tells how X is stored.  Writes `out` (nM x R FP32) using `ws`
// (at least contract_ws_bytes) for partial sums and quantised fragments.
size_t contract_ws_bytes(const ContractPlan& p, int prec);
// transposed: mode 2 of an FP8 tensor read from its per-slice transposed copy
// (element (i,j,k) at (i*K + k)*J + j), which makes the reduction over j contiguous.
ContractPlan make_plan(const int64_t dims[3], int R, int mode, int prec, bool x_aligned16,
                       bool transposed = false);
// `job` (optional, R <= kJobMaxRank): the inversion of an update's V, run
// by one extra workgroup of the same launch so that it overlaps the
// contraction (results in job->vinv once the launch has completed).
constexpr int kJobMaxRank = 32;
hipError_t launch_contract(const ContractPlan& p, int prec, int mode, const void* X,
                           const int32_t* slice_exp, const float* frag_src,
                           const float* weight, float* out, void* ws, hipStream_t st,
                           const FactorArgs* job = nullptr);
// out[e] = sum over s in order of part[s * n + e], e < n.
hipError_t launch_slice_reduce(const float* part, int slices, int64_t n, float* out, hipStream_t st);

// Dimension-tree sweep (dimtree.hip): the mode-0 and mode-1 MTTKRPs from
// Y = X x3 C (I*J x R, at the start of `ws`).  form_y: form Y first; else Y
// must still be in ws from an earlier call on the same stream with the same
// X and C (the mode-1 update of a sweep reuses the mode-0 update's Y).
// FP32 / BF16X3, FP32 tensor.  `ws`: dimtree_ws_bytes.  `job` (R <=
// kJobMaxRank) rides in the mode-0 Y launch or the mode-1 sum.
// An MTTKRP result as handed to an update: `slices` split-K partial slices
// (`sstride` floats apart) that the update adds in the split-K reduction's
// order, bit for bit; slices == 1 is the plain n x R matrix.
struct MSlices {
  const float* p;
  int slices;
  int64_t sstride;
};
// Largest dims[0]*dims[1] (rows of Y) the tree takes.
constexpr int64_t kDimtreeMaxRows = (int64_t)1 << 36;
bool dimtree_used(const int64_t dims[3], int R, int prec);
size_t dimtree_ws_bytes(const int64_t dims[3], int R);
// defer != nullptr: the sum's split-K slices are left in ws and described in
// *defer for an update to add (no reduction launch); out is then unused
// unless the sum has a single slice.
hipError_t launch_dimtree_mttkrp(int mode, bool form_y, const float* X, bool x_aligned16, const int64_t dims[3],
                                 const float* const factors[3], int R, int prec, float* out, void* ws,
                                 hipStream_t st, const FactorArgs* job, MSlices* defer = nullptr);

// N-way MTTKRP (nway.hip): Khatri-Rao product of n consecutive modes'
// factors (first mode's index slowest), rows = prod dims, into out (rows x R).
constexpr int kMaxNwayModes = 8;
hipError_t launch_kr_rows(const float* const* factors, const int64_t* dims, int n, int R, float* out,
                          hipStream_t st);

// FP8 tensor preparation (per mode-1 slice power-of-two scaled e4m3).
hipError_t launch_quantize_slices(const float* x, int64_t I, int64_t J, int64_t K, uint8_t* q,
                                  uint8_t* qt, int32_t* exps, hipStream_t st);

// FP64 Gram / solve pieces.  `status` points to a zeroed 1 KiB device
// block: word 0 is the sticky status, words 64..191 are the counters of the
// kernels' last-workgroup reductions (each reduction returns its counter to
// zero, so the block stays valid across launches and graph replays).
// `ws` holds solve_ws_bytes(maxdim, R) bytes laid out for that maxdim; the
// Gram matrices of the three factors persist there between launches.
constexpr int kStatusWords = 256;
size_t solve_ws_bytes(int64_t maxdim, int R);
// Gram matrices of factors ma and (if mb >= 0) mb into their slots.
hipError_t launch_grams(const float* const factors[3], const int64_t dims[3], int R, int ma, int mb, int64_t maxdim,
                        void* ws, int* status, hipStream_t st);
// Update of factor `mode` from its MTTKRP M, using the Gram slots of the two
// other factors: V^{-1} (LDL^T elimination in Gauss-Jordan form),
// F = M V^{-1}, lambda, the normalised FP32 factor, and the Gram slot of the
// new factor.
// with_ip: also form <F, M> (F = M V^{-1} before normalising) into the solve
// region's scalar (solve_ip); used by the last update of a sweep, where
// ||X||^2 - <F, M> is the squared residual of the updated model.
hipError_t launch_update(const int64_t dims[3], int R, int mode, const float* M, float* factor_out, double* lambda,
                         int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip = false);
// launch_update in two halves: the factorisation (V^{-1} by LDL^T /
// Gauss-Jordan elimination; reads only the Gram slots of the other two
// factors, so it may run concurrently with the mode's MTTKRP) and the rest
// (needs M).
FactorArgs factor_args(const int64_t dims[3], int R, int mode, int64_t maxdim, void* ws, int* status);
hipError_t launch_factor(const int64_t dims[3], int R, int mode, int64_t maxdim, void* ws, int* status,
                         hipStream_t st);
hipError_t launch_apply(const int64_t dims[3], int R, int mode, const float* M, float* factor_out, double* lambda,
                        int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip = false);
hipError_t launch_apply(const int64_t dims[3], int R, int mode, const MSlices& m, float* factor_out, double* lambda,
                        int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip = false);
hipError_t launch_update(const int64_t dims[3], int R, int mode, const MSlices& m, float* factor_out,
                         double* lambda, int64_t maxdim, void* ws, int* status, hipStream_t st, bool with_ip = false);
// Device address of the <F, M> scalar in a solve region laid out for maxdim.
const double* solve_ip(int64_t maxdim, int R, void* ws);
// launch_grams of the two other factors followed by launch_update.
hipError_t launch_gram_solve(const float* const factors[3], const int64_t dims[3], int R,
                             int mode, const float* M, float* factor_out, double* lambda,
                             void* ws, int* status, hipStream_t st);
size_t fit_ws_bytes(const int64_t dims[3]);
hipError_t launch_fit(const void* X, int fmt, const int32_t* slice_exp, const int64_t dims[3],
                      const float* const factors[3], const double* lambda, int R,
                      double* acc2 /* [2]: residual^2, norm^2 */, void* ws, hipStream_t st);
// acc2[1] = ||X||^2 (FP64; acc2[0] = 0); ws: fit_ws_bytes.
hipError_t launch_sumsq(const void* X, int fmt, const int32_t* slice_exp, const int64_t dims[3], double* acc2,
                        void* ws, hipStream_t st);

}  // namespace mtk

// The opaque context behind mtk_ctx* (C ABI).
struct mtk_ctx {
  int device = 0;
  void* ws = nullptr;             // workspace (partials, fragments, solve scratch)
  size_t ws_bytes = 0;
  int* d_status = nullptr;        // sticky status word + reduction counters (kStatusWords ints)
  double* d_fit = nullptr;        // fit accumulators
  std::string last_error;
  std::vector<void*> retired_ws;  // outgrown workspace blocks (freed by mtk_graph_reset / mtk_destroy)
  void* scratch = nullptr;        // device address of mttkrp_noalloc's static scratch on this device
  void* graph_cache = nullptr;    // als_sweep graph cache (see api.hip)
  hipStream_t side = nullptr;     // second stream of the captured sweep (factorisation)
  hipEvent_t fork_ev[3] = {nullptr, nullptr, nullptr};
  hipEvent_t join_ev[3] = {nullptr, nullptr, nullptr};
};
