// Grouped launches of the serving loop (server.hip).
//
// The server advances every resident request by one CP-ALS sweep per
// scheduler step.  A step is a fixed sequence of launches, each covering the
// work of all resident requests at once from a device table with one entry
// per request and update: for each of the sweep's three updates, the mode-n
// contraction of every request (grouped contraction), the inversion of
// every request's V (one workgroup each; inside the contraction launch when
// every rank fits its LDS, else a parallel branch), F = M V^{-1} for every
// request (grouped apply) and the normalisation with the new factor's Gram
// partials (grouped normalise).  Each launch has a fixed grid whose
// workgroups stride over the step's work items and find their request by a
// binary search over the entries' first work items, so the step is captured
// once as a HIP graph and replayed for any set of requests.  A request's
// work items, plan and summation orders depend only on its own shape, rank,
// mode and precision, so its result is the same alone and beside any other
// requests.
#pragma once

#include "mtk_internal.h"

namespace mtk {

// Most requests a step can carry.
constexpr int kSrvMaxReq = 64;

// One request's mode-n contraction this step (the fields of the contraction
// launch, see mttkrp_kernels.hip), cut into work items of one workgroup and
// one 16-column tile each.
struct SrvContract {
  const float* X;
  const float* frag;        // factor inside the MFMA (nRed x R)
  const float* weight;      // factor of the epilogue (nLoop x R)
  float* part;              // split-K partial slices (slices x nM x R), or M if slices == 1
  int64_t sM, sRed, sLoop;
  int nM, nRed, nLoop, R;
  int wr, mt_per_wg, n_rg, n_mg, loop_block, n_lb, nct, slices;
  int mode, prec, form;     // form: 0 contiguous 16-byte loads, 1 contiguous, 2 strided reduction
};

// One request's update of factor `mode` this step.
struct SrvUpdate {
  FactorArgs fa;            // V^{-1} from the Gram partials of the two other factors
  const float* M;           // the contraction's partial slices (added in split-K order)
  int S;
  int64_t sstride;
  int64_t n;                // rows of the factor
  int R;
  int nblk;                 // apply row blocks (16 rows)
  int nrb;                  // Gram row blocks of the new factor
  double* F;
  double* colsq;
  double* lam;
  float* fout;
  double* gram_out;         // Gram partial slot of the new factor
  const int* status;
};

struct SrvEntry {
  SrvContract c;
  SrvUpdate u;
  int64_t wi0;              // first contraction work item
  int64_t ab0;              // first apply workgroup
  int64_t nb0;              // first normalise workgroup
};

// A step's table: entry e[q][u] is request q's update u (mode u) of the sweep.
struct SrvTable {
  int nreq;
  int pad_;
  int64_t n_wi[3], n_ab[3], n_nb[3];   // work items of the strided launches, per update
  SrvEntry e[kSrvMaxReq][3];
};

// Bytes of a table holding n requests (the part the host copies each step).
inline size_t srv_table_bytes(int n) { return offsetof(SrvTable, e) + (size_t)n * 3 * sizeof(SrvEntry); }

// Contraction plan of one request in the grouped step (host): nv = 8, one
// 16-column tile per workgroup, strided or contiguous reduction; the
// partial slices need slices * nM * R floats.
SrvContract srv_contract_plan(const int64_t dims[3], int R, int mode, int prec, bool x_aligned16);
// The update of `mode` for a request whose solve region (solve_ws_bytes
// laid out for maxdim) is `solve_ws`; S / sstride describe the contraction's
// partial slices (S == 1: M itself).
SrvUpdate srv_update(const int64_t dims[3], int R, int mode, int64_t maxdim, void* solve_ws, const float* M,
                     int S, int64_t sstride, float* fout, double* lam, int* status);
int64_t srv_apply_blocks(const SrvUpdate& u);
int64_t srv_normalize_blocks(const SrvUpdate& u);
int64_t srv_contract_items(const SrvContract& c);

// Launch sizes (fixed, so a captured step fits any table).
constexpr int kSrvContractGrid = 2048;
constexpr int kSrvApplyGrid = 1024;
constexpr int kSrvNormalizeGrid = 1024;
size_t srv_contract_lds_bytes();
size_t srv_factor_lds_bytes(int max_rank);
// Largest rank whose inversion fits the contraction launch's LDS.
constexpr int kSrvFusedMaxRank = 64;

// Update u of the step in table t.  with_factor: the contraction launch's
// first nreq work items invert the requests' V (every R <= kSrvFusedMaxRank);
// otherwise launch_srv_factor does it.
hipError_t launch_srv_contract(const SrvTable* t, int u, bool with_factor, hipStream_t st);
hipError_t launch_srv_factor(const SrvTable* t, int u, int max_rank, hipStream_t st);
hipError_t launch_srv_apply(const SrvTable* t, int u, hipStream_t st);
hipError_t launch_srv_normalize(const SrvTable* t, int u, hipStream_t st);

// Device: index of the entry whose work items [first, next first) hold w.
template <class First>
__device__ __forceinline__ int srv_find(int n, int64_t w, First first) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(mid) <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace mtk
