// Sparse three-way MTTKRP over coordinates (mtk_coo_create / mttkrp_coo).
//
// M(i, r) = sum over stored entries (i, j, k, v) of v * B(j, r) * C(k, r)
// for mode 0, and the same with the roles exchanged for modes 1 and 2: the
// dense definition with the sum restricted to the stored entries (repeated
// coordinates add).
//
// Layout.  mtk_coo_create keeps, for each mode n, a copy of the entries
// sorted by their mode-n index (stable: entries with equal index keep the
// input order), each entry 16 bytes {row, a, b, value} where row is the
// mode-n index and a, b the indices of the two other modes in increasing
// mode order.  Where a gathered factor is too large for one XCD's L2, the
// mode is partitioned: the entries are first ordered by which of 8 equal
// index ranges of that factor they fall in (part; of the two gathered
// factors the one that spreads the entries more evenly), rows ascending
// within each part,
// part p is walked by workgroups of XCD p, each part writes its own partial
// output, and the partials are added in part order.  The sort is an LSD radix sort on 8-bit digits written here
// (histogram per 4096-entry tile, exclusive scan, stable scatter with
// per-wave ballot ranking).
//
// Contraction.  The sorted entries are cut into segments of L entries (L a
// multiple of 64 fixed by nnz alone).  A segment is walked by a group of RL
// lanes (RL = 8, 16, 32 or 64 by R; lane c holds columns c, c + RL, ...):
// entries are staged through LDS 16 bytes at a time and read back as a
// broadcast, both factor rows are gathered with coalesced loads, and the
// products are added in entry order.  A row that starts and ends inside a
// segment is written directly; the segment's first and last rows (which may
// continue in the neighbouring segments) go to two carry slots.  Passes over
// the carry slots, 32 at a time, reduce them the same way (rows inside a
// group written, the group's first and last rows carried on) until one
// group remains, so a heavy row that spans many segments is added along a
// tree rather than by one group in sequence.  The output is zeroed first (rows
// with no entries stay zero), every row with entries is then written by
// exactly one group, and the result does not depend on timing.  The bound is the
// gather of the factor rows (2 R floats per entry, served by L2 for factors
// that fit there) and the entry stream from HBM (16 bytes per entry).

#include <algorithm>
#include <cstring>

#include "mtk_internal.h"

namespace mtk {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 entries per tile
constexpr int kScanTile = 4096;                       // elements per scan block
constexpr int kCooMaxSeg = 1024;                      // longest segment (entries)
constexpr int kCooParts = 8;                          // parts of a partitioned mode (one per XCD)

// ----------------------------------------------------------- preparation ---

// Entries with any index outside [0, dims) are counted into *bad.
__global__ __launch_bounds__(256) void coo_range_kernel(const int32_t* __restrict__ i0, const int32_t* __restrict__ i1,
                                                        const int32_t* __restrict__ i2, int64_t nnz, int32_t d0,
                                                        int32_t d1, int32_t d2, int* bad) {
  int cnt = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = i0[e], b = i1[e], c = i2[e];
    cnt += (a < 0 || a >= d0 || b < 0 || b >= d1 || c < 0 || c >= d2) ? 1 : 0;
  }
  if (cnt) atomicAdd(bad, cnt);
}

// Digit histogram of one 4096-entry tile: hist[d * ntiles + tile].
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const int32_t* __restrict__ keys, int64_t n,
                                                                  int shift, int* __restrict__ hist, int64_t ntiles) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t e = base + (int64_t)i * kSortThreads + threadIdx.x;
    if (e < n) atomicAdd(&h[((uint32_t)keys[e] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix of x over the 256 threads of a block; *total gets the sum.
__device__ int block_excl_scan(int x, int* lds, int* total) {
  const int t = threadIdx.x;
  lds[t] = x;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int y = t >= off ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += y;
    __syncthreads();
  }
  const int incl = lds[t];
  *total = lds[255];
  __syncthreads();
  return incl - x;
}

// Exclusive scan of a[0, n) in blocks of kScanTile; sums[b] = block b's total.
__global__ __launch_bounds__(256) void scan_tiles_kernel(int* __restrict__ a, int64_t n, int* __restrict__ sums) {
  __shared__ int lds[256];
  constexpr int per = kScanTile / 256;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * per;
  int v[per];
  int s = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    v[i] = base + i < n ? a[base + i] : 0;
    s += v[i];
  }
  int total;
  int run = block_excl_scan(s, lds, &total);
#pragma unroll
  for (int i = 0; i < per; ++i) {
    if (base + i < n) a[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of sums[0, nb) by one block, in chunks of 256.
__global__ __launch_bounds__(256) void scan_sums_kernel(int* __restrict__ sums, int64_t nb) {
  __shared__ int lds[256];
  int carry = 0;
  for (int64_t base = 0; base < nb; base += 256) {
    const int64_t e = base + threadIdx.x;
    const int x = e < nb ? sums[e] : 0;
    int total;
    const int ex = block_excl_scan(x, lds, &total);
    if (e < nb) sums[e] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(256) void scan_add_kernel(int* __restrict__ a, int64_t n, const int* __restrict__ sums) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    a[e] += sums[e / kScanTile];
}

// Stable scatter of one 8-bit digit pass.  Wave w of a tile takes entries
// [tile*4096 + w*1024, + 1024) in 16 steps of 64 consecutive entries; an
// entry's rank among the equal digits before it is counted with ballots, so
// the order within a digit is the input order.  perm_in == nullptr: the
// payload is the entry's own position.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(const int32_t* __restrict__ keys_in,
                                                                     const int32_t* __restrict__ perm_in, int64_t n,
                                                                     int shift, const int* __restrict__ offs,
                                                                     int64_t ntiles, int32_t* __restrict__ keys_out,
                                                                     int32_t* __restrict__ perm_out) {
  __shared__ int cnt[4][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) cnt[q][t] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * (kSortTile / 4);
  int32_t kk[kSortItems], pp[kSortItems];
  int rk[kSortItems];
#pragma unroll
  for (int s = 0; s < kSortItems; ++s) {
    const int64_t e = base + (int64_t)s * 64 + lane;
    const bool valid = e < n;
    kk[s] = valid ? keys_in[e] : 0;
    pp[s] = valid ? (perm_in ? perm_in[e] : (int32_t)e) : 0;
    const uint32_t d = ((uint32_t)kk[s] >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    // All lanes read the running count before the group's leader adds to it.
    const int before = cnt[w][d];
    rk[s] = before + __popcll(m & lt);
    __builtin_amdgcn_wave_barrier();
    if (valid && lane == __ffsll((unsigned long long)m) - 1) cnt[w][d] = before + __popcll(m);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    int run = offs[(int64_t)t * ntiles + blockIdx.x];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = cnt[q][t];
      cnt[q][t] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kSortItems; ++s) {
    const int64_t e = base + (int64_t)s * 64 + lane;
    if (e < n) {
      const int pos = cnt[w][((uint32_t)kk[s] >> shift) & 255u] + rk[s];
      keys_out[pos] = kk[s];
      perm_out[pos] = pp[s];
    }
  }
}

// Sorted entries of one mode: ent[p] = {idx_n, idx_a, idx_b, value} of input
// entry perm[p] (p itself when perm is null).
__global__ __launch_bounds__(256) void coo_gather_kernel(const int32_t* __restrict__ perm, const int32_t* __restrict__ in,
                                                         const int32_t* __restrict__ ia,
                                                         const int32_t* __restrict__ ib, const float* __restrict__ v,
                                                         int64_t nnz, int4* __restrict__ ent) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = perm ? perm[p] : p;
    ent[p] = make_int4(in[o], ia[o], ib[o], __float_as_int(v[o]));
  }
}


// Part of each entry for a partitioned mode: which of `parts` equal ranges
// of the first gathered factor's rows its index a falls in.
__global__ __launch_bounds__(256) void coo_part_key_kernel(const int32_t* __restrict__ perm,
                                                           const int32_t* __restrict__ ia, int64_t da, int parts,
                                                           int64_t nnz, int32_t* __restrict__ key) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = perm ? perm[p] : p;
    key[p] = (int32_t)((int64_t)ia[o] * parts / da);
  }
}

// Entries per part if the parts are the equal index ranges of ia
// (integer counts: order does not matter).
__global__ __launch_bounds__(256) void coo_part_count_kernel(const int32_t* __restrict__ ia, int64_t da, int parts,
                                                             int64_t nnz, int* __restrict__ cnt) {
  __shared__ int c[kCooParts];
  if (threadIdx.x < kCooParts) c[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&c[(int64_t)ia[p] * parts / da], 1);
  __syncthreads();
  if (threadIdx.x < kCooParts && c[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], c[threadIdx.x]);
}

// ----------------------------------------------------------- contraction ---

template <int RL, int T>
__device__ __forceinline__ void store_row(float* __restrict__ dst, const float (&acc)[T], int R, int c0) {
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int c = c0 + t * RL;
    if (c < R) dst[c] = acc[t];
  }
}

constexpr int kCooUnroll = 4;

// Segments of one mode: part p holds entries [ent[p], ent[p+1]) and
// segments [seg[p], seg[p+1]) of the global segment numbering (carry slots).
struct CooSegs {
  int64_t ent[kCooParts + 1];
  int64_t seg[kCooParts + 1];
  int parts;
  int64_t nrows;
};

// Output row `row` of part p goes to row p * nrows + row of the partial
// outputs (the output itself with one part); carry slots hold that key.
template <int RL, int T>
__global__ __launch_bounds__(256) void coo_mttkrp_kernel(const int4* __restrict__ ent, CooSegs sg, int L,
                                                         const float* __restrict__ fa, const float* __restrict__ fb,
                                                         int R, float* __restrict__ out, float* __restrict__ cval,
                                                         int64_t* __restrict__ crow) {
  constexpr int G = kWave / RL;
  __shared__ int4 stage[4][kWave];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / RL, c0 = lane % RL;
  // Workgroups are handed to the XCDs in turn, so workgroup b runs on XCD
  // b mod 8: part p is walked by XCD p, whose L2 then holds that part's
  // share of the gathered factor.
  const int part = sg.parts > 1 ? (int)(blockIdx.x % (unsigned)sg.parts) : 0;
  const int64_t lb = sg.parts > 1 ? blockIdx.x / (unsigned)sg.parts : blockIdx.x;
  const int64_t ls = (lb * 4 + w) * G + g;
  if (ls >= sg.seg[part + 1] - sg.seg[part]) return;
  const int64_t seg = sg.seg[part] + ls;
  const int64_t e0 = sg.ent[part] + ls * L, e1 = min(e0 + (int64_t)L, sg.ent[part + 1]);
  const int64_t kbase = (int64_t)part * sg.nrows;
  int4* my = stage[w] + g * RL;
  float acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = 0.0f;
  int64_t cur = ent[e0].x;
  bool first = true;
  for (int64_t cb = e0; cb < e1; cb += RL) {
    const int64_t e = cb + c0;
    my[c0] = e < e1 ? ent[e] : make_int4(-1, 0, 0, 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int n = (int)min((int64_t)RL, e1 - cb);
    for (int i = 0; i < n; i += kCooUnroll) {
      int4 q[kCooUnroll];
      float pa[kCooUnroll][T], pb[kCooUnroll][T];
#pragma unroll
      for (int u = 0; u < kCooUnroll; ++u) {
        q[u] = my[min(i + u, RL - 1)];
        if (i + u >= n) q[u].x = -1;
      }
#pragma unroll
      for (int u = 0; u < kCooUnroll; ++u)
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int c = c0 + t * RL;
          const bool ok = q[u].x >= 0 && c < R;
          pa[u][t] = ok ? fa[(int64_t)q[u].y * R + c] : 0.0f;
          pb[u][t] = ok ? fb[(int64_t)q[u].z * R + c] : 0.0f;
        }
#pragma unroll
      for (int u = 0; u < kCooUnroll; ++u) {
        if (q[u].x < 0) break;
        if (q[u].x != cur) {
          if (first) {
            store_row<RL, T>(cval + (2 * seg) * R, acc, R, c0);
            if (c0 == 0) crow[2 * seg] = kbase + cur;
          } else {
            store_row<RL, T>(out + (kbase + cur) * R, acc, R, c0);
          }
          first = false;
          cur = q[u].x;
#pragma unroll
          for (int t = 0; t < T; ++t) acc[t] = 0.0f;
        }
        const float v = __int_as_float(q[u].w);
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] += v * pa[u][t] * pb[u][t];
      }
    }
    // The next chunk overwrites this group's slots only after every lane has read them.
    __builtin_amdgcn_wave_barrier();
  }
  if (first) {
    store_row<RL, T>(cval + (2 * seg) * R, acc, R, c0);
    if (c0 == 0) {
      crow[2 * seg] = kbase + cur;
      crow[2 * seg + 1] = -1;
    }
  } else {
    store_row<RL, T>(cval + (2 * seg + 1) * R, acc, R, c0);
    if (c0 == 0) crow[2 * seg + 1] = kbase + cur;
  }
}

// One level of the carry reduction.  The slots (key, R values; key -1 =
// empty) are cut into groups of kCarryGroup consecutive slots, each walked
// by RL lanes like a segment of entries: a key that starts and ends inside
// the group is written to out, the group's first and last keys go to two
// slots of the next level.  With a single group (final) every key is
// written.  Each level keeps the slot order, so a row's partial sums are
// added in segment order along a tree fixed by nnz.
constexpr int kCarryGroup = 32;

template <int RL, int T>
__global__ __launch_bounds__(256) void coo_carry_kernel(const float* __restrict__ cin, const int64_t* __restrict__ rin,
                                                        int64_t nin, int final_, int R, float* __restrict__ out,
                                                        float* __restrict__ cout, int64_t* __restrict__ rout) {
  constexpr int G = kWave / RL;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c0 = lane % RL;
  const int64_t gi = ((int64_t)blockIdx.x * 4 + w) * G + lane / RL;
  const int64_t s0 = gi * kCarryGroup;
  if (s0 >= nin) return;
  const int64_t s1 = min(s0 + (int64_t)kCarryGroup, nin);
  float acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = 0.0f;
  int64_t cur = -1;
  bool first = true;
  for (int64_t k = s0; k < s1; ++k) {
    const int64_t r = rin[k];
    if (r < 0) continue;
    float v[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int c = c0 + t * RL;
      v[t] = c < R ? cin[k * R + c] : 0.0f;
    }
    if (cur >= 0 && r != cur) {
      if (first && !final_) {
        store_row<RL, T>(cout + (2 * gi) * R, acc, R, c0);
        if (c0 == 0) rout[2 * gi] = cur;
      } else {
        store_row<RL, T>(out + cur * R, acc, R, c0);
      }
      first = false;
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = 0.0f;
    }
    cur = r;
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] += v[t];
  }
  if (final_) {
    store_row<RL, T>(out + cur * R, acc, R, c0);
  } else if (first) {
    store_row<RL, T>(cout + (2 * gi) * R, acc, R, c0);
    if (c0 == 0) {
      rout[2 * gi] = cur;
      rout[2 * gi + 1] = -1;
    }
  } else {
    store_row<RL, T>(cout + (2 * gi + 1) * R, acc, R, c0);
    if (c0 == 0) rout[2 * gi + 1] = cur;
  }
}

// out[e] = sum over parts p, in order, of part[p * n + e].
__global__ __launch_bounds__(256) void coo_part_sum_kernel(const float* __restrict__ part, int parts, int64_t n,
                                                           float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    float s = part[e];
    for (int p = 1; p < parts; ++p) s += part[p * n + e];
    out[e] = s;
  }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(float* __restrict__ out, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = 0.0f;
}

int64_t grid_of(int64_t items, int per_block, int64_t cap = (int64_t)1 << 20) {
  return std::max<int64_t>(1, std::min<int64_t>(cap, (items + per_block - 1) / per_block));
}

}  // namespace

// Entries per segment: a multiple of 64 set by nnz only, so that the
// partition (and with it the order of every sum) is the same for every R.
int coo_segment_len(int64_t nnz) {
  const int64_t want = (nnz + 32767) / 32768;
  return (int)std::min<int64_t>(kCooMaxSeg, std::max<int64_t>(64, (want + 63) / 64 * 64));
}

// A mode may be partitioned when the partial outputs (one per part, each
// zeroed, written and read: 3 x 8 x rows x R floats) stay small next to the
// entries (16 bytes each): 8 x rows x 64 <= nnz.  A gathered factor
// qualifies when it is large enough to overflow an XCD's 4 MB L2 (8192 rows
// and more) but an eighth of it fits there at the usual ranks (at most
// 131072 rows: 2 MB per part at R = 32).
bool coo_may_partition(const int64_t dims[3], int64_t nnz, int mode) {
  return (int64_t)kCooParts * dims[mode] * 64 <= nnz;
}
constexpr int64_t kCooPartMinRows = 8192;
constexpr int64_t kCooPartMaxRows = 131072;

}  // namespace mtk

// ------------------------------------------------------------------ C ABI ---

struct mtk_coo {
  int device = 0;
  int64_t dims[3] = {0, 0, 0};
  int64_t nnz = 0;
  int seg_len = 64;
  mtk::CooSegs segs[3] = {};                    // per mode: parts, entry and segment ranges
  int64_t max_nseg = 0;                         // most segments of any mode
  int4* ent[3] = {nullptr, nullptr, nullptr};  // per mode, sorted by (part, that mode's index)
  float* cval = nullptr;                        // 2 * max_nseg carry slots of up to kMaxRank floats
  int64_t* crow = nullptr;                      // their keys (-1: empty)
  float* cval2 = nullptr;                       // the next level's slots (levels alternate)
  int64_t* crow2 = nullptr;
  void* block = nullptr;                        // the one allocation behind all of the above
  float* part = nullptr;                        // partial outputs of a partitioned mode (grown on demand)
  size_t part_bytes = 0;
};

namespace {

mtk_status coo_fail(mtk_ctx* c, mtk_status s, const std::string& msg) {
  c->last_error = msg;
  return s;
}

mtk_status coo_hip_fail(mtk_ctx* c, hipError_t e, const char* where) {
  return coo_fail(c, e == hipErrorOutOfMemory ? MTK_ENOMEM : MTK_EHIP,
                  std::string(where) + ": " + hipGetErrorString(e));
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

int digit_passes(int64_t d) {
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < d) ++bits;  // indices are < d <= 2^bits
  return (bits + 7) / 8;
}

}  // namespace

extern "C" {

mtk_status mtk_coo_create(mtk_ctx* c, const int64_t dims[3], int64_t nnz, const int32_t* const idx[3],
                          const float* vals, void* stream, mtk_coo** out) {
  using namespace mtk;
  if (!c) return MTK_EINVAL;
  if (!dims || !out) return coo_fail(c, MTK_EINVAL, "NULL argument");
  *out = nullptr;
  for (int m = 0; m < 3; ++m)
    if (dims[m] < 1 || dims[m] > 0x7fffffff) return coo_fail(c, MTK_EINVAL, "dims must be in [1, 2^31 - 1]");
  if (nnz < 0 || nnz > 0x7fffffff) return coo_fail(c, MTK_EINVAL, "nnz must be in [0, 2^31 - 1]");
  if (nnz > 0) {
    if (!idx || !idx[0] || !idx[1] || !idx[2] || !vals) return coo_fail(c, MTK_EINVAL, "NULL index or value array");
    for (int m = 0; m < 3; ++m)
      if (reinterpret_cast<uintptr_t>(idx[m]) & 3) return coo_fail(c, MTK_EINVAL, "index array not 4-byte aligned");
    if (reinterpret_cast<uintptr_t>(vals) & 3) return coo_fail(c, MTK_EINVAL, "value array not 4-byte aligned");
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return coo_hip_fail(c, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);

  mtk_coo* t = new mtk_coo;
  t->device = c->device;
  std::memcpy(t->dims, dims, sizeof(t->dims));
  t->nnz = nnz;
  t->seg_len = coo_segment_len(nnz);
  // Segment count bound: each part rounds its segments up once.
  t->max_nseg = (nnz + t->seg_len - 1) / t->seg_len + kCooParts;
  const size_t ent_b = up256((size_t)nnz * sizeof(int4));
  const int64_t nslot = 2 * t->max_nseg;
  const int64_t nslot2 = 2 * ((nslot + kCarryGroup - 1) / kCarryGroup);
  const size_t cval_b = up256((size_t)nslot * kMaxRank * sizeof(float));
  const size_t crow_b = up256((size_t)nslot * sizeof(int64_t));
  const size_t cval2_b = up256((size_t)nslot2 * kMaxRank * sizeof(float));
  const size_t crow2_b = up256((size_t)nslot2 * sizeof(int64_t));
  if ((e = hipMalloc(&t->block, 3 * ent_b + cval_b + crow_b + cval2_b + crow2_b + 256)) != hipSuccess) {
    delete t;
    return coo_hip_fail(c, e, "mtk_coo_create: allocation");
  }
  char* p = static_cast<char*>(t->block);
  for (int m = 0; m < 3; ++m, p += ent_b) t->ent[m] = reinterpret_cast<int4*>(p);
  t->cval = reinterpret_cast<float*>(p);
  t->crow = reinterpret_cast<int64_t*>(p + cval_b);
  t->cval2 = reinterpret_cast<float*>(p + cval_b + crow_b);
  t->crow2 = reinterpret_cast<int64_t*>(p + cval_b + crow_b + cval2_b);
  for (int m = 0; m < 3; ++m) {
    CooSegs& sg = t->segs[m];
    sg.parts = 1;
    sg.nrows = dims[m];
  }
  if (nnz == 0) {
    *out = t;
    return MTK_OK;
  }

  // Temporaries of the sort: ping-pong keys and payloads, digit histograms,
  // scan block sums, the range-check counter and the part counts.
  const int64_t ntiles = (nnz + kSortTile - 1) / kSortTile;
  const int64_t nhist = 256 * ntiles;
  const int64_t nsums = (nhist + kScanTile - 1) / kScanTile;
  const size_t kb = up256((size_t)nnz * 4);
  void* tmp = nullptr;
  if ((e = hipMalloc(&tmp, 5 * kb + up256(nhist * 4) + up256(nsums * 4) + 512)) != hipSuccess) {
    hipFree(t->block);
    delete t;
    return coo_hip_fail(c, e, "mtk_coo_create: sort temporaries");
  }
  char* q = static_cast<char*>(tmp);
  int32_t* kbuf[2] = {reinterpret_cast<int32_t*>(q), reinterpret_cast<int32_t*>(q + kb)};
  int32_t* pbuf[2] = {reinterpret_cast<int32_t*>(q + 2 * kb), reinterpret_cast<int32_t*>(q + 3 * kb)};
  int32_t* pkey = reinterpret_cast<int32_t*>(q + 4 * kb);
  int* hist = reinterpret_cast<int*>(q + 5 * kb);
  int* sums = reinterpret_cast<int*>(q + 5 * kb + up256(nhist * 4));
  int* bad = reinterpret_cast<int*>(q + 5 * kb + up256(nhist * 4) + up256(nsums * 4));
  int* pcnt = bad + 64;

  auto done = [&](mtk_status s) {
    hipStreamSynchronize(st);
    hipFree(tmp);
    if (s != MTK_OK) {
      hipFree(t->block);
      delete t;
    } else {
      *out = t;
    }
    return s;
  };
  int hbad = 0;
  fill_zero_kernel<<<1, 64, 0, st>>>(reinterpret_cast<float*>(bad), 1);
  coo_range_kernel<<<grid_of(nnz, 256, 4096), 256, 0, st>>>(idx[0], idx[1], idx[2], nnz, (int32_t)dims[0],
                                                             (int32_t)dims[1], (int32_t)dims[2], bad);
  if ((e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return done(coo_hip_fail(c, e, "mtk_coo_create: index check"));
  if (hbad != 0)
    return done(coo_fail(c, MTK_EINVAL, "mtk_coo_create: " + std::to_string(hbad) + " entries have an index outside dims"));

  auto radix_pass = [&](const int32_t* keys, const int32_t* perm, int shift, int32_t* ko, int32_t* po) {
    radix_hist_kernel<<<ntiles, kSortThreads, 0, st>>>(keys, nnz, shift, hist, ntiles);
    scan_tiles_kernel<<<nsums, 256, 0, st>>>(hist, nhist, sums);
    scan_sums_kernel<<<1, 256, 0, st>>>(sums, nsums);
    scan_add_kernel<<<grid_of(nhist, 256), 256, 0, st>>>(hist, nhist, sums);
    radix_scatter_kernel<<<ntiles, kSortThreads, 0, st>>>(keys, perm, nnz, shift, hist, ntiles, ko, po);
  };
  for (int m = 0; m < 3; ++m) {
    const int oa = m == 0 ? 1 : 0, ob = m == 2 ? 1 : 2;
    const int passes = digit_passes(dims[m]);
    const int32_t* keys = idx[m];
    const int32_t* perm = nullptr;
    int buf = 0;
    for (int ps = 0; ps < passes; ++ps, buf ^= 1) {
      radix_pass(keys, perm, 8 * ps, kbuf[buf], pbuf[buf]);
      keys = kbuf[buf];
      perm = pbuf[buf];
    }
    CooSegs& sg = t->segs[m];
    sg.parts = 1;
    int64_t cnt[kCooParts] = {nnz};
    if (coo_may_partition(dims, nnz, m)) {
      // Of the two gathered factors, partition by the one whose index ranges
      // spread the entries most evenly over the parts (a skewed index would
      // leave one XCD most of the work); none if even that one is lopsided.
      int best = -1;
      int64_t best_max = 0;
      int64_t best_cnt[kCooParts] = {};
      for (int cand : {oa, ob}) {
        if (dims[cand] < kCooPartMinRows || dims[cand] > kCooPartMaxRows) continue;
        int hc[kCooParts] = {};
        fill_zero_kernel<<<1, 64, 0, st>>>(reinterpret_cast<float*>(pcnt), kCooParts);
        coo_part_count_kernel<<<grid_of(nnz, 256, 1024), 256, 0, st>>>(idx[cand], dims[cand], kCooParts, nnz, pcnt);
        if ((e = hipMemcpyAsync(hc, pcnt, sizeof(hc), hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
          return done(coo_hip_fail(c, e, "mtk_coo_create: part counts"));
        const int64_t mx = *std::max_element(hc, hc + kCooParts);
        if (best < 0 || mx < best_max) {
          best = cand;
          best_max = mx;
          for (int pp = 0; pp < kCooParts; ++pp) best_cnt[pp] = hc[pp];
        }
      }
      if (best >= 0 && best_max * 4 * kCooParts <= 5 * nnz) {
        // One more stable pass orders the entries by part, rows ascending within each.
        sg.parts = kCooParts;
        coo_part_key_kernel<<<grid_of(nnz, 256), 256, 0, st>>>(perm, idx[best], dims[best], sg.parts, nnz, pkey);
        radix_pass(pkey, perm, 0, kbuf[buf], pbuf[buf]);
        perm = pbuf[buf];
        for (int pp = 0; pp < kCooParts; ++pp) cnt[pp] = best_cnt[pp];
      }
    }
    sg.ent[0] = 0;
    sg.seg[0] = 0;
    for (int pp = 0; pp < kCooParts; ++pp) {
      const int64_t n = pp < sg.parts ? cnt[pp] : 0;
      sg.ent[pp + 1] = sg.ent[pp] + n;
      sg.seg[pp + 1] = sg.seg[pp] + (n + t->seg_len - 1) / t->seg_len;
    }
    coo_gather_kernel<<<grid_of(nnz, 256), 256, 0, st>>>(perm, idx[m], idx[oa], idx[ob], vals, nnz, t->ent[m]);
  }
  if ((e = hipGetLastError()) != hipSuccess) return done(coo_hip_fail(c, e, "mtk_coo_create: sort launch"));
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return done(coo_hip_fail(c, e, "mtk_coo_create: sort"));
  return done(MTK_OK);
}

mtk_status mtk_coo_destroy(mtk_coo* t) {
  if (!t) return MTK_OK;
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(t->device);
  hipFree(t->block);
  if (t->part) hipFree(t->part);
  hipSetDevice(prev);
  delete t;
  return MTK_OK;
}

int64_t mtk_coo_nnz(const mtk_coo* t) { return t ? t->nnz : -1; }

mtk_status mttkrp_coo(mtk_ctx* c, const mtk_coo* tc, const float* const factors[3], int64_t R, int mode, float* out,
                      void* stream) {
  using namespace mtk;
  if (!c) return MTK_EINVAL;
  if (!tc || !factors || !out) return coo_fail(c, MTK_EINVAL, "NULL argument");
  mtk_coo* t = const_cast<mtk_coo*>(tc);   // the partial-output buffer is grown on demand
  if (t->device != c->device) return coo_fail(c, MTK_EINVAL, "tensor and context are on different devices");
  if (mode < 0 || mode > 2) return coo_fail(c, MTK_EINVAL, "mode must be 0, 1 or 2");
  if (R < 1 || R > kMaxRank) return coo_fail(c, MTK_EINVAL, "R must be in [1, 128]");
  const int oa = mode == 0 ? 1 : 0, ob = mode == 2 ? 1 : 2;
  if (!factors[oa] || !factors[ob]) return coo_fail(c, MTK_EINVAL, "NULL factor pointer");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return coo_hip_fail(c, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nrows = t->dims[mode];
  const CooSegs& sg = t->segs[mode];
  const bool parts = t->nnz > 0 && sg.parts > 1;
  float* base = out;
  if (parts) {
    const size_t need = (size_t)sg.parts * nrows * R * sizeof(float);
    if (need > t->part_bytes) {
      if (t->part) {
        hipFree(t->part);          // waits for the work that used it
        t->part = nullptr;
        t->part_bytes = 0;
      }
      if ((e = hipMalloc(&t->part, need)) != hipSuccess) return coo_hip_fail(c, e, "mttkrp_coo: partial outputs");
      t->part_bytes = need;
    }
    base = t->part;
  }
  const int64_t nbase = (parts ? sg.parts : 1) * nrows * R;
  fill_zero_kernel<<<grid_of(nbase, 256, 4096), 256, 0, st>>>(base, nbase);
  if (t->nnz > 0) {
    const int r = (int)R;
    const int4* ent = t->ent[mode];
    const float* fa = factors[oa];
    const float* fb = factors[ob];
    const int64_t nslot = 2 * sg.seg[kCooParts];
    int64_t most = 0;
    for (int pp = 0; pp < sg.parts; ++pp) most = std::max<int64_t>(most, sg.seg[pp + 1] - sg.seg[pp]);
#define MTK_COO_LAUNCH(RL, T)                                                                           \
  do {                                                                                                  \
    const int64_t gpb = 4 * (kWave / RL);                                                               \
    coo_mttkrp_kernel<RL, T><<<sg.parts * ((most + gpb - 1) / gpb), 256, 0, st>>>(ent, sg, t->seg_len, fa, \
                                                                                  fb, r, base, t->cval, t->crow); \
    float* cv[2] = {t->cval, t->cval2};                                                                 \
    int64_t* cr[2] = {t->crow, t->crow2};                                                               \
    int64_t nin = nslot;                                                                                \
    for (int lv = 0;; ++lv) {                                                                           \
      const int64_t groups = (nin + kCarryGroup - 1) / kCarryGroup;                                     \
      const int fin = groups == 1;                                                                      \
      coo_carry_kernel<RL, T><<<(groups + gpb - 1) / gpb, 256, 0, st>>>(                                \
          cv[lv & 1], cr[lv & 1], nin, fin, r, base, cv[(lv + 1) & 1], cr[(lv + 1) & 1]);               \
      if (fin) break;                                                                                   \
      nin = 2 * groups;                                                                                 \
    }                                                                                                   \
  } while (0)
    if (r <= 8)
      MTK_COO_LAUNCH(8, 1);
    else if (r <= 16)
      MTK_COO_LAUNCH(16, 1);
    else if (r <= 32)
      MTK_COO_LAUNCH(32, 1);
    else if (r <= 64)
      MTK_COO_LAUNCH(64, 1);
    else
      MTK_COO_LAUNCH(64, 2);
#undef MTK_COO_LAUNCH
    if (parts) coo_part_sum_kernel<<<grid_of(nrows * R, 256, 4096), 256, 0, st>>>(base, sg.parts, nrows * R, out);
  }
  if ((e = hipGetLastError()) != hipSuccess) return coo_hip_fail(c, e, "mttkrp_coo launch");
  return MTK_OK;
}

mtk_status als_sweep_coo(mtk_ctx* c, const mtk_coo* t, float* const factors[3], double* lambda, int64_t R,
                         int nsweeps, void* stream) {
  if (!c) return MTK_EINVAL;
  if (!t || !factors || !factors[0] || !factors[1] || !factors[2] || !lambda)
    return coo_fail(c, MTK_EINVAL, "NULL argument");
  if (nsweeps < 0) return coo_fail(c, MTK_EINVAL, "nsweeps must be >= 0");
  if (R < 1 || R > mtk::kMaxRank) return coo_fail(c, MTK_EINVAL, "R must be in [1, 128]");
  for (int m = 0; m < 3; ++m)
    if (t->dims[m] > (1 << 30)) return coo_fail(c, MTK_EUNSUPPORTED, "als_sweep_coo: a dimension exceeds 2^30");
  const float* const cf[3] = {factors[0], factors[1], factors[2]};
  for (int s = 0; s < nsweeps; ++s)
    for (int mode = 0; mode < 3; ++mode) {
      // The mode's MTTKRP goes straight into its factor (which it does not
      // read), and the update overwrites it in place.
      mtk_status st = mttkrp_coo(c, t, cf, R, mode, factors[mode], stream);
      if (st == MTK_OK) st = gram_solve(c, cf, t->dims, R, mode, factors[mode], factors[mode], lambda, stream);
      if (st != MTK_OK) return st;
    }
  return mtk_check(c, stream);
}

}  // extern "C"
