// Continuous-batching server for CP-ALS decompositions (C ABI: mtk_server_*).
//
// A worker thread owns the device side.  Requests are admitted in arrival
// order when (a) a slot is free and (b) the request's device bytes fit in
// the HBM budget next to the resident requests.  Admission carves the
// request's buffers out of a device arena, queues its upload, all of its
// ALS sweeps, the final fit and the download on the slot's own stream, and
// records an event.  Resident requests therefore run concurrently on the
// device; the worker polls the events, retires finished requests (freeing
// their memory and slot) and admits more.  Each request runs exactly the
// kernels and summation orders of a lone als_sweep call on the same shape,
// so its result does not depend on what runs beside it.

#include "mtk_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit sub-allocator over a growing list of chunks (device or pinned
// host memory).  Free blocks are coalesced with their neighbours.
class Arena {
 public:
  using AllocFn = void* (*)(size_t);
  using FreeFn = void (*)(void*);
  Arena(AllocFn a, FreeFn f, size_t chunk) : alloc_(a), free_(f), chunk_(chunk) {}
  ~Arena() {
    for (auto& c : chunks_) free_(c.base);
  }
  void* alloc(size_t bytes) {
    bytes = r256(std::max<size_t>(bytes, 256));
    for (auto& c : chunks_)
      if (void* p = take(c, bytes)) return p;
    const size_t sz = std::max(chunk_, bytes);
    void* base = alloc_(sz);
    if (!base) return nullptr;
    chunks_.push_back(Chunk{static_cast<char*>(base), sz, {{0, sz}}});
    return take(chunks_.back(), bytes);
  }
  void release(void* p) {
    char* q = static_cast<char*>(p);
    for (auto& c : chunks_) {
      if (q < c.base || q >= c.base + c.size) continue;
      auto it = c.used.find((size_t)(q - c.base));
      if (it == c.used.end()) return;
      size_t off = it->first, len = it->second;
      c.used.erase(it);
      // insert into free map and coalesce
      auto nx = c.free.lower_bound(off);
      if (nx != c.free.end() && off + len == nx->first) { len += nx->second; nx = c.free.erase(nx); }
      if (nx != c.free.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) { pv->second += len; return; }
      }
      c.free[off] = len;
      return;
    }
  }

 private:
  struct Chunk {
    char* base;
    size_t size;
    std::map<size_t, size_t> free;   // offset -> length
    std::map<size_t, size_t> used;
  };
  void* take(Chunk& c, size_t bytes) {
    for (auto it = c.free.begin(); it != c.free.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      c.free.erase(it);
      if (len > bytes) c.free[off + bytes] = len - bytes;
      c.used[off] = bytes;
      return c.base + off;
    }
    return nullptr;
  }
  AllocFn alloc_;
  FreeFn free_;
  size_t chunk_;
  std::vector<Chunk> chunks_;
};

void* dev_alloc(size_t b) {
  void* p = nullptr;
  if (hipMalloc(&p, b) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  return p;
}
void dev_free(void* p) { (void)hipFree(p); }
void* host_alloc(size_t b) {
  void* p = nullptr;
  if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  return p;
}
void host_free(void* p) { (void)hipHostFree(p); }

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Req {
  int64_t id = 0;
  int64_t dims[3] = {0, 0, 0};
  int R = 0, prec = 0, sweeps = 0;
  size_t dev_bytes = 0;
  char* hbuf = nullptr;            // pinned: X, init factors, then results
  float* out_f[3] = {nullptr, nullptr, nullptr};
  double* out_lambda = nullptr;
  mtk_result res{};
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  int* d_status = nullptr;
  double* d_fit = nullptr;
  char* dbuf = nullptr;            // arena block of the resident request
  std::unique_ptr<Req> req;
};

size_t elem_count(const int64_t d[3]) { return (size_t)d[0] * d[1] * d[2]; }

size_t host_bytes(const Req& r) {
  size_t b = r256(elem_count(r.dims) * sizeof(float));
  for (int m = 0; m < 3; ++m) b += r256((size_t)r.dims[m] * r.R * sizeof(float));
  b += r256((size_t)r.R * sizeof(double)) + r256(2 * sizeof(double)) + 256;
  return b;
}

// Contraction / fit scratch of a request, rounded to 256 bytes.
size_t contract_region_bytes(const int64_t dims[3], int R, int prec) {
  size_t b = 0;
  for (int m = 0; m < 3; ++m) {
    mtk::ContractPlan p = mtk::make_plan(dims, R, m, prec, true);
    b = std::max(b, mtk::contract_ws_bytes(p, prec));
  }
  b = std::max(b, mtk::fit_ws_bytes(dims));
  return r256(b);
}

// The solve region (which keeps the Gram matrices across the MTTKRPs)
// follows the contraction region, then the dimension-tree region when the
// sweep uses one.
size_t scratch_bytes(const int64_t dims[3], int R, int prec) {
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  const size_t dt = mtk::dimtree_used(dims, R, prec) ? mtk::dimtree_ws_bytes(dims, R) : 0;
  return contract_region_bytes(dims, R, prec) + mtk::solve_ws_bytes(maxdim, R) + dt;
}

size_t device_bytes(const int64_t dims[3], int R, int prec) {
  const int64_t maxdim = std::max(dims[0], std::max(dims[1], dims[2]));
  size_t b = r256(elem_count(dims) * sizeof(float));
  for (int m = 0; m < 3; ++m) b += r256((size_t)dims[m] * R * sizeof(float));
  b += r256((size_t)R * sizeof(double));
  b += r256((size_t)maxdim * R * sizeof(float));
  b += scratch_bytes(dims, R, prec);
  return b + 256;
}

}  // namespace

struct mtk_server {
  int device = 0;
  uint64_t budget = 0;
  int max_slots = 1;
  std::chrono::steady_clock::time_point t0;
  std::unique_ptr<Arena> darena, harena;
  std::vector<Slot> slots;
  std::mutex mu;                   // guards pending, finished, harena, counters
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Req>> pending;
  std::deque<mtk_result> finished;
  std::atomic<bool> stop{false};
  uint64_t in_use = 0, peak = 0;
  int resident = 0;
  int64_t outstanding = 0;         // submitted and not yet finished
  std::thread worker;
  std::string err;

  // Queue the whole decomposition of `r` on slot `s` (device buffers in s.dbuf).
  hipError_t launch(Slot& s) {
    Req& r = *s.req;
    const int R = r.R;
    const size_t nx = elem_count(r.dims);
    char* d = s.dbuf;
    char* h = r.hbuf;
    float* X = reinterpret_cast<float*>(d); d += r256(nx * sizeof(float));
    const float* hx = reinterpret_cast<const float*>(h); h += r256(nx * sizeof(float));
    float* f[3];
    float* hf[3];
    for (int m = 0; m < 3; ++m) {
      f[m] = reinterpret_cast<float*>(d);
      hf[m] = reinterpret_cast<float*>(h);
      d += r256((size_t)r.dims[m] * R * sizeof(float));
      h += r256((size_t)r.dims[m] * R * sizeof(float));
    }
    double* lam = reinterpret_cast<double*>(d); d += r256((size_t)R * sizeof(double));
    double* hlam = reinterpret_cast<double*>(h); h += r256((size_t)R * sizeof(double));
    double* hfit = reinterpret_cast<double*>(h);
    const int64_t maxdim = std::max(r.dims[0], std::max(r.dims[1], r.dims[2]));
    float* M = reinterpret_cast<float*>(d); d += r256((size_t)maxdim * R * sizeof(float));
    void* scratch = d;

    hipError_t e;
    if ((e = hipMemsetAsync(s.d_status, 0, sizeof(int), s.st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(X, hx, nx * sizeof(float), hipMemcpyHostToDevice, s.st)) != hipSuccess) return e;
    for (int m = 0; m < 3; ++m)
      if ((e = hipMemcpyAsync(f[m], hf[m], (size_t)r.dims[m] * R * sizeof(float), hipMemcpyHostToDevice, s.st)) !=
          hipSuccess)
        return e;
    const float* cf[3] = {f[0], f[1], f[2]};
    void* solve_ws = static_cast<char*>(scratch) + contract_region_bytes(r.dims, R, r.prec);
    if (r.sweeps > 0 && (e = mtk::launch_grams(cf, r.dims, R, 1, 2, maxdim, solve_ws, s.d_status, s.st)) != hipSuccess)
      return e;
    // The same kernels in the same order as a lone als_sweep of this request.
    void* dt_ws = mtk::dimtree_used(r.dims, R, r.prec)
                      ? static_cast<char*>(solve_ws) + mtk::solve_ws_bytes(maxdim, R)
                      : nullptr;
    for (int sw = 0; sw < r.sweeps; ++sw) {
      for (int n = 0; n < 3; ++n) {
        const mtk::FactorArgs job = mtk::factor_args(r.dims, R, n, maxdim, solve_ws, s.d_status);
        const mtk::FactorArgs* jp = R <= mtk::kJobMaxRank ? &job : nullptr;
        mtk::MSlices ms{M, 1, 0};
        if (dt_ws && n < 2) {
          e = mtk::launch_dimtree_mttkrp(n, n == 0, X, true, r.dims, cf, R, r.prec, M, dt_ws, s.st, jp, &ms);
        } else {
          const float* fr = n == 2 ? f[1] : f[2];
          const float* wt = n == 0 ? f[1] : f[0];
          mtk::ContractPlan p = mtk::make_plan(r.dims, R, n, r.prec, true);
          e = mtk::launch_contract(p, r.prec, n, X, nullptr, fr, wt, M, scratch, s.st, jp);
        }
        if (e != hipSuccess) return e;
        e = jp ? mtk::launch_apply(r.dims, R, n, ms, f[n], lam, maxdim, solve_ws, s.d_status, s.st)
               : mtk::launch_update(r.dims, R, n, ms, f[n], lam, maxdim, solve_ws, s.d_status, s.st);
        if (e != hipSuccess) return e;
      }
    }
    if ((e = mtk::launch_fit(X, MTK_FP32, nullptr, r.dims, cf, lam, R, s.d_fit, scratch, s.st)) != hipSuccess)
      return e;
    for (int m = 0; m < 3; ++m)
      if ((e = hipMemcpyAsync(hf[m], f[m], (size_t)r.dims[m] * R * sizeof(float), hipMemcpyDeviceToHost, s.st)) !=
          hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(hlam, lam, (size_t)R * sizeof(double), hipMemcpyDeviceToHost, s.st)) != hipSuccess)
      return e;
    if ((e = hipMemcpyAsync(hfit, s.d_fit, 2 * sizeof(double), hipMemcpyDeviceToHost, s.st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(reinterpret_cast<char*>(hfit) + 2 * sizeof(double), s.d_status, sizeof(int),
                            hipMemcpyDeviceToHost, s.st)) != hipSuccess)
      return e;
    return hipEventRecord(s.done, s.st);
  }

  void retire(Slot& s) {
    Req& r = *s.req;
    const int R = r.R;
    const size_t nx = elem_count(r.dims);
    const char* h = r.hbuf + r256(nx * sizeof(float));
    for (int m = 0; m < 3; ++m) {
      const size_t b = (size_t)r.dims[m] * R * sizeof(float);
      if (r.out_f[m]) std::memcpy(r.out_f[m], h, b);
      h += r256(b);
    }
    if (r.out_lambda) std::memcpy(r.out_lambda, h, (size_t)R * sizeof(double));
    h += r256((size_t)R * sizeof(double));
    const double* fit = reinterpret_cast<const double*>(h);
    int st = 0;
    std::memcpy(&st, h + 2 * sizeof(double), sizeof(int));
    r.res.fit = 1.0 - std::sqrt(fit[0]) / std::sqrt(fit[1]);
    if (st & mtk::kStatusNotSPD) r.res.status = MTK_ENOTSPD;
    r.res.t_done = now_s(t0);
    darena->release(s.dbuf);
    s.dbuf = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    harena->release(r.hbuf);
    in_use -= r.dev_bytes;
    --resident;
    --outstanding;
    finished.push_back(r.res);
    s.req.reset();
    cv_done.notify_all();
  }

  void run() {
    (void)hipSetDevice(device);
    while (true) {
      bool did = false;
      // Retire finished requests.
      for (auto& s : slots) {
        if (!s.req) continue;
        if (hipEventQuery(s.done) == hipSuccess) { retire(s); did = true; }
      }
      // Admit in arrival order while a slot and the budget allow.
      while (true) {
        std::unique_ptr<Req> r;
        {
          std::lock_guard<std::mutex> lk(mu);
          if (pending.empty()) break;
          Req& head = *pending.front();
          if (resident >= max_slots || in_use + head.dev_bytes > budget) break;
          r = std::move(pending.front());
          pending.pop_front();
          in_use += r->dev_bytes;
          peak = std::max(peak, in_use);
          ++resident;
        }
        Slot* s = nullptr;
        for (auto& q : slots)
          if (!q.req) { s = &q; break; }
        s->dbuf = static_cast<char*>(darena->alloc(r->dev_bytes));
        r->res.t_admit = now_s(t0);
        s->req = std::move(r);
        hipError_t e = s->dbuf ? launch(*s) : hipErrorOutOfMemory;
        if (e != hipSuccess) {
          // Could not run: report and release everything of this request.
          (void)hipStreamSynchronize(s->st);
          s->req->res.status = s->dbuf ? MTK_EHIP : MTK_ENOMEM;
          s->req->res.t_done = now_s(t0);
          if (s->dbuf) darena->release(s->dbuf);
          s->dbuf = nullptr;
          std::lock_guard<std::mutex> lk(mu);
          harena->release(s->req->hbuf);
          in_use -= s->req->dev_bytes;
          --resident;
          --outstanding;
          finished.push_back(s->req->res);
          s->req.reset();
          cv_done.notify_all();
        }
        did = true;
      }
      if (did) continue;
      std::unique_lock<std::mutex> lk(mu);
      if (stop && pending.empty() && resident == 0) break;
      cv_work.wait_for(lk, std::chrono::microseconds(resident > 0 ? 50 : 2000));
    }
  }
};

extern "C" {

mtk_status mtk_server_create(mtk_server** out, int device, uint64_t budget_bytes, int max_slots) {
  if (!out || max_slots < 1 || budget_bytes == 0) return MTK_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MTK_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return MTK_EHIP;
  auto* s = new (std::nothrow) mtk_server();
  if (!s) return MTK_ENOMEM;
  s->device = device;
  s->budget = budget_bytes;
  s->max_slots = max_slots;
  s->t0 = std::chrono::steady_clock::now();
  s->darena.reset(new Arena(dev_alloc, dev_free, (size_t)1 << 30));
  s->harena.reset(new Arena(host_alloc, host_free, (size_t)1 << 30));
  s->slots.resize(max_slots);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&sl.d_status, mtk::kStatusWords * sizeof(int)) != hipSuccess ||
        hipMemset(sl.d_status, 0, mtk::kStatusWords * sizeof(int)) != hipSuccess ||
        hipMalloc(&sl.d_fit, 256) != hipSuccess) {
      mtk_server_destroy(s);
      return MTK_EHIP;
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return MTK_OK;
}

mtk_status mtk_server_submit(mtk_server* s, int64_t id, const float* x, const int64_t dims[3], int64_t R, int prec,
                             int sweeps, const float* const init[3], float* const factors_out[3],
                             double* lambda_out) {
  if (!s || !x || !dims || !init || !init[0] || !init[1] || !init[2]) return MTK_EINVAL;
  if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || R < 1 || R > mtk::kMaxRank || sweeps < 0) return MTK_EINVAL;
  if (prec != MTK_FP32 && prec != MTK_BF16X3) return MTK_EINVAL;
  auto r = std::make_unique<Req>();
  r->id = id;
  for (int m = 0; m < 3; ++m) r->dims[m] = dims[m];
  r->R = (int)R;
  r->prec = prec;
  r->sweeps = sweeps;
  r->dev_bytes = device_bytes(dims, (int)R, prec);
  if (r->dev_bytes > s->budget) return MTK_EBUDGET;
  for (int m = 0; m < 3; ++m) r->out_f[m] = factors_out ? factors_out[m] : nullptr;
  r->out_lambda = lambda_out;
  r->res.id = id;
  r->res.status = MTK_OK;
  r->res.R = (int)R;
  for (int m = 0; m < 3; ++m) r->res.dims[m] = dims[m];
  r->res.t_submit = now_s(s->t0);
  const size_t hb = host_bytes(*r);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->hbuf = static_cast<char*>(s->harena->alloc(hb));
  }
  if (!r->hbuf) return MTK_ENOMEM;
  const size_t nx = elem_count(dims);
  std::memcpy(r->hbuf, x, nx * sizeof(float));
  char* h = r->hbuf + r256(nx * sizeof(float));
  for (int m = 0; m < 3; ++m) {
    const size_t b = (size_t)dims[m] * R * sizeof(float);
    std::memcpy(h, init[m], b);
    h += r256(b);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->outstanding;
    s->pending.push_back(std::move(r));
  }
  s->cv_work.notify_one();
  return MTK_OK;
}

mtk_status mtk_server_poll(mtk_server* s, mtk_result* out, int cap, int* n, double timeout_s) {
  if (!s || !n || (cap > 0 && !out)) return MTK_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->finished.empty() && timeout_s > 0)
    s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [s] { return !s->finished.empty(); });
  int k = 0;
  while (k < cap && !s->finished.empty()) {
    out[k++] = s->finished.front();
    s->finished.pop_front();
  }
  *n = k;
  return k > 0 ? MTK_OK : MTK_EAGAIN;
}

mtk_status mtk_server_stats(mtk_server* s, int* resident, uint64_t* bytes_in_use, uint64_t* peak_bytes) {
  if (!s) return MTK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (resident) *resident = s->resident;
  if (bytes_in_use) *bytes_in_use = s->in_use;
  if (peak_bytes) *peak_bytes = s->peak;
  return MTK_OK;
}

mtk_status mtk_server_destroy(mtk_server* s) {
  if (!s) return MTK_OK;
  if (s->worker.joinable()) {
    s->stop = true;
    s->cv_work.notify_all();
    s->worker.join();
  }
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (auto& sl : s->slots) {
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.d_status) (void)hipFree(sl.d_status);
    if (sl.d_fit) (void)hipFree(sl.d_fit);
  }
  s->darena.reset();
  s->harena.reset();
  delete s;
  return MTK_OK;
}

}  // extern "C"
