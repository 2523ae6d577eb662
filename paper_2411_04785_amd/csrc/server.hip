// Continuous-batching server for CP-ALS decompositions (C ABI: mtk_server_*).
//
// A worker thread owns the device side and runs a scheduler loop:
//  - admission: requests are admitted in arrival order when a slot is free
//    and their device block can be carved out of the server's arena without
//    the arena's device footprint passing the HBM budget.  Admission queues
//    the upload of the request's tensor and initial factors and the Gram
//    matrices of its factors 1 and 2 on the copy stream;
//  - steps: every uploaded request advances by one CP-ALS sweep (three mode
//    updates) per step.  A step is one HIP graph, captured when the server
//    is created and replayed for every step: for each update, the grouped
//    contraction of all resident requests with the grouped inversion of
//    their V (inside the contraction launch when every rank is at most 64,
//    else on a parallel branch), then the grouped apply (F = M V^{-1}) and
//    the grouped normalisation with the new factor's Gram partials
//    (srv_internal.h).  The host writes the step's request table into
//    pinned memory and copies it to the device before each replay; two
//    tables alternate, so the worker prepares a step while the previous one
//    runs;
//  - completion: after a request's last update its fit (direct residual) and
//    the download of its factors, lambda, fit and status are queued behind
//    the step, and an event marks the request done; the worker then retires
//    it (results to the caller's buffers, memory and slot freed).
// A request's work items, plans and summation orders depend only on its own
// shape, rank, mode and precision, never on the other entries of a step, so
// its result is bitwise the same alone and in any mix.  Factor state stays
// on the device from admission to completion.

#include "mtk_internal.h"
#include "srv_internal.h"

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

// First-fit sub-allocator over a list of chunks (device or pinned host
// memory).  Free blocks are coalesced with their neighbours.  Chunks are
// never returned (freeing device memory synchronises the device), and the
// total of the chunks -- the arena's footprint -- is kept at or below
// `limit`: an allocation that would need a chunk past it fails instead.
class Arena {
 public:
  using AllocFn = void* (*)(size_t);
  using FreeFn = void (*)(void*);
  Arena(AllocFn a, FreeFn f, size_t chunk, size_t limit) : alloc_(a), free_(f), chunk_(chunk), limit_(limit) {}
  ~Arena() {
    for (auto& c : chunks_) free_(c.base);
  }
  void* alloc(size_t bytes) {
    bytes = r256(std::max<size_t>(bytes, 256));
    for (auto& c : chunks_)
      if (void* p = take(c, bytes)) return p;
    const size_t sz = std::max(chunk_, bytes);
    if (footprint_ + sz > limit_) return nullptr;
    void* base = alloc_(sz);
    if (!base) return nullptr;
    chunks_.push_back(Chunk{static_cast<char*>(base), sz, {{0, sz}}, {}});
    footprint_ += sz;
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
  size_t footprint() const { return footprint_; }
  // Return every chunk that holds no block (hipFree synchronises the device;
  // called only when nothing is resident).
  void trim() {
    for (auto it = chunks_.begin(); it != chunks_.end();) {
      if (it->used.empty()) {
        free_(it->base);
        footprint_ -= it->size;
        it = chunks_.erase(it);
      } else {
        ++it;
      }
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
  size_t chunk_, limit_;
  size_t footprint_ = 0;
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

size_t elem_count(const int64_t d[3]) { return (size_t)d[0] * d[1] * d[2]; }
int64_t max_dim(const int64_t d[3]) { return std::max(d[0], std::max(d[1], d[2])); }

// Device block of a request: X, factors, lambda, the contraction's partial
// slices (M itself when a mode has one slice), the solve region, the fit
// scratch, and a 256-byte status block (status word, then the two fit sums).
struct Layout {
  size_t x, f[3], lam, part, solve, fit, status, total;
};

Layout layout(const int64_t dims[3], int R, int prec) {
  Layout L{};
  size_t o = 0;
  L.x = o; o += r256(elem_count(dims) * sizeof(float));
  for (int m = 0; m < 3; ++m) { L.f[m] = o; o += r256((size_t)dims[m] * R * sizeof(float)); }
  L.lam = o; o += r256((size_t)R * sizeof(double));
  size_t part = 0;
  for (int m = 0; m < 3; ++m) {
    const mtk::SrvContract c = mtk::srv_contract_plan(dims, R, m, prec, true);
    part = std::max(part, (size_t)std::max(1, c.slices) * c.nM * R * sizeof(float));
  }
  L.part = o; o += r256(part);
  L.solve = o; o += r256(mtk::solve_ws_bytes(max_dim(dims), R));
  L.fit = o; o += r256(mtk::fit_ws_bytes(dims));
  L.status = o; o += 256;
  L.total = o;
  return L;
}

// Pinned host block of a request: X, the three initial factors (overwritten
// by the results), lambda, then the fit sums and status copied back.
size_t host_bytes(const int64_t dims[3], int R) {
  size_t b = r256(elem_count(dims) * sizeof(float));
  for (int m = 0; m < 3; ++m) b += r256((size_t)dims[m] * R * sizeof(float));
  return b + r256((size_t)R * sizeof(double)) + 256;
}

enum State { kPending = 0, kUploading, kRunning, kFinishing };

struct Req {
  int64_t id = 0;
  int64_t dims[3] = {0, 0, 0};
  int R = 0, prec = 0, sweeps = 0;
  size_t dev_bytes = 0;
  char* hbuf = nullptr;
  float* out_f[3] = {nullptr, nullptr, nullptr};
  double* out_lambda = nullptr;
  mtk_result res{};
  // device side
  char* dbuf = nullptr;
  Layout L{};
  mtk::SrvContract plan[3];
  int state = kPending;
  int done_sweeps = 0;             // sweeps queued so far
};

struct Slot {
  hipEvent_t ready = nullptr;      // upload done
  hipEvent_t done = nullptr;       // results downloaded
  std::unique_ptr<Req> req;
};

}  // namespace

struct mtk_server {
  int device = 0;
  uint64_t budget = 0;
  int max_slots = 1;
  int max_rank = mtk::kMaxRank;
  std::chrono::steady_clock::time_point t0;
  std::unique_ptr<Arena> darena, harena;
  std::vector<Slot> slots;
  hipStream_t copy = nullptr, compute = nullptr, cap = nullptr, side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // Two alternating step tables: pinned host copy, device copy, the captured
  // step that reads it, and the event that marks that step done.
  mtk::SrvTable* htab[2] = {nullptr, nullptr};
  mtk::SrvTable* dtab[2] = {nullptr, nullptr};
  // Captured steps per table and variant: [0] inversion inside the
  // contraction launch (every R <= 64), [1] on a parallel branch (any R).
  hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipEvent_t step_ev[2] = {nullptr, nullptr};
  bool step_pending[2] = {false, false};
  int next_tab = 0;
  std::mutex mu;                   // guards pending, finished, harena, counters
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Req>> pending;
  std::deque<mtk_result> finished;
  std::atomic<bool> stop{false};
  uint64_t in_use = 0, peak = 0;
  uint64_t steps = 0;
  int max_batch = 0;
  int resident = 0;
  std::thread worker;

  hipError_t capture_steps() {
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 2; ++v) {
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = hipSuccess;
        for (int u = 0; u < 3 && le == hipSuccess; ++u) {
          if (v == 0) {
            le = mtk::launch_srv_contract(dtab[b], u, true, cap);
          } else {
            le = hipEventRecord(fork_ev, cap);
            if (le == hipSuccess) le = hipStreamWaitEvent(side, fork_ev, 0);
            if (le == hipSuccess) le = mtk::launch_srv_factor(dtab[b], u, max_rank, side);
            if (le == hipSuccess) le = mtk::launch_srv_contract(dtab[b], u, false, cap);
            if (le == hipSuccess) le = hipEventRecord(join_ev, side);
            if (le == hipSuccess) le = hipStreamWaitEvent(cap, join_ev, 0);
          }
          if (le == hipSuccess) le = mtk::launch_srv_apply(dtab[b], u, cap);
          if (le == hipSuccess) le = mtk::launch_srv_normalize(dtab[b], u, cap);
        }
        e = hipStreamEndCapture(cap, &graph[b][v]);
        if (le != hipSuccess) return le;
        if (e != hipSuccess) return e;
        if ((e = hipGraphInstantiate(&exec[b][v], graph[b][v], nullptr, nullptr, 0)) != hipSuccess) return e;
      }
    return hipSuccess;
  }

  void bind(Req& r) {
    r.L = layout(r.dims, r.R, r.prec);
    for (int m = 0; m < 3; ++m) r.plan[m] = mtk::srv_contract_plan(r.dims, r.R, m, r.prec, true);
  }
  float* X(Req& r) { return reinterpret_cast<float*>(r.dbuf + r.L.x); }
  float* F(Req& r, int m) { return reinterpret_cast<float*>(r.dbuf + r.L.f[m]); }
  double* lam(Req& r) { return reinterpret_cast<double*>(r.dbuf + r.L.lam); }
  int* status(Req& r) { return reinterpret_cast<int*>(r.dbuf + r.L.status); }
  double* fit_acc(Req& r) { return reinterpret_cast<double*>(r.dbuf + r.L.status + 16); }

  // Upload X and the initial factors, then the Gram partials of factors 1
  // and 2 (the first update needs them), on the copy stream.
  hipError_t start_upload(Slot& s) {
    Req& r = *s.req;
    const int R = r.R;
    const size_t nx = elem_count(r.dims);
    const char* h = r.hbuf;
    hipError_t e;
    if ((e = hipMemsetAsync(status(r), 0, 256, copy)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(X(r), h, nx * sizeof(float), hipMemcpyHostToDevice, copy)) != hipSuccess) return e;
    h += r256(nx * sizeof(float));
    for (int m = 0; m < 3; ++m) {
      const size_t b = (size_t)r.dims[m] * R * sizeof(float);
      if ((e = hipMemcpyAsync(F(r, m), h, b, hipMemcpyHostToDevice, copy)) != hipSuccess) return e;
      h += r256(b);
    }
    if ((e = hipMemcpyAsync(lam(r), h, (size_t)R * sizeof(double), hipMemcpyHostToDevice, copy)) != hipSuccess)
      return e;
    const float* cf[3] = {F(r, 0), F(r, 1), F(r, 2)};
    if ((e = mtk::launch_grams(cf, r.dims, R, 1, 2, max_dim(r.dims), r.dbuf + r.L.solve, status(r), copy)) !=
        hipSuccess)
      return e;
    return hipEventRecord(s.ready, copy);
  }

  // The table entry of request r for update (mode) n of its next sweep.
  void fill_entry(Req& r, int n, mtk::SrvEntry& en) {
    mtk::SrvContract c = r.plan[n];
    c.X = X(r);
    c.frag = n == 2 ? F(r, 1) : F(r, 2);
    c.weight = n == 0 ? F(r, 1) : F(r, 0);
    c.part = reinterpret_cast<float*>(r.dbuf + r.L.part);
    en.c = c;
    en.u = mtk::srv_update(r.dims, r.R, n, max_dim(r.dims), r.dbuf + r.L.solve, c.part, c.slices,
                           (int64_t)c.nM * r.R, F(r, n), lam(r), status(r));
  }

  // Fit and download of a request behind the step that made its last update.
  hipError_t finish(Slot& s) {
    Req& r = *s.req;
    const int R = r.R;
    const float* cf[3] = {F(r, 0), F(r, 1), F(r, 2)};
    hipError_t e = mtk::launch_fit(X(r), MTK_FP32, nullptr, r.dims, cf, lam(r), R, fit_acc(r), r.dbuf + r.L.fit,
                                   compute);
    if (e != hipSuccess) return e;
    char* h = r.hbuf + r256(elem_count(r.dims) * sizeof(float));
    for (int m = 0; m < 3; ++m) {
      const size_t b = (size_t)r.dims[m] * R * sizeof(float);
      if ((e = hipMemcpyAsync(h, F(r, m), b, hipMemcpyDeviceToHost, compute)) != hipSuccess) return e;
      h += r256(b);
    }
    if ((e = hipMemcpyAsync(h, lam(r), (size_t)R * sizeof(double), hipMemcpyDeviceToHost, compute)) != hipSuccess)
      return e;
    h += r256((size_t)R * sizeof(double));
    if ((e = hipMemcpyAsync(h, r.dbuf + r.L.status, 32, hipMemcpyDeviceToHost, compute)) != hipSuccess) return e;
    r.state = kFinishing;
    return hipEventRecord(s.done, compute);
  }

  void release(Slot& s) {
    Req& r = *s.req;
    if (r.dbuf) darena->release(r.dbuf);
    r.dbuf = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    harena->release(r.hbuf);
    in_use -= r.dev_bytes;
    --resident;
    finished.push_back(r.res);
    s.req.reset();
    cv_done.notify_all();
  }

  void retire(Slot& s) {
    Req& r = *s.req;
    const int R = r.R;
    const char* h = r.hbuf + r256(elem_count(r.dims) * sizeof(float));
    for (int m = 0; m < 3; ++m) {
      const size_t b = (size_t)r.dims[m] * R * sizeof(float);
      if (r.out_f[m]) std::memcpy(r.out_f[m], h, b);
      h += r256(b);
    }
    if (r.out_lambda) std::memcpy(r.out_lambda, h, (size_t)R * sizeof(double));
    h += r256((size_t)R * sizeof(double));
    int st = 0;
    double fit[2];
    std::memcpy(&st, h, sizeof(int));
    std::memcpy(fit, h + 16, sizeof(fit));
    r.res.fit = 1.0 - std::sqrt(fit[0]) / std::sqrt(fit[1]);
    if (st & mtk::kStatusNotSPD) r.res.status = MTK_ENOTSPD;
    r.res.t_done = now_s(t0);
    release(s);
  }

  void fail_slot(Slot& s, mtk_status st) {
    (void)hipStreamSynchronize(copy);
    (void)hipStreamSynchronize(compute);
    s.req->res.status = st;
    s.req->res.t_done = now_s(t0);
    release(s);
  }

  // One scheduler step (a sweep) over the running requests; false if none runs.
  bool step() {
    std::vector<Slot*> run;
    for (auto& s : slots)
      if (s.req && s.req->state == kRunning) run.push_back(&s);
    if (run.empty()) return false;
    const int b = next_tab;
    next_tab ^= 1;
    if (step_pending[b]) {            // the table's last copy must have been read
      (void)hipEventSynchronize(step_ev[b]);
      step_pending[b] = false;
    }
    mtk::SrvTable* t = htab[b];
    t->nreq = (int)run.size();
    int rmax = 0;
    for (int u = 0; u < 3; ++u) {
      int64_t wi = 0, ab = 0, nb = 0;
      for (size_t q = 0; q < run.size(); ++q) {
        mtk::SrvEntry& en = t->e[q][u];
        fill_entry(*run[q]->req, u, en);
        en.wi0 = wi;
        en.ab0 = ab;
        en.nb0 = nb;
        wi += mtk::srv_contract_items(en.c);
        ab += mtk::srv_apply_blocks(en.u);
        nb += mtk::srv_normalize_blocks(en.u);
      }
      t->n_wi[u] = wi;
      t->n_ab[u] = ab;
      t->n_nb[u] = nb;
    }
    for (Slot* s : run) rmax = std::max(rmax, s->req->R);
    const int v = rmax <= mtk::kSrvFusedMaxRank ? 0 : 1;
    hipError_t e = hipMemcpyAsync(dtab[b], t, mtk::srv_table_bytes(t->nreq), hipMemcpyHostToDevice, compute);
    if (e == hipSuccess) e = hipGraphLaunch(exec[b][v], compute);
    if (e == hipSuccess) e = hipEventRecord(step_ev[b], compute);
    if (e != hipSuccess) {
      for (Slot* s : run) fail_slot(*s, MTK_EHIP);
      return true;
    }
    step_pending[b] = true;
    ++steps;
    max_batch = std::max(max_batch, (int)run.size());
    for (Slot* s : run) {
      Req& r = *s->req;
      if (++r.done_sweeps == r.sweeps && finish(*s) != hipSuccess) fail_slot(*s, MTK_EHIP);
    }
    return true;
  }

  void run() {
    (void)hipSetDevice(device);
    while (true) {
      bool did = false;
      for (auto& s : slots) {
        if (!s.req) continue;
        if (s.req->state == kFinishing && hipEventQuery(s.done) == hipSuccess) {
          retire(s);
          did = true;
        } else if (s.req->state == kUploading && hipEventQuery(s.ready) == hipSuccess) {
          s.req->state = kRunning;
          if (s.req->sweeps == 0 && finish(s) != hipSuccess) fail_slot(s, MTK_EHIP);
          did = true;
        }
      }
      // Admit in arrival order while a slot is free and the arena (kept
      // within the budget) has room.
      while (true) {
        Slot* s = nullptr;
        for (auto& q : slots)
          if (!q.req) { s = &q; break; }
        if (!s) break;
        std::unique_ptr<Req> r;
        {
          std::lock_guard<std::mutex> lk(mu);
          if (pending.empty()) break;
          char* d = static_cast<char*>(darena->alloc(pending.front()->dev_bytes));
          if (!d && resident == 0 && darena->footprint() > 0) {
            // Nothing resident: every chunk is free, so give them back and
            // let the head request take a chunk of its own size.
            darena->trim();
            d = static_cast<char*>(darena->alloc(pending.front()->dev_bytes));
          }
          if (!d) break;
          r = std::move(pending.front());
          pending.pop_front();
          r->dbuf = d;
          in_use += r->dev_bytes;
          peak = std::max(peak, in_use);
          ++resident;
        }
        bind(*r);
        r->res.t_admit = now_s(t0);
        r->state = kUploading;
        s->req = std::move(r);
        if (start_upload(*s) != hipSuccess) fail_slot(*s, MTK_EHIP);
        did = true;
      }
      if (step()) continue;
      if (did) continue;
      std::unique_lock<std::mutex> lk(mu);
      if (stop && pending.empty() && resident == 0) break;
      cv_work.wait_for(lk, std::chrono::microseconds(resident > 0 ? 50 : 2000));
    }
  }
};

extern "C" {

mtk_status mtk_server_create(mtk_server** out, int device, uint64_t budget_bytes, int max_slots) {
  if (!out || max_slots < 1 || max_slots > mtk::kSrvMaxReq || budget_bytes == 0) return MTK_EINVAL;
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
  // Chunks of 1 GiB, or an eighth of a smaller budget (at least 1 MiB, at
  // most the budget).
  const size_t chunk = std::min<size_t>(
      {(size_t)1 << 30, std::max<size_t>(budget_bytes / 8, (size_t)1 << 20), (size_t)budget_bytes});
  s->darena.reset(new Arena(dev_alloc, dev_free, chunk, budget_bytes));
  s->harena.reset(new Arena(host_alloc, host_free, (size_t)1 << 30, ~(size_t)0));
  s->slots.resize(max_slots);
  bool ok = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming) == hipSuccess;
  for (int b = 0; b < 2 && ok; ++b)
    ok = hipHostMalloc((void**)&s->htab[b], sizeof(mtk::SrvTable), hipHostMallocDefault) == hipSuccess &&
         hipMalloc((void**)&s->dtab[b], sizeof(mtk::SrvTable)) == hipSuccess &&
         hipEventCreateWithFlags(&s->step_ev[b], hipEventDisableTiming) == hipSuccess;
  for (auto& sl : s->slots) {
    if (!ok) break;
    ok = hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
  }
  if (ok) ok = s->capture_steps() == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    mtk_server_destroy(s);
    return MTK_EHIP;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return MTK_OK;
}

mtk_status mtk_server_submit(mtk_server* s, int64_t id, const float* x, const int64_t dims[3], int64_t R, int prec,
                             int sweeps, const float* const init[3], float* const factors_out[3],
                             double* lambda_out) {
  if (!s || !x || !dims || !init || !init[0] || !init[1] || !init[2]) return MTK_EINVAL;
  if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || R < 1 || R > s->max_rank || sweeps < 0) return MTK_EINVAL;
  if (dims[0] > (1 << 24) || dims[1] > (1 << 24) || dims[2] > (1 << 24)) return MTK_EINVAL;
  if (prec != MTK_FP32 && prec != MTK_BF16X3) return MTK_EINVAL;
  auto r = std::make_unique<Req>();
  r->id = id;
  for (int m = 0; m < 3; ++m) r->dims[m] = dims[m];
  r->R = (int)R;
  r->prec = prec;
  r->sweeps = sweeps;
  r->dev_bytes = layout(dims, (int)R, prec).total;
  if (r->dev_bytes > s->budget) return MTK_EBUDGET;
  for (int m = 0; m < 3; ++m) r->out_f[m] = factors_out ? factors_out[m] : nullptr;
  r->out_lambda = lambda_out;
  r->res.id = id;
  r->res.status = MTK_OK;
  r->res.R = (int)R;
  for (int m = 0; m < 3; ++m) r->res.dims[m] = dims[m];
  r->res.t_submit = now_s(s->t0);
  const size_t hb = host_bytes(dims, (int)R);
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
  double* lam0 = reinterpret_cast<double*>(h);       // lambda starts at 1
  for (int64_t c = 0; c < R; ++c) lam0[c] = 1.0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->pending.push_back(std::move(r));
  }
  s->cv_work.notify_one();
  return MTK_OK;
}

uint64_t mtk_server_request_bytes(const int64_t dims[3], int64_t R, int prec) {
  if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || R < 1 || R > mtk::kMaxRank) return 0;
  if (dims[0] > (1 << 24) || dims[1] > (1 << 24) || dims[2] > (1 << 24)) return 0;
  if (prec != MTK_FP32 && prec != MTK_BF16X3) return 0;
  return layout(dims, (int)R, prec).total;
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

mtk_status mtk_server_stats(mtk_server* s, mtk_server_stat* out) {
  if (!s || !out) return MTK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->resident = s->resident;
  out->max_batch = s->max_batch;
  out->bytes_in_use = s->in_use;
  out->peak_bytes_in_use = s->peak;
  out->device_bytes = s->darena ? s->darena->footprint() : 0;
  out->steps = s->steps;
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
  for (int b = 0; b < 2; ++b) {
    for (int v = 0; v < 2; ++v) {
      if (s->exec[b][v]) (void)hipGraphExecDestroy(s->exec[b][v]);
      if (s->graph[b][v]) (void)hipGraphDestroy(s->graph[b][v]);
    }
    if (s->htab[b]) (void)hipHostFree(s->htab[b]);
    if (s->dtab[b]) (void)hipFree(s->dtab[b]);
    if (s->step_ev[b]) (void)hipEventDestroy(s->step_ev[b]);
  }
  for (auto& sl : s->slots) {
    if (sl.ready) (void)hipEventDestroy(sl.ready);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  for (hipStream_t st : {s->copy, s->compute, s->cap, s->side})
    if (st) (void)hipStreamDestroy(st);
  if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
  if (s->join_ev) (void)hipEventDestroy(s->join_ev);
  s->darena.reset();
  s->harena.reset();
  delete s;
  return MTK_OK;
}

}  // extern "C"
