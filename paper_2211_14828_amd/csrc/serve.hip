// Request server for many small decompositions (continuous batching).
//
// The server owns one device arena of a fixed HBM budget and a pool of
// slots; each slot is a worker thread with its own HIP stream (default
// priority) and a pinned host block for its results.  Requests are queued by
// rbki_server_submit.  A free worker takes the oldest queued request as soon
// as the request's footprint (the workspace of rbki_tucker for its shape)
// fits into the arena's free memory, carves that workspace out of the arena
// (first fit), enqueues the whole decomposition on its stream and waits for
// that stream only.  Requests admitted by different workers run concurrently
// on the device; finishing one frees its memory and its slot, which admits
// the next.  No device memory is allocated after rbki_server_create.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rbki_api_internal.h"

namespace {

using clk = std::chrono::steady_clock;

// First-fit allocator over [0, cap) with coalescing of freed neighbours.
class ArenaAlloc {
 public:
  explicit ArenaAlloc(size_t cap) { free_[0] = cap; }
  bool alloc(size_t bytes, size_t& off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_[off] = bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, size = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + size) {
      size += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = size;
  }

 private:
  std::map<size_t, size_t> free_;   // offset -> size
  std::map<size_t, size_t> used_;
};

struct Request {
  uint64_t id = 0;
  const void* X = nullptr;
  int xtype = 0;
  std::vector<int64_t> dims, ranks;
  rbki_params prm{};
  void* core = nullptr;
  std::vector<void*> factors;
  int out_type = RBKI_F32;
  size_t bytes = 0;
  clk::time_point t_submit, t_done;
  bool done = false;
  rbki_status status = RBKI_OK;
  std::string err;
  double rel_err = 0.0;
};

}  // namespace

// One worker's resources: its non-blocking stream, a blocking-sync event (the worker
// sleeps on it while its solve runs: many workers spinning in a stream
// synchronisation would starve the host threads that enqueue other solves)
// and a pinned block for the results read back at the end of a solve.
namespace rbki {
struct ServerSlot {
  hipStream_t stream = nullptr;
  hipEvent_t fin = nullptr;
  HostResult* hr = nullptr;
};
}  // namespace rbki

struct rbki_server {
  int device = 0;
  std::vector<rbki::ServerSlot> slots;
  char* arena = nullptr;
  size_t cap = 0;
  std::unique_ptr<ArenaAlloc> alloc;
  std::mutex mu;
  std::condition_variable cv_work;   // queue changed or memory freed
  std::condition_variable cv_done;   // a request finished
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_id = 1;
  int inflight = 0;
};

namespace {

void worker_main(rbki_server* sv, rbki::ServerSlot* slot) {
  (void)hipSetDevice(sv->device);
  hipStream_t st = slot->stream;
  hipEvent_t fin = slot->fin;
  rbki::HostResult* hr = slot->hr;
  for (;;) {
    Request* r = nullptr;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      // admission: the oldest request, once its footprint fits the free
      // memory; on shutdown the queue is drained first
      bool got = false;
      sv->cv_work.wait(lk, [&] {
        if (!sv->queue.empty() && sv->alloc->alloc(sv->reqs[sv->queue.front()]->bytes, off)) {
          got = true;
          return true;
        }
        return sv->stop && sv->queue.empty();
      });
      if (!got) break;
      r = sv->reqs[sv->queue.front()].get();
      sv->queue.pop_front();
      ++sv->inflight;
    }
    rbki_status s = rbki::tucker_enqueue(r->X, r->xtype, &r->prm, r->core, r->factors.data(), r->out_type,
                                         sv->arena + off, r->bytes, st, hr);
    std::string msg;
    if (s == RBKI_OK) {
      hipError_t e = hipEventRecord(fin, st);
      if (e == hipSuccess) e = hipEventSynchronize(fin);
      if (e != hipSuccess) {
        s = RBKI_E_HIP;
        msg = hipGetErrorString(e);
      } else {
        s = rbki::finish_result(*hr, &r->rel_err);
        if (s != RBKI_OK) msg = rbki_last_error();
      }
    } else {
      msg = rbki_last_error();
      (void)hipStreamSynchronize(st);                    // nothing of it may still run on the arena
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->alloc->release(off);
      r->status = s;
      r->err = msg;
      r->t_done = clk::now();
      r->done = true;
      --sv->inflight;
    }
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
  }
  (void)hipStreamSynchronize(st);
}

void free_slots(rbki_server* sv) {
  for (auto& sl : sv->slots) {
    if (sl.fin) (void)hipEventDestroy(sl.fin);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.hr) (void)hipHostFree(sl.hr);
  }
  sv->slots.clear();
}

}  // namespace

extern "C" {

size_t rbki_server_request_bytes(const rbki_params* prm, int xtype) { return rbki_tucker_workspace(prm, xtype); }

rbki_status rbki_server_create(size_t hbm_budget_bytes, int slots, rbki_server** out) {
  if (!out || slots < 1 || slots > 64 || hbm_budget_bytes < ((size_t)1 << 20)) {
    rbki::set_error(RBKI_E_INVALID, "server: need out != NULL, 1 <= slots <= 64, budget >= 1 MiB");
    return RBKI_E_INVALID;
  }
  auto sv = std::make_unique<rbki_server>();
  if (hipGetDevice(&sv->device) != hipSuccess) {
    rbki::set_error(RBKI_E_HIP, "server: no current device");
    return RBKI_E_HIP;
  }
  sv->cap = hbm_budget_bytes & ~(size_t)255;
  if (hipMalloc((void**)&sv->arena, sv->cap) != hipSuccess) {
    rbki::set_error(RBKI_E_NOMEM, "server: cannot allocate the arena");
    return RBKI_E_NOMEM;
  }
  sv->alloc = std::make_unique<ArenaAlloc>(sv->cap);
  sv->slots.resize(slots);
  for (auto& sl : sv->slots) {
    // non-blocking: work a caller puts on the legacy default stream neither
    // waits for the server's solves nor makes them wait
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.fin, hipEventBlockingSync | hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.hr, sizeof(rbki::HostResult)) != hipSuccess) {
      free_slots(sv.get());
      (void)hipFree(sv->arena);
      rbki::set_error(RBKI_E_HIP, "server: cannot create the worker streams");
      return RBKI_E_HIP;
    }
  }
  for (auto& sl : sv->slots) sv->workers.emplace_back(worker_main, sv.get(), &sl);
  *out = sv.release();
  return RBKI_OK;
}

rbki_status rbki_server_submit(rbki_server* sv, const void* X, int xtype, const rbki_params* prm, void* core,
                               void* const* factors, int out_type, uint64_t* ticket) {
  if (!sv || !X || !prm || !ticket) {
    rbki::set_error(RBKI_E_INVALID, "server_submit: NULL argument");
    return RBKI_E_INVALID;
  }
  const size_t bytes = rbki_tucker_workspace(prm, xtype);   // validates the problem
  if (bytes == 0) return RBKI_E_INVALID;
  if (out_type != RBKI_F64 && out_type != RBKI_F32) {
    rbki::set_error(RBKI_E_INVALID, "server_submit: out_type must be F64 or F32");
    return RBKI_E_INVALID;
  }
  if (bytes > sv->cap) {
    rbki::set_error(RBKI_E_INVALID, "server_submit: request footprint exceeds the server budget");
    return RBKI_E_INVALID;
  }
  auto r = std::make_unique<Request>();
  r->X = X;
  r->xtype = xtype;
  r->dims.assign(prm->dims, prm->dims + prm->order);
  r->ranks.assign(prm->ranks, prm->ranks + prm->order);
  r->prm = *prm;
  r->prm.dims = r->dims.data();
  r->prm.ranks = r->ranks.data();
  r->core = core;
  if (factors) r->factors.assign(factors, factors + prm->order);
  else r->factors.assign(prm->order, nullptr);
  r->out_type = out_type;
  r->bytes = bytes;
  r->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      rbki::set_error(RBKI_E_INVALID, "server_submit: server is stopping");
      return RBKI_E_INVALID;
    }
    r->id = sv->next_id++;
    *ticket = r->id;
    sv->queue.push_back(r->id);
    sv->reqs[r->id] = std::move(r);
  }
  sv->cv_work.notify_all();
  return RBKI_OK;
}

static rbki_status collect(rbki_server* sv, std::unique_lock<std::mutex>& lk, uint64_t ticket, double* rel_err,
                           double* latency_ms) {
  auto it = sv->reqs.find(ticket);
  Request* r = it->second.get();
  const rbki_status s = r->status;
  if (rel_err) *rel_err = r->rel_err;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  const std::string err = r->err;
  sv->reqs.erase(it);
  lk.unlock();
  if (s != RBKI_OK) rbki::set_error(s, err.c_str());
  return s;
}

rbki_status rbki_server_poll(rbki_server* sv, uint64_t ticket, int* done, double* rel_err, double* latency_ms) {
  if (!sv || !done) {
    rbki::set_error(RBKI_E_INVALID, "server_poll: NULL argument");
    return RBKI_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) {
    rbki::set_error(RBKI_E_INVALID, "server_poll: unknown ticket");
    return RBKI_E_INVALID;
  }
  *done = it->second->done ? 1 : 0;
  if (!*done) return RBKI_OK;
  return collect(sv, lk, ticket, rel_err, latency_ms);
}

rbki_status rbki_server_wait(rbki_server* sv, uint64_t ticket, double* rel_err, double* latency_ms) {
  if (!sv) {
    rbki::set_error(RBKI_E_INVALID, "server_wait: NULL server");
    return RBKI_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) {
    rbki::set_error(RBKI_E_INVALID, "server_wait: unknown ticket");
    return RBKI_E_INVALID;
  }
  Request* r = it->second.get();
  sv->cv_done.wait(lk, [&] { return r->done; });
  return collect(sv, lk, ticket, rel_err, latency_ms);
}

rbki_status rbki_server_destroy(rbki_server* sv) {
  if (!sv) return RBKI_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  free_slots(sv);
  (void)hipFree(sv->arena);
  delete sv;
  return RBKI_OK;
}

}  // extern "C"
