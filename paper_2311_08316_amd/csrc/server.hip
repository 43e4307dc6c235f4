// Serving form of the factorization (derived from the serving goal; not in
// the paper): requests of uneven shape arrive at any time, are admitted in
// arrival order as a slot and enough device memory free up, and run
// concurrently, each on its slot's stream, so work of different requests
// overlaps on the device.
//
//   * Memory: one arena of the budget size is allocated at creation and
//     carved first-fit into per-request workspaces (256-byte aligned, freed
//     blocks coalesced), so admission never calls the HIP allocator.
//   * Slots: max_slots streams (default priority) with one completion event
//     each. A request occupies a slot from admission to completion.
//   * A scheduler thread retires finished requests (event query), then
//     admits the oldest pending request while it fits (no overtaking, so no
//     request starves), launching its stream-ordered factorization.
//   * Results do not depend on the mix: every kernel of the factorization
//     has a fixed reduction order and touches only its own request's
//     buffers, so a request returns the same bits alone and among others.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size): free blocks keyed by offset.
class Arena {
 public:
  static constexpr size_t kNone = ~(size_t)0;
  explicit Arena(size_t size) { free_[0] = size; }

  size_t alloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return off;
      }
    }
    return kNone;
  }

  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  const double* A = nullptr;
  int64_t lda = 0, m = 0, n = 0, d = 0;
  int32_t nnz = 0;
  uint64_t seed = 0;
  double tol = 0.0;
  double* Q = nullptr;
  int64_t ldq = 0;
  double* R = nullptr;
  int64_t ldr = 0;
  int64_t* J = nullptr;
  cqrrpt_info_t* info = nullptr;
  size_t ws_bytes = 0;
  size_t ws_off = 0;
  int slot = -1;
  int state = 0;  // 0 pending, 1 running, 2 done
  int rc = 0;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

}  // namespace

struct cqrrpt_server {
  int device = 0;
  cqrrpt_mode_t mode = CQRRPT_FP64;
  size_t budget = 0;
  char* base = nullptr;
  Arena* arena = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done_ev;
  std::vector<Request*> slot_req;
  // Per slot, pinned host copy of the running request's device status word
  // (info->status), copied on the slot's stream before its completion event.
  int32_t* status_host = nullptr;

  std::mutex mu;
  std::condition_variable cv;       // wakes the scheduler
  std::condition_variable done_cv;  // wakes drain()
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> all;
  uint64_t next_ticket = 1;
  int running = 0;
  bool stop = false;
  std::thread worker;

  void schedule();
  bool retire_locked();
  void admit_locked();
};

bool cqrrpt_server::retire_locked() {
  bool any = false;
  for (size_t s = 0; s < slot_req.size(); ++s) {
    Request* r = slot_req[s];
    if (!r) continue;
    const hipError_t q = hipEventQuery(done_ev[s]);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess && r->rc == 0) r->rc = CQRRPT_EHIP;
    // Device-side failures (non-finite input, barrier timeout) become the
    // request's status.
    if (q == hipSuccess && r->rc == 0 && status_host[s] != 0) r->rc = status_host[s];
    r->t_done = now_ms();
    r->state = 2;
    arena->release(r->ws_off, r->ws_bytes);
    slot_req[s] = nullptr;
    --running;
    any = true;
  }
  return any;
}

void cqrrpt_server::admit_locked() {
  while (!pending.empty()) {
    int slot = -1;
    for (size_t s = 0; s < slot_req.size(); ++s)
      if (!slot_req[s]) {
        slot = (int)s;
        break;
      }
    if (slot < 0) return;
    Request* r = pending.front();
    const size_t off = arena->alloc(r->ws_bytes);
    if (off == Arena::kNone) return;  // wait for memory; no overtaking
    pending.pop_front();
    r->ws_off = off;
    r->slot = slot;
    r->t_admit = now_ms();
    status_host[slot] = 0;
    r->rc = cqrrpt_factor_ex(r->A, r->lda, r->m, r->n, r->d, r->nnz, r->seed, r->tol, r->Q,
                             r->ldq, r->R, r->ldr, r->J, mode, base + off, r->ws_bytes,
                             streams[slot], r->info);
    if (r->rc == CQRRPT_OK &&
        hipMemcpyAsync(&status_host[slot], &r->info->status, sizeof(int32_t),
                       hipMemcpyDeviceToHost, streams[slot]) != hipSuccess)
      r->rc = CQRRPT_EHIP;
    if (r->rc == CQRRPT_OK && hipEventRecord(done_ev[slot], streams[slot]) != hipSuccess)
      r->rc = CQRRPT_EHIP;
    if (r->rc != CQRRPT_OK) {
      // Nothing (or not everything) was enqueued: finish at once.
      (void)hipStreamSynchronize(streams[slot]);
      r->t_done = now_ms();
      r->state = 2;
      arena->release(off, r->ws_bytes);
      continue;
    }
    r->state = 1;
    slot_req[slot] = r;
    ++running;
  }
}

void cqrrpt_server::schedule() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lock(mu);
  while (true) {
    retire_locked();
    admit_locked();
    done_cv.notify_all();
    if (stop && pending.empty() && running == 0) break;
    if (running == 0 && pending.empty()) {
      cv.wait(lock);
    } else {
      // Requests in flight: poll their events at a fine interval.
      lock.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lock.lock();
    }
  }
  done_cv.notify_all();
}

extern "C" {

cqrrpt_server_t* cqrrpt_server_create(size_t hbm_budget_bytes, int32_t max_slots,
                                      cqrrpt_mode_t mode) {
  if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 64) return nullptr;
  if (mode != CQRRPT_FP64 && mode != CQRRPT_MIXED && mode != CQRRPT_MIXED_CHECKED &&
      mode != CQRRPT_MIXED_FP32_CHOLQR2)
    return nullptr;
  cqrrpt_server_t* sv = new cqrrpt_server_t();
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return nullptr;
  }
  sv->mode = mode;
  sv->budget = (hbm_budget_bytes + 255) & ~(size_t)255;
  if (hipMalloc((void**)&sv->base, sv->budget) != hipSuccess) {
    delete sv;
    return nullptr;
  }
  if (hipHostMalloc((void**)&sv->status_host, sizeof(int32_t) * max_slots, 0) != hipSuccess) {
    (void)hipFree(sv->base);
    delete sv;
    return nullptr;
  }
  sv->arena = new Arena(sv->budget);
  sv->streams.resize(max_slots);
  sv->done_ev.resize(max_slots);
  sv->slot_req.assign(max_slots, nullptr);
  for (int s = 0; s < max_slots; ++s) {
    if (hipStreamCreateWithFlags(&sv->streams[s], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sv->done_ev[s], hipEventDisableTiming) != hipSuccess) {
      for (int t = 0; t <= s; ++t) {
        if (sv->streams[t]) (void)hipStreamDestroy(sv->streams[t]);
        if (sv->done_ev[t]) (void)hipEventDestroy(sv->done_ev[t]);
      }
      (void)hipFree(sv->base);
      (void)hipHostFree(sv->status_host);
      delete sv->arena;
      delete sv;
      return nullptr;
    }
  }
  sv->worker = std::thread([sv] { sv->schedule(); });
  return sv;
}

int cqrrpt_server_submit(cqrrpt_server_t* sv, const double* A, int64_t lda, int64_t m, int64_t n,
                         int64_t d, int32_t nnz, uint64_t seed, double tol, double* Q,
                         int64_t ldq, double* R, int64_t ldr, int64_t* J, cqrrpt_info_t* info,
                         uint64_t* ticket) {
  if (!sv) return -1;
  if (!ticket) return -17;
  const size_t wsb = cqrrpt_workspace_bytes(m, n, d, nnz, sv->mode);
  if (wsb == 0) return -5;  // shape or sketch parameters out of range
  if (((wsb + 255) & ~(size_t)255) > sv->budget) return CQRRPT_EBUDGET;
  if (!A || !Q || !R || !J || !info) return -2;
  Request* r = new Request();
  r->A = A;
  r->lda = lda;
  r->m = m;
  r->n = n;
  r->d = d;
  r->nnz = nnz;
  r->seed = seed;
  r->tol = tol;
  r->Q = Q;
  r->ldq = ldq;
  r->R = R;
  r->ldr = ldr;
  r->J = J;
  r->info = info;
  r->ws_bytes = wsb;
  r->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->stop) {
      delete r;
      return -1;
    }
    r->ticket = sv->next_ticket++;
    sv->all[r->ticket] = r;
    sv->pending.push_back(r);
  }
  sv->cv.notify_one();
  *ticket = r->ticket;
  return CQRRPT_OK;
}

int cqrrpt_server_poll(cqrrpt_server_t* sv, uint64_t ticket, int32_t* done) {
  if (!sv || !done) return -1;
  std::lock_guard<std::mutex> lock(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return -2;
  *done = it->second->state == 2 ? 1 : 0;
  return it->second->state == 2 ? it->second->rc : CQRRPT_OK;
}

int cqrrpt_server_ticket_times(cqrrpt_server_t* sv, uint64_t ticket, double* ms3) {
  if (!sv || !ms3) return -1;
  std::lock_guard<std::mutex> lock(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return -2;
  const Request* r = it->second;
  ms3[0] = r->t_submit;
  ms3[1] = r->t_admit;
  ms3[2] = r->t_done;
  return CQRRPT_OK;
}

int cqrrpt_server_release(cqrrpt_server_t* sv, uint64_t ticket) {
  if (!sv) return -1;
  std::lock_guard<std::mutex> lock(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return -2;
  if (it->second->state != 2) return -3;
  delete it->second;
  sv->all.erase(it);
  return CQRRPT_OK;
}

int cqrrpt_server_drain(cqrrpt_server_t* sv) {
  if (!sv) return -1;
  std::unique_lock<std::mutex> lock(sv->mu);
  sv->cv.notify_one();
  sv->done_cv.wait(lock, [sv] { return sv->pending.empty() && sv->running == 0; });
  int rc = CQRRPT_OK;
  for (auto& kv : sv->all)
    if (kv.second->rc != CQRRPT_OK && rc == CQRRPT_OK) rc = kv.second->rc;
  return rc;
}

void cqrrpt_server_destroy(cqrrpt_server_t* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lock(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_one();
  if (sv->worker.joinable()) sv->worker.join();
  for (size_t s = 0; s < sv->streams.size(); ++s) {
    (void)hipStreamSynchronize(sv->streams[s]);
    (void)hipStreamDestroy(sv->streams[s]);
    (void)hipEventDestroy(sv->done_ev[s]);
  }
  (void)hipFree(sv->base);
  (void)hipHostFree(sv->status_host);
  for (auto& kv : sv->all) delete kv.second;
  delete sv->arena;
  delete sv;
}

}  // extern "C"
