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
//     admits pending requests in arrival order while slots and memory allow
//     (no overtaking, so no request starves). The requests admitted together
//     form a batch: each runs its sketch, its rank stage, preconditioning
//     solve and Gram, and its Q and R products on its own slot stream, while
//     their QRCPs and their Cholesky steps run as one cooperative launch each
//     (one gang of workgroups per request) on the server's small-step
//     stream, ordered by events. Cooperative launches of separate requests
//     would run one after another; in one launch they run side by side.
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
  cqh::Phased* ph = nullptr;
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
  std::vector<hipEvent_t> front_ev;  // per slot: sketch done / Gram done
  std::vector<Request*> slot_req;
  hipStream_t small = nullptr;         // batched QRCP and Cholesky launches
  hipEvent_t small_ev = nullptr;
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
  void launch_batch(std::vector<Request*>& batch);
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
  std::vector<Request*> batch;
  std::vector<char> taken(slot_req.size(), 0);
  while (!pending.empty()) {
    int slot = -1;
    for (size_t s = 0; s < slot_req.size(); ++s)
      if (!slot_req[s] && !taken[s]) {
        slot = (int)s;
        break;
      }
    if (slot < 0) break;
    Request* r = pending.front();
    const size_t off = arena->alloc(r->ws_bytes);
    if (off == Arena::kNone) break;  // wait for memory; no overtaking
    pending.pop_front();
    r->ws_off = off;
    r->slot = slot;
    r->t_admit = now_ms();
    taken[slot] = 1;
    batch.push_back(r);
  }
  if (!batch.empty()) launch_batch(batch);
}

// Enqueues a batch: per request, its phases on its slot stream; the QRCPs
// and Cholesky steps of the batch in one launch each on the small-step
// stream, which waits for the requests' earlier phases and which the slot
// streams wait for in turn. A request whose setup fails finishes at once.
void cqrrpt_server::launch_batch(std::vector<Request*>& batch) {
  std::vector<Request*> live;
  for (Request* r : batch) {
    const int slot = r->slot;
    status_host[slot] = 0;
    int rc = CQRRPT_OK;
    r->ph = cqh::phased_begin(r->A, r->lda, r->m, r->n, r->d, r->nnz, r->seed, r->tol, r->Q,
                              r->ldq, r->R, r->ldr, r->J, mode, base + r->ws_off, r->ws_bytes,
                              streams[slot], r->info, &rc);
    if (r->ph && rc == CQRRPT_OK) rc = cqh::phased_sketch(r->ph);
    if (rc == CQRRPT_OK && hipEventRecord(front_ev[slot], streams[slot]) != hipSuccess)
      rc = CQRRPT_EHIP;
    r->rc = rc;
    if (rc != CQRRPT_OK) {
      // Nothing (or not everything) was enqueued: finish at once.
      (void)hipStreamSynchronize(streams[slot]);
      if (r->ph) cqh::phased_end(r->ph);
      r->ph = nullptr;
      r->t_done = now_ms();
      r->state = 2;
      arena->release(r->ws_off, r->ws_bytes);
      continue;
    }
    r->state = 1;
    slot_req[slot] = r;
    ++running;
    live.push_back(r);
  }
  if (live.empty()) return;
  auto fail = [&](Request* r, int rc) {
    if (r->rc == CQRRPT_OK) r->rc = rc;
  };
  // QRCPs: the register-resident ones batched, the others on their own
  // streams.
  std::vector<cqh::QrcpBatchItem> qitems;
  for (Request* r : live) {
    if (!cqh::phased_batchable(r->ph)) continue;
    if (hipStreamWaitEvent(small, front_ev[r->slot], 0) != hipSuccess) fail(r, CQRRPT_EHIP);
    qitems.push_back(cqh::phased_qrcp_item(r->ph));
  }
  bool qok = true;
  if (!qitems.empty()) {
    qok = cqh::launch_qrcp_batch(qitems.data(), (int)qitems.size(), small) == hipSuccess &&
          hipEventRecord(small_ev, small) == hipSuccess;
  }
  for (Request* r : live) {
    hipStream_t st = streams[r->slot];
    int rc = CQRRPT_OK;
    if (cqh::phased_batchable(r->ph)) {
      if (!qok || hipStreamWaitEvent(st, small_ev, 0) != hipSuccess) rc = CQRRPT_EHIP;
      cqh::phased_mark(r->ph, 2);
    } else {
      rc = cqh::phased_qrcp(r->ph);
    }
    if (rc == CQRRPT_OK) rc = cqh::phased_tall(r->ph);
    if (rc == CQRRPT_OK && hipEventRecord(front_ev[r->slot], st) != hipSuccess) rc = CQRRPT_EHIP;
    if (rc != CQRRPT_OK) fail(r, rc);
  }
  // Cholesky steps, batched.
  std::vector<cqh::CholBatchItem> citems;
  for (Request* r : live) {
    if (hipStreamWaitEvent(small, front_ev[r->slot], 0) != hipSuccess) fail(r, CQRRPT_EHIP);
    citems.push_back(cqh::phased_chol_item(r->ph));
  }
  const bool cok = cqh::launch_cholesky_batch(citems.data(), (int)citems.size(), small) ==
                       hipSuccess &&
                   hipEventRecord(small_ev, small) == hipSuccess;
  for (Request* r : live) {
    const int slot = r->slot;
    hipStream_t st = streams[slot];
    int rc = CQRRPT_OK;
    if (!cok || hipStreamWaitEvent(st, small_ev, 0) != hipSuccess) rc = CQRRPT_EHIP;
    cqh::phased_mark(r->ph, 6);
    if (rc == CQRRPT_OK) rc = cqh::phased_tail(r->ph);
    if (rc != CQRRPT_OK) fail(r, rc);
    if (hipMemcpyAsync(&status_host[slot], &r->info->status, sizeof(int32_t),
                       hipMemcpyDeviceToHost, st) != hipSuccess)
      fail(r, CQRRPT_EHIP);
    if (hipEventRecord(done_ev[slot], st) != hipSuccess) {
      // The request cannot be tracked on the device: wait for it here.
      fail(r, CQRRPT_EHIP);
      (void)hipStreamSynchronize(st);
      (void)hipEventRecord(done_ev[slot], nullptr);
    }
    cqh::phased_end(r->ph);
    r->ph = nullptr;
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
  sv->streams.assign(max_slots, nullptr);
  sv->done_ev.assign(max_slots, nullptr);
  sv->front_ev.assign(max_slots, nullptr);
  sv->slot_req.assign(max_slots, nullptr);
  auto cleanup = [sv]() {
    for (size_t t = 0; t < sv->streams.size(); ++t) {
      if (sv->streams[t]) (void)hipStreamDestroy(sv->streams[t]);
      if (sv->done_ev[t]) (void)hipEventDestroy(sv->done_ev[t]);
      if (sv->front_ev[t]) (void)hipEventDestroy(sv->front_ev[t]);
    }
    if (sv->small) (void)hipStreamDestroy(sv->small);
    if (sv->small_ev) (void)hipEventDestroy(sv->small_ev);
    (void)hipFree(sv->base);
    (void)hipHostFree(sv->status_host);
    delete sv->arena;
    delete sv;
  };
  bool ok = hipStreamCreateWithFlags(&sv->small, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&sv->small_ev, hipEventDisableTiming) == hipSuccess;
  for (int s = 0; ok && s < max_slots; ++s)
    ok = hipStreamCreateWithFlags(&sv->streams[s], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&sv->done_ev[s], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sv->front_ev[s], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    cleanup();
    return nullptr;
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
  (void)hipStreamSynchronize(sv->small);
  for (size_t s = 0; s < sv->streams.size(); ++s) {
    (void)hipStreamSynchronize(sv->streams[s]);
    (void)hipStreamDestroy(sv->streams[s]);
    (void)hipEventDestroy(sv->done_ev[s]);
    (void)hipEventDestroy(sv->front_ev[s]);
  }
  (void)hipStreamDestroy(sv->small);
  (void)hipEventDestroy(sv->small_ev);
  (void)hipFree(sv->base);
  (void)hipHostFree(sv->status_host);
  for (auto& kv : sv->all) delete kv.second;
  delete sv->arena;
  delete sv;
}

}  // extern "C"
