// Continuous-batching server over the batched form (declared in
// include/soap_dp.h).  Every slot has its own worker thread, context,
// stream and pinned host staging.  A free slot's worker takes the requests
// that have arrived, in submission order, while the merged batch stays
// within the slot's limits and its device buffers fit the free part of the
// server's device memory (one arena shared by the batches in flight).  It
// uploads the batch into its arena region, enqueues the batched alignment
// and the result copies on its stream, waits for them, hands each request
// its slice and frees the region.  Slots work concurrently, so batches of
// different sizes overlap on the device and the host work of one slot
// (staging, result hand-off) overlaps the others.
//
// The slot contexts are reserved, warmed up and frozen at creation: while
// serving, no worker allocates or frees device memory, captures a graph or
// synchronises the whole device (each only waits for its own stream).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/soap_dp.h"
#include "batch.h"
#include "ctx_internal.h"
#include "serve_host.h"
#include "serve_rest.h"

using soapdp::serve::Arena;
using soapdp::serve::BatchLayout;
using soapdp::serve::Request;

namespace {

uint64_t now_ns() {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now().time_since_epoch())
                      .count());
}

struct TicketState {
  bool done = false;
  int rc = SOAP_DP_OK;
  uint64_t done_ns = 0;
};

template <class T>
bool halloc(T **p, size_t n) {
  return hipHostMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T),
                       hipHostMallocDefault) == hipSuccess;
}

// Device pointers of one batch inside the arena.
struct DeviceBatch {
  uint32_t *reads = nullptr;
  uint64_t *rwo = nullptr, *rbo = nullptr;
  int32_t *rl = nullptr, *ml = nullptr;
  int32_t *i32 = nullptr;   // score | begin | end | cigar_len, `tasks` each
  uint8_t *status = nullptr;
  uint32_t *cigar = nullptr, *head = nullptr, *rest = nullptr;
  int32_t *rest_hdr = nullptr;
  soapdp::RestRow *rest_rows = nullptr;
};

DeviceBatch carve(char *base, const BatchLayout &L) {
  DeviceBatch d;
  d.reads = reinterpret_cast<uint32_t *>(base + L.reads);
  d.rwo = reinterpret_cast<uint64_t *>(base + L.rwo);
  d.rbo = reinterpret_cast<uint64_t *>(base + L.rbo);
  d.rl = reinterpret_cast<int32_t *>(base + L.rl);
  d.ml = reinterpret_cast<int32_t *>(base + L.ml);
  d.i32 = reinterpret_cast<int32_t *>(base + L.i32);
  d.status = reinterpret_cast<uint8_t *>(base + L.status);
  d.cigar = reinterpret_cast<uint32_t *>(base + L.cigar);
  d.head = reinterpret_cast<uint32_t *>(base + L.head);
  d.rest_hdr = reinterpret_cast<int32_t *>(base + L.rest_hdr);
  d.rest_rows = reinterpret_cast<soapdp::RestRow *>(base + L.rest_rows);
  d.rest = reinterpret_cast<uint32_t *>(base + L.rest);
  return d;
}

struct Slot {
  soap_dp_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
  // pinned host staging, sized for the slot limits
  uint32_t *h_reads = nullptr;
  uint64_t *h_rwo = nullptr, *h_rbo = nullptr;
  int32_t *h_rl = nullptr, *h_ml = nullptr;
  int32_t *h_i32 = nullptr;              // 4 x max_tasks
  uint32_t *h_head = nullptr;            // max_tasks x kCigarHeadWords
  int32_t *h_rest_hdr = nullptr;         // 2
  soapdp::RestRow *h_rest_rows = nullptr;
  uint32_t *h_rest = nullptr;
  uint8_t *h_status = nullptr;
  // batch in flight
  std::vector<std::unique_ptr<Request>> reqs;
  std::vector<int32_t> first_task;
  int32_t tasks = 0;
  size_t region = 0;      // arena offset of the batch's device buffers
  BatchLayout layout{};
  DeviceBatch dev{};
};

constexpr int32_t kMaxRestRows = 1024, kMaxRestWords = 32768;   // batch_layout's caps

}  // namespace

struct soap_dp_server {
  soap_dp_server_config cfg{};
  int32_t stride = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Request>> queue;
  std::unordered_map<uint64_t, TicketState> tickets;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::vector<std::thread> workers;
  soap_dp_server_stats stats{};
  int fatal = SOAP_DP_OK;
  char *arena_base = nullptr;   // device memory of the batches in flight
  Arena arena;
};

namespace {

void free_slot(Slot &s) {
  if (s.ctx) soap_dp_destroy(s.ctx);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.start) (void)hipEventDestroy(s.start);
  if (s.done) (void)hipEventDestroy(s.done);
  for (void *p : {(void *)s.h_reads, (void *)s.h_rwo, (void *)s.h_rbo, (void *)s.h_rl, (void *)s.h_ml,
                  (void *)s.h_i32, (void *)s.h_head, (void *)s.h_rest_hdr, (void *)s.h_rest_rows,
                  (void *)s.h_rest, (void *)s.h_status})
    if (p) (void)hipHostFree(p);
  s = Slot{};
}

int init_slot(soap_dp_server *srv, Slot &s) {
  const auto &c = srv->cfg;
  const size_t T = size_t(c.max_tasks), Wd = size_t(c.max_read_words);
  int rc = soap_dp_create(&s.ctx, c.device_ordinal);
  if (rc) return rc;
  if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s.start, hipEventDefault) != hipSuccess ||
      hipEventCreateWithFlags(&s.done, hipEventDefault) != hipSuccess)
    return SOAP_DP_EHIP;
  const bool ok = halloc(&s.h_reads, Wd) && halloc(&s.h_rwo, T) && halloc(&s.h_rbo, T) &&
                  halloc(&s.h_rl, T) && halloc(&s.h_ml, T) && halloc(&s.h_i32, 4 * T) &&
                  halloc(&s.h_head, T * soapdp::kCigarHeadWords) && halloc(&s.h_rest_hdr, 2) &&
                  halloc(&s.h_rest_rows, size_t(kMaxRestRows)) &&
                  halloc(&s.h_rest, size_t(kMaxRestWords)) && halloc(&s.h_status, T);
  if (!ok) {
    (void)hipGetLastError();
    return SOAP_DP_ENOMEM;
  }
  return SOAP_DP_OK;
}

// Enqueue the batch `s.reqs` (already merged into the staging arrays, nt
// tasks, nw read words) in its arena region: uploads, the batched form,
// the CIGAR head gather and rest packing, and the copies back.
int enqueue_batch(soap_dp_server *srv, Slot &s, int32_t nt, uint64_t nw) {
  const auto &c = srv->cfg;
  const int32_t C = c.max_tasks, S = srv->stride;
  const DeviceBatch &d = s.dev;
  const BatchLayout &L = s.layout;
  hipStream_t st = s.stream;
  bool ok = hipEventRecord(s.start, st) == hipSuccess &&
            hipMemcpyAsync(d.reads, s.h_reads, std::max<uint64_t>(nw, 1) * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(d.rwo, s.h_rwo, size_t(nt) * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(d.rbo, s.h_rbo, size_t(nt) * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(d.rl, s.h_rl, size_t(nt) * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(d.ml, s.h_ml, size_t(nt) * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  if (!ok) return SOAP_DP_EHIP;
  soap_dp_batch in{};
  in.read_codes = d.reads;
  in.read_word_off = d.rwo;
  in.read_len = d.rl;
  in.ref_codes = c.genome;
  in.ref_base_off = d.rbo;
  in.ref_len = d.ml;
  in.n_tasks = nt;
  in.max_n = c.max_n;
  in.max_m = c.max_m;
  in.read_words = std::max<uint64_t>(nw, 1);
  in.ref_words = c.genome_words;
  soap_dp_result out{};
  out.score = d.i32;
  out.ref_begin = d.i32 + nt;
  out.ref_end = d.i32 + 2 * size_t(nt);
  out.cigar_len = d.i32 + 3 * size_t(nt);
  out.cigar = d.cigar;
  out.cigar_stride = S;
  out.status = d.status;
  const int rc = soap_dp_align_batch(s.ctx, &in, &c.scoring, &out, st, SOAP_DP_BATCHED | c.align_flags);
  if (rc) return rc;
  ok = soapdp::launch_gather_cigar_head(d.cigar, S, out.cigar_len, nt, d.head, st) == hipSuccess &&
       soapdp::launch_pack_cigar_rest(d.cigar, S, out.cigar_len, nt, soapdp::kCigarHeadWords,
                                      d.rest_hdr, d.rest_rows, L.rest_rows_cap, d.rest,
                                      L.rest_words_cap, st) == hipSuccess;
  for (int a = 0; ok && a < 4; ++a)
    ok = hipMemcpyAsync(s.h_i32 + size_t(a) * C, d.i32 + size_t(a) * nt, size_t(nt) * 4,
                        hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok &&
       hipMemcpyAsync(s.h_status, d.status, size_t(nt), hipMemcpyDeviceToHost, st) == hipSuccess &&
       hipMemcpyAsync(s.h_head, d.head, size_t(nt) * soapdp::kCigarHeadWords * 4,
                      hipMemcpyDeviceToHost, st) == hipSuccess &&
       hipMemcpyAsync(s.h_rest_hdr, d.rest_hdr, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                      st) == hipSuccess &&
       hipMemcpyAsync(s.h_rest_rows, d.rest_rows, size_t(L.rest_rows_cap) * sizeof(soapdp::RestRow),
                      hipMemcpyDeviceToHost, st) == hipSuccess &&
       hipMemcpyAsync(s.h_rest, d.rest, size_t(L.rest_words_cap) * 4, hipMemcpyDeviceToHost,
                      st) == hipSuccess &&
       hipEventRecord(s.done, st) == hipSuccess;
  return ok ? SOAP_DP_OK : SOAP_DP_EHIP;
}

// Merge the taken requests into the slot's staging and enqueue the batch.
int launch(soap_dp_server *srv, Slot &s) {
  uint64_t nw = 0;
  const soapdp::serve::Staging st{s.h_reads, s.h_rwo, s.h_rbo, s.h_rl, s.h_ml};
  const int32_t nt = soapdp::serve::merge(s.reqs, srv->cfg.max_n, st, s.first_task, &nw);
  s.tasks = nt;
  s.dev = carve(srv->arena_base + s.region, s.layout);
  const int rc = enqueue_batch(srv, s, nt, nw);
  const uint64_t t = now_ns();
  for (auto &q : s.reqs) q->launched_ns = t;
  return rc;
}

// Finished batch: copy each request's slice to its caller buffers, then
// free the batch's device region.  The rests of long CIGAR rows come from
// the area packed on the device; a row that did not fit it is fetched on
// the slot's own stream.
void retire(soap_dp_server *srv, Slot &s) {
  const int32_t listed = std::max(0, std::min(s.h_rest_hdr[0], s.layout.rest_rows_cap));
  std::sort(s.h_rest_rows, s.h_rest_rows + listed,
            [](const soapdp::RestRow &a, const soapdp::RestRow &b) { return a.task < b.task; });
  const soapdp::serve::BatchHost b{srv->cfg.max_tasks, srv->stride, s.h_i32, s.h_status, s.h_head,
                                   s.h_rest_rows, listed, s.h_rest, s.layout.rest_words_cap};
  struct Finished {
    uint64_t ticket;
    int rc;
    uint64_t done_ns;   // when the request's results were all in its buffers
  };
  std::vector<Finished> finished;
  std::vector<soapdp::serve::Fetch> fetch;
  for (size_t r = 0; r < s.reqs.size(); ++r) {
    Request &q = *s.reqs[r];
    fetch.clear();
    int rc = soapdp::serve::hand_off(b, s.first_task[r], q, fetch);
    bool ok = true;
    for (const auto &f : fetch)
      ok = ok && hipMemcpyAsync(f.dst, s.dev.cigar + int64_t(f.task) * srv->stride +
                                           soapdp::kCigarHeadWords,
                                size_t(f.words) * 4, hipMemcpyDeviceToHost, s.stream) == hipSuccess;
    if (!fetch.empty()) ok = ok && hipStreamSynchronize(s.stream) == hipSuccess;
    if (!ok) rc = SOAP_DP_EHIP;
    const uint64_t t = now_ns();
    if (q.stamps) *q.stamps = soap_dp_request_stamps{q.arrival_ns, q.taken_ns, q.launched_ns,
                                                     q.device_ns, t};
    finished.push_back(Finished{q.ticket, rc, t});
  }
  // device time of the batch, for the stats only
  float ms = 0;
  (void)hipEventElapsedTime(&ms, s.start, s.done);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (const Finished &fq : finished) {
      TicketState &ts = srv->tickets[fq.ticket];
      ts.done = true;
      ts.rc = fq.rc;
      ts.done_ns = fq.done_ns;
    }
    srv->stats.completed += finished.size();
    srv->stats.batches += 1;
    srv->stats.tasks += uint64_t(s.tasks);
    for (auto &q : s.reqs) srv->stats.cells += uint64_t(q->cells);
    srv->stats.device_busy_s += double(ms) * 1e-3;
    srv->arena.release(s.region);
  }
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();   // device memory was freed
  s.reqs.clear();
  s.first_task.clear();
  s.tasks = 0;
}

// Fail a slot's requests with `rc` (its batch could not be run).
void fail_batch(soap_dp_server *srv, Slot &s, int rc) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->fatal = rc;
    for (auto &q : s.reqs) {
      TicketState &ts = srv->tickets[q->ticket];
      ts.done = true;
      ts.rc = rc;
      ts.done_ns = now_ns();
    }
    srv->stats.completed += s.reqs.size();
    srv->arena.release(s.region);
  }
  s.reqs.clear();
  s.first_task.clear();
  s.tasks = 0;
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();
}

void slot_worker(soap_dp_server *srv, size_t k) {
  (void)hipSetDevice(srv->cfg.device_ordinal);
  Slot &s = srv->slots[k];
  const soapdp::serve::Limits lim{srv->cfg.max_tasks, uint64_t(srv->cfg.max_read_words),
                                  srv->stride};
  constexpr uint64_t kSpin = 200000;   // ns: poll closely when an arrival is this near
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      for (;;) {
        if (srv->queue.empty()) {
          if (srv->stopping) return;
          srv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
          continue;
        }
        const uint64_t now = now_ns(), next = srv->queue.front()->arrival_ns;
        if (next > now) {
          if (next > now + kSpin) {
            srv->cv_work.wait_for(lk, std::chrono::nanoseconds(next - now - kSpin / 2));
          } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
          }
          continue;
        }
        if (soapdp::serve::take_arrived(srv->queue, now, lim, srv->arena, s.reqs, &s.region,
                                        &s.layout))
          break;
        // the head has arrived but its batch does not fit the free device
        // memory: wait for a batch in flight to retire
        srv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
      }
      srv->stats.device_bytes_peak = srv->arena.peak();
    }
    uint64_t t0 = now_ns();
    for (auto &q : s.reqs) q->taken_ns = t0;
    const int rc = launch(srv, s);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->stats.host_launch_s += double(now_ns() - t0) * 1e-9;
    }
    if (rc) {
      fail_batch(srv, s, rc);
      continue;
    }
    // another request may have arrived meanwhile: let a free slot take it
    srv->cv_work.notify_one();
    if (hipEventSynchronize(s.done) != hipSuccess) {
      fail_batch(srv, s, SOAP_DP_EHIP);
      continue;
    }
    t0 = now_ns();
    for (auto &q : s.reqs) q->device_ns = t0;
    retire(srv, s);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->stats.host_retire_s += double(now_ns() - t0) * 1e-9;
    }
  }
}

// The first large host<->device copies on a stream cost milliseconds once
// (the copy path is set up on first use); a served batch should not pay
// that.  Move every staging buffer to and from the device once at its full
// size (or the largest batch the device budget holds), on the slot's stream.
int warm_copies(soap_dp_server *srv, Slot &s) {
  int64_t tasks = srv->cfg.max_tasks;
  uint64_t words = uint64_t(srv->cfg.max_read_words);
  size_t region = 0;
  soapdp::serve::BatchLayout L = soapdp::serve::batch_layout(tasks, words, srv->stride);
  while (!srv->arena.alloc(L.bytes, &region)) {
    if (tasks == 1 && words == 1) return SOAP_DP_OK;   // the budget holds only tiny batches
    tasks = std::max<int64_t>(1, tasks / 2);
    words = std::max<uint64_t>(1, words / 2);
    L = soapdp::serve::batch_layout(tasks, words, srv->stride);
  }
  const DeviceBatch d = carve(srv->arena_base + region, L);
  const size_t T = size_t(tasks);
  hipStream_t st = s.stream;
  const bool ok =
      hipMemcpyAsync(d.reads, s.h_reads, words * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
      hipMemcpyAsync(d.rwo, s.h_rwo, T * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
      hipMemcpyAsync(d.rbo, s.h_rbo, T * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
      hipMemcpyAsync(d.rl, s.h_rl, T * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
      hipMemcpyAsync(d.ml, s.h_ml, T * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
      hipMemcpyAsync(s.h_i32, d.i32, 4 * T * 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
      hipMemcpyAsync(s.h_status, d.status, T, hipMemcpyDeviceToHost, st) == hipSuccess &&
      hipMemcpyAsync(s.h_head, d.head, T * soapdp::kCigarHeadWords * 4, hipMemcpyDeviceToHost,
                     st) == hipSuccess &&
      hipMemcpyAsync(s.h_rest, d.rest, size_t(L.rest_words_cap) * 4, hipMemcpyDeviceToHost,
                     st) == hipSuccess &&
      hipStreamSynchronize(st) == hipSuccess;
  srv->arena.release(region);
  return ok ? SOAP_DP_OK : SOAP_DP_EHIP;
}

// Run one batch of a single empty read through a slot at creation, before
// the workers start: every kernel a batch launches is loaded, and the
// context's stream set is made, on the creating thread.
int warm_up(soap_dp_server *srv, Slot &s) {
  auto q = std::make_unique<Request>();
  q->n_tasks = 1;
  q->reads.assign(1, 0u);
  q->rwo.assign(1, 0);
  q->rl.assign(1, 0);   // empty read: the kernels report INVALID_LEN
  q->rbo.assign(1, 0);
  q->ml.assign(1, 1);
  std::vector<std::unique_ptr<Request>> one;
  one.push_back(std::move(q));
  s.layout = soapdp::serve::batch_layout(1, 1, srv->stride);
  if (!srv->arena.alloc(s.layout.bytes, &s.region)) return SOAP_DP_E2BIG;
  s.reqs = std::move(one);
  int rc = launch(srv, s);
  if (!rc && hipStreamSynchronize(s.stream) != hipSuccess) rc = SOAP_DP_EHIP;
  if (!rc && s.h_status[0] != SOAP_DP_TASK_INVALID_LEN) rc = SOAP_DP_EHIP;
  srv->arena.release(s.region);
  s.reqs.clear();
  s.first_task.clear();
  if (!rc) rc = warm_copies(srv, s);
  return rc;
}

void destroy_all(soap_dp_server *srv) {
  for (auto &s : srv->slots) free_slot(s);
  if (srv->arena_base) (void)hipFree(srv->arena_base);
  delete srv;
}

}  // namespace

extern "C" {

uint64_t soap_dp_now_ns(void) { return now_ns(); }

constexpr int kMaxSlots = 8;

int soap_dp_server_create(soap_dp_server **out, const soap_dp_server_config *cfg) {
  if (!out || !cfg) return SOAP_DP_EINVAL;
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > kMaxSlots || cfg->max_tasks < 1 || cfg->max_read_words < 1 ||
      cfg->max_n < 1 || cfg->max_n > SOAP_DP_MAX_READ || cfg->max_m < 1 ||
      cfg->max_m > SOAP_DP_MAX_WINDOW || !cfg->genome || cfg->genome_words == 0 ||
      (cfg->align_flags & ~SOAP_DP_FULL_WINDOW) != 0)
    return SOAP_DP_EINVAL;
  auto *srv = new (std::nothrow) soap_dp_server();
  if (!srv) return SOAP_DP_ENOMEM;
  srv->cfg = *cfg;
  srv->stride = 2 * cfg->max_n - 1;
  const size_t full =
      soapdp::serve::batch_layout(cfg->max_tasks, uint64_t(cfg->max_read_words), srv->stride).bytes;
  const size_t budget = cfg->device_bytes ? size_t(cfg->device_bytes) : size_t(cfg->n_slots) * full;
  if (budget < soapdp::serve::batch_layout(1, 1, srv->stride).bytes) {
    delete srv;
    return SOAP_DP_E2BIG;
  }
  (void)hipSetDevice(cfg->device_ordinal);
  if (hipMalloc(reinterpret_cast<void **>(&srv->arena_base), budget) != hipSuccess) {
    (void)hipGetLastError();
    delete srv;
    return SOAP_DP_ENOMEM;
  }
  srv->arena = Arena(budget);
  srv->stats.device_bytes = srv->arena.capacity();
  srv->slots.resize(size_t(cfg->n_slots));
  int rc = SOAP_DP_OK;
  for (auto &s : srv->slots) {
    rc = init_slot(srv, s);
    if (rc) break;
  }
  // shapes first (autotuned on one slot, copied to the others), then every
  // workspace is reserved for those shapes, then each slot runs one batch
  if (!rc && cfg->autotune) {
    rc = soap_dp_autotune(srv->slots[0].ctx, nullptr, 1);
    if (!rc) {
      soap_dp_class_info info[64];
      const int n = soap_dp_get_classes(srv->slots[0].ctx, info, 64);
      for (size_t k = 1; k < srv->slots.size() && !rc; ++k)
        for (int q = 0; q < n && !rc; ++q)
          rc = soap_dp_set_class_shape(srv->slots[k].ctx, info[q].precision, info[q].capacity,
                                       info[q].lanes, info[q].cells);
    }
  }
  for (size_t k = 0; k < srv->slots.size() && !rc; ++k)
    rc = soapdp::ctx_reserve_for(srv->slots[k].ctx, cfg->max_tasks, cfg->max_n, cfg->max_m,
                                 SOAP_DP_BATCHED | cfg->align_flags, &cfg->scoring);
  for (size_t k = 0; k < srv->slots.size() && !rc; ++k) {
    soapdp::ctx_set_frozen(srv->slots[k].ctx, true);
    rc = warm_up(srv, srv->slots[k]);
  }
  if (rc) {
    destroy_all(srv);
    return rc;
  }
  for (size_t k = 0; k < srv->slots.size(); ++k) srv->workers.emplace_back(slot_worker, srv, k);
  *out = srv;
  return SOAP_DP_OK;
}

int soap_dp_server_submit(soap_dp_server *srv, const soap_dp_request *req, uint64_t *ticket) {
  if (!srv || !req || !ticket || req->n_tasks < 1) return SOAP_DP_EINVAL;
  const auto &c = srv->cfg;
  if (!req->read_codes || !req->read_word_off || !req->read_len || !req->ref_base_off ||
      !req->ref_len || !req->out.score || !req->out.ref_begin || !req->out.ref_end ||
      !req->out.cigar || !req->out.cigar_len || !req->out.status || req->out.cigar_capacity < 0)
    return SOAP_DP_EINVAL;
  if (req->n_tasks > c.max_tasks || req->read_words > uint64_t(c.max_read_words) ||
      soapdp::serve::batch_layout(req->n_tasks, req->read_words, srv->stride).bytes >
          srv->arena.capacity()) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.rejected += 1;
    return SOAP_DP_E2BIG;
  }
  auto q = std::make_unique<Request>();
  const size_t n = size_t(req->n_tasks);
  q->n_tasks = req->n_tasks;
  q->reads.assign(req->read_codes, req->read_codes + req->read_words);
  q->rwo.assign(req->read_word_off, req->read_word_off + n);
  q->rl.assign(req->read_len, req->read_len + n);
  q->rbo.assign(req->ref_base_off, req->ref_base_off + n);
  q->ml.assign(req->ref_len, req->ref_len + n);
  q->out = req->out;
  q->stamps = req->stamps;
  q->arrival_ns = req->arrival_ns ? req->arrival_ns : now_ns();
  for (size_t t = 0; t < n; ++t) q->cells += int64_t(q->rl[t]) * int64_t(q->ml[t]);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return SOAP_DP_ESTOPPED;
    if (srv->fatal) return srv->fatal;
    q->ticket = srv->next_ticket++;
    *ticket = q->ticket;
    srv->tickets[q->ticket] = TicketState{};
    srv->queue.push_back(std::move(q));
    srv->stats.submitted += 1;
  }
  srv->cv_work.notify_one();
  return SOAP_DP_OK;
}

int soap_dp_server_poll(soap_dp_server *srv, uint64_t ticket) {
  if (!srv) return SOAP_DP_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return SOAP_DP_EINVAL;
  if (!it->second.done) return 0;
  return it->second.rc ? it->second.rc : 1;
}

int soap_dp_server_wait(soap_dp_server *srv, uint64_t ticket, uint64_t *done_ns) {
  if (!srv) return SOAP_DP_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return SOAP_DP_EINVAL;
  srv->cv_done.wait(lk, [&] { return srv->tickets[ticket].done; });
  const TicketState ts = srv->tickets[ticket];
  srv->tickets.erase(ticket);
  if (done_ns) *done_ns = ts.done_ns;
  return ts.rc;
}

int soap_dp_server_drain(soap_dp_server *srv) {
  if (!srv) return SOAP_DP_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->stats.completed + 0 >= srv->stats.submitted || srv->fatal; });
  return srv->fatal;
}

int soap_dp_server_stats_get(soap_dp_server *srv, soap_dp_server_stats *out) {
  if (!srv || !out) return SOAP_DP_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  out->device_bytes_peak = srv->arena.peak();
  return SOAP_DP_OK;
}

int soap_dp_server_destroy(soap_dp_server *srv) {
  if (!srv) return SOAP_DP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  for (auto &w : srv->workers)
    if (w.joinable()) w.join();
  (void)hipSetDevice(srv->cfg.device_ordinal);
  for (auto &s : srv->slots)
    if (s.stream) (void)hipStreamSynchronize(s.stream);
  destroy_all(srv);
  return SOAP_DP_OK;
}

}  // extern "C"
