// Continuous-batching server over the batched form (declared in
// include/soap_dp.h).  Every slot has its own worker thread, context,
// stream and buffers.  A worker takes the requests that have arrived, in
// submission order, up to its slot's capacity, merges them into one batch,
// uploads it, enqueues the batched alignment and the result copies on its
// stream, waits for them and hands each request its slice of the results.
// Slots work concurrently, so batches overlap on the device and the host
// work of one slot (staging, result hand-off) overlaps the others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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
#include "serve_rest.h"

namespace {


uint64_t now_ns() {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now().time_since_epoch())
                      .count());
}

struct Request {
  uint64_t ticket = 0;
  int32_t n_tasks = 0;
  std::vector<uint32_t> reads;
  std::vector<uint64_t> rwo;
  std::vector<int32_t> rl, ml;
  std::vector<uint64_t> rbo;
  soap_dp_host_result out{};
  uint64_t arrival_ns = 0;
  int64_t cells = 0;
};

struct TicketState {
  bool done = false;
  int rc = SOAP_DP_OK;
  uint64_t done_ns = 0;
};

template <class T>
bool dalloc(T **p, size_t n) {
  return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T)) == hipSuccess;
}
template <class T>
bool halloc(T **p, size_t n) {
  return hipHostMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T),
                       hipHostMallocDefault) == hipSuccess;
}

struct Slot {
  soap_dp_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
  // device inputs and outputs
  uint32_t *d_reads = nullptr;
  uint64_t *d_rwo = nullptr, *d_rbo = nullptr;
  int32_t *d_rl = nullptr, *d_ml = nullptr;
  int32_t *d_i32 = nullptr;   // score | begin | end | cigar_len
  uint32_t *d_cigar = nullptr;
  uint32_t *d_head = nullptr;     // first CIGAR words of every task (dense)
  uint8_t *d_status = nullptr;
  // rests of the rows longer than the head, packed on the device
  int32_t rest_rows = 0, rest_words = 0;   // capacities
  int32_t batch_rest_rows = 0, batch_rest_words = 0;   // the part the batch in flight uses
  int32_t *d_rest_hdr = nullptr;
  soapdp::RestRow *d_rest_rows = nullptr;
  uint32_t *d_rest = nullptr;
  // pinned host staging
  uint32_t *h_reads = nullptr;
  uint64_t *h_rwo = nullptr, *h_rbo = nullptr;
  int32_t *h_rl = nullptr, *h_ml = nullptr;
  int32_t *h_i32 = nullptr;
  uint32_t *h_head = nullptr;     // copy of d_head
  int32_t *h_rest_hdr = nullptr;  // copies of d_rest_hdr, d_rest_rows, d_rest
  soapdp::RestRow *h_rest_rows = nullptr;
  uint32_t *h_rest = nullptr;
  uint8_t *h_status = nullptr;
  // batch in flight
  bool busy = false;
  std::vector<std::unique_ptr<Request>> reqs;
  std::vector<int32_t> first_task;
  int32_t tasks = 0;
};

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
};

namespace {

void free_slot(Slot &s) {
  if (s.ctx) soap_dp_destroy(s.ctx);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.start) (void)hipEventDestroy(s.start);
  if (s.done) (void)hipEventDestroy(s.done);
  for (void *p : {(void *)s.d_reads, (void *)s.d_rwo, (void *)s.d_rbo, (void *)s.d_rl, (void *)s.d_ml,
                  (void *)s.d_i32, (void *)s.d_cigar, (void *)s.d_status, (void *)s.d_head,
                  (void *)s.d_rest_hdr, (void *)s.d_rest_rows, (void *)s.d_rest})
    if (p) (void)hipFree(p);
  for (void *p : {(void *)s.h_reads, (void *)s.h_rwo, (void *)s.h_rbo, (void *)s.h_rl, (void *)s.h_ml,
                  (void *)s.h_i32, (void *)s.h_head, (void *)s.h_rest_hdr, (void *)s.h_rest_rows,
                  (void *)s.h_rest, (void *)s.h_status})
    if (p) (void)hipHostFree(p);
  s = Slot{};
}

int init_slot(soap_dp_server *srv, Slot &s) {
  const auto &c = srv->cfg;
  const size_t T = size_t(c.max_tasks), Wd = size_t(c.max_read_words), S = size_t(srv->stride);
  int rc = soap_dp_create(&s.ctx, c.device_ordinal);
  if (rc) return rc;
  if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s.start, hipEventDefault) != hipSuccess ||
      hipEventCreateWithFlags(&s.done, hipEventDefault) != hipSuccess)
    return SOAP_DP_EHIP;
  // room for the rests of up to 1,024 long rows per batch (fewer for small
  // slots), 128 KB of words
  s.rest_rows = int32_t(std::min<size_t>(T, 1024));
  s.rest_words = int32_t(std::min<size_t>(T * soapdp::kCigarHeadWords, 32768));
  const bool ok = dalloc(&s.d_reads, Wd) && dalloc(&s.d_rwo, T) && dalloc(&s.d_rbo, T) &&
                  dalloc(&s.d_rl, T) && dalloc(&s.d_ml, T) && dalloc(&s.d_i32, 4 * T) &&
                  dalloc(&s.d_cigar, T * S) && dalloc(&s.d_status, T) &&
                  dalloc(&s.d_head, T * soapdp::kCigarHeadWords) &&
                  dalloc(&s.d_rest_hdr, 2) && dalloc(&s.d_rest_rows, size_t(s.rest_rows)) &&
                  dalloc(&s.d_rest, size_t(s.rest_words)) &&
                  halloc(&s.h_reads, Wd) && halloc(&s.h_rwo, T) && halloc(&s.h_rbo, T) &&
                  halloc(&s.h_rl, T) && halloc(&s.h_ml, T) && halloc(&s.h_i32, 4 * T) &&
                  halloc(&s.h_head, T * soapdp::kCigarHeadWords) &&
                  halloc(&s.h_rest_hdr, 2) && halloc(&s.h_rest_rows, size_t(s.rest_rows)) &&
                  halloc(&s.h_rest, size_t(s.rest_words)) &&
                  halloc(&s.h_status, T);
  if (!ok) {
    (void)hipGetLastError();
    return SOAP_DP_ENOMEM;
  }
  return soap_dp_reserve(s.ctx, c.max_tasks, c.max_n, c.max_m, SOAP_DP_BATCHED);
}

// Finished batch: copy each request's slice to its caller buffers.  CIGARs
// come from the dense head copy; the rests of the rare longer rows were
// packed on the device and came back with the batch.  A long row that did
// not fit that area is fetched on its own, with a synchronous copy.
void retire(soap_dp_server *srv, Slot &s) {
  const int32_t T = srv->cfg.max_tasks;
  const int32_t S = srv->stride;
  constexpr int32_t H = soapdp::kCigarHeadWords;
  std::unordered_map<int32_t, int32_t> rest_at;   // task -> offset in h_rest
  const int32_t listed = std::min(s.h_rest_hdr[0], s.batch_rest_rows);
  for (int32_t k = 0; k < listed; ++k)
    if (s.h_rest_rows[k].off >= 0) rest_at.emplace(s.h_rest_rows[k].task, s.h_rest_rows[k].off);
  struct Finished {
    uint64_t ticket;
    int rc;
    uint64_t done_ns;   // when the request's results were all in its buffers
  };
  std::vector<Finished> finished;
  for (size_t r = 0; r < s.reqs.size(); ++r) {
    Request &q = *s.reqs[r];
    const int32_t f = s.first_task[r], n = q.n_tasks;
    const soap_dp_host_result &o = q.out;
    std::memcpy(o.score, s.h_i32 + f, size_t(n) * 4);
    std::memcpy(o.ref_begin, s.h_i32 + T + f, size_t(n) * 4);
    std::memcpy(o.ref_end, s.h_i32 + 2 * T + f, size_t(n) * 4);
    std::memcpy(o.cigar_len, s.h_i32 + 3 * T + f, size_t(n) * 4);
    std::memcpy(o.status, s.h_status + f, size_t(n));
    int64_t words = 0;
    int rc = SOAP_DP_OK;
    const int32_t *lens = s.h_i32 + 3 * T + f;
    const uint32_t *head = s.h_head + int64_t(f) * H;
    int64_t total = 0;
    for (int32_t t = 0; t < n; ++t) total += std::min(std::max(lens[t], 0), S);
    // A row whose full head (H words) ends within the request's packed
    // CIGARs is copied whole, with no length-dependent branch; the words
    // past the row are rewritten by the rows after it, which are copied
    // later.  Other rows, and every row of a request that does not fit its
    // buffer, are copied word by word up to their length.
    const bool whole = total <= o.cigar_capacity;
    for (int32_t t = 0; t < n; ++t) {
      const int32_t len = std::min(std::max(lens[t], 0), S);
      if (words + len > o.cigar_capacity) {
        rc = SOAP_DP_E2BIG;   // keeps counting; writes nothing past the buffer
      } else {
        uint32_t *dst = o.cigar + words;
        const uint32_t *src = head + int64_t(t) * H;
        if (whole && words + H <= total) {
          std::memcpy(dst, src, sizeof(uint32_t) * H);
        } else {
          const int32_t hn = std::min(len, H);
          for (int32_t k = 0; k < hn; ++k) dst[k] = src[k];
        }
        if (len > H) {
          auto it = rest_at.find(f + t);
          uint32_t *rdst = dst + H;
          if (it != rest_at.end())
            std::memcpy(rdst, s.h_rest + it->second, size_t(len - H) * 4);
          else if (hipMemcpy(rdst, s.d_cigar + int64_t(f + t) * S + H, size_t(len - H) * 4,
                             hipMemcpyDeviceToHost) != hipSuccess)
            rc = SOAP_DP_EHIP;
        }
      }
      words += len;
    }
    finished.push_back(Finished{q.ticket, rc, now_ns()});
  }
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
  }
  srv->cv_done.notify_all();
  // device time of the batch, for the stats only: taken after the results
  // are handed over (the runtime call can wait on other threads' calls)
  float ms = 0;
  (void)hipEventElapsedTime(&ms, s.start, s.done);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.device_busy_s += double(ms) * 1e-3;
  }
  s.reqs.clear();
  s.first_task.clear();
  s.tasks = 0;
  s.busy = false;
}

// Merge queued requests (FIFO) into the free slot and launch the batch.
int launch(soap_dp_server *srv, Slot &s, std::vector<std::unique_ptr<Request>> &take) {
  const auto &c = srv->cfg;
  const int32_t T = c.max_tasks, S = srv->stride;
  int32_t nt = 0;
  uint64_t nw = 0;
  for (auto &q : take) {
    s.first_task.push_back(nt);
    std::memcpy(s.h_reads + nw, q->reads.data(), q->reads.size() * 4);
    for (int32_t t = 0; t < q->n_tasks; ++t) {
      s.h_rwo[nt + t] = q->rwo[size_t(t)] + nw;
      s.h_rl[nt + t] = q->rl[size_t(t)];
      s.h_rbo[nt + t] = q->rbo[size_t(t)];
      s.h_ml[nt + t] = q->ml[size_t(t)];
    }
    nt += q->n_tasks;
    nw += q->reads.size();
    s.reqs.push_back(std::move(q));
  }
  take.clear();
  s.tasks = nt;
  // Every batch of a slot has the slot's full capacity: the tail past the
  // merged requests holds zero-length reads, which the bucketing marks
  // invalid and skips.  The call is then identical from batch to batch
  // (same buffers, same sizes), so the slot's graph is captured once and
  // replayed.
  std::memset(s.h_rl + nt, 0, size_t(T - nt) * 4);
  hipStream_t st = s.stream;
  bool ok = hipEventRecord(s.start, st) == hipSuccess &&
            hipMemcpyAsync(s.d_reads, s.h_reads, std::max<uint64_t>(nw, 1) * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(s.d_rwo, s.h_rwo, size_t(nt) * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(s.d_rbo, s.h_rbo, size_t(nt) * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(s.d_rl, s.h_rl, size_t(T) * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(s.d_ml, s.h_ml, size_t(nt) * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  if (!ok) return SOAP_DP_EHIP;
  soap_dp_batch in{};
  in.read_codes = s.d_reads;
  in.read_word_off = s.d_rwo;
  in.read_len = s.d_rl;
  in.ref_codes = c.genome;
  in.ref_base_off = s.d_rbo;
  in.ref_len = s.d_ml;
  in.n_tasks = T;
  in.max_n = c.max_n;
  in.max_m = c.max_m;
  in.read_words = uint64_t(c.max_read_words);
  in.ref_words = c.genome_words;
  soap_dp_result out{};
  out.score = s.d_i32;
  out.ref_begin = s.d_i32 + T;
  out.ref_end = s.d_i32 + 2 * T;
  out.cigar_len = s.d_i32 + 3 * T;
  out.cigar = s.d_cigar;
  out.cigar_stride = S;
  out.status = s.d_status;
  const int rc = soap_dp_align_batch(s.ctx, &in, &c.scoring, &out, st, SOAP_DP_BATCHED);
  if (rc) return rc;
  // the rest area this batch may use, and copy back, grows with its tasks
  s.batch_rest_rows = std::min(s.rest_rows, std::max(16, nt / 64));
  s.batch_rest_words = std::min(s.rest_words, std::max(512, nt / 4));
  ok = soapdp::launch_gather_cigar_head(s.d_cigar, S, s.d_i32 + 3 * T, nt, s.d_head, st) == hipSuccess &&
       soapdp::launch_pack_cigar_rest(s.d_cigar, S, s.d_i32 + 3 * T, nt, soapdp::kCigarHeadWords,
                                      s.d_rest_hdr, s.d_rest_rows, s.batch_rest_rows, s.d_rest,
                                      s.batch_rest_words, st) == hipSuccess;
  for (int a = 0; ok && a < 4; ++a)
    ok = hipMemcpyAsync(s.h_i32 + size_t(a) * T, s.d_i32 + size_t(a) * T, size_t(nt) * 4,
                        hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok &&
       hipMemcpyAsync(s.h_status, s.d_status, size_t(nt), hipMemcpyDeviceToHost, st) == hipSuccess &&
       hipMemcpyAsync(s.h_head, s.d_head, size_t(nt) * soapdp::kCigarHeadWords * 4,
                      hipMemcpyDeviceToHost, st) == hipSuccess &&
       hipMemcpyAsync(s.h_rest_hdr, s.d_rest_hdr, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                      st) == hipSuccess &&
       hipMemcpyAsync(s.h_rest_rows, s.d_rest_rows,
                      size_t(s.batch_rest_rows) * sizeof(soapdp::RestRow), hipMemcpyDeviceToHost,
                      st) == hipSuccess &&
       hipMemcpyAsync(s.h_rest, s.d_rest, size_t(s.batch_rest_words) * 4, hipMemcpyDeviceToHost,
                      st) == hipSuccess &&
       hipEventRecord(s.done, st) == hipSuccess;
  if (!ok) return SOAP_DP_EHIP;
  s.busy = true;
  return SOAP_DP_OK;
}

// Fail a slot's requests with `rc` (its batch could not be run).
void fail_batch(soap_dp_server *srv, Slot &s, int rc) {
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->fatal = rc;
  for (auto &q : s.reqs) {
    TicketState &ts = srv->tickets[q->ticket];
    ts.done = true;
    ts.rc = rc;
    ts.done_ns = now_ns();
  }
  srv->stats.completed += s.reqs.size();
  s.reqs.clear();
  s.first_task.clear();
  s.tasks = 0;
  s.busy = false;
  srv->cv_done.notify_all();
}

// Take the arrived requests at the queue's head that fit one batch (caller
// holds the lock).
void take_arrived(soap_dp_server *srv, std::vector<std::unique_ptr<Request>> &take) {
  const auto &c = srv->cfg;
  int32_t nt = 0;
  uint64_t nw = 0;
  const uint64_t now = now_ns();
  while (!srv->queue.empty()) {
    Request &q = *srv->queue.front();
    if (q.arrival_ns > now) break;   // not arrived yet
    if (nt + q.n_tasks > c.max_tasks || nw + q.reads.size() > uint64_t(c.max_read_words)) break;
    nt += q.n_tasks;
    nw += q.reads.size();
    take.push_back(std::move(srv->queue.front()));
    srv->queue.pop_front();
  }
}

void slot_worker(soap_dp_server *srv, size_t k) {
  (void)hipSetDevice(srv->cfg.device_ordinal);
  Slot &s = srv->slots[k];
  std::vector<std::unique_ptr<Request>> take;
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
        if (next <= now) break;
        if (next > now + kSpin) {
          srv->cv_work.wait_for(lk, std::chrono::nanoseconds(next - now - kSpin / 2));
        } else {
          lk.unlock();
          std::this_thread::yield();
          lk.lock();
        }
      }
      take_arrived(srv, take);
    }
    if (take.empty()) continue;
    uint64_t t0 = now_ns();
    const int rc = launch(srv, s, take);
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
    retire(srv, s);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->stats.host_retire_s += double(now_ns() - t0) * 1e-9;
    }
  }
}

}  // namespace

extern "C" {

uint64_t soap_dp_now_ns(void) { return now_ns(); }

// Slot counts run and checked: 1 to 4.  A run with 6 slots of 32,768 reads
// ended in a host crash whose cause is not known; larger counts are refused
// until it is.
constexpr int kMaxSlots = 4;

int soap_dp_server_create(soap_dp_server **out, const soap_dp_server_config *cfg) {
  if (!out || !cfg) return SOAP_DP_EINVAL;
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > kMaxSlots || cfg->max_tasks < 1 || cfg->max_read_words < 1 ||
      cfg->max_n < 1 || cfg->max_n > SOAP_DP_MAX_READ || cfg->max_m < 1 ||
      cfg->max_m > SOAP_DP_MAX_WINDOW || !cfg->genome || cfg->genome_words == 0)
    return SOAP_DP_EINVAL;
  auto *srv = new (std::nothrow) soap_dp_server();
  if (!srv) return SOAP_DP_ENOMEM;
  srv->cfg = *cfg;
  srv->stride = 2 * cfg->max_n - 1;
  srv->slots.resize(size_t(cfg->n_slots));
  int rc = SOAP_DP_OK;
  (void)hipSetDevice(cfg->device_ordinal);
  for (auto &s : srv->slots) {
    rc = init_slot(srv, s);
    if (rc) break;
  }
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
  if (rc) {
    for (auto &s : srv->slots) free_slot(s);
    delete srv;
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
  if (req->n_tasks > c.max_tasks || req->read_words > uint64_t(c.max_read_words)) {
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
  (void)hipDeviceSynchronize();
  for (auto &s : srv->slots) free_slot(s);
  delete srv;
  return SOAP_DP_OK;
}

}  // extern "C"
