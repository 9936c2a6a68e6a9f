// CPU check of the server's host bookkeeping (paper_1302_5507_amd/csrc/
// serve_host.cpp), built by tests/test_serve_host.py with AddressSanitizer
// and UndefinedBehaviorSanitizer.  Several worker threads share one request
// queue and one device-memory arena, as the server's slot workers do; each
// takes batches, merges them into its own staging, fabricates the outputs a
// device would produce for every merged task, hands them off and checks
// every request's buffers word by word.  Exit status 0 when every check
// holds.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "serve_host.h"

using namespace soapdp;
using namespace soapdp::serve;

namespace {

std::atomic<int> g_fail{0};

#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      g_fail.fetch_add(1);                                                    \
    }                                                                         \
  } while (0)

constexpr int32_t kMaxN = 250;
constexpr int32_t kStride = 2 * kMaxN - 1;
constexpr int32_t kGuard = 64;   // words after each CIGAR buffer that must stay untouched
constexpr uint32_t kGuardWord = 0xdeadbeefu;

uint32_t mix(uint64_t a, uint64_t b, uint64_t c) {
  uint64_t z = a * 0x9e3779b97f4a7c15ull ^ (b + 0x632be59bd9b4e019ull) * 0xbf58476d1ce4e5b9ull ^
               (c + 7) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return uint32_t(z * 0xd6e8feb86659fd93ull >> 32);
}

// What the device returns for task t of request `ticket`: a CIGAR length in
// [0, kStride] (several longer than the head) and its words.
int32_t fake_len(uint64_t ticket, int32_t t) {
  const uint32_t h = mix(ticket, uint64_t(t), 1);
  if (h % 7 == 0) return int32_t(kCigarHeadWords + 1 + h % 60);   // a long row
  return int32_t(h % (kCigarHeadWords + 1));
}
uint32_t fake_word(uint64_t ticket, int32_t t, int32_t k) { return mix(ticket, uint64_t(t), 100 + k); }

struct Owned {
  std::unique_ptr<Request> req;   // moved into the queue on submit
  Request *r = nullptr;
  std::vector<int32_t> score, begin, end, clen;
  std::vector<uint8_t> status;
  std::vector<uint32_t> cigar;    // capacity + guard
  int64_t capacity = 0;
  std::vector<uint64_t> expected_rwo;   // rebased later; kBadReadOffset marks a bad one
};

std::unique_ptr<Owned> make_request(std::mt19937_64 &rng, uint64_t ticket) {
  auto o = std::make_unique<Owned>();
  auto q = std::make_unique<Request>();
  const int32_t n = 1 + int32_t(rng() % 300);
  q->ticket = ticket;
  q->n_tasks = n;
  uint64_t words = 0;
  for (int32_t t = 0; t < n; ++t) {
    int32_t len = 1 + int32_t(rng() % kMaxN);
    const uint32_t pick = uint32_t(rng() % 40);
    if (pick == 0) len = 0;             // empty read
    if (pick == 1) len = kMaxN + 5;     // longer than max_n
    const uint64_t need = len >= 1 && len <= kMaxN ? uint64_t((len + 15) / 16) : 0;
    q->rl.push_back(len);
    q->rwo.push_back(words);
    words += need;
    q->rbo.push_back(rng() % 1000000);
    q->ml.push_back(1 + int32_t(rng() % 410));
  }
  for (uint64_t w = 0; w < words; ++w) q->reads.push_back(mix(ticket, w, 7));
  // a few tasks point outside their own read words
  for (int32_t t = 0; t < n; ++t) {
    const uint32_t pick = uint32_t(rng() % 25);
    if (pick == 0) q->rwo[size_t(t)] = words;                 // starts at the end
    if (pick == 1) q->rwo[size_t(t)] = words + 1000;           // far past it
    if (pick == 2 && words) q->rwo[size_t(t)] = words - 1;     // runs past the end
  }
  for (int32_t t = 0; t < n; ++t) {
    const int32_t len = q->rl[size_t(t)];
    const bool len_ok = len >= 1 && len <= kMaxN;
    const uint64_t need = len_ok ? uint64_t((len + 15) / 16) : 0;
    const uint64_t r = q->rwo[size_t(t)];
    const bool inside = r <= words && need <= words - r;
    o->expected_rwo.push_back(len_ok && !inside ? kBadReadOffset : r);
  }
  int64_t total = 0;
  for (int32_t t = 0; t < n; ++t) total += fake_len(ticket, t);
  o->capacity = (rng() % 6 == 0) ? std::max<int64_t>(0, total - 1 - int64_t(rng() % 40)) : total + int64_t(rng() % 3);
  o->score.assign(size_t(n), -1);
  o->begin.assign(size_t(n), -1);
  o->end.assign(size_t(n), -1);
  o->clen.assign(size_t(n), -1);
  o->status.assign(size_t(n), 255);
  o->cigar.assign(size_t(o->capacity + kGuard), kGuardWord);
  q->out = soap_dp_host_result{o->score.data(), o->begin.data(), o->end.data(), o->clen.data(),
                               o->status.data(), o->cigar.data(), o->capacity};
  q->arrival_ns = ticket;   // every request has arrived by `now` below
  o->r = q.get();
  o->req = std::move(q);
  return o;
}

void check_arena() {
  std::mt19937_64 rng(5);
  Arena a(1 << 20);
  std::vector<size_t> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 2) {
      size_t off = 0;
      const size_t bytes = 1 + rng() % 70000;
      if (a.alloc(bytes, &off)) {
        CHECK(off % 256 == 0 && off + bytes <= a.capacity());
        live.push_back(off);
      } else {
        CHECK(a.largest_free() < bytes);
      }
    } else {
      const size_t k = rng() % live.size();
      a.release(live[k]);
      live.erase(live.begin() + long(k));
    }
    CHECK(a.used() <= a.capacity() && a.used() <= a.peak());
  }
  for (size_t off : live) a.release(off);
  CHECK(a.used() == 0 && a.largest_free() == a.capacity());
}

struct Shared {
  std::mutex mu;
  std::deque<std::unique_ptr<Request>> queue;
  Arena arena;
  Limits lim;
  std::vector<uint64_t> taken_order;   // tickets in the order batches took them
  size_t peak_seen = 0;
};

void worker(Shared *sh, std::vector<std::unique_ptr<Owned>> *owned, uint64_t seed) {
  const Limits lim = sh->lim;
  std::vector<uint32_t> reads(size_t(lim.max_read_words));
  std::vector<uint64_t> rwo(size_t(lim.max_tasks)), rbo(size_t(lim.max_tasks));
  std::vector<int32_t> rl(size_t(lim.max_tasks)), ml(size_t(lim.max_tasks));
  std::vector<int32_t> i32(4 * size_t(lim.max_tasks));
  std::vector<uint8_t> status(size_t(lim.max_tasks));
  std::vector<uint32_t> head(size_t(lim.max_tasks) * kCigarHeadWords);
  std::vector<RestRow> rows;
  std::vector<uint32_t> rest;
  std::mt19937_64 rng(seed);
  for (;;) {
    std::vector<std::unique_ptr<Request>> take;
    size_t region = 0;
    BatchLayout lay{};
    {
      std::lock_guard<std::mutex> lk(sh->mu);
      if (sh->queue.empty()) return;
      if (!take_arrived(sh->queue, ~uint64_t(0), lim, sh->arena, take, &region, &lay)) continue;
      for (auto &q : take) sh->taken_order.push_back(q->ticket);
      sh->peak_seen = std::max(sh->peak_seen, sh->arena.used());
      CHECK(sh->arena.used() <= sh->arena.capacity());
    }
    std::vector<int32_t> first;
    uint64_t nw = 0;
    const Staging st{reads.data(), rwo.data(), rbo.data(), rl.data(), ml.data()};
    const int32_t nt = merge(take, kMaxN, st, first, &nw);
    CHECK(nt <= lim.max_tasks && nw <= lim.max_read_words);
    CHECK(lay.bytes == batch_layout(nt, nw, lim.stride).bytes);
    // merged inputs
    uint64_t wbase = 0;
    for (size_t r = 0; r < take.size(); ++r) {
      const Request &q = *take[r];
      const Owned &o = *(*owned)[size_t(q.ticket)];
      for (int32_t t = 0; t < q.n_tasks; ++t) {
        const int32_t b = first[r] + t;
        const uint64_t e = o.expected_rwo[size_t(t)];
        CHECK(rwo[size_t(b)] == (e == kBadReadOffset ? e : e + wbase));
        CHECK(rl[size_t(b)] == q.rl[size_t(t)] && ml[size_t(b)] == q.ml[size_t(t)] &&
              rbo[size_t(b)] == q.rbo[size_t(t)]);
      }
      for (size_t w = 0; w < q.reads.size(); ++w) CHECK(reads[size_t(wbase + w)] == q.reads[w]);
      wbase += q.reads.size();
    }
    // fabricated device outputs, laid out with the slot capacity
    const int32_t C = lim.max_tasks;
    rows.clear();
    rest.clear();
    std::vector<std::pair<int32_t, int32_t>> unpacked;   // long rows left to fetch
    for (size_t r = 0; r < take.size(); ++r) {
      const Request &q = *take[r];
      for (int32_t t = 0; t < q.n_tasks; ++t) {
        const int32_t b = first[r] + t, len = fake_len(q.ticket, t);
        i32[size_t(b)] = int32_t(mix(q.ticket, uint64_t(t), 2) % 1000) - 500;
        i32[size_t(C + b)] = int32_t(mix(q.ticket, uint64_t(t), 3) % 400);
        i32[size_t(2 * C + b)] = int32_t(mix(q.ticket, uint64_t(t), 4) % 400);
        i32[size_t(3 * C + b)] = len;
        status[size_t(b)] = uint8_t(mix(q.ticket, uint64_t(t), 5) % 6);
        for (int32_t k = 0; k < kCigarHeadWords; ++k)
          head[size_t(b) * kCigarHeadWords + size_t(k)] = k < len ? fake_word(q.ticket, t, k) : 0u;
        if (len > kCigarHeadWords) {
          const uint32_t how = uint32_t(rng() % 4);
          if (how == 0) continue;                                   // not listed
          if (how == 1) { rows.push_back(RestRow{b, -1}); continue; }   // area was full
          const int32_t off = int32_t(rest.size());
          for (int32_t k = kCigarHeadWords; k < len; ++k) rest.push_back(fake_word(q.ticket, t, k));
          rows.push_back(RestRow{b, off});
        }
      }
    }
    std::sort(rows.begin(), rows.end(), [](const RestRow &x, const RestRow &y) { return x.task < y.task; });
    const int32_t rest_valid = int32_t(rest.size()) - int32_t(rng() % 3 == 0 ? std::min<size_t>(rest.size(), 20) : 0);
    const BatchHost bh{C, kStride, i32.data(), status.data(), head.data(), rows.data(),
                       int32_t(rows.size()), rest.data(), rest_valid};
    std::vector<Fetch> fetch;
    for (size_t r = 0; r < take.size(); ++r) {
      const Request &q = *take[r];
      Owned &o = *(*owned)[size_t(q.ticket)];
      fetch.clear();
      const int rc = hand_off(bh, first[r], q, fetch);
      // the device copies of the rests the packed area did not hold
      for (const Fetch &f : fetch) {
        const int32_t t = f.task - first[r];
        CHECK(t >= 0 && t < q.n_tasks);
        CHECK(f.words == fake_len(q.ticket, t) - kCigarHeadWords);
        CHECK(f.dst >= o.cigar.data() && f.dst + f.words <= o.cigar.data() + o.capacity);
        for (int32_t k = 0; k < f.words; ++k) f.dst[k] = fake_word(q.ticket, t, kCigarHeadWords + k);
      }
      int64_t total = 0;
      for (int32_t t = 0; t < q.n_tasks; ++t) total += fake_len(q.ticket, t);
      CHECK(rc == (total <= o.capacity ? SOAP_DP_OK : SOAP_DP_E2BIG));
      int64_t w = 0;
      for (int32_t t = 0; t < q.n_tasks; ++t) {
        const int32_t b = first[r] + t, len = fake_len(q.ticket, t);
        CHECK(o.score[size_t(t)] == i32[size_t(b)] && o.begin[size_t(t)] == i32[size_t(C + b)] &&
              o.end[size_t(t)] == i32[size_t(2 * C + b)] && o.clen[size_t(t)] == len &&
              o.status[size_t(t)] == status[size_t(b)]);
        if (w + len <= o.capacity)
          for (int32_t k = 0; k < len; ++k) CHECK(o.cigar[size_t(w + k)] == fake_word(q.ticket, t, k));
        w += len;
      }
      for (int32_t g = 0; g < kGuard; ++g) CHECK(o.cigar[size_t(o.capacity + g)] == kGuardWord);
    }
    {
      std::lock_guard<std::mutex> lk(sh->mu);
      sh->arena.release(region);
    }
  }
}

}  // namespace

int main() {
  check_arena();
  // every request fits the arena on its own; several batches fit at once
  Shared sh;
  sh.lim = Limits{1200, 1200 * 16, kStride};
  sh.arena = Arena(3 * batch_layout(900, 900 * 16, kStride).bytes);
  std::mt19937_64 rng(11);
  std::vector<std::unique_ptr<Owned>> owned;
  const int kRequests = 3000;
  for (int k = 0; k < kRequests; ++k) {
    owned.push_back(make_request(rng, uint64_t(k)));
    sh.queue.push_back(std::move(owned.back()->req));
  }
  // a request whose batch cannot fit the arena must not be taken
  {
    Arena tiny(batch_layout(1, 1, kStride).bytes);
    std::deque<std::unique_ptr<Request>> q1;
    auto big = make_request(rng, 999999);
    while (big->r->n_tasks < 2) big = make_request(rng, 999999);
    q1.push_back(std::move(big->req));
    std::vector<std::unique_ptr<Request>> take;
    size_t off = 0;
    BatchLayout lay{};
    CHECK(!take_arrived(q1, ~uint64_t(0), sh.lim, tiny, take, &off, &lay));
    CHECK(take.empty() && tiny.used() == 0);
    // not yet arrived: nothing is taken
    Arena roomy(1 << 30);
    q1.front()->arrival_ns = 1000;
    CHECK(!take_arrived(q1, 999, sh.lim, roomy, take, &off, &lay) && take.empty());
  }
  std::vector<std::thread> th;
  for (int k = 0; k < 6; ++k) th.emplace_back(worker, &sh, &owned, 100 + uint64_t(k));
  for (auto &t : th) t.join();
  // first in, first out: every ticket taken exactly once, in submission order
  CHECK(sh.taken_order.size() == size_t(kRequests));
  for (size_t k = 0; k < sh.taken_order.size(); ++k) CHECK(sh.taken_order[k] == k);
  CHECK(sh.arena.used() == 0 && sh.peak_seen <= sh.arena.capacity());
  CHECK(sh.arena.peak() > batch_layout(900, 900 * 16, kStride).bytes);   // batches overlapped
  if (g_fail.load()) {
    std::fprintf(stderr, "%d checks failed\n", g_fail.load());
    return 1;
  }
  std::printf("serve_host_check ok: %d requests, peak %zu of %zu arena bytes\n", kRequests,
              sh.arena.peak(), sh.arena.capacity());
  return 0;
}
