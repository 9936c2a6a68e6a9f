// Host-side bookkeeping of the continuous-batching server (no HIP calls;
// declared in serve_host.h).
#include "serve_host.h"

#include <algorithm>
#include <cstring>
#include <iterator>

namespace soapdp {
namespace serve {

namespace {

constexpr size_t kGranule = 256;

size_t round_up(size_t b) { return (b + kGranule - 1) / kGranule * kGranule; }

}  // namespace

BatchLayout batch_layout(int64_t tasks, uint64_t words, int32_t stride) {
  const size_t T = size_t(std::max<int64_t>(tasks, 1));
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(std::max<size_t>(bytes, 1));
    return at;
  };
  L.rest_rows_cap = int32_t(std::min<int64_t>(1024, std::max<int64_t>(16, int64_t(T) / 64)));
  L.rest_words_cap = int32_t(std::min<int64_t>(32768, std::max<int64_t>(512, int64_t(T) / 4)));
  L.reads = take(size_t(std::max<uint64_t>(words, 1)) * 4);
  L.rwo = take(T * 8);
  L.rbo = take(T * 8);
  L.rl = take(T * 4);
  L.ml = take(T * 4);
  L.i32 = take(4 * T * 4);
  L.status = take(T);
  L.cigar = take(T * size_t(std::max(stride, 1)) * 4);
  L.head = take(T * size_t(kCigarHeadWords) * 4);
  L.rest_hdr = take(2 * 4);
  L.rest_rows = take(size_t(L.rest_rows_cap) * sizeof(RestRow));
  L.rest = take(size_t(L.rest_words_cap) * 4);
  L.bytes = off;
  return L;
}

Arena::Arena(size_t capacity) : cap_(capacity / kGranule * kGranule) {
  if (cap_) free_.emplace(0, cap_);
}

bool Arena::alloc(size_t bytes, size_t *off) {
  const size_t need = round_up(std::max<size_t>(bytes, 1));
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < need) continue;
    const size_t at = it->first, left = it->second - need;
    free_.erase(it);
    if (left) free_.emplace(at + need, left);
    live_.emplace(at, need);
    used_ += need;
    peak_ = std::max(peak_, used_);
    *off = at;
    return true;
  }
  return false;
}

void Arena::release(size_t off) {
  auto it = live_.find(off);
  if (it == live_.end()) return;
  size_t at = it->first, len = it->second;
  used_ -= len;
  live_.erase(it);
  auto nx = free_.lower_bound(at);
  if (nx != free_.end() && nx->first == at + len) {   // merge with the block after
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {                            // and with the block before
    auto pv = std::prev(nx);
    if (pv->first + pv->second == at) {
      at = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_.emplace(at, len);
}

size_t Arena::largest_free() const {
  size_t best = 0;
  for (const auto &f : free_) best = std::max(best, f.second);
  return best;
}

bool take_arrived(std::deque<std::unique_ptr<Request>> &queue, uint64_t now, const Limits &lim,
                  Arena &arena, std::vector<std::unique_ptr<Request>> &take, size_t *off,
                  BatchLayout *layout) {
  int64_t nt = 0;
  uint64_t nw = 0;
  size_t k = 0;
  const size_t room = arena.largest_free();
  for (; k < queue.size(); ++k) {
    const Request &q = *queue[k];
    if (q.arrival_ns > now) break;   // not arrived yet
    const int64_t t2 = nt + q.n_tasks;
    const uint64_t w2 = nw + q.reads.size();
    if (t2 > lim.max_tasks || w2 > lim.max_read_words) break;
    if (batch_layout(t2, w2, lim.stride).bytes > room) break;
    nt = t2;
    nw = w2;
  }
  if (k == 0) return false;
  *layout = batch_layout(nt, nw, lim.stride);
  if (!arena.alloc(layout->bytes, off)) return false;   // cannot happen: it fit `room`
  for (size_t j = 0; j < k; ++j) {
    take.push_back(std::move(queue.front()));
    queue.pop_front();
  }
  return true;
}

int32_t merge(const std::vector<std::unique_ptr<Request>> &reqs, int32_t max_n, const Staging &st,
              std::vector<int32_t> &first_task, uint64_t *words) {
  int32_t nt = 0;
  uint64_t nw = 0;
  first_task.clear();
  for (const auto &qp : reqs) {
    const Request &q = *qp;
    first_task.push_back(nt);
    const uint64_t qw = q.reads.size();
    if (qw) std::memcpy(st.reads + nw, q.reads.data(), qw * 4);
    for (int32_t t = 0; t < q.n_tasks; ++t) {
      const int32_t n = q.rl[size_t(t)];
      const uint64_t r = q.rwo[size_t(t)];
      // a read of valid length must lie inside its own request's words;
      // a length outside 1..max_n is reported by the kernels first
      const bool len_ok = n >= 1 && n <= max_n;
      const uint64_t need = len_ok ? uint64_t((n + 15) >> 4) : 0;
      const bool inside = r <= qw && need <= qw - r;
      st.rwo[nt + t] = (len_ok && !inside) ? kBadReadOffset : r + nw;
      st.rl[nt + t] = n;
      st.rbo[nt + t] = q.rbo[size_t(t)];
      st.ml[nt + t] = q.ml[size_t(t)];
    }
    nt += q.n_tasks;
    nw += qw;
  }
  *words = nw;
  return nt;
}

int hand_off(const BatchHost &b, int32_t first, const Request &q, std::vector<Fetch> &fetch) {
  const int32_t n = q.n_tasks, C = b.cap, S = b.stride;
  constexpr int32_t H = kCigarHeadWords;
  const soap_dp_host_result &o = q.out;
  std::memcpy(o.score, b.i32 + first, size_t(n) * 4);
  std::memcpy(o.ref_begin, b.i32 + C + first, size_t(n) * 4);
  std::memcpy(o.ref_end, b.i32 + 2 * size_t(C) + first, size_t(n) * 4);
  std::memcpy(o.cigar_len, b.i32 + 3 * size_t(C) + first, size_t(n) * 4);
  std::memcpy(o.status, b.status + first, size_t(n));
  const int32_t *lens = b.i32 + 3 * size_t(C) + first;
  const uint32_t *head = b.head + int64_t(first) * H;
  int64_t total = 0;
  for (int32_t t = 0; t < n; ++t) total += std::min(std::max(lens[t], 0), S);
  // A row whose full head (H words) ends within the request's packed CIGARs
  // is copied whole, with no length-dependent branch; the words past the
  // row are rewritten by the rows after it, which are copied later.  Other
  // rows, and every row of a request that does not fit its buffer, are
  // copied word by word up to their length.
  const bool whole = total <= o.cigar_capacity;
  int rc = SOAP_DP_OK;
  int64_t words = 0;
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
        const int32_t task = first + t, need = len - H;
        int32_t off = -1;
        const RestRow *end = b.rows + b.n_rows;
        const RestRow *it = std::lower_bound(
            b.rows, end, task, [](const RestRow &r, int32_t v) { return r.task < v; });
        if (it != end && it->task == task) off = it->off;
        if (off >= 0 && int64_t(off) + need <= b.rest_words)
          std::memcpy(dst + H, b.rest + off, size_t(need) * 4);
        else
          fetch.push_back(Fetch{task, dst + H, need});
      }
    }
    words += len;
  }
  return rc;
}

}  // namespace serve
}  // namespace soapdp
