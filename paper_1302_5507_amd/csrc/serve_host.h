// Host-side bookkeeping of the continuous-batching server, kept free of HIP
// calls so that it can be built and checked on a CPU alone: the request
// record, admission of queued requests into one batch by slot capacity and
// by device memory, the device-memory arena the batches in flight share,
// the merge of requests into one batch's staging arrays, and the hand-off
// of a finished batch's results into each request's buffers.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "../../include/soap_dp.h"

namespace soapdp {

// First CIGAR words of every task that a served batch copies back densely.
constexpr int32_t kCigarHeadWords = 16;

// One long CIGAR row packed on the device: task index in the batch and the
// offset of its words past the head in the packed word area (-1: the area
// was full and the row was not packed).
struct RestRow {
  int32_t task;
  int32_t off;
};

namespace serve {

struct Request {
  uint64_t ticket = 0;
  int32_t n_tasks = 0;
  std::vector<uint32_t> reads;
  std::vector<uint64_t> rwo;
  std::vector<int32_t> rl, ml;
  std::vector<uint64_t> rbo;
  soap_dp_host_result out{};
  soap_dp_request_stamps *stamps = nullptr;   // caller's, optional
  uint64_t arrival_ns = 0;
  uint64_t taken_ns = 0, launched_ns = 0, device_ns = 0;
  int64_t cells = 0;
};

// Device regions of one batch of `tasks` tasks and `words` packed read
// words inside the arena, as byte offsets from the batch's base (each
// region 256-byte aligned), and the capacities of its long-row rest area.
struct BatchLayout {
  size_t reads, rwo, rbo, rl, ml, i32, status, cigar, head, rest_hdr, rest_rows, rest;
  size_t bytes;
  int32_t rest_rows_cap, rest_words_cap;
};
BatchLayout batch_layout(int64_t tasks, uint64_t words, int32_t stride);

// First-fit allocator over [0, capacity) bytes of one device allocation,
// 256-byte granules.  Not thread-safe (the server holds its lock).
class Arena {
 public:
  explicit Arena(size_t capacity = 0);
  // Reserve `bytes`; false when no free block is large enough.
  bool alloc(size_t bytes, size_t *off);
  void release(size_t off);
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t largest_free() const;

 private:
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;   // offset -> size, coalesced
  std::map<size_t, size_t> live_;   // offset -> size
};

// Slot limits of one batch.
struct Limits {
  int32_t max_tasks;
  uint64_t max_read_words;
  int32_t stride;
};

// Move the requests at the head of `queue` that have arrived by `now` into
// `take`, in order, while the merged batch stays within the slot limits and
// its device regions fit one free block of `arena`; the block is reserved
// and its offset returned in *off.  Stops at the first request that does
// not fit (first in, first out).  Returns false, taking nothing, when the
// head request has not arrived or does not fit.
bool take_arrived(std::deque<std::unique_ptr<Request>> &queue, uint64_t now, const Limits &lim,
                  Arena &arena, std::vector<std::unique_ptr<Request>> &take, size_t *off,
                  BatchLayout *layout);

// Staging arrays of one batch (host memory, slot capacity).
struct Staging {
  uint32_t *reads;
  uint64_t *rwo, *rbo;
  int32_t *rl, *ml;
};

// Read offset given to a task whose read words lie outside its request:
// past any read buffer, so the kernels report SOAP_DP_TASK_INVALID_OFFSET,
// as soap_dp_align_batch does for a request aligned on its own.
constexpr uint64_t kBadReadOffset = uint64_t(1) << 62;

// Copy `reqs` into the staging arrays, rebasing read offsets into the
// merged read buffer.  first_task[r] receives request r's first task.
// Returns the task count; *words receives the merged read words.
int32_t merge(const std::vector<std::unique_ptr<Request>> &reqs, int32_t max_n, const Staging &st,
              std::vector<int32_t> &first_task, uint64_t *words);

// Host copies of a finished batch's outputs (`cap`: the slot capacity the
// per-task arrays are laid out with: score | begin | end | cigar_len).
struct BatchHost {
  int32_t cap;
  int32_t stride;
  const int32_t *i32;
  const uint8_t *status;
  const uint32_t *head;                // kCigarHeadWords per task
  const RestRow *rows;                 // packed long rows, sorted by task
  int32_t n_rows;
  const uint32_t *rest;                // their words past the head
  int32_t rest_words;                  // valid words of `rest`
};

// A CIGAR rest that the hand-off could not take from the packed area and
// that the caller must fetch from the device: words [kCigarHeadWords, len)
// of batch task `task`'s row, to `dst`.
struct Fetch {
  int32_t task;
  uint32_t *dst;
  int32_t words;
};

// Copy the results of the request whose tasks start at batch task `first`
// into its buffers.  CIGARs are packed: a task's runs follow the previous
// task's.  Returns SOAP_DP_OK or SOAP_DP_E2BIG when the CIGARs exceed the
// request's capacity (nothing is written past it; the other outputs are
// complete).  Rests to fetch are appended to `fetch`.
int hand_off(const BatchHost &b, int32_t first, const Request &q, std::vector<Fetch> &fetch);

}  // namespace serve
}  // namespace soapdp
