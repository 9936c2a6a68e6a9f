// Length classes of the batched form and the device buffers of its bucketing.
#pragma once
#include "dp_internal.h"

namespace soapdp {

constexpr int kMaxClasses = 32;

// Classes in the order tried: int16 classes by ascending capacity, then
// int32 classes by ascending capacity.  A class's capacity is its upper
// bound on read length; `cols` is lanes * cells of its current shape.
struct ClassTable {
  int32_t count;
  int32_t cap[kMaxClasses];
  int32_t cols[kMaxClasses];
  int32_t prec[kMaxClasses];
};

struct BucketBuffers {
  uint8_t *task_class;    // n_tasks
  int32_t *task_list;     // n_tasks, class segments
  int32_t *hist;          // kMaxClasses: tasks per class
  int32_t *offset;        // kMaxClasses: segment starts
  int32_t *cursor;        // kMaxClasses
  int32_t *work_counter;  // kMaxClasses: persistent-kernel work queues
};

// Enqueue: zero the histogram, classify (invalid tasks get their outputs),
// scan, scatter.  `p` carries the batch, scoring and outputs.
hipError_t launch_bucketing(const DpParams &p, const ClassTable &ct, const BucketBuffers &b,
                            hipStream_t stream);
hipError_t launch_zero(int32_t *a, int n, hipStream_t stream);
// Pack the CIGAR rows of tasks [0, n) back to back (at most out_cap words).
hipError_t launch_compact_cigar(const uint32_t *cigar, int32_t stride, const int32_t *cigar_len,
                                int32_t n, uint32_t *out, int64_t out_cap, hipStream_t stream);

}  // namespace soapdp
