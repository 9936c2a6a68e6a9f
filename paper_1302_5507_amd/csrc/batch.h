// Length classes of the batched form and the device buffers of its bucketing.
#pragma once
#include "dp_internal.h"
#include "serve_host.h"

namespace soapdp {

constexpr int kMaxClasses = 48;

// Class kinds (ClassTable::prec): packed int16 in the offset form, packed
// int16 in the direct form (saturating, with the int32 re-run of tasks too
// close to the floor), int32.
constexpr int kPrecI16 = 16;
constexpr int kPrecI16Direct = 17;
constexpr int kPrecI32 = 32;
__host__ __device__ inline bool packed16(int prec) { return prec == kPrecI16 || prec == kPrecI16Direct; }

// Classes in the order tried: int16 classes (offset form) by ascending
// capacity, then int16 classes in the direct form, then int32 classes.  A class's capacity is its upper
// bound on read length; `cols` is lanes * cells of its current shape.
//
// The launch fields describe each class kernel as the host enqueues it:
// tasks per work item, grid, the most work items a workgroup may defer
// before tracing back (64 / tasks per item), lanes per task and decision
// dwords per sweep step; a slot holds (longest window + lanes - 1) steps
// rounded up to whole blocks.
// `budget_dwords` is the scratch the context holds for all class kernels.
struct ClassTable {
  int32_t count;
  int32_t cap[kMaxClasses];
  int32_t cols[kMaxClasses];
  int32_t prec[kMaxClasses];
  int32_t per_item[kMaxClasses];
  int32_t grid[kMaxClasses];
  int32_t max_defer[kMaxClasses];
  int32_t lanes[kMaxClasses];
  int32_t step_dwords[kMaxClasses];   // decision dwords per sweep step
  int32_t step_block[kMaxClasses];    // slots hold whole blocks of this many steps
  uint64_t budget_dwords;
};

// Device buffers of the bucketing and of the class plans; `hist` and
// `max_m` are adjacent (one fill clears both).
struct BucketBuffers {
  uint8_t *task_class;    // n_tasks
  int32_t *task_list;     // n_tasks, class segments
  int32_t *hist;          // kMaxClasses: tasks per class
  int32_t *max_m;         // kMaxClasses: longest window per class
  int32_t *offset;        // kMaxClasses: segment starts
  int32_t *cursor;        // kMaxClasses
  int32_t *work_counter;  // kMaxClasses: persistent-kernel work queues
  int32_t *defer;         // kMaxClasses: deferral of each class kernel
  uint64_t *slot_dwords;  // kMaxClasses: decision-slot size of each class
  uint64_t *scratch_off;  // kMaxClasses: scratch region of each class (dwords)
  int32_t *redo_list;     // n_tasks: tasks the direct-form kernels flag
  int32_t *redo_count;    // their count (cleared by the bucketing)
  int32_t *redo_work_counter;   // work queue of the int32 re-run (cleared likewise)
};

// Round a region to 64 dwords (256 bytes).
__host__ __device__ inline uint64_t round64(uint64_t dwords) { return (dwords + 63) & ~uint64_t(63); }

// Enqueue: zero the histogram, classify (invalid tasks get their outputs),
// scan and plan, scatter.  `p` carries the batch, scoring and outputs.  The
// class lists take the tasks in `order` (nullptr: index order).
hipError_t launch_bucketing(const DpParams &p, const ClassTable &ct, const BucketBuffers &b,
                            const int32_t *order, hipStream_t stream);
hipError_t launch_zero(int32_t *a, int n, hipStream_t stream);
// First CIGAR words of every task, gathered densely for one small copy back
// to the host: head[t * kCigarHeadWords + k] = word k of task t's row for
// k < cigar_len[t], else 0; tasks [0, n).
hipError_t launch_gather_cigar_head(const uint32_t *cigar, int32_t stride, const int32_t *cigar_len,
                                    int32_t n, uint32_t *head, hipStream_t stream);

}  // namespace soapdp
