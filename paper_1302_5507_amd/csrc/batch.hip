// Device-side length bucketing for the batched form.  Every task is put in
// the smallest length class whose kernel shape holds its read: a packed
// int16 class in the offset form when the task's values stay inside int16
// (int16_fits), else one in the direct form when its read keeps every value
// below the int16 ceiling (int16_direct_fits), else an int32 class.
// Invalid tasks get their status and zero outputs here.
// The class segments of one task list are built with per-workgroup
// histograms and one atomic per class and workgroup, so nothing depends on
// the host and the whole sequence can be replayed as a graph.
#include "dp_device.h"
#include "batch.h"

namespace soapdp {

namespace {

constexpr int kBlock = 256;

__device__ int class_of(const ClassTable &ct, int32_t n, int32_t m, int32_t ma, int32_t mi,
                        int32_t go, int32_t ge) {
  // int16 offset-form classes first (ascending capacity), then the direct
  // form, then int32 classes
  for (int k = 0; k < ct.count; ++k) {
    if (ct.prec[k] != kPrecI16 || ct.cap[k] < n) continue;
    if (int16_fits(n, m, ct.cols[k], ma, mi, go, ge)) return k;
    break;   // a wider int16 shape only narrows the range
  }
  if (int16_direct_fits(n, ma, mi, go, ge))
    for (int k = 0; k < ct.count; ++k)
      if (ct.prec[k] == kPrecI16Direct && ct.cap[k] >= n) return k;
  for (int k = 0; k < ct.count; ++k)
    if (ct.prec[k] == kPrecI32 && ct.cap[k] >= n) return k;
  return -1;
}

__global__ void zero_kernel(int32_t *a, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = 0;
}

__global__ __launch_bounds__(kBlock) void classify_kernel(DpParams p, ClassTable ct,
                                                          uint8_t *task_class, int32_t *hist,
                                                          int32_t *max_m) {
  __shared__ int32_t s_hist[kMaxClasses], s_maxm[kMaxClasses];
  for (int k = threadIdx.x; k < kMaxClasses; k += kBlock) { s_hist[k] = 0; s_maxm[k] = 0; }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < p.n_tasks) {
    const int32_t n = p.read_len[t];
    const int32_t m = p.ref_len[t];
    const uint64_t rwo = p.read_word_off[t];
    const uint64_t rbo = p.ref_base_off[t];
    uint8_t st = kTaskOk;
    int k = -1;
    if (n < 1 || m < 1 || n > p.max_n || m > p.max_m)
      st = kTaskInvalidLen;
    else if (!read_in_bounds(rwo, n, p.read_words, p.read_stride) ||
             rbo + (uint64_t)m > p.ref_words * 16)
      st = kTaskInvalidOffset;
    else {
      k = class_of(ct, n, m, p.ma, p.mi, p.go, p.ge);
      if (k < 0) st = kTaskInvalidLen;
    }
    if (st != kTaskOk) {
      p.score[t] = 0; p.ref_begin[t] = 0; p.ref_end[t] = 0; p.cigar_len[t] = 0;
      p.status[t] = st;
      task_class[t] = 0xff;
    } else {
      task_class[t] = (uint8_t)k;
      atomicAdd(&s_hist[k], 1);
      atomicMax(&s_maxm[k], m);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ct.count; k += kBlock)
    if (s_hist[k]) {
      atomicAdd(&hist[k], s_hist[k]);
      atomicMax(&max_m[k], s_maxm[k]);
    }
}

// One thread: class offsets (exclusive scan of the histogram), the cursors
// the scatter advances, and the launch plan of every class from its actual
// tasks.  A class with h tasks has ceil(h / per_item) work items, so
// g = min(grid, items) workgroups do work, each deferring up to
// min(max_defer, ceil(items / g)) items into slots sized for the class's
// longest window.  While the regions g * defer * slot exceed the budget, the
// largest region's deferral drops by one; with every deferral at 1 the
// regions fit, because the budget covers every live class's full grid of
// slots for the batch's longest window.  Regions are laid out back to back,
// 64-dword aligned.
__global__ void scan_kernel(ClassTable ct, const int32_t *hist, const int32_t *max_m,
                            int32_t *offset, int32_t *cursor, int32_t *work_counter,
                            int32_t *defer, uint64_t *slot_dwords, uint64_t *scratch_off) {
  if (threadIdx.x != 0) return;
  int32_t acc = 0;
  uint64_t region[kMaxClasses];   // dwords per unit of deferral
  uint64_t total = 0;
  for (int k = 0; k < ct.count; ++k) {
    offset[k] = acc;
    cursor[k] = acc;
    work_counter[k] = 0;
    acc += hist[k];
    const int64_t items = (int64_t(hist[k]) + ct.per_item[k] - 1) / ct.per_item[k];
    const int64_t g = items < ct.grid[k] ? items : ct.grid[k];
    int64_t d = g > 0 ? (items + g - 1) / g : 1;
    d = d < ct.max_defer[k] ? d : ct.max_defer[k];
    d = d > 1 ? d : 1;
    const uint64_t B = uint64_t(ct.step_block[k]);
    const uint64_t steps = (uint64_t(max_m[k] + ct.lanes[k] - 1) + B - 1) / B * B;
    const uint64_t slot = hist[k] > 0 ? steps * uint64_t(ct.step_dwords[k]) : 0;
    defer[k] = int32_t(d);
    slot_dwords[k] = slot;
    region[k] = uint64_t(g) * slot;
    total += region[k] * uint64_t(d);
  }
  while (total > ct.budget_dwords) {
    int worst = -1;
    for (int k = 0; k < ct.count; ++k)
      if (defer[k] > 1 && (worst < 0 || region[k] * uint64_t(defer[k]) >
                                             region[worst] * uint64_t(defer[worst])))
        worst = k;
    if (worst < 0) break;
    total -= region[worst];
    --defer[worst];
  }
  uint64_t off = 0;
  for (int k = 0; k < ct.count; ++k) {
    scratch_off[k] = off;
    off += round64(region[k] * uint64_t(defer[k]));
  }
}

// Class lists follow `order` (nullptr: task index order) up to the
// interleaving of workgroups.
__global__ __launch_bounds__(kBlock) void scatter_kernel(const uint8_t *task_class, int64_t n_tasks,
                                                         const int32_t *order, int32_t *cursor,
                                                         int32_t *task_list) {
  __shared__ int32_t s_cnt[kMaxClasses], s_base[kMaxClasses];
  for (int k = threadIdx.x; k < kMaxClasses; k += kBlock) s_cnt[k] = 0;
  __syncthreads();
  const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t t = -1;
  int k = 0xff, rank = 0;
  if (x < n_tasks) {
    t = order ? (int64_t)order[x] : x;
    k = task_class[t];
    if (k != 0xff) rank = atomicAdd(&s_cnt[k], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kMaxClasses; c += kBlock)
    s_base[c] = s_cnt[c] ? atomicAdd(&cursor[c], s_cnt[c]) : 0;
  __syncthreads();
  if (x < n_tasks && k != 0xff) task_list[s_base[k] + rank] = (int32_t)t;
}

__global__ __launch_bounds__(kBlock) void gather_cigar_head_kernel(const uint32_t *cigar,
                                                                   int32_t stride,
                                                                   const int32_t *cigar_len,
                                                                   int32_t n, uint32_t *head) {
  const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t t = x / kCigarHeadWords;
  const int32_t k = (int32_t)(x % kCigarHeadWords);
  if (t >= n) return;
  const int32_t len = min(cigar_len[t], stride);
  head[x] = k < len ? cigar[t * stride + k] : 0u;
}

}  // namespace

hipError_t launch_gather_cigar_head(const uint32_t *cigar, int32_t stride, const int32_t *cigar_len,
                                    int32_t n, uint32_t *head, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t threads = int64_t(n) * kCigarHeadWords;
  hipLaunchKernelGGL(gather_cigar_head_kernel, dim3((uint32_t)((threads + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, stream, cigar, stride, cigar_len, n, head);
  return hipGetLastError();
}

hipError_t launch_bucketing(const DpParams &p, const ClassTable &ct, const BucketBuffers &b,
                            const int32_t *order, hipStream_t stream) {
  const int64_t blocks = (p.n_tasks + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, stream, b.hist, 2 * kMaxClasses);
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, stream, b.redo_count, 2);
  hipLaunchKernelGGL(classify_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, p, ct,
                     b.task_class, b.hist, b.max_m);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(64), 0, stream, ct, b.hist, b.max_m, b.offset,
                     b.cursor, b.work_counter, b.defer, b.slot_dwords, b.scratch_off);
  hipLaunchKernelGGL(scatter_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, b.task_class,
                     p.n_tasks, order, b.cursor, b.task_list);
  return hipGetLastError();
}

hipError_t launch_zero(int32_t *a, int n, hipStream_t stream) {
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, stream, a, n);
  return hipGetLastError();
}

}  // namespace soapdp
