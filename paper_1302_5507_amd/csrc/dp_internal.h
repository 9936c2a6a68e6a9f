// Internal declarations shared by the HIP kernels and the host library.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace soapdp {

constexpr int kWave = 64;
constexpr int32_t kNeg32 = -(1 << 30);  // minus infinity in the int32 kernels

// Per-task status values (mirrors the public header).
constexpr uint8_t kTaskOk = 0;
constexpr uint8_t kTaskInvalidLen = 1;
constexpr uint8_t kTaskRedone = 2;
constexpr uint8_t kTaskInvalidOffset = 3;
constexpr uint8_t kTaskBelowCutoff = 5;
// Internal: an int16 kernel in the direct form found the task's score too
// close to the saturation floor for its outputs to be exact; the int32
// re-run overwrites this status.
constexpr uint8_t kTaskNeedsRedo = 0xfe;

// Arguments of every DP kernel, passed by value.
struct DpParams {
  const uint32_t *read_codes;
  const uint64_t *read_word_off;
  const int32_t *read_len;
  const uint32_t *ref_codes;
  const uint64_t *ref_base_off;
  const int32_t *ref_len;
  int64_t n_tasks;
  uint64_t read_words;
  uint64_t ref_words;
  int32_t max_n, max_m;
  int32_t ma, mi, go, ge;
  int32_t *score;
  int32_t *ref_begin;
  int32_t *ref_end;
  uint32_t *cigar;
  int32_t cigar_stride;
  int32_t *cigar_len;
  uint8_t *status;
  // Decision-bit scratch: `defer` slots of `slot_dwords` per workgroup of the
  // grid.  A workgroup sweeps up to `defer` work items (one per slot) before
  // it traces them back together; 1 <= defer <= 64 / tasks per work item.
  uint32_t *scratch;
  uint64_t slot_dwords;
  int32_t defer;
  // Device-planned launch (batched form): when non-null, the deferral, the
  // slot size and the offset (dwords) of this kernel's scratch region are
  // read from here instead.
  const int32_t *defer_dev;
  const uint64_t *slot_dwords_dev;
  const uint64_t *scratch_off_dev;
  // Optional task order (nullptr: identity) and its length; work items are
  // groups of (tasks per wave) consecutive entries of that order.
  const int32_t *task_list;
  const int32_t *task_count;   // device count overriding n_tasks when non-null
  // When non-null, the task order starts at task_list + *task_off (a class
  // segment of the batched form, located on the device).
  const int32_t *task_off;
  // Optional dynamic work counter (nullptr: static grid-stride schedule).
  int32_t *work_counter;
  // Status written for a task this kernel completes (kTaskOk, or kTaskRedone
  // when the int32 kernel re-runs tasks outside the int16 range).
  uint8_t ok_status;
  // Nonzero: score and end only (ref_begin -1, cigar_len 0, no CIGAR, no
  // decision scratch).
  uint8_t score_only;
  // Tasks scoring below this get kTaskBelowCutoff and no traceback
  // (INT32_MIN: no cutoff).
  int32_t min_score;
  // int16 direct form: tasks whose score lies too close to the saturation
  // floor are appended here (atomically counted) for the int32 re-run.
  int32_t *redo_list;
  int32_t *redo_count;
  // Word k of read t is read_codes[read_word_off[t] + k * read_stride]: 1
  // for reads stored one after another, kReadGroup for reads interleaved
  // word by word in groups.
  uint32_t read_stride;
};

// Reads interleaved word by word in groups of this many (the paper's
// layout for a warp of one-problem threads).
constexpr uint32_t kReadGroup = 32;

// The words of an n-base read at word offset rwo, stride `stride`, lie
// inside a buffer of read_words words.
__host__ __device__ inline bool read_in_bounds(uint64_t rwo, int32_t n, uint64_t read_words,
                                               uint32_t stride) {
  const uint64_t nw = (uint64_t)((n + 15) >> 4);
  return nw == 0 || rwo + (nw - 1) * stride < read_words;
}

// Decision words are stored in blocks of `step_block(K)` sweep steps: within
// a block each lane's words for consecutive steps are contiguous, so the
// traceback fetches one lane's block in one piece.  Eight steps while a lane
// has at most two column groups (W = ceil(K/8) words per step), else four
// (bounds the LDS staging buffer).  Slots hold whole blocks.
__host__ __device__ constexpr int step_block(int K) { return (K + 7) / 8 <= 2 ? 8 : 4; }

// A kernel shape: L lanes cooperate on one task, each owning K read columns.
struct Shape {
  int lanes;
  int cells;
};

// The sweeps carry M as G = X - (i+j) S_GE + (S_GO - S_GE): the value that
// opens a gap next to the cell, so the cells to the right and below use it
// without another add.  The diagonal constants relative to it are
// S_MA - S_GE - S_GO on a match, S_MI - S_GE - S_GO on a mismatch and
// -S_GE - S_GO left of the read.  True when they fit an unsigned byte, so
// one byte permute looks them up.
__host__ __device__ inline bool byte_delta_fits(int32_t ma, int32_t mi, int32_t go, int32_t ge) {
  const int64_t d_ma = int64_t(ma) - int64_t(ge) - int64_t(go);
  const int64_t d_mi = int64_t(mi) - int64_t(ge) - int64_t(go);
  const int64_t d_v = -int64_t(ge) - int64_t(go);
  return d_mi >= 0 && d_ma <= 255 && d_v <= 255;
}

// int16 form: a task (read of n bases, window of m) can run in packed int16
// iff the diagonal constants fit a byte table (byte_delta_fits) and every
// value the kernel forms stays inside int16: real cells lie between the
// lowest possible maximum and n S_MA, shifted up by at most (m + n) |S_GE|;
// virtual columns hold (i+j) |S_GE| with j down to -cols; each bound is
// widened by twice the largest constant added (S_GO - S_GE, the diagonal
// constants, S_GE).  Evaluated identically on host and device.
__host__ __device__ inline bool int16_fits(int32_t n, int32_t m, int32_t cols, int32_t ma,
                                           int32_t mi, int32_t go, int32_t ge) {
  if (!byte_delta_fits(ma, mi, go, ge)) return false;
  const int64_t d_ma = int64_t(ma) - int64_t(ge) - int64_t(go);
  auto iabs = [](int64_t v) { return v < 0 ? -v : v; };
  int64_t s = iabs(int64_t(go) - ge);
  s = s > d_ma ? s : d_ma;
  s = s > iabs(ge) ? s : iabs(ge);
  const int64_t lo = 2 * int64_t(go) + int64_t(n - 1) * ge - int64_t(cols) * iabs(ge);
  const int64_t hi = int64_t(n) * ma + (int64_t(m) + n + cols) * iabs(ge);
  return lo - 2 * s > -32000 && hi + 2 * s < 32000;
}

// The int16 direct form keeps the true values, with M carried as
// G = M + S_GO, and saturates.  Its diagonal constants relative to G are
// S_MA - S_GO (match), S_MI - S_GO (mismatch) and -S_GO (left of the read,
// where M stays 0).  They are formed as e * g + b from a byte e looked up
// per column pair (one byte permute, one packed multiply-add): b is the
// smallest constant, g the greatest common divisor of the others' distances
// to it, and every e must fit a byte.
struct DirectDelta {
  int32_t g, b, e_ma, e_mi, e_v;
};

__host__ __device__ inline int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a < 0 ? -a : a;
}

__host__ __device__ inline bool direct_delta(int32_t ma, int32_t mi, int32_t go, DirectDelta *d) {
  const int64_t c_ma = int64_t(ma) - go, c_mi = int64_t(mi) - go, c_v = -int64_t(go);
  int64_t b = c_ma < c_mi ? c_ma : c_mi;
  b = b < c_v ? b : c_v;
  const int64_t g0 = gcd64(gcd64(c_ma - b, c_mi - b), c_v - b);
  const int64_t g = g0 ? g0 : 1;
  const int64_t e_ma = (c_ma - b) / g, e_mi = (c_mi - b) / g, e_v = (c_v - b) / g;
  if (d) *d = DirectDelta{int32_t(g), int32_t(b), int32_t(e_ma), int32_t(e_mi), int32_t(e_v)};
  auto in16 = [](int64_t v) { return v >= -32000 && v <= 32000; };
  return e_ma <= 255 && e_mi <= 255 && e_v <= 255 && in16(c_ma) && in16(c_mi) && in16(c_v) &&
         in16(g) && in16(b);
}

// int16 direct form: a task runs there when the offset form's rule
// (int16_fits) fails but its read cannot push any value above int16: every
// value is at most n S_MA (plus the constants added on the way, bounded by
// |S_GO| + |S_GE|).  Low values saturate at -32768 instead of being ruled
// out: a saturated value only ever rises, and by at most S_MA per read
// column, so every value of column j that is wrong stays at or below
// B_j = -32768 + |S_GO| + j S_MA.  A cell of an optimal alignment of score
// S lies at or above S - (n - j) S_MA, so when S > B_n every such cell, and
// every comparison it wins or ties, is exact, and so are the score, the end
// and the traceback; tasks with S <= B_n (decided on the computed score,
// which exceeds B_n exactly when the true one does) are re-run in int32.
__host__ __device__ inline bool int16_direct_fits(int32_t n, int32_t ma, int32_t mi, int32_t go,
                                                  int32_t ge) {
  if (!direct_delta(ma, mi, go, nullptr)) return false;
  const int64_t hi = int64_t(n) * ma - int64_t(go) - int64_t(ge);
  return hi < 32000;
}

// The saturation floor of the direct form's result column, B_n above.
__host__ __device__ inline int32_t direct_floor(int32_t n, int32_t ma, int32_t go) {
  return -32768 - go + n * ma;
}

// Launch the int32 kernel of shape `s` (must be one of the compiled shapes);
// the variant with the byte-table diagonal runs when the scoring allows it
// (byte_delta_fits).
hipError_t launch_dp_i32(Shape s, int grid, hipStream_t stream, const DpParams &p);
// Occupancy (workgroups of one wave per CU) of the int32 kernel of shape `s`,
// byte-table variant or general one, full or score-only.
int occupancy_dp_i32(Shape s, bool byte_delta, bool score_only);
// The compiled int32 shapes.
const Shape *shapes_i32(int *count);

// Same for the packed int16 kernel (two tasks per lane, lo and hi halves),
// offset form or direct form.  `dense` asks for the variant built for more
// waves per SIMD where the shape has one (kernels with traceback at 13-14,
// 19-20 and 32 columns); other shapes ignore it.
hipError_t launch_dp_i16(Shape s, int grid, hipStream_t stream, const DpParams &p, bool direct,
                         bool dense);
int occupancy_dp_i16(Shape s, bool score_only, bool direct, bool dense);
// Whether the int16 kernel with traceback of shape `s` has the denser variant.
bool has_dense_dp_i16(Shape s);
const Shape *shapes_i16(int *count);
// Decision-scratch dwords of one workgroup slot.
uint64_t slot_dwords_i32(Shape s, int32_t max_m);
uint64_t slot_dwords_i16(Shape s, int32_t max_m);

}  // namespace soapdp
