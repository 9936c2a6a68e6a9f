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
  // Decision-bit scratch: one slot of `slot_dwords` per workgroup of the grid.
  uint32_t *scratch;
  uint64_t slot_dwords;
  // Optional task order (nullptr: identity) and its length; work items are
  // groups of (tasks per wave) consecutive entries of that order.
  const int32_t *task_list;
  const int32_t *task_count;   // device count overriding n_tasks when non-null
  // Optional dynamic work counter (nullptr: static grid-stride schedule).
  int32_t *work_counter;
};

// A kernel shape: L lanes cooperate on one task, each owning K read columns.
struct Shape {
  int lanes;
  int cells;
};

// Launch the int32 kernel of shape `s` (must be one of the compiled shapes).
hipError_t launch_dp_i32(Shape s, int grid, hipStream_t stream, const DpParams &p);
// Occupancy (workgroups of one wave per CU) of the int32 kernel of shape `s`.
int occupancy_dp_i32(Shape s);
// The compiled int32 shapes.
const Shape *shapes_i32(int *count);

}  // namespace soapdp
