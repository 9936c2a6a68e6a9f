// Device helpers shared by the DP kernels.
#pragma once
#include "dp_internal.h"

namespace soapdp {

__device__ __forceinline__ int32_t wave_shr1(int32_t v) {
  // DPP wave_shr:1 -- lane k receives lane k-1; lane 0 receives 0.
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}

// Shift every value one lane to the right inside groups of L lanes: lane k
// receives lane k-1, and the first lane of each group receives `first_val`.
// With L = 16 the groups are DPP rows and with L = 64 the whole wavefront,
// so the DPP "old" operand supplies the boundary at no cost; other group
// sizes patch the first lanes with one select.
template <int L>
__device__ __forceinline__ int32_t group_shr1(int32_t v, int32_t first_val, bool first) {
  if constexpr (L == 16) {
    return __builtin_amdgcn_update_dpp(first_val, v, 0x111, 0xf, 0xf, false);   // row_shr:1
  } else if constexpr (L == 64) {
    return __builtin_amdgcn_update_dpp(first_val, v, 0x138, 0xf, 0xf, false);   // wave_shr:1
  } else {
    const int32_t s = __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
    return first ? first_val : s;
  }
}

// First work item of a persistent workgroup is its own index; later ones
// come from the shared counter (so a launch with no work makes no atomics).
__device__ __forceinline__ int64_t next_item(int32_t *counter, int lane) {
  int32_t v = 0;
  if (lane == 0) v = atomicAdd(counter, 1);
  return (int64_t)__builtin_amdgcn_readfirstlane(v) + gridDim.x;
}

__device__ __forceinline__ uint32_t push_sign(uint32_t acc, int32_t diff) {
  // (acc << 1) | (diff < 0): shift the sign bit of `diff` into the accumulator.
  return __builtin_amdgcn_alignbit(acc, (uint32_t)diff, 31);
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Walk the decision nibbles of one task back from (end, n) and write its
// CIGAR.  `nib_at(i, j)` returns the decision nibble of cell (i, j):
// bit3 I extended, bit2 D extended, bit1 M not from the diagonal, bit0 M not
// from D.  One iteration per emitted operation; the state update is
// select-based so that lanes tracing different tasks stay converged.
template <class NibFn>
__device__ void traceback_task(const DpParams &p, int64_t task, int32_t n, int32_t end,
                               NibFn nib_at) {
  uint32_t *row = p.cigar + task * (int64_t)p.cigar_stride;
  int32_t wpos = p.cigar_stride;  // runs are written backward from the row end
  int32_t cur = 3, run = 0;       // current run (3: none yet)
  int32_t i = end, j = n, state = 0;  // 0 = M, 1 = D, 2 = I
  // Cells (i, j) with 1 <= i <= max_m and 1 <= j <= n lie inside the task's
  // decision slot; an end or length outside that range is never walked.
  bool bad = end < 1 || end > p.max_m || n < 1 || n > p.max_n;
  // Every iteration lowers i or j, so the walk ends within n + end steps.
  // The guard keeps a corrupted decision from reading outside the task.
  for (int32_t guard = bad ? 0 : n + end + 1; guard > 0; --guard) {
    if (state == 0 && (i == 0 || j == 0)) break;
    if (i < 1 || j < 1) { bad = true; break; }
    const uint32_t nib = nib_at(i, j);
    const bool in_m = state == 0;
    const bool diag = in_m && !(nib & 2u);
    const bool to_d = in_m ? ((nib & 3u) == 2u) : state == 1;   // M from D, or still in D
    const int32_t op = diag ? 0 : (to_d ? 2 : 1);              // M = 0, I = 1, D = 2
    const int32_t next = diag ? 0 : (to_d ? ((nib & 4u) ? 1 : 0) : ((nib & 8u) ? 2 : 0));
    if (op != cur && run > 0) {
      if (wpos > 0) row[--wpos] = (uint32_t)run << 4 | (uint32_t)cur;
      else bad = true;
    }
    run = op == cur ? run + 1 : 1;
    cur = op;
    i -= op != 1;   // M and D consume a region base
    j -= op != 2;   // M and I consume a read base
    state = next;
  }
  int32_t begin = i;
  if (!bad && state == 0 && i == 0 && j > 0) {   // base case M(0, j): j insertions
    if (cur == 1) {
      run += j;
    } else {
      if (run > 0) {
        if (wpos > 0) row[--wpos] = (uint32_t)run << 4 | (uint32_t)cur;
        else bad = true;
      }
      cur = 1;
      run = j;
    }
    begin = 0;
  }
  if (run > 0) {
    if (wpos > 0) row[--wpos] = (uint32_t)run << 4 | (uint32_t)cur;
    else bad = true;
  }
  const int32_t cnt = p.cigar_stride - wpos;
  for (int32_t k = 0; k < cnt; ++k) row[k] = row[wpos + k];
  p.cigar_len[task] = bad ? 0 : cnt;
  p.ref_begin[task] = bad ? 0 : begin;
  if (bad) p.status[task] = kTaskInvalidLen;
}

// Per-lane cache of one (lane, column-group) word over four consecutive
// sweep steps [top - 3, top], held in LDS (`slots` points at this lane's four
// entries): a diagonal or vertical move of the traceback usually stays inside
// it, and a refill issues its four loads at once.
template <class Word>
struct StepCache {
  int32_t lq = -1, w = -1, top = -1;
  // `base` points at step 0 of this (lq, w); consecutive steps are `stride`
  // Words apart.  Steps below 0 are clamped to 0 (never used).
  __device__ __forceinline__ Word get(Word *slots, const Word *base, int32_t ts, int32_t lq_,
                                      int32_t w_, uint32_t stride) {
    uint32_t d = (uint32_t)(top - ts);
    if (lq_ != lq || w_ != w || d > 3u) {
      lq = lq_;
      w = w_;
      top = ts;
      d = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t tk = ts - k > 0 ? ts - k : 0;
        slots[k] = base[(uint64_t)(uint32_t)tk * stride];
      }
    }
    return slots[d];
  }
};

// Resolve the task order of a work item: entry `tix` of the (segment of the)
// task list, or `tix` itself.
__device__ __forceinline__ int64_t task_at(const DpParams &p, const int32_t *list, int64_t tix) {
  return list ? (int64_t)list[tix] : tix;
}

// The read words covering columns q0 .. q0+K-1 of a lane's strip (q = 0-based
// read index; negative q lie left of the read).  A strip of K <= 32 columns
// spans at most three words.  Loads stay inside the read's own words.
struct StripWords {
  uint32_t w0, w1, w2;
  int32_t base;  // word index of w0
  __device__ __forceinline__ void load(const uint32_t *codes, uint64_t first_word, int32_t n,
                                       int32_t q0) {
    const int32_t last = (n - 1) >> 4;
    base = (q0 > 0 ? q0 : 0) >> 4;
    const int32_t i0 = base < last ? base : last;
    const int32_t i1 = base + 1 < last ? base + 1 : last;
    const int32_t i2 = base + 2 < last ? base + 2 : last;
    w0 = codes[first_word + (uint64_t)i0];
    w1 = codes[first_word + (uint64_t)i1];
    w2 = codes[first_word + (uint64_t)i2];
  }
  // code of read index q (0 <= q < n)
  __device__ __forceinline__ uint32_t code(int32_t q) const {
    const int32_t k = (q >> 4) - base;
    const uint32_t w = k == 0 ? w0 : (k == 1 ? w1 : w2);
    return (w >> ((q & 15) * 2)) & 3u;
  }
};

}  // namespace soapdp
