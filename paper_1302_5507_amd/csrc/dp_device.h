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
// CIGAR.  The decision nibble of cell (i, j) has bit3 I extended, bit2 D
// extended, bit1 M not from the diagonal, bit0 M not from D.  `tr` serves
// nibbles from a window of cached decision words: `tr.get(i, j, nib)`
// returns false when the cell is outside the window, after which
// `tr.fill()` loads the window that holds it.
//
// The walk runs in rounds: every lane advances on cached words until it
// misses or finishes, then all missing lanes of the wavefront refill at once
// and wait for memory once.  One iteration per emitted operation; the state
// update is select-based so that lanes tracing different tasks stay
// converged.
template <class Tracer>
__device__ __forceinline__ void traceback_task(const DpParams &p, int64_t task, int32_t n, int32_t end,
                               int32_t slot_rows, Tracer &tr) {
  uint32_t *row = p.cigar + task * (int64_t)p.cigar_stride;
  int32_t wpos = p.cigar_stride;  // runs are written backward from the row end
  int32_t cur = 3, run = 0;       // current run (3: none yet)
  int32_t i = end, j = n, state = 0;  // 0 = M, 1 = D, 2 = I
  // Cells (i, j) with 1 <= i <= slot_rows and 1 <= j <= n lie inside the
  // task's decision slot; an end or length outside that range is never walked.
  bool bad = end < 1 || end > slot_rows || n < 1 || n > p.max_n;
  // Every iteration lowers i or j, so the walk ends within n + end steps.
  // The guard keeps a corrupted decision from reading outside the task.
  int32_t guard = bad ? 0 : n + end + 1;
  for (;;) {
    bool miss = false;
    for (; guard > 0; --guard) {
      if (state == 0 && (i == 0 || j == 0)) { guard = 0; break; }
      if (i < 1 || j < 1) { bad = true; guard = 0; break; }
      uint32_t nib;
      if (!tr.get(i, j, nib)) { miss = true; break; }
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
    if (!miss) break;
    tr.fill(i, j);
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

// Decision slot layout.  A slot holds ceil(steps / B) blocks of B sweep
// steps; block b, column group w is a run of 64 lanes x B words, lane-major:
// word (lane, u) of that run is the decision word of `lane` at step
// b * B + u.  The sweep writes one step at a time into an LDS staging
// buffer (`stage`, row stride kStageRow words so that rows start in
// different banks) and flushes a whole block with coalesced stores.
constexpr int kStageRow = kWave + 1;

template <class Word, int W, int B>
__device__ __forceinline__ void stage_step(Word *stage, int lane, int u, const Word (&v)[W]) {
#pragma unroll
  for (int w = 0; w < W; ++w) stage[(w * B + u) * kStageRow + lane] = v[w];
}

// Flush the staged block to `dst` (the block's first word).  Must be called
// by the whole wavefront; staged writes of all lanes are complete on entry.
// The run is written in 8-byte chunks, consecutive lanes to consecutive
// chunks (each store covers 512 contiguous bytes).  Chunk ci = lane + 64 s
// holds lane ci / CHUNKS's steps from (ci % CHUNKS) * PER on; since 64 is a
// multiple of CHUNKS, all chunks of a lane are one LDS base plus constant
// offsets.
template <class Word, int W, int B>
__device__ __forceinline__ void flush_block(const Word *stage, int lane, Word *dst) {
  constexpr int PER = 8 / (int)sizeof(Word);    // words per 8-byte chunk
  constexpr int CHUNKS = B / PER;              // chunks per lane and group
  static_assert(B % PER == 0 && kWave % CHUNKS == 0, "whole chunks per lane");
  const Word *src = stage + (lane % CHUNKS) * PER * kStageRow + lane / CHUNKS;
  uint2 *out = reinterpret_cast<uint2 *>(dst) + lane;
#pragma unroll
  for (int w = 0; w < W; ++w) {
#pragma unroll
    for (int s = 0; s < CHUNKS; ++s) {
      Word v[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) v[k] = src[(w * B + k) * kStageRow + s * (kWave / CHUNKS)];
      uint2 q;
      __builtin_memcpy(&q, v, 8);
      out[(w * CHUNKS + s) * kWave] = q;
      // one chunk at a time: the flush runs while the sweep's registers are
      // live, so it must not hold more than one chunk
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Decision words of one task as the traceback reads them.  Cell (i, j) (j
// counted from the read's first base) lies in strip column jp = j + pad - 1,
// i.e. lane lq = jp / K, column c = jp % K, group w = c / 8, and was computed
// at step ts = i - 1 + lq.  A block is the B steps of one (lq, w) holding ts.
// A refill loads up to NB blocks at once into this lane's LDS cache: the
// missed block, the one before it (the walk only goes to lower steps and
// columns), and the same two of the column group to the left (the previous
// lane's last group when w = 0, whose steps are one lower): one memory wait
// serves a diagonal run of about 2B rows and 16 columns.  `Decode(word, c)`
// extracts the nibble of column c.
// Blocks one refill loads: up to four, as many as the sweep's staging
// buffer (W groups of B steps per lane) has room for.
__host__ __device__ constexpr int tracer_blocks(int W) { return W < 4 ? W : 4; }

template <class Word, int K, int W, int B, class Decode>
struct BlockTracer {
  static constexpr int NB = tracer_blocks(W);
  const Word *slot;   // the task's slot
  Word *cache;        // NB * B LDS entries, 16-byte aligned
  int32_t lane0;      // first lane of the task in the wavefront
  int32_t pad;
  Decode decode;
  int32_t tag[NB];    // cached block k: (lq * W + w) << 20 | blk, -1 if none

  __device__ __forceinline__ static int32_t key(int32_t lq, int32_t w, int32_t blk) {
    return (lq * W + w) << 20 | blk;
  }
  // strip lane, column group, column and sweep step of cell (i, j)
  __device__ __forceinline__ void locate(int32_t i, int32_t j, int32_t &lq, int32_t &w, uint32_t &c,
                                         int32_t &ts) const {
    const uint32_t jp = (uint32_t)(j + pad - 1);
    lq = (int32_t)(jp / K);
    c = jp - (uint32_t)lq * K;
    w = (int32_t)(c >> 3);
    ts = i - 1 + lq;   // >= 0: i >= 1
  }
  __device__ __forceinline__ bool get(int32_t i, int32_t j, uint32_t &nib) {
    int32_t lq, w, ts;
    uint32_t c;
    locate(i, j, lq, w, c, ts);
    const int32_t k_ = key(lq, w, ts / B);
    int32_t hit = -1;
#pragma unroll
    for (int k = 0; k < NB; ++k) hit = tag[k] == k_ ? k : hit;
    if (hit < 0) return false;
    nib = decode(cache[hit * B + (ts & (B - 1))], c);
    return true;
  }
  // Refill after get(i, j) missed.
  __device__ __forceinline__ void fill(int32_t i, int32_t j) {
    constexpr int V = B * (int)sizeof(Word) / 16;
    int32_t lq0, w0, ts0;
    uint32_t c0;
    locate(i, j, lq0, w0, c0, ts0);
    // candidate blocks: (lq, w) at the missed step's block and the one
    // before, then the group to the left at its own steps
    const bool left_lane = w0 == 0;
    const int32_t lq2 = left_lane ? lq0 - 1 : lq0;
    const int32_t w2 = left_lane ? W - 1 : w0 - 1;
    const int32_t ts2 = left_lane ? ts0 - 1 : ts0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int32_t lq = k < 2 ? lq0 : lq2;
      const int32_t w = k < 2 ? w0 : w2;
      const int32_t blk = (k < 2 ? ts0 : ts2) / B - (k & 1);
      const bool ok = lq >= 0 && blk >= 0 && (k < 2 || ts2 >= 0);
      tag[k] = ok ? key(lq, w, blk) : -1;
      if (ok) {
        const uint4 *src = reinterpret_cast<const uint4 *>(
            slot + ((uint64_t)(blk * W + w) * kWave + (uint64_t)(lane0 + lq)) * B);
        uint4 *dst = reinterpret_cast<uint4 *>(cache + k * B);
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v] = src[v];
      }
    }
  }
};

template <class Word, int K, int W, int B, class Decode>
__device__ __forceinline__ BlockTracer<Word, K, W, B, Decode> make_tracer(
    const Word *slot, Word *cache, int32_t lane0, int32_t pad, Decode dec) {
  BlockTracer<Word, K, W, B, Decode> t{slot, cache, lane0, pad, dec};
#pragma unroll
  for (int k = 0; k < t.NB; ++k) t.tag[k] = -1;
  return t;
}

// LDS of one wavefront shared by the sweep's staging buffer and the
// traceback's block caches (never live at the same time).
template <class Word, int W, int B>
struct StageOrCache {
  static constexpr int kStageWords = W * B * kStageRow;
  static constexpr int kCacheWords = kWave * B * tracer_blocks(W);
  static constexpr int kWords = kStageWords > kCacheWords ? kStageWords : kCacheWords;
};

// Resolve the task order of a work item: entry `tix` of the (segment of the)
// task list, or `tix` itself.
__device__ __forceinline__ int64_t task_at(const DpParams &p, const int32_t *list, int64_t tix) {
  return list ? (int64_t)list[tix] : tix;
}

// The read words covering columns q0 .. q0+K-1 of a lane's strip (q = 0-based
// read index; negative q lie left of the read).  A strip of K <= 48 columns
// spans at most four words.  Loads stay inside the read's own words.
struct StripWords {
  uint32_t w0, w1, w2, w3;
  int32_t base;  // word index of w0
  // word i of the read is codes[first_word + i * stride]
  __device__ __forceinline__ void load(const uint32_t *codes, uint64_t first_word, int32_t n,
                                       int32_t q0, uint32_t stride) {
    const int32_t last = (n - 1) >> 4;
    base = (q0 > 0 ? q0 : 0) >> 4;
    const int32_t i0 = base < last ? base : last;
    const int32_t i1 = base + 1 < last ? base + 1 : last;
    const int32_t i2 = base + 2 < last ? base + 2 : last;
    const int32_t i3 = base + 3 < last ? base + 3 : last;
    w0 = codes[first_word + (uint64_t)i0 * stride];
    w1 = codes[first_word + (uint64_t)i1 * stride];
    w2 = codes[first_word + (uint64_t)i2 * stride];
    w3 = codes[first_word + (uint64_t)i3 * stride];
  }
  // code of read index q (0 <= q < n)
  __device__ __forceinline__ uint32_t code(int32_t q) const {
    const int32_t k = (q >> 4) - base;
    const uint32_t w = k == 0 ? w0 : (k == 1 ? w1 : (k == 2 ? w2 : w3));
    return (w >> ((q & 15) * 2)) & 3u;
  }
};

}  // namespace soapdp
