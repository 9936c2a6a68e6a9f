// Kernels of the multi-candidate call: reverse complements, ranking of each
// read's candidate regions by support with the effort-limit ceiling (paper,
// Methods section 4), the best / second-best reduction over the score-only
// pass, and the final fix-up.  One thread per read throughout; the
// alignments themselves run in the batched form's kernels.
#include "multi.h"

#include "../../include/soap_dp.h"

namespace soapdp {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ bool read_ok(const MultiIn &in, int64_t r, uint8_t *status) {
  const int32_t n = in.read_len[r];
  if (n < 1 || n > in.max_n) {
    *status = kTaskInvalidLen;
    return false;
  }
  if (in.read_word_off[r] + (uint64_t)((n + 15) >> 4) > in.read_words) {
    *status = kTaskInvalidOffset;
    return false;
  }
  *status = kTaskOk;
  return true;
}

__global__ __launch_bounds__(kBlock) void revcomp_kernel(MultiIn in, MultiWork w) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  uint8_t st;
  if (!read_ok(in, r, &st)) return;
  const int32_t n = in.read_len[r];
  const uint64_t off = in.read_word_off[r];
  const uint32_t *src = in.read_codes + off;
  uint32_t *dst = w.reads2 + in.read_words + off;
  for (int32_t q = 0; q < (n + 15) / 16; ++q) {
    uint32_t word = 0;
    for (int32_t b = 0; b < 16; ++b) {
      const int32_t j = q * 16 + b;        // position in the reverse complement
      if (j >= n) break;
      const int32_t s = n - 1 - j;         // its source base
      const uint32_t code = (src[s >> 4] >> (2 * (s & 15))) & 3u;
      word |= (3u - code) << (2 * b);
    }
    dst[q] = word;
  }
}

__device__ __forceinline__ bool cand_ok(const MultiIn &in, int64_t c) {
  const int32_t m = in.cand_len[c];
  return m >= 1 && m <= in.max_m && in.cand_base_off[c] + (uint64_t)m <= in.ref_words * 16;
}

// Per read: validity and the number of valid candidates kept under the
// ceiling (its task count).  A list that runs backwards (cand_start[r+1] <
// cand_start[r]) makes the lists of other reads overlap, whatever read r's
// own status: its count is written as -1, which the scan turns into the
// mark kBadList that condemns the whole call.
__global__ __launch_bounds__(kBlock) void count_kernel(MultiIn in, MultiWork w, MultiOut out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  const int64_t a = in.cand_start[r], b = in.cand_start[r + 1];
  uint8_t st;
  int64_t valid = 0;
  if (read_ok(in, r, &st)) {
    if (a < 0 || b < a || b > in.n_cands)
      st = kTaskInvalidOffset;
    else
      for (int64_t c = a; c < b; ++c) valid += cand_ok(in, c) ? 1 : 0;
  }
  const int32_t cnt = st == kTaskOk ? (int32_t)min(valid, (int64_t)in.ceiling) : 0;
  out.n_aligned[r] = b < a ? -1 : cnt;
  w.flag[r] = st != kTaskOk ? st : (cnt == 0 ? (uint8_t)SOAP_DP_TASK_NO_CANDIDATE : kTaskOk);
}

// Exclusive scan of the task counts in three steps: within blocks of
// kScanBlock reads, over the block sums (one workgroup), then the block
// offsets added back.  Every sum saturates at kBadList, far above any real
// total (at most n_reads * ceiling), so a backwards list anywhere leaves
// the total, off[n_reads], at exactly kBadList without overflow; a
// well-formed call never reaches it.
constexpr int kScanPer = 4;
constexpr int kScanBlock = kBlock * kScanPer;
constexpr int64_t kBadList = int64_t(1) << 48;

__device__ __forceinline__ int64_t sat_add(int64_t x, int64_t y) { return min(x + y, kBadList); }

__device__ __forceinline__ bool call_is_bad(const MultiIn &in, const MultiWork &w) {
  return w.off[in.n_reads] >= kBadList;
}

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *s_tmp, int64_t *total) {
  // Hillis-Steele over the workgroup in LDS
  const int x = threadIdx.x;
  s_tmp[x] = v;
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {
    const int64_t add = x >= d ? s_tmp[x - d] : 0;
    __syncthreads();
    s_tmp[x] = sat_add(s_tmp[x], add);
    __syncthreads();
  }
  const int64_t incl = s_tmp[x];
  *total = s_tmp[kBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kBlock) void scan_local_kernel(MultiIn in, MultiWork w, MultiOut out) {
  __shared__ int64_t s_tmp[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer], sum = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int32_t n = base + j < in.n_reads ? out.n_aligned[base + j] : 0;
    v[j] = n < 0 ? kBadList : n;
    sum = sat_add(sum, v[j]);
  }
  int64_t total;
  int64_t run = block_exclusive_scan(sum, s_tmp, &total);
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    if (base + j < in.n_reads) w.off[base + j] = run;
    run = sat_add(run, v[j]);
  }
  if (threadIdx.x == 0) w.bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void scan_blocks_kernel(MultiIn in, MultiWork w, int64_t nb) {
  __shared__ int64_t s_tmp[kBlock];
  // each thread scans a contiguous chunk of the block sums
  const int64_t per = (nb + kBlock - 1) / kBlock;
  const int64_t a = min((int64_t)threadIdx.x * per, nb), b = min(a + per, nb);
  int64_t sum = 0;
  for (int64_t k = a; k < b; ++k) sum = sat_add(sum, w.bsum[k]);
  int64_t total;
  int64_t run = block_exclusive_scan(sum, s_tmp, &total);
  for (int64_t k = a; k < b; ++k) {
    const int64_t c = w.bsum[k];
    w.bsum[k] = run;
    run = sat_add(run, c);
  }
  if (threadIdx.x == 0) w.off[in.n_reads] = total;
}

__global__ __launch_bounds__(kBlock) void scan_add_kernel(MultiIn in, MultiWork w) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  w.off[r] = sat_add(w.off[r], w.bsum[r / kScanBlock]);
}

// Every slot emptied (a zero-length task the batched form skips) before
// the ranking fills the live ones: slots past the last task stay empty, and
// a malformed candidate list cannot leave an earlier call's task behind.
__global__ __launch_bounds__(kBlock) void pad_kernel(MultiIn in, MultiWork w) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= in.n_slots) return;
  w.t_rwo[t] = 0;
  w.t_rl[t] = 0;
  w.t_rbo[t] = 0;
  w.t_ml[t] = 0;
  w.t_cand[t] = -1;
}

// Per candidate: its rank among the valid candidates of its read by
// (support desc, index asc) -- the number of valid candidates ahead of it;
// a rank under the ceiling places the candidate at task off[r] + rank.
__global__ __launch_bounds__(kBlock) void rank_kernel(MultiIn in, MultiWork w) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= in.n_cands || call_is_bad(in, w)) return;
  // owning read: the last r with cand_start[r] <= c (cand_start is
  // non-decreasing in a call that is not condemned)
  int64_t lo = 0, hi = in.n_reads - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (in.cand_start[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int64_t r = lo;
  if (w.flag[r] != kTaskOk || !cand_ok(in, c)) return;
  const int64_t a = in.cand_start[r], b = in.cand_start[r + 1];
  if (c < a || c >= b) return;
  const int32_t s = in.cand_support[c];
  const int32_t C = in.ceiling;
  int32_t rank = 0;
  for (int64_t d = a; d < b && rank < C; ++d) {
    if (d == c || !cand_ok(in, d)) continue;
    const int32_t sd = in.cand_support[d];
    rank += (sd > s || (sd == s && d < c)) ? 1 : 0;
  }
  const int64_t t = w.off[r] + rank;
  if (rank >= C || t >= in.n_slots) return;   // (t < n_slots holds here; kept as a guard)
  w.t_rwo[t] = in.read_word_off[r] + (in.cand_strand[c] ? in.read_words : 0);
  w.t_rl[t] = in.read_len[r];
  w.t_rbo[t] = in.cand_base_off[c];
  w.t_ml[t] = in.cand_len[c];
  w.t_cand[t] = c;
}

// Highest score, ties to the earlier rank; every other aligned candidate
// contributes to the second best.  The final task of a read is its best
// (read, candidate) pair, or a zero-length task.
__global__ __launch_bounds__(kBlock) void reduce_kernel(MultiIn in, MultiWork w, MultiOut out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  int32_t best = -1, best_s = 0, second = INT32_MIN;
  const int64_t t0 = w.off[r];
  if (call_is_bad(in, w)) {
    w.flag[r] = kTaskInvalidOffset;   // overlapping lists: every read rejected
  } else if (w.flag[r] == kTaskOk) {
    const int32_t cnt = out.n_aligned[r];
    for (int32_t k = 0; k < cnt && t0 + k < in.n_slots; ++k) {
      const int64_t t = t0 + k;
      const uint8_t ts = w.p_status[t];
      if (ts != kTaskOk && ts != kTaskRedone) continue;
      const int32_t s = w.p_score[t];
      if (best < 0 || s > best_s) {
        if (best >= 0) second = max(second, best_s);
        best = k;
        best_s = s;
      } else {
        second = max(second, s);
      }
    }
    if (best < 0) w.flag[r] = SOAP_DP_TASK_NO_CANDIDATE;
  }
  if (best >= 0) {
    const int64_t t = t0 + best;
    w.f_rwo[r] = w.t_rwo[t];
    w.f_rl[r] = w.t_rl[t];
    w.f_rbo[r] = w.t_rbo[t];
    w.f_ml[r] = w.t_ml[t];
    out.best_cand[r] = w.t_cand[t];
  } else {
    w.f_rwo[r] = 0;
    w.f_rl[r] = 0;
    w.f_rbo[r] = 0;
    w.f_ml[r] = 0;
    out.best_cand[r] = -1;
  }
  out.second_score[r] = second;
}

__global__ __launch_bounds__(kBlock) void fixup_kernel(MultiIn in, MultiWork w, MultiOut out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  const uint8_t f = w.flag[r];
  if (f == kTaskOk) return;
  out.status[r] = f;
  out.score[r] = 0;
  out.ref_begin[r] = 0;
  out.ref_end[r] = 0;
  out.cigar_len[r] = 0;
  out.best_cand[r] = -1;
  out.second_score[r] = INT32_MIN;
  if (f != SOAP_DP_TASK_NO_CANDIDATE) out.n_aligned[r] = 0;
}

dim3 grid_of(int64_t n) { return dim3((uint32_t)((n + kBlock - 1) / kBlock)); }

}  // namespace

hipError_t launch_revcomp(const MultiIn &in, const MultiWork &w, hipStream_t stream) {
  hipLaunchKernelGGL(revcomp_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w);
  return hipGetLastError();
}

hipError_t launch_select(const MultiIn &in, const MultiWork &w, const MultiOut &out,
                         hipStream_t stream) {
  const int64_t nb = (in.n_reads + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(count_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w, out);
  hipLaunchKernelGGL(scan_local_kernel, dim3((uint32_t)nb), dim3(kBlock), 0, stream, in, w, out);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kBlock), 0, stream, in, w, nb);
  hipLaunchKernelGGL(scan_add_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w);
  if (in.n_slots > 0)
    hipLaunchKernelGGL(pad_kernel, grid_of(in.n_slots), dim3(kBlock), 0, stream, in, w);
  if (in.n_cands > 0)
    hipLaunchKernelGGL(rank_kernel, grid_of(in.n_cands), dim3(kBlock), 0, stream, in, w);
  return hipGetLastError();
}

hipError_t launch_reduce(const MultiIn &in, const MultiWork &w, const MultiOut &out,
                         hipStream_t stream) {
  hipLaunchKernelGGL(reduce_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w, out);
  return hipGetLastError();
}

hipError_t launch_fixup(const MultiIn &in, const MultiWork &w, const MultiOut &out,
                        hipStream_t stream) {
  hipLaunchKernelGGL(fixup_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w, out);
  return hipGetLastError();
}

}  // namespace soapdp
