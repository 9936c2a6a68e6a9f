// Kernels of the multi-candidate call: reverse complements, ranking of each
// read's candidate regions by support with the effort-limit ceiling (paper,
// Methods section 4), the best / second-best reduction over the score-only
// pass, and the final fix-up.  One thread per read throughout; the
// alignments themselves run in the batched form's kernels.
#include "multi.h"

#include "../../include/soap_dp.h"

namespace soapdp {

namespace {

constexpr int kBlock = 64;

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

// Rank the valid candidates of read r by (support desc, index asc) and keep
// the first `ceiling` in a sorted list in LDS; candidates arrive in index
// order, so equal support never moves a later one ahead.
__global__ __launch_bounds__(kBlock) void select_kernel(MultiIn in, MultiWork w, MultiOut out) {
  // list entry k of thread x at [k][x]: the threads of a wavefront touch
  // consecutive words
  __shared__ int64_t s_idx[SOAP_DP_MAX_CEILING][kBlock];
  __shared__ int32_t s_sup[SOAP_DP_MAX_CEILING][kBlock];
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  const int x = threadIdx.x;
  auto idx = [&](int32_t k) -> int64_t & { return s_idx[k][x]; };
  auto sup = [&](int32_t k) -> int32_t & { return s_sup[k][x]; };
  const int32_t C = in.ceiling;
  uint8_t st;
  int32_t cnt = 0;
  if (read_ok(in, r, &st)) {
    const int64_t a = in.cand_start[r], b = in.cand_start[r + 1];
    if (a < 0 || b < a || b > in.n_cands) {
      st = kTaskInvalidOffset;
    } else {
      for (int64_t c = a; c < b; ++c) {
        const int32_t m = in.cand_len[c];
        if (m < 1 || m > in.max_m || in.cand_base_off[c] + (uint64_t)m > in.ref_words * 16) continue;
        const int32_t s = in.cand_support[c];
        if (cnt == C && s <= sup(C - 1)) continue;
        int32_t k = cnt < C ? cnt : C - 1;
        while (k > 0 && sup(k - 1) < s) {
          idx(k) = idx(k - 1);
          sup(k) = sup(k - 1);
          --k;
        }
        idx(k) = c;
        sup(k) = s;
        if (cnt < C) ++cnt;
      }
    }
  }
  const int32_t n = in.read_len[r];
  const uint64_t off = in.read_word_off[r];
  for (int32_t k = 0; k < C; ++k) {
    const int64_t t = r * C + k;
    if (k < cnt) {
      const int64_t c = idx(k);
      w.t_rwo[t] = off + (in.cand_strand[c] ? in.read_words : 0);
      w.t_rl[t] = n;
      w.t_rbo[t] = in.cand_base_off[c];
      w.t_ml[t] = in.cand_len[c];
      w.t_cand[t] = c;
    } else {   // empty slot: a zero-length task the batched form skips
      w.t_rwo[t] = 0;
      w.t_rl[t] = 0;
      w.t_rbo[t] = 0;
      w.t_ml[t] = 0;
      w.t_cand[t] = -1;
    }
  }
  out.n_aligned[r] = cnt;
  w.flag[r] = st != kTaskOk ? st : (cnt == 0 ? (uint8_t)SOAP_DP_TASK_NO_CANDIDATE : kTaskOk);
}

// Highest score, ties to the earlier rank; every other aligned candidate
// contributes to the second best.  The final task of a read is its best
// (read, candidate) pair, or a zero-length task.
__global__ __launch_bounds__(kBlock) void reduce_kernel(MultiIn in, MultiWork w, MultiOut out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  const int32_t C = in.ceiling;
  int32_t best = -1, best_s = 0, second = INT32_MIN;
  if (w.flag[r] == kTaskOk) {
    const int32_t cnt = out.n_aligned[r];
    for (int32_t k = 0; k < cnt; ++k) {
      const int64_t t = r * C + k;
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
    const int64_t t = r * C + best;
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
  hipLaunchKernelGGL(select_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w, out);
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
