// Kernels of the mate-rescue call.  One thread per pair: the candidate
// region where the fragment length range and the orientation place the
// unaligned end (paper, Results: step 2; Methods: paired-end alignment),
// its strand, the reverse complement of a reverse-strand mate, and the
// pair's task for the batched or plain form.
#include "mate.h"

#include "../../include/soap_dp.h"

namespace soapdp {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void mate_window_kernel(MateIn in, MateWork w, MateOut out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  const int32_t n = in.read_len[r];
  const int32_t n1 = in.mate_len[r];
  const uint64_t off = in.read_word_off[r];
  uint8_t flag = kTaskOk;
  int64_t lo = 0, hi = 0;
  uint8_t strand = 0;
  if (n < 1 || n > in.max_n || n1 < 1) {
    flag = kTaskInvalidLen;
  } else if (off + (uint64_t)((n + 15) >> 4) > in.read_words) {
    flag = kTaskInvalidOffset;
  } else {
    const int64_t G = (int64_t)in.ref_len;
    // any start at or past `far` leaves the region empty in both
    // directions, so clamping keeps the arithmetic in range
    const uint64_t far = in.ref_len + (uint64_t)max(in.max_frag, in.max_n) + 1;
    const int64_t p = (int64_t)min(in.mate_pos[r], far);
    const uint8_t s = in.mate_strand[r] ? 1 : 0;
    const bool higher = (s == 0) != in.upstream;
    if (higher) {
      lo = p + in.min_frag - n;
      hi = p + in.max_frag;
    } else {
      lo = p + n1 - in.max_frag;
      hi = p + n1 - in.min_frag + n;
    }
    lo = max(lo, (int64_t)0);
    hi = min(hi, G);
    strand = in.same_strand ? s : (uint8_t)(1 - s);
    if (hi <= lo) flag = (uint8_t)SOAP_DP_TASK_NO_CANDIDATE;
  }
  w.flag[r] = flag;
  if (flag != kTaskOk) {   // a zero-length task; the fix-up writes the outputs
    w.t_rwo[r] = 0;
    w.t_rl[r] = 0;
    w.t_rbo[r] = 0;
    w.t_ml[r] = 0;
    return;
  }
  if (strand) {   // reverse complement beside the copy of the reads
    const uint32_t *src = in.read_codes + off;
    uint32_t *dst = w.reads2 + in.read_words + off;
    for (int32_t q = 0; q < (n + 15) / 16; ++q) {
      uint32_t word = 0;
      for (int32_t b = 0; b < 16; ++b) {
        const int32_t j = q * 16 + b;   // position in the reverse complement
        if (j >= n) break;
        const int32_t k = n - 1 - j;    // its source base
        word |= (3u - ((src[k >> 4] >> (2 * (k & 15))) & 3u)) << (2 * b);
      }
      dst[q] = word;
    }
  }
  w.t_rwo[r] = off + (strand ? in.read_words : 0);
  w.t_rl[r] = n;
  w.t_rbo[r] = (uint64_t)lo;
  w.t_ml[r] = (int32_t)(hi - lo);
  out.window_off[r] = (uint64_t)lo;
  out.window_len[r] = (int32_t)(hi - lo);
  out.strand[r] = strand;
}

__global__ __launch_bounds__(kBlock) void mate_fixup_kernel(MateIn in, MateWork w, MateOut out) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= in.n_reads) return;
  const uint8_t f = w.flag[r];
  if (f == kTaskOk) return;
  out.status[r] = f;
  out.score[r] = 0;
  out.ref_begin[r] = 0;
  out.ref_end[r] = 0;
  out.cigar_len[r] = 0;
  out.window_off[r] = 0;
  out.window_len[r] = 0;
  out.strand[r] = 0;
}

dim3 grid_of(int64_t n) { return dim3((uint32_t)((n + kBlock - 1) / kBlock)); }

}  // namespace

hipError_t launch_mate_windows(const MateIn &in, const MateWork &w, const MateOut &out,
                               hipStream_t stream) {
  hipLaunchKernelGGL(mate_window_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w, out);
  return hipGetLastError();
}

hipError_t launch_mate_fixup(const MateIn &in, const MateWork &w, const MateOut &out,
                             hipStream_t stream) {
  hipLaunchKernelGGL(mate_fixup_kernel, grid_of(in.n_reads), dim3(kBlock), 0, stream, in, w, out);
  return hipGetLastError();
}

}  // namespace soapdp
