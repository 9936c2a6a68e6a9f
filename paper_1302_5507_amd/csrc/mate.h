// Kernels of the mate-rescue call: candidate regions from the aligned end,
// the fragment length range and the orientation (paper, Results: step 2;
// Methods: paired-end alignment), and the final fix-up.
#pragma once
#include "dp_internal.h"

namespace soapdp {

// Inputs (device pointers; see soap_dp_mate_batch).
struct MateIn {
  const uint32_t *read_codes;
  const uint64_t *read_word_off;
  const int32_t *read_len;
  uint64_t read_words;
  const uint64_t *mate_pos;
  const int32_t *mate_len;
  const uint8_t *mate_strand;
  uint64_t ref_len;
  int64_t n_reads;
  int32_t max_n, min_frag, max_frag;
  bool same_strand;   // the mate lies on the aligned end's strand
  bool upstream;      // the mate lies upstream of the aligned end
};

// Work arrays: one task per pair; `reads2` holds the reads (words
// [0, read_words)) and the reverse complements of the reverse-strand mates
// at the same offsets plus read_words.
struct MateWork {
  uint32_t *reads2;
  uint64_t *t_rwo, *t_rbo;
  int32_t *t_rl, *t_ml;
  uint8_t *flag;   // per pair: 0, or the pair's final status
};

// Outputs written beside the alignment (see soap_dp_mate_result).
struct MateOut {
  int32_t *score, *ref_begin, *ref_end, *cigar_len;
  uint8_t *status;
  uint64_t *window_off;
  int32_t *window_len;
  uint8_t *strand;
};

// Regions, strands, reverse complements and tasks (after the reads were
// copied into reads2).
hipError_t launch_mate_windows(const MateIn &in, const MateWork &w, const MateOut &out,
                               hipStream_t stream);
// Pairs without a result: status and zero outputs.
hipError_t launch_mate_fixup(const MateIn &in, const MateWork &w, const MateOut &out,
                             hipStream_t stream);

}  // namespace soapdp
