// Kernels of the multi-candidate call (effort limit: only the best
// `ceiling` candidate regions of a read, ranked by support, are aligned).
#pragma once
#include "dp_internal.h"

namespace soapdp {

// Inputs of the candidate stage (device pointers; see soap_dp_multi_batch).
struct MultiIn {
  const uint32_t *read_codes;
  const uint64_t *read_word_off;
  const int32_t *read_len;
  uint64_t read_words;
  const int64_t *cand_start;
  const uint64_t *cand_base_off;
  const int32_t *cand_len;
  const int32_t *cand_support;
  const uint8_t *cand_strand;
  uint64_t ref_words;
  int64_t n_reads, n_cands;
  int32_t max_n, max_m, ceiling;
  int64_t n_slots;   // task slots: min(n_cands, n_reads * ceiling)
};

// Work arrays.  Tasks are dense: read r's ranked candidates are tasks
// off[r] .. off[r] + n_aligned[r] - 1 (rank order), and slots from
// off[n_reads] on are zero-length.  The read buffer `reads2` holds the reads
// (words [0, read_words)) and their reverse complements at the same offsets
// plus read_words.
struct MultiWork {
  uint32_t *reads2;
  int64_t *off;    // n_reads + 1 task offsets
  int64_t *bsum;   // per block of reads: count, then its exclusive offset
  uint64_t *t_rwo, *t_rbo;
  int32_t *t_rl, *t_ml;
  int64_t *t_cand;
  int32_t *p_score, *p_begin, *p_end, *p_clen;   // score-only pass results
  uint8_t *p_status;
  uint64_t *f_rwo, *f_rbo;                        // final task per read
  int32_t *f_rl, *f_ml;
  uint8_t *flag;                                  // per read: 0 or the read's final status
};

// Outputs written beside the final alignment (see soap_dp_multi_result).
struct MultiOut {
  int32_t *score, *ref_begin, *ref_end, *cigar_len;
  uint8_t *status;
  int64_t *best_cand;
  int32_t *second_score;
  int32_t *n_aligned;
};

// Reverse complements of the valid reads into reads2 (after the reads were
// copied there).
hipError_t launch_revcomp(const MultiIn &in, const MultiWork &w, hipStream_t stream);
// Count, place and rank each read's candidates under the ceiling; fill the
// task slots.
hipError_t launch_select(const MultiIn &in, const MultiWork &w, const MultiOut &out,
                         hipStream_t stream);
// Best and second best per read from the score-only pass; final tasks.
hipError_t launch_reduce(const MultiIn &in, const MultiWork &w, const MultiOut &out,
                         hipStream_t stream);
// Reads without a result: status and zero outputs.
hipError_t launch_fixup(const MultiIn &in, const MultiWork &w, const MultiOut &out,
                        hipStream_t stream);

}  // namespace soapdp
