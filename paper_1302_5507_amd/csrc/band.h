// Kernels of the two-pass traceback: a score-only pass gives each task its
// score S and end e; only window rows [i0, e) can hold an optimal alignment,
// and the pass with decision bits and traceback runs on that sub-window.
//
// Why the band holds (paper, Methods section 3, recurrences and base cases):
// an alignment of the whole read that deletes k >= 1 window bases scores at
// most n S_MA + S_GO + (k - 1) S_GE, since every read base adds at most S_MA
// and k deleted bases in g runs cost g S_GO + (k - g) S_GE <= S_GO +
// (k - 1) S_GE.  An optimal alignment scores S, so with S_GE < 0 it deletes
// at most Dmax = 1 + floor((n S_MA + S_GO - S) / |S_GE|) bases (none when
// n S_MA + S_GO < S) and spans at most n + Dmax window rows ending at e:
// every optimal alignment ending at e starts at row >= i0 = max(0, e - n -
// Dmax).  Every cell on an optimal path then has an optimal prefix inside
// the band, and any candidate that ties with it does too, so the sub-window
// run takes the same tie-broken decisions, reaches the same score, and its
// smallest best end is e - i0.  With S_GE = 0 nothing bounds the deletions
// and the whole window is kept.
#pragma once
#include "dp_internal.h"

namespace soapdp {

constexpr int kBandBins = 256;   // band-length bins of the pass-2 task order

// Work arrays of a two-pass call (context-owned, n_tasks entries each).
struct BandWork {
  int32_t *p_score, *p_begin, *p_end, *p_clen;   // pass-1 (score-only) results
  uint8_t *p_status;
  uint64_t *b_rbo;    // pass-2 window: base offset ...
  int32_t *b_ml;      // ... and length (0: the task is final after pass 1)
  int32_t *b_i0;      // rows dropped before the band (-1: not banded)
  int32_t *order;     // pass-2 task order, by band length
  int32_t *bins;      // kBandBins counts, then kBandBins cursors
};

// Inputs the band kernel reads besides the pass-1 results.
struct BandIn {
  const uint64_t *ref_base_off;
  const int32_t *read_len;
  const int32_t *ref_len;
  int64_t n_tasks;
  int32_t max_m;
  int32_t ma, go, ge;
};

// Bands of every task, then the pass-2 order (tasks grouped by band length,
// so that a work item's tasks sweep similar numbers of rows).
hipError_t launch_band(const BandIn &in, const BandWork &w, hipStream_t stream);

// Merge: banded tasks get pass-2 outputs shifted back to window
// coordinates; the others keep their pass-1 outputs.
struct BandOut {
  int32_t *score, *ref_begin, *ref_end, *cigar_len;
  uint8_t *status;
};
hipError_t launch_band_fixup(int64_t n_tasks, const BandWork &w, const BandOut &out,
                             hipStream_t stream);

}  // namespace soapdp
