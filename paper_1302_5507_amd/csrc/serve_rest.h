// Packing, on the device, of the CIGAR words past the dense head of the
// rare rows longer than it, so that a served batch brings them back with
// its other copies and the host needs no further transfer or wait.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "serve_host.h"

namespace soapdp {

// Enqueue on `stream`: hdr[0] and hdr[1] are cleared, then every task
// t < n whose row (cigar_len[t], clamped to the stride) is longer than
// `head` words reserves a row entry (hdr[0]) and room for its rest
// (hdr[1]) and copies words [head, len) of its row to words[off ..].
// Rows past `max_rows` entries are not listed; a listed row whose rest
// does not fit `max_words` gets off = -1.  hdr[0] ends as the number of
// long rows and hdr[1] as the words the listed ones asked for (at most
// max_rows * stride); either may exceed its capacity.  The order of the
// listed rows is not fixed.
hipError_t launch_pack_cigar_rest(const uint32_t *cigar, int32_t stride, const int32_t *cigar_len,
                                  int32_t n, int32_t head, int32_t *hdr, RestRow *rows,
                                  int32_t max_rows, uint32_t *words, int32_t max_words,
                                  hipStream_t stream);

}  // namespace soapdp
