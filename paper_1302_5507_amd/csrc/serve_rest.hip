// Device-side packing of the long CIGAR rows' rests for the served form.
#include "serve_rest.h"

namespace soapdp {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(64) void clear_hdr_kernel(int32_t *hdr) {
  if (threadIdx.x < 2) hdr[threadIdx.x] = 0;
}

// One thread per task; only the long rows (a few per hundred thousand for
// short reads) reserve and copy.
__global__ __launch_bounds__(kBlock) void pack_rest_kernel(const uint32_t *cigar, int32_t stride,
                                                           const int32_t *cigar_len, int32_t n,
                                                           int32_t head, int32_t *hdr,
                                                           RestRow *rows, int32_t max_rows,
                                                           uint32_t *words, int32_t max_words) {
  const int32_t t = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
  if (t >= n) return;
  const int32_t len = min(max(cigar_len[t], 0), stride);
  if (len <= head) return;
  const int32_t need = len - head;
  const int32_t k = atomicAdd(&hdr[0], 1);
  if (k >= max_rows) return;
  const int32_t off = atomicAdd(&hdr[1], need);
  const bool fits = off <= max_words - need;
  rows[k] = RestRow{t, fits ? off : -1};
  if (!fits) return;
  const uint32_t *src = cigar + (int64_t)t * stride + head;
  for (int32_t w = 0; w < need; ++w) words[off + w] = src[w];
}

}  // namespace

hipError_t launch_pack_cigar_rest(const uint32_t *cigar, int32_t stride, const int32_t *cigar_len,
                                  int32_t n, int32_t head, int32_t *hdr, RestRow *rows,
                                  int32_t max_rows, uint32_t *words, int32_t max_words,
                                  hipStream_t stream) {
  hipLaunchKernelGGL(clear_hdr_kernel, dim3(1), dim3(64), 0, stream, hdr);
  if (n > 0)
    hipLaunchKernelGGL(pack_rest_kernel, dim3((uint32_t)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, stream, cigar, stride, cigar_len, n, head, hdr, rows, max_rows, words,
                       max_words);
  return hipGetLastError();
}

}  // namespace soapdp
