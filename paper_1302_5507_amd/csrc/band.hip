// Band kernels of the two-pass traceback (see band.h for why the band holds
// every optimal alignment).
#include "band.h"

namespace soapdp {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int band_bin(int32_t len, int32_t max_m) {
  const int64_t b = int64_t(len) * kBandBins / (int64_t(max_m) + 1);
  return int(b < kBandBins ? b : kBandBins - 1);
}

__global__ void band_zero_kernel(int32_t *bins) {
  for (int i = threadIdx.x; i < 2 * kBandBins; i += blockDim.x) bins[i] = 0;
}

// One thread per task: the rows [i0, e) that can hold an optimal alignment
// of a task pass 1 scored; a task pass 1 left final (invalid, below the
// score threshold, or traced back already: ref_begin >= 0) gets an empty
// window and is restored by the fixup.
__global__ __launch_bounds__(kBlock) void band_kernel(BandIn in, BandWork w) {
  __shared__ int32_t s_cnt[kBandBins];
  for (int k = threadIdx.x; k < kBandBins; k += kBlock) s_cnt[k] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < in.n_tasks) {
    const uint8_t st = w.p_status[t];
    uint64_t rbo = in.ref_base_off[t];
    int32_t len = 0, i0 = -1;
    if ((st == kTaskOk || st == kTaskRedone) && w.p_begin[t] < 0) {
      const int64_t n = in.read_len[t], S = w.p_score[t], e = w.p_end[t];
      int64_t lo = 0;
      if (in.ge < 0) {
        const int64_t num = n * in.ma + in.go - S;
        const int64_t dmax = num < 0 ? 0 : 1 + num / (-int64_t(in.ge));
        lo = e - n - dmax;
        lo = lo > 0 ? lo : 0;
      }
      i0 = (int32_t)lo;
      rbo += (uint64_t)lo;
      len = (int32_t)(e - lo);
    }
    w.b_rbo[t] = rbo;
    w.b_ml[t] = len;
    w.b_i0[t] = i0;
    atomicAdd(&s_cnt[band_bin(len, in.max_m)], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kBandBins; k += kBlock)
    if (s_cnt[k]) atomicAdd(&w.bins[k], s_cnt[k]);
}

// One thread: bin counts to starting cursors.
__global__ void band_scan_kernel(int32_t *bins) {
  if (threadIdx.x != 0) return;
  int32_t acc = 0;
  for (int k = 0; k < kBandBins; ++k) {
    bins[kBandBins + k] = acc;
    acc += bins[k];
  }
}

__global__ __launch_bounds__(kBlock) void band_scatter_kernel(BandIn in, BandWork w) {
  __shared__ int32_t s_cnt[kBandBins], s_base[kBandBins];
  for (int k = threadIdx.x; k < kBandBins; k += kBlock) s_cnt[k] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int b = 0, rank = 0;
  if (t < in.n_tasks) {
    b = band_bin(w.b_ml[t], in.max_m);
    rank = atomicAdd(&s_cnt[b], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kBandBins; k += kBlock)
    s_base[k] = s_cnt[k] ? atomicAdd(&w.bins[kBandBins + k], s_cnt[k]) : 0;
  __syncthreads();
  if (t < in.n_tasks) w.order[s_base[b] + rank] = (int32_t)t;
}

__global__ __launch_bounds__(kBlock) void band_fixup_kernel(int64_t n_tasks, BandWork w,
                                                            BandOut out) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n_tasks) return;
  const int32_t i0 = w.b_i0[t];
  if (i0 >= 0) {
    const uint8_t st = out.status[t];
    if (st == kTaskOk || st == kTaskRedone) {
      out.ref_end[t] += i0;
      out.ref_begin[t] += i0;
      // the int32 kernels served this task in either pass
      out.status[t] = (st == kTaskRedone || w.p_status[t] == kTaskRedone) ? kTaskRedone : kTaskOk;
    }
  } else {
    out.score[t] = w.p_score[t];
    out.ref_begin[t] = w.p_begin[t];
    out.ref_end[t] = w.p_end[t];
    out.cigar_len[t] = w.p_clen[t];
    out.status[t] = w.p_status[t];
  }
}

}  // namespace

hipError_t launch_band(const BandIn &in, const BandWork &w, hipStream_t stream) {
  if (in.n_tasks <= 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)((in.n_tasks + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(band_zero_kernel, dim3(1), dim3(128), 0, stream, w.bins);
  hipLaunchKernelGGL(band_kernel, dim3(blocks), dim3(kBlock), 0, stream, in, w);
  hipLaunchKernelGGL(band_scan_kernel, dim3(1), dim3(64), 0, stream, w.bins);
  hipLaunchKernelGGL(band_scatter_kernel, dim3(blocks), dim3(kBlock), 0, stream, in, w);
  return hipGetLastError();
}

hipError_t launch_band_fixup(int64_t n_tasks, const BandWork &w, const BandOut &out,
                             hipStream_t stream) {
  if (n_tasks <= 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)((n_tasks + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(band_fixup_kernel, dim3(blocks), dim3(kBlock), 0, stream, n_tasks, w, out);
  return hipGetLastError();
}

}  // namespace soapdp
