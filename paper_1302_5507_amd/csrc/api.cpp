// Host side of the C ABI declared in include/soap_dp.h: argument checking,
// the context and its workspace, kernel-shape choice and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/soap_dp.h"
#include "dp_internal.h"

using namespace soapdp;

struct soap_dp_ctx {
  int device = 0;
  int cu_count = 0;
  int last_hip_error = 0;
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  void *small = nullptr;       // counters and other small device state
  size_t small_bytes = 0;
};

namespace {

constexpr size_t kSmallBytes = 4096;

// Scratch budget: the decision bits of every workgroup in flight.
constexpr size_t kScratchCap = size_t(8) << 30;

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool scoring_ok(const soap_dp_scoring *sc) {
  if (!sc) return false;
  const int32_t lim = SOAP_DP_MAX_SCORE_ABS;
  auto in = [&](int32_t v) { return v >= -lim && v <= lim; };
  return in(sc->match) && in(sc->mismatch) && in(sc->gap_open) && in(sc->gap_extend) &&
         sc->match > 0 && sc->mismatch < sc->match && sc->gap_open < 0 &&
         sc->gap_open <= sc->gap_extend && sc->gap_extend <= 0;
}

int batch_ok(const soap_dp_batch *in, const soap_dp_result *out) {
  if (!in || !out) return SOAP_DP_EINVAL;
  if (in->n_tasks < 0 || in->n_tasks > (int64_t(1) << 31) - 1) return SOAP_DP_EINVAL;
  if (in->max_n < 1 || in->max_n > SOAP_DP_MAX_READ) return SOAP_DP_EINVAL;
  if (in->max_m < 1 || in->max_m > SOAP_DP_MAX_WINDOW) return SOAP_DP_EINVAL;
  if (out->cigar_stride < 2 * in->max_n - 1) return SOAP_DP_EINVAL;
  if (in->n_tasks == 0) return SOAP_DP_OK;
  if (!in->read_codes || !in->read_word_off || !in->read_len || !in->ref_codes ||
      !in->ref_base_off || !in->ref_len || in->read_words == 0 || in->ref_words == 0)
    return SOAP_DP_EINVAL;
  if (!out->score || !out->ref_begin || !out->ref_end || !out->cigar || !out->cigar_len ||
      !out->status)
    return SOAP_DP_EINVAL;
  return SOAP_DP_OK;
}

// Plain form: the compiled shape covering max_n with the least work per task
// (columns times sweep steps, the anti-diagonal skew included).
Shape plain_shape(int32_t max_n, int32_t max_m) {
  int cnt = 0;
  const Shape *all = shapes_i32(&cnt);
  Shape best{0, 0};
  double best_cost = 0;
  for (int k = 0; k < cnt; ++k) {
    const Shape s = all[k];
    if (s.lanes * s.cells < max_n) continue;
    if (s.lanes == 1 && max_n > 8) continue;
    const double cost = double(s.lanes) * s.cells * double(max_m + s.lanes - 1);
    if (best.lanes == 0 || cost < best_cost) { best = s; best_cost = cost; }
  }
  return best;
}

uint64_t slot_dwords_for(Shape s, int32_t max_m) {
  const uint64_t steps = uint64_t(max_m) + uint64_t(s.lanes) - 1;
  const uint64_t w = uint64_t((s.cells + 7) / 8);
  return steps * w * kWave;
}

int grid_for(const soap_dp_ctx *ctx, Shape s, int64_t n_tasks, int32_t max_m) {
  const int64_t per_wave = kWave / s.lanes;
  const int64_t items = (n_tasks + per_wave - 1) / per_wave;
  int occ = occupancy_dp_i32(s);
  if (occ < 1) occ = 1;
  int64_t grid = int64_t(ctx->cu_count) * occ;
  const uint64_t slot_bytes = slot_dwords_for(s, max_m) * 4;
  const int64_t cap = int64_t(kScratchCap / slot_bytes);
  grid = std::min<int64_t>(grid, std::max<int64_t>(cap, 1));
  grid = std::min<int64_t>(grid, std::max<int64_t>(items, 1));
  return int(grid);
}

int hip_fail(soap_dp_ctx *ctx, hipError_t e) {
  ctx->last_hip_error = int(e);
  return SOAP_DP_EHIP;
}

int ensure_scratch(soap_dp_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return SOAP_DP_OK;
  if (ctx->scratch) {
    // earlier work may still read the old buffer
    if (hipDeviceSynchronize() != hipSuccess) return SOAP_DP_EHIP;
    (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return SOAP_DP_ENOMEM;
  }
  ctx->scratch = p;
  ctx->scratch_bytes = bytes;
  return SOAP_DP_OK;
}

DpParams make_params(const soap_dp_batch *in, const soap_dp_scoring *sc, const soap_dp_result *out) {
  DpParams p{};
  p.read_codes = in->read_codes;
  p.read_word_off = in->read_word_off;
  p.read_len = in->read_len;
  p.ref_codes = in->ref_codes;
  p.ref_base_off = in->ref_base_off;
  p.ref_len = in->ref_len;
  p.n_tasks = in->n_tasks;
  p.read_words = in->read_words;
  p.ref_words = in->ref_words;
  p.max_n = in->max_n;
  p.max_m = in->max_m;
  p.ma = sc->match;
  p.mi = sc->mismatch;
  p.go = sc->gap_open;
  p.ge = sc->gap_extend;
  p.score = out->score;
  p.ref_begin = out->ref_begin;
  p.ref_end = out->ref_end;
  p.cigar = out->cigar;
  p.cigar_stride = out->cigar_stride;
  p.cigar_len = out->cigar_len;
  p.status = out->status;
  return p;
}

int align_plain(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                const soap_dp_result *out, hipStream_t stream) {
  const Shape s = plain_shape(in->max_n, in->max_m);
  if (s.lanes == 0) return SOAP_DP_EINVAL;
  const int grid = grid_for(ctx, s, in->n_tasks, in->max_m);
  const uint64_t slot = slot_dwords_for(s, in->max_m);
  const int rc = ensure_scratch(ctx, size_t(grid) * slot * 4);
  if (rc) return rc;
  DpParams p = make_params(in, sc, out);
  p.scratch = static_cast<uint32_t *>(ctx->scratch);
  p.slot_dwords = slot;
  const hipError_t e = launch_dp_i32(s, grid, stream, p);
  if (e != hipSuccess) return hip_fail(ctx, e);
  return SOAP_DP_OK;
}

}  // namespace

extern "C" {

int soap_dp_create(soap_dp_ctx **out, int device_ordinal) {
  if (!out) return SOAP_DP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return SOAP_DP_ENODEV;
  }
  if (device_ordinal < 0 || device_ordinal >= ndev) return SOAP_DP_EINVAL;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device_ordinal) != hipSuccess) return SOAP_DP_ENODEV;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SOAP_DP_ENODEV;
  auto *ctx = new (std::nothrow) soap_dp_ctx();
  if (!ctx) return SOAP_DP_ENOMEM;
  ctx->device = device_ordinal;
  ctx->cu_count = prop.multiProcessorCount;
  {
    DeviceGuard dg(device_ordinal);
    if (hipMalloc(&ctx->small, kSmallBytes) != hipSuccess) {
      delete ctx;
      return SOAP_DP_ENOMEM;
    }
    ctx->small_bytes = kSmallBytes;
  }
  *out = ctx;
  return SOAP_DP_OK;
}

int soap_dp_destroy(soap_dp_ctx *ctx) {
  if (!ctx) return SOAP_DP_EINVAL;
  {
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->small) (void)hipFree(ctx->small);
  }
  delete ctx;
  return SOAP_DP_OK;
}

int soap_dp_align_batch(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                        const soap_dp_result *out, void *stream, uint32_t flags) {
  if (!ctx) return SOAP_DP_EINVAL;
  if (!scoring_ok(sc)) return SOAP_DP_EINVAL;
  int rc = batch_ok(in, out);
  if (rc) return rc;
  if (flags != SOAP_DP_PLAIN && flags != SOAP_DP_BATCHED) return SOAP_DP_EINVAL;
  if (in->n_tasks == 0) return SOAP_DP_OK;
  DeviceGuard dg(ctx->device);
  return align_plain(ctx, in, sc, out, static_cast<hipStream_t>(stream));
}

size_t soap_dp_workspace_bytes(const soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n,
                               int32_t max_m, uint32_t flags) {
  (void)flags;
  if (!ctx || n_tasks <= 0 || max_n < 1 || max_n > SOAP_DP_MAX_READ || max_m < 1 ||
      max_m > SOAP_DP_MAX_WINDOW)
    return 0;
  const Shape s = plain_shape(max_n, max_m);
  if (s.lanes == 0) return 0;
  const int grid = grid_for(ctx, s, n_tasks, max_m);
  return size_t(grid) * slot_dwords_for(s, max_m) * 4 + ctx->small_bytes;
}

int soap_dp_reserve(soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                    uint32_t flags) {
  if (!ctx) return SOAP_DP_EINVAL;
  const size_t b = soap_dp_workspace_bytes(ctx, n_tasks, max_n, max_m, flags);
  if (b == 0) return SOAP_DP_EINVAL;
  DeviceGuard dg(ctx->device);
  return ensure_scratch(ctx, b - ctx->small_bytes);
}

const char *soap_dp_strerror(int code) {
  switch (code) {
    case SOAP_DP_OK: return "ok";
    case SOAP_DP_EINVAL: return "invalid argument (scoring, pointer, size or stride)";
    case SOAP_DP_ENOMEM: return "device workspace allocation failed";
    case SOAP_DP_EHIP: return "HIP runtime error";
    case SOAP_DP_ENODEV: return "no usable gfx950 device";
    default: return "unknown error";
  }
}

int soap_dp_last_hip_error(const soap_dp_ctx *ctx) { return ctx ? ctx->last_hip_error : 0; }

}  // extern "C"
