// Host side of the C ABI declared in include/soap_dp.h: argument checking,
// the context and its workspace, kernel-shape choice, the batched form's
// class launches and graph cache, and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/soap_dp.h"
#include "band.h"
#include "batch.h"
#include "ctx_internal.h"
#include "dp_internal.h"
#include "mate.h"
#include "multi.h"

using namespace soapdp;

namespace {

constexpr size_t kScratchCap = size_t(16) << 30;  // decision-bit scratch budget
constexpr size_t kForkStreams = 2;   // forked streams of a large batched call (see enqueue_batched)
constexpr int64_t kSpreadTasks = 262144;   // below: one forked stream per class
// Small device buffer (int32 units): hist | max_m | offset | cursor |
// work_counter | defer, then two uint64 tables (slot_dwords, scratch_off),
// then the int32 re-run's task count and work counter.
constexpr int kSmallInts = 6 * kMaxClasses + 4 * kMaxClasses + 4;
constexpr int kGraphCacheMax = 16;

// Kernel kind of a launch: which int32 diagonal variant (byte table,
// general, or -- for sizing before the scoring is known -- whichever holds
// more workgroups; int16 kernels have one) and whether only scores are
// computed.
enum Variant { kGeneral = 0, kByte = 1, kEither = 2 };

struct ClassSpec {
  int prec;          // kPrecI16 (offset form), kPrecI16Direct or kPrecI32
  int cap;           // upper bound on read length
  Shape shape;       // kernel shape with traceback
  Shape score_shape; // kernel shape of the score-only kernels ({0, 0}: as `shape`)
  // int32 classes under scorings that need the general (compare and
  // select) diagonal: their own shapes ({0, 0}: as above)
  Shape gen_shape{0, 0};
  Shape gen_score_shape{0, 0};
};

// The shape a class runs with: score-only kernels carry no decision words,
// so fewer lanes with more columns each can pay off for them; the int32
// general diagonal holds a code and a constant per column, so it may prefer
// other shapes than the byte table.
Shape shape_of(const ClassSpec &c, bool score, Variant v = kByte) {
  if (v == kGeneral && c.prec == kPrecI32) {
    const Shape g = score && c.gen_score_shape.lanes ? c.gen_score_shape : c.gen_shape;
    if (g.lanes) return g;
  }
  return score && c.score_shape.lanes ? c.score_shape : c.shape;
}

// What the class kernels of one batched call compute: everything, score and
// end only, or -- the first pass of a two-pass call -- per class: score and
// end where the windows are long against the class's reads (the band pass
// will then trace back over a fraction of them), everything where they are
// not (the band would cover most of the window, so one pass is cheaper).
enum Mode { kModeFull = 0, kModeScore = 1, kModeMixed = 2 };
// A class takes two passes when the batch's windows reach this many times
// its longest read.  The score pass costs about half a decision pass per
// cell, so two passes pay off while the band is under about half the
// window; with the band about n + a few dozen rows, that is m >= 3 n or so.
constexpr int32_t kBandRatio = 3;
// Autotuner: rank of an int16 shape with traceback that has a denser
// variant, relative to its timing (see autotune).
constexpr double kDenseRank = 1.02;

bool class_score(const ClassSpec &c, int32_t max_m, Mode mode) {
  return mode == kModeScore || (mode == kModeMixed && int64_t(max_m) >= int64_t(kBandRatio) * c.cap);
}

// Default classes: int16 in the offset form by ascending capacity, the same
// capacities and shapes in the direct form (tasks the offset form's range
// rule excludes), then the int32 classes for tasks neither int16 form
// covers.  Shapes are replaced by the autotuner; a direct-form class always
// runs the shape of the offset-form class of its capacity.
const ClassSpec kDefaultClasses[] = {
    {16, 16, {2, 8}},    {16, 32, {4, 8}},    {16, 40, {4, 10}},   {16, 56, {8, 7}},
    {16, 64, {8, 8}},    {16, 80, {8, 10}},   {16, 104, {8, 13}},  {16, 128, {8, 16}},
    {16, 152, {8, 19}},  {16, 192, {16, 12}}, {16, 256, {16, 16}}, {16, 320, {32, 10}},
    {16, 384, {32, 12}}, {16, 512, {32, 16}},
    {17, 16, {2, 8}},    {17, 32, {4, 8}},    {17, 40, {4, 10}},   {17, 56, {8, 7}},
    {17, 64, {8, 8}},    {17, 80, {8, 10}},   {17, 104, {8, 13}},  {17, 128, {8, 16}},
    {17, 152, {8, 19}},  {17, 192, {16, 12}}, {17, 256, {16, 16}}, {17, 320, {32, 10}},
    {17, 384, {32, 12}}, {17, 512, {32, 16}},
    {32, 36, {4, 9}},    {32, 56, {8, 7}},    {32, 80, {8, 10}},   {32, 104, {8, 13}},
    {32, 152, {8, 19}},  {32, 256, {16, 16}}, {32, 512, {32, 16}},
};
static_assert(sizeof(kDefaultClasses) / sizeof(kDefaultClasses[0]) <= kMaxClasses, "class table");

// Direct-form classes mirror the offset-form class of the same capacity.
void mirror_direct_shapes(std::vector<ClassSpec> &cls) {
  for (auto &d : cls)
    if (d.prec == kPrecI16Direct)
      for (const auto &o : cls)
        if (o.prec == kPrecI16 && o.cap == d.cap) {
          d.shape = o.shape;
          d.score_shape = o.score_shape;
        }
}

// What a captured batched call depends on: every pointer and size of the
// batch and the outputs, the scoring, the context's buffer epoch and the
// flags.  Compared field by field (the ABI structs carry padding whose
// bytes are unspecified).
struct GraphKey {
  soap_dp_batch in;
  soap_dp_scoring sc;
  soap_dp_result out;
  const int32_t *order;
  uint64_t epoch;
  uint32_t flags;
  uint32_t read_stride;
};

bool same_batch(const soap_dp_batch &a, const soap_dp_batch &b) {
  return a.read_codes == b.read_codes && a.read_word_off == b.read_word_off &&
         a.read_len == b.read_len && a.ref_codes == b.ref_codes &&
         a.ref_base_off == b.ref_base_off && a.ref_len == b.ref_len && a.n_tasks == b.n_tasks &&
         a.max_n == b.max_n && a.max_m == b.max_m && a.read_words == b.read_words &&
         a.ref_words == b.ref_words;
}

bool same_scoring(const soap_dp_scoring &a, const soap_dp_scoring &b) {
  return a.match == b.match && a.mismatch == b.mismatch && a.gap_open == b.gap_open &&
         a.gap_extend == b.gap_extend && a.min_score == b.min_score;
}

bool same_result(const soap_dp_result &a, const soap_dp_result &b) {
  return a.score == b.score && a.ref_begin == b.ref_begin && a.ref_end == b.ref_end &&
         a.cigar == b.cigar && a.cigar_stride == b.cigar_stride && a.cigar_len == b.cigar_len &&
         a.status == b.status;
}

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
  uint64_t last_use;
};

bool same_key(const GraphKey &a, const GraphKey &b) {
  return same_batch(a.in, b.in) && same_scoring(a.sc, b.sc) && same_result(a.out, b.out) &&
         a.order == b.order && a.epoch == b.epoch && a.flags == b.flags &&
         a.read_stride == b.read_stride;
}

}  // namespace

struct soap_dp_ctx {
  int device = 0;
  int cu_count = 0;
  int last_hip_error = 0;
  std::string arch;
  // workspace
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  int32_t *small = nullptr;          // bucketing tables and class plans (kSmallInts)
  uint8_t *task_class = nullptr;
  int32_t *task_list = nullptr;
  int32_t *redo_list = nullptr;   // tasks the direct-form kernels flag for the int32 re-run
  int64_t task_cap = 0;
  // batched form
  std::vector<ClassSpec> classes;
  hipStream_t capture_stream = nullptr;
  // class kernels run on streams forked from the caller's stream after
  // bucketing (one join event each; see enqueue_batched)
  std::vector<hipStream_t> class_streams;
  std::vector<hipEvent_t> join_events;
  hipEvent_t fork_event = nullptr;
  std::vector<GraphEntry> graphs;
  uint64_t epoch = 1;   // bumped whenever buffers or shapes change
  // occupancy per kernel shape (key prec << 16 | lanes << 8 | cells), queried
  // once: launch planning runs on every call
  mutable std::unordered_map<uint32_t, int> occupancy;
  uint64_t use_clock = 0;
  // Replay batched calls as captured hipGraphs (opt-in, SOAPDP_GRAPHS=1):
  // off by default since host crashes of unknown cause were seen only in
  // processes that captured and replayed graphs.
  bool use_graphs = false;
  // serving: no growth, no graph capture (see ctx_set_frozen)
  bool frozen = false;
  // multi-candidate work arrays (task slots, reverse complements)
  void *multi = nullptr;
  size_t multi_bytes = 0;
  // two-pass work arrays (pass-1 results, bands, pass-2 order)
  void *band = nullptr;
  size_t band_bytes = 0;
  // this device's copy of the fixed array behind soap_dp_align_batch_noalloc
  char *fixed = nullptr;
};

namespace {

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

// The scoring the kernels see: min_score only counts under SOAP_DP_MIN_SCORE.
soap_dp_scoring effective_scoring(const soap_dp_scoring *sc, uint32_t flags) {
  soap_dp_scoring s = *sc;
  if ((flags & SOAP_DP_MIN_SCORE) == 0) s.min_score = INT32_MIN;
  return s;
}

int batch_ok(const soap_dp_batch *in, const soap_dp_result *out, bool score_only) {
  if (!in || !out) return SOAP_DP_EINVAL;
  if (in->n_tasks < 0 || in->n_tasks > (int64_t(1) << 31) - 1) return SOAP_DP_EINVAL;
  if (in->max_n < 1 || in->max_n > SOAP_DP_MAX_READ) return SOAP_DP_EINVAL;
  if (in->max_m < 1 || in->max_m > SOAP_DP_MAX_WINDOW) return SOAP_DP_EINVAL;
  if (!score_only && out->cigar_stride < 2 * in->max_n - 1) return SOAP_DP_EINVAL;
  if (in->n_tasks == 0) return SOAP_DP_OK;
  if (!in->read_codes || !in->read_word_off || !in->read_len || !in->ref_codes ||
      !in->ref_base_off || !in->ref_len || in->read_words == 0 || in->ref_words == 0)
    return SOAP_DP_EINVAL;
  if (!out->score || !out->ref_begin || !out->ref_end || !out->cigar_len || !out->status ||
      (!score_only && !out->cigar))
    return SOAP_DP_EINVAL;
  return SOAP_DP_OK;
}

bool shape_compiled(int prec, Shape s) {
  int cnt = 0;
  const Shape *all = packed16(prec) ? shapes_i16(&cnt) : shapes_i32(&cnt);
  for (int k = 0; k < cnt; ++k)
    if (all[k].lanes == s.lanes && all[k].cells == s.cells) return true;
  return false;
}

struct Kind {
  Variant v;
  bool score;
  bool dense = false;   // int16 kernels with traceback: the variant for more waves per SIMD
};

Kind kind_for(const soap_dp_scoring *sc, bool score) {
  return Kind{byte_delta_fits(sc->match, sc->mismatch, sc->gap_open, sc->gap_extend) ? kByte
                                                                                      : kGeneral,
              score};
}

int occupancy(const soap_dp_ctx *ctx, int prec, Shape s, Kind k) {
  if (prec == 32 && k.v == kEither)
    return std::max(occupancy(ctx, prec, s, Kind{kGeneral, k.score}),
                    occupancy(ctx, prec, s, Kind{kByte, k.score}));
  const bool dense = k.dense && packed16(prec);
  const uint32_t key = uint32_t(dense) << 27 | uint32_t(k.score) << 26 | uint32_t(k.v) << 24 |
                       uint32_t(prec) << 16 | uint32_t(s.lanes) << 8 | uint32_t(s.cells);
  auto it = ctx->occupancy.find(key);
  if (it != ctx->occupancy.end()) return it->second;
  int o = packed16(prec) ? occupancy_dp_i16(s, k.score, prec == kPrecI16Direct, dense)
                         : occupancy_dp_i32(s, k.v == kByte, k.score);
  o = o < 1 ? 1 : o;
  ctx->occupancy.emplace(key, o);
  return o;
}

uint64_t slot_dwords(int prec, Shape s, int32_t max_m) {
  return packed16(prec) ? slot_dwords_i16(s, max_m) : slot_dwords_i32(s, max_m);
}

// Plain form: the compiled int32 shape covering max_n with the least work
// per task (columns times sweep steps, the anti-diagonal skew included).
// Among shapes of equal columns that prefers fewer lanes with more columns
// each, which also spreads each step's fixed work (neighbour shifts, table,
// end tracking) over more columns.
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

// Persistent grid of one launch: every resident workgroup slot, limited by
// the scratch budget and by the work available.
int grid_for(const soap_dp_ctx *ctx, int prec, Shape s, int64_t n_tasks, int32_t max_m, Kind k) {
  const int64_t per_wave = (packed16(prec) ? 2 : 1) * kWave / s.lanes;
  const int64_t items = (n_tasks + per_wave - 1) / per_wave;
  int64_t grid = int64_t(ctx->cu_count) * occupancy(ctx, prec, s, k);
  const uint64_t slot_bytes = slot_dwords(prec, s, max_m) * 4;
  grid = std::min<int64_t>(grid, std::max<int64_t>(int64_t(kScratchCap / slot_bytes), 1));
  grid = std::min<int64_t>(grid, std::max<int64_t>(items, 1));
  return int(grid);
}

int hip_fail(soap_dp_ctx *ctx, hipError_t e) {
  ctx->last_hip_error = int(e);
  (void)hipGetLastError();
  return SOAP_DP_EHIP;
}

// Drop every cached graph.  A cached graph may have been launched moments
// ago (the caller's stream does not wait for the host), so the device is
// synchronised before an executable graph is destroyed.
void clear_graphs(soap_dp_ctx *ctx) {
  if (!ctx->graphs.empty()) (void)hipDeviceSynchronize();
  for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
  ++ctx->epoch;
}

int ensure_scratch(soap_dp_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return SOAP_DP_OK;
  if (ctx->frozen) return SOAP_DP_ENOMEM;
  if (ctx->scratch) {
    if (hipDeviceSynchronize() != hipSuccess) return SOAP_DP_EHIP;   // earlier work may read it
    (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  clear_graphs(ctx);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return SOAP_DP_ENOMEM;
  }
  ctx->scratch = p;
  ctx->scratch_bytes = bytes;
  return SOAP_DP_OK;
}

int ensure_task_buffers(soap_dp_ctx *ctx, int64_t n_tasks) {
  if (n_tasks <= ctx->task_cap) return SOAP_DP_OK;
  if (ctx->frozen) return SOAP_DP_ENOMEM;
  if (ctx->task_list) {
    if (hipDeviceSynchronize() != hipSuccess) return SOAP_DP_EHIP;
    (void)hipFree(ctx->task_list);
    (void)hipFree(ctx->task_class);
    (void)hipFree(ctx->redo_list);
    ctx->task_list = nullptr;
    ctx->task_class = nullptr;
    ctx->redo_list = nullptr;
    ctx->task_cap = 0;
  }
  clear_graphs(ctx);
  const int64_t cap = std::max<int64_t>(n_tasks, 1024);
  if (hipMalloc(reinterpret_cast<void **>(&ctx->task_list), size_t(cap) * 4) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&ctx->task_class), size_t(cap)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&ctx->redo_list), size_t(cap) * 4) != hipSuccess) {
    (void)hipGetLastError();
    if (ctx->task_list) (void)hipFree(ctx->task_list);
    if (ctx->task_class) (void)hipFree(ctx->task_class);
    ctx->task_list = nullptr;
    ctx->task_class = nullptr;
    ctx->redo_list = nullptr;
    return SOAP_DP_ENOMEM;
  }
  ctx->task_cap = cap;
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
  p.ok_status = kTaskOk;
  p.min_score = sc->min_score;
  p.defer = 1;
  p.read_stride = 1;
  return p;
}

// Work items of one launch and the tasks each serves.
int64_t tasks_per_item(int prec, Shape s) { return (packed16(prec) ? 2 : 1) * kWave / s.lanes; }

// Grid, traceback deferral and scratch of one kernel launch.
struct LaunchPlan {
  int grid = 0;
  int defer = 1;
  uint64_t slot_dwords = 0;
  size_t bytes() const { return (size_t(grid) * size_t(defer) * slot_dwords * 4 + 255) & ~size_t(255); }
};

// Deferral: as many slots per workgroup as one traceback pass has lanes for,
// but no more than the work items a workgroup can expect, and within
// `budget` bytes of scratch.
LaunchPlan plan_launch(const soap_dp_ctx *ctx, int prec, Shape s, int64_t n_tasks, int32_t max_m,
                       Kind k, size_t budget) {
  LaunchPlan q;
  q.grid = grid_for(ctx, prec, s, n_tasks, max_m, k);
  if (k.score) {   // no decision scratch
    q.slot_dwords = 0;
    q.defer = 1;
    return q;
  }
  q.slot_dwords = slot_dwords(prec, s, max_m);
  const int64_t per = tasks_per_item(prec, s);
  const int64_t items = (n_tasks + per - 1) / per;
  const int64_t per_block = (items + q.grid - 1) / q.grid;
  q.defer = int(std::max<int64_t>(1, std::min<int64_t>(kWave / per, per_block)));
  while (q.defer > 1 && q.bytes() > budget) --q.defer;
  return q;
}

hipError_t launch_shape(int prec, Shape s, int grid, hipStream_t stream, const DpParams &p,
                        bool dense = false) {
  return packed16(prec) ? launch_dp_i16(s, grid, stream, p, prec == kPrecI16Direct, dense)
                        : launch_dp_i32(s, grid, stream, p);
}

// Device tables of the bucketing and the class plans, carved from `small`.
BucketBuffers bucket_buffers(const soap_dp_ctx *ctx) {
  BucketBuffers b{};
  b.task_class = ctx->task_class;
  b.task_list = ctx->task_list;
  b.hist = ctx->small;
  b.max_m = ctx->small + kMaxClasses;
  b.offset = ctx->small + 2 * kMaxClasses;
  b.cursor = ctx->small + 3 * kMaxClasses;
  b.work_counter = ctx->small + 4 * kMaxClasses;
  b.defer = ctx->small + 5 * kMaxClasses;
  b.slot_dwords = reinterpret_cast<uint64_t *>(ctx->small + 6 * kMaxClasses);
  b.scratch_off = reinterpret_cast<uint64_t *>(ctx->small + 8 * kMaxClasses);
  b.redo_count = ctx->small + 10 * kMaxClasses;
  b.redo_work_counter = ctx->small + 10 * kMaxClasses + 1;
  b.redo_list = ctx->redo_list;
  return b;
}

// ------------------------------------------------------------------ plain

size_t plain_scratch_bytes(const soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                           Kind k) {
  const Shape s = plain_shape(max_n, max_m);
  if (s.lanes == 0) return 0;
  return plan_launch(ctx, 32, s, n_tasks, max_m, k, kScratchCap).bytes();
}

int align_plain(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                const soap_dp_result *out, hipStream_t stream, bool score,
                const int32_t *order = nullptr, uint32_t read_stride = 1) {
  const Shape s = plain_shape(in->max_n, in->max_m);
  if (s.lanes == 0) return SOAP_DP_EINVAL;
  const LaunchPlan q = plan_launch(ctx, 32, s, in->n_tasks, in->max_m, kind_for(sc, score), kScratchCap);
  const int rc = ensure_scratch(ctx, q.bytes());
  if (rc) return rc;
  DpParams p = make_params(in, sc, out);
  p.score_only = score;
  p.scratch = static_cast<uint32_t *>(ctx->scratch);
  p.slot_dwords = q.slot_dwords;
  p.defer = q.defer;
  // work queue: waves share SIMDs unevenly, so a static split of the work
  // items would leave the launch waiting on the most crowded SIMDs
  p.work_counter = bucket_buffers(ctx).work_counter;
  p.task_list = order;   // work items take consecutive tasks of this order
  p.read_stride = read_stride;
  hipError_t e = launch_zero(p.work_counter, 1, stream);
  if (e == hipSuccess) e = launch_dp_i32(s, q.grid, stream, p);
  if (e != hipSuccess) return hip_fail(ctx, e);
  return SOAP_DP_OK;
}

// ---------------------------------------------------------------- batched

// Classes a batch with these bounds can populate: a class receives reads
// longer than the previous class of its kind, so classes starting at or
// above max_n stay empty.  A direct-form class is needed when some task of
// its capacity (read up to max_n, window up to max_m) falls outside the
// offset form's range and the direct form's static rule admits the class's
// shortest read; int32 classes when the direct form's rule fails for some
// read up to max_n.  The int32 re-run of flagged tasks is not a class (see
// enqueue_batched).
std::vector<int> live_classes(const soap_dp_ctx *ctx, int32_t max_n, int32_t max_m,
                              const soap_dp_scoring *sc, Mode mode) {
  std::vector<int> live;
  const int32_t ma = sc->match, mi = sc->mismatch, go = sc->gap_open, ge = sc->gap_extend;
  bool need32 = false;
  std::vector<int> direct_caps;   // capacities whose direct-form class is needed
  int prev16 = 0;
  for (size_t k = 0; k < ctx->classes.size(); ++k) {
    const ClassSpec &c = ctx->classes[k];
    if (c.prec != kPrecI16) continue;
    if (prev16 < max_n) {
      live.push_back(int(k));
      const int32_t n_hi = std::min(c.cap, max_n);
      const Shape sh = shape_of(c, class_score(c, max_m, mode));
      if (!int16_fits(n_hi, max_m, sh.lanes * sh.cells, ma, mi, go, ge)) {
        if (int16_direct_fits(prev16 + 1, ma, mi, go, ge)) direct_caps.push_back(c.cap);
        if (!int16_direct_fits(n_hi, ma, mi, go, ge)) need32 = true;
      }
    }
    prev16 = c.cap;
  }
  for (size_t k = 0; k < ctx->classes.size(); ++k) {
    const ClassSpec &c = ctx->classes[k];
    if (c.prec == kPrecI16Direct &&
        std::find(direct_caps.begin(), direct_caps.end(), c.cap) != direct_caps.end())
      live.push_back(int(k));
  }
  if (need32) {
    int prev32 = 0;
    for (size_t k = 0; k < ctx->classes.size(); ++k) {
      const ClassSpec &c = ctx->classes[k];
      if (c.prec != kPrecI32) continue;
      if (prev32 < max_n) live.push_back(int(k));
      prev32 = c.cap;
    }
  }
  return live;
}

bool any_direct(const soap_dp_ctx *ctx, const std::vector<int> &live) {
  for (int k : live)
    if (ctx->classes[size_t(k)].prec == kPrecI16Direct) return true;
  return false;
}

// Scratch of the batched form.  The live classes run concurrently, each in
// its own region, and their plans (deferral, slot size, region) are made on
// the device from the actual split of the tasks (the scan kernel).  The host
// reserves a budget that holds every live class's full grid of slots for
// the batch's longest window at deferral 1, whatever the split, and
// otherwise room for every class to reach full deferral as if it held the
// whole batch, up to the scratch cap; plus slack for region rounding.
// When a direct-form class is live, the int32 re-run of its flagged tasks
// follows the class kernels with the plain form's shape for the batch's
// bounds and reuses the scratch from its start (the class kernels are done
// by then), at deferral 1; the budget holds its full grid of slots too.
struct BatchedPlan {
  Variant v = kByte;             // int32 diagonal of the call's scoring
  bool dense = false;            // large call: int16 kernels with traceback at more waves per SIMD
  std::vector<char> cls_score;   // per class: score-only kernel (no decision scratch)
  std::vector<int> grids;
  uint64_t budget_dwords = 0;
  bool redo = false;
  bool redo_score = false;
  Shape redo_shape{0, 0};
  LaunchPlan redo_plan;
  size_t bytes() const { return size_t(budget_dwords + 64 * kMaxClasses) * 4; }
};

BatchedPlan batched_plan(const soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                         Variant v, Mode mode, const std::vector<int> &live, bool redo) {
  BatchedPlan bp;
  bp.v = v;
  bp.dense = n_tasks >= kSpreadTasks;
  for (const ClassSpec &c : ctx->classes) bp.cls_score.push_back(class_score(c, max_m, mode));
  uint64_t need = 0, want = 0;
  for (int cls : live) {
    const ClassSpec &c = ctx->classes[size_t(cls)];
    const Kind k{v, bp.cls_score[size_t(cls)] != 0, bp.dense};
    const LaunchPlan q =
        plan_launch(ctx, c.prec, shape_of(c, k.score, v), n_tasks, max_m, k, SIZE_MAX);
    bp.grids.push_back(q.grid);
    need += round64(uint64_t(q.grid) * q.slot_dwords);
    want += round64(uint64_t(q.grid) * uint64_t(q.defer) * q.slot_dwords);
  }
  bp.redo = redo;
  // the re-run traces back unless every class of the call is score-only
  bp.redo_score = mode == kModeScore;
  if (redo) {
    bp.redo_shape = plain_shape(max_n, max_m);
    bp.redo_plan = plan_launch(ctx, kPrecI32, bp.redo_shape, n_tasks, max_m,
                               Kind{v, bp.redo_score}, 0);
    bp.redo_plan.defer = 1;
    need = std::max<uint64_t>(need, round64(uint64_t(bp.redo_plan.grid) * bp.redo_plan.slot_dwords));
  }
  bp.budget_dwords = std::max<uint64_t>(need, std::min<uint64_t>(want, kScratchCap / 4));
  return bp;
}

size_t batched_scratch_bytes(const soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                             Kind k, const std::vector<int> &live, bool redo) {
  if (k.v == kEither)   // the scoring is not known: room for either diagonal's shapes
    return std::max(batched_scratch_bytes(ctx, n_tasks, max_n, max_m, Kind{kByte, k.score}, live, redo),
                    batched_scratch_bytes(ctx, n_tasks, max_n, max_m, Kind{kGeneral, k.score}, live,
                                          redo));
  return batched_plan(ctx, n_tasks, max_n, max_m, k.v, k.score ? kModeScore : kModeFull, live, redo)
      .bytes();
}

int ensure_class_streams(soap_dp_ctx *ctx, size_t n) {
  if (ctx->frozen && (ctx->class_streams.size() < n || !ctx->fork_event)) return SOAP_DP_ENOMEM;
  if (!ctx->fork_event &&
      hipEventCreateWithFlags(&ctx->fork_event, hipEventDisableTiming) != hipSuccess)
    return hip_fail(ctx, hipGetLastError());
  while (ctx->class_streams.size() < n) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
      return hip_fail(ctx, hipGetLastError());
    ctx->class_streams.push_back(st);
    ctx->join_events.push_back(ev);
  }
  return SOAP_DP_OK;
}

// Class table of one batched call: classes, and for the live ones the launch
// fields the device planner needs (dead classes get grid 0 and no tasks).
ClassTable class_table(const soap_dp_ctx *ctx, const std::vector<int> &live,
                       const BatchedPlan &bp) {
  ClassTable ct{};
  ct.count = int32_t(ctx->classes.size());
  for (size_t k = 0; k < ctx->classes.size(); ++k) {
    const ClassSpec &c = ctx->classes[k];
    const bool score = bp.cls_score[k] != 0;
    const Shape sh = shape_of(c, score, bp.v);
    ct.cap[k] = c.cap;
    ct.cols[k] = sh.lanes * sh.cells;
    ct.prec[k] = c.prec;
    ct.per_item[k] = int32_t(tasks_per_item(c.prec, sh));
    ct.grid[k] = 0;
    ct.max_defer[k] = kWave / ct.per_item[k];
    ct.lanes[k] = sh.lanes;
    ct.step_block[k] = step_block(sh.cells);
    ct.step_dwords[k] =
        score ? 0 : int32_t(uint64_t((sh.cells + 7) / 8) * kWave * (packed16(c.prec) ? 2 : 1));
    if (score) ct.max_defer[k] = 1;
  }
  for (size_t li = 0; li < live.size(); ++li) ct.grid[live[li]] = bp.grids[li];
  ct.budget_dwords = bp.budget_dwords;
  return ct;
}


// Enqueue the whole batched sequence on `stream` (also used under capture,
// so the launch plans are computed beforehand: no runtime queries in between).
hipError_t enqueue_batched(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                           const soap_dp_result *out, const std::vector<int> &live,
                           const BatchedPlan &bp, const int32_t *order, uint32_t read_stride,
                           hipStream_t stream) {
  DpParams p = make_params(in, sc, out);
  p.read_stride = read_stride;
  const BucketBuffers b = bucket_buffers(ctx);
  p.redo_list = b.redo_list;
  p.redo_count = b.redo_count;
  hipError_t e = launch_bucketing(p, class_table(ctx, live, bp), b, order, stream);
  if (e != hipSuccess) return e;
  // Class kernels, largest capacity first.  A large batch runs its largest
  // live class on the caller's stream and the others, taking turns, on
  // kForkStreams forked streams, which wait for the bucketing only; the
  // caller's stream joins them at the end.  The classes that have work
  // overlap (one kernel's tail leaves CUs that another fills), while at
  // most kForkStreams kernels sit pending beside the largest class: with
  // one stream per class, a batch of 100 bp reads (all in one class) had a
  // dozen kernels of empty classes pending beside its class kernel and took
  // 8.0 ms per call against 7.5, and with one forked stream the uneven batch
  // lost its overlap (20.9 against 19.7 ms).  A small batch (under
  // kSpreadTasks reads, as served batches are) gives every class its own
  // forked stream: its class kernels are short, and running them all at
  // once sets its latency (served p50 at 26,000 requests/s: 2.7 ms against
  // 4.7 with the large-batch arrangement).
  const bool spread = in->n_tasks < kSpreadTasks;
  if ((e = hipEventRecord(ctx->fork_event, stream)) != hipSuccess) return e;
  p.task_list = ctx->task_list;
  p.scratch = static_cast<uint32_t *>(ctx->scratch);
  const size_t nl = live.size();
  for (size_t li = nl; li-- > 0;) {
    const int k = live[li];
    const ClassSpec &c = ctx->classes[size_t(k)];
    const size_t turn = nl - 2 - li;   // launch order among the forked classes
    const size_t fs = spread ? li : turn % kForkStreams;
    const bool on_caller = !spread && li == nl - 1;
    hipStream_t cs = on_caller ? stream : ctx->class_streams[fs];
    if (!on_caller && (spread || turn < kForkStreams) &&
        (e = hipStreamWaitEvent(cs, ctx->fork_event, 0)) != hipSuccess)
      return e;
    DpParams q = p;
    q.task_off = b.offset + k;
    q.task_count = b.hist + k;
    q.work_counter = b.work_counter + k;
    q.defer_dev = b.defer + k;
    q.slot_dwords_dev = b.slot_dwords + k;
    q.scratch_off_dev = b.scratch_off + k;
    q.ok_status = packed16(c.prec) ? kTaskOk : kTaskRedone;
    q.score_only = bp.cls_score[size_t(k)];
    if ((e = launch_shape(c.prec, shape_of(c, q.score_only != 0, bp.v), bp.grids[li], cs, q,
                          bp.dense)) != hipSuccess)
      return e;
    // join a forked stream after its last kernel
    if (on_caller || (!spread && turn + kForkStreams < nl - 1)) continue;
    if ((e = hipEventRecord(ctx->join_events[fs], cs)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(stream, ctx->join_events[fs], 0)) != hipSuccess) return e;
  }
  if (bp.redo) {
    // the int32 re-run of the tasks the direct-form kernels flagged, after
    // every class kernel, on the whole scratch
    DpParams q = p;
    q.task_list = b.redo_list;
    q.task_count = b.redo_count;
    q.work_counter = b.redo_work_counter;
    q.scratch_off_dev = nullptr;
    q.defer = 1;
    q.slot_dwords = bp.redo_plan.slot_dwords;
    q.ok_status = kTaskRedone;
    q.score_only = bp.redo_score;
    if ((e = launch_dp_i32(bp.redo_shape, bp.redo_plan.grid, stream, q)) != hipSuccess) return e;
  }
  return hipSuccess;
}

int align_batched(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                  const soap_dp_result *out, hipStream_t stream, Mode mode,
                  const int32_t *order = nullptr, uint32_t read_stride = 1) {
  const std::vector<int> live = live_classes(ctx, in->max_n, in->max_m, sc, mode);
  int rc = ensure_task_buffers(ctx, in->n_tasks);
  if (rc) return rc;
  rc = ensure_class_streams(ctx, in->n_tasks < kSpreadTasks ? live.size() : kForkStreams);
  if (rc) return rc;
  const BatchedPlan bp = batched_plan(ctx, in->n_tasks, in->max_n, in->max_m,
                                      kind_for(sc, mode == kModeScore).v, mode, live,
                                      any_direct(ctx, live));
  rc = ensure_scratch(ctx, bp.bytes());
  if (rc) return rc;
  if (!ctx->use_graphs || ctx->frozen) {
    const hipError_t e = enqueue_batched(ctx, in, sc, out, live, bp, order, read_stride, stream);
    return e == hipSuccess ? SOAP_DP_OK : hip_fail(ctx, e);
  }
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.in = *in;
  key.sc = *sc;
  key.out = *out;
  key.order = order;
  key.read_stride = read_stride;
  key.epoch = ctx->epoch;
  key.flags = uint32_t(mode);
  GraphEntry *hit = nullptr;
  for (auto &g : ctx->graphs)
    if (same_key(g.key, key)) { hit = &g; break; }
  if (!hit) {
    if (!ctx->capture_stream &&
        hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess)
      return hip_fail(ctx, hipGetLastError());
    hipError_t e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(ctx, e);
    const hipError_t le =
        enqueue_batched(ctx, in, sc, out, live, bp, order, read_stride, ctx->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(ctx, le != hipSuccess ? le : e);
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(ctx, e);
    if (int(ctx->graphs.size()) >= kGraphCacheMax) {
      auto oldest = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                     [](const GraphEntry &a, const GraphEntry &b) {
                                       return a.last_use < b.last_use;
                                     });
      // its last launch may still run: wait before destroying it
      if ((e = hipDeviceSynchronize()) != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return hip_fail(ctx, e);
      }
      (void)hipGraphExecDestroy(oldest->exec);
      ctx->graphs.erase(oldest);
    }
    ctx->graphs.push_back(GraphEntry{key, exec, 0});
    hit = &ctx->graphs.back();
  }
  hit->last_use = ++ctx->use_clock;
  const hipError_t e = hipGraphLaunch(hit->exec, stream);
  if (e != hipSuccess) return hip_fail(ctx, e);
  return SOAP_DP_OK;
}

// ---------------------------------------------------------------- autotune

uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

struct TuneData {
  uint32_t *reads = nullptr, *genome = nullptr;
  uint64_t *rwo = nullptr, *rbo = nullptr;
  int32_t *rl = nullptr, *ml = nullptr, *i32 = nullptr;
  uint32_t *cigar = nullptr;
  uint8_t *status = nullptr;
  int64_t tasks = 0;
  int32_t max_m = 0;
  double cells = 0;
  ~TuneData() {
    for (void *q : {(void *)reads, (void *)genome, (void *)rwo, (void *)rbo, (void *)rl, (void *)ml,
                    (void *)i32, (void *)cigar, (void *)status})
      if (q) (void)hipFree(q);
  }
};

// Window lengths a class is timed on.  Kernels with traceback: half of the
// tasks have windows of n + 160 (short windows, as in uneven and served
// batches), half of 4 n + 160 (long windows, as in low-similarity batches),
// so a shape is chosen for both.  Score-only kernels mostly run the first
// pass of two-pass calls, which a class takes only when its windows reach
// three times its reads: they are timed on windows of 6 n + 160.
int32_t tune_window(int32_t n, int64_t t, int64_t tasks, bool score) {
  if (score) return std::min<int32_t>(6 * n + 160, SOAP_DP_MAX_WINDOW);
  return t < tasks / 2 ? n + 160 : std::min<int32_t>(4 * n + 160, SOAP_DP_MAX_WINDOW);
}

// Synthetic tasks for timing one class: reads of length n copied from random
// windows (tune_window) with 5% substitutions.
bool make_tune_data(TuneData &d, int32_t n, int64_t tasks, bool score) {
  const int64_t glen = 1 << 20;
  uint64_t seed = 0x5eed0000u + uint64_t(n);
  std::vector<uint8_t> g(static_cast<size_t>(glen));
  for (auto &x : g) x = uint8_t(splitmix(seed) & 3);
  const int32_t nw = (n + 15) / 16;
  std::vector<uint32_t> gw(static_cast<size_t>(glen / 16), 0u), rw(static_cast<size_t>(tasks * nw), 0u);
  for (int64_t k = 0; k < glen; ++k) gw[size_t(k / 16)] |= uint32_t(g[size_t(k)]) << (2 * (k % 16));
  std::vector<uint64_t> rwo(static_cast<size_t>(tasks)), rbo(static_cast<size_t>(tasks));
  std::vector<int32_t> rl(static_cast<size_t>(tasks), n), ml(static_cast<size_t>(tasks), 0);
  d.max_m = 0;
  d.cells = 0;
  for (int64_t t = 0; t < tasks; ++t) {
    const int32_t m = tune_window(n, t, tasks, score);
    ml[size_t(t)] = m;
    d.max_m = std::max(d.max_m, m);
    d.cells += double(n) * double(m);
    const uint64_t off = splitmix(seed) % uint64_t(glen - m);
    const uint64_t s = splitmix(seed) % uint64_t(m - n + 1);
    rbo[size_t(t)] = off;
    rwo[size_t(t)] = uint64_t(t) * uint64_t(nw);
    for (int32_t q = 0; q < n; ++q) {
      uint32_t b = g[size_t(off + s + uint64_t(q))];
      if (splitmix(seed) % 100 < 5) b = (b + 1 + uint32_t(splitmix(seed) % 3)) & 3;
      rw[size_t(t * nw + q / 16)] |= b << (2 * (q % 16));
    }
  }
  auto up = [](void **dst, const void *src, size_t bytes) {
    return hipMalloc(dst, bytes) == hipSuccess &&
           hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  d.tasks = tasks;
  return up((void **)&d.genome, gw.data(), gw.size() * 4) && up((void **)&d.reads, rw.data(), rw.size() * 4) &&
         up((void **)&d.rwo, rwo.data(), rwo.size() * 8) && up((void **)&d.rbo, rbo.data(), rbo.size() * 8) &&
         up((void **)&d.rl, rl.data(), rl.size() * 4) && up((void **)&d.ml, ml.data(), ml.size() * 4) &&
         hipMalloc((void **)&d.i32, size_t(tasks) * 4 * 4) == hipSuccess &&
         hipMalloc((void **)&d.cigar, size_t(tasks) * size_t(2 * n) * 4) == hipSuccess &&
         hipMalloc((void **)&d.status, size_t(tasks)) == hipSuccess;
}

std::string cache_header(const soap_dp_ctx *ctx) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "\"arch\": \"%s\", \"cus\": %d, \"version\": 4", ctx->arch.c_str(),
                ctx->cu_count);
  return buf;
}

bool load_cache(soap_dp_ctx *ctx, const char *path) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  if (text.find(cache_header(ctx)) == std::string::npos) return false;
  std::vector<ClassSpec> cls = ctx->classes;
  size_t pos = 0;
  int found = 0;
  auto usable = [](int prec, int cap, Shape s) {
    return s.lanes * s.cells >= cap && shape_compiled(prec, s);
  };
  while ((pos = text.find("{\"prec\":", pos)) != std::string::npos) {
    int prec = 0, cap = 0, lanes = 0, cells = 0, sl = 0, sk = 0, gl = 0, gk = 0, gsl = 0, gsk = 0;
    if (std::sscanf(text.c_str() + pos,
                    "{\"prec\": %d, \"cap\": %d, \"lanes\": %d, \"cells\": %d, "
                    "\"score_lanes\": %d, \"score_cells\": %d, \"gen_lanes\": %d, "
                    "\"gen_cells\": %d, \"gen_score_lanes\": %d, \"gen_score_cells\": %d",
                    &prec, &cap, &lanes, &cells, &sl, &sk, &gl, &gk, &gsl, &gsk) == 10) {
      for (auto &c : cls)
        if (c.prec == prec && c.cap == cap && usable(prec, cap, Shape{lanes, cells}) &&
            usable(prec, cap, Shape{sl, sk})) {
          c.shape = Shape{lanes, cells};
          c.score_shape = Shape{sl, sk};
          // general-diagonal shapes: int32 classes only, when tuned
          const bool gen = prec == kPrecI32 && usable(prec, cap, Shape{gl, gk}) &&
                           usable(prec, cap, Shape{gsl, gsk});
          c.gen_shape = gen ? Shape{gl, gk} : Shape{0, 0};
          c.gen_score_shape = gen ? Shape{gsl, gsk} : Shape{0, 0};
          ++found;
        }
    }
    ++pos;
  }
  if (found == 0) return false;
  mirror_direct_shapes(cls);
  ctx->classes = cls;
  return true;
}

bool save_cache(const soap_dp_ctx *ctx, const char *path, const std::vector<double> &gcups,
                const std::vector<double> &gcups_score) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{%s, \"classes\": [\n", cache_header(ctx).c_str());
  std::vector<size_t> keep;
  for (size_t k = 0; k < ctx->classes.size(); ++k)
    if (ctx->classes[k].prec != kPrecI16Direct) keep.push_back(k);
  for (size_t q = 0; q < keep.size(); ++q) {
    const size_t k = keep[q];
    const ClassSpec &c = ctx->classes[k];
    const Shape ss = shape_of(c, true);
    std::fprintf(f,
                 "  {\"prec\": %d, \"cap\": %d, \"lanes\": %d, \"cells\": %d, \"score_lanes\": %d, "
                 "\"score_cells\": %d, \"gen_lanes\": %d, \"gen_cells\": %d, "
                 "\"gen_score_lanes\": %d, \"gen_score_cells\": %d, \"gcups\": %.1f, "
                 "\"score_gcups\": %.1f}%s\n",
                 c.prec, c.cap, c.shape.lanes, c.shape.cells, ss.lanes, ss.cells, c.gen_shape.lanes,
                 c.gen_shape.cells, c.gen_score_shape.lanes, c.gen_score_shape.cells,
                 k < gcups.size() ? gcups[k] : 0.0, k < gcups_score.size() ? gcups_score[k] : 0.0,
                 q + 1 < keep.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return std::rename(tmp.c_str(), path) == 0;
}

// Measure one shape on the class's synthetic tasks: best of three launches.
double time_shape(soap_dp_ctx *ctx, int prec, Shape s, const TuneData &d, int32_t n, hipStream_t st,
                  bool score, const soap_dp_scoring &sc) {
  const int32_t m = d.max_m;
  DpParams p{};
  p.read_codes = d.reads; p.read_word_off = d.rwo; p.read_len = d.rl;
  p.ref_codes = d.genome; p.ref_base_off = d.rbo; p.ref_len = d.ml;
  p.n_tasks = d.tasks;
  p.read_words = uint64_t(d.tasks) * uint64_t((n + 15) / 16);
  p.ref_words = (1u << 20) / 16;
  p.max_n = n; p.max_m = m;
  p.ma = sc.match; p.mi = sc.mismatch; p.go = sc.gap_open; p.ge = sc.gap_extend;
  p.score = d.i32; p.ref_begin = d.i32 + d.tasks; p.ref_end = d.i32 + 2 * d.tasks;
  p.cigar_len = d.i32 + 3 * d.tasks; p.cigar = d.cigar; p.cigar_stride = 2 * n;
  p.status = d.status;
  p.ok_status = kTaskOk;
  p.min_score = INT32_MIN;
  p.score_only = score;
  const LaunchPlan q = plan_launch(ctx, prec, s, d.tasks, m, kind_for(&sc, score), kScratchCap);
  const int grid = q.grid;
  p.slot_dwords = q.slot_dwords;
  p.defer = q.defer;
  if (ensure_scratch(ctx, q.bytes())) return 0;
  p.scratch = static_cast<uint32_t *>(ctx->scratch);
  p.work_counter = bucket_buffers(ctx).work_counter;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  double best_ms = 1e30;
  for (int rep = 0; rep < 4; ++rep) {
    if (launch_zero(p.work_counter, 1, st) != hipSuccess) break;
    (void)hipEventRecord(a, st);
    if (launch_shape(prec, s, grid, st, p) != hipSuccess) break;
    (void)hipEventRecord(b, st);
    if (hipEventSynchronize(b) != hipSuccess) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    if (rep > 0) best_ms = std::min(best_ms, double(ms));   // first launch warms up
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipGetLastError();
  if (best_ms >= 1e29) return 0;
  return d.cells / (best_ms * 1e-3) / 1e9;
}

int autotune(soap_dp_ctx *ctx, std::vector<double> &gcups, std::vector<double> &gcups_score) {
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return hip_fail(ctx, hipGetLastError());
  gcups.assign(ctx->classes.size(), 0.0);
  gcups_score.assign(ctx->classes.size(), 0.0);
  // SOAPDP_TUNE_LOG=1: every timed candidate on stderr
  const char *tl = std::getenv("SOAPDP_TUNE_LOG");
  const bool tune_log = tl && tl[0] && tl[0] != '0';
  int rc = SOAP_DP_OK;
  for (size_t k = 0; k < ctx->classes.size() && rc == SOAP_DP_OK; ++k) {
    ClassSpec &c = ctx->classes[k];
    if (c.prec == kPrecI16Direct) continue;   // runs its offset-form class's shapes
    const int32_t n = c.cap;
    // about 1.2e10 cells with traceback and 6e10 score only (a few ms per
    // launch either way), and never fewer than 65,536 tasks: enough work
    // items that the persistent grid runs many rounds, as it does on real
    // batches (with too few, the last round's tail decides: a score-only
    // shape with fewer, longer work items was timed 20% below its speed in
    // a 500,000-read batch)
    auto tasks_for = [&](bool score) {
      const double m = 0.5 * (tune_window(n, 0, 2, score) + tune_window(n, 1, 2, score));
      const double cells = score ? 6e10 : 1.2e10;
      return std::max<int64_t>(65536, std::min<int64_t>(1 << 20, int64_t(cells / (double(n) * m))));
    };
    TuneData dt, ds;   // windows of the kernels with traceback / score only
    if (!make_tune_data(dt, n, tasks_for(false), false) || !make_tune_data(ds, n, tasks_for(true), true)) {
      rc = SOAP_DP_ENOMEM;
      break;
    }
    int cnt = 0;
    const Shape *all = c.prec == 16 ? shapes_i16(&cnt) : shapes_i32(&cnt);
    // with traceback, then score only: the best shape of each kind, timed
    // with the benchmark scoring (byte-table diagonal); int32 classes also
    // with a scoring that needs the general diagonal
    const soap_dp_scoring byte_sc{1, -3, -5, -2, INT32_MIN};
    const soap_dp_scoring gen_sc{1, -9, -3, -1, INT32_MIN};   // S_MI - S_GE - S_GO < 0
    for (int kind = 0; kind < (c.prec == kPrecI32 ? 4 : 2); ++kind) {
      const bool score = kind & 1, general = kind >= 2;
      const soap_dp_scoring &sc = general ? gen_sc : byte_sc;
      const TuneData &d = score ? ds : dt;
      Shape &slot = general ? (score ? c.gen_score_shape : c.gen_shape)
                            : (score ? c.score_shape : c.shape);
      double best = -1, best_rank = -1;
      Shape best_s = shape_of(c, score, general ? kGeneral : kByte);
      for (int q = 0; q < cnt; ++q) {
        const Shape s = all[q];
        const int cols = s.lanes * s.cells;
        if (cols < c.cap || cols > c.cap + std::max(c.cap / 6, 8)) continue;
        if (c.prec == 16 && !int16_fits(n, d.max_m, cols, sc.match, sc.mismatch, sc.gap_open,
                                        sc.gap_extend))
          continue;
        const double g = time_shape(ctx, c.prec, s, d, n, st, score, sc);
        if (tune_log)
          std::fprintf(stderr, "autotune: int%d class %d %s%s %dx%d: %.1f GCUPS\n",
                       c.prec == kPrecI32 ? 32 : 16, c.cap, score ? "score-only" : "traceback",
                       general ? " general" : "", s.lanes, s.cells, g);
        // Large calls run the int16 kernels with traceback of some shapes in
        // a variant for more waves per SIMD, 3-7% faster there, which these
        // isolated launches do not show: such shapes rank 2% above their
        // timing, so near-ties go to them.
        const double rank =
            g * (c.prec == 16 && !score && has_dense_dp_i16(s) ? kDenseRank : 1.0);
        if (rank > best_rank) { best_rank = rank; best = g; best_s = s; }
      }
      slot = best_s;
      if (!general) (score ? gcups_score : gcups)[k] = best;
    }
  }
  (void)hipStreamDestroy(st);
  mirror_direct_shapes(ctx->classes);
  clear_graphs(ctx);
  return rc;
}

// Work arrays of a multi-candidate call with R reads, T task slots and W
// read words, laid out 256-byte aligned from `base`; returns the bytes
// needed (with base == nullptr only the size is computed).
size_t multi_layout(int64_t R, int64_t T, uint64_t W, char *base, MultiWork *w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  MultiWork m{};
  m.reads2 = reinterpret_cast<uint32_t *>(take(2 * W * 4));
  m.off = reinterpret_cast<int64_t *>(take(size_t(R + 1) * 8));
  m.bsum = reinterpret_cast<int64_t *>(take(size_t(R / 1024 + 2) * 8));
  m.t_rwo = reinterpret_cast<uint64_t *>(take(T * 8));
  m.t_rbo = reinterpret_cast<uint64_t *>(take(T * 8));
  m.t_rl = reinterpret_cast<int32_t *>(take(T * 4));
  m.t_ml = reinterpret_cast<int32_t *>(take(T * 4));
  m.t_cand = reinterpret_cast<int64_t *>(take(T * 8));
  m.p_score = reinterpret_cast<int32_t *>(take(T * 4));
  m.p_begin = reinterpret_cast<int32_t *>(take(T * 4));
  m.p_end = reinterpret_cast<int32_t *>(take(T * 4));
  m.p_clen = reinterpret_cast<int32_t *>(take(T * 4));
  m.p_status = reinterpret_cast<uint8_t *>(take(T));
  m.f_rwo = reinterpret_cast<uint64_t *>(take(size_t(R) * 8));
  m.f_rbo = reinterpret_cast<uint64_t *>(take(size_t(R) * 8));
  m.f_rl = reinterpret_cast<int32_t *>(take(size_t(R) * 4));
  m.f_ml = reinterpret_cast<int32_t *>(take(size_t(R) * 4));
  m.flag = reinterpret_cast<uint8_t *>(take(size_t(R)));
  if (w) *w = m;
  return off;
}

// Work arrays of a mate-rescue call with R pairs and W read words, laid
// out like multi_layout.
size_t mate_layout(int64_t R, uint64_t W, char *base, MateWork *w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  MateWork m{};
  m.reads2 = reinterpret_cast<uint32_t *>(take(2 * W * 4));
  m.t_rwo = reinterpret_cast<uint64_t *>(take(size_t(R) * 8));
  m.t_rbo = reinterpret_cast<uint64_t *>(take(size_t(R) * 8));
  m.t_rl = reinterpret_cast<int32_t *>(take(size_t(R) * 4));
  m.t_ml = reinterpret_cast<int32_t *>(take(size_t(R) * 4));
  m.flag = reinterpret_cast<uint8_t *>(take(size_t(R)));
  if (w) *w = m;
  return off;
}

int ensure_multi(soap_dp_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->multi_bytes) return SOAP_DP_OK;
  if (ctx->frozen) return SOAP_DP_ENOMEM;
  if (ctx->multi) {
    if (hipDeviceSynchronize() != hipSuccess) return SOAP_DP_EHIP;
    (void)hipFree(ctx->multi);
    ctx->multi = nullptr;
    ctx->multi_bytes = 0;
  }
  clear_graphs(ctx);   // graphs hold pointers into the old arrays
  if (hipMalloc(&ctx->multi, bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->multi = nullptr;
    return SOAP_DP_ENOMEM;
  }
  ctx->multi_bytes = bytes;
  return SOAP_DP_OK;
}

// Work arrays of a two-pass call over T tasks, laid out like multi_layout.
size_t band_layout(int64_t T, char *base, BandWork *w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  BandWork b{};
  const size_t n = size_t(std::max<int64_t>(T, 1));
  b.p_score = reinterpret_cast<int32_t *>(take(n * 4));
  b.p_begin = reinterpret_cast<int32_t *>(take(n * 4));
  b.p_end = reinterpret_cast<int32_t *>(take(n * 4));
  b.p_clen = reinterpret_cast<int32_t *>(take(n * 4));
  b.p_status = reinterpret_cast<uint8_t *>(take(n));
  b.b_rbo = reinterpret_cast<uint64_t *>(take(n * 8));
  b.b_ml = reinterpret_cast<int32_t *>(take(n * 4));
  b.b_i0 = reinterpret_cast<int32_t *>(take(n * 4));
  b.order = reinterpret_cast<int32_t *>(take(n * 4));
  b.bins = reinterpret_cast<int32_t *>(take(2 * kBandBins * 4));
  if (w) *w = b;
  return off;
}

int ensure_band(soap_dp_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->band_bytes) return SOAP_DP_OK;
  if (ctx->frozen) return SOAP_DP_ENOMEM;
  if (ctx->band) {
    if (hipDeviceSynchronize() != hipSuccess) return SOAP_DP_EHIP;
    (void)hipFree(ctx->band);
    ctx->band = nullptr;
    ctx->band_bytes = 0;
  }
  clear_graphs(ctx);   // graphs hold pointers into the old arrays
  if (hipMalloc(&ctx->band, bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->band = nullptr;
    return SOAP_DP_ENOMEM;
  }
  ctx->band_bytes = bytes;
  return SOAP_DP_OK;
}

// Alignment with traceback in two passes (band.h): score and end of every
// task without decision bits, then decision bits and traceback only over
// the window rows that can hold an optimal alignment, in an order that
// groups tasks of similar band lengths.  Either form runs both passes.
int align_two_pass(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                   const soap_dp_result *out, hipStream_t stream, bool batched,
                   uint32_t read_stride) {
  int rc = ensure_band(ctx, band_layout(in->n_tasks, nullptr, nullptr));
  if (rc) return rc;
  BandWork w{};
  band_layout(in->n_tasks, static_cast<char *>(ctx->band), &w);
  // pass 1: score and end (batched form: per class, where two passes pay;
  // the other classes trace back into the caller's CIGAR rows already)
  const soap_dp_result r1{w.p_score, w.p_begin, w.p_end, out->cigar, out->cigar_stride, w.p_clen,
                          w.p_status};
  rc = batched ? align_batched(ctx, in, sc, &r1, stream, kModeMixed, nullptr, read_stride)
               : align_plain(ctx, in, sc, &r1, stream, true, nullptr, read_stride);
  if (rc) return rc;
  const BandIn bi{in->ref_base_off, in->read_len, in->ref_len, in->n_tasks, in->max_m,
                  sc->match, sc->gap_open, sc->gap_extend};
  hipError_t e = launch_band(bi, w, stream);
  if (e != hipSuccess) return hip_fail(ctx, e);
  // pass 2 sees only tasks at or above any threshold: no cutoff there
  soap_dp_scoring s2 = *sc;
  s2.min_score = INT32_MIN;
  const soap_dp_batch b2{in->read_codes, in->read_word_off, in->read_len, in->ref_codes, w.b_rbo,
                         w.b_ml, in->n_tasks, in->max_n, in->max_m, in->read_words, in->ref_words};
  rc = batched ? align_batched(ctx, &b2, &s2, out, stream, kModeFull, w.order, read_stride)
               : align_plain(ctx, &b2, &s2, out, stream, false, w.order, read_stride);
  if (rc) return rc;
  const BandOut bo{out->score, out->ref_begin, out->ref_end, out->cigar_len, out->status};
  if ((e = launch_band_fixup(in->n_tasks, w, bo, stream)) != hipSuccess) return hip_fail(ctx, e);
  return SOAP_DP_OK;
}

// Flags of soap_dp_align_batch and soap_dp_mate_rescue to the path taken.
int align_dispatch(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                   const soap_dp_result *out, hipStream_t stream, uint32_t flags) {
  const bool batched = (flags & SOAP_DP_BATCHED) != 0;
  const bool score = (flags & SOAP_DP_SCORE_ONLY) != 0;
  const uint32_t stride = (flags & SOAP_DP_READS_INTERLEAVED) ? kReadGroup : 1u;
  if (!score && (flags & SOAP_DP_FULL_WINDOW) == 0)
    return align_two_pass(ctx, in, sc, out, stream, batched, stride);
  return batched ? align_batched(ctx, in, sc, out, stream, score ? kModeScore : kModeFull,
                                 nullptr, stride)
                 : align_plain(ctx, in, sc, out, stream, score, nullptr, stride);
}

// Classes a batched call with these bounds can populate: for a known
// scoring exactly those live_classes gives for both kinds of kernel, else
// every class of every kind up to max_n.
std::vector<int> reserve_classes(const soap_dp_ctx *ctx, int32_t max_n, int32_t max_m,
                                 const soap_dp_scoring *sc, bool *redo) {
  std::vector<int> live;
  if (sc) {
    for (Mode mode : {kModeFull, kModeScore})
      for (int k : live_classes(ctx, max_n, max_m, sc, mode))
        if (std::find(live.begin(), live.end(), k) == live.end()) live.push_back(k);
    *redo = any_direct(ctx, live);
    return live;
  }
  int prev[3] = {0, 0, 0};
  for (size_t k = 0; k < ctx->classes.size(); ++k) {
    const ClassSpec &c = ctx->classes[k];
    int &pv = prev[c.prec == kPrecI16 ? 0 : (c.prec == kPrecI16Direct ? 1 : 2)];
    if (pv < max_n) live.push_back(int(k));
    pv = c.cap;
  }
  *redo = true;
  return live;
}

size_t workspace_bytes_for(const soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                           uint32_t flags, const soap_dp_scoring *sc) {
  if (!ctx || n_tasks <= 0 || max_n < 1 || max_n > SOAP_DP_MAX_READ || max_m < 1 ||
      max_m > SOAP_DP_MAX_WINDOW)
    return 0;
  const size_t small = kSmallInts * sizeof(int32_t);
  const bool score = (flags & SOAP_DP_SCORE_ONLY) != 0;
  const Kind k = sc ? kind_for(sc, score) : Kind{kEither, score};
  // two-pass work arrays
  const size_t band = (flags & (SOAP_DP_SCORE_ONLY | SOAP_DP_FULL_WINDOW)) == 0
                          ? band_layout(n_tasks, nullptr, nullptr)
                          : 0;
  if ((flags & SOAP_DP_BATCHED) == 0)
    return plain_scratch_bytes(ctx, n_tasks, max_n, max_m, k) + small + band;
  bool redo = false;
  const std::vector<int> live = reserve_classes(ctx, max_n, max_m, sc, &redo);
  return batched_scratch_bytes(ctx, n_tasks, max_n, max_m, k, live, redo) + size_t(n_tasks) * 9 +
         small + band;
}

}  // namespace

int soapdp::ctx_reserve_for(soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                            uint32_t flags, const soap_dp_scoring *sc) {
  if (!ctx) return SOAP_DP_EINVAL;
  const size_t b = workspace_bytes_for(ctx, n_tasks, max_n, max_m, flags, sc);
  if (b == 0) return SOAP_DP_EINVAL;
  DeviceGuard dg(ctx->device);
  const size_t small = kSmallInts * sizeof(int32_t);
  size_t scratch = b - small;
  if ((flags & (SOAP_DP_SCORE_ONLY | SOAP_DP_FULL_WINDOW)) == 0) {
    const size_t band = band_layout(n_tasks, nullptr, nullptr);
    scratch -= band;
    const int rc = ensure_band(ctx, band);
    if (rc) return rc;
  }
  if (flags & SOAP_DP_BATCHED) {
    scratch -= size_t(n_tasks) * 9;
    int rc = ensure_task_buffers(ctx, n_tasks);
    if (rc) return rc;
    // the forked streams of the class kernels: one per class a call with
    // these bounds can populate (small batches), at least kForkStreams
    bool redo = false;
    const size_t n_live = reserve_classes(ctx, max_n, max_m, sc, &redo).size();
    if ((rc = ensure_class_streams(ctx, std::max(n_live, kForkStreams))) != SOAP_DP_OK) return rc;
  }
  return ensure_scratch(ctx, scratch);
}

// Fixed device memory of soap_dp_align_batch_noalloc: a 256-byte block for
// the work counter, then the decision slots.  Each device that loads the
// library holds its own copy until the process ends.  In host code the
// array's name is no device address: the address of a device's copy comes
// from hipGetSymbolAddress (fixed_array_of) and only that is used.
static __device__ __align__(256) uint32_t scratch[SOAP_DP_NOALLOC_BYTES / 4];

namespace {

constexpr size_t kFixedHead = 256;   // work counter block
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
char *g_fixed[kMaxDevices] = {};

// Address of `device`'s copy of the fixed array, looked up once per device
// with that device current.
int fixed_array_of(int device, char **out) {
  if (device < 0 || device >= kMaxDevices) return SOAP_DP_EINVAL;
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (!g_fixed[device]) {
    DeviceGuard dg(device);
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return SOAP_DP_EHIP;
    }
    g_fixed[device] = static_cast<char *>(p);
  }
  *out = g_fixed[device];
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
  ctx->arch = "gfx950";
  ctx->classes.assign(std::begin(kDefaultClasses), std::end(kDefaultClasses));
  const char *ug = std::getenv("SOAPDP_GRAPHS");
  ctx->use_graphs = ug && ug[0] && ug[0] != '0';
  if (const int frc = fixed_array_of(device_ordinal, &ctx->fixed)) {
    delete ctx;
    return frc;
  }
  {
    DeviceGuard dg(device_ordinal);
    if (hipMalloc(reinterpret_cast<void **>(&ctx->small), kSmallInts * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      delete ctx;
      return SOAP_DP_ENOMEM;
    }
  }
  *out = ctx;
  return SOAP_DP_OK;
}

int soap_dp_destroy(soap_dp_ctx *ctx) {
  if (!ctx) return SOAP_DP_EINVAL;
  {
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    clear_graphs(ctx);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto st : ctx->class_streams) (void)hipStreamDestroy(st);
    for (auto ev : ctx->join_events) (void)hipEventDestroy(ev);
    if (ctx->fork_event) (void)hipEventDestroy(ctx->fork_event);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->small) (void)hipFree(ctx->small);
    if (ctx->task_list) (void)hipFree(ctx->task_list);
    if (ctx->task_class) (void)hipFree(ctx->task_class);
    if (ctx->redo_list) (void)hipFree(ctx->redo_list);
    if (ctx->multi) (void)hipFree(ctx->multi);
    if (ctx->band) (void)hipFree(ctx->band);
  }
  delete ctx;
  return SOAP_DP_OK;
}

int soap_dp_align_multi(soap_dp_ctx *ctx, const soap_dp_multi_batch *in, const soap_dp_scoring *sc,
                        const soap_dp_multi_result *out, void *stream) {
  if (!ctx || !in || !out || !scoring_ok(sc)) return SOAP_DP_EINVAL;
  if (in->n_reads < 0 || in->n_cands < 0 || in->ceiling < 1 || in->ceiling > SOAP_DP_MAX_CEILING)
    return SOAP_DP_EINVAL;
  if (in->max_n < 1 || in->max_n > SOAP_DP_MAX_READ || in->max_m < 1 || in->max_m > SOAP_DP_MAX_WINDOW)
    return SOAP_DP_EINVAL;
  if (out->cigar_stride < 2 * in->max_n - 1) return SOAP_DP_EINVAL;
  if (in->n_reads > (int64_t(1) << 31) - 1 || in->n_cands > (int64_t(1) << 40)) return SOAP_DP_EINVAL;
  // task slots: at most one per candidate, at most `ceiling` per read
  const int64_t T = std::min<int64_t>(in->n_cands, in->n_reads * int64_t(in->ceiling));
  if (T > (int64_t(1) << 31) - 1) return SOAP_DP_EINVAL;
  if (in->n_reads == 0) return SOAP_DP_OK;
  if (!in->read_codes || !in->read_word_off || !in->read_len || !in->cand_start ||
      (in->n_cands > 0 && (!in->cand_base_off || !in->cand_len || !in->cand_support ||
                           !in->cand_strand)) ||
      !in->ref_codes || in->read_words == 0 || in->ref_words == 0)
    return SOAP_DP_EINVAL;
  if (!out->score || !out->ref_begin || !out->ref_end || !out->best_cand || !out->second_score ||
      !out->n_aligned || !out->cigar || !out->cigar_len || !out->status)
    return SOAP_DP_EINVAL;
  DeviceGuard dg(ctx->device);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t C = in->ceiling;
  int rc = ensure_multi(ctx, multi_layout(in->n_reads, T, in->read_words, nullptr, nullptr));
  if (rc) return rc;
  MultiWork w{};
  multi_layout(in->n_reads, T, in->read_words, static_cast<char *>(ctx->multi), &w);
  const MultiIn mi{in->read_codes, in->read_word_off, in->read_len, in->read_words, in->cand_start,
                   in->cand_base_off, in->cand_len, in->cand_support, in->cand_strand,
                   in->ref_words, in->n_reads, in->n_cands, in->max_n, in->max_m, C, T};
  const MultiOut mo{out->score, out->ref_begin, out->ref_end, out->cigar_len, out->status,
                    out->best_cand, out->second_score, out->n_aligned};
  // reads and their reverse complements, candidate ranking into task slots
  hipError_t e = hipMemcpyAsync(w.reads2, in->read_codes, in->read_words * 4,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = launch_revcomp(mi, w, st);
  if (e == hipSuccess) e = launch_select(mi, w, mo, st);
  if (e != hipSuccess) return hip_fail(ctx, e);
  // every ranked (read, candidate) pair, score only
  const soap_dp_batch b1{w.reads2, w.t_rwo, w.t_rl, in->ref_codes, w.t_rbo, w.t_ml,
                         T, in->max_n, in->max_m, 2 * in->read_words, in->ref_words};
  const soap_dp_result r1{w.p_score, w.p_begin, w.p_end, nullptr, 0, w.p_clen, w.p_status};
  const soap_dp_scoring es = effective_scoring(sc, 0);   // no cutoff here
  if (T > 0 && (rc = align_batched(ctx, &b1, &es, &r1, st, kModeScore)) != SOAP_DP_OK) return rc;
  if ((e = launch_reduce(mi, w, mo, st)) != hipSuccess) return hip_fail(ctx, e);
  // each read's best pair again, with traceback, into the caller's outputs
  const soap_dp_batch b2{w.reads2, w.f_rwo, w.f_rl, in->ref_codes, w.f_rbo, w.f_ml,
                         in->n_reads, in->max_n, in->max_m, 2 * in->read_words, in->ref_words};
  const soap_dp_result r2{out->score, out->ref_begin, out->ref_end, out->cigar, out->cigar_stride,
                          out->cigar_len, out->status};
  rc = align_batched(ctx, &b2, &es, &r2, st, kModeFull);
  if (rc) return rc;
  if ((e = launch_fixup(mi, w, mo, st)) != hipSuccess) return hip_fail(ctx, e);
  return SOAP_DP_OK;
}

int soap_dp_mate_rescue(soap_dp_ctx *ctx, const soap_dp_mate_batch *in, const soap_dp_scoring *sc,
                        const soap_dp_mate_result *out, void *stream, uint32_t flags) {
  if (!ctx || !in || !out || !scoring_ok(sc)) return SOAP_DP_EINVAL;
  if (flags & ~(SOAP_DP_BATCHED | SOAP_DP_SCORE_ONLY | SOAP_DP_MIN_SCORE | SOAP_DP_FULL_WINDOW))
    return SOAP_DP_EINVAL;
  const bool score = (flags & SOAP_DP_SCORE_ONLY) != 0;
  if (in->n_reads < 0 || in->n_reads > (int64_t(1) << 31) - 1) return SOAP_DP_EINVAL;
  if (in->max_n < 1 || in->max_n > SOAP_DP_MAX_READ) return SOAP_DP_EINVAL;
  if (in->min_frag < 1 || in->max_frag < in->min_frag ||
      int64_t(in->max_frag) - in->min_frag + in->max_n > SOAP_DP_MAX_WINDOW)
    return SOAP_DP_EINVAL;
  if (in->orientation < SOAP_DP_ORIENT_FR || in->orientation > SOAP_DP_ORIENT_FF_UP)
    return SOAP_DP_EINVAL;
  if (in->ref_len < 1 || in->ref_len > (uint64_t(1) << 40)) return SOAP_DP_EINVAL;
  if (!score && (!out->cigar || out->cigar_stride < 2 * in->max_n - 1)) return SOAP_DP_EINVAL;
  if (in->n_reads == 0) return SOAP_DP_OK;
  if (!in->read_codes || !in->read_word_off || !in->read_len || in->read_words == 0 ||
      !in->mate_pos || !in->mate_len || !in->mate_strand || !in->ref_codes)
    return SOAP_DP_EINVAL;
  if (!out->score || !out->ref_begin || !out->ref_end || !out->cigar_len || !out->status ||
      !out->window_off || !out->window_len || !out->strand)
    return SOAP_DP_EINVAL;
  DeviceGuard dg(ctx->device);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ensure_multi(ctx, mate_layout(in->n_reads, in->read_words, nullptr, nullptr));
  if (rc) return rc;
  MateWork w{};
  mate_layout(in->n_reads, in->read_words, static_cast<char *>(ctx->multi), &w);
  const MateIn mi{in->read_codes, in->read_word_off, in->read_len, in->read_words, in->mate_pos,
                  in->mate_len, in->mate_strand, in->ref_len, in->n_reads, in->max_n,
                  in->min_frag, in->max_frag,
                  in->orientation == SOAP_DP_ORIENT_FF || in->orientation == SOAP_DP_ORIENT_FF_UP,
                  in->orientation == SOAP_DP_ORIENT_RF || in->orientation == SOAP_DP_ORIENT_FF_UP};
  const MateOut mo{out->score, out->ref_begin, out->ref_end, out->cigar_len, out->status,
                   out->window_off, out->window_len, out->strand};
  hipError_t e = hipMemcpyAsync(w.reads2, in->read_codes, in->read_words * 4,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = launch_mate_windows(mi, w, mo, st);
  if (e != hipSuccess) return hip_fail(ctx, e);
  const soap_dp_batch b{w.reads2, w.t_rwo, w.t_rl, in->ref_codes, w.t_rbo, w.t_ml, in->n_reads,
                        in->max_n, in->max_frag - in->min_frag + in->max_n, 2 * in->read_words,
                        (in->ref_len + 15) / 16};
  const soap_dp_result r{out->score, out->ref_begin, out->ref_end, out->cigar, out->cigar_stride,
                         out->cigar_len, out->status};
  if ((rc = batch_ok(&b, &r, score)) != SOAP_DP_OK) return rc;
  const soap_dp_scoring es = effective_scoring(sc, flags);
  rc = align_dispatch(ctx, &b, &es, &r, st, flags);
  if (rc) return rc;
  if ((e = launch_mate_fixup(mi, w, mo, st)) != hipSuccess) return hip_fail(ctx, e);
  return SOAP_DP_OK;
}

int soap_dp_align_batch(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                        const soap_dp_result *out, void *stream, uint32_t flags) {
  if (!ctx) return SOAP_DP_EINVAL;
  if (!scoring_ok(sc)) return SOAP_DP_EINVAL;
  if (flags & ~(SOAP_DP_BATCHED | SOAP_DP_SCORE_ONLY | SOAP_DP_MIN_SCORE | SOAP_DP_FULL_WINDOW |
                SOAP_DP_READS_INTERLEAVED))
    return SOAP_DP_EINVAL;
  const bool score = (flags & SOAP_DP_SCORE_ONLY) != 0;
  const int rc = batch_ok(in, out, score);
  if (rc) return rc;
  if (in->n_tasks == 0) return SOAP_DP_OK;
  DeviceGuard dg(ctx->device);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const soap_dp_scoring es = effective_scoring(sc, flags);
  return align_dispatch(ctx, in, &es, out, st, flags);
}

int soap_dp_align_batch_noalloc(soap_dp_ctx *ctx, const soap_dp_batch *in,
                                const soap_dp_scoring *sc, const soap_dp_result *out,
                                void *stream, uint32_t flags) {
  if (!ctx || !scoring_ok(sc)) return SOAP_DP_EINVAL;
  if (flags & ~(SOAP_DP_SCORE_ONLY | SOAP_DP_MIN_SCORE | SOAP_DP_FULL_WINDOW |
                SOAP_DP_READS_INTERLEAVED))
    return SOAP_DP_EINVAL;
  const bool score = (flags & SOAP_DP_SCORE_ONLY) != 0;
  const int rc = batch_ok(in, out, score);
  if (rc) return rc;
  if (in->n_tasks == 0) return SOAP_DP_OK;
  if (!ctx->fixed) return SOAP_DP_EHIP;
  DeviceGuard dg(ctx->device);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const soap_dp_scoring es = effective_scoring(sc, flags);
  // the plain form in one pass (whole windows), its decision slots in the
  // fixed array: fewer workgroups when all of them would not fit
  const Shape s = plain_shape(in->max_n, in->max_m);
  if (s.lanes == 0) return SOAP_DP_EINVAL;
  const size_t avail = SOAP_DP_NOALLOC_BYTES - kFixedHead;
  LaunchPlan q = plan_launch(ctx, 32, s, in->n_tasks, in->max_m, kind_for(&es, score), avail);
  if (!score) {
    const uint64_t slot = q.slot_dwords * 4;
    if (slot > avail) return SOAP_DP_E2BIG;
    q.grid = int(std::min<uint64_t>(uint64_t(q.grid), avail / slot));
    while (q.defer > 1 && q.bytes() > avail) --q.defer;
  }
  DpParams p = make_params(in, &es, out);
  p.score_only = score;
  p.work_counter = reinterpret_cast<int32_t *>(ctx->fixed);
  p.scratch = reinterpret_cast<uint32_t *>(ctx->fixed + kFixedHead);
  p.slot_dwords = q.slot_dwords;
  p.defer = q.defer;
  p.read_stride = (flags & SOAP_DP_READS_INTERLEAVED) ? kReadGroup : 1u;
  // the previous call left its count: clear it (a kernel, so that a
  // captured call replays the clear)
  hipError_t e = launch_zero(p.work_counter, 1, st);
  if (e == hipSuccess) e = launch_dp_i32(s, q.grid, st, p);
  if (e != hipSuccess) return hip_fail(ctx, e);
  return SOAP_DP_OK;
}

size_t soap_dp_workspace_bytes(const soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n,
                               int32_t max_m, uint32_t flags) {
  return workspace_bytes_for(ctx, n_tasks, max_n, max_m, flags, nullptr);
}

int soap_dp_reserve(soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                    uint32_t flags) {
  return soapdp::ctx_reserve_for(ctx, n_tasks, max_n, max_m, flags, nullptr);
}

int soap_dp_autotune(soap_dp_ctx *ctx, const char *cache_path, int force) {
  if (!ctx) return SOAP_DP_EINVAL;
  DeviceGuard dg(ctx->device);
  if (cache_path && !force && load_cache(ctx, cache_path)) {
    clear_graphs(ctx);
    return SOAP_DP_OK;
  }
  std::vector<double> gcups, gcups_score;
  const int rc = autotune(ctx, gcups, gcups_score);
  if (rc) return rc;
  if (cache_path && !save_cache(ctx, cache_path, gcups, gcups_score)) return SOAP_DP_EINVAL;
  return SOAP_DP_OK;
}

int soap_dp_get_classes(const soap_dp_ctx *ctx, soap_dp_class_info *out, int32_t n_max) {
  if (!ctx) return SOAP_DP_EINVAL;
  // the direct-form classes run their int16 class's shapes and are not listed
  int32_t cnt = 0;
  for (const ClassSpec &c : ctx->classes) {
    if (c.prec == kPrecI16Direct) continue;
    if (out && cnt < n_max)
      out[cnt] = soap_dp_class_info{c.prec, c.cap, c.shape.lanes, c.shape.cells};
    ++cnt;
  }
  return cnt;
}

int soap_dp_set_class_shape(soap_dp_ctx *ctx, int32_t precision, int32_t capacity, int32_t lanes,
                            int32_t cells) {
  if (!ctx) return SOAP_DP_EINVAL;
  const Shape s{lanes, cells};
  if ((precision != 16 && precision != 32) || !shape_compiled(precision, s) ||
      lanes * cells < capacity)
    return SOAP_DP_EINVAL;
  for (auto &c : ctx->classes)
    if (c.prec == precision && c.cap == capacity) {
      c.shape = s;
      c.score_shape = s;
      c.gen_shape = Shape{0, 0};
      c.gen_score_shape = Shape{0, 0};
      mirror_direct_shapes(ctx->classes);
      clear_graphs(ctx);
      return SOAP_DP_OK;
    }
  return SOAP_DP_EINVAL;
}

int soap_dp_list_shapes(int32_t precision, soap_dp_class_info *out, int32_t n_max) {
  if (precision != 16 && precision != 32) return SOAP_DP_EINVAL;
  int cnt = 0;
  const Shape *all = precision == 16 ? shapes_i16(&cnt) : shapes_i32(&cnt);
  for (int k = 0; out && k < cnt && k < n_max; ++k) {
    out[k].precision = precision;
    out[k].capacity = all[k].lanes * all[k].cells;
    out[k].lanes = all[k].lanes;
    out[k].cells = all[k].cells;
  }
  return cnt;
}

const char *soap_dp_strerror(int code) {
  switch (code) {
    case SOAP_DP_OK: return "ok";
    case SOAP_DP_EINVAL: return "invalid argument (scoring, pointer, size or stride)";
    case SOAP_DP_ENOMEM: return "device workspace allocation failed";
    case SOAP_DP_EHIP: return "HIP runtime error";
    case SOAP_DP_ENODEV: return "no usable gfx950 device";
    case SOAP_DP_E2BIG: return "request larger than a slot, the device budget or the fixed scratch";
    case SOAP_DP_ESTOPPED: return "server is shutting down";
    default: return "unknown error";
  }
}

int soap_dp_last_hip_error(const soap_dp_ctx *ctx) { return ctx ? ctx->last_hip_error : 0; }

}  // extern "C"

void soapdp::ctx_set_frozen(soap_dp_ctx *ctx, bool frozen) {
  if (ctx) ctx->frozen = frozen;
}
