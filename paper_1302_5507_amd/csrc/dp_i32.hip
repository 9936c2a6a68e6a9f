// int32 fill + traceback kernel for batched read-vs-window affine-gap
// alignment (paper, Methods section 3: recurrences for I, D, M, base cases,
// result max_i M(i, n); traceback from the D and M decisions).
//
// Mapping onto a 64-lane CDNA wavefront:
//  * A task is served by L consecutive lanes (64/L tasks per wavefront).  The
//    read is right-aligned onto the L*K columns the lanes own (K per lane),
//    so read column n is always the last column of the last lane and the
//    result row is read from a fixed register.  Columns left of the read are
//    "virtual": their delta is 0 and their M stays 0, which reproduces the
//    boundary M(i,0) = 0 exactly, and I there never beats opening a gap.
//    (In offset form a virtual column's M^ is -(i+j)*S_GE, kept by its
//    diagonal constant -2 S_GE.)
//  * Values are kept in the offset form  X^(i,j) = X(i,j) - (i+j)*S_GE  for
//    X = M, I, D (exact, and an order-preserving shift within each cell).
//    Gap extension then adds nothing:  I^(i,j) = max(M^(i,j-1) + S_GO - S_GE,
//    I^(i,j-1)),  D^(i,j) = max(M^(i-1,j) + S_GO - S_GE, D^(i-1,j)),  and the
//    diagonal adds delta - 2 S_GE.  The result row compares M^(i,n) + i*S_GE.
//  * The window (rows i = 1..m) is swept along anti-diagonals: at step t lane
//    l of a task computes row t + 1 - l for its K columns, left to right.  The
//    only value crossing lanes is the left neighbour's last column (M and I
//    of the current row) plus the window base of that row; it moves with one
//    DPP wave_shr:1 per value and step.  The diagonal M of the first column is
//    the value received one step earlier.  D and M of the previous row stay in
//    the lane's registers.
//  * Each cell yields four decision bits, taken as the sign of a difference
//    that is zero exactly when the tie-broken option wins: bit3 I extended,
//    bit2 D extended, bit1 M did not come from the diagonal, bit0 M did not
//    come from D.  They are packed 8 cells to a dword (first cell in the top
//    nibble) and written step-major, so every store of the wavefront is 256
//    contiguous bytes.
//  * A wavefront sweeps up to 64/G work items into consecutive scratch slots,
//    then one lane per task of all of them walks the decisions back from
//    (ref_end, n) and writes the run-length CIGAR, so the walk, which is
//    bound by dependent loads, keeps every lane busy.
#include "dp_device.h"

namespace soapdp {

// Waves per SIMD asked of the register allocator.  The byte-table variant
// fits five (96 VGPRs) up to 16 columns per lane without spilling once the
// compiler is asked to.  The score-only 4 x 25 sweep fits four instead of
// three with its few spills outside the row loop, which made the
// mate-rescue plain call 2% faster; asked the same, the 4 x 38 and 8 x 32
// score sweeps ran 4% and 2% slower, so they keep the default.  The
// byte-table kernels with traceback above 16 columns are asked for four:
// 4 x 25 and 8 x 32 then fit without spilling and 4 x 38 spills 72 bytes,
// and the plain calls ran 1.2% (low-similarity) and 1.2-2.0% (mate rescue)
// faster.  Their general-table twins would spill 100-300 bytes at four and
// keep the default.
// kScore: score and end only -- no decision bits, no scratch, no traceback.
template <int L, int K, bool kByte, bool kScore>
__global__ __launch_bounds__(kWave)
__attribute__((amdgpu_waves_per_eu((kByte || kScore) && K <= 16 ? 5 : (kByte && (!kScore || (K >= 20 && K <= 25)) ? 4 : 1))))
void dp_i32_kernel(DpParams p) {
  static_assert(kWave % L == 0, "lanes per task must divide the wavefront");
  constexpr int G = kWave / L;       // tasks per wavefront
  constexpr int W = (K + 7) / 8;     // decision dwords per lane per step
  const int lane = threadIdx.x;
  const int g = lane / L;
  const int lg = lane % L;
  const bool first = lg == 0;
  const bool last = lg == L - 1;

  // bookkeeping of the deferred work items, entry r * G + g
  __shared__ int64_t s_task[kWave];
  __shared__ int32_t s_n[kWave], s_pad[kWave], s_end[kWave], s_score[kWave];
  __shared__ uint8_t s_st[kWave];
  constexpr int B = step_block(K);   // sweep steps per stored block
  // staging buffer of the sweep, or the traceback's block caches
  __shared__ __align__(16) uint32_t s_lds[kScore ? 4 : StageOrCache<uint32_t, W, B>::kWords];

  // `defer` work items are swept into consecutive slots before one
  // traceback pass serves all their tasks, one lane per task
  const int32_t defer = kScore ? 1 : min(max(p.defer_dev ? *p.defer_dev : p.defer, 1), kWave / G);
  const uint64_t slot_dwords = p.slot_dwords_dev ? *p.slot_dwords_dev : p.slot_dwords;
  uint32_t *const slots = p.scratch + (p.scratch_off_dev ? *p.scratch_off_dev : 0) +
                          (uint64_t)blockIdx.x * slot_dwords * (uint64_t)defer;
  // window rows a slot can hold: (rows + L - 1) steps of W * 64 lanes
  const int64_t slot_rows =
      kScore ? INT64_MAX : (int64_t)(slot_dwords / (uint64_t)(W * kWave * 1)) - (L - 1);
  int32_t r = 0;   // slot of the current work item
  const int64_t n_tasks = p.task_count ? (int64_t)*p.task_count : p.n_tasks;
  const int32_t *const list = (p.task_list && p.task_off) ? p.task_list + *p.task_off : p.task_list;
  const int64_t n_items = (n_tasks + G - 1) / G;

  int64_t item = blockIdx.x;
  while (item < n_items) {
    // ---------------- task set-up
    const int64_t tix = item * G + g;
    int64_t task = -1;
    int32_t n = 0, m = 0;
    uint64_t rwo = 0, rbo = 0;
    uint8_t st = kTaskOk;
    if (tix < n_tasks) {
      task = task_at(p, list, tix);
      n = p.read_len[task];
      m = p.ref_len[task];
      rwo = p.read_word_off[task];
      rbo = p.ref_base_off[task];
      if (n < 1 || m < 1 || n > p.max_n || m > p.max_m || n > L * K || m > slot_rows)
        st = kTaskInvalidLen;
      else if (!read_in_bounds(rwo, n, p.read_words, p.read_stride) ||
               rbo + (uint64_t)m > p.ref_words * 16)
        st = kTaskInvalidOffset;
    }
    const bool valid = task >= 0 && st == kTaskOk;
    const int32_t mg = valid ? m : 0;
    const int32_t pad = L * K - n;
    // uniform trip count: keeps the step loop under scalar control
    const int32_t steps = __builtin_amdgcn_readfirstlane(wave_max(mg)) + L - 1;
    // bookkeeping for the traceback goes to LDS now, out of the sweep's registers
    const int u0 = r * G + g;
    if (first) { s_task[u0] = task; s_n[u0] = n; s_pad[u0] = pad; s_st[u0] = st; }

    StripWords rw{0, 0, 0, 0};
    if (valid) rw.load(p.read_codes, rwo, n, lg * K - pad, p.read_stride);
    const int32_t ge = p.ge;
    const int32_t c_go = p.go - ge;          // gap open in offset form
    // H holds G = M^ + c_go: the gap-open candidate of the cell to the right
    // (same row) and of the cell below (next row) without another add.  The
    // diagonal constants are taken relative to it: delta - 2 S_GE - c_go.
    const int32_t c_ma = p.ma - 2 * ge - c_go;
    // Read codes (4 left of the read, never a window base).  General
    // variant: one register per column plus its mismatch constant.  Byte
    // variant: four columns' codes per register, one byte each.
    constexpr int Q = (K + 3) / 4;
    int32_t Rc[kByte ? 1 : K], Mi[kByte ? 1 : K], H[K], F[K];
    uint32_t R4[kByte ? Q : 1];
#pragma unroll
    for (int q = 0; q < (kByte ? Q : 1); ++q) R4[q] = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const int32_t q = lg * K + c - pad;  // 0-based read index of this column
      const bool real = valid && q >= 0;
      const uint32_t code = real ? rw.code(q) : 4u;
      if constexpr (kByte) {
        R4[c / 4] |= code << (8 * (c % 4));
      } else {
        Rc[c] = (int32_t)code;
        Mi[c] = real ? p.mi - 2 * ge - c_go : -2 * ge - c_go;
      }
      // M^(0, j), j = q + 1: S_GO + (j-1) S_GE - j S_GE, or 0 - j S_GE left
      // of the read; held as G = M^ + c_go
      H[c] = (real ? c_go : -(q + 1) * ge) + c_go;
      F[c] = kNeg32;                       // D(0, j)
      // finish each column before the next: bounds live registers in set-up
      if constexpr (kByte)
        asm volatile("" : "+v"(R4[c / 4]), "+v"(H[c]));
      else
        asm volatile("" : "+v"(Rc[c]), "+v"(Mi[c]), "+v"(H[c]));
      __builtin_amdgcn_sched_barrier(0);
    }
    // Byte variant: the diagonal constant of code x at window base b is byte
    // x of the table (tab_hi:tab_lo) with byte b of tab_lo holding the match
    // value, the other bytes of tab_lo the mismatch value and tab_hi (codes
    // 4..7) the value left of the read.
    const uint32_t d_mi = (uint32_t)(p.mi - 2 * ge - c_go) & 0xffu;
    const uint32_t tab_mis = d_mi * 0x01010101u;
    const uint32_t tab_flip = ((uint32_t)c_ma & 0xffu) ^ d_mi;
    const uint32_t tab_hi = ((uint32_t)(-2 * ge - c_go) & 0xffu) * 0x01010101u;

    // window bases, 16 at a time, realigned from the base offset
    const uint64_t wlim = p.ref_words - 1;
    const int32_t wsh = (int32_t)(rbo & 15) * 2;
    auto load_block = [&](int32_t b, uint32_t &w0, uint32_t &w1) {
      const uint64_t wi = (rbo >> 4) + (uint64_t)b;
      w0 = p.ref_codes[wi < wlim ? wi : wlim];
      w1 = p.ref_codes[wi + 1 < wlim ? wi + 1 : wlim];
    };
    uint32_t tn0, tn1, tw = 0;
    load_block(0, tn0, tn1);

    int32_t hl_out = H[K - 1];   // G(0, last column of the strip)
    int32_t el_out = kNeg32;
    int32_t t_out = 0;
    // left boundary M^(i, -pad) = -(i - pad) S_GE (true value 0), as G: row 0
    // is the first lane's first diagonal, row 1 its first left neighbour
    int32_t hl_prev = pad * ge + c_go;
    int32_t bnd = (pad - 1) * ge + c_go;
    int32_t rge = (1 - lg) * ge - c_go;   // i * S_GE of the current row, minus c_go
    int32_t best = INT32_MIN, endi = 0;
    uint32_t acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;

    uint32_t *sp = slots + (uint64_t)r * slot_dwords;
    for (int32_t t = 0; t < steps; ++t) {
      if ((t & 15) == 0) {
        tw = __builtin_amdgcn_alignbit(tn1, tn0, wsh);
        load_block((t >> 4) + 1, tn0, tn1);
      }
      const int32_t tfirst = (int32_t)((tw >> ((t & 15) * 2)) & 3u);
      // the first lane of a task receives the left boundary (M = 0, I = -inf)
      // and the row's window base; its diagonal is the boundary received one
      // step earlier
      int32_t hl = group_shr1<L>(hl_out, bnd, first);
      int32_t el = group_shr1<L>(el_out, kNeg32, first);
      const int32_t T = group_shr1<L>(t_out, tfirst, first);
      const int32_t hd = hl_prev;
      hl_prev = hl;
      t_out = T;
      const int32_t i = t + 1 - lg;
      if ((uint32_t)(t - lg) < (uint32_t)mg) {   // 1 <= i <= mg
        uint32_t d4[kByte ? Q : 1];
        if constexpr (kByte) {
          // this row's table, then four columns' constants per byte permute
          const uint32_t tab_lo = tab_mis ^ (tab_flip << (8 * T));
#pragma unroll
          for (int q = 0; q < Q; ++q) d4[q] = __builtin_amdgcn_perm(tab_hi, tab_lo, R4[q]);
        }
        auto delta = [&](int c) -> int32_t {
          if constexpr (kByte)
            return (int32_t)((d4[c / 4] >> (8 * (c % 4))) & 0xffu);
          else
            return Rc[c] == T ? c_ma : Mi[c];
        };
        // The diagonal candidate of column c+1 is formed from the old H[c]
        // before H[c] is overwritten, so every update happens in place.
        int32_t diag = hd + delta(0);
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int32_t ad = H[c];   // G of the cell above: D-open candidate
          int32_t diag_next = 0;
          if (c + 1 < K) diag_next = H[c] + delta(c + 1);
          const int32_t ai = hl;     // G of the cell to the left: I-open candidate
          el = max(ai, el);
          const int32_t f = max(ad, F[c]);
          // score-only: the old H[c] is dead once the next diagonal and the
          // D-open candidate are formed; keeping the rest below lets the new
          // G take its register (otherwise it costs a copy per column)
          if constexpr (kScore) __builtin_amdgcn_sched_barrier(0);
          const int32_t h = max(max(diag, el), f);
          if constexpr (!kScore) {
            uint32_t a = acc[c / 8];
            a = push_sign(a, ai - el);
            a = push_sign(a, ad - f);
            a = push_sign(a, diag - h);
            a = push_sign(a, f - h);
            acc[c / 8] = a;
          }
          H[c] = h + c_go;
          F[c] = f;
          diag = diag_next;
          // keep each column's decisions next to its scores: without this the
          // optimiser sinks them below all columns and every column's
          // candidates stay live (bounds live registers)
          if constexpr (!kScore) asm volatile("" : "+v"(acc[c / 8]));
          else asm volatile("" : "+v"(H[c]));
          hl = H[c];   // read after the asm above, so it is the register H[c] holds
          __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (!kScore)
          if (K % 8) acc[W - 1] <<= 4 * (8 - K % 8);
        hl_out = hl;
        el_out = el;
        // M(i, n) - n S_GE = M^(i, n) + i S_GE = G - c_go + i S_GE
        const int32_t v = H[K - 1] + rge;
        if (last && v > best) { best = v; endi = i; }
      }
      if constexpr (!kScore) {
        const int u = t & (B - 1);
        stage_step<uint32_t, W, B>(s_lds, lane, u, acc);
        if (u == B - 1 || t == steps - 1) {   // block complete (or last step)
          __syncthreads();
          flush_block<uint32_t, W, B>(s_lds, lane, sp);
          sp += W * kWave * B;
          __syncthreads();
        }
      }
      bnd -= ge;
      rge += ge;
    }

    if (last) { s_end[u0] = endi; s_score[u0] = best; }
    ++r;
    item = p.work_counter ? next_item(p.work_counter, lane) : item + gridDim.x;
    if (r < defer && item < n_items) continue;

    // ---------------- traceback of the deferred items, one lane per task
    __syncthreads();
    if (lane < r * G) {
      const int64_t tk = s_task[lane];
      if (tk >= 0) {
        const uint8_t tst = s_st[lane];
        if (tst != kTaskOk) {
          p.score[tk] = 0; p.ref_begin[tk] = 0; p.ref_end[tk] = 0; p.cigar_len[tk] = 0;
          p.status[tk] = tst;
        } else {
          const int32_t tn = s_n[lane], tpad = s_pad[lane], tend = s_end[lane];
          const int32_t tscore = s_score[lane] + tn * p.ge;
          p.score[tk] = tscore;
          p.ref_end[tk] = tend;
          p.status[tk] = tscore < p.min_score ? kTaskBelowCutoff : p.ok_status;
          if (tscore < p.min_score) {   // below the cutoff: no traceback
            (void)tpad;
            p.ref_begin[tk] = -1;
            p.cigar_len[tk] = 0;
          } else if constexpr (kScore) {   // begin and CIGAR are not computed
            (void)tpad;
            p.ref_begin[tk] = -1;
            p.cigar_len[tk] = 0;
          } else {
            const int rs = lane / G, gq = lane % G;
            const uint32_t *slot = slots + (uint64_t)rs * slot_dwords;
            auto tr = make_tracer<uint32_t, K, W, B>(
                slot, s_lds + lane * B * tracer_blocks(W), gq * L, tpad,
                [](uint32_t wd, uint32_t c) { return (wd >> (4 * (7 - (c & 7)))) & 15u; });
            traceback_task(p, tk, tn, tend, (int32_t)slot_rows, tr);
          }
        }
      }
    }
    __syncthreads();
    r = 0;
  }
}

// ---------------------------------------------------------------- dispatch

#define SOAPDP_I32_SHAPES(X) \
  X(1, 8) X(2, 8) X(4, 9) X(4, 13) X(4, 19) X(4, 25) X(4, 38) X(8, 7) X(8, 10) X(8, 13) \
  X(8, 19) X(8, 32) X(16, 10) X(16, 16) X(32, 16) X(64, 8)

static const Shape kShapesI32[] = {
#define X(l, k) {l, k},
    SOAPDP_I32_SHAPES(X)
#undef X
};

uint64_t slot_dwords_i32(Shape s, int32_t max_m) {
  const uint64_t B = uint64_t(step_block(s.cells));
  const uint64_t steps = (uint64_t(max_m) + uint64_t(s.lanes) - 1 + B - 1) / B * B;
  return steps * uint64_t((s.cells + 7) / 8) * kWave;
}

const Shape *shapes_i32(int *count) {
  *count = (int)(sizeof(kShapesI32) / sizeof(kShapesI32[0]));
  return kShapesI32;
}

template <int L, int K>
hipError_t launch_i32(int grid, hipStream_t stream, const DpParams &p, bool byte, bool score) {
  if (byte && score)
    hipLaunchKernelGGL((dp_i32_kernel<L, K, true, true>), dim3(grid), dim3(kWave), 0, stream, p);
  else if (byte)
    hipLaunchKernelGGL((dp_i32_kernel<L, K, true, false>), dim3(grid), dim3(kWave), 0, stream, p);
  else if (score)
    hipLaunchKernelGGL((dp_i32_kernel<L, K, false, true>), dim3(grid), dim3(kWave), 0, stream, p);
  else
    hipLaunchKernelGGL((dp_i32_kernel<L, K, false, false>), dim3(grid), dim3(kWave), 0, stream, p);
  return hipGetLastError();
}

template <int L, int K>
int occupancy_i32(bool byte, bool score) {
  int blocks = 0;
  hipError_t e;
  if (byte && score)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, dp_i32_kernel<L, K, true, true>, kWave, 0);
  else if (byte)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, dp_i32_kernel<L, K, true, false>, kWave, 0);
  else if (score)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, dp_i32_kernel<L, K, false, true>, kWave, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, dp_i32_kernel<L, K, false, false>, kWave, 0);
  return e == hipSuccess ? blocks : 0;
}

hipError_t launch_dp_i32(Shape s, int grid, hipStream_t stream, const DpParams &p) {
  const bool byte = byte_delta_fits(p.ma, p.mi, p.go, p.ge);
#define X(l, k) \
  if (s.lanes == l && s.cells == k) return launch_i32<l, k>(grid, stream, p, byte, p.score_only != 0);
  SOAPDP_I32_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

int occupancy_dp_i32(Shape s, bool byte_delta, bool score_only) {
#define X(l, k) \
  if (s.lanes == l && s.cells == k) return occupancy_i32<l, k>(byte_delta, score_only);
  SOAPDP_I32_SHAPES(X)
#undef X
  return 0;
}

}  // namespace soapdp
