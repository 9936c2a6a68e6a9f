// Packed int16 fill + traceback kernel (batched form).  Same recurrences and
// tie-breaks as the int32 kernel (paper, Methods section 3), two tasks per
// lane: the low and high 16-bit halves of every register belong to two
// different tasks that share the lane geometry, so each packed VALU
// instruction advances two cells.
//
// Two forms.  The offset form (below) is the cheaper one and serves every
// task whose values provably stay inside int16.  The direct form (kDirect)
// keeps the true values, so nothing drifts with the window length, and lets
// low values saturate: it serves tasks the offset form's rule excludes,
// flags those whose score lies too close to the saturation floor to be
// exact (int16_direct_fits, direct_floor) and appends them to a list the
// int32 kernel re-runs.  It differs from the offset form in four places:
// gap extensions add S_GE, M is carried as G = M + S_GO, the left boundary
// is the constant M = 0, and the diagonal constant of a column pair is
// e * g + b from a byte table (one v_perm_b32 and one v_pk_mad_u16).
//
// Same offset form as the int32 kernel, X^(i,j) = X(i,j) - (i+j)*S_GE, so
// gap extension adds nothing.  Differences from the int32 kernel, all exact:
//  * The diagonal adds delta - 2 S_GE: S_MA - 2 S_GE on a match and
//    S_MI - 2 S_GE on a mismatch, small non-negative numbers read from an
//    8-byte table with one v_perm_b32 indexed by (read code XOR window base).
//    Columns left of the read (virtual, true value 0) index the table's upper
//    half, which holds -2 S_GE.
//  * Adds and subtracts saturate (v_pk_*_i16 clamp).  A task runs here only
//    if every value, widened by the largest constant added, stays well inside
//    int16 and the table entries fit a byte (int16_fits); clamped candidates
//    then always lose, and -32768 serves as minus infinity.  Other tasks are
//    left to the int32 kernel.
//  * Decision bits: the sign of each packed difference is replicated into a
//    byte with v_perm_b32 (selectors 8..11) and merged with v_and_or_b32 into
//    bit c%8 of that byte.  Per 8 columns a lane writes two dwords:
//      A: byte h = D extended, byte 2+h = I extended        (h = 0 low task,
//      B: byte h = not from D, byte 2+h = not diagonal         1 high task)
#include "dp_device.h"

namespace soapdp {

namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 v2(uint32_t x) { return __builtin_bit_cast(s16x2, x); }
__device__ __forceinline__ uint32_t u32(s16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t add16(uint32_t a, uint32_t b) {
  return u32(__builtin_elementwise_add_sat(v2(a), v2(b)));
}
__device__ __forceinline__ uint32_t sub16(uint32_t a, uint32_t b) {
  return u32(__builtin_elementwise_sub_sat(v2(a), v2(b)));
}
__device__ __forceinline__ uint32_t max16(uint32_t a, uint32_t b) {
  return u32(__builtin_elementwise_max(v2(a), v2(b)));
}
__device__ __forceinline__ uint32_t pack16(int32_t lo, int32_t hi) {
  return ((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16);
}
__device__ __forceinline__ int32_t clamp16(int32_t v) { return v < -32768 ? -32768 : (v > 32767 ? 32767 : v); }
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
// e * g + b on both halves, modulo 2^16 (the exact 16-bit pattern of a
// constant inside int16)
__device__ __forceinline__ uint32_t mad16(uint32_t e, uint32_t g, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, e) * __builtin_bit_cast(u16x2, g) +
                                          __builtin_bit_cast(u16x2, b));
}

constexpr uint32_t kNeg16x2 = 0x80008000u;   // (-32768, -32768)
constexpr uint32_t kSignSel = 0x0b0a0908u;   // v_perm: replicate the four sign bits

}  // namespace

// Waves per SIMD asked of the register allocator.  Shapes with at most 8
// columns per lane fit five (96 VGPRs) without spilling once the compiler
// is asked to.  The offset-form score sweeps are asked for three: the
// 4 x 38 one then spills a few values outside its row loop and made the
// low-similarity batched call 0.8% faster.  The kernels with traceback at
// 13-14 and 19-20 columns sit a few registers above four and three waves;
// their dense variant (kDense) is asked for those and fits without
// spilling.  At 32 columns the dense variant runs three waves instead of
// two with about 100 bytes spilled, mostly outside the row loop (the
// uneven batch ran 3% faster).  It serves large calls only: there each
// class kernel has work for many times its resident waves.  In served
// batches, whose class kernels are short and run side by side, it ran 2%
// below capacity and slower at low load, so small calls keep the default.
constexpr int waves_i16(int K, bool score, bool direct, bool dense) {
  return K <= 8 ? 5 : (score && !direct ? 3 : (!dense ? 1 : (K <= 16 ? 4 : 3)));
}
constexpr bool has_dense_i16(int K) { return K == 13 || K == 14 || K == 19 || K == 20 || K == 32; }

// kScore: score and end only -- no decision bits, no scratch, no traceback.
template <int L, int K, bool kScore, bool kDirect, bool kDense>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(waves_i16(K, kScore, kDirect, kDense))))
void dp_i16_kernel(DpParams p) {
  static_assert(kWave % L == 0, "lanes per task must divide the wavefront");
  constexpr int G = kWave / L;       // lane groups per wavefront
  constexpr int TPW = 2 * G;         // tasks per wavefront (low and high halves)
  static_assert(TPW <= kWave, "one traceback lane per task");
  constexpr int W = (K + 7) / 8;     // 8-column groups per lane
  const int lane = threadIdx.x;
  const int g = lane / L;
  const int lg = lane % L;
  const bool first = lg == 0;
  const bool last = lg == L - 1;

  // bookkeeping of the deferred work items, entry r * TPW + h * G + g
  __shared__ int64_t s_task[kWave];
  __shared__ int32_t s_n[kWave], s_pad[kWave], s_end[kWave], s_score[kWave];
  __shared__ uint8_t s_st[kWave];
  constexpr int B = step_block(K);   // sweep steps per stored block
  // staging buffer of the sweep, or the traceback's block caches
  __shared__ __align__(16) uint2 s_lds[kScore ? 2 : StageOrCache<uint2, W, B>::kWords];

  // `defer` work items are swept into consecutive slots before one
  // traceback pass serves all their tasks, one lane per task
  const int32_t defer = kScore ? 1 : min(max(p.defer_dev ? *p.defer_dev : p.defer, 1), kWave / TPW);
  const uint64_t slot_dwords = p.slot_dwords_dev ? *p.slot_dwords_dev : p.slot_dwords;
  uint32_t *const slots = p.scratch + (p.scratch_off_dev ? *p.scratch_off_dev : 0) +
                          (uint64_t)blockIdx.x * slot_dwords * (uint64_t)defer;
  // window rows a slot can hold: (rows + L - 1) steps of W * 64 lanes
  const int64_t slot_rows =
      kScore ? INT64_MAX : (int64_t)(slot_dwords / (uint64_t)(W * kWave * 2)) - (L - 1);
  int32_t r = 0;   // slot of the current work item
  const int64_t n_tasks = p.task_count ? (int64_t)*p.task_count : p.n_tasks;
  const int32_t *const list = (p.task_list && p.task_off) ? p.task_list + *p.task_off : p.task_list;
  const int64_t n_items = (n_tasks + TPW - 1) / TPW;

  const int32_t ma = p.ma, mi = p.mi, go = p.go, ge = p.ge;
  const int32_t go1 = go - ge;                        // gap open, offset form
  // H holds G = M^ + (S_GO - S_GE) (offset form) or G = M + S_GO (direct
  // form): the gap-open candidate of the cell to the right (same row) and
  // of the cell below (next row) without another add.
  const int32_t gadd = kDirect ? go : go1;
  const uint32_t c_go = pack16(gadd, gadd);
  const uint32_t c_ge = pack16(ge, ge);
  const uint32_t c_nge = pack16(-ge, -ge);
  // Diagonal constants relative to G, byte x = (read code XOR window base):
  // x = 0 match, 1..3 mismatch, 4..7 left of the read.  Offset form: the
  // constants themselves, delta - 2 S_GE - (S_GO - S_GE).  Direct form: the
  // multipliers e of e * g + b for delta - S_GO (0 - S_GO left of the read).
  DirectDelta dd{1, 0, 0, 0, 0};
  if constexpr (kDirect) direct_delta(ma, mi, go, &dd);
  const uint32_t tab_lo =
      kDirect ? ((uint32_t)dd.e_ma & 0xffu) | ((uint32_t)dd.e_mi & 0xffu) * 0x01010100u
              : ((uint32_t)(ma - 2 * ge - go1) & 0xffu) |
                    ((uint32_t)(mi - 2 * ge - go1) & 0xffu) * 0x01010100u;
  const uint32_t tab_hi = kDirect ? ((uint32_t)dd.e_v & 0xffu) * 0x01010101u
                                  : ((uint32_t)(-2 * ge - go1) & 0xffu) * 0x01010101u;
  const uint32_t c_dg = pack16(dd.g, dd.g), c_db = pack16(dd.b, dd.b);
  // diagonal constants of a column pair from the selector (code ^ base)
  auto dconst = [&](uint32_t sel) {
    const uint32_t e = __builtin_amdgcn_perm(tab_hi, tab_lo, sel);
    if constexpr (kDirect) return mad16(e, c_dg, c_db);
    else return e;
  };

  int64_t item = blockIdx.x;
  while (item < n_items) {
    // ---------------- set-up of the two tasks of this lane group
    int64_t task[2];
    int32_t n[2], m[2], pad[2], mg[2];
    uint64_t rwo[2], rbo[2];
    uint8_t st[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t tix = item * TPW + h * G + g;
      task[h] = -1; n[h] = 0; m[h] = 0; rwo[h] = 0; rbo[h] = 0; st[h] = kTaskOk;
      if (tix < n_tasks) {
        task[h] = task_at(p, list, tix);
        n[h] = p.read_len[task[h]];
        m[h] = p.ref_len[task[h]];
        rwo[h] = p.read_word_off[task[h]];
        rbo[h] = p.ref_base_off[task[h]];
        if (n[h] < 1 || m[h] < 1 || n[h] > p.max_n || m[h] > p.max_m || n[h] > L * K ||
            m[h] > slot_rows)
          st[h] = kTaskInvalidLen;
        else if (!read_in_bounds(rwo[h], n[h], p.read_words, p.read_stride) ||
                 rbo[h] + (uint64_t)m[h] > p.ref_words * 16)
          st[h] = kTaskInvalidOffset;
        else if (kDirect ? !int16_direct_fits(n[h], ma, mi, go, ge)
                         : !int16_fits(n[h], m[h], L * K, ma, mi, go, ge))
          task[h] = -1;   // outside this form's range: another kernel owns it
      }
      const bool valid = task[h] >= 0 && st[h] == kTaskOk;
      mg[h] = valid ? m[h] : 0;
      pad[h] = valid ? L * K - n[h] : 0;
    }
    const int32_t mlane = max(mg[0], mg[1]);
    // uniform trip count: keeps the step loop under scalar control
    const int32_t steps = __builtin_amdgcn_readfirstlane(wave_max(mlane)) + L - 1;
    // per-task bookkeeping for the traceback goes to LDS now, so it does not
    // occupy registers during the sweep
    if (first) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int u = r * TPW + h * G + g;
        s_task[u] = task[h]; s_n[u] = n[h]; s_pad[u] = pad[h]; s_st[u] = st[h];
      }
    }

    StripWords rw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      rw[h] = StripWords{0, 0, 0, 0};
      if (mg[h] > 0) rw[h].load(p.read_codes, rwo[h], n[h], lg * K - pad[h], p.read_stride);
    }
    uint32_t Rc[K], H[K], F[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      int32_t hv[2];
      uint32_t code[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int32_t q = lg * K + c - pad[h];   // 0-based read index of this column
        const bool real = mg[h] > 0 && q >= 0;
        code[h] = real ? rw[h].code(q) : 4u;     // virtual: table entries 4..7
        // offset form: M^(0, j), j = q + 1: S_GO + (j-1) S_GE - j S_GE, or
        // 0 - j S_GE left of the read, held as G = M^ + (S_GO - S_GE);
        // direct form: M(0, j) = S_GO + (j-1) S_GE (0 left of the read) as
        // G = M + S_GO, saturated
        hv[h] = kDirect ? clamp16((real ? go + q * ge : 0) + go)
                        : (real ? go1 : -(q + 1) * ge) + go1;
      }
      Rc[c] = (code[0] | 0x0c00u) | ((code[1] | 0x0c00u) << 16);
      H[c] = pack16(hv[0], hv[1]);
      F[c] = kNeg16x2;
      // finish each column before the next: bounds live registers in set-up
      asm volatile("" : "+v"(Rc[c]), "+v"(H[c]));
      __builtin_amdgcn_sched_barrier(0);
    }
    // left boundary M^(i, -pad) = -(i - pad) S_GE (true value 0), as G: row 0
    // is the first lane's first diagonal, row 1 its first left neighbour
    // (direct form: the constant M = 0 as G = S_GO)
    uint32_t bnd = kDirect ? pack16(go, go) : pack16((pad[0] - 1) * ge + go1, (pad[1] - 1) * ge + go1);
    // i * S_GE of this lane's row, minus (S_GO - S_GE) (direct form: -S_GO,
    // so that G + rge is M)
    uint32_t rge = kDirect ? pack16(-go, -go) : pack16((1 - lg) * ge - go1, (1 - lg) * ge - go1);

    // window bases, 16 at a time per task, realigned from the base offset
    const uint64_t wlim = p.ref_words - 1;
    const int32_t wsh0 = (int32_t)(rbo[0] & 15) * 2, wsh1 = (int32_t)(rbo[1] & 15) * 2;
    auto ldw = [&](uint64_t wi) { return p.ref_codes[wi < wlim ? wi : wlim]; };
    uint32_t a0 = ldw(rbo[0] >> 4), a1 = ldw((rbo[0] >> 4) + 1);
    uint32_t b0 = ldw(rbo[1] >> 4), b1 = ldw((rbo[1] >> 4) + 1);
    uint32_t twa = 0, twb = 0;

    uint32_t hl_out = H[K - 1];
    uint32_t el_out = kNeg16x2;
    uint32_t t_out = 0;
    uint32_t hl_prev = kDirect ? pack16(go, go) : pack16(pad[0] * ge + go1, pad[1] * ge + go1);
    int32_t best0 = INT32_MIN, best1 = INT32_MIN;
    uint32_t accA[W], accB[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { accA[w] = 0; accB[w] = 0; }

    uint2 *sp = reinterpret_cast<uint2 *>(slots + (uint64_t)r * slot_dwords);
    for (int32_t t = 0; t < steps; ++t) {
      if ((t & 15) == 0) {
        twa = __builtin_amdgcn_alignbit(a1, a0, wsh0);
        twb = __builtin_amdgcn_alignbit(b1, b0, wsh1);
        const uint64_t nb = (uint64_t)(t >> 4) + 1;
        a0 = ldw((rbo[0] >> 4) + nb); a1 = ldw((rbo[0] >> 4) + nb + 1);
        b0 = ldw((rbo[1] >> 4) + nb); b1 = ldw((rbo[1] >> 4) + nb + 1);
      }
      const uint32_t sh = (uint32_t)(t & 15) * 2;
      const uint32_t tfirst = ((twa >> sh) & 3u) | (((twb >> sh) & 3u) << 16);
      // the first lane of a task receives the left boundary and the row's
      // window base; its diagonal is the boundary received one step earlier
      uint32_t hl = (uint32_t)group_shr1<L>((int32_t)hl_out, (int32_t)bnd, first);
      uint32_t el = (uint32_t)group_shr1<L>((int32_t)el_out, (int32_t)kNeg16x2, first);
      const uint32_t T = (uint32_t)group_shr1<L>((int32_t)t_out, (int32_t)tfirst, first);
      const uint32_t hd = hl_prev;
      hl_prev = hl;
      t_out = T;
      const int32_t i = t + 1 - lg;
      if ((uint32_t)(t - lg) < (uint32_t)mlane) {   // 1 <= i <= mlane
        // The diagonal candidate of column c+1 is formed from the old H[c]
        // before H[c] is overwritten, so every update happens in place.
        uint32_t diag = add16(hd, dconst(Rc[0] ^ T));
        if constexpr (kScore) {
          // Score only: the same recurrences in a fixed issue order.  A
          // packed result read by the next packed instruction costs a wait
          // state, so the serial chain of a column (I, max, max, new G, then
          // the next column's I) is interleaved with independent work: the
          // next column's diagonal constant and this column's D candidate.
          // The next diagonal reads the old H[c] before the new G overwrites
          // it, so the update stays in place.
#pragma unroll
          for (int c = 0; c < K; ++c) {
            uint32_t fg = F[c], eg = el;
            if constexpr (kDirect) {
              fg = add16(F[c], c_ge);
              __builtin_amdgcn_sched_barrier(0);
              eg = add16(el, c_ge);
              __builtin_amdgcn_sched_barrier(0);
            }
            const uint32_t f = max16(H[c], fg);      // D: open from above or extend
            __builtin_amdgcn_sched_barrier(0);
            el = max16(hl, eg);                      // I: open from the left or extend
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t x = c + 1 < K ? Rc[c + 1] ^ T : 0u;
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t tv = max16(diag, el);
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t dc = c + 1 < K ? dconst(x) : 0u;
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t hv = max16(tv, f);
            __builtin_amdgcn_sched_barrier(0);
            if (c + 1 < K) diag = add16(H[c], dc);
            __builtin_amdgcn_sched_barrier(0);
            H[c] = add16(hv, c_go);
            F[c] = f;
            hl = H[c];
            __builtin_amdgcn_sched_barrier(0);
          }
        } else
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const uint32_t ad = H[c];   // G of the cell above: D-open candidate
          uint32_t diag_next = 0;
          if (c + 1 < K) diag_next = add16(H[c], dconst(Rc[c + 1] ^ T));
          const uint32_t ai = hl;     // G of the cell to the left: I-open candidate
          // gap extension: free in the offset form, + S_GE in the direct form
          el = max16(ai, kDirect ? add16(el, c_ge) : el);
          const uint32_t f = max16(ad, kDirect ? add16(F[c], c_ge) : F[c]);
          const uint32_t hv = max16(max16(diag, el), f);
          // differences against the maxima, so the old I and D die at the max
          // and the new values take their registers
          {
            const uint32_t tA = __builtin_amdgcn_perm(sub16(ai, el), sub16(ad, f), kSignSel);
            const uint32_t tB = __builtin_amdgcn_perm(sub16(diag, hv), sub16(f, hv), kSignSel);
            const uint32_t msk = 0x01010101u << (c & 7);
            if ((c & 7) == 0) {
              accA[c / 8] = tA & msk;
              accB[c / 8] = tB & msk;
            } else {
              accA[c / 8] |= tA & msk;
              accB[c / 8] |= tB & msk;
            }
          }
          H[c] = add16(hv, c_go);
          F[c] = f;
          diag = diag_next;
          // keep each column's decisions next to its scores: without this the
          // optimiser sinks them below all columns and every column's
          // candidates stay live (bounds live registers)
          asm volatile("" : "+v"(accA[c / 8]), "+v"(accB[c / 8]));
          hl = H[c];
          __builtin_amdgcn_sched_barrier(0);
        }
        hl_out = hl;
        el_out = el;
        if (last) {
          // key = ((M^(i, n) + i S_GE) << 16) | (0xffff - i): the max is the
          // best score M(i, n) - n S_GE, then the smallest row (H holds
          // M^ + (S_GO - S_GE), which rge takes off again)
          const uint32_t inv = 0xffffu - (uint32_t)i;
          const uint32_t v = add16(H[K - 1], rge);
          const int32_t k0 = (int32_t)((v << 16) | inv);
          const int32_t k1 = (int32_t)((v & 0xffff0000u) | inv);
          if (i <= mg[0]) best0 = max(best0, k0);
          if (i <= mg[1]) best1 = max(best1, k1);
        }
      }
      if constexpr (!kScore) {
        uint2 v[W];
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] = make_uint2(accA[w], accB[w]);
        const int u = t & (B - 1);
        stage_step<uint2, W, B>(s_lds, lane, u, v);
        if (u == B - 1 || t == steps - 1) {   // block complete (or last step)
          __syncthreads();
          flush_block<uint2, W, B>(s_lds, lane, sp);
          sp += W * kWave * B;
          __syncthreads();
        }
      }
      if constexpr (!kDirect) {
        bnd = add16(bnd, c_nge);
        rge = add16(rge, c_ge);
      }
    }

#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int u = r * TPW + h * G + g;
      if (last) {
        const int32_t b = h ? best1 : best0;
        s_end[u] = 0xffff - (b & 0xffff);
        s_score[u] = b >> 16;   // M(end, n) - n S_GE; the traceback lane adds n S_GE
      }
    }
    ++r;
    item = p.work_counter ? next_item(p.work_counter, lane) : item + gridDim.x;
    if (r < defer && item < n_items) continue;

    // ---------------- traceback of the deferred items, one lane per task
    __syncthreads();
    if (lane < r * TPW) {
      const int64_t tk = s_task[lane];
      if (tk >= 0) {
        const uint8_t tst = s_st[lane];
        if (tst != kTaskOk) {
          p.score[tk] = 0; p.ref_begin[tk] = 0; p.ref_end[tk] = 0; p.cigar_len[tk] = 0;
          p.status[tk] = tst;
        } else {
          const int rs = lane / TPW, ui = lane % TPW;
          const int h = ui / G, gq = ui % G;
          const int32_t tn = s_n[lane], tpad = s_pad[lane], tend = s_end[lane];
          const int32_t tscore = kDirect ? s_score[lane] : s_score[lane] + tn * ge;
          p.score[tk] = tscore;
          p.ref_end[tk] = tend;
          p.status[tk] = tscore < p.min_score ? kTaskBelowCutoff : p.ok_status;
          if (kDirect && tscore <= direct_floor(tn, ma, go)) {
            // too close to the saturation floor to be exact: int32 re-run
            (void)tpad;
            p.status[tk] = kTaskNeedsRedo;
            p.ref_begin[tk] = -1;
            p.cigar_len[tk] = 0;
            p.redo_list[atomicAdd(p.redo_count, 1)] = (int32_t)tk;
          } else if (tscore < p.min_score) {   // below the cutoff: no traceback
            (void)tpad;
            p.ref_begin[tk] = -1;
            p.cigar_len[tk] = 0;
          } else if constexpr (kScore) {   // begin and CIGAR are not computed
            (void)rs; (void)h; (void)gq; (void)tpad;
            p.ref_begin[tk] = -1;
            p.cigar_len[tk] = 0;
          } else {
            const uint2 *slot = reinterpret_cast<const uint2 *>(slots + (uint64_t)rs * slot_dwords);
            const uint32_t shA = 8u * (2 + h), shD = 8u * h;
            auto tr = make_tracer<uint2, K, W, B>(
                slot, s_lds + lane * B * tracer_blocks(W), gq * L, tpad, [shA, shD](uint2 v, uint32_t c) {
                  const uint32_t b = c & 7u;
                  return ((v.x >> (shA + b)) & 1u) << 3 | ((v.x >> (shD + b)) & 1u) << 2 |
                         ((v.y >> (shA + b)) & 1u) << 1 | ((v.y >> (shD + b)) & 1u);
                });
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

#define SOAPDP_I16_SHAPES(X)                                                            \
  X(2, 8) X(4, 4) X(4, 8) X(2, 16) X(4, 10) X(8, 5) X(4, 14) X(8, 7) X(4, 16) X(8, 8)   \
  X(4, 20) X(8, 10) X(8, 13) X(4, 26) X(16, 7) X(8, 16) X(4, 32) X(16, 8) X(8, 19)      \
  X(16, 10) X(8, 24) X(4, 38) X(8, 32)                                                  \
  X(16, 12) X(16, 16) X(32, 8) X(16, 20) X(32, 10) X(16, 24) X(32, 12) X(32, 16) X(64, 8)

static const Shape kShapesI16[] = {
#define X(l, k) {l, k},
    SOAPDP_I16_SHAPES(X)
#undef X
};

const Shape *shapes_i16(int *count) {
  *count = (int)(sizeof(kShapesI16) / sizeof(kShapesI16[0]));
  return kShapesI16;
}

uint64_t slot_dwords_i16(Shape s, int32_t max_m) {
  const uint64_t B = uint64_t(step_block(s.cells));
  const uint64_t steps = (uint64_t(max_m) + uint64_t(s.lanes) - 1 + B - 1) / B * B;
  return steps * uint64_t((s.cells + 7) / 8) * kWave * 2;
}

template <int L, int K, bool kScore, bool kDirect>
void launch_v16(int grid, hipStream_t stream, const DpParams &p, bool dense) {
  if constexpr (!kScore && has_dense_i16(K)) {
    if (dense) {
      hipLaunchKernelGGL((dp_i16_kernel<L, K, kScore, kDirect, true>), dim3(grid), dim3(kWave), 0,
                         stream, p);
      return;
    }
  }
  hipLaunchKernelGGL((dp_i16_kernel<L, K, kScore, kDirect, false>), dim3(grid), dim3(kWave), 0,
                     stream, p);
}

template <int L, int K>
hipError_t launch_i16(int grid, hipStream_t stream, const DpParams &p, bool direct, bool dense) {
  const bool score = p.score_only != 0;
  if (score && direct)
    launch_v16<L, K, true, true>(grid, stream, p, dense);
  else if (score)
    launch_v16<L, K, true, false>(grid, stream, p, dense);
  else if (direct)
    launch_v16<L, K, false, true>(grid, stream, p, dense);
  else
    launch_v16<L, K, false, false>(grid, stream, p, dense);
  return hipGetLastError();
}

template <int L, int K, bool kScore, bool kDirect>
hipError_t occupancy_v16(int *blocks, bool dense) {
  if constexpr (!kScore && has_dense_i16(K)) {
    if (dense)
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          blocks, dp_i16_kernel<L, K, kScore, kDirect, true>, kWave, 0);
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks, dp_i16_kernel<L, K, kScore, kDirect, false>, kWave, 0);
}

template <int L, int K>
int occupancy_i16(bool score, bool direct, bool dense) {
  int blocks = 0;
  hipError_t e;
  if (score && direct)
    e = occupancy_v16<L, K, true, true>(&blocks, dense);
  else if (score)
    e = occupancy_v16<L, K, true, false>(&blocks, dense);
  else if (direct)
    e = occupancy_v16<L, K, false, true>(&blocks, dense);
  else
    e = occupancy_v16<L, K, false, false>(&blocks, dense);
  return e == hipSuccess ? blocks : 0;
}

hipError_t launch_dp_i16(Shape s, int grid, hipStream_t stream, const DpParams &p, bool direct,
                         bool dense) {
#define X(l, k) \
  if (s.lanes == l && s.cells == k) return launch_i16<l, k>(grid, stream, p, direct, dense);
  SOAPDP_I16_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

bool has_dense_dp_i16(Shape s) { return has_dense_i16(s.cells); }

int occupancy_dp_i16(Shape s, bool score_only, bool direct, bool dense) {
#define X(l, k) \
  if (s.lanes == l && s.cells == k) return occupancy_i16<l, k>(score_only, direct, dense);
  SOAPDP_I16_SHAPES(X)
#undef X
  return 0;
}

}  // namespace soapdp
