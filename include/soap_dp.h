/*
 * soap_dp.h -- C ABI of libsoapdp, batched read-vs-window affine-gap
 * alignment on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, Methods section 3, "GPU-accelerated dynamic
 * programming"): for each task, a read R of length n and a candidate region
 * (reference window) T of length m, find the sub-region T' of T whose
 * alignment score with the whole of R is maximal.  With delta(x,y) = S_MA if
 * x == y else S_MI, and gap scores S_GO (first base of a gap) and S_GE (each
 * further base):
 *
 *   I(i,j) = max(M(i,j-1) + S_GO, I(i,j-1) + S_GE)
 *   D(i,j) = max(M(i-1,j) + S_GO, D(i-1,j) + S_GE)
 *   M(i,j) = max(M(i-1,j-1) + delta(T[i], R[j]), I(i,j), D(i,j))
 *   I(i,0) = D(0,j) = -inf,  M(i,0) = 0,  M(0,j) = S_GO + (j-1) S_GE
 *
 * score = max_{1<=i<=m} M(i,n).  The read is aligned end to end; the window
 * is free at both ends; there is no zero floor.
 *
 * Outputs are exact integers and deterministic:
 *   ref_end    the smallest i reaching the score (0-based exclusive end)
 *   ref_begin  0-based start of T', so T' = T[ref_begin, ref_end)
 *   cigar      BAM-encoded runs (len << 4 | op), op M = 0, I = 1, D = 2,
 *              no soft clips (a leading or trailing I is kept)
 * Ties in the traceback prefer, at an M cell, the diagonal, then D, then I;
 * inside a gap, opening before extending.
 *
 * Sequences are 2-bit codes A=0, C=1, G=2, T=3, sixteen to a 32-bit word,
 * base k of a word in bits [2k, 2k+2).
 *
 * All functions return SOAP_DP_OK (0) or a negative error code; on error
 * nothing has been enqueued.  Per-task problems do not fail a batch: they
 * are reported in result.status.
 */
#ifndef SOAP_DP_H
#define SOAP_DP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes (return values) ---- */
#define SOAP_DP_OK 0
#define SOAP_DP_EINVAL (-1)   /* bad scoring, null pointer, size or stride */
#define SOAP_DP_ENOMEM (-2)   /* workspace could not be allocated */
#define SOAP_DP_EHIP (-3)     /* HIP runtime error; see soap_dp_last_hip_error */
#define SOAP_DP_ENODEV (-4)   /* no usable gfx950 device */

/* ---- per-task status (result.status) ---- */
#define SOAP_DP_TASK_OK 0
#define SOAP_DP_TASK_INVALID_LEN 1     /* n or m < 1, or above the batch bounds / limits */
#define SOAP_DP_TASK_OK_REDONE_INT32 2 /* OK; the int16 form's range did not cover this task,
                                          so it was computed by the exact int32 kernel */
#define SOAP_DP_TASK_INVALID_OFFSET 3  /* read or window lies outside its buffer */
#define SOAP_DP_TASK_NO_CANDIDATE 4    /* multi-candidate call: the read has no valid
                                          candidate region; mate rescue: the region
                                          lies outside the sequence */
#define SOAP_DP_TASK_BELOW_CUTOFF 5    /* SOAP_DP_MIN_SCORE: the best score is below
                                          scoring.min_score; score and ref_end are
                                          reported, ref_begin is -1, no CIGAR */

/* ---- limits ---- */
#define SOAP_DP_MAX_READ 512      /* n; the paper does not recommend reads over 500 bp */
#define SOAP_DP_MAX_WINDOW 8192   /* m */
#define SOAP_DP_MAX_SCORE_ABS 16384
#define SOAP_DP_NOALLOC_BYTES ((size_t)256 << 20)   /* fixed memory of soap_dp_align_batch_noalloc */

/* ---- flags for soap_dp_align_batch ---- */
#define SOAP_DP_PLAIN 0u    /* one int32 launch, one kernel shape for the whole batch */
#define SOAP_DP_BATCHED 1u  /* device-side length bucketing, packed int16 with int32 redo of
                               tasks outside the int16 range, persistent kernels with a
                               work queue, autotuned shapes; with SOAPDP_GRAPHS=1 in the
                               environment each distinct call is captured once and
                               replayed as a hipGraph */
#define SOAP_DP_SCORE_ONLY 2u  /* OR-ed with either form: score and ref_end only (same values
                                  as the full call); no traceback: ref_begin is -1, cigar_len
                                  0, `cigar` untouched and may be NULL with any stride */
#define SOAP_DP_MIN_SCORE 4u   /* OR-ed with either form: a task whose best score is below
                                  scoring.min_score is reported without traceback, with
                                  status SOAP_DP_TASK_BELOW_CUTOFF (score and ref_end as
                                  usual, ref_begin -1, cigar_len 0); the paper's aligner
                                  accepts an alignment only above a score threshold (its
                                  default limits for a 100 bp read, one gap of up to 68 bp
                                  or up to 23 one-base gaps, meet at one threshold) */
#define SOAP_DP_FULL_WINDOW 8u /* OR-ed with either form: decision bits for every cell of the
                                  window in one pass.  Without it a call with traceback runs
                                  two passes: score and end of every task first (no decision
                                  bits), then decision bits and traceback only over the window
                                  rows an optimal alignment can reach.  With S_GE < 0 an
                                  alignment of score S deletes at most
                                  Dmax = 1 + (n S_MA + S_GO - S) / |S_GE| window bases (none
                                  when n S_MA + S_GO < S), so it starts at row
                                  max(0, end - n - Dmax) or later; with S_GE = 0 the band is the
                                  whole window.  Outputs are identical either way. */
#define SOAP_DP_READS_INTERLEAVED 16u /* soap_dp_align_batch only, OR-ed with either form:
                                  word k of read t is read_codes[read_word_off[t] + 32 k]
                                  instead of read_codes[read_word_off[t] + k], i.e. reads
                                  stored word by word in groups of 32 (the paper's layout
                                  for a warp of one-problem threads, Methods section 1).
                                  A read whose last word lies at or past read_words gets
                                  SOAP_DP_TASK_INVALID_OFFSET.  Outputs are the same as
                                  for the same reads stored one after another. */

/*
 * Scores, all signed and added.  A gap of k bases scores
 * gap_open + (k-1) * gap_extend.  Valid: 0 < match <= 2^14,
 * mismatch < match, gap_open <= gap_extend <= 0, gap_open < 0,
 * |every score| <= 2^14.  (BWA's "open q, extend r" convention maps to
 * gap_open = -(q + r), gap_extend = -r.)  min_score is read only under
 * SOAP_DP_MIN_SCORE: scores >= min_score pass.
 */
typedef struct {
  int32_t match;
  int32_t mismatch;
  int32_t gap_open;
  int32_t gap_extend;
  int32_t min_score;
} soap_dp_scoring;

/*
 * A batch of tasks.  Array pointers are DEVICE pointers, caller-owned, read
 * only to the library, and must stay valid until the enqueued work has
 * completed.  Scalars are host values.
 *   read_codes     packed reads; read t starts at word read_word_off[t]
 *   read_len       n_t, 1 <= n_t <= max_n
 *   ref_codes      packed windows or a packed genome; window t starts at
 *                  BASE offset ref_base_off[t] (any alignment), so windows
 *                  can be cut from a device-resident genome without copies
 *   ref_len        m_t, 1 <= m_t <= max_m
 *   n_tasks        number of tasks (0 is a no-op)
 *   max_n, max_m   host-side bounds on every n_t and m_t (1..512, 1..8192);
 *                  they size the workspace and the plain kernel's shape.
 *                  A task above them gets SOAP_DP_TASK_INVALID_LEN.
 *   read_words     words in read_codes, ref_words words in ref_codes; a task
 *                  whose data would lie outside gets SOAP_DP_TASK_INVALID_OFFSET
 */
typedef struct {
  const uint32_t *read_codes;
  const uint64_t *read_word_off;
  const int32_t *read_len;
  const uint32_t *ref_codes;
  const uint64_t *ref_base_off;
  const int32_t *ref_len;
  int64_t n_tasks;
  int32_t max_n;
  int32_t max_m;
  uint64_t read_words;
  uint64_t ref_words;
} soap_dp_batch;

/*
 * Outputs, DEVICE pointers, caller-owned, n_tasks entries each (cigar:
 * n_tasks * cigar_stride words).  cigar_stride >= 2 * max_n - 1, the most
 * runs an alignment of an n-base read can have.  Every task's outputs are
 * written, zeros for an invalid task.
 */
typedef struct {
  int32_t *score;
  int32_t *ref_begin;
  int32_t *ref_end;
  uint32_t *cigar;
  int32_t cigar_stride;
  int32_t *cigar_len;
  uint8_t *status;
} soap_dp_result;

typedef struct soap_dp_ctx soap_dp_ctx;

/* Create a context on HIP device `device_ordinal`.  The context owns the
 * device workspace (decision-bit scratch, bucketing arrays), the autotune
 * table and the graph cache.  Returns SOAP_DP_ENODEV unless the device is
 * gfx950. */
int soap_dp_create(soap_dp_ctx **ctx, int device_ordinal);

/* Release everything the context owns (synchronises the device first). */
int soap_dp_destroy(soap_dp_ctx *ctx);

/*
 * Enqueue the alignment of `in` on `stream` (a hipStream_t; NULL is the null
 * stream) and return.  Results are valid once the stream has synchronised.
 * `flags` is SOAP_DP_PLAIN or SOAP_DP_BATCHED (both give identical outputs),
 * optionally OR-ed with SOAP_DP_SCORE_ONLY and SOAP_DP_MIN_SCORE; other bits
 * are SOAP_DP_EINVAL.
 * The library keeps no pointer to caller buffers after the work completes.
 * One context serves one stream at a time: calls on a context must not
 * overlap in time on different streams (use one context per stream).
 */
int soap_dp_align_batch(soap_dp_ctx *ctx, const soap_dp_batch *in, const soap_dp_scoring *sc,
                        const soap_dp_result *out, void *stream, uint32_t flags);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, hosts that forbid allocation): the plain
 * form of soap_dp_align_batch with the same outputs, which allocates
 * nothing.  Its work counter and decision slots live in one fixed device
 * array of SOAP_DP_NOALLOC_BYTES per device (256 MiB), which each device
 * holds from soap_dp_create until the process ends.
 *  - flags: SOAP_DP_SCORE_ONLY, SOAP_DP_MIN_SCORE, SOAP_DP_READS_INTERLEAVED
 *    and SOAP_DP_FULL_WINDOW as for soap_dp_align_batch; SOAP_DP_BATCHED and
 *    other bits are SOAP_DP_EINVAL.  The call always sweeps whole windows in
 *    one pass (the two-pass arrays would need memory per task).
 *  - When the decision slots of every workgroup do not fit the array, fewer
 *    workgroups run (slower, same results).  A window so long that one
 *    workgroup's slot exceeds the array is SOAP_DP_E2BIG.
 *  - Every call on one device shares that device's array and overwrites
 *    what the last call left there: calls that overlap in time on one
 *    device, from any context or stream, race and give wrong results.
 *    Order them (one stream, or events).
 * Argument meaning, layout, ownership and the other errors are those of
 * soap_dp_align_batch.
 */
int soap_dp_align_batch_noalloc(soap_dp_ctx *ctx, const soap_dp_batch *in,
                                const soap_dp_scoring *sc, const soap_dp_result *out,
                                void *stream, uint32_t flags);

/* Device bytes of workspace a call with these bounds needs (allocated by the
 * context on first use and kept). */
size_t soap_dp_workspace_bytes(const soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n,
                               int32_t max_m, uint32_t flags);

/* Allocate the workspace for these bounds now, so later calls allocate
 * nothing (needed before capturing a call into a hipGraph). */
int soap_dp_reserve(soap_dp_ctx *ctx, int64_t n_tasks, int32_t max_n, int32_t max_m,
                    uint32_t flags);

/*
 * Length classes of the batched form.  Each task goes to the smallest class
 * whose capacity (upper bound on read length) holds its read: an int16 class
 * when all of the task's values fit int16, else an int32 class.  Each class
 * runs one kernel shape: `lanes` lanes of a 64-wide wavefront cooperate on a
 * task, each owning `cells` read columns (lanes * cells >= capacity).
 */
typedef struct {
  int32_t precision;  /* 16 or 32 */
  int32_t capacity;
  int32_t lanes;
  int32_t cells;
} soap_dp_class_info;

/* Choose the fastest compiled shape for every class by timing each candidate
 * on synthetic reads of the class's capacity on this device, once for the
 * kernels with traceback and once for the score-only kernels
 * (SOAP_DP_SCORE_ONLY), which may run a different shape.  With a non-NULL
 * `cache_path`, a cache written earlier for the same device kind is loaded
 * instead (unless `force`), and a fresh result is written there (JSON).
 * Synchronises the device; replaces cached graphs. */
int soap_dp_autotune(soap_dp_ctx *ctx, const char *cache_path, int force);

/* Copy up to n_max class descriptions (the shapes with traceback); returns
 * the number of classes. */
int soap_dp_get_classes(const soap_dp_ctx *ctx, soap_dp_class_info *out, int32_t n_max);

/* Set the shape of the class (precision, capacity), for both kinds of
 * kernel; the shape must be a compiled one with lanes * cells >= capacity
 * (see soap_dp_list_shapes). */
int soap_dp_set_class_shape(soap_dp_ctx *ctx, int32_t precision, int32_t capacity, int32_t lanes,
                            int32_t cells);

/* The compiled shapes of a precision (capacity = lanes * cells); returns the
 * count, writes up to n_max. */
int soap_dp_list_shapes(int32_t precision, soap_dp_class_info *out, int32_t n_max);

/* ------------------------------------------------------------------------
 * Multi-candidate alignment with an effort limit (paper, Methods section 4:
 * candidate regions are ranked by their number of supporting seeds and only
 * the best `ceiling` of them are aligned by dynamic programming).
 *
 * Read r owns candidates [cand_start[r], cand_start[r+1]).  A candidate is
 * valid if 1 <= cand_len <= max_m and its window lies inside ref_codes;
 * invalid candidates are skipped before ranking.  The valid ones are ranked
 * by cand_support, highest first, ties by lower candidate index, and the
 * first min(count, ceiling) are aligned: strand 0 aligns the read, strand 1
 * its reverse complement (codes 3 - c, reversed), against the window as
 * stored.  The result is the best of them -- highest score, ties to the
 * earlier rank -- with its begin, end (window coordinates of that
 * candidate) and CIGAR, plus the best score among the other aligned
 * candidates.  Statuses: SOAP_DP_TASK_OK (or OK_REDONE_INT32),
 * INVALID_LEN / INVALID_OFFSET for the read itself, NO_CANDIDATE.
 * ------------------------------------------------------------------------ */
#define SOAP_DP_MAX_CEILING 64

typedef struct {
  /* reads, DEVICE pointers, caller-owned, as in soap_dp_batch */
  const uint32_t *read_codes;
  const uint64_t *read_word_off;
  const int32_t *read_len;
  uint64_t read_words;
  /* candidate regions, DEVICE pointers, caller-owned */
  const int64_t *cand_start;       /* n_reads + 1 entries, non-decreasing, last = n_cands */
  const uint64_t *cand_base_off;   /* window start, in bases into ref_codes */
  const int32_t *cand_len;         /* window length m */
  const int32_t *cand_support;     /* ranking key (e.g. supporting seeds) */
  const uint8_t *cand_strand;      /* 0: the read, 1: its reverse complement */
  const uint32_t *ref_codes;       /* packed sequence the windows index */
  uint64_t ref_words;
  int64_t n_reads;
  int64_t n_cands;
  int32_t max_n, max_m;            /* bounds on read and window lengths */
  int32_t ceiling;                 /* 1 .. SOAP_DP_MAX_CEILING */
} soap_dp_multi_batch;

/* Outputs, DEVICE pointers, caller-owned, n_reads entries each (cigar:
 * n_reads * cigar_stride words, cigar_stride >= 2 * max_n - 1). */
typedef struct {
  int32_t *score;
  int32_t *ref_begin;
  int32_t *ref_end;
  int64_t *best_cand;      /* candidate index of the result, -1 if none */
  int32_t *second_score;   /* best score of the other aligned candidates, INT32_MIN if none */
  int32_t *n_aligned;      /* candidates aligned for the read */
  uint32_t *cigar;
  int32_t cigar_stride;
  int32_t *cigar_len;
  uint8_t *status;
} soap_dp_multi_result;

/* Enqueue on `stream` like soap_dp_align_batch: all candidates are first
 * scored (score-only batched form), then each read's best one is aligned
 * again with traceback.  Same error codes; the context's workspace grows
 * with the reads and min(n_cands, n_reads * ceiling).  cand_start must be
 * non-decreasing, so that the lists do not overlap; if any entry is smaller
 * than the one before it, every read of the call gets
 * SOAP_DP_TASK_INVALID_OFFSET (n_aligned 0).  Otherwise a read whose list
 * lies outside [0, n_cands) gets SOAP_DP_TASK_INVALID_OFFSET on its own. */
int soap_dp_align_multi(soap_dp_ctx *ctx, const soap_dp_multi_batch *in, const soap_dp_scoring *sc,
                        const soap_dp_multi_result *out, void *stream);

/* ------------------------------------------------------------------------
 * Mate rescue (paper, Results: step 2 of the three-step pipeline; Methods:
 * paired-end alignment).  For a pair with one end aligned, the other end
 * is aligned against the region where the expected fragment length range
 * [min_frag, max_frag] (the -v / -u settings) and the orientation of the
 * ends place it.  The regions are computed on the device.
 *
 * Pair r's aligned end covers forward-strand bases [mate_pos, mate_pos +
 * mate_len) of ref_codes, on strand mate_strand (0 forward, 1 reverse).  A
 * fragment runs from the outer end of one read to the outer end of the
 * other; its length L satisfies min_frag <= L <= max_frag.  The
 * orientation says where the unaligned end (the mate, length n) lies,
 * relative to the aligned end: on the same or the opposite strand, and
 * downstream (further along the aligned end's own strand) or upstream.
 * The mate lies toward higher coordinates when it is downstream of a
 * forward end or upstream of a reverse one.  The region is the union of
 * the mate's placements over all L:
 *   toward higher coordinates: [mate_pos + min_frag - n, mate_pos + max_frag)
 *   toward lower coordinates:  [mate_pos + mate_len - max_frag,
 *                               mate_pos + mate_len - min_frag + n)
 * clipped to [0, ref_len).  A mate on the reverse strand is aligned as its
 * reverse complement (codes 3 - c, reversed) against the region as stored.
 * Outputs: the region's start, length and the mate's strand, and the
 * alignment in region coordinates (score, begin, end, CIGAR), as from
 * soap_dp_align_batch.  Statuses: SOAP_DP_TASK_OK (or OK_REDONE_INT32);
 * INVALID_LEN for n outside 1..max_n or mate_len < 1; INVALID_OFFSET for a
 * read outside read_codes; NO_CANDIDATE when the clipped region is empty.
 * Pairs with a non-OK status have zero outputs.
 * ------------------------------------------------------------------------ */
#define SOAP_DP_ORIENT_FR 0     /* opposite strand, downstream (Illumina paired ends) */
#define SOAP_DP_ORIENT_FF 1     /* same strand, downstream (SOLiD) */
#define SOAP_DP_ORIENT_RF 2     /* opposite strand, upstream (outward-facing) */
#define SOAP_DP_ORIENT_FF_UP 3  /* same strand, upstream */

typedef struct {
  /* unaligned ends, DEVICE pointers, caller-owned, as in soap_dp_batch */
  const uint32_t *read_codes;
  const uint64_t *read_word_off;
  const int32_t *read_len;
  uint64_t read_words;
  /* aligned ends, DEVICE pointers, caller-owned, n_reads entries each */
  const uint64_t *mate_pos;     /* leftmost forward-strand base */
  const int32_t *mate_len;
  const uint8_t *mate_strand;   /* 0 forward, 1 reverse */
  /* packed sequence, DEVICE pointer, caller-owned, (ref_len + 15) / 16 words */
  const uint32_t *ref_codes;
  uint64_t ref_len;             /* in bases, at most 2^40 */
  int64_t n_reads;
  int32_t max_n;                /* bound on the unaligned ends' lengths */
  int32_t min_frag, max_frag;   /* 1 <= min_frag <= max_frag, and
                                   max_frag - min_frag + max_n <= SOAP_DP_MAX_WINDOW */
  int32_t orientation;          /* SOAP_DP_ORIENT_* */
} soap_dp_mate_batch;

/* Outputs, DEVICE pointers, caller-owned, n_reads entries each (cigar:
 * n_reads * cigar_stride words, cigar_stride >= 2 * max_n - 1, or NULL with
 * stride 0 under SOAP_DP_SCORE_ONLY). */
typedef struct {
  int32_t *score;
  int32_t *ref_begin;
  int32_t *ref_end;
  uint32_t *cigar;
  int32_t cigar_stride;
  int32_t *cigar_len;
  uint8_t *status;
  uint64_t *window_off;         /* region start in ref_codes */
  int32_t *window_len;
  uint8_t *strand;              /* 1: the read's reverse complement was aligned */
} soap_dp_mate_result;

/* Enqueue on `stream`.  flags as for soap_dp_align_batch (SOAP_DP_PLAIN or
 * SOAP_DP_BATCHED, optionally | SOAP_DP_SCORE_ONLY).  Same error codes; the
 * context's workspace grows with the reads. */
int soap_dp_mate_rescue(soap_dp_ctx *ctx, const soap_dp_mate_batch *in, const soap_dp_scoring *sc,
                        const soap_dp_mate_result *out, void *stream, uint32_t flags);

/* ------------------------------------------------------------------------
 * Serving: continuous batching over a device-resident genome.
 *
 * A server owns `n_slots` slots, each with its own worker thread, stream,
 * library context and pinned host staging for up to `max_tasks` tasks and
 * `max_read_words` packed read words per batch.  Requests are queued on
 * submit.  A free slot's worker takes the requests that have arrived, first
 * in first out, and merges them into one batch while the batch stays within
 * the slot's limits and its device buffers (reads, task arrays, outputs and
 * CIGAR rows) fit the free part of the server's device memory budget
 * (`device_bytes`, shared by all batches in flight).  It uploads the batch,
 * runs the batched form on the slot's stream, copies the results back and
 * hands each request its slice; the batch's device memory is then free for
 * the next one.  Batches of different sizes therefore overlap on the device
 * as memory and slots free up, while new requests keep arriving.  Windows
 * are base offsets into the resident genome: no sequence is copied for them.
 * Results are written into the caller's host buffers, which must stay valid
 * until the request completes; a request completes when
 * soap_dp_server_wait returns for it.
 *
 * A task of a request gets the same outputs whatever else is served with
 * it, and the same as soap_dp_align_batch(SOAP_DP_BATCHED) gives for the
 * request on its own (with read_words = the request's read_words): a task
 * whose read lies outside the request's read words gets
 * SOAP_DP_TASK_INVALID_OFFSET.
 *
 * The slots' contexts reserve their workspace and stream set at creation
 * (after autotuning, when asked) and warm every kernel up there; serving
 * then allocates nothing, captures no graph and never synchronises the
 * whole device.
 * ------------------------------------------------------------------------ */
#define SOAP_DP_E2BIG (-5)   /* request larger than a slot or than the device budget */
#define SOAP_DP_ESTOPPED (-6) /* server is shutting down */

typedef struct soap_dp_server soap_dp_server;

typedef struct {
  int device_ordinal;
  int n_slots;                 /* batches in flight at once (worker threads, streams), 1..8 */
  int32_t max_tasks;           /* tasks per merged batch */
  int64_t max_read_words;      /* packed read words per merged batch */
  int32_t max_n, max_m;        /* bounds on every task of every request */
  soap_dp_scoring scoring;
  const uint32_t *genome;      /* DEVICE pointer, packed, caller-owned, resident */
  uint64_t genome_words;
  int autotune;                /* nonzero: autotune the slots' shapes at start */
  uint64_t device_bytes;       /* device memory for the batches in flight, shared by the
                                  slots; 0: room for n_slots batches at the slot limits.
                                  It must hold at least one batch of one largest request;
                                  the contexts' decision scratch is reserved apart from it */
  uint32_t align_flags;        /* OR-ed into every batch's SOAP_DP_BATCHED call: 0 or
                                  SOAP_DP_FULL_WINDOW (one pass per batch); other bits are
                                  SOAP_DP_EINVAL */
} soap_dp_server_config;

/* HOST results of one served request.  CIGARs are packed: task t's runs
 * start at the sum of cigar_len over the tasks before it.  If they need more
 * than cigar_capacity words the request fails with SOAP_DP_E2BIG (its other
 * outputs are still written); n_tasks * (2 * max_n - 1) words always
 * suffice. */
typedef struct {
  int32_t *score;
  int32_t *ref_begin;
  int32_t *ref_end;
  int32_t *cigar_len;
  uint8_t *status;
  uint32_t *cigar;
  int64_t cigar_capacity;
} soap_dp_host_result;

/* Where a served request's time went, on soap_dp_now_ns's clock. */
typedef struct {
  uint64_t arrival_ns;   /* when it was due (admitted no earlier) */
  uint64_t taken_ns;     /* a free slot's worker took it into a batch */
  uint64_t launched_ns;  /* its batch's uploads, kernels and copies back were enqueued */
  uint64_t device_ns;    /* the worker saw its batch's results arrive in host memory */
  uint64_t done_ns;      /* its results were all in its buffers */
} soap_dp_request_stamps;

typedef struct {
  /* HOST arrays describing the request's tasks */
  const uint32_t *read_codes;     /* packed reads, read t at word read_word_off[t] */
  const uint64_t *read_word_off;
  const int32_t *read_len;
  uint64_t read_words;            /* words in read_codes */
  const uint64_t *ref_base_off;   /* base offsets into the resident genome */
  const int32_t *ref_len;
  int32_t n_tasks;
  soap_dp_host_result out;
  uint64_t arrival_ns;            /* arrival time on the soap_dp_now_ns() clock: the
                                     request is admitted no earlier (0: on submission);
                                     requests are admitted in submission order */
  soap_dp_request_stamps *stamps; /* HOST, optional: filled when the request completes */
} soap_dp_request;

typedef struct {
  uint64_t submitted, completed, rejected, batches;
  uint64_t tasks, cells;
  double device_busy_s;   /* sum over batches of upload start .. results copied
                             (slots overlap, so this can exceed wall time) */
  double host_launch_s;   /* worker time merging and enqueueing batches */
  double host_retire_s;   /* worker time handing results to requests */
  uint64_t device_bytes;       /* the budget the batches in flight share */
  uint64_t device_bytes_peak;  /* most of it the batches in flight held at once */
} soap_dp_server_stats;

/* Monotonic clock used for arrival and completion times (nanoseconds). */
uint64_t soap_dp_now_ns(void);

int soap_dp_server_create(soap_dp_server **srv, const soap_dp_server_config *cfg);

/* Queue a request; returns a ticket.  SOAP_DP_E2BIG if it can never fit a
 * slot or the device budget.  The request's host arrays are copied before
 * this returns; the result arrays (and stamps) are written when it
 * completes. */
int soap_dp_server_submit(soap_dp_server *srv, const soap_dp_request *req, uint64_t *ticket);

/* 1 when the request has completed (results written), 0 while pending,
 * a negative code if it failed. */
int soap_dp_server_poll(soap_dp_server *srv, uint64_t ticket);

/* Block until the request has completed and release its ticket; its
 * completion time (when its results were all in the caller's buffers, on
 * soap_dp_now_ns's clock) goes to *done_ns when non-NULL.  Returns the
 * request's result code. */
int soap_dp_server_wait(soap_dp_server *srv, uint64_t ticket, uint64_t *done_ns);

/* Block until every submitted request has completed. */
int soap_dp_server_drain(soap_dp_server *srv);

int soap_dp_server_stats_get(soap_dp_server *srv, soap_dp_server_stats *out);

/* Stop accepting requests, finish the queued ones, release everything. */
int soap_dp_server_destroy(soap_dp_server *srv);

/* Human-readable text for an error code. */
const char *soap_dp_strerror(int code);

/* The HIP error code behind the last SOAP_DP_EHIP on this context. */
int soap_dp_last_hip_error(const soap_dp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* SOAP_DP_H */
