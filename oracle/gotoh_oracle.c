/*
 * CPU oracle: plain three-table affine-gap dynamic programming.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code with
 * the GPU path.
 *
 * It computes exactly the paper's recurrences (Methods section 3,
 * "GPU-accelerated dynamic programming"), in the loop order of the
 * straightforward three-table algorithm given there: region position i
 * outer (1..m), read position j inner (1..n), with
 *
 *   I(i,j) = max( M(i,j-1) + S_GO,  I(i,j-1) + S_GE )     read base j vs a space
 *   D(i,j) = max( M(i-1,j) + S_GO,  D(i-1,j) + S_GE )     region base i vs a space
 *   M(i,j) = max( M(i-1,j-1) + delta(T[i], R[j]),  I(i,j),  D(i,j) )
 *
 * and the base cases I(i,0) = -inf, D(0,j) = -inf, M(i,0) = 0 (i = 0..m),
 * M(0,j) = S_GO + (j-1) S_GE.  The result is max_{1<=i<=m} M(i,n).
 *
 * Readings taken where the paper is silent or garbled:
 *  - delta is applied to (T[i], R[j]); the printed argument order swaps the
 *    indices, but i ranges over the region and j over the read.
 *  - the gap scores are signed and added ("penalty scores" inside a max).
 *  - no zero floor: the whole read is aligned, the region is free at both
 *    ends; scores may be negative.
 *  - end position: the smallest i reaching the maximum.
 *  - tie-breaks, used both to record decisions and for the traceback: at an
 *    M cell diagonal before D before I; inside a gap, open before extend.
 *    Ties are resolved with >= so that the earlier option wins.
 *  - traceback: from (ref_end, n) in state M.  State M at j = 0 stops with
 *    ref_begin = i; at i = 0 (j > 0) it emits j insertions (base case
 *    M(0,j)) and stops with ref_begin = 0.  Otherwise it follows the
 *    recorded source.  State D emits D, moves to M if the gap was opened,
 *    then i -= 1.  State I emits I, moves to M if opened, then j -= 1.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define SRC_DIAG 0
#define SRC_D 1
#define SRC_I 2

static int32_t max2(int32_t a, int32_t b) { return a >= b ? a : b; }

typedef struct {
  int32_t *M, *I, *D;
  uint8_t *dec;
  size_t cap; /* cells */
} tables;

static int ensure(tables *t, size_t cells) {
  if (cells <= t->cap) return 0;
  free(t->M); free(t->I); free(t->D); free(t->dec);
  t->M = malloc(cells * sizeof(int32_t));
  t->I = malloc(cells * sizeof(int32_t));
  t->D = malloc(cells * sizeof(int32_t));
  t->dec = malloc(cells);
  t->cap = (t->M && t->I && t->D && t->dec) ? cells : 0;
  return t->cap ? 0 : -1;
}

static void release(tables *t) {
  free(t->M); free(t->I); free(t->D); free(t->dec);
  memset(t, 0, sizeof(*t));
}

/* Fill all three tables and the decisions.  W = n + 1 is the row width. */
static void fill(const uint8_t *R, int32_t n, const uint8_t *T, int32_t m,
                 const oracle_scoring *sc, int32_t *M, int32_t *I, int32_t *D, uint8_t *dec) {
  const int32_t W = n + 1;
  /* base cases */
  for (int32_t i = 0; i <= m; ++i) {
    M[i * W + 0] = 0;
    I[i * W + 0] = ORACLE_NEG_INF;
    D[i * W + 0] = ORACLE_NEG_INF; /* never read by the recurrences */
    dec[i * W + 0] = 0;
  }
  for (int32_t j = 1; j <= n; ++j) {
    M[0 * W + j] = sc->gap_open + (j - 1) * sc->gap_extend;
    D[0 * W + j] = ORACLE_NEG_INF;
    I[0 * W + j] = ORACLE_NEG_INF; /* never read by the recurrences */
    dec[0 * W + j] = 0;
  }
  for (int32_t i = 1; i <= m; ++i) {
    for (int32_t j = 1; j <= n; ++j) {
      const int32_t i_open = M[i * W + (j - 1)] + sc->gap_open;
      const int32_t i_ext = I[i * W + (j - 1)] + sc->gap_extend;
      const int32_t vi = max2(i_open, i_ext);
      const int32_t d_open = M[(i - 1) * W + j] + sc->gap_open;
      const int32_t d_ext = D[(i - 1) * W + j] + sc->gap_extend;
      const int32_t vd = max2(d_open, d_ext);
      const int32_t delta = (T[i - 1] == R[j - 1]) ? sc->match : sc->mismatch;
      const int32_t diag = M[(i - 1) * W + (j - 1)] + delta;
      int32_t vm;
      uint8_t src;
      if (diag >= vd && diag >= vi) { vm = diag; src = SRC_DIAG; }
      else if (vd >= vi) { vm = vd; src = SRC_D; }
      else { vm = vi; src = SRC_I; }
      I[i * W + j] = vi;
      D[i * W + j] = vd;
      M[i * W + j] = vm;
      dec[i * W + j] = (uint8_t)(src | ((i_open >= i_ext) ? 0 : 1) << 2 | ((d_open >= d_ext) ? 0 : 1) << 3);
    }
  }
}

int oracle_fill_tables(const uint8_t *R, int32_t n, const uint8_t *T, int32_t m,
                       const oracle_scoring *sc, int32_t *M, int32_t *I, int32_t *D,
                       uint8_t *dec) {
  if (n < 1 || m < 1 || !R || !T || !sc) return -1;
  tables t = {0};
  const size_t cells = (size_t)(n + 1) * (size_t)(m + 1);
  if (ensure(&t, cells)) return -1;
  fill(R, n, T, m, sc, t.M, t.I, t.D, t.dec);
  if (M) memcpy(M, t.M, cells * sizeof(int32_t));
  if (I) memcpy(I, t.I, cells * sizeof(int32_t));
  if (D) memcpy(D, t.D, cells * sizeof(int32_t));
  if (dec) memcpy(dec, t.dec, cells);
  release(&t);
  return 0;
}

/* Append one operation to a reversed run-length list. */
typedef struct {
  uint32_t *runs; /* reversed order while tracing */
  int32_t count, cap;
  int overflow;
} cigar_acc;

static void push(cigar_acc *c, int op, int32_t len) {
  if (len <= 0) return;
  if (c->count > 0 && (int)(c->runs[c->count - 1] & 0xF) == op) {
    c->runs[c->count - 1] += (uint32_t)len << 4;
    return;
  }
  if (c->count >= c->cap) { c->overflow = 1; return; }
  c->runs[c->count++] = (uint32_t)len << 4 | (uint32_t)op;
}

static void align_one(const uint8_t *R, int32_t n, const uint8_t *T, int32_t m,
                      const oracle_scoring *sc, tables *tb,
                      int32_t *score, int32_t *ref_begin, int32_t *ref_end,
                      uint32_t *cigar, int32_t cigar_stride, int32_t *cigar_len, uint8_t *status) {
  *score = 0; *ref_begin = 0; *ref_end = 0; *cigar_len = 0; *status = ORACLE_OK;
  if (n < 1 || m < 1) { *status = ORACLE_INVALID_LEN; return; }
  const size_t cells = (size_t)(n + 1) * (size_t)(m + 1);
  if (ensure(tb, cells)) { *status = ORACLE_INVALID_LEN; return; }
  const int32_t W = n + 1;
  fill(R, n, T, m, sc, tb->M, tb->I, tb->D, tb->dec);

  /* result: max over i of M(i, n), smallest i on ties */
  int32_t best = tb->M[1 * W + n], end = 1;
  for (int32_t i = 2; i <= m; ++i)
    if (tb->M[i * W + n] > best) { best = tb->M[i * W + n]; end = i; }

  /* traceback */
  cigar_acc acc = { cigar, 0, cigar_stride, 0 };
  int32_t i = end, j = n;
  int state = SRC_DIAG; /* 0 = M, 1 = D, 2 = I */
  int32_t begin = 0;
  for (;;) {
    if (state == SRC_DIAG) {
      if (j == 0) { begin = i; break; }
      if (i == 0) { push(&acc, ORACLE_OP_I, j); begin = 0; break; }
      const int src = tb->dec[i * W + j] & 3;
      if (src == SRC_DIAG) { push(&acc, ORACLE_OP_M, 1); --i; --j; }
      else state = src;
    } else if (state == SRC_D) {
      push(&acc, ORACLE_OP_D, 1);
      if (!((tb->dec[i * W + j] >> 3) & 1)) state = SRC_DIAG;
      --i;
    } else {
      push(&acc, ORACLE_OP_I, 1);
      if (!((tb->dec[i * W + j] >> 2) & 1)) state = SRC_DIAG;
      --j;
    }
  }
  if (acc.overflow) { *status = ORACLE_INVALID_LEN; *cigar_len = 0; return; }
  /* reverse into forward order */
  for (int32_t a = 0, b = acc.count - 1; a < b; ++a, --b) {
    uint32_t t = cigar[a]; cigar[a] = cigar[b]; cigar[b] = t;
  }
  *score = best;
  *ref_end = end;
  *ref_begin = begin;
  *cigar_len = acc.count;
}

typedef struct {
  const uint8_t *read_codes; const int64_t *read_off; const int32_t *read_len;
  const uint8_t *ref_codes; const int64_t *ref_off; const int32_t *ref_len;
  int64_t n_tasks; const oracle_scoring *sc;
  int32_t *score, *ref_begin, *ref_end; uint32_t *cigar; int32_t cigar_stride;
  int32_t *cigar_len; uint8_t *status;
  _Atomic int64_t next;
} job;

#define CHUNK 64

static void *worker(void *arg) {
  job *jb = (job *)arg;
  tables tb = {0};
  for (;;) {
    const int64_t s = atomic_fetch_add(&jb->next, CHUNK);
    if (s >= jb->n_tasks) break;
    const int64_t e = s + CHUNK < jb->n_tasks ? s + CHUNK : jb->n_tasks;
    for (int64_t t = s; t < e; ++t) {
      align_one(jb->read_codes + jb->read_off[t], jb->read_len[t],
                jb->ref_codes + jb->ref_off[t], jb->ref_len[t], jb->sc, &tb,
                &jb->score[t], &jb->ref_begin[t], &jb->ref_end[t],
                jb->cigar + t * (int64_t)jb->cigar_stride, jb->cigar_stride,
                &jb->cigar_len[t], &jb->status[t]);
    }
  }
  release(&tb);
  return NULL;
}

int oracle_default_threads(void) {
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  return c > 0 ? (int)c : 1;
}

int oracle_align_batch(const uint8_t *read_codes, const int64_t *read_off, const int32_t *read_len,
                       const uint8_t *ref_codes, const int64_t *ref_off, const int32_t *ref_len,
                       int64_t n_tasks, const oracle_scoring *sc,
                       int32_t *score, int32_t *ref_begin, int32_t *ref_end,
                       uint32_t *cigar, int32_t cigar_stride, int32_t *cigar_len,
                       uint8_t *status, int n_threads) {
  if (n_tasks < 0 || !sc || cigar_stride < 1) return -1;
  if (n_tasks == 0) return 0;
  if (!read_off || !read_len || !ref_off || !ref_len || !score || !ref_begin || !ref_end ||
      !cigar || !cigar_len || !status)
    return -1;
  if (n_threads <= 0) n_threads = oracle_default_threads();
  if (n_threads > n_tasks / CHUNK + 1) n_threads = (int)(n_tasks / CHUNK + 1);
  job jb = { read_codes, read_off, read_len, ref_codes, ref_off, ref_len, n_tasks, sc,
             score, ref_begin, ref_end, cigar, cigar_stride, cigar_len, status, 0 };
  if (n_threads == 1) { worker(&jb); return 0; }
  pthread_t *th = malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return -1;
  int started = 0;
  for (int k = 0; k < n_threads; ++k)
    if (pthread_create(&th[k], NULL, worker, &jb) == 0) ++started;
  if (started == 0) worker(&jb);
  for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
  free(th);
  return 0;
}
