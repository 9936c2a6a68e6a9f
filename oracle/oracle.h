/*
 * CPU oracle for read-vs-window affine-gap alignment.  TEST INFRASTRUCTURE
 * ONLY: the tests, the smoke check and the benchmark's CPU baseline use it;
 * the GPU library never links, loads or calls it, and it shares no code,
 * header or constant with that library.
 *
 * The problem (paper, Methods section 3 "GPU-accelerated dynamic
 * programming"): given a candidate region T of length m and a read R of
 * length n, find the sub-region T' of T whose alignment score with the whole
 * of R is maximal.  Scores: delta(x,y) = S_MA if x == y else S_MI; a run of
 * k read bases against spaces, or of k region bases against spaces, scores
 * S_GO + (k-1) * S_GE.  All four scores are signed and added.
 *
 * Bases are codes 0..3, one per byte.
 */
#ifndef SOAPDP_ORACLE_H
#define SOAPDP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t match;       /* S_MA */
  int32_t mismatch;    /* S_MI */
  int32_t gap_open;    /* S_GO: score of the first base of a gap */
  int32_t gap_extend;  /* S_GE: score of each further base of the gap */
} oracle_scoring;

/* Value standing for minus infinity in the tables. */
#define ORACLE_NEG_INF (-(1 << 30))

/* Per-task status. */
#define ORACLE_OK 0
#define ORACLE_INVALID_LEN 1

/* CIGAR operation codes (BAM numbering). */
#define ORACLE_OP_M 0
#define ORACLE_OP_I 1
#define ORACLE_OP_D 2

/*
 * Align every task t: read read_codes[read_off[t] .. +read_len[t]) against
 * window ref_codes[ref_off[t] .. +ref_len[t]).  Outputs per task:
 *   score[t]      max over 1 <= i <= m of M(i, n)
 *   ref_end[t]    the smallest such i (0-based exclusive end of T')
 *   ref_begin[t]  0-based start of T'
 *   cigar[t*cigar_stride ..] BAM-encoded (len << 4 | op) runs, cigar_len[t] of them
 *   status[t]     ORACLE_OK, or ORACLE_INVALID_LEN when n < 1 or m < 1
 *                 (outputs zero), or when the CIGAR would not fit the stride.
 * Tasks are spread over n_threads POSIX threads (<= 0: one per online CPU).
 * Returns 0, or -1 on a bad argument.
 */
int oracle_align_batch(const uint8_t *read_codes, const int64_t *read_off, const int32_t *read_len,
                       const uint8_t *ref_codes, const int64_t *ref_off, const int32_t *ref_len,
                       int64_t n_tasks, const oracle_scoring *sc,
                       int32_t *score, int32_t *ref_begin, int32_t *ref_end,
                       uint32_t *cigar, int32_t cigar_stride, int32_t *cigar_len,
                       uint8_t *status, int n_threads);

/*
 * The three score tables of one task, each (m+1) x (n+1) row-major with
 * row i = region position, column j = read position, ORACLE_NEG_INF where a
 * base case is minus infinity, and the traceback decisions of every cell:
 * dec[i*(n+1)+j] = msrc | iext << 2 | dext << 3 with msrc 0 = diagonal,
 * 1 = from D, 2 = from I; iext/dext 1 = the gap was extended, 0 = opened.
 * Any output pointer may be NULL.  Returns 0, or -1 if n < 1 or m < 1.
 */
int oracle_fill_tables(const uint8_t *R, int32_t n, const uint8_t *T, int32_t m,
                       const oracle_scoring *sc, int32_t *M, int32_t *I, int32_t *D,
                       uint8_t *dec);

/* Number of online CPUs the batch call would use by default. */
int oracle_default_threads(void);

#ifdef __cplusplus
}
#endif
#endif
