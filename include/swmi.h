/*
 * swmi -- Smith-Waterman protein database search on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  All sizes are in elements; every pointer is a host pointer unless its name
 * ends in `_dev`.  Every call returns 0 on success or a negative SW_E* code, never
 * throws across the ABI and never aborts the process.  On error no output buffer is
 * written.
 *
 * What is computed (Rucci et al., "First Experiences Optimizing Smith-Waterman on
 * Intel's Knights Landing Processor", Section 2, Eqs. 1-3): for a query S1 of length
 * m and a database sequence S2 of length n,
 *
 *   H[i][j] = max{0, H[i-1][j-1] + SM(S1[i], S2[j]), E[i][j], F[i][j]}
 *   E[i][j] = max{H[i][j-1] - Goe, E[i][j-1] - Ge}
 *   F[i][j] = max{H[i-1][j] - Goe, F[i-1][j] - Ge}
 *
 * with H = E = F = 0 on row 0 and column 0, Goe = gap_open + gap_extend and
 * Ge = gap_extend.  The score of the pair is the maximum entry of H (0 if either
 * sequence is empty).  A search scores one query against every database sequence
 * (Section 4, "SW stage"); scores are exact integers.
 */
#ifndef SWMI_H
#define SWMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ error codes */
#define SW_OK        0
#define SW_EINVAL   (-1) /* bad argument: NULL pointer, bad offsets, residue >= alphabet,
                            negative length or penalty, gap_open + gap_extend > 16383,
                            |matrix entry| > 127, alphabet outside [1, 31],
                            query_len > 2^24 */
#define SW_ENOMEM   (-2) /* device memory could not be allocated (admission refused) */
#define SW_EDEVICE  (-3) /* a HIP runtime call failed, or no usable gfx950 device */
#define SW_ENODB    (-4) /* the database handle is NULL or was not loaded */

#define SW_MAX_ALPHABET   31
#define SW_MAX_QUERY_LEN  (1 << 24)
#define SW_MAX_GOE        16383
#define SW_MAX_ABS_SCORE  127

/* Opaque database handle.  Owns device (HBM) memory until sw_db_free. */
typedef struct sw_db sw_db;

/*
 * sw_db_load -- pre-processing stage (Section 4, step 1; the grouping of Section 4
 * before "Multiple Parallelism Levels"): sort the sequences by length, split off the
 * very long ones, group the rest 64 to a group, pad each group to its longest member
 * with a reserved padding code and copy the packed, interleaved result to HBM, where
 * it stays resident for any number of searches.
 *
 *   residues  host, uint8[offsets[n_seqs]]: concatenated residue codes, each in
 *             [0, alphabet).
 *   offsets   host, int64[n_seqs + 1]: offsets[0] == 0, non-decreasing; sequence k
 *             is residues[offsets[k] .. offsets[k+1]).  Empty sequences are allowed
 *             (they score 0).
 *   n_seqs    number of sequences, >= 0 (0 gives an empty database).
 *   alphabet  number of residue codes, 1..31 (code 31 is reserved for padding).
 *   out       receives the new handle; untouched on error.
 *
 * The caller keeps ownership of residues and offsets; nothing is retained after the
 * call returns.  Errors: SW_EINVAL, SW_ENOMEM, SW_EDEVICE.
 */
int sw_db_load(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs,
               int32_t alphabet, sw_db **out);

/* Number of sequences in the database (or a negative SW_E* code). */
int64_t sw_db_size(const sw_db *db);

/* Releases the handle and its device memory.  NULL is a no-op. */
void sw_db_free(sw_db *db);

/*
 * sw_search -- SW stage of Section 4: score one query against every database
 * sequence and return the scores in the caller's original database order.
 *
 *   query       host, uint8[query_len], codes in [0, alphabet).  query_len 0 gives
 *               all-zero scores.  query_len <= 2^24.
 *   matrix      host, int32[alphabet * alphabet], row-major, SM(S1[i], S2[j]) =
 *               matrix[S1[i] * alphabet + S2[j]] (row = query residue); |entry| <= 127.
 *   gap_open, gap_extend   >= 0 with gap_open + gap_extend <= 16383 (Section 2:
 *               Goe = gap_open + gap_extend, Ge = gap_extend).
 *   scores_out  host, int32[sw_db_size(db)], caller-allocated, fully written on
 *               success.
 *
 * Blocks until the scores are on the host.  Safe to call concurrently from several
 * host threads on one handle (the database is read-only; each call takes its own
 * device workspace).  Errors: SW_ENODB, SW_EINVAL, SW_ENOMEM, SW_EDEVICE.
 */
int sw_search(const sw_db *db, const uint8_t *query, int32_t query_len,
              const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
              int32_t *scores_out);

/*
 * sw_search_async -- the same search, enqueued on a caller's HIP stream, with the
 * scores written to device memory.
 *
 *   query, matrix, gap_open, gap_extend   as for sw_search (host memory, validated
 *               and copied before the call returns, so the caller may reuse them).
 *   scores_dev  device, int32[sw_db_size(db)], written in the caller's database order
 *               when the stream reaches the end of the enqueued work.
 *   hip_stream  a hipStream_t (NULL = the default stream).
 *
 * Returns once the work is enqueued.  The device workspace of the call is recycled
 * only after the stream has passed it.  Errors as for sw_search.
 */
int sw_search_async(const sw_db *db, const uint8_t *query, int32_t query_len,
                    const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                    int32_t *scores_dev, void *hip_stream);

/*
 * sw_search_batch -- many queries against the database in one launch of the search
 * kernels (work items are (query, sequence group) pairs, longest first).
 *
 *   queries        host, uint8: the queries concatenated.
 *   query_offsets  host, int64[n_queries + 1], offsets[0] == 0, non-decreasing.
 *   n_queries      >= 0.
 *   matrix, gap_open, gap_extend   as for sw_search; shared by all queries.
 *   scores_out     host, int32[n_queries * sw_db_size(db)]; row q holds query q's
 *                  scores in the caller's database order.
 *
 * Results are identical to n_queries separate sw_search calls.  Errors as for
 * sw_search.
 */
int sw_search_batch(const sw_db *db, const uint8_t *queries, const int64_t *query_offsets,
                    int64_t n_queries, const int32_t *matrix, int32_t gap_open,
                    int32_t gap_extend, int32_t *scores_out);

/* Static message for an error code. */
const char *sw_strerror(int code);

/*
 * Kernel timing of the inter-task DP kernel (the dominant kernel), measured with HIP
 * events recorded on the stream that launches it.  sw_timing_enable(db, 1) turns the
 * events on and clears the totals; sw_timing_read reports the number of launches and
 * the summed device time in milliseconds since then.  Not thread-safe with concurrent
 * searches on the same handle.
 */
int sw_timing_enable(sw_db *db, int32_t enable);
int sw_timing_read(const sw_db *db, int64_t *launches, double *total_ms);

/*
 * Tuning and debug knobs (process-wide; read at the next search):
 *   SW_KNOB_INTRA_MIN_LEN  database sequences longer than this go to the intra-task
 *                          kernel (read at sw_db_load; default 8192);
 *   SW_KNOB_RECOMPUTE_ALL  non-zero: recompute every score in int32 (debug; the
 *                          result must not change);
 *   SW_KNOB_STRIP_ROWS     rows per inter-task strip (0 = automatic choice);
 *   SW_KNOB_GRID_WAVES     persistent waves per compute unit (0 = automatic);
 *   SW_KNOB_MEM_CAP_MB     refuse workspaces beyond this many MiB (0 = no cap);
 *   SW_KNOB_ROUTE_LEN      database groups whose longest sequence exceeds this go to the
 *                          intra-task kernel for the search (0 = automatic: about twice
 *                          the residues per inter-task lane).
 */
#define SW_KNOB_INTRA_MIN_LEN  1
#define SW_KNOB_RECOMPUTE_ALL  2
#define SW_KNOB_STRIP_ROWS     3
#define SW_KNOB_GRID_WAVES     4
#define SW_KNOB_MEM_CAP_MB     5
#define SW_KNOB_ROUTE_LEN      6
int sw_set_knob(int32_t knob, int64_t value);
int64_t sw_get_knob(int32_t knob);

#ifdef __cplusplus
}
#endif

#endif /* SWMI_H */
