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
 * (Section 4, the alignment stage); scores are exact integers.
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
 * sw_db_load -- pre-processing stage (Section 4, first stage, and its grouping of
 * sequences by lane count): sort the sequences by length, split off the
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
 * device workspace).  Errors: SW_ENODB, SW_EINVAL, SW_ENOMEM, SW_EDEVICE (also when a
 * bounded wait between the workgroups of a split pair gave up; see
 * SW_KNOB_SPIN_LIMIT); scores_out is then left untouched.
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
 * only after the stream has passed it.  Errors as for sw_search, except that a bounded
 * wait that gives up on the device cannot be reported by an asynchronous call (its
 * default limit, 2^24 polls, is seconds beyond any legitimate wait).
 */
int sw_search_async(const sw_db *db, const uint8_t *query, int32_t query_len,
                    const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                    int32_t *scores_dev, void *hip_stream);

/*
 * sw_search_batch -- many queries against the database in one launch of the search
 * kernels.  The queries are paired longest first and each pair shares the lanes of the
 * inter-task kernel, one query per int16 half (SW_KNOB_QUERY_PAIRS; 0 = one query per
 * lane); work items are (query pair, sequence group), longest first.
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

/*
 * Plans: a search captured once into a HIP graph and replayed.
 *
 * sw_plan_create runs the (batched) search once, sizing a workspace that the plan owns,
 * then captures the whole launch sequence of the search (query profiles, inter-task
 * kernel, intra-task kernel on a second stream, saturation recompute) into a hipGraph.
 * Arguments are those of sw_search_batch, except that the scores go to device memory:
 *   scores_dev  device, int32[n_queries * sw_db_size(db)], written by the eager run and
 *               by every replay (row q = query q, caller's database order).
 * The queries, matrix and penalties are copied; the caller may reuse its buffers.  The
 * plan keeps using scores_dev and the database until sw_plan_free.  Knob values in force
 * at creation (strip height, waves per CU, routing) are baked into the plan.
 * sw_plan_launch enqueues one replay on hip_stream (NULL = default stream); replays on
 * different streams must not overlap (they share the plan's workspace).
 * Errors: as for sw_search_batch; SW_EINVAL for a NULL plan.
 */
typedef struct sw_plan sw_plan;
int sw_plan_create(const sw_db *db, const uint8_t *queries, const int64_t *query_offsets,
                   int64_t n_queries, const int32_t *matrix, int32_t gap_open,
                   int32_t gap_extend, int32_t *scores_dev, sw_plan **out);
int sw_plan_launch(sw_plan *plan, void *hip_stream);
void sw_plan_free(sw_plan *plan);

/*
 * Serving: continuous batching over a resident database (not in the paper, whose queries
 * run one after another).
 *
 * sw_server_create starts a worker thread that serves queries submitted with
 * sw_server_submit, in one of two modes chosen from the database:
 *
 *   Session mode, for a database whose groups of 64 sequences fill the device's
 *   persistent waves at least four times over and that holds no sequence above the
 *   intra-task threshold (SW_KNOB_INTRA_MIN_LEN), when the session's device scratch fits
 *   the free device memory and `mem_budget_bytes` (if > 0): one persistent kernel launch
 *   serves every query admitted while it runs.  Queued queries become records (one
 *   query, or two of similar length sharing the lanes of the two-query strip loop when
 *   `max_batch` >= 2) that are appended to the running launch's work list, so a query
 *   that arrives while others are on the device joins the same launch right behind them.
 *   A record is published when the device is about to run out of published work, with
 *   at most 4 x `slots` records in flight; the budget also bounds the host rows that
 *   receive the scores.  The launch ends once the server is idle; a query longer than
 *   16,384 residues, or one with a score at the int16 ceiling (Section 4.2), is
 *   searched (again) by the standard path, exactly, after the launch has drained.
 *
 *   Batch mode, otherwise: `slots` (1..16) stream slots each own a device workspace;
 *   whenever a slot is free, every queued query it can admit (at most `max_batch`,
 *   1..4096, and only while the device bytes of the batches in flight fit the budget and
 *   the free device memory) is launched as one batched search, so requests that arrive
 *   while others are on the GPU run next to them.  A batch stops growing once its
 *   inter-task work items fill every wave slot of the device four times over, and no
 *   further batch is launched while the batches in flight do.
 *
 * A query that alone exceeds the budget completes with SW_ENOMEM.  All searches use
 * `matrix`, `gap_open` and `gap_extend` (validated as for sw_search).  The database must
 * outlive the server.  While a session launch runs, other searches on the same device
 * wait for free compute units, i.e. until the server is idle.
 *
 * sw_server_submit copies the query (validated as for sw_search) and returns a ticket;
 * `scores_out` (host, int32[sw_db_size(db)]) must stay valid until sw_server_wait for
 * that ticket returns, and is fully written when the request completes.
 * sw_server_wait blocks until the request completes and returns its status (SW_OK or a
 * negative code, SW_EDEVICE when a wait on the device timed out); latency_ms (submission
 * to completion) and queue_ms (submission to launch or publication) are filled if
 * non-NULL.  Each ticket can be waited on once.
 * sw_server_stats reports the number of kernel launches (batches, or session launches),
 * the largest number of batches or records in flight at once and the number of refused
 * requests.  sw_server_free drains the queue, waits for the work in flight and releases
 * the server.  Scores are identical to those of sw_search for the same query.
 */
typedef struct sw_server sw_server;
int sw_server_create(sw_db *db, const int32_t *matrix, int32_t gap_open, int32_t gap_extend,
                     int32_t slots, int32_t max_batch, int64_t mem_budget_bytes,
                     sw_server **out);
int sw_server_submit(sw_server *server, const uint8_t *query, int32_t query_len,
                     int32_t *scores_out, uint64_t *ticket);
int sw_server_wait(sw_server *server, uint64_t ticket, double *latency_ms, double *queue_ms);
int sw_server_stats(sw_server *server, int64_t *launches, int64_t *max_in_flight,
                    int64_t *refused);
void sw_server_free(sw_server *server);

/*
 * sw_server_counters -- the server's counters, written to values[0 .. min(n, 9)):
 *   SW_SC_LAUNCHES      kernel launches (batch mode: batched searches; session mode:
 *                       session launches, each serving every query admitted while it ran)
 *   SW_SC_MAX_IN_FLIGHT largest number of batches (batch mode) or records (session mode)
 *                       on the device at once
 *   SW_SC_REFUSED       requests refused with SW_ENOMEM
 *   SW_SC_SESSION_MODE  1 if the server runs sessions, 0 if batches
 *   SW_SC_RECORDS       records published (session mode)
 *   SW_SC_PAIRED        of those, records holding two queries
 *   SW_SC_EXACT_RUNS    queries served by the standard search path (a score at the int16
 *                       ceiling, or a query longer than a session takes)
 *   SW_SC_WAVES         persistent waves of a session launch (0 in batch mode)
 *   SW_SC_COPY_US       host microseconds spent copying session scores to the callers
 * Errors: SW_EINVAL (NULL server or values, n < 0).
 */
#define SW_SC_LAUNCHES       0
#define SW_SC_MAX_IN_FLIGHT  1
#define SW_SC_REFUSED        2
#define SW_SC_SESSION_MODE   3
#define SW_SC_RECORDS        4
#define SW_SC_PAIRED         5
#define SW_SC_EXACT_RUNS     6
#define SW_SC_WAVES          7
#define SW_SC_COPY_US        8
#define SW_SERVER_NCOUNTERS  9
int sw_server_counters(sw_server *server, int64_t *values, int32_t n);

/*
 * sw_topk -- sorting stage (Section 4, step 3: scores sorted in descending order),
 * restricted to the k best hits: selects, on the device, the min(k, n_seqs) highest
 * scores of a search and returns them sorted by score descending, ties by database index
 * ascending.
 *
 *   scores_dev  device, int32[sw_db_size(db)]: scores in the caller's order (for example
 *               the output of sw_search_async; the call orders itself after earlier work
 *               on hip_stream).
 *   k           1..4096.
 *   hit_index, hit_score   host, int32[k]: database index and score of each hit.
 *   n_hits      host: number of hits written (min(k, n_seqs)).
 *   hip_stream  a hipStream_t (NULL = default stream); the call blocks until done.
 *
 * Calls on one database handle are serialised.  Errors: SW_ENODB, SW_EINVAL (k out of
 * range or NULL output), SW_ENOMEM, SW_EDEVICE.
 */
int sw_topk(const sw_db *db, const int32_t *scores_dev, int32_t k, int32_t *hit_index,
            int32_t *hit_score, int32_t *n_hits, void *hip_stream);

/*
 * sw_topk_noalloc -- sw_topk for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, results and errors, with every scratch buffer of the selection in a fixed
 * device array of the library (65 KiB per device, held until the process ends) instead
 * of memory allocated on first use.  k above 4096 (the array's limit) is rejected with
 * SW_EINVAL.  Calls on one device share that device's array: they are serialised inside
 * the library, and work that overlaps on the device from outside it (another process's
 * copy of the library excepted) would race; the selection state is cleared at the start
 * of every call.
 */
int sw_topk_noalloc(const sw_db *db, const int32_t *scores_dev, int32_t k, int32_t *hit_index,
                    int32_t *hit_score, int32_t *n_hits, void *hip_stream);

/* Static message for an error code. */
const char *sw_strerror(int code);

/*
 * Kernel timing of the inter-task DP kernel (the dominant kernel), measured with HIP
 * events recorded on the stream that launches it.  sw_timing_enable(db, 1) turns the
 * events on, clears the totals and creates the events of the next 128 timed launches
 * (so that no search in a timed region creates one); sw_timing_read reports the number
 * of launches and the summed device time in milliseconds since then.  Not thread-safe
 * with concurrent searches on the same handle.
 */
int sw_timing_enable(sw_db *db, int32_t enable);
int sw_timing_read(const sw_db *db, int64_t *launches, double *total_ms);

/*
 * The same totals for one kernel: SW_KERNEL_INTER16 (packed-int16 inter-task kernel),
 * SW_KERNEL_INTRA_LONG (int32 intra-task kernel over long and routed sequences, on the
 * second stream) or SW_KERNEL_RECOMPUTE (int32 recompute of saturated alignments).
 * Errors: SW_ENODB, SW_EINVAL (unknown kernel or NULL output), SW_EDEVICE.
 */
#define SW_KERNEL_INTER16     0
#define SW_KERNEL_INTRA_LONG  1
#define SW_KERNEL_RECOMPUTE   2
int sw_timing_read_kernel(const sw_db *db, int32_t kernel, int64_t *launches,
                          double *total_ms);

/*
 * sw_search_stats -- how the latest search enqueued on the handle was laid out, written
 * to values[0 .. min(n, 10)) (algorithmic cells count query rows x unpadded residues):
 *   SW_ST_CELLS_INTER16  cells of the packed-int16 inter-task launch
 *   SW_ST_CELLS_INTRA32  int32 cells of the main intra-task launch
 *   SW_ST_CELLS_INTRA16  cells of its two-pairs-per-wave (packed int16) items
 *   SW_ST_CELLS_CRIT     cells of the critical-pair launch (finer bands)
 *   SW_ST_INTRA_ROWS     query rows per lane of the main intra-task launch
 *   SW_ST_MAIN_WAVES     waves per workgroup of that launch
 *   SW_ST_ROUTED_GROUPS  database groups routed to the intra-task kernel
 *   SW_ST_STRIP_ROWS     strip rows of the inter-task launch
 *   SW_ST_QUERY_PAIRS    1 if the inter-task launch ran two queries per lane
 *   SW_ST_BIG_WAVES      waves of that launch with boundary slots for the widest groups,
 *                        when the others' slots are narrower (0: one slot width)
 * Errors: SW_ENODB, SW_EINVAL (NULL values or n < 0).
 */
#define SW_ST_CELLS_INTER16   0
#define SW_ST_CELLS_INTRA32   1
#define SW_ST_CELLS_INTRA16   2
#define SW_ST_CELLS_CRIT      3
#define SW_ST_INTRA_ROWS      4
#define SW_ST_MAIN_WAVES      5
#define SW_ST_ROUTED_GROUPS   6
#define SW_ST_STRIP_ROWS      7
#define SW_ST_QUERY_PAIRS     8
#define SW_ST_BIG_WAVES       9
#define SW_SEARCH_NSTATS      10
int sw_search_stats(const sw_db *db, int64_t *values, int32_t n);

/*
 * Tuning and debug knobs (process-wide; read at the next search):
 *   SW_KNOB_INTRA_MIN_LEN  database sequences longer than this go to the intra-task
 *                          kernel (read at sw_db_load; default 8192);
 *   SW_KNOB_RECOMPUTE_ALL  non-zero: recompute every score in int32 (debug; the
 *                          result must not change);
 *   SW_KNOB_STRIP_ROWS     rows per inter-task strip half: 8, 16, 24, 32 or 40, and 28
 *                          for searches that pair their queries (a height a search's
 *                          kernel lacks is chosen automatically); 0 = automatic;
 *   SW_KNOB_GRID_WAVES     persistent waves per compute unit (0 = automatic);
 *   SW_KNOB_MEM_CAP_MB     refuse workspaces beyond this many MiB (0 = no cap);
 *   SW_KNOB_ROUTE_LEN      database groups whose longest sequence exceeds this go to the
 *                          intra-task kernel for the search (0 = automatic: about twice
 *                          the residues per inter-task lane);
 *   SW_KNOB_WIDE_LEN       intra-task pairs at least this long (with two or more query
 *                          bands) are swept by a whole workgroup, shorter ones by one
 *                          wave (0 = automatic: 1152);
 *   SW_KNOB_MAX_SEGMENTS   most workgroups one intra-task pair may be split across
 *                          (0 = automatic, 1 = never split);
 *   SW_KNOB_INTRA_ROWS     query rows per lane of the intra-task kernel: 2, 4, 8 or 16
 *                          (bands of 128, 256, 512 or 1024 rows; 0 = chosen per search);
 *   SW_KNOB_INTRA_PAIRS    1 (default): when a search has many narrow intra-task pairs,
 *                          short ones run two per wave in packed int16 (saturated halves
 *                          recomputed in int32); 0: every intra-task pair runs alone in
 *                          int32; 2: every unsplit pair is paired (for tests);
 *   SW_KNOB_SPIN_LIMIT     polls after which a workgroup waiting for the previous
 *                          segment of a split intra-task pair gives up (1..2^24; 0 =
 *                          2^24).  A wait that gives up marks the search failed (a
 *                          blocking search returns SW_EDEVICE) and every kernel still
 *                          runs to its end; tiny values exist to test that path.
 *   SW_KNOB_QUERY_PAIRS    1 (default): a search of two or more queries runs the
 *                          inter-task DP two queries per lane (the queries paired
 *                          longest first, both in packed int16 at the same database
 *                          column); 0: one query per lane.  Scores are the same.
 *   SW_KNOB_MAIN_WAVES     waves per workgroup of the intra-task launch over long and
 *                          routed sequences: 8 (one workgroup per compute unit) or 4
 *                          (two per compute unit); 0 (default) = 4 when the search is
 *                          estimated throughput-bound, 8 when the longest pair's
 *                          pipeline bounds it.  Scores are the same.
 *   SW_KNOB_PRIO_COLS      inter-task work items (and serving-session items) of database
 *                          groups at least this many columns wide run at raised wave
 *                          priority on their SIMDs (0 = automatic: the width at which one
 *                          wave's item takes a quarter of the launch; a value above every
 *                          group's width turns it off).  Scores are the same.
 *   SW_KNOB_FLAG_CAP       entries of the list of saturated pairs recomputed in int32
 *                          (0 = 2^20); pairs beyond it are marked in the scores and
 *                          recomputed by a pass over all pairs.  Scores are the same.
 *   SW_KNOB_CRIT_ROWS      query rows per lane of the critical-pair launch: 4 or 8 (bands
 *                          of 256 or 512 rows); 0 (default) = 8.  Scores are the same.
 *   SW_KNOB_CRIT_SHARE     a split long pair whose band pipeline is estimated to take more
 *                          than this percentage of the whole intra-task search runs in
 *                          the critical-pair launch (1..100; 0 = automatic, 20).  Scores
 *                          are the same.
 *   SW_KNOB_INTRA_PRIO     1 (default): the intra-task kernel sweeps the critical pairs at
 *                          the highest wave priority, the main launch's wide items (a
 *                          whole workgroup per pair, the longest pairs) above its narrow
 *                          ones, and the narrow items within 70% of the longest narrow
 *                          one's cost above the others; 0: every wave at the default
 *                          priority.  Scores are the same.
 *   SW_KNOB_INTRA_CHAIN    1 (default): a pair the intra-task kernel sweeps with one wave
 *                          (at least 192 residues, two or more query bands) runs its
 *                          bands back to back as one stream instead of one band after
 *                          another, which saves each band's fill and drain; 0: one band
 *                          after another.  Scores are the same.
 */
#define SW_KNOB_INTRA_MIN_LEN  1
#define SW_KNOB_RECOMPUTE_ALL  2
#define SW_KNOB_STRIP_ROWS     3
#define SW_KNOB_GRID_WAVES     4
#define SW_KNOB_MEM_CAP_MB     5
#define SW_KNOB_ROUTE_LEN      6
#define SW_KNOB_WIDE_LEN       7
#define SW_KNOB_MAX_SEGMENTS   8
#define SW_KNOB_INTRA_ROWS     9
#define SW_KNOB_INTRA_PAIRS    10
#define SW_KNOB_SPIN_LIMIT     11
#define SW_KNOB_QUERY_PAIRS    12
#define SW_KNOB_MAIN_WAVES     13
#define SW_KNOB_PRIO_COLS      14
#define SW_KNOB_FLAG_CAP       15
#define SW_KNOB_CRIT_ROWS      16
#define SW_KNOB_CRIT_SHARE     17
#define SW_KNOB_INTRA_PRIO     18
#define SW_KNOB_INTRA_CHAIN    19
int sw_set_knob(int32_t knob, int64_t value);
int64_t sw_get_knob(int32_t knob);

#ifdef __cplusplus
}
#endif

#endif /* SWMI_H */
