/*
 * sw.h -- C ABI of the batched Smith-Waterman library (gfx950 / MI355X).
 *
 * The library aligns many candidate protein pairs of uneven length with local
 * (Smith-Waterman) alignment, the BLOSUM62 matrix and affine (Gotoh) gaps, in
 * exact int32 arithmetic, and returns for every pair the best score and the
 * start and end of the aligned region in both sequences.  This is the batch
 * alignment stage of the paper's pipeline (section "Protein similarity search
 * pipeline", stage (ii); section "Load balancing techniques": the full m x n
 * matrix is computed for every pair, so the cost of a pair is m*n).
 *
 * Conventions shared by every entry point:
 *  - Pointers named *_dev are device pointers (HBM of the current HIP device);
 *    every other pointer is host memory.  The caller owns all buffers; the
 *    library keeps no caller pointer after the work it enqueued completes.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *    asynchronously; results are valid once the caller has synchronised it.
 *  - Every function returns an int status (SW_OK or a negative SW_E* code);
 *    no C++ exception crosses the interface.
 *  - Residues are ASCII letters of the 24-symbol BLOSUM62 alphabet
 *    A R N D C Q E G H I L K M F P S T W Y V B Z X *  (upper case only).
 *  - A gap run of k residues costs gap_open + (k-1)*gap_extend, with
 *    1 <= gap_open <= 2^20 and 0 <= gap_extend <= gap_open (the paper's
 *    program-parameter table, section "Similarity search at scale", uses
 *    separate open and extension penalties; this model is Gotoh's).
 *  - Tie rule (the paper does not fix one): the end is the lexicographically
 *    smallest (query, reference) cell reaching the best score; the start is
 *    the largest (query, then reference) start among optimal alignments that
 *    end there.  Coordinates are 0-based and inclusive; score 0 reports all
 *    coordinates as -1.
 */
#ifndef SW_H
#define SW_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define SW_API __attribute__((visibility("default")))
#else
#define SW_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SW_OK 0
#define SW_EINVAL (-1)    /* null pointer, negative size, bad scoring, bad flags */
#define SW_ERANGE (-2)    /* pair index outside [0, n_seqs) or sequence longer than SW_MAX_SEQ_LEN */
#define SW_ECODE (-3)     /* a residue that is not a symbol of the alphabet */
#define SW_ENOMEM (-4)    /* device workspace or caller buffer too small */
#define SW_EDEVICE (-5)   /* a HIP runtime error (see sw_last_device_error) */
#define SW_ETIMEOUT (-6)  /* a wait ran out of time */
#define SW_EAGAIN (-7)    /* serving: the request is not admissible right now */
#define SW_ECANCELED (-8) /* serving: the server was shut down */

#define SW_MAX_SEQ_LEN 65535 /* keeps coordinates in 16 bits and scores far below 2^31 */

/* Result of one pair; 20 bytes, fields in this order. */
typedef struct {
    int32_t score;
    int32_t q_start, q_end;
    int32_t r_start, r_end;
} sw_result;

typedef struct {
    int32_t matrix_id;  /* 0 = BLOSUM62, the only matrix */
    int32_t gap_open;   /* cost of the first residue of a gap run */
    int32_t gap_extend; /* cost of every further residue of the run */
} sw_scoring;

/* flags of sw_batch_align */
#define SW_PERSISTENT 0u /* default: persistent launches over a device work queue, replayed as HIP graphs */
#define SW_PLAIN 1u      /* one launch per length bucket, static work split, no queue, no graph */
#define SW_VALIDATE 2u   /* synchronise before returning and report SW_ERANGE / SW_ECODE found on the device */
#define SW_NO_GRAPH 4u   /* persistent form without HIP-graph capture */
#define SW_TIMED 8u      /* bracket the alignment kernels of this call with HIP events (see sw_timing_read) */

/*
 * Bytes a packed buffer needs for n_residues residues (header, two residue
 * planes, guard and slack).  The paper's alignment driver packs the sequences
 * before handing them to the GPU kernels (section "Software stack and
 * parallelism"); this is the size of that packed form.
 */
SW_API size_t sw_packed_bytes(int64_t n_residues);

/*
 * Packing step of the alignment driver (section "Software stack and
 * parallelism": the driver between the application and the kernels packs the
 * data and moves it to the GPU).
 * Encode a concatenated ASCII buffer of n_residues residues (device memory)
 * into the library's packed 5-bit form: a 4-bit plane (8 residues per 32-bit
 * word) followed by a 1-bit plane (32 residues per word), the layout being
 * described in the library source.  Residue positions are unchanged, so the
 * same int64 offsets index sequences in the ASCII and in the packed buffer.
 * packed_dev must be 16-byte aligned and packed_cap at least
 * sw_packed_bytes(n_residues).  Letters outside the alphabet are stored as a
 * padding symbol that scores -4 (the lowest BLOSUM62 score) against every
 * residue; they are reported as SW_ECODE by the next sw_check on this device
 * or by sw_batch_align with SW_VALIDATE, and the results of pairs holding
 * them are not defined.  Errors: SW_EINVAL (null or misaligned pointer,
 * n_residues < 0), SW_ENOMEM (packed_cap too small), SW_EDEVICE.
 */
SW_API int sw_pack(const char* ascii_dev, int64_t n_residues, void* packed_dev, size_t packed_cap,
            void* stream);

/*
 * Batch alignment of candidate pairs, stage (ii) of the paper's pipeline
 * (section "Protein similarity search pipeline"), over the whole m x n matrix
 * of every pair (section "Load balancing techniques").
 * Align n_pairs candidate pairs.
 *   packed_dev    buffer written by sw_pack (16-byte aligned)
 *   offsets_dev   int64[n_seqs + 1]: sequence k is residues offsets[k] ..
 *                 offsets[k+1]-1 of the packed buffer (non-decreasing)
 *   pairs_dev     int32[2 * n_pairs]: (query index, reference index) per pair
 *   scoring       host struct (see above)
 *   out_dev       sw_result[n_pairs], written in pair order
 *   flags         SW_PERSISTENT (0) | SW_PLAIN | SW_VALIDATE | SW_NO_GRAPH |
 *                 SW_TIMED
 * The persistent form runs every forward pass first and then the start
 * passes, regrouped by the size of their regions; the plain form runs both
 * passes of a pair together.
 * A pair with an index outside [0, n_seqs) or a sequence longer than
 * SW_MAX_SEQ_LEN gets score -1 and coordinates -1 and raises SW_ERANGE on the
 * next check; an empty sequence gives score 0.  n_pairs == 0 does nothing.
 * Errors returned directly: SW_EINVAL, SW_ENOMEM, SW_EDEVICE; with
 * SW_VALIDATE the call synchronises `stream` and also returns SW_ERANGE or
 * SW_ECODE.  The SW_PLAIN form reads the bucket sizes back to the host (one
 * synchronisation of `stream` inside the call).
 */
SW_API int sw_batch_align(const void* packed_dev, const int64_t* offsets_dev, int64_t n_seqs,
                   const int32_t* pairs_dev, int64_t n_pairs, const sw_scoring* scoring,
                   sw_result* out_dev, void* stream, uint32_t flags);

/*
 * The search of one sequence set against another (section "Overview of the
 * Problem": queries against references, or a set against itself).
 * Align pairs drawn from two sequence sets, each packed by sw_pack into its
 * own buffer (for instance a query batch against a reference set that stays
 * resident in HBM).  pairs_dev[2k] indexes the query set (n_q sequences,
 * q_offsets_dev int64[n_q + 1]) and pairs_dev[2k+1] the reference set.
 * Results, flags and errors as for sw_batch_align, which is this call with
 * both sets equal.  The device workspace (sort tables, the pair permutation
 * and one boundary-row slot per resident block, about 3 GiB on a 256-CU GPU)
 * belongs to the library: allocated on the first call on a stream, grown to
 * the largest call and kept.
 */
SW_API int sw_align_sets(const void* q_packed_dev, const int64_t* q_offsets_dev, int64_t n_q,
                         const void* r_packed_dev, const int64_t* r_offsets_dev, int64_t n_r,
                         const int32_t* pairs_dev, int64_t n_pairs, const sw_scoring* scoring,
                         sw_result* out_dev, void* stream, uint32_t flags);

/*
 * Device workspace of a caller-owned alignment call (the driver role of
 * section "Software stack and parallelism", with the memory left to the
 * caller).  *bytes (host) receives the size that lets sw_align_sets_ws run
 * n_pairs pairs on the full persistent grid of the current tuning, with
 * boundary-row slots large enough that every pair whose reference holds up
 * to max_len residues takes the fastest whole-wave form.  Smaller buffers
 * still work (see sw_align_sets_ws).
 * Errors: SW_EINVAL (null pointer, negative argument), SW_ERANGE (max_len
 * above SW_MAX_SEQ_LEN, n_pairs of 2^31 - 64 or more), SW_EDEVICE.
 */
SW_API int sw_workspace_size(int64_t n_pairs, int64_t max_len, size_t* bytes);

/*
 * sw_align_sets with the device workspace in workspace_dev (device memory,
 * 256-byte aligned, workspace_bytes long, owned by the caller; the library
 * allocates no device memory for the call and keeps no pointer into the
 * buffer after the enqueued work completes).  The buffer holds the sort
 * tables, the three pair arrays and then as many boundary-row slots of at
 * least 1,280 KiB as fit, up to one per resident block of the persistent grid:
 * a buffer below the sw_workspace_size figure runs a smaller grid (fewer
 * blocks at once, same results).  Two calls in flight at the same time must
 * not share a buffer.  Arguments, results and flags as for sw_align_sets.
 * Errors: as sw_align_sets, plus SW_EINVAL (workspace_dev NULL or not
 * 256-byte aligned) and SW_ENOMEM (not even one slot fits).
 */
SW_API int sw_align_sets_ws(const void* q_packed_dev, const int64_t* q_offsets_dev, int64_t n_q,
                            const void* r_packed_dev, const int64_t* r_offsets_dev, int64_t n_r,
                            const int32_t* pairs_dev, int64_t n_pairs, const sw_scoring* scoring,
                            sw_result* out_dev, void* workspace_dev, size_t workspace_bytes, void* stream,
                            uint32_t flags);

/*
 * For callers that cannot allocate device memory (code under HIP-graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sw_align_sets
 * with its device workspace in a fixed array that the library holds on every
 * device it is loaded on (384 MiB, kept until the process ends).  The call
 * allocates nothing, host or device: it runs the persistent form without HIP
 * graphs and a smaller grid than sw_align_sets (as many blocks as boundary-row
 * slots fit the array), with the same results.  Every call on a device shares
 * that device's array and leaves its contents behind (each call clears what
 * it needs): calls that overlap in time on one device -- on two streams, or
 * from two host threads -- race and must not be issued.
 * flags: SW_VALIDATE, SW_NO_GRAPH (implied); SW_PLAIN and SW_TIMED are refused
 * (SW_EINVAL: both need host state the library would allocate).
 * Errors: as sw_align_sets, plus SW_ENOMEM (with a message in
 * sw_last_device_error) for more than 4,194,304 pairs, the most the array
 * holds.
 */
SW_API int sw_align_sets_static(const void* q_packed_dev, const int64_t* q_offsets_dev, int64_t n_q,
                                const void* r_packed_dev, const int64_t* r_offsets_dev, int64_t n_r,
                                const int32_t* pairs_dev, int64_t n_pairs, const sw_scoring* scoring,
                                sw_result* out_dev, void* stream, uint32_t flags);

/*
 * Error check of the driver (section "Software stack and parallelism"): the
 * kernels record invalid input in a device word instead of stopping.
 * Synchronise `stream`, then return and clear the device-detected errors
 * (SW_ERANGE, SW_ECODE) raised by earlier calls on the current device.
 */
SW_API int sw_check(void* stream);

/*
 * Timers of the kernels (section "How Performance Was Measured": cell updates
 * per second use the time of the alignment kernel alone).
 * Device time of the alignment kernels of the calls made with SW_TIMED on
 * `stream` since the previous read: the two persistent launches of each
 * persistent call (forward passes, then start passes; the sorting kernels
 * before each are not included -- with graph replay every part is its own
 * graph, with the events between them), or the per-bucket launch series of
 * each SW_PLAIN call.  Synchronises `stream`, writes the summed milliseconds
 * to *kernel_ms and the number of calls to *calls, and forgets them.  At most
 * 4096 timed calls may be outstanding on a stream; a further SW_TIMED call
 * returns SW_ENOMEM before launching anything.
 * Errors: SW_EINVAL (null output pointer), SW_EDEVICE.
 */
SW_API int sw_timing_read(void* stream, double* kernel_ms, int64_t* calls);

/*
 * The same read, split by pass (the paper's cell-update rate counts the
 * forward scoring time only, section "How Performance Was Measured"):
 * *forward_ms sums the forward launches of
 * persistent calls (and the whole launch series of SW_PLAIN calls, which run
 * both passes together), *start_ms the start-pass launches.  Synchronises
 * `stream`, forgets the timed calls.  Errors: SW_EINVAL, SW_EDEVICE.
 */
SW_API int sw_timing_read_passes(void* stream, double* forward_ms, double* start_ms, int64_t* calls);

/*
 * Kernel shape (the split of work between lanes, the paper's inter- and
 * intra-task parallelism of section "Software stack and parallelism"), used
 * by later calls on the current device.  rows_per_lane is
 * the number of query rows each lane keeps in registers (8 or 16);
 * inter_max_len is the longest pair (max of both lengths, 64..1024, at most
 * 64 rows_per_lane) that is aligned one pair per lane; longer pairs up to
 * group8_max_len are spread over a group of 8 lanes, longer ones up to
 * group16_max_len over a group of 16 lanes (both powers of two, 64..4096;
 * both 2048 by default, which leaves no pair to 16-lane groups: a 4096-residue
 * pair on 16 lanes outlasts the rest of a launch), longer ones over a whole
 * 64-lane wave; blocks_per_cu sets the
 * persistent grid (1..8; -1 goes back to the occupancy-derived value, which
 * is the default).  A field of 0 (and any other field <= 0) keeps the current
 * value.
 * bucket_lanes[b] overrides that rule for length bucket b, the pairs whose
 * longer sequence has 2^(b-1) + 1 .. 2^b residues (bucket 0: one residue):
 * 1, 8, 16 or 64 lanes per pair, or 0 for the rule above.  One lane needs
 * 2^b <= 1024 and 2^b <= 64 rows_per_lane; 8 or 16 lanes need 2^b <= 4096;
 * 64 lanes fit every bucket.  In sw_set_tuning every entry is applied as
 * given (0 included), so a caller that only changes the other fields passes
 * the table sw_get_tuning returned.  Errors: SW_EINVAL for a value outside
 * these sets, SW_EDEVICE.  Results never depend on any of these values.
 */
#define SW_NUM_BUCKETS 17
typedef struct {
    int32_t rows_per_lane;
    int32_t inter_max_len;
    int32_t blocks_per_cu;
    int32_t group16_max_len;
    int32_t group8_max_len;
    int8_t bucket_lanes[SW_NUM_BUCKETS];
} sw_tuning;
SW_API int sw_set_tuning(const sw_tuning* t);
SW_API int sw_get_tuning(sw_tuning* t);

/*
 * Autotuner of the batching pattern: per length bucket, how many lanes align
 * one pair (the paper balances its alignment work by the cost of each pair,
 * m*n, section "Load balancing techniques").
 * For rows_per_lane 16 and 8 (the occupancy-derived grid), every length
 * bucket that holds pairs of this workload is timed alone with each lane
 * count the bucket allows (1, 8, 16, 64), and keeps the fastest.  A bucket
 * is timed on a filled device: the persistent form over its pairs repeated
 * until a call holds at least 4e9 cells and four one-lane items per block
 * (at most 1.6e10 cells and 2^21 pairs), one untimed call then `reps` timed
 * ones.  Then the
 * whole workload is timed with the current tuning and with each
 * rows_per_lane and its table; the fastest of the three becomes the current
 * tuning (sw_get_tuning shows it).
 * Every candidate must give byte-identical results (else SW_EDEVICE and the
 * previous tuning is restored).  out_dev receives the results of the whole
 * workload under the chosen tuning.
 * cache_path (may be NULL): a JSON file of earlier choices, one entry per
 * (GPU architecture, compute units, blocks per CU, rows_per_lane, gap_open,
 * gap_extend, bucket) with its lane count and time; buckets found there are
 * not timed again, new choices are added and the file rewritten.
 * *chosen receives the tuning, *best_ms (may be NULL) the time of one call of
 * the whole workload with it, *bucket_trials (may be NULL) the number of
 * (bucket, lane count) candidates timed in this call (0 when the cache held
 * every bucket).  Synchronises `stream`.
 * Errors: SW_EINVAL (null pointer, n_pairs <= 0), SW_EDEVICE (a HIP error or
 * results that differ between candidates), SW_ENOMEM, and those of
 * sw_batch_align; an unreadable cache is ignored, an unwritable one is
 * SW_EINVAL after the tuning is applied.
 */
SW_API int sw_autotune(const void* packed_dev, const int64_t* offsets_dev, int64_t n_seqs,
                       const int32_t* pairs_dev, int64_t n_pairs, const sw_scoring* scoring,
                       sw_result* out_dev, void* stream, int32_t reps, const char* cache_path,
                       sw_tuning* chosen, float* best_ms, int32_t* bucket_trials);

/*
 * The scoring matrix (the paper does not name one; BLOSUM62 is used).
 * The library's substitution matrix in the alphabet order above
 * (scores[24*q + r], query symbol q, reference symbol r) and the alphabet
 * itself (25 bytes including the terminating zero).  Host memory.
 */
SW_API int sw_matrix(int32_t matrix_id, int8_t* scores, char* letters);

/* ---------------------------------------------------------- candidate discovery
 * Which pairs to align: every (query, reference) pair whose sequences have at
 * least min_shared DISTINCT k-mers (runs of k consecutive residues) in
 * common.  This is the overlap product of the paper's sequence-by-k-mer
 * matrix with itself (section "Protein similarity search pipeline": the
 * product counts common k-mers; section "Similarity search at scale":
 * k = 6, threshold 2).  A sequence that repeats a k-mer holds it once; a
 * sequence shorter than k has none.
 *
 * Inputs are two sets packed by sw_pack (they may be the same buffer and
 * offsets: a self search), with int64 device offsets as for sw_align_sets.
 * mode selects the pairs of a self search (section "Load balancing
 * techniques": the overlap matrix is symmetric, one alignment per unordered
 * pair suffices):
 *   SW_DISCOVER_ALL     every (q, r) pair, the diagonal of a self search
 *                       included;
 *   SW_DISCOVER_UPPER   q < r only (the triangularity scheme);
 *   SW_DISCOVER_PARITY  the index-based scheme: q > r with equal index
 *                       parities, or q < r with different ones.
 * The two self-search modes need n_q == n_r and keep exactly one of every
 * unordered pair {i, j}, i != j.
 *
 * Output: pairs_out_dev int32[2 * out_cap] receives (query, reference) index
 * pairs -- the layout sw_align_sets takes -- and shared_out_dev int32[out_cap]
 * (may be NULL) the count of distinct shared k-mers of each.  The ORDER of the
 * pairs is unspecified (it varies from call to call); the set is exact.
 * *n_found (host) receives the total number of qualifying pairs; when it
 * exceeds out_cap only out_cap of them are written and the call returns
 * SW_ENOMEM, so a caller may size its buffers with out_cap = 0 first.
 *
 * The call is synchronous with respect to the host (it reads table sizes
 * back between its launches) and enqueues everything on `stream`.  Its
 * workspace (hash tables of twice the number of k-mer windows and of twice
 * the number of k-mer matches, two int32 arrays of 24^k entries) grows to the
 * largest call seen on the stream and is kept for reuse.
 *
 * table_budget_bytes bounds the (query, reference) counter table, the part
 * that grows with the number of k-mer matches (12 bytes per slot, twice as
 * many slots as matches, rounded up to a power of two).  0 means no bound.
 * When the whole table would exceed it, the queries are cut into contiguous
 * ranges whose tables fit, and each range is counted and written in a pass
 * of its own (the overlap product formed block by block, as the paper does
 * to bound the memory of discovery, section "Blocked 2D Sparse SUMMA").  A
 * single query whose matches alone exceed the budget forms a range with a
 * table of its own size.  The result does not depend on the budget.
 *
 * Errors: SW_EINVAL (null pointer, k outside 1..6, min_shared < 1, unknown
 * mode, a self-search mode with n_q != n_r), SW_ERANGE (offsets not
 * increasing or beyond the packed buffer, 2^31 or more k-mer windows in the
 * reference set), SW_ECODE (a residue that is not a symbol), SW_ENOMEM
 * (device memory, or out_cap too small), SW_EDEVICE.
 */
#define SW_DISCOVER_ALL 0
#define SW_DISCOVER_UPPER 1
#define SW_DISCOVER_PARITY 2

SW_API int sw_discover(const void* q_packed_dev, const int64_t* q_offsets_dev, int64_t n_q,
                       const void* r_packed_dev, const int64_t* r_offsets_dev, int64_t n_r,
                       int32_t k, int32_t min_shared, int32_t mode, int32_t* pairs_out_dev,
                       int32_t* shared_out_dev, int64_t out_cap, int64_t* n_found,
                       size_t table_budget_bytes, void* stream);

/* ------------------------------------------------------ identity and coverage
 * The alignment metrics the paper forms its similarity graph from (section
 * "Protein similarity search pipeline": identity and coverage of each
 * aligned pair, kept above thresholds -- 0.30 and 0.70 in the program
 * parameters of section "Similarity search at scale").
 *
 * For every pair whose aligned score (aligned_dev, this library's results for
 * the same pairs, sets and scoring) is positive, the pass takes the box the
 * aligner reported, q[q_start..q_end] x r[r_start..r_end], and among all
 * global alignments of that box picks the best by score, then by the number
 * of identical aligned pairs, then by the fewest columns (aligned pairs plus
 * gap positions).  Its score equals the aligned score.  The record holds
 * that score, the matches, the columns, and keep = 1 when
 *   1000 * matches >= ani_permille * columns,
 *   1000 * (q_end - q_start + 1) >= cov_permille * (query length), and
 *   1000 * (r_end - r_start + 1) >= cov_permille * (reference length)
 * (identity and both coverages at least the thresholds, given in
 * thousandths; integer arithmetic).  A pair with score 0 gets all zeros.
 *
 * Sets, offsets and pairs as for sw_align_sets; out_dev receives n_pairs
 * records.  Asynchronous on `stream` like sw_align_sets; with SW_VALIDATE the
 * call synchronises and reports device-found errors.  With SW_COVERAGE_FIRST
 * a pair whose coverage already misses the threshold is not swept: its
 * record is {score, -1, -1, 0} (keep is 0 either way, so every keep flag is
 * the same as without the flag).  Workspace: one scratch
 * row pair of 65,536 int64 per resident wave (4 GiB on a 256-CU GPU),
 * allocated on the first call on a stream and kept.
 *
 * Errors: SW_EINVAL (null pointer, bad scoring or flags, thresholds outside
 * 0..1000), SW_ERANGE (pair index or coordinates outside the sequences, or a
 * box whose best score differs from the aligned score: found on the device,
 * reported under SW_VALIDATE or by sw_check), SW_ECODE, SW_ENOMEM, SW_EDEVICE.
 */
#define SW_COVERAGE_FIRST 16u /* sw_identity: skip the sweep of pairs that fail coverage */

typedef struct {
    int32_t score;   /* best global score of the box (the aligned score) */
    int32_t matches; /* identical aligned pairs */
    int32_t columns; /* aligned pairs plus gap positions */
    int32_t keep;    /* 1: identity and both coverages reach the thresholds */
} sw_identity_result;

SW_API int sw_identity(const void* q_packed_dev, const int64_t* q_offsets_dev, int64_t n_q,
                       const void* r_packed_dev, const int64_t* r_offsets_dev, int64_t n_r,
                       const int32_t* pairs_dev, int64_t n_pairs, const sw_scoring* scoring,
                       const sw_result* aligned_dev, int32_t ani_permille, int32_t cov_permille,
                       sw_identity_result* out_dev, void* stream, uint32_t flags);

/* ------------------------------------------------------------ whole search
 * The paper's search pipeline on one GPU (section "Protein similarity search
 * pipeline": discovery of candidate pairs by shared k-mers, their batch
 * alignment, then the identity and coverage filter that makes the edges of
 * the similarity graph), formed block by block with the next block made
 * ready while the current one aligns (section "Pre-blocking").
 * The queries are cut into contiguous blocks of block_queries queries (0:
 * half of them).  For each block, sw_discover's pairs (k, min_shared,
 * mode as there; the mode filters use the global query index) are handed on
 * the device to the aligner (persistent form) and to sw_identity
 * (ani_permille, cov_permille as there), and the pairs it keeps are appended
 * to the outputs: edges_dev int32[2 * edge_cap] (query, reference),
 * edge_results_dev sw_result[edge_cap], edge_ident_dev
 * sw_identity_result[edge_cap], in no particular order (the set is exact).
 * Discovery runs on `stream` (after the work already enqueued on it); each
 * block's alignment and filter run on one of two internal streams,
 * alternately, so the discovery of block b+1 overlaps the alignment of
 * block b and block b+1's launches fill the compute units that block b's
 * last long items leave idle; two sets of block buffers, kept by the
 * library and grown to the largest block, bound the memory.  The call
 * returns when everything is done.  HIP maps streams onto GPU_MAX_HW_QUEUES
 * hardware queues (4 by default) and two streams on one queue run one after
 * the other: with more streams alive in the process (the library's graph
 * capture stream, server slots, the caller's own) the two internal streams
 * may share a queue, and the blocks then no longer overlap.
 * *stats receives the candidates, the edges (all of them, also when more
 * than edge_cap: then only edge_cap are written and the call returns
 * SW_ENOMEM) and the number of blocks.  Calls on one device run one at a
 * time.  Errors: those of sw_discover, sw_align_sets and sw_identity.
 */
typedef struct {
    int64_t candidates; /* pairs discovery found */
    int64_t edges;      /* pairs the filter kept */
    int32_t blocks;     /* query blocks */
    int32_t reserved;
} sw_search_stats;

SW_API int sw_search(const void* q_packed_dev, const int64_t* q_offsets_dev, int64_t n_q,
                     const void* r_packed_dev, const int64_t* r_offsets_dev, int64_t n_r, int32_t k,
                     int32_t min_shared, int32_t mode, const sw_scoring* scoring, int32_t ani_permille,
                     int32_t cov_permille, int64_t block_queries, int32_t* edges_dev,
                     sw_result* edge_results_dev, sw_identity_result* edge_ident_dev, int64_t edge_cap,
                     sw_search_stats* stats, void* stream);

/* ------------------------------------------------------------------ serving
 * Continuous batching against a reference set resident in HBM.  The server
 * keeps `max_slots` HIP streams, each with its own alignment workspace, and an
 * arena of hbm_budget_bytes for the device state of admitted requests (query
 * ASCII, packed queries, offsets, candidate pairs, results; see
 * sw_server_request_bytes).  A request is admitted when its state fits in the
 * part of the budget not held by earlier unfinished requests; admitted
 * requests queue in arrival order, and whenever a slot is free all queued
 * requests (up to 2^24 pairs) are merged into one launch on it.  A request
 * that arrives while the device is busy therefore joins the next launch, and
 * launches on different slots overlap.  Completions are collected and new
 * launches started inside submit, poll, wait and stats.  Results of a request
 * do not depend on what else is in flight.  The reference buffers (from
 * sw_pack) stay owned by the caller and must outlive the server.  Servers are
 * not shareable between devices; calls on one server are serialised by the
 * server.
 */
typedef struct sw_server sw_server;

/* A resident reference set and its request loop: the paper's search aligns
 * query batches against a reference set one block at a time (sections
 * "Blocked 2D Sparse SUMMA" and "Pre-blocking": the next batch is made ready
 * while the current one aligns).
 * Errors: SW_EINVAL (bad argument or scoring), SW_ENOMEM (arena allocation),
 * SW_EDEVICE. */
SW_API int sw_server_create(const void* refs_packed_dev, const int64_t* ref_offsets_dev, int64_t n_refs,
                            const sw_scoring* scoring, size_t hbm_budget_bytes, int max_slots,
                            sw_server** server);

/* Admission of one query batch with its candidate list (the pairs stage (i)
 * of section "Protein similarity search pipeline" discovered).
 * Submit n_q query sequences (host ASCII, host int64 offsets[n_q + 1] with
 * offsets[0] == 0) with n_cand candidate pairs (host int32 [query index within
 * the request, reference index]).  On SW_OK *ticket identifies the request and
 * out_host (host, n_cand results) is written when the request completes
 * (poll/wait); the library copies the inputs before returning.  SW_EAGAIN: not
 * enough free budget now, retry after a completion.  SW_ENOMEM: the request
 * can never fit the budget.  SW_ERANGE: a query index outside [0, n_q), or
 * more than 2^24 pairs.  SW_ECANCELED after destroy began.  A reference index
 * outside the resident set gives score -1 for that pair. */
SW_API int sw_server_submit(sw_server* server, const char* q_ascii, const int64_t* q_offsets, int64_t n_q,
                            const int32_t* cand, int64_t n_cand, sw_result* out_host, uint64_t* ticket);

/* Completion of a request (its alignments, stage (ii) of section "Protein
 * similarity search pipeline").
 * SW_OK once the request is complete (results copied, resources freed; the
 * ticket is then retired), SW_EAGAIN while it waits or runs, SW_EINVAL for an
 * unknown ticket; a launch that failed returns its error (SW_EDEVICE,
 * SW_ENOMEM) for each of its requests. */
SW_API int sw_server_poll(sw_server* server, uint64_t ticket);

/* Bounded wait for a request (as sw_server_poll, section "Protein similarity
 * search pipeline" stage (ii)).
 * Poll until complete or until timeout_us elapses (SW_ETIMEOUT); a negative
 * timeout waits without limit. */
SW_API int sw_server_wait(sw_server* server, uint64_t ticket, int64_t timeout_us);

/* Memory held by requests in flight (the paper bounds the memory of the
 * blocks in flight, section "Pre-blocking": extra memory for the next block).
 * Requests admitted and not complete, budget bytes they hold and the budget
 * (any pointer may be NULL). */
SW_API int sw_server_stats(sw_server* server, int64_t* inflight, int64_t* bytes_in_use, int64_t* budget);

/* Admission size of a request (section "Pre-blocking": memory of a block in
 * flight).  Arena bytes a request of this size needs (0 for negative
 * arguments). */
SW_API size_t sw_server_request_bytes(int64_t n_residues, int64_t n_q, int64_t n_cand);

/* End of the request loop (section "Pre-blocking"): wait for every request
 * in flight, then free the server. */
SW_API int sw_server_destroy(sw_server* server);

/* Error reporting of the driver (section "Software stack and parallelism":
 * the layer between the application and the kernels).  Text of a status
 * code; never NULL. */
SW_API const char* sw_strerror(int status);

/* The same driver's record of the last HIP runtime error (or refusal with a
 * message) seen by the library on this thread. */
SW_API const char* sw_last_device_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SW_H */
