/*
 * fastcount.h -- C ABI of the MI355X (gfx950) exact counting library.
 *
 * Method: Karan, Eichhorn, Hurlburt, Iraci, Zola, "Fast Counting in Machine
 * Learning Applications" (UAI 2018, arXiv 1804.04640).
 *
 * Data model (Section 2).  A complete categorical database D of n variables
 * and m instances; variable v has arity r_v in 1..255 and every instance
 * holds a state 0 <= s < r_v (the paper numbers states 1..r_v; state s here
 * is the paper's s+1).  A query is an ordered list of k distinct variables,
 * 1 <= k <= FC_MAX_VARS.  Query(X_i, Pa) of Sections 3.1-3.3 is the list
 * Pa ++ [X_i]: the child is the last variable.
 *
 * Dense table layout.  The contingency table of a query has prod r_v cells
 * (q_i * r_i, Section 2), int32, mixed-radix with vars[0] the most
 * significant digit and the child the least significant one (the MSD digit
 * order of Section 3.3):
 *     idx = ((s_0 * r_1 + s_1) * r_2 + ...) * r_{k-1} + s_{k-1}
 * so row j (one parent configuration) is the contiguous slice
 * [j * r_i, (j + 1) * r_i).
 *
 * Pointers.  Query descriptions (vars, var_off, table_off, items, states)
 * are host memory.  Output buffers (tables, scores, err, gram, pair records)
 * may be device memory (for example a torch tensor's data_ptr) or host
 * memory; the library tells them apart with hipPointerGetAttributes.  With
 * device outputs a call is asynchronous on `stream` (a hipStream_t; NULL is
 * the null stream); with host outputs it returns after the results are in
 * place.  Every output buffer is owned by the caller.
 *
 * Errors.  Every int-returning call returns FC_OK (0) or a negative FC_ERR_*
 * code and never aborts.  A batch is validated as a whole before anything
 * is launched, so a rejected call has no effect; fc_last_error() then holds
 * a message (per host thread) that names the first offending query index.
 *
 * Threads.  An fc_db is immutable once created.  Calls on one fc_db from
 * several host threads, each on its own stream, may run concurrently: every
 * call owns its scratch memory (the independent function objects of
 * Section 3.1).
 */
#ifndef FASTCOUNT_H
#define FASTCOUNT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fc_db fc_db;

/* Status codes. */
#define FC_OK 0
#define FC_ERR_INVALID (-1) /* malformed argument or query            */
#define FC_ERR_RANGE (-2)   /* a size beyond what the library handles  */
#define FC_ERR_NOMEM (-3)   /* device or pinned host allocation failed */
#define FC_ERR_DEVICE (-4)  /* a HIP runtime call failed               */

#define FC_MAX_VARS 8

/* fc_db_create layouts. */
#define FC_COL_MAJOR 0 /* data[v * m + p]: n columns of m states       */
#define FC_ROW_MAJOR 1 /* data[p * n + v]: m instances of n states     */

/* fc_db_create flags. */
#define FC_DB_BITVECTORS 1u     /* also build per-state bit-vectors        */
#define FC_DB_DATA_ON_DEVICE 2u /* `data` is a device pointer              */

/* Strategy field of the batch flags (low 4 bits).  FC_STRAT_AUTO chooses per
 * query shape (tuning below); in a large batch on a handle with bit-vectors
 * it may also count every one- and two-variable query at once as the Gram
 * of their variables' state bit-vectors (Section 3.2's two-vector
 * intersections on the matrix cores).  Every strategy yields identical
 * counts. */
#define FC_STRAT_AUTO 0u      /* per-query choice by the cost model / tuner */
#define FC_STRAT_HIST 1u      /* joint key + LDS histogram (Section 3.3)    */
#define FC_STRAT_BITMAP 2u    /* AND of bit-vectors + popcount (Sec. 3.2)   */
#define FC_STRAT_PARTITION 3u /* MSD partition by the top key digits: keys */
                              /* formed in one pass and moved to their      */
                              /* parts, each part counted in LDS (Section   */
                              /* 3.3); beyond 2^25 cells, key windows that  */
                              /* each rescan the columns                    */
#define FC_STRAT_SORT FC_STRAT_PARTITION
#define FC_STRAT_MASK 0xFu

/* Reducers (bit mask; several may be fused into one counting pass). */
#define FC_RED_LL 1u   /* log-likelihood of Eq. (1), bits (Fig. 2)          */
#define FC_RED_MDL 2u  /* -LL + 1/2 log2(m) q (r-1), bits, minimised        */
#define FC_RED_BDEU 4u /* BDeu log marginal likelihood, nats, maximised     */
#define FC_RED_MI 8u   /* mutual information child ; parents, nats          */

typedef struct fc_reduce_params {
    double ess; /* BDeu equivalent sample size alpha (> 0); 1.0 if NULL */
} fc_reduce_params;

typedef struct fc_pair_rec {
    int32_t a, b;     /* item indices into the `items` list, a < b     */
    int32_t n_ab;     /* Count(X_a = 1 AND X_b = 1)                     */
    float support;    /* n_ab / m                                       */
    float conf_ab;    /* n_ab / Count(X_a = 1): confidence of a => b    */
    float conf_ba;    /* n_ab / Count(X_b = 1): confidence of b => a    */
} fc_pair_rec;

/*
 * Make D resident on the current HIP device (Section 2 database; the
 * column-major layout and precomputed per-variable partitions of Section
 * 3.3; the per-state bitmaps of Section 3.2 when FC_DB_BITVECTORS is set).
 *
 * data    n*m states, FC_COL_MAJOR or FC_ROW_MAJOR; host memory unless
 *         FC_DB_DATA_ON_DEVICE.  The caller keeps ownership; it is copied.
 * m       instances, 0 <= m < 2^31 (counts are int32).
 * n       variables, n >= 1.
 * arity   host array of n arities, each 1..255.
 * stream  stream for the upload and preprocessing kernels; the call
 *         synchronises it before returning.
 * out     receives the handle.
 * Fails with FC_ERR_INVALID on a bad argument or when a state is not below
 * its variable's arity (the database must be complete), FC_ERR_RANGE when
 * m >= 2^31, FC_ERR_NOMEM when device memory runs out.
 */
int fc_db_create(const uint8_t *data, int64_t m, int32_t n,
                 const uint8_t *arity, int32_t layout, uint32_t flags,
                 void *stream, fc_db **out);

/*
 * Append m_new instances to a database (the extension noted in Section 6:
 * the bitmaps are updated, a column scan needs nothing else).  data, layout
 * and FC_DB_DATA_ON_DEVICE are as in fc_db_create; the new states are
 * validated before anything changes, so a rejected append leaves the handle
 * as it was.  Columns, marginals, entropies and bit-vectors are updated in
 * place; their allocation grows 1.5x at a time when the rows outgrow it, so
 * appends cost O(m_new) amortised.  Graphs captured before
 * the append are invalidated: fc_graph_launch then fails with
 * FC_ERR_INVALID.  Must not run concurrently with other calls on the handle;
 * synchronises the device.
 */
int fc_db_append(fc_db *db, const uint8_t *data, int64_t m_new, int32_t layout,
                 uint32_t flags, void *stream);

/* Free every device and host resource of the handle (NULL is a no-op). */
void fc_db_destroy(fc_db *db);

/*
 * Release the handle's idle device workspaces.  Batches take their plan,
 * the tables their reducers consume, and sort or descriptor scratch from up
 * to four workspaces that the handle keeps between calls (allocation and
 * release cost more host time than small batches take), so after a batch
 * the handle holds device memory up to a few times its largest batch
 * footprint (fc_batch_footprint) beyond the database; fc_db_info's device
 * bytes include it.  Waits for each workspace's last use, frees it, and
 * leaves workspaces in use by concurrent calls alone.  Later calls allocate
 * again as needed.
 */
int fc_db_trim(fc_db *db);

/*
 * Database facts: instances, variables, whether bit-vectors exist, and the
 * device bytes held.  Any output pointer may be NULL.
 */
int fc_db_info(const fc_db *db, int64_t *m, int32_t *n, int32_t *has_bits,
               int64_t *device_bytes);

/*
 * Host copies of the per-variable marginal counts (sum of arities int64
 * values, variable-major) and entropies in bits (n floats), computed on the
 * device at creation; the entropy order drives the Bitmap traversal order of
 * Section 3.2.  Either pointer may be NULL.
 */
int fc_db_marginals(const fc_db *db, int64_t *counts, float *entropy_bits);

/*
 * Number of cells prod r_v of the query's table (q_i * r_i, Section 2), or a
 * negative FC_ERR_* code for an invalid query.
 */
int64_t fc_table_cells(const fc_db *db, const int32_t *vars, int32_t k);

/*
 * One query, one dense int32 table (Section 2 definition; the per-query
 * path).  `cells` must equal fc_table_cells(db, vars, k).  `table` is
 * overwritten.
 */
int fc_count(fc_db *db, const int32_t *vars, int32_t k, int32_t *table,
             int64_t cells, void *stream);

/*
 * Count((X_vars[0] = states[0]) AND ...): the single-assignment query of
 * Section 2, answered by one path of bit-vector intersections and a
 * popcount (the single-path specialisation closing Section 3.3).  Uses the
 * bit-vectors when the handle has them, the state columns otherwise.  The
 * result is written to the host int64 `*count`; the call synchronises.
 */
int fc_count_assignment(fc_db *db, const int32_t *vars, const uint8_t *states,
                        int32_t k, int64_t *count, void *stream);

/*
 * Sparse table of one query for key spaces far beyond the data (prod r_v up
 * to 2^63, e.g. many high-arity variables): the distinct configurations that
 * occur -- at most min(q_i r_i, m), Section 3.2 -- as mixed-radix keys (int64,
 * same digit order as the dense table) in increasing order with their int32
 * counts, found by sorting the instances' keys and run-length encoding them
 * (the MSD order of Section 3.3 carried to the last digit).  keys and counts
 * (device or host memory) hold `cap` entries; *nnz receives the number of
 * distinct configurations, which may exceed cap (then the cap smallest keys
 * are written).  Synchronises `stream`.
 */
int fc_count_sparse(fc_db *db, const int32_t *vars, int32_t k, int64_t *keys,
                    int32_t *counts, int64_t cap, int64_t *nnz, void *stream);

/*
 * Sparse tables of many queries in one submission (the sparse form of
 * Section 3.2 for a batch, as fc_count_batch is for dense tables).  Query i
 * is vars_flat[var_off[i] .. var_off[i+1]) (1..FC_MAX_VARS distinct
 * variables, key space below 2^63); var_off holds nq+1 int64 values starting
 * at 0.  The pairs of all queries are packed in query order: query i's
 * (key, count) pairs, keys increasing, occupy [out_off[i], out_off[i+1]) of
 * keys (int64) and counts (int32); out_off is host memory of nq+1 entries,
 * *total_nnz = out_off[nq].  keys and counts are both device or both host
 * memory and hold `cap` entries (total_nnz <= nq * m always).  When the
 * total exceeds cap the call returns FC_ERR_RANGE with out_off and
 * *total_nnz set and keys/counts unspecified, so the caller can size and
 * call again.  Queries are grouped (ordered by key space within windows
 * of consecutive queries); a group shares one radix sort of composite keys
 * (its offset in the group plus the query's key, at most 2^26 keys per
 * sort).  The grouping affects speed only.  Synchronises `stream`.
 */
int fc_count_sparse_batch(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                          int64_t nq, int64_t *keys, int32_t *counts, int64_t cap,
                          int64_t *out_off, int64_t *total_nnz, void *stream);

/*
 * Many single-assignment counts in one submission (the queries of the
 * association-rule search of Section 4.3, each a path of |Pa|+1 bitmap
 * intersections and a popcount).  Query i assigns states_flat[var_off[i] ..
 * var_off[i+1]) to vars_flat[var_off[i] .. var_off[i+1]); counts[i] (int64,
 * device or host memory) receives Count(...).  Uses the bit-vectors when the
 * handle has them, the state columns otherwise.
 */
int fc_count_assignments(fc_db *db, const int32_t *vars_flat,
                         const int64_t *var_off, const uint8_t *states_flat,
                         int64_t nq, int64_t *counts, void *stream);

/*
 * Many queries of uneven size in one submission (concurrent query groups,
 * Section 3.1).  Query i is vars_flat[var_off[i] .. var_off[i+1]); its table
 * is written at tables[table_off[i] .. table_off[i] + cells_i).  var_off and
 * table_off hold nq+1 int64 values; table_off may be NULL, meaning tables are
 * packed back to back in query order.  flags: an FC_STRAT_* value (forced
 * strategies exist for testing; every strategy returns identical tables;
 * where a forced strategy cannot hold a table -- Bitmap beyond 128 cells,
 * histogram beyond LDS -- the next one that can is used).
 */
int fc_count_batch(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                   int64_t nq, int32_t *tables, const int64_t *table_off,
                   uint32_t flags, void *stream);

/*
 * Query(X_i, Pa, F) with F drawn from a fixed set of reducers (Sections 3.1,
 * Fig. 2, Eq. (1); MDL and BDeu of Section 4.2; mutual information of
 * Section 1): counts every query's table and streams it into each reducer in
 * the `reducers` mask.  Scores are float32 computed with compensated
 * summation; for the j-th set bit of the mask (ascending), scores[j*nq + i]
 * is query i's score and, if err is not NULL, err[j*nq + i] an upper
 * estimate of its absolute rounding error.  `tables` may be NULL: the counts
 * are then consumed and never stored (Section 3.1); otherwise it receives the
 * tables as in fc_count_batch.  p may be NULL (ess = 1).
 */
int fc_count_reduce(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                    int64_t nq, uint32_t reducers, const fc_reduce_params *p,
                    float *scores, float *err, int32_t *tables,
                    const int64_t *table_off, uint32_t flags, void *stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fc_count_reduce with the tables consumed, allocating no device or pinned
 * host memory.  The plan image and the tables live in one statically sized
 * device array of FC_NOALLOC_SCRATCH_BYTES per GPU, which the library holds
 * from its first use on that GPU until the process ends.
 *
 * Arguments are those of fc_count_reduce without tables/table_off; scores
 * ([slot][nq] floats) and err (same layout, may be NULL) must be device
 * memory.  Results are bitwise those of fc_count_reduce for the same batch
 * and tuning.  Asynchronous on `stream`.  The plan image is copied from
 * pageable host memory, so the host thread waits for that copy.
 *
 * Errors: those of fc_count_reduce; FC_ERR_INVALID for host-memory scores
 * or err; FC_ERR_RANGE when the batch needs more scratch than
 * FC_NOALLOC_SCRATCH_BYTES (plan image plus 4 bytes per table cell; the
 * message gives the figure), before anything is launched.
 *
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or host threads without ordering) race and give
 * wrong results.  Calls on one stream are ordered and safe.
 */
#define FC_NOALLOC_SCRATCH_BYTES (64ll << 20)
int fc_count_reduce_noalloc(fc_db *db, const int32_t *vars_flat,
                            const int64_t *var_off, int64_t nq, uint32_t reducers,
                            const fc_reduce_params *p, float *scores, float *err,
                            uint32_t flags, void *stream);

/*
 * Exact parent-set search support (Section 4.2): the scores of every parent
 * set of `size` variables drawn from cand[0..ncand-1] (distinct, not the
 * child) for one child, enumerated by the library.  Set i is the i-th
 * `size`-subset of the positions 0..ncand-1 in lexicographic order; the query
 * counted for it is the subset's variables (in cand order) followed by the
 * child.  nsets must equal C(ncand, size), and size + 1 <= FC_MAX_VARS.
 * scores (device or host) receives, for the j-th set bit of `reducers`,
 * scores[j*nsets + i], exactly the values fc_count_reduce gives for the same
 * queries.  prune_mdl > 0 (only with reducers == FC_RED_MDL): a set whose MDL
 * penalty 1/2 log2(m) q (r-1) alone is >= prune_mdl is not counted and
 * scores +infinity (its MDL, and every superset's, is at least that bound).
 * The stream is synchronised when scores is a host pointer.
 */
int fc_score_parent_sets(fc_db *db, int32_t child, const int32_t *cand,
                         int32_t ncand, int32_t size, uint32_t reducers,
                         const fc_reduce_params *p, double prune_mdl,
                         float *scores, int64_t nsets, void *stream);

/*
 * All 2-itemset supports of binary items (association rule mining, Section
 * 4.3) from the co-occurrence Gram matrix A^T A of the one-hot instance x item
 * matrix, computed exactly on the FP4 matrix cores (0/1 operands, fp32
 * partial sums of at most 2^24 instances, int32 totals).  items lists
 * ni distinct variables of arity 2 (state 1 = item present); NULL means all
 * variables.  gram (nullable, ni*ni int32, row-major) receives the full
 * symmetric matrix.  Every pair a < b with n_ab / m > minsup is written to
 * out (ordered by a, then b) up to `cap` records; *n_out receives the total
 * number of qualifying pairs (which may exceed cap).  Needs bit-vectors.
 */
int fc_pairs(fc_db *db, const int32_t *items, int32_t ni, double minsup,
             int32_t *gram, fc_pair_rec *out, int64_t cap, int64_t *n_out,
             void *stream);

/*
 * Bottom-up association-rule mining over binary items (Section 4.3), the
 * whole level-wise search in one call.  Level 1 comes from the marginals,
 * level 2 from the co-occurrence Gram (as fc_pairs), and every level k >= 3
 * joins the frequent (k-1)-itemsets that share their first k-2 items, keeps
 * a candidate only when all its (k-1)-subsets are frequent, and counts the
 * candidates as batched single-assignment queries Count(X_a = 1 AND ...)
 * (as fc_count_assignments).  An itemset S is frequent when Count(S)/m >
 * minsup; a rule S - {X} => X is kept when Count(S)/Count(S - {X}) >
 * minconf (both binary64).  Itemsets have at most max_size items
 * (1..FC_MAX_VARS; the paper mines rules of fewer than seven items).
 *
 * items   host array of ni distinct variables, each of arity 2 (item a is
 *         present in an instance when X_a = 1).  Needs bit-vectors.
 * out     receives a result owned by the caller (fc_arm_free); read it with
 *         fc_arm_sizes and fc_arm_read.  Synchronises `stream`.
 * Fails with FC_ERR_INVALID on a bad argument (unknown, repeated or
 * non-binary item, max_size out of range).
 */
typedef struct fc_arm_result fc_arm_result;
int fc_mine(fc_db *db, const int32_t *items, int32_t ni, double minsup,
            double minconf, int32_t max_size, fc_arm_result **out, void *stream);

/*
 * Sizes of a mining result: itemsets, items over all itemsets, rules, and
 * antecedent items over all rules.
 */
int fc_arm_sizes(const fc_arm_result *r, int64_t *n_sets, int64_t *n_set_items,
                 int64_t *n_rules, int64_t *n_rule_items);

/*
 * Copies a mining result into host arrays sized by fc_arm_sizes (any
 * pointer may be NULL to skip that array):
 *   set_items[n_set_items], set_off[n_sets+1], set_count[n_sets]: itemset i
 *     is set_items[set_off[i] .. set_off[i+1]) (increasing item ids) with
 *     Count = set_count[i]; itemsets come level by level, lexicographic
 *     within a level;
 *   rule_items[n_rule_items], rule_off[n_rules+1], rule_cons[n_rules],
 *   rule_support[n_rules], rule_conf[n_rules]: rule j is antecedent
 *     rule_items[rule_off[j] .. rule_off[j+1]) => rule_cons[j], support
 *     Count(S)/m, confidence Count(S)/Count(antecedent); rules are ordered by
 *     antecedent (item by item, a proper prefix first), then consequent.
 */
int fc_arm_read(const fc_arm_result *r, int32_t *set_items, int64_t *set_off,
                int64_t *set_count, int32_t *rule_items, int64_t *rule_off,
                int32_t *rule_cons, double *rule_support, double *rule_conf);

/* Releases a mining result (NULL is ignored). */
void fc_arm_free(fc_arm_result *r);

/*
 * Device bytes a batch needs beyond the resident database: tables and
 * scratch of fc_count_reduce with tables == NULL, the work plan, and the
 * staging of host outputs.  Used by callers that admit work by memory.
 */
int fc_batch_footprint(const fc_db *db, const int32_t *vars_flat,
                       const int64_t *var_off, int64_t nq, uint32_t flags,
                       int64_t *bytes);

/*
 * Captured batch (hipGraph).  fc_graph_create plans a batch once, uploads its
 * plan into buffers the graph owns and records every device step -- table
 * zeroing, counting, reducers -- into a graph; each fc_graph_launch replays
 * all of that work on `stream` with no host planning, for callers that run
 * the same batch repeatedly.  Arguments are those of fc_count_reduce
 * (reducers may be 0: counts only, then `tables` is required); every output
 * buffer must be device memory and stay valid while the graph exists.  The
 * graph reads the database, which must outlive it.
 */
typedef struct fc_graph fc_graph;

int fc_graph_create(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                    int64_t nq, uint32_t reducers, const fc_reduce_params *p,
                    float *scores, float *err, int32_t *tables,
                    const int64_t *table_off, uint32_t flags, void *stream,
                    fc_graph **out);

/* Replay the captured batch on `stream` (asynchronous). */
int fc_graph_launch(fc_graph *g, void *stream);

/* Wait for the graph's launches, then free it (NULL is a no-op). */
void fc_graph_destroy(fc_graph *g);

/*
 * Tuning of one database handle: which strategy FC_STRAT_AUTO gives each
 * query shape (Section 3.1: the traversal can be switched per query context)
 * and the row-chunk sizes of the counting launches.  Counts never depend on
 * these values, only the time they take.
 */
typedef struct fc_tuning {
    int64_t chunk_rows;        /* histogram instances per workgroup, >= 4096 */
    int64_t bitmap_chunk_rows; /* bitmap instances per workgroup, >= 4096    */
    int32_t bitmap_words;      /* 64-instance words per tree walk: 1, 2 or 4 */
    int32_t persistent_max_queries; /* batches of at most this many queries
                                  count their small tables in one persistent
                                  launch fed by per-XCD work queues (0: never) */
    /* bitmap_cells[k-1][b]: FC_STRAT_AUTO counts a query of k variables with
     * the Bitmap strategy when its table has at most 2^(b+2) cells and this
     * entry is non-zero (b = 0..5: up to 4, 8, 16, 32, 64, 128 cells).      */
    uint8_t bitmap_cells[FC_MAX_VARS][6];
    int32_t packed_columns;    /* 1: histogram kernels read the 4-bit packed
                                  columns when the database has them, 0: the
                                  byte columns                            */
    int32_t bitmap_order;      /* 1: the Bitmap tree walks a query's
                                  variables by ascending marginal entropy
                                  (Section 3.2; ties by lower variable
                                  index), 0: in the query's order.  Either
                                  order gives the same table.              */
    int32_t derive_tables;     /* 1: an automatic plan sums the table of a
                                  query of 3 or 4 variables out of the table
                                  of another query of the batch whose
                                  variables contain its own (or of an equal
                                  query), instead of counting it from the
                                  instances; 0: every query is counted.
                                  The tables are the same.                 */
    int32_t one_pass_partition; /* 1: tables beyond the LDS classes (up to
                                  2^25 cells) are counted by the one-pass
                                  partition (columns read once, keys moved
                                  to their parts); 0: by key windows, each
                                  a scan of the columns.  Same tables.     */
    int32_t row_sweep;         /* 1: the histogram workgroups resident on an
                                  XCD start their row chunks where the
                                  workgroups they replace ended, so they
                                  read the same rows at the same time and
                                  share them in the XCD's L2; 0: every
                                  workgroup starts at its chunk's first row.
                                  Same tables.                             */
} fc_tuning;

/*
 * How a batch would be answered, planned but not launched (flags as in
 * fc_count_batch): out[0] queries counted by LDS-histogram kernels (whole,
 * in key windows or by the one-pass partition), out[1] by Bitmap tree walks (Alg. 1), out[2] from the
 * Gram of the state bit-vectors, out[3] summed out of another query's
 * table (derive_tables).  out[0..3] add up to nq.  Errors as fc_count_batch.
 */
int fc_plan_summary(const fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                    int64_t nq, uint32_t flags, int64_t *out);

int fc_db_get_tuning(const fc_db *db, fc_tuning *t);

/* Validates and installs `t` (FC_ERR_INVALID on an out-of-range field). */
int fc_db_set_tuning(fc_db *db, const fc_tuning *t);

/*
 * Autotuner: times a representative batch (vars_flat/var_off as in
 * fc_count_batch) on the device with every candidate -- Bitmap against
 * histogram per (k, table-size bucket), the row-chunk sizes, then row
 * sweeps on or off -- and installs the fastest choices in the handle.
 * Choices that change only device work are compared by the summed
 * event-timed durations of the batch's kernel launches, the persistent
 * threshold and the strategy mix by wall time per batch.  Synchronises
 * `stream`.
 */
int fc_autotune(fc_db *db, const int32_t *vars_flat, const int64_t *var_off,
                int64_t nq, void *stream);

/*
 * Launch profiling (observability).  While enabled, the library brackets
 * every kernel launch with a pair of HIP events on the launch's stream and
 * attributes to it the algorithmic work it performs: bytes of state columns
 * a column scan must read (k bytes per query and instance) for counting
 * kernels, and m n (n + 1) matrix-core operations (2 per item pair and
 * instance over the upper triangle with the diagonal) for the co-occurrence
 * Gram.
 */
typedef struct fc_kernel_stat {
    char name[48];     /* kernel instance, e.g. "k_hist<3,1>"              */
    int64_t launches;  /* launches timed since the last reset              */
    double ms;         /* summed event-measured duration                   */
    double alg_bytes;  /* summed algorithmic bytes                         */
    double alg_ops;    /* summed algorithmic matrix-core operations        */
} fc_kernel_stat;

/* Turn launch profiling on (1) or off (0) for the whole process. */
int fc_profile_enable(int on);

/*
 * Synchronise the recorded events and write up to `cap` per-kernel
 * aggregates to `out`; returns the number of distinct kernels (which may
 * exceed cap) or a negative FC_ERR_* code.  reset != 0 clears the totals.
 */
int fc_profile_read(fc_kernel_stat *out, int32_t cap, int32_t reset);

/* Message of the last failed call on this host thread ("" if none). */
const char *fc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTCOUNT_H */
