/*
 * mapsq.h -- C ABI of libmapsq.so, an MI355X (gfx950) implementation of the
 * MapReduce-based join of MapSQ (Feng, Zhang and Feng, "MapSQ: A
 * MapReduce-based Framework for SPARQL Queries on GPU", arXiv 1702.03484).
 *
 * What the library computes
 *   Section 1 of the paper: every triple pattern of a SPARQL basic graph
 *   pattern yields a table of partial matches whose key is the variable it
 *   shares with another pattern and whose value is its other variables; the
 *   answer is the join of those tables (Table 1).  Section 2, Algorithm 1:
 *   the join runs as Map (emit key/value records labelled LEFT or RIGHT),
 *   Sort (group by key) and ReduceDuplicate (per key, pair every LEFT record
 *   with every RIGHT record).  Section 2, text after Algorithm 1: results are
 *   merged pattern by pattern on one shared variable; the CPU assigns the
 *   subqueries and the GPU joins them (abstract).
 *
 * Conventions
 *   - Every call returns a mapsq_status; 0 is success, negative values are
 *     errors.  The message of the last error of a context is returned by
 *     mapsq_last_error().  No C++ exception crosses this boundary.
 *   - Arguments are checked before any GPU work is enqueued.  On error every
 *     output struct is zeroed and nothing the library owns is left
 *     half-written.
 *   - Terms of a triple pattern: a value >= 0 is a constant (a dictionary
 *     ID); a value < 0 is the variable number -t-1 (so -1 is variable 0).
 *     IDs must lie in [0, 2^31 - 1).
 *   - Tables are SoA: column c holds nrows int32 values in device memory and
 *     carries the variable var[c].  A join's result has the columns
 *     [key, left's other variables in left order, right's variables that the
 *     left does not bind, in right order], as in Table 1(c).  Row order is
 *     deterministic but not part of the result's meaning.
 *   - Bag semantics: every matching triple, and every pair of matching rows,
 *     gives one row; nothing is de-duplicated unless MAPSQ_LOAD_DEDUP asks
 *     for set semantics at load time.
 *
 * Memory and streams
 *   The caller owns all device memory.  mapsq_create() receives one device
 *   arena (for instance a torch uint8 tensor) and a hipStream_t; the library
 *   sub-allocates the store, its scratch buffers and result tables inside
 *   that arena and never calls hipMalloc.  Host-side bookkeeping is the only
 *   host allocation.  All GPU work of a context is enqueued on its stream.
 *   A context is externally synchronised: one thread at a time per context.
 *   Several contexts may share a device.
 */
#ifndef MAPSQ_H
#define MAPSQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mapsq_status;

#define MAPSQ_OK 0
#define MAPSQ_ERR_INVALID_ARG (-1) /* a pointer, size or term is invalid */
#define MAPSQ_ERR_UNSUPPORTED (-2) /* valid but not supported (e.g. a pattern with no variable) */
#define MAPSQ_ERR_CAPACITY (-3)    /* the arena has no room for the request */
#define MAPSQ_ERR_TOO_LARGE (-4)   /* the exact result exceeds the arena or 2^40 rows */
#define MAPSQ_ERR_HIP (-5)         /* a HIP runtime call failed */
#define MAPSQ_ERR_STATE (-6)       /* call out of order (e.g. no store loaded) */

#define MAPSQ_MAX_COLS 16

/* mapsq_load_triples flags */
#define MAPSQ_LOAD_DEVICE_PTRS 1u /* s, p, o are device pointers (else host pointers) */
#define MAPSQ_LOAD_DEDUP 2u       /* drop repeated triples (RDF set semantics) */

typedef struct mapsq_ctx mapsq_ctx; /* opaque */

/* A triple pattern (Section 1): each term a constant ID (>= 0) or a variable (< 0). */
typedef struct {
    int32_t s, p, o;
} mapsq_pattern;

/* A binding table in device memory (SoA int32 columns). */
typedef struct {
    int64_t nrows;
    int32_t ncols;
    int32_t owned;              /* 1: columns live in the context arena; release with mapsq_table_free.
                                   0: a view (of the loaded store, or caller-owned columns). */
    int32_t var[MAPSQ_MAX_COLS];/* variable number of each column */
    int32_t* col[MAPSQ_MAX_COLS];/* device pointer of each column */
    uint64_t block;             /* library bookkeeping (arena block id); 0 for views */
    int32_t key_max;            /* upper bound of the IDs in the table, -1 if unknown */
    int32_t sorted_col;         /* 1 + a column whose values ascend over the rows, 0 if none is known.
                                   Set by the library on index views (the index's next sort column)
                                   and on join results (column 0, the key).  A caller that sets it on
                                   its own table asserts that order; mapsq_join then pairs the two
                                   tables' key runs directly when both are sorted on the key (a wrong
                                   claim gives wrong rows, never an out-of-range access). */
} mapsq_table;

/* Facts about the loaded store. */
typedef struct {
    int64_t n_triples;
    int64_t n_predicates;  /* distinct predicate IDs */
    int32_t max_id;        /* largest ID over s, p, o */
    int32_t id_bits;       /* bit length of max_id */
    uint64_t device_bytes; /* arena bytes held by the store and its indexes */
} mapsq_store_facts;

/* What the last join of a context did (filled by mapsq_join and mapsq_query;
 * after a mapsq_join_batch that ran joins in the batched kernels, the sums
 * over those joins, path MAPSQ_PATH_SEMIJOIN when any of them was filtered). */
typedef struct {
    int64_t left_rows, right_rows;
    int64_t segments;      /* distinct keys among the |L|+|R| sorted records */
    int64_t out_rows;      /* exact |RS| = sum over keys of cL * cR (before equality filters) */
    int32_t radix_bits;    /* digit width of the sort */
    int32_t passes;        /* radix passes */
    int32_t key_bits;      /* bits sorted */
    int32_t path;          /* MAPSQ_PATH_*: how the records were grouped by key */
    int64_t sorted_records; /* records that went through the shuffle (0 for a merge join) */
} mapsq_join_stats;

#define MAPSQ_PATH_SORT 0     /* LSD radix sort of both sides' records */
#define MAPSQ_PATH_SEMIJOIN 1 /* the same after the semi-join reduction of the larger side */
#define MAPSQ_PATH_MERGE 2    /* both sides already sorted on the key: runs paired directly */
#define MAPSQ_PATH_COMPOSITE 3 /* radix sort on a composite key of two shared variables */

/* Create a context on `device`.  `arena` is device memory of `arena_bytes`
 * bytes owned by the caller and kept alive until mapsq_destroy; it must be
 * 256-byte aligned.  `hip_stream` is a hipStream_t (NULL = the null stream).
 * Returns INVALID_ARG for a NULL out/arena, a misaligned arena or fewer than
 * 64 MiB; HIP when the device cannot be selected. */
mapsq_status mapsq_create(int device, void* arena, size_t arena_bytes, void* hip_stream, mapsq_ctx** out);

/* Destroy a context (synchronises its stream first).  NULL is accepted. */
mapsq_status mapsq_destroy(mapsq_ctx* ctx);

/* Message of the last error of `ctx` ("" if none); valid until the next call. */
const char* mapsq_last_error(const mapsq_ctx* ctx);

/* Load a dictionary-encoded store of n triples (s[i], p[i], o[i]) and build
 * its indexes: the raw SoA columns, a copy sorted by (p, s, o) and one
 * sorted by (p, o, s), with the predicate ranges.  Replaces any store loaded
 * before (tables that view the old store become invalid).  s, p, o are host
 * pointers unless MAPSQ_LOAD_DEVICE_PTRS is set; the library copies them
 * and the caller keeps ownership.  INVALID_ARG for n < 0, NULL columns with
 * n > 0, n >= 2^31 or an ID outside [0, 2^31 - 1); CAPACITY when the arena
 * cannot hold 28 bytes per triple plus scratch.  Synchronises once. */
mapsq_status mapsq_load_triples(mapsq_ctx* ctx, const int32_t* s, const int32_t* p, const int32_t* o,
                                int64_t n, uint32_t flags);

mapsq_status mapsq_store_info(mapsq_ctx* ctx, mapsq_store_facts* out);

/* Statistics of one predicate of the loaded store (computed at load time
 * when the store has at most 4096 distinct predicates): its triples and its
 * distinct subjects and objects.  A predicate absent from the store gives
 * zeros.  UNSUPPORTED when the statistics were not computed. */
mapsq_status mapsq_predicate_stats(mapsq_ctx* ctx, int32_t predicate, int64_t* triples, int64_t* distinct_s,
                                   int64_t* distinct_o);

/* Map (Section 1 partial matches; Algorithm 1's Map): the table of matches
 * of one triple pattern, key variable `key_var` first (-1: no key, columns
 * in first-appearance order over s, p, o), then the other variables in
 * first-appearance order.  Constants are not materialised.  A pattern whose
 * constants form a prefix of one index order and that has no repeated
 * variable returns a view of the store (owned = 0); any other pattern is
 * scanned and compacted into an owned table.  UNSUPPORTED for a pattern
 * without variables; STATE without a store.  Synchronises once. */
mapsq_status mapsq_map_pattern(mapsq_ctx* ctx, const mapsq_pattern* pattern, int32_t key_var, mapsq_table* out);

/* Join (Algorithm 1): RS = left JOIN right on variable `key_var`, which both
 * tables must bind.  When both tables bind a further variable, the join is
 * on the composite key (key_var, k2), k2 being the first such variable in
 * the left table's column order: the records are sorted on both variables
 * (as one packed word when their two ranges fit 32 bits, else on k2 and
 * then stably on key_var) and only pairs that agree on both meet, so the
 * result is the natural join and right's copy of k2 is never materialised
 * (stats path MAPSQ_PATH_COMPOSITE; mapsq_set_join_options can ask for the
 * single-variable join plus an equality filter instead).  Any third shared
 * variable is filtered for equality after the join.  Tables may be views, owned results or
 * caller-owned columns (owned = 0, key_max = bound or -1).  Each side may
 * hold at most 2^31 - 1 rows.  TOO_LARGE when |RS| exceeds the arena's free
 * space or 2^40 rows (nothing is allocated then).  Enqueues the sort and the
 * counting, synchronises once to read the exact |RS|, then enqueues the
 * materialisation and returns without waiting for it. */
mapsq_status mapsq_join(mapsq_ctx* ctx, const mapsq_table* left, const mapsq_table* right, int32_t key_var,
                        mapsq_table* out);

/* Join into caller memory, allocating nothing: for callers that cannot
 * allocate device memory at call time (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The same join as
 * mapsq_join -- the same rows in the same order -- except
 * that the result is written to the caller's columns out_cols[0 ..
 * left->ncols + right->ncols - 2], each a device array of out_capacity
 * int32 values owned by the caller, in the column order of mapsq_join, and
 * that every scratch buffer comes from a fixed device array of the library
 * (MAPSQ_JOIN_INTO_SCRATCH_BYTES per device, held from the first context on
 * the device until the process ends) instead of the context's arena.  No
 * device memory is allocated and the arena is not touched.  On success *out
 * is a view (owned = 0) of out_cols with the exact row count.
 * Limits and errors: at most MAPSQ_JOIN_INTO_MAX_RECORDS rows over both
 * tables (else CAPACITY); the tables share only the key variable (else
 * UNSUPPORTED); TOO_LARGE when |RS| exceeds out_capacity (the exact count
 * is then in mapsq_last_join_stats().out_rows); INVALID_ARG for null
 * output columns when out_capacity > 0.  All calls on one device share the
 * scratch array: calls that overlap on one device (several host threads,
 * or contexts on different streams without ordering) race.  Like
 * mapsq_join, it synchronises once and returns with the materialisation
 * enqueued on the context's stream. */
#define MAPSQ_JOIN_INTO_SCRATCH_BYTES (64ull << 20)
#define MAPSQ_JOIN_INTO_MAX_RECORDS (1ull << 21)
mapsq_status mapsq_join_into(mapsq_ctx* ctx, const mapsq_table* left, const mapsq_table* right, int32_t key_var,
                             int32_t* const* out_cols, int64_t out_capacity, mapsq_table* out);

/* Query (Section 2: pattern-by-pattern merging, CPU plans, GPU joins): the
 * bag of solutions of the basic graph pattern pats[0..npats), projected on
 * select_vars[0..nselect) in that order (nselect = 0: every variable, in
 * first-appearance order).  The host maps every pattern, then joins greedily
 * from the smallest partial-match table, always taking the smallest table
 * connected to the bound variables; further shared variables are filtered
 * by equality; an unconnected pattern joins by cross product.
 * Intermediate tables are freed; the result is owned. */
mapsq_status mapsq_query(mapsq_ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* select_vars,
                         int32_t nselect, mapsq_table* out);

/* Join order of mapsq_query (the host's share of the CPU/GPU split: the
 * CPU assigns the subqueries, the GPU joins them; abstract and Section 2).
 * MAPSQ_PLAN_SIZES (the default): greedy on the exact partial-match sizes
 * -- start from the smallest table, then take the smallest table that
 * shares a variable with the bound ones.  MAPSQ_PLAN_EXACT: greedy on exact
 * join sizes counted on the GPU -- the first join is the pair of connected
 * tables with the smallest exact |RS|, and every later step joins the
 * connected table whose exact |RS| with the running result is smallest;
 * each candidate is counted by the join's own path up to the exact count
 * (a merge of key runs for index views in key order, dense per-key counts
 * where the key range allows, else sort and count), without writing rows.
 * Ties go to the lowest pattern index.  A table that shares nothing joins
 * by cross product last.  Both give the same bag.  The serving loop plans
 * with MAPSQ_PLAN_SIZES (it sizes queries before running them).
 * INVALID_ARG for another mode. */
#define MAPSQ_PLAN_SIZES 0
#define MAPSQ_PLAN_EXACT 1
mapsq_status mapsq_set_planner(mapsq_ctx* ctx, int32_t mode);

/* One step of the plan mapsq_query ran: step 0 is the start pattern (its
 * partial-match rows, key_var -1); step k >= 1 joins pattern `pattern` on
 * key_var (-1 for a cross product) and gives `rows` rows; `candidates` is
 * the number of join sizes counted on the GPU to choose it (0 when the plan
 * came from pattern sizes). */
typedef struct {
    int32_t pattern;
    int32_t key_var;
    int64_t rows;
    int32_t candidates;
    int32_t reserved;
} mapsq_plan_step;

/* The plan of the context's last successful mapsq_query: its steps are
 * copied to out[0 .. min(n, cap)) and *n is set to the step count (the
 * number of patterns).  STATE when no query has completed. */
mapsq_status mapsq_last_plan(mapsq_ctx* ctx, mapsq_plan_step* out, int32_t cap, int32_t* n);

/* One join of a batch: left JOIN right on key_var (see mapsq_join). */
typedef struct {
    const mapsq_table* left;
    const mapsq_table* right;
    int32_t key_var;
    int32_t reserved;
} mapsq_join_desc;

/* Batched joins (the batched form of Algorithm 1): the n independent joins
 * run together as one captured hipGraph launch (radix passes, counting,
 * device-side placement of every result in one output region and the
 * materialisation), then the stream is synchronised once and outs[i] is
 * filled.  Each join's result equals what mapsq_join returns for it, row for
 * row.  Semi-join reduction (mapsq_set_join_options' semijoin: automatic
 * when a join's larger side has at least twice the smaller side's rows):
 * a blocked Bloom filter of the smaller side's keys (16 bits per row) drops
 * the larger side's records whose key it cannot hold before the sort; it
 * has no false negatives, so the rows and their order do not change.
 * Joins the batched kernels do not cover (more than 8 output columns
 * or a further shared variable) and results that do not fit the output
 * region run through the plain path afterwards.  The result tables of one
 * batch share an arena block that is released when the last of them is
 * freed.  On error every outs[i] is zeroed and nothing stays allocated.
 * The caller's tables must stay valid until the call returns. */
mapsq_status mapsq_join_batch(mapsq_ctx* ctx, const mapsq_join_desc* joins, int32_t n, mapsq_table* outs);

/* ---- serving: continuous batching over the resident store -------------
 * Queries are queued by mapsq_submit.  Each mapsq_serve_step is one
 * scheduling round: waiting queries get exact pattern sizes from the index
 * ranges and a predicted intermediate-byte cost (greedy plan, join sizes
 * estimated from per-predicate distinct counts); they are admitted in
 * arrival order while the predicted bytes of all admitted queries stay
 * within the budget, a later query that fits going ahead of one that does
 * not (at most 8 rounds in a row, then admission waits for the older one).
 * A query predicted above the whole budget reserves nothing: the exact size
 * of each of its joins decides.  Newly admitted queries map their patterns;
 * then the next join step of every admitted query runs: small steps
 * together in one batched launch, steps of 2^20 records or more and steps
 * whose inputs are already in key order through the plain join path.  A
 * step that finds no memory waits while other queries hold memory, unless
 * its exact output could not fit even if they let go of everything (free
 * space plus every block only they reference); while other queries wait to
 * be admitted it first frees what it holds and goes behind them (at most
 * twice), and after 8 rounds of waiting admission pauses until it runs.  A
 * step held up only by results not yet polled tries again next round; a
 * query alone whose own tables split the free space starts over once.  When
 * a round makes no progress at all, the most recently admitted waiting
 * query frees what it holds and is queued again at the head, and nothing is
 * admitted until some query ends.  A query fails with TOO_LARGE when a join
 * output cannot fit or an intermediate reaches 2^31 rows.  A query that
 * arrives while others are in flight joins the next round.  Each result is
 * exactly what mapsq_query returns for the query alone.  Serving calls use
 * the context like every other call: one thread at a time. */

/* Budget of predicted intermediate bytes (0: 60% of the arena's free space
 * at the first round) and the most queries in flight (0: 256). */
mapsq_status mapsq_serve_config(mapsq_ctx* ctx, uint64_t budget_bytes, int32_t max_active);

/* Queue a query (arguments as mapsq_query); *ticket identifies it. */
mapsq_status mapsq_submit(mapsq_ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* select_vars,
                          int32_t nselect, uint64_t* ticket);

/* One scheduling round (synchronises the stream once per batched launch);
 * reports the queries in flight and still waiting. */
mapsq_status mapsq_serve_step(mapsq_ctx* ctx, int32_t* active, int32_t* waiting);

/* *done = 0: still pending.  *done = 1 and OK: the result moves to *out (an
 * owned table or a view) and the ticket is retired.  *done = 1 and an error
 * status: the query failed with that status and the ticket is retired. */
mapsq_status mapsq_poll(mapsq_ctx* ctx, uint64_t ticket, int32_t* done, mapsq_table* out);

/* The next query to end, in the order queries ended (one call per finished
 * query instead of one per pending ticket).  *done = 0: none has ended that
 * is not yet retired (*ticket = 0).  *done = 1: *ticket names it and the
 * call returns what mapsq_poll(ctx, *ticket, ...) would: OK with the result
 * in *out, or the query's error status.  INVALID_ARG (with *ticket = 0) for
 * null outputs. */
mapsq_status mapsq_poll_next(mapsq_ctx* ctx, uint64_t* ticket, int32_t* done, mapsq_table* out);

/* ---- term dictionary --------------------------------------------------
 * Table 1 writes the example with string terms; the join works on their
 * identifiers.  A context holds one dictionary on the device that maps byte
 * strings to dense identifiers 0, 1, 2, ... in order of first appearance
 * and back: a batch of terms is hashed (FNV-1a, 64-bit) and inserted into an
 * open-addressing table with a 64-bit CAS per claimed slot, the first
 * occurrences of terms it did not hold are numbered in batch order after the
 * terms it held, and their bytes are appended to its byte store.  Encoding a
 * batch and then another gives the identifiers of encoding both at once.
 * Terms are arbitrary byte strings (no terminator; the empty string is a
 * term).  A batch is bytes plus n + 1 int64 offsets starting at 0 and never
 * decreasing: term i is bytes[offsets[i] .. offsets[i + 1]). */
#define MAPSQ_DICT_DEVICE_PTRS 1u /* every buffer of the call is device memory (else host) */
#define MAPSQ_DICT_LOOKUP 2u      /* encode without adding: an unknown term gives -1 */

/* (Re)create the context's dictionary, empty, with room for max_terms terms
 * (1 .. 2^30) and max_bytes bytes of term text (0 .. 2^40) in the arena:
 * 16 bytes per term of hash table and 8 of offsets, plus the text.  Drops
 * any dictionary the context had.  CAPACITY when the arena has no room. */
mapsq_status mapsq_dict_create(mapsq_ctx* ctx, int64_t max_terms, int64_t max_bytes);

/* Identifiers of a batch of n terms (n <= min(2^26, max_terms)), written to
 * ids[0 .. n) (int32).  Terms the dictionary lacks are added (unless
 * MAPSQ_DICT_LOOKUP) and *n_new (may be NULL) gets their number.
 * INVALID_ARG for bad offsets (checked before any byte is read); CAPACITY
 * when the new terms would exceed max_terms or max_bytes (the dictionary is
 * then left exactly as it was); STATE without a dictionary.  Synchronises. */
mapsq_status mapsq_dict_encode(mapsq_ctx* ctx, const uint8_t* bytes, const int64_t* offsets, int64_t n,
                               uint32_t flags, int32_t* ids, int64_t* n_new);

/* Terms of n identifiers (n <= 2^26): their bytes back to back in
 * bytes[0 .. need) and n + 1 offsets in offsets[] (starting at 0).  *need
 * (may be NULL) gets the byte count; TOO_LARGE when it exceeds cap_bytes
 * (nothing is written then); INVALID_ARG for an identifier outside
 * [0, terms).  Synchronises. */
mapsq_status mapsq_dict_decode(mapsq_ctx* ctx, const int32_t* ids, int64_t n, uint32_t flags, int64_t* offsets,
                               uint8_t* bytes, int64_t cap_bytes, int64_t* need);

/* Terms and bytes of text the dictionary holds (STATE without one). */
mapsq_status mapsq_dict_info(mapsq_ctx* ctx, int64_t* terms, int64_t* bytes);

/* Release an owned table (views are left alone); the struct is zeroed. */
mapsq_status mapsq_table_free(mapsq_ctx* ctx, mapsq_table* t);

/* Statistics of the most recent join of the context. */
mapsq_status mapsq_last_join_stats(mapsq_ctx* ctx, mapsq_join_stats* out);

/* Radix digit width (4..11 bits; 0 = automatic) and keys per thread of the
 * sort tiles (8 or 16; 0 = automatic: the autotuner table or 16 for
 * mapsq_join, 32 for mapsq_join_batch) used by later joins.  Every choice
 * gives the same rows in the same order. */
mapsq_status mapsq_set_tuning(mapsq_ctx* ctx, int32_t radix_bits, int32_t keys_per_thread);

/* How mapsq_join / mapsq_query group records by key; every choice of
 * semijoin, merge and precount gives the same rows in the same order (or the
 * same error); composite gives the same rows (the same bag).
 * semijoin: a record whose key the other side lacks meets no partner in
 *   Reduce (Algorithm 1), so it can be left out of the shuffle.  0 =
 *   automatic (the larger side has at least 2^16 records and 4 times the
 *   smaller side's, and the key bitmap is no larger than the larger side's
 *   key column), 1 = never, 2 = whenever the bitmap fits in 1 GiB.  In
 *   mapsq_join_batch (a Bloom filter per join): 0 = when the larger side
 *   has at least twice the smaller side's rows, 1 = never, 2 = every join.
 * merge: 0 = pair the key runs directly when both tables are sorted on the
 *   key (sorted_col), 1 = always shuffle.
 * precount: before a shuffle, count |RS| exactly from dense per-key counts
 *   (two passes over the keys), so that a join with no key in common, or
 *   whose result cannot fit in the arena, ends without sorting.  0 =
 *   automatic: shuffles of at least 2^24 records, except the join steps of
 *   mapsq_query and of the server whose planned output (the System-R
 *   estimate of the pattern-size plan, or the exact planner's count) would
 *   take at most 1/8 of the arena's free space; 1 = never, 2 = every
 *   shuffle.  Without it the same outcome comes after the sort.
 * composite: 0 = a second variable both tables bind is part of the join key
 *   (see mapsq_join), 1 = join on key_var alone and filter the second
 *   variable for equality afterwards (the larger intermediate the paper's
 *   one-variable merge implies).
 * INVALID_ARG for other values. */
mapsq_status mapsq_set_join_options(mapsq_ctx* ctx, int32_t semijoin, int32_t merge, int32_t precount,
                                    int32_t composite);

/* Per-phase device time and algorithmic bytes, accumulated while profiling
 * is on.  Phases: 0 map (range location and scan/compaction), 1 sort
 * (histogram and radix passes), 2 count (segment heads, LEFT/RIGHT split,
 * count and offset scan), 3 materialize, 4 equality filter, 5 index build.
 * Times come from hipEvents recorded on the context's stream around each
 * phase's launches; 6 is a whole batched launch (mapsq_join_batch); 7 is
 * the gather of value cells into sorted record order that precedes
 * materialisation when the result has at least as many rows as records;
 * 8 is the semi-join reduction (key bitmap and filtered records).  A merge
 * join's segment pass counts under 2 (count).
 * Algorithmic bytes are what each phase must move given
 * the exact sizes (formulas in the design notes of the repository). */
#define MAPSQ_NPHASES 9
typedef struct {
    double ms[MAPSQ_NPHASES];
    double bytes[MAPSQ_NPHASES];
    int64_t launches[MAPSQ_NPHASES]; /* timed intervals per phase */
    int64_t joins;
    int64_t rows_out;                /* sum of exact |RS| over the joins */
} mapsq_profile;

/* Turn profiling on (1) or off (0); either way the accumulators are reset. */
mapsq_status mapsq_profile_enable(mapsq_ctx* ctx, int32_t on);

/* Synchronise the context's stream and return the accumulators. */
mapsq_status mapsq_profile_read(mapsq_ctx* ctx, mapsq_profile* out);

/* Autotuner table: for sorts of keys of `key_bits` bits over about
 * 2^(log2_records-1) .. 2^log2_records records, use digit width `radix_bits`
 * (4..11) and `keys_per_thread` (8 or 16).  Consulted when no explicit
 * mapsq_set_tuning is in force.  radix_bits = 0 removes the entry. */
mapsq_status mapsq_tune_record(mapsq_ctx* ctx, int32_t key_bits, int32_t log2_records, int32_t radix_bits,
                               int32_t keys_per_thread);

/* Grid cap of the materialisation launches (their waves stride over the
 * output's work items): 64 .. 65536 blocks, or 0 for automatic (the
 * autotuned entry for the output's size class, else 8192).  Every choice
 * gives the same rows in the same order. */
mapsq_status mapsq_set_mat_tuning(mapsq_ctx* ctx, int32_t max_blocks);

/* Autotuner table of the materialisation grid cap: for outputs of about
 * 2^(log2_rows-1) .. 2^log2_rows rows use max_blocks (64 .. 65536);
 * max_blocks = 0 removes the entry. */
mapsq_status mapsq_tune_record_mat(mapsq_ctx* ctx, int32_t log2_rows, int32_t max_blocks);

/* Bytes of the arena still free, and the largest free block. */
mapsq_status mapsq_arena_free_bytes(mapsq_ctx* ctx, uint64_t* free_bytes, uint64_t* largest_block);

/* Fault injection for tests of the error paths: after `after` more arena
 * allocations of this context succeed, the next one fails as if the arena
 * were full (once; after < 0 disables).  The environment variable
 * MAPSQ_FAULT=alloc:N sets the same at mapsq_create.  Every call must then
 * end with its documented status (CAPACITY or TOO_LARGE for memory), free
 * everything it allocated, and leave the context usable. */
mapsq_status mapsq_debug_fail_alloc(mapsq_ctx* ctx, int64_t after);

#ifdef __cplusplus
}
#endif

#endif /* MAPSQ_H */
