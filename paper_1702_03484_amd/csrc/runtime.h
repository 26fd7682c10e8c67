// Host runtime of libmapsq: the context, the arena sub-allocator and the
// internal entry points shared by the plain, batched and serving paths.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mapsq.h"
#include "kernels.h"

namespace mq {

constexpr size_t ARENA_ALIGN = 256;
constexpr uint64_t SAT40_HOST = (1ull << 40) - 1ull;  // saturation cap of device row counts

// First-fit sub-allocator over the caller's arena.  All users of a context
// enqueue on one stream, so a block freed on the host can be handed out
// again at once: later work on the stream runs after earlier work.
class Arena {
   public:
    void init(char* base, size_t size);
    // returns offset or SIZE_MAX
    size_t alloc(size_t bytes);
    void free(size_t off);
    // shrink an allocated block to `bytes` (returns the tail to the free list)
    void shrink(size_t off, size_t bytes);
    char* ptr(size_t off) const { return base_ + off; }
    size_t free_bytes() const;
    size_t largest() const;
    // size of the allocated block at `off` (0 if none)
    size_t block_size(size_t off) const {
        auto it = used_.find(off);
        return it == used_.end() ? 0 : it->second;
    }
    char* base() const { return base_; }
    size_t size() const { return size_; }
    // Fault injection: when >= 0, each allocation counts it down and the one
    // that finds it at 0 fails as if the arena were full (then it is -1).
    int64_t fail_after = -1;

   private:
    char* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;           // offset -> size
    std::unordered_map<size_t, size_t> used_;  // offset -> size
};

struct Ctx;
struct Server;

// A block of the arena freed when the guard goes out of scope (unless released).
struct Block {
    Ctx* ctx = nullptr;
    size_t off = SIZE_MAX;
    Block() = default;
    Block(const Block&) = delete;
    Block& operator=(const Block&) = delete;
    Block(Block&& o) noexcept : ctx(o.ctx), off(o.off) { o.off = SIZE_MAX; }
    Block& operator=(Block&& o) noexcept {
        if (this != &o) {
            reset();
            ctx = o.ctx;
            off = o.off;
            o.off = SIZE_MAX;
        }
        return *this;
    }
    ~Block() { reset(); }
    void reset();
    bool ok() const { return off != SIZE_MAX; }
    template <typename T>
    T* as() const;
    size_t release() {
        size_t o = off;
        off = SIZE_MAX;
        return o;
    }
};

struct Store {
    bool loaded = false;
    int64_t n = 0;
    int32_t max_id = 0;
    int32_t id_bits = 0;
    int32_t *s = nullptr, *p = nullptr, *o = nullptr;            // raw SoA
    int32_t *pso_s = nullptr, *pso_o = nullptr;                  // sorted by (p, s, o)
    int32_t *pos_o = nullptr, *pos_s = nullptr;                  // sorted by (p, o, s)
    std::vector<int32_t> preds;                                  // distinct predicates, ascending
    std::vector<int64_t> pred_off;                               // preds.size() + 1 offsets
    std::vector<int64_t> pred_ds, pred_do;                       // distinct subjects / objects per predicate
    std::vector<size_t> blocks;
    uint64_t bytes = 0;
};

// The term dictionary of a context (mapsq_dict_*): arena blocks holding the
// hash table, the offsets and the bytes of the terms in identifier order.
struct Dict {
    bool made = false;
    int64_t cap_terms = 0, cap_bytes = 0;
    size_t table_off = SIZE_MAX, off_off = SIZE_MAX, bytes_off = SIZE_MAX;
    uint64_t* table = nullptr;
    uint64_t slots = 0;  // a power of two above 2 * cap_terms
    int64_t* off = nullptr;
    uint8_t* bytes = nullptr;
    int64_t nterms = 0, nbytes = 0;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    std::string err;
    Store store;
    // persistent look-back status words (epoch-tagged, never cleared between uses)
    size_t status_off = SIZE_MAX;
    uint64_t* status = nullptr;
    size_t status_words = 0;
    uint32_t epoch = 0;
    // small per-call device area: counters, histograms and scalars
    size_t small_off = SIZE_MAX;
    uint32_t* small = nullptr;
    // pinned host staging for read-backs
    void* pinned = nullptr;
    int32_t tune_rb = 0, tune_kpt = 0;
    int32_t semijoin = 0;    // 0 automatic, 1 never, 2 always
    int32_t merge_mode = 0;  // 0 merge join of key-sorted tables, 1 never
    int32_t precount = 0;    // exact |RS| before shuffles: 0 of 2^24+ records, 1 never, 2 always
    // The caller's estimate of the next join's output rows (the planner's and
    // the server's plans set it; < 0: none), read and cleared by join_tables:
    // in automatic mode the exact pre-count is skipped when the output at
    // that size would take at most 1/8 of the arena's free space.
    double join_est_rows = -1.0;
    int32_t composite = 0;   // 0 a second shared variable joins as part of the key, 1 it is filtered
    int32_t planner = 0;     // mapsq_query join order: 0 pattern sizes, 1 exact join sizes
    // join_tables stops once the exact |RS| is known (nrows set, no columns)
    bool count_only = false;
    // the plan mapsq_query ran last: start pattern, then each join step
    std::vector<mapsq_plan_step> last_plan;
    // autotuned choices: (key bits << 8 | log2 records) -> (rb << 8 | kpt)
    std::map<uint32_t, uint32_t> tuned;
    // materialisation grid cap: explicit (0: automatic), and autotuned by
    // log2 of the output rows
    int32_t tune_mat_blocks = 0;
    std::map<uint32_t, uint32_t> mat_tuned;
    uint32_t mat_blocks(uint64_t rows) const;
    mapsq_join_stats last{};
    // profiling: pairs of events around phases, harvested after a sync
    bool prof = false;
    struct Interval {
        hipEvent_t a, b;
        int phase;
        double bytes;
    };
    std::vector<Interval> pending;
    std::vector<hipEvent_t> event_pool;
    mapsq_profile acc{};
    // tables of one batch share an arena block: offset -> tables still alive
    std::unordered_map<size_t, uint32_t> shared_refs;
    // batched joins: a fixed device header (so captured graphs can be
    // replayed), pinned staging for descriptor uploads, cached graphs
    size_t bhdr_off = SIZE_MAX;
    BatchHdr* bhdr = nullptr;
    void* stage = nullptr;
    size_t stage_bytes = 0;
    std::map<uint64_t, hipGraphExec_t> graphs;
    bool use_graph = true;
    void release_graphs();
    // serving scheduler (created on first use)
    Server* server = nullptr;
    Dict dict;
    // When set, the next join result is written to these caller-owned
    // columns (out_cap rows each) instead of an arena table.
    int32_t* const* out_cols = nullptr;
    int64_t out_cap = 0;
    // returns an interval handle (-1 when profiling is off)
    int prof_begin(int phase);
    void prof_end(int h, double bytes);
    void prof_harvest();  // caller has synchronised the stream
    void prof_release();

    mapsq_status fail(mapsq_status code, const std::string& msg) {
        err = msg;
        return code;
    }
    // make sure the status array holds `words` words; returns false on CAPACITY
    bool ensure_status(size_t words);
    uint32_t next_epoch();
};

// layout of the small device area (u32 words)
// automatic semi-join reduction: the larger side has at least this many
// records and SEMI_RATIO times the smaller side's, and the key bitmap is no
// larger than the larger side's key column
constexpr uint32_t SEMI_MIN_RECORDS = 1u << 16;
constexpr uint64_t SEMI_RATIO = 4;
// exact output size before the shuffle of at least this many records, when
// the key range needs at most PRECOUNT_MAX_RANGE counters
constexpr uint64_t PRECOUNT_MIN_RECORDS = uint64_t(1) << 24;
constexpr uint64_t PRECOUNT_MAX_RANGE = uint64_t(1) << 28;
// a count-only join of two key-sorted tables whose smaller side has at
// least this many rows counts densely instead of merging
constexpr uint32_t COUNT_DENSE_MIN = 1u << 16;
// materialisation with one 256-row sub-chunk per wave when the output has
// fewer rows than this per segment on average (per-row segment searches)
constexpr uint64_t SPARSE_ROWS_PER_SEG = 64;

constexpr size_t SMALL_HIST = 0;                  // up to 8 passes x 2048 buckets
constexpr size_t SMALL_HIST_WORDS = 8 * 2048;
constexpr size_t SMALL_CTR = SMALL_HIST + SMALL_HIST_WORDS;  // 32 tile counters
constexpr size_t SMALL_SCALARS = SMALL_CTR + 32;             // 64 words of device scalars
constexpr size_t SMALL_WORDS = SMALL_SCALARS + 64;

template <typename T>
T* Block::as() const {
    return reinterpret_cast<T*>(ctx->arena.ptr(off));
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int bitlen(uint64_t v) {
    int b = 0;
    while (v) {
        b++;
        v >>= 1;
    }
    return b;
}

// internal entry points (return mapsq_status, set ctx->err)
mapsq_status join_tables(Ctx* ctx, const mapsq_table* L, const mapsq_table* R, int32_t key_var, mapsq_table* out);
mapsq_status map_pattern(Ctx* ctx, const mapsq_pattern* pat, int32_t key_var, mapsq_table* out);
// mapsq_join_into (noalloc.hip): the scratch array's address on the current
// device, looked up once per device; the join into caller columns
mapsq_status join_into_setup(int device);
mapsq_status join_into(Ctx* ctx, const mapsq_table* L, const mapsq_table* R, int32_t key_var,
                       int32_t* const* out_cols, int64_t out_capacity, mapsq_table* out);
// The plan of one pattern's map: which rows of the store to read and, for a
// scan, which equality tests to apply (set up by map_plan together with the
// output table's metadata).
struct MapPlan {
    bool empty = false;                        // the predicate does not occur
    int64_t lo = 0, rows = 0;                  // rows [lo, lo + rows) of the source columns
    const int32_t* col[3] = {nullptr, nullptr, nullptr};  // source of s, p, o (p is null on an index)
    int src_pos[MAPSQ_MAX_COLS] = {};          // output column c comes from position src_pos[c]
    int nterm = 0;                             // 0: the range itself is the answer (a view)
    int32_t ta[6] = {}, tb[6] = {}, tc[6] = {};  // tests: pos ta == constant tc (tb < 0) or == pos tb
};
mapsq_status map_plan(Ctx* ctx, const mapsq_pattern* pat, int32_t key_var, mapsq_table* out, MapPlan* mp);
CompactArgs map_scan_args(const MapPlan& mp, int ncols, int32_t* const* out_cols, uint64_t* count);
double map_test_bytes(const MapPlan& mp);
mapsq_status free_table(Ctx* ctx, mapsq_table* t);
// an owned table of rows x ncols in one arena block (CAPACITY when it does not fit)
mapsq_status alloc_table(Ctx* ctx, int64_t rows, int ncols, mapsq_table* t);
mapsq_status load_triples(Ctx* ctx, const int32_t* s, const int32_t* p, const int32_t* o, int64_t n,
                          uint32_t flags);
mapsq_status query(Ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                   mapsq_table* out);
// per_join == nullptr: any failing join fails the whole batch.  Otherwise a
// join that fails leaves its status there (and a zeroed table) while the
// others complete, and need_rows (if given) gets each failed join's exact
// output row count when it was counted (0 otherwise).
mapsq_status join_batch(Ctx* ctx, const mapsq_join_desc* d, int32_t n, mapsq_table* outs,
                        mapsq_status* per_join = nullptr, int64_t* need_rows = nullptr);
struct PlanStep {
    int pick;     // table joined at this step
    int32_t key;  // join variable (-1 for a cross product)
    bool cross;
};
void greedy_plan(const std::vector<std::vector<int32_t>>& vars, const std::vector<int64_t>& rows,
                 const std::vector<int32_t>& qvars, int* start, std::vector<PlanStep>* steps);
mapsq_status cross_join(Ctx* ctx, const mapsq_table& a, const mapsq_table& b, mapsq_table* out);
mapsq_table project_table(const mapsq_table& cur, const std::vector<int32_t>& want);
mapsq_status key_sort_views(Ctx* ctx, const mapsq_pattern* pats, mapsq_table* tabs, int start,
                            const std::vector<PlanStep>& steps);
// System-R estimates of a plan's step outputs (rows), from the patterns'
// partial-match sizes and the store's per-predicate distinct subjects and
// objects; *scan_bytes (if given) gets the bytes the plan's scans write.
std::vector<double> estimate_steps(const Ctx* ctx, const mapsq_pattern* pats, const std::vector<int64_t>& rows,
                                   int start, const std::vector<PlanStep>& steps, double* scan_bytes = nullptr,
                                   std::vector<size_t>* out_cols = nullptr);
bool ensure_stage(Ctx* ctx, size_t bytes);
// [lo, hi) of each index lookup (2 int64 per query in out); one synchronisation
mapsq_status locate_ranges(Ctx* ctx, const LocateQuery* q, size_t n, int64_t* out);
// term dictionary (dict.cpp)
mapsq_status dict_create(Ctx* ctx, int64_t max_terms, int64_t max_bytes);
mapsq_status dict_encode(Ctx* ctx, const uint8_t* bytes, const int64_t* offsets, int64_t n, uint32_t flags,
                         int32_t* ids, int64_t* n_new);
mapsq_status dict_decode(Ctx* ctx, const int32_t* ids, int64_t n, uint32_t flags, int64_t* offsets, uint8_t* bytes,
                         int64_t cap_bytes, int64_t* need_bytes);
void dict_release(Ctx* ctx);
// serving (serve.cpp)
mapsq_status serve_config(Ctx* ctx, uint64_t budget_bytes, int32_t max_active);
mapsq_status submit(Ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                    uint64_t* ticket);
mapsq_status serve_step(Ctx* ctx, int32_t* n_active, int32_t* n_waiting);
mapsq_status poll(Ctx* ctx, uint64_t ticket, int32_t* done, mapsq_table* out);
mapsq_status poll_next(Ctx* ctx, uint64_t* ticket, int32_t* done, mapsq_table* out);
void destroy_server(Ctx* ctx);
mapsq_status query_vars(Ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                        std::vector<int32_t>* qvars, std::vector<int32_t>* want);
mapsq_status check_table(Ctx* ctx, const mapsq_table* t, const char* name);
void pick_tuning(Ctx* ctx, int key_bits, int& rb, int& kpt, uint64_t nrec = 0);
int col_of(const mapsq_table* t, int32_t v);
Block alloc_block(Ctx* ctx, size_t bytes);

}  // namespace mq

struct mapsq_ctx {
    mq::Ctx impl;
};
