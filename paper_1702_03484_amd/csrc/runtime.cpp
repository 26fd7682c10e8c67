// Host runtime of libmapsq: arena, store loading and indexing, the map of a
// triple pattern, and the plain join driver (Map -> Sort -> ReduceDuplicate
// of Algorithm 1, with one read-back of the exact output size per join).
#include "runtime.h"

#include <algorithm>
#include <climits>
#include <cstring>

namespace mq {

uint32_t Ctx::next_epoch() {
    if (++epoch >= (1u << 22)) {
        // every word of the status array is re-tagged as unpublished
        (void)launch_fill_u64(status, status_words, 0ull, stream);
        epoch = 1;
    }
    return epoch;
}

bool Ctx::ensure_status(size_t words) {
    if (words <= status_words) return true;
    size_t want = std::max(words, status_words * 3 / 2);
    size_t off = arena.alloc(want * 8);
    if (off == SIZE_MAX) {
        want = words;
        off = arena.alloc(want * 8);
        if (off == SIZE_MAX) return false;
    }
    if (status_off != SIZE_MAX) arena.free(status_off);
    status_off = off;
    status = reinterpret_cast<uint64_t*>(arena.ptr(off));
    status_words = want;
    (void)launch_fill_u64(status, want, 0ull, stream);
    return true;
}

int Ctx::prof_begin(int phase) {
    if (!prof) return -1;
    hipEvent_t ev[2];
    for (auto& e : ev) {
        if (!event_pool.empty()) {
            e = event_pool.back();
            event_pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            return -1;
        }
    }
    (void)hipEventRecord(ev[0], stream);
    pending.push_back(Interval{ev[0], ev[1], phase, 0.0});
    return (int)pending.size() - 1;
}

void Ctx::prof_end(int h, double bytes) {
    if (h < 0 || h >= (int)pending.size()) return;
    (void)hipEventRecord(pending[h].b, stream);
    pending[h].bytes = bytes;
}

void Ctx::prof_harvest() {
    for (auto& iv : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, iv.a, iv.b) == hipSuccess) {
            acc.ms[iv.phase] += ms;
            acc.bytes[iv.phase] += iv.bytes;
            acc.launches[iv.phase] += 1;
        }
        event_pool.push_back(iv.a);
        event_pool.push_back(iv.b);
    }
    pending.clear();
}

void Ctx::prof_release() {
    for (auto& iv : pending) {
        event_pool.push_back(iv.a);
        event_pool.push_back(iv.b);
    }
    pending.clear();
    for (auto e : event_pool) (void)hipEventDestroy(e);
    event_pool.clear();
}

#define HIPCHK(x)                                                                                     \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) return ctx->fail(MAPSQ_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static inline uint64_t* scalar64(Ctx* ctx, int word) {
    return reinterpret_cast<uint64_t*>(ctx->small + SMALL_SCALARS + word);
}
static inline uint32_t* scalar32(Ctx* ctx, int word) { return ctx->small + SMALL_SCALARS + word; }
static inline uint32_t* counter(Ctx* ctx, int i) { return ctx->small + SMALL_CTR + i; }

// scalar slots (u32 word index inside the scalar area)
enum { SC_NSEG = 0, SC_TOTAL = 2, SC_COUNT = 4, SC_MINMAX = 6, SC_BAD = 8, SC_NPRED = 9, SC_MINMAX2 = 10, SC_SEMI = 12, SC_PRECOUNT = 14, SC_MAXPAIRS = 16, SC_MINMAX3 = 18 };
// counter slots
enum { CT_PASS0 = 0, CT_COUNT = 9, CT_SEMI = 11 };

static mapsq_status readback(Ctx* ctx, const void* dev, size_t bytes, void* host) {
    HIPCHK(hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::memcpy(host, ctx->pinned, bytes);
    return MAPSQ_OK;
}

// ------------------------------------------------------------ radix sort ---

struct SortBufs {
    uint32_t* k[2];
    uint32_t* v[2];
};

uint32_t Ctx::mat_blocks(uint64_t rows) const {
    if (tune_mat_blocks) return (uint32_t)tune_mat_blocks;
    auto it = mat_tuned.find((uint32_t)bitlen(rows));
    return it == mat_tuned.end() ? 0u : it->second;
}

void pick_tuning(Ctx* ctx, int key_bits, int& rb, int& kpt, uint64_t nrec) {
    rb = ctx->tune_rb;
    kpt = ctx->tune_kpt;
    if (!rb && !kpt && nrec) {
        // an autotuned entry for this key width and size class
        auto it = ctx->tuned.find(((uint32_t)key_bits << 8) | (uint32_t)bitlen(nrec));
        if (it != ctx->tuned.end()) {
            rb = (int)(it->second >> 8);
            kpt = (int)(it->second & 0xff);
        }
    }
    if (!kpt) kpt = 16;
    if (!rb) {
        // fewest passes with digits of at most 8 bits, spread evenly
        int passes = std::max(1, (key_bits + 7) / 8);
        rb = std::max(4, (key_bits + passes - 1) / passes);
    }
}

// Sort n records.  src != nullptr: first pass reads keys from src and
// generates payloads; else the input sits in b.k[0], b.v[0].  Result buffer
// index in *res.  Zeroes the histogram and tile counters itself.
static mapsq_status radix_sort(Ctx* ctx, const SortSrc* src, uint32_t n, int key_bits, int rb, int kpt,
                               SortBufs& b, int* res, int* passes_out) {
    const int passes = std::max(1, (key_bits + rb - 1) / rb);
    *passes_out = passes;
    *res = 0;
    if (n == 0) return MAPSQ_OK;
    const size_t buckets = size_t(1) << rb;
    if (passes * buckets > SMALL_HIST_WORDS) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "radix digit width too small");
    if (!ctx->ensure_status(size_t(radix_tiles(n, kpt, rb, true)) * buckets))  // the most tiles of any pass
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for sort status words");
    HIPCHK(launch_fill_u32(ctx->small + SMALL_CTR, SMALL_SCALARS - SMALL_CTR, 0u, ctx->stream));
    SortSrc none{};
    Block part = alloc_block(ctx, size_t(radix_hist_part_words(rb, passes)) * 4);
    if (!part.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for histogram partials");
    HIPCHK(launch_radix_hist(src ? *src : none, src ? nullptr : b.k[0], n, rb, passes, part.as<uint32_t>(),
                             ctx->small + SMALL_HIST, ctx->stream));
    int cur = 0;
    for (int p = 0; p < passes; p++) {
        const bool gen = src && p == 0;
        int dst = gen ? 0 : 1 - cur;
        HIPCHK(launch_radix_pass(rb, kpt, gen ? *src : none, gen ? nullptr : b.k[cur], gen ? nullptr : b.v[cur],
                                 b.k[dst], b.v[dst], n, p, ctx->small + SMALL_HIST + p * buckets, ctx->status,
                                 counter(ctx, CT_PASS0 + p), ctx->next_epoch(), ctx->stream));
        cur = dst;
    }
    *res = cur;
    return MAPSQ_OK;
}

// --------------------------------------------------------- store loading ---

static void free_store(Ctx* ctx) {
    for (size_t off : ctx->store.blocks) ctx->arena.free(off);
    ctx->store = Store{};
}

// Sort the store by (p, first, second) with three stable LSD sorts (second,
// then first, then p - pmin) and gather the `first`/`second` columns in that
// order.  On return b.v[*res] holds the permutation (sorted position ->
// triple) and b.k[*res] the sorted p - pmin.
static mapsq_status build_order(Ctx* ctx, int64_t n, const int32_t* first, const int32_t* second, int32_t so_max,
                                int32_t pmin, int32_t pmax, SortBufs& b, int32_t* out_first, int32_t* out_second,
                                bool want_preds, int* res_out) {
    int rb, kpt, res, passes;
    const int so_bits = bitlen((uint32_t)so_max);
    const int p_bits = bitlen((uint32_t)(pmax - pmin));
    SortSrc src{second, (uint32_t)n, nullptr, 0, 0};
    pick_tuning(ctx, so_bits, rb, kpt);
    mapsq_status st = radix_sort(ctx, &src, (uint32_t)n, so_bits, rb, kpt, b, &res, &passes);
    if (st) return st;
    auto to_front = [&]() {
        if (res != 0) {
            std::swap(b.k[0], b.k[1]);
            std::swap(b.v[0], b.v[1]);
        }
    };
    to_front();
    // then by `first` (stable)
    HIPCHK(launch_gather(first, b.v[0], reinterpret_cast<int32_t*>(b.k[0]), n, 0, ctx->stream));
    st = radix_sort(ctx, nullptr, (uint32_t)n, so_bits, rb, kpt, b, &res, &passes);
    if (st) return st;
    to_front();
    // then by p - pmin (stable)
    HIPCHK(launch_gather(ctx->store.p, b.v[0], reinterpret_cast<int32_t*>(b.k[0]), n, pmin, ctx->stream));
    pick_tuning(ctx, p_bits, rb, kpt);
    st = radix_sort(ctx, nullptr, (uint32_t)n, p_bits, rb, kpt, b, &res, &passes);
    if (st) return st;
    *res_out = res;
    HIPCHK(launch_gather(first, b.v[res], out_first, n, 0, ctx->stream));
    HIPCHK(launch_gather(second, b.v[res], out_second, n, 0, ctx->stream));
    if (want_preds) {
        const uint32_t cap = (uint32_t)std::min<int64_t>(n, 1 << 22);
        Block vals = alloc_block(ctx, size_t(cap) * 4);
        Block pos = alloc_block(ctx, size_t(cap) * 8);
        if (!vals.ok() || !pos.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for predicate table");
        HIPCHK(launch_fill_u32(scalar32(ctx, SC_NPRED), 1, 0u, ctx->stream));
        HIPCHK(launch_run_bounds(reinterpret_cast<const int32_t*>(b.k[res]), n, vals.as<int32_t>(),
                                 pos.as<int64_t>(), scalar32(ctx, SC_NPRED), cap, ctx->stream));
        uint32_t np = 0;
        if ((st = readback(ctx, scalar32(ctx, SC_NPRED), 4, &np))) return st;
        if (np > cap) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 2^22 distinct predicates");
        std::vector<int32_t> pv(np);
        std::vector<int64_t> pp(np);
        HIPCHK(hipMemcpyAsync(pv.data(), vals.as<int32_t>(), size_t(np) * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(pp.data(), pos.as<int64_t>(), size_t(np) * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        std::vector<uint32_t> ord(np);
        for (uint32_t i = 0; i < np; i++) ord[i] = i;
        std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t c) { return pp[a] < pp[c]; });
        ctx->store.preds.resize(np);
        ctx->store.pred_off.resize(np + 1);
        for (uint32_t i = 0; i < np; i++) {
            ctx->store.preds[i] = pv[ord[i]] + pmin;
            ctx->store.pred_off[i] = pp[ord[i]];
        }
        ctx->store.pred_off[np] = n;
    }
    return MAPSQ_OK;
}

mapsq_status load_triples(Ctx* ctx, const int32_t* s, const int32_t* p, const int32_t* o, int64_t n,
                          uint32_t flags) {
    if (n < 0 || n >= (int64_t(1) << 31)) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "n must be in [0, 2^31)");
    if (n > 0 && (!s || !p || !o)) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null triple column");
    if (flags & ~(MAPSQ_LOAD_DEVICE_PTRS | MAPSQ_LOAD_DEDUP)) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "unknown flag");
    free_store(ctx);
    Store& S = ctx->store;
    const size_t cb = align_up(size_t(std::max<int64_t>(n, 1)) * 4, ARENA_ALIGN);
    auto take = [&](int32_t*& dst) -> bool {
        size_t off = ctx->arena.alloc(cb);
        if (off == SIZE_MAX) return false;
        S.blocks.push_back(off);
        dst = reinterpret_cast<int32_t*>(ctx->arena.ptr(off));
        S.bytes += cb;
        return true;
    };
    if (!take(S.s) || !take(S.p) || !take(S.o)) {
        free_store(ctx);
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the raw triples");
    }
    const hipMemcpyKind kind = (flags & MAPSQ_LOAD_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    mapsq_status st;
#define LCHK(x)                   \
    do {                          \
        st = (x);                 \
        if (st) {                 \
            free_store(ctx);      \
            return st;            \
        }                         \
    } while (0)
#define LHIP(x)                                                                                       \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) {                                                                       \
            free_store(ctx);                                                                          \
            return ctx->fail(MAPSQ_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));          \
        }                                                                                             \
    } while (0)
    if (n > 0) {
        LHIP(hipMemcpyAsync(S.s, s, size_t(n) * 4, kind, ctx->stream));
        LHIP(hipMemcpyAsync(S.p, p, size_t(n) * 4, kind, ctx->stream));
        LHIP(hipMemcpyAsync(S.o, o, size_t(n) * 4, kind, ctx->stream));
    }
    // ID range check and bounds
    {
        // words SC_MINMAX .. SC_MINMAX+5: min/max of s and o, bad-ID count, (unused), min/max of p
        int32_t init[6] = {INT32_MAX, INT32_MIN, 0, 0, INT32_MAX, INT32_MIN};
        static_assert(SC_BAD == SC_MINMAX + 2 && SC_MINMAX2 == SC_MINMAX + 4, "scalar layout");
        std::memcpy(ctx->pinned, init, sizeof(init));
        LHIP(hipMemcpyAsync(scalar32(ctx, SC_MINMAX), ctx->pinned, sizeof(init), hipMemcpyHostToDevice,
                            ctx->stream));
        LHIP(hipStreamSynchronize(ctx->stream));
    }
    LHIP(launch_check_ids(S.s, n, scalar32(ctx, SC_BAD), ctx->stream));
    LHIP(launch_check_ids(S.p, n, scalar32(ctx, SC_BAD), ctx->stream));
    LHIP(launch_check_ids(S.o, n, scalar32(ctx, SC_BAD), ctx->stream));
    LHIP(launch_minmax(S.s, n, S.o, n, reinterpret_cast<int32_t*>(scalar32(ctx, SC_MINMAX)), ctx->stream));
    LHIP(launch_minmax(S.p, n, nullptr, 0, reinterpret_cast<int32_t*>(scalar32(ctx, SC_MINMAX2)), ctx->stream));
    uint32_t sc[6];
    LCHK(readback(ctx, scalar32(ctx, SC_MINMAX), 24, sc));  // minmax(2), bad, npred, minmax2(2)
    if (sc[2] != 0) {
        free_store(ctx);
        return ctx->fail(MAPSQ_ERR_INVALID_ARG, "an ID lies outside [0, 2^31 - 1)");
    }
    int32_t so_max = n ? (int32_t)sc[1] : 0, pmin = n ? (int32_t)sc[4] : 0, pmax = n ? (int32_t)sc[5] : 0;
    S.n = n;
    S.max_id = std::max(so_max, pmax);
    S.id_bits = bitlen((uint32_t)S.max_id);

    // sort scratch: two key and two payload buffers
    Block sk0 = alloc_block(ctx, cb), sk1 = alloc_block(ctx, cb), sv0 = alloc_block(ctx, cb),
          sv1 = alloc_block(ctx, cb);
    if (!sk0.ok() || !sk1.ok() || !sv0.ok() || !sv1.ok()) {
        free_store(ctx);
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for index-build scratch");
    }
    SortBufs b{{sk0.as<uint32_t>(), sk1.as<uint32_t>()}, {sv0.as<uint32_t>(), sv1.as<uint32_t>()}};

    if ((flags & MAPSQ_LOAD_DEDUP) && n > 0) {
        // order by (p, s, o), flag the first triple of every run of equal
        // triples, and keep the flagged triples in input order
        Block t1 = alloc_block(ctx, cb), t2 = alloc_block(ctx, cb), keep = alloc_block(ctx, cb);
        Block ns = alloc_block(ctx, cb), np_ = alloc_block(ctx, cb), no = alloc_block(ctx, cb);
        if (!t1.ok() || !t2.ok() || !keep.ok() || !ns.ok() || !np_.ok() || !no.ok()) {
            free_store(ctx);
            return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for de-duplication");
        }
        int res = 0;
        LCHK(build_order(ctx, n, S.s, S.o, so_max, pmin, pmax, b, t1.as<int32_t>(), t2.as<int32_t>(), false, &res));
        LHIP(launch_dup_flags(reinterpret_cast<const int32_t*>(b.k[res]), t1.as<int32_t>(), t2.as<int32_t>(),
                              b.v[res], n, keep.as<int32_t>(), ctx->stream));
        CompactArgs c{};
        c.nin = 4;
        c.in[0] = S.s;
        c.in[1] = S.p;
        c.in[2] = S.o;
        c.in[3] = keep.as<int32_t>();
        c.n = (uint64_t)n;
        c.nterm = 1;
        c.term_a[0] = 3;
        c.term_b[0] = -1;
        c.term_c[0] = 1;
        c.nout = 3;
        for (int i = 0; i < 3; i++) c.out_src[i] = i;
        c.out[0] = ns.as<int32_t>();
        c.out[1] = np_.as<int32_t>();
        c.out[2] = no.as<int32_t>();
        c.count = scalar64(ctx, SC_COUNT);
        Block cs = alloc_block(ctx, compact_scratch_words((uint64_t)n) * 8);
        if (!cs.ok()) {
            free_store(ctx);
            return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for de-duplication");
        }
        LHIP(launch_fill_u32(scalar32(ctx, SC_COUNT), 2, 0u, ctx->stream));
        LHIP(launch_compact(c, cs.as<uint64_t>(), ctx->stream));
        uint64_t kept = 0;
        LCHK(readback(ctx, scalar64(ctx, SC_COUNT), 8, &kept));
        LHIP(hipMemcpyAsync(S.s, ns.as<int32_t>(), kept * 4, hipMemcpyDeviceToDevice, ctx->stream));
        LHIP(hipMemcpyAsync(S.p, np_.as<int32_t>(), kept * 4, hipMemcpyDeviceToDevice, ctx->stream));
        LHIP(hipMemcpyAsync(S.o, no.as<int32_t>(), kept * 4, hipMemcpyDeviceToDevice, ctx->stream));
        n = (int64_t)kept;
        S.n = n;
    }

    if (!take(S.pso_s) || !take(S.pso_o) || !take(S.pos_o) || !take(S.pos_s)) {
        free_store(ctx);
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the PSO/POS indexes");
    }
    if (n > 0) {
        int res = 0;
        int ph = ctx->prof_begin(5);
        LCHK(build_order(ctx, n, S.s, S.o, so_max, pmin, pmax, b, S.pso_s, S.pso_o, true, &res));
        LCHK(build_order(ctx, n, S.o, S.s, so_max, pmin, pmax, b, S.pos_o, S.pos_s, false, &res));
        ctx->prof_end(ph, 0.0);
    }
    // per-predicate statistics for the planner's size estimates: distinct
    // subjects (runs in the PSO subject column) and objects (POS object column)
    if (n > 0 && S.preds.size() <= 4096) {
        const size_t np = S.preds.size();
        Block cnt = alloc_block(ctx, np * 16);
        if (!cnt.ok()) {
            free_store(ctx);
            return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for predicate statistics");
        }
        unsigned long long* c = cnt.as<unsigned long long>();
        LHIP(launch_fill_u64(reinterpret_cast<uint64_t*>(c), np * 2, 0ull, ctx->stream));
        for (size_t i = 0; i < np; i++) {
            LHIP(launch_count_runs(S.pso_s, S.pred_off[i], S.pred_off[i + 1], c + i, ctx->stream));
            LHIP(launch_count_runs(S.pos_o, S.pred_off[i], S.pred_off[i + 1], c + np + i, ctx->stream));
        }
        std::vector<int64_t> h(np * 2);
        LHIP(hipMemcpyAsync(h.data(), c, np * 16, hipMemcpyDeviceToHost, ctx->stream));
        LHIP(hipStreamSynchronize(ctx->stream));
        S.pred_ds.assign(h.begin(), h.begin() + np);
        S.pred_do.assign(h.begin() + np, h.end());
    }
    LHIP(hipStreamSynchronize(ctx->stream));
    S.loaded = true;
#undef LCHK
#undef LHIP
    return MAPSQ_OK;
}

// -------------------------------------------------------------------- map ---

static void zero_table(mapsq_table* t) { std::memset(t, 0, sizeof(*t)); }

static int find_pred(const Store& S, int32_t p) {
    auto it = std::lower_bound(S.preds.begin(), S.preds.end(), p);
    if (it == S.preds.end() || *it != p) return -1;
    return int(it - S.preds.begin());
}

// What a pattern's map needs: the output's metadata (in `out`), the row
// range of the store to read, and for a scan the equality tests and the
// source columns.  An empty predicate range leaves rows = 0.
mapsq_status map_plan(Ctx* ctx, const mapsq_pattern* pat, int32_t key_var, mapsq_table* out, MapPlan* mp) {
    zero_table(out);
    *mp = MapPlan{};
    if (!ctx->store.loaded) return ctx->fail(MAPSQ_ERR_STATE, "no store loaded");
    const Store& S = ctx->store;
    const int32_t term[3] = {pat->s, pat->p, pat->o};
    // variables in first-appearance order and their first position
    std::vector<int32_t> vars;
    std::vector<int> first_pos;
    int rep_a[3], rep_b[3], nrep = 0;
    for (int pos = 0; pos < 3; pos++) {
        if (term[pos] < 0) {
            int32_t v = -term[pos] - 1;
            auto it = std::find(vars.begin(), vars.end(), v);
            if (it == vars.end()) {
                vars.push_back(v);
                first_pos.push_back(pos);
            } else {
                rep_a[nrep] = first_pos[it - vars.begin()];
                rep_b[nrep] = pos;
                nrep++;
            }
        } else if (term[pos] == INT32_MAX) {
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "constant outside [0, 2^31 - 1)");
        }
    }
    if (vars.empty()) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a triple pattern without variables");
    // output column order: key first, then the others
    std::vector<int> order;  // index into vars
    if (key_var >= 0) {
        auto it = std::find(vars.begin(), vars.end(), key_var);
        if (it == vars.end()) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "key variable not in the pattern");
        order.push_back(int(it - vars.begin()));
    }
    for (int i = 0; i < (int)vars.size(); i++)
        if (std::find(order.begin(), order.end(), i) == order.end()) order.push_back(i);
    const int ncols = (int)vars.size();
    out->ncols = ncols;
    out->key_max = S.max_id;
    for (int c = 0; c < ncols; c++) {
        out->var[c] = vars[order[c]];
        mp->src_pos[c] = first_pos[order[c]];
    }

    // the three source columns and the row range to scan
    const int32_t* col[3] = {S.s, S.p, S.o};
    int64_t lo = 0, hi = S.n;
    bool s_const = term[0] >= 0, p_const = term[1] >= 0, o_const = term[2] >= 0;
    int sorted_pos = -1;  // the store position whose values ascend over the rows, if any
    if (p_const) {
        int pi = find_pred(S, term[1]);
        if (pi < 0) {
            mp->empty = true;
            return MAPSQ_OK;
        }
        lo = S.pred_off[pi];
        hi = S.pred_off[pi + 1];
        LocateQuery q{};
        q.lo = lo;
        q.hi = hi;
        if (s_const) {  // PSO: (p, s[, o])
            col[0] = S.pso_s;
            col[2] = S.pso_o;
            q.col1 = S.pso_s;
            q.v1 = term[0];
            if (o_const) {
                q.col2 = S.pso_o;
                q.v2 = term[2];
            }
            sorted_pos = 2;
        } else if (o_const) {  // POS: (p, o)
            col[0] = S.pos_s;
            col[2] = S.pos_o;
            q.col1 = S.pos_o;
            q.v1 = term[2];
            sorted_pos = 0;
        } else if (key_var >= 0 && term[2] == -key_var - 1 && term[0] != term[2]) {
            // POS, so that the rows come sorted on the key (the object)
            col[0] = S.pos_s;
            col[2] = S.pos_o;
            sorted_pos = 2;
        } else {
            col[0] = S.pso_s;
            col[2] = S.pso_o;
            sorted_pos = 0;
        }
        col[1] = nullptr;
        if (q.col1) {
            LocateQuery* qd = reinterpret_cast<LocateQuery*>(ctx->small + SMALL_SCALARS + 16);
            int64_t* od = reinterpret_cast<int64_t*>(ctx->small + SMALL_SCALARS + 48);
            std::memcpy(ctx->pinned, &q, sizeof(q));
            HIPCHK(hipMemcpyAsync(qd, ctx->pinned, sizeof(q), hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(launch_locate(qd, 1, od, ctx->stream));
            int64_t r[2];
            mapsq_status st = readback(ctx, od, 16, r);
            if (st) return st;
            lo = r[0];
            hi = r[1];
        }
    } else {
        // variable predicate: full scan of the raw columns, constants tested
        for (int pos = 0; pos < 3; pos++)
            if (term[pos] >= 0) {
                mp->ta[mp->nterm] = pos;
                mp->tb[mp->nterm] = -1;
                mp->tc[mp->nterm] = term[pos];
                mp->nterm++;
            }
    }
    for (int r = 0; r < nrep; r++) {
        mp->ta[mp->nterm] = rep_a[r];
        mp->tb[mp->nterm] = rep_b[r];
        mp->tc[mp->nterm] = 0;
        mp->nterm++;
    }
    // rows of an index range (and any order-preserving compaction of them)
    // ascend on the index's next sort column
    if (sorted_pos >= 0 && term[sorted_pos] < 0)
        for (int c = 0; c < ncols; c++)
            if (out->var[c] == -term[sorted_pos] - 1) out->sorted_col = c + 1;
    for (int pos = 0; pos < 3; pos++) mp->col[pos] = col[pos];
    mp->lo = lo;
    mp->rows = hi - lo;
    return MAPSQ_OK;
}

CompactArgs map_scan_args(const MapPlan& mp, int ncols, int32_t* const* out_cols, uint64_t* count) {
    CompactArgs a{};
    a.nin = 3;
    for (int pos = 0; pos < 3; pos++) a.in[pos] = mp.col[pos] ? mp.col[pos] + mp.lo : nullptr;
    a.n = (uint64_t)mp.rows;
    a.nterm = mp.nterm;
    for (int i = 0; i < mp.nterm; i++) {
        a.term_a[i] = mp.ta[i];
        a.term_b[i] = mp.tb[i];
        a.term_c[i] = mp.tc[i];
    }
    a.nout = ncols;
    for (int c = 0; c < ncols; c++) {
        a.out_src[c] = mp.src_pos[c];
        a.out[c] = out_cols[c];
    }
    a.count = count;
    return a;
}

double map_test_bytes(const MapPlan& mp) {
    // every row reads the columns its equality tests use
    bool used[3] = {false, false, false};
    for (int i = 0; i < mp.nterm; i++) {
        used[mp.ta[i]] = true;
        if (mp.tb[i] >= 0) used[mp.tb[i]] = true;
    }
    return 4.0 * ((int)used[0] + (int)used[1] + (int)used[2]) * (double)mp.rows;
}

mapsq_status map_pattern(Ctx* ctx, const mapsq_pattern* pat, int32_t key_var, mapsq_table* out) {
    MapPlan mp;
    if (mapsq_status st = map_plan(ctx, pat, key_var, out, &mp)) {
        zero_table(out);
        return st;
    }
    const int ncols = out->ncols;
    if (mp.empty) {
        out->nrows = 0;
        return MAPSQ_OK;
    }
    if (mp.nterm == 0) {
        // a view of the store
        out->owned = 0;
        out->nrows = mp.rows;
        for (int c = 0; c < ncols; c++) out->col[c] = const_cast<int32_t*>(mp.col[mp.src_pos[c]]) + mp.lo;
        return MAPSQ_OK;
    }
    // scan + compaction into an owned table laid out for the whole range
    mapsq_table t{};
    if (alloc_table(ctx, mp.rows, ncols, &t)) {
        zero_table(out);
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the map output");
    }
    CompactArgs a = map_scan_args(mp, ncols, t.col, scalar64(ctx, SC_COUNT));
    Block cs = alloc_block(ctx, compact_scratch_words((uint64_t)mp.rows) * 8);
    if (!cs.ok()) {
        free_table(ctx, &t);
        zero_table(out);
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the map's row masks");
    }
    int ph = ctx->prof_begin(0);
    hipError_t e = launch_fill_u32(scalar32(ctx, SC_COUNT), 2, 0u, ctx->stream);
    if (e == hipSuccess) e = launch_compact(a, cs.as<uint64_t>(), ctx->stream);
    ctx->prof_end(ph, map_test_bytes(mp));
    if (e != hipSuccess) {
        free_table(ctx, &t);
        zero_table(out);
        return ctx->fail(MAPSQ_ERR_HIP, std::string("map scan: ") + hipGetErrorString(e));
    }
    uint64_t kept = 0;
    mapsq_status st = readback(ctx, scalar64(ctx, SC_COUNT), 8, &kept);
    if (st) {
        free_table(ctx, &t);
        zero_table(out);
        return st;
    }
    // kept rows also read and write their output columns
    if (ph >= 0) ctx->pending[ph].bytes += 8.0 * ncols * (double)kept;
    // columns were laid out for the whole range; only the row count changes
    out->owned = 1;
    out->block = t.block;
    out->nrows = (int64_t)kept;
    for (int c = 0; c < ncols; c++) out->col[c] = t.col[c];
    return MAPSQ_OK;
}

// Row ranges of index lookups (one launch, one synchronisation): for each
// query the [lo, hi) part of its range whose sort columns equal v1 (and v2).
mapsq_status locate_ranges(Ctx* ctx, const LocateQuery* lq, size_t n, int64_t* out) {
    if (n == 0) return MAPSQ_OK;
    Block buf = alloc_block(ctx, n * (sizeof(LocateQuery) + 16));
    if (!buf.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for range queries");
    LocateQuery* qd = buf.as<LocateQuery>();
    int64_t* od = reinterpret_cast<int64_t*>(qd + n);
    const size_t up = n * sizeof(LocateQuery), down = n * 16;
    if (!ensure_stage(ctx, std::max(up, down))) return ctx->fail(MAPSQ_ERR_HIP, "pinned staging allocation failed");
    std::memcpy(ctx->stage, lq, up);
    hipError_t e = hipMemcpyAsync(qd, ctx->stage, up, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = launch_locate(qd, (int32_t)n, od, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->stage, od, down, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return ctx->fail(MAPSQ_ERR_HIP, std::string("range location: ") + hipGetErrorString(e));
    std::memcpy(out, ctx->stage, down);
    return MAPSQ_OK;
}

// ------------------------------------------------------------------- join ---

mapsq_status check_table(Ctx* ctx, const mapsq_table* t, const char* name) {
    if (!t) return ctx->fail(MAPSQ_ERR_INVALID_ARG, std::string(name) + " is null");
    if (t->ncols < 1 || t->ncols > MAPSQ_MAX_COLS)
        return ctx->fail(MAPSQ_ERR_INVALID_ARG, std::string(name) + ": ncols must be in [1, 16]");
    if (t->nrows < 0) return ctx->fail(MAPSQ_ERR_INVALID_ARG, std::string(name) + ": negative nrows");
    if (t->nrows >= (int64_t(1) << 31))
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, std::string(name) + ": a join input of 2^31 rows or more");
    for (int c = 0; c < t->ncols; c++) {
        if (t->nrows > 0 && !t->col[c]) return ctx->fail(MAPSQ_ERR_INVALID_ARG, std::string(name) + ": null column");
        for (int d = 0; d < c; d++)
            if (t->var[d] == t->var[c])
                return ctx->fail(MAPSQ_ERR_INVALID_ARG, std::string(name) + ": a variable appears twice");
    }
    return MAPSQ_OK;
}

// Room for a join result of `rows` rows x `nc` columns: the caller's output
// columns when the call writes there, else the arena's largest free block.
static mapsq_status result_room(Ctx* ctx, uint64_t rows, int nc) {
    if (ctx->out_cols) {
        if (rows > (uint64_t)ctx->out_cap)
            return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result (" + std::to_string(rows) +
                                                      " rows) exceeds the output capacity (" +
                                                      std::to_string(ctx->out_cap) + " rows)");
        return MAPSQ_OK;
    }
    if (ctx->arena.largest() < align_up(size_t(rows) * 4, ARENA_ALIGN) * nc)
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result (" + std::to_string(rows) +
                                                  " rows) exceeds the arena's free space");
    return MAPSQ_OK;
}

mapsq_status join_tables(Ctx* ctx, const mapsq_table* L, const mapsq_table* R, int32_t key_var, mapsq_table* out) {
    zero_table(out);
    const double est_rows = ctx->join_est_rows;  // this call's estimate only
    ctx->join_est_rows = -1.0;
    mapsq_status st;
    if ((st = check_table(ctx, L, "left")) || (st = check_table(ctx, R, "right"))) return st;
    const int lk = col_of(L, key_var), rk = col_of(R, key_var);
    if (lk < 0 || rk < 0) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "both tables must bind the key variable");
    // output columns: key, L's others, R's vars not in L; R's vars in L are filtered
    std::vector<int> lv, rv, extra_l, extra_r;
    for (int c = 0; c < L->ncols; c++)
        if (c != lk) lv.push_back(c);
    for (int c = 0; c < R->ncols; c++) {
        if (c == rk) continue;
        int cl = col_of(L, R->var[c]);
        if (cl >= 0) {
            extra_l.push_back(cl);
            extra_r.push_back(c);
        }
        rv.push_back(c);  // materialised (filtered copies dropped afterwards)
    }
    // Further variables both tables bind join as part of a composite key
    // (key_var, then the others in the left table's column order) instead
    // of being filtered after a join on key_var alone: only pairs that agree
    // on every shared variable meet.  The right table's copies are then
    // neither materialised nor filtered.
    int kl[MAX_KEY_WORDS] = {lk, -1, -1}, kr[MAX_KEY_WORDS] = {rk, -1, -1};
    int nkeys = 1;
    if (ctx->composite == 0 && !extra_r.empty()) {
        for (int c = 0; c < L->ncols && nkeys < MAX_KEY_WORDS; c++) {
            if (c == lk) continue;
            const int cr = col_of(R, L->var[c]);
            if (cr >= 0) {
                kl[nkeys] = c;
                kr[nkeys] = cr;
                nkeys++;
            }
        }
        for (int j = 1; j < nkeys; j++) {
            for (size_t i = 0; i < extra_r.size(); i++)
                if (extra_r[i] == kr[j]) {
                    extra_r.erase(extra_r.begin() + i);
                    extra_l.erase(extra_l.begin() + i);
                    break;
                }
            rv.erase(std::find(rv.begin(), rv.end(), kr[j]));
        }
    }
    const bool composite = nkeys > 1;
    const int nc_mat = 1 + (int)lv.size() + (int)rv.size();
    const int nc_out = nc_mat - (int)extra_r.size();
    if (nc_mat > MAPSQ_MAX_COLS) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 16 columns in the join");
    if (ctx->out_cols && !extra_r.empty())  // the filter needs a materialised copy of its own
        return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a join into caller columns shares only the key variable");
    const uint32_t nL = (uint32_t)L->nrows, nR = (uint32_t)R->nrows;
    const uint32_t N = nL + nR;

    std::vector<int32_t> mat_vars;
    mat_vars.push_back(key_var);
    for (int c : lv) mat_vars.push_back(L->var[c]);
    for (int c : rv) mat_vars.push_back(R->var[c]);
    auto set_meta = [&](mapsq_table* t) {
        int k = 0;
        for (int c = 0; c < nc_mat; c++) {
            bool drop = c >= 1 + (int)lv.size() &&
                        std::find(extra_r.begin(), extra_r.end(), rv[c - 1 - lv.size()]) != extra_r.end();
            if (!drop) t->var[k++] = mat_vars[c];
        }
        t->ncols = nc_out;
        t->key_max = (L->key_max >= 0 && R->key_max >= 0) ? std::max(L->key_max, R->key_max) : -1;
        t->sorted_col = 1;  // rows come out grouped by ascending key
    };
    // The materialised result m (nc_mat columns, total rows): further shared
    // variables keep the rows where both copies agree and drop R's copy.
    auto finish = [&](mapsq_table& m, uint64_t total) -> mapsq_status {
        hipError_t e;
        int ph;
        if (extra_r.empty()) {
            out->owned = m.owned;
            out->block = m.block;
            out->nrows = (int64_t)total;
            for (int c = 0; c < nc_mat; c++) out->col[c] = m.col[c];
            return MAPSQ_OK;
        }
        // further shared variables: keep rows where both copies agree, drop R's copy
        mapsq_table f{};
        if (alloc_table(ctx, (int64_t)total, nc_out, &f)) {
            free_table(ctx, &m);
            return ctx->fail(MAPSQ_ERR_TOO_LARGE, "filtered join result exceeds the arena's free space");
        }
        CompactArgs c{};
        c.nin = nc_mat;
        for (int i = 0; i < nc_mat; i++) c.in[i] = m.col[i];
        c.n = total;
        c.nterm = 0;
        for (size_t i = 0; i < extra_r.size(); i++) {
            if (c.nterm >= 6) {
                free_table(ctx, &m);
                free_table(ctx, &f);
                return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 6 further shared variables");
            }
            int li = 1 + int(std::find(lv.begin(), lv.end(), extra_l[i]) - lv.begin());
            int ri = 1 + (int)lv.size() + int(std::find(rv.begin(), rv.end(), extra_r[i]) - rv.begin());
            c.term_a[c.nterm] = li;
            c.term_b[c.nterm] = ri;
            c.nterm++;
        }
        c.nout = 0;
        for (int i = 0; i < nc_mat; i++) {
            bool drop = i >= 1 + (int)lv.size() &&
                        std::find(extra_r.begin(), extra_r.end(), rv[i - 1 - lv.size()]) != extra_r.end();
            if (!drop) {
                c.out_src[c.nout] = i;
                c.out[c.nout] = f.col[c.nout];
                c.nout++;
            }
        }
        c.count = scalar64(ctx, SC_COUNT);
        uint64_t kept = 0;
        e = hipSuccess;
        Block cs = alloc_block(ctx, compact_scratch_words((uint64_t)total) * 8);
        if (!cs.ok()) {
            free_table(ctx, &m);
            free_table(ctx, &f);
            return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the equality filter's row masks");
        }
        ph = ctx->prof_begin(4);
        if (e == hipSuccess) e = launch_fill_u32(scalar32(ctx, SC_COUNT), 2, 0u, ctx->stream);
        if (e == hipSuccess) e = launch_compact(c, cs.as<uint64_t>(), ctx->stream);
        ctx->prof_end(ph, 4.0 * (double)c.nterm * 2 * total);
        if (e == hipSuccess) st = readback(ctx, scalar64(ctx, SC_COUNT), 8, &kept);
        if (ph >= 0) ctx->pending[ph].bytes += 8.0 * (double)c.nout * (double)kept;
        free_table(ctx, &m);
        if (e != hipSuccess || st) {
            free_table(ctx, &f);
            return e != hipSuccess ? ctx->fail(MAPSQ_ERR_HIP, "equality filter launch failed") : st;
        }
        out->owned = 1;
        out->block = f.block;
        out->nrows = (int64_t)kept;
        for (int i = 0; i < nc_out; i++) out->col[i] = f.col[i];
        return MAPSQ_OK;
    };
    mapsq_join_stats js{};
    js.left_rows = nL;
    js.right_rows = nR;
    ctx->last = js;
    if (nL == 0 || nR == 0) {
        set_meta(out);
        out->owned = 1;
        out->nrows = 0;
        return MAPSQ_OK;
    }

    // Both tables already in key order (PSO/POS views, results of a join on
    // this key): Reduce straight from the two sides' key runs, no shuffle.
    const int32_t* lkey = L->col[lk];
    const int32_t* rkey = R->col[rk];
    // A count-only call on two large sorted tables counts from dense per-key
    // counts instead (two streaming passes over the keys), when the key range
    // allows: the merge pass searches the larger table once per key run of
    // the smaller one, which costs far more there.
    const bool dense_count = ctx->count_only && std::min(nL, nR) >= COUNT_DENSE_MIN &&
                             L->key_max >= 0 && R->key_max >= 0 &&
                             (uint64_t)std::max(L->key_max, R->key_max) < PRECOUNT_MAX_RANGE;
    if (!composite && !dense_count && ctx->merge_mode == 0 && L->sorted_col == lk + 1 && R->sorted_col == rk + 1) {
        const bool small_left = nL <= nR;
        const uint32_t nsm = small_left ? nL : nR, nbg = small_left ? nR : nL;
        const size_t sb4 = align_up(size_t(nsm) * 4, ARENA_ALIGN);
        Block seg = alloc_block(ctx, sb4 * 4 + align_up(size_t(nsm) * 8, ARENA_ALIGN));
        if (!seg.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for merge segments");
        if (!ctx->ensure_status(2 * size_t(merge_tiles(nsm)) + 2))
            return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: status words");
        char* sp = ctx->arena.ptr(seg.off);
        uint32_t* seg_ls = reinterpret_cast<uint32_t*>(sp);
        uint32_t* seg_lc = reinterpret_cast<uint32_t*>(sp + sb4);
        uint32_t* seg_rs = reinterpret_cast<uint32_t*>(sp + 2 * sb4);
        uint32_t* seg_rc = reinterpret_cast<uint32_t*>(sp + 3 * sb4);
        uint64_t* seg_off = reinterpret_cast<uint64_t*>(sp + 4 * sb4);
        MergeArgs ma{small_left ? lkey : rkey, nsm, small_left ? rkey : lkey, nbg, small_left ? 1 : 0,
                     seg_ls, seg_lc, seg_rs, seg_rc, seg_off, scalar32(ctx, SC_NSEG), scalar64(ctx, SC_TOTAL)};
        int ph = ctx->prof_begin(2);
        HIPCHK(launch_fill_u32(counter(ctx, CT_COUNT), 1, 0u, ctx->stream));
        HIPCHK(launch_merge_segments(ma, ctx->status, counter(ctx, CT_COUNT), ctx->next_epoch(), ctx->stream));
        ctx->prof_end(ph, 0.0);
        uint32_t sc[4];
        if ((st = readback(ctx, scalar32(ctx, SC_NSEG), 16, sc))) return st;
        const uint32_t nseg = sc[0];
        uint64_t total;
        std::memcpy(&total, &sc[2], 8);
        // reads the smaller side's keys; writes 24 B per segment
        if (ph >= 0) ctx->pending[ph].bytes = 4.0 * nsm + 24.0 * nseg;
        js.segments = nseg;
        js.out_rows = (int64_t)total;
        js.path = MAPSQ_PATH_MERGE;
        js.sorted_records = 0;
        ctx->last = js;
        if (total >= SAT40_HOST) return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds 2^40 rows");
        set_meta(out);
        if (total == 0 || ctx->count_only) {
            out->owned = 1;
            out->nrows = (int64_t)total;
            return MAPSQ_OK;
        }
        mapsq_table m{};
        if ((st = result_room(ctx, total, nc_mat))) return st;
        if (alloc_table(ctx, (int64_t)total, nc_mat, &m))
            return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds the arena's free space");
        MatArgs a{};
        a.keys = reinterpret_cast<const uint32_t*>(lkey);
        a.seg_start = seg_ls;
        a.seg_split = seg_rs;
        a.seg_cl = seg_lc;
        a.seg_cr = seg_rc;
        a.seg_off = seg_off;
        a.nseg = scalar32(ctx, SC_NSEG);
        a.key_base = 0;
        a.nl = (int)lv.size();
        a.nr = (int)rv.size();
        for (int i = 0; i < a.nl; i++) a.lcol[i] = L->col[lv[i]];
        for (int i = 0; i < a.nr; i++) a.rcol[i] = R->col[rv[i]];
        for (int c = 0; c < nc_mat; c++) a.out[c] = m.col[c];
        a.row_begin = 0;
        a.row_end = total;
        a.sparse = total < SPARSE_ROWS_PER_SEG * (uint64_t)nseg ? 1 : 0;
        a.max_blocks = ctx->mat_blocks(total);
        ph = ctx->prof_begin(3);
        hipError_t e = launch_materialize(a, ctx->stream);
        // writes 4 B per output cell and reads the segment table (the value
        // cells of the matched runs are not counted)
        ctx->prof_end(ph, 4.0 * nc_mat * (double)total + 24.0 * nseg);
        ctx->acc.joins += 1;
        ctx->acc.rows_out += (int64_t)total;
        if (e != hipSuccess) {
            free_table(ctx, &m);
            return ctx->fail(MAPSQ_ERR_HIP, std::string("materialize: ") + hipGetErrorString(e));
        }
        return finish(m, total);
    }

    // key range: known bound, else a min/max pass (a composite key: every
    // variable's range from one read-back)
    int32_t kmin = 0, kmax;
    int32_t wmin[MAX_KEY_WORDS] = {0, 0, 0}, wmax[MAX_KEY_WORDS] = {0, 0, 0};
    if (composite) {
        static_assert(MAX_KEY_WORDS == 3, "one scalar pair per key word");
        const int slot[MAX_KEY_WORDS] = {SC_MINMAX, SC_MINMAX2, SC_MINMAX3};
        int32_t init[2] = {INT32_MAX, INT32_MIN};
        std::memcpy(ctx->pinned, init, 8);
        for (int j = 0; j < nkeys; j++) {
            int32_t* mm = reinterpret_cast<int32_t*>(scalar32(ctx, slot[j]));
            HIPCHK(hipMemcpyAsync(mm, ctx->pinned, 8, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(launch_minmax(L->col[kl[j]], nL, R->col[kr[j]], nR, mm, ctx->stream));
        }
        int32_t r[SC_MINMAX3 + 2 - SC_MINMAX];  // scalar words SC_MINMAX .. SC_MINMAX3 + 1
        if ((st = readback(ctx, scalar32(ctx, SC_MINMAX), sizeof(r), r))) return st;
        for (int j = 0; j < nkeys; j++) {
            wmin[j] = r[slot[j] - SC_MINMAX];
            wmax[j] = r[slot[j] - SC_MINMAX + 1];
        }
        kmin = wmin[0];
        kmax = wmax[0];
    } else if (L->key_max >= 0 && R->key_max >= 0) {
        kmax = std::max(L->key_max, R->key_max);
    } else {
        int32_t init[2] = {INT32_MAX, INT32_MIN};
        int32_t* mm = reinterpret_cast<int32_t*>(scalar32(ctx, SC_MINMAX));
        std::memcpy(ctx->pinned, init, 8);
        HIPCHK(hipMemcpyAsync(mm, ctx->pinned, 8, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(launch_minmax(lkey, nL, rkey, nR, mm, ctx->stream));
        int32_t r[2];
        if ((st = readback(ctx, mm, 8, r))) return st;
        kmin = r[0];
        kmax = r[1];
    }
    // bits of each key variable's relative range; a composite key whose
    // ranges fit side by side in one 32-bit word is sorted packed (key_var
    // highest), otherwise word by word from the last variable to key_var
    int wbits[MAX_KEY_WORDS] = {bitlen((uint64_t)((int64_t)kmax - (int64_t)kmin)), 0, 0};
    int key_bits = wbits[0];
    for (int j = 1; j < nkeys; j++) {
        wbits[j] = bitlen((uint64_t)((int64_t)wmax[j] - (int64_t)wmin[j]));
        key_bits += wbits[j];
    }
    const int low_bits = key_bits - wbits[0];  // the shift of key_var in a packed word
    const bool packed = composite && key_bits <= 32 && low_bits <= 31;
    int rb, kpt;
    pick_tuning(ctx, key_bits, rb, kpt, (uint64_t)nL + nR);

    // A large shuffle first gets the exact |RS| from two passes over the
    // keys (dense key counts of one side, summed over the other side's
    // records): a join with no key in common, or whose output cannot fit in
    // the arena's free space at all, then ends without sorting anything.
    // On a join that fits it costs about as much as the count phase.
    // (a count-only call takes it whenever the key range allows: it is the
    // whole answer there)
    // (automatic mode skips it when the caller's estimate of the output is
    // far below the free space: the pre-count then mostly costs time)
    const bool est_small = est_rows >= 0.0 && est_rows * 4.0 * nc_mat * 8.0 < (double)ctx->arena.free_bytes();
    const bool precount = !composite && (ctx->precount == 2 || ctx->count_only ||
                                         (ctx->precount == 0 && (uint64_t)N >= PRECOUNT_MIN_RECORDS && !est_small));
    if (precount) {
        const uint64_t range = (uint64_t)((int64_t)kmax - (int64_t)kmin) + 1;
        Block cnt;
        if (range <= PRECOUNT_MAX_RANGE) cnt = alloc_block(ctx, size_t(range) * 4);
        if (cnt.ok()) {
            // count a side sorted on the key (its hot keys come in runs), else the smaller one
            const bool ls = L->sorted_col == lk + 1, rs = R->sorted_col == rk + 1;
            const bool count_left = ls && rs ? nL <= nR : (ls || (!rs && nL <= nR));
            const int ph = ctx->prof_begin(2);
            HIPCHK(launch_fill_u32(cnt.as<uint32_t>(), range, 0u, ctx->stream));
            HIPCHK(launch_fill_u32(scalar32(ctx, SC_PRECOUNT), 2, 0u, ctx->stream));
            HIPCHK(launch_key_count(count_left ? lkey : rkey, count_left ? nL : nR, kmin, range, cnt.as<uint32_t>(),
                                    ctx->stream));
            HIPCHK(launch_key_dot(count_left ? rkey : lkey, count_left ? nR : nL, kmin, range, cnt.as<uint32_t>(),
                                  scalar64(ctx, SC_PRECOUNT), ctx->stream));
            // clears the counts, reads both key columns and one count per record of the other side
            ctx->prof_end(ph, 4.0 * range + 4.0 * N + 4.0 * (count_left ? nR : nL));
            uint64_t total = 0;
            if ((st = readback(ctx, scalar64(ctx, SC_PRECOUNT), 8, &total))) return st;
            cnt.reset();
            js.out_rows = (int64_t)std::min<uint64_t>(total, SAT40_HOST);
            ctx->last = js;
            if (total >= SAT40_HOST) return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds 2^40 rows");
            if (total == 0 || ctx->count_only) {
                set_meta(out);
                out->owned = 1;
                out->nrows = (int64_t)total;
                return MAPSQ_OK;
            }
            if (ctx->out_cols ? total > (uint64_t)ctx->out_cap
                              : (double)align_up(size_t(total) * 4, ARENA_ALIGN) * nc_mat >
                                    (double)ctx->arena.free_bytes())
                return result_room(ctx, total, nc_mat);
        }
    }

    // scratch: sort buffers (16 N) and segment offsets (8 N); the spare sort
    // buffers later hold the segment starts and splits
    const size_t nb4 = align_up(size_t(N) * 4, ARENA_ALIGN);
    Block scratch = alloc_block(ctx, nb4 * 4 + nb4 * 2);
    if (!scratch.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for join scratch");
    char* sb = ctx->arena.ptr(scratch.off);
    SortBufs b{{reinterpret_cast<uint32_t*>(sb), reinterpret_cast<uint32_t*>(sb + nb4)},
               {reinterpret_cast<uint32_t*>(sb + 2 * nb4), reinterpret_cast<uint32_t*>(sb + 3 * nb4)}};
    uint64_t* seg_off = reinterpret_cast<uint64_t*>(sb + 4 * nb4);

    // Semi-join reduction: when one side is much larger, only its records
    // whose key the other side has are sorted (same rows, same order).
    uint32_t Ns = N;  // records that go through the shuffle
    uint32_t nLs = nL, nRs = nR;  // of which LEFT and RIGHT
    int ph;
    {
        const bool left_big = nL >= nR;
        const uint32_t nb = left_big ? nL : nR, nsm = left_big ? nR : nL;
        const uint64_t range = (uint64_t)((int64_t)kmax - (int64_t)kmin) + 1;
        const uint64_t words = (range + 31) / 32;
        bool semi = false;
        if (composite)
            semi = false;
        else if (ctx->semijoin == 0)
            semi = nb >= SEMI_MIN_RECORDS && (uint64_t)nsm * SEMI_RATIO <= nb && words <= (uint64_t)nb;
        else if (ctx->semijoin == 2)
            semi = words * 4 <= (uint64_t(1) << 30);
        Block bm;
        if (semi) bm = alloc_block(ctx, words * 4);
        if (bm.ok()) {
            ph = ctx->prof_begin(8);
            uint32_t* bits = bm.as<uint32_t>();
            HIPCHK(launch_fill_u32(bits, words, 0u, ctx->stream));
            HIPCHK(launch_fill_u32(counter(ctx, CT_SEMI), 1, 0u, ctx->stream));
            HIPCHK(launch_bitmap_set(left_big ? rkey : lkey, nsm, kmin, range, bits, ctx->stream));
            if (!ctx->ensure_status(semi_filter_tiles(nb) + 1))
                return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: status words");
            const uint32_t at = left_big ? 0u : nL;
            SemiArgs sa{left_big ? lkey : rkey, nb, kmin, range, bits, at, b.k[0] + at, b.v[0] + at,
                        scalar32(ctx, SC_SEMI)};
            HIPCHK(launch_semi_filter(sa, ctx->status, counter(ctx, CT_SEMI), ctx->next_epoch(), ctx->stream));
            if (left_big)  // the RIGHT records follow the kept LEFT ones
                HIPCHK(launch_side_records(rkey, nR, kmin, nL, scalar32(ctx, SC_SEMI), b.k[0], b.v[0], ctx->stream));
            else
                HIPCHK(launch_side_records(lkey, nL, kmin, 0u, nullptr, b.k[0], b.v[0], ctx->stream));
            // bitmap cleared, set and read once; the small side's keys read
            // twice and its records written; the big side's keys read
            ctx->prof_end(ph, 8.0 * words + 16.0 * nsm + 4.0 * nb);
            uint32_t kept = 0;
            if ((st = readback(ctx, scalar32(ctx, SC_SEMI), 4, &kept))) return st;
            if (ph >= 0) ctx->pending[ph].bytes += 8.0 * kept;
            Ns = kept + nsm;
            (left_big ? nLs : nRs) = kept;
            js.path = MAPSQ_PATH_SEMIJOIN;
            js.sorted_records = Ns;
            ctx->last = js;
            if (kept == 0) {  // no key in common
                set_meta(out);
                out->owned = 1;
                out->nrows = 0;
                return MAPSQ_OK;
            }
        }
    }
    js.sorted_records = Ns;

    // Map + Sort: the first pass reads the LEFT then the RIGHT key column
    // (or the records the semi-join kept).  When each side has at most one
    // value column the records carry that value instead of their position
    // (the side moves into the key's low bit), so Reduce reads the values
    // in sorted order instead of gathering them through the positions.
    const bool carry =
        !composite && js.path != MAPSQ_PATH_SEMIJOIN && lv.size() <= 1 && rv.size() <= 1 && key_bits <= 31;
    const int sort_bits = carry ? key_bits + 1 : key_bits;
    if (carry) pick_tuning(ctx, sort_bits, rb, kpt, (uint64_t)Ns);
    SortSrc src{lkey, nL, rkey, nR, kmin, nullptr, nullptr, carry ? 1 : 0};
    if (carry) {
        src.v0 = lv.empty() ? lkey : L->col[lv[0]];  // payloads of a side without values go unused
        src.v1 = rv.empty() ? rkey : R->col[rv[0]];
    }
    int res, passes;
    const uint8_t* brk = nullptr;  // break flags of a composite key sorted word by word
    Block cbuf;                    // packed composite keys, or those flags
    if (composite) {
        js.path = MAPSQ_PATH_COMPOSITE;
        cbuf = alloc_block(ctx, packed ? nb4 : align_up(size_t(N), ARENA_ALIGN));
        if (!cbuf.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for composite keys");
    }
    ph = ctx->prof_begin(1);
    double sort_bytes;
    if (packed) {
        // one key word per record: the variables' relative values side by
        // side, key_var in the highest bits
        uint32_t* pk = cbuf.as<uint32_t>();
        PackArgs pl{}, pr{};
        pl.ncols = pr.ncols = nkeys;
        for (int j = 0, sh = low_bits; j < nkeys; j++) {
            pl.col[j] = L->col[kl[j]];
            pr.col[j] = R->col[kr[j]];
            pl.base[j] = pr.base[j] = wmin[j];
            pl.shift[j] = pr.shift[j] = wbits[j] ? sh : 0;  // a zero-width word adds nothing
            if (j + 1 < nkeys) sh -= wbits[j + 1];
        }
        HIPCHK(launch_pack_keys(pl, nL, pk, ctx->stream));
        HIPCHK(launch_pack_keys(pr, nR, pk + nL, ctx->stream));
        SortSrc ps{reinterpret_cast<const int32_t*>(pk), nL, reinterpret_cast<const int32_t*>(pk) + nL, nR, 0,
                   nullptr, nullptr, 0};
        if ((st = radix_sort(ctx, &ps, Ns, key_bits, rb, kpt, b, &res, &passes))) return st;
        // packing reads every key column and writes the packed word
        sort_bytes = 4.0 * (nkeys + 1) * Ns + 16.0 * Ns * passes;
    } else if (composite) {
        // LSD over the words: a stable sort on the last variable, then on
        // each earlier one of the records in the order so far (its cells
        // gathered through the record ids), ending with key_var; records end
        // grouped by the whole key, LEFT ahead of RIGHT inside each group
        int rbj, kptj, rj, pj;
        passes = 0;
        const int last = nkeys - 1;
        pick_tuning(ctx, wbits[last], rbj, kptj, (uint64_t)Ns);
        SortSrc sl{L->col[kl[last]], nL, R->col[kr[last]], nR, wmin[last], nullptr, nullptr, 0};
        if ((st = radix_sort(ctx, &sl, Ns, wbits[last], rbj, kptj, b, &rj, &pj))) return st;
        passes += pj;
        for (int j = last - 1; j >= 0; j--) {
            HIPCHK(launch_side_gather(L->col[kl[j]], R->col[kr[j]], nL, b.v[rj], Ns, wmin[j], b.k[1 - rj],
                                      ctx->stream));
            SortBufs bj{{b.k[1 - rj], b.k[rj]}, {b.v[rj], b.v[1 - rj]}};
            pick_tuning(ctx, wbits[j], rbj, kptj, (uint64_t)Ns);
            if ((st = radix_sort(ctx, nullptr, Ns, wbits[j], rbj, kptj, bj, &rj, &pj))) return st;
            b = bj;
            passes += pj;
        }
        res = rj;
        rb = rbj;
        BreakArgs ba{};
        ba.n_left = nL;
        ba.nw = nkeys - 1;
        for (int j = 1; j < nkeys; j++) {
            ba.lcol[j - 1] = L->col[kl[j]];
            ba.rcol[j - 1] = R->col[kr[j]];
        }
        uint8_t* fl = cbuf.as<uint8_t>();
        HIPCHK(launch_key_breaks(ba, b.v[res], Ns, fl, ctx->stream));
        brk = fl;
        // every sort, the gather of each earlier variable between them
        // (read 4N ids, 4N cells, write 4N), and the break flags (read 4N
        // ids and 4N cells per further variable, write N)
        sort_bytes = 16.0 * Ns * passes + 12.0 * (nkeys - 1) * Ns + (4.0 + 4.0 * (nkeys - 1) + 1.0) * Ns;
    } else {
        if ((st = radix_sort(ctx, js.path == MAPSQ_PATH_SEMIJOIN ? nullptr : &src, Ns, sort_bits, rb, kpt, b, &res,
                             &passes)))
            return st;
        // histogram reads 4N; the first pass reads 4N keys (8N records after a
        // semi-join, plus the carried value cells), later passes 8N; every pass
        // writes 8N
        sort_bytes = 16.0 * Ns * passes + (js.path == MAPSQ_PATH_SEMIJOIN ? 4.0 * Ns : 0.0) +
                     (carry ? 4.0 * (lv.size() * (double)nL + rv.size() * (double)nR) : 0.0);
    }
    ctx->prof_end(ph, sort_bytes);
    const uint32_t* skeys = b.k[res];
    const uint32_t* svals = b.v[res];
    uint32_t* seg_start = b.k[1 - res];
    uint32_t* seg_split = b.v[1 - res];
    // ReduceDuplicate: segments, counts, offsets
    Block ss = alloc_block(ctx, seg_scratch_bytes(Ns));
    if (!ss.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the segment scans");
    ph = ctx->prof_begin(2);
    HIPCHK(launch_seg_heads(skeys, svals, Ns, nL, carry ? 1 : 0, seg_start, seg_split, scalar32(ctx, SC_NSEG),
                            ss.as<void>(), ctx->stream, brk));
    HIPCHK(launch_seg_count(Ns, seg_start, scalar32(ctx, SC_NSEG), Ns, seg_split, seg_off, scalar64(ctx, SC_TOTAL),
                            scalar64(ctx, SC_MAXPAIRS), ss.as<void>(), ctx->stream));
    uint32_t sc[SC_MAXPAIRS + 2];  // scalar words 0 .. SC_MAXPAIRS + 1
    {
        // bytes are filled in once the segment count is known (below)
        ctx->prof_end(ph, 0.0);
    }
    if ((st = readback(ctx, scalar32(ctx, SC_NSEG), sizeof(sc), sc))) return st;
    uint64_t max_pairs;
    std::memcpy(&max_pairs, &sc[SC_MAXPAIRS], 8);
    const uint32_t nseg = sc[0];
    // heads: read 4N keys and 4N payloads, write 4S starts and 4S splits;
    // count: read 8S starts and 4S splits, write 8S offsets
    if (ph >= 0) ctx->pending[ph].bytes = (brk ? 9.0 : 8.0) * Ns + 28.0 * nseg;
    uint64_t total;
    std::memcpy(&total, &sc[2], 8);
    js.segments = nseg;
    js.out_rows = (int64_t)total;
    js.radix_bits = rb;
    js.passes = passes;
    js.key_bits = key_bits;
    ctx->last = js;
    if (total >= SAT40_HOST) return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds 2^40 rows");
    set_meta(out);
    if (total == 0 || ctx->count_only) {
        out->owned = 1;
        out->nrows = (int64_t)total;
        return MAPSQ_OK;
    }
    mapsq_table m{};
    if ((st = result_room(ctx, total, nc_mat))) return st;
    if (alloc_table(ctx, (int64_t)total, nc_mat, &m))
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds the arena's free space");
    MatArgs a{};
    a.keys = skeys;
    a.vals = svals;
    a.seg_start = seg_start;
    a.seg_split = seg_split;
    a.seg_off = seg_off;
    a.nseg = scalar32(ctx, SC_NSEG);
    a.n = Ns;
    a.n_left = nL;
    a.key_base = kmin;
    a.key_shift = carry ? 1 : (packed ? low_bits : 0);
    a.nl = (int)lv.size();
    a.nr = (int)rv.size();
    for (int i = 0; i < a.nl; i++) a.lcol[i] = L->col[lv[i]];
    for (int i = 0; i < a.nr; i++) a.rcol[i] = R->col[rv[i]];
    for (int c = 0; c < nc_mat; c++) a.out[c] = m.col[c];
    a.row_begin = 0;
    a.row_end = total;
    a.sparse = total < SPARSE_ROWS_PER_SEG * (uint64_t)nseg ? 1 : 0;
    a.seg_major = mat_seg_use(total, nseg, max_pairs) ? 1 : 0;
    a.seg_count = nseg;
    a.max_blocks = ctx->mat_blocks(total);
    // values in sorted record order when output rows outnumber records
    // (each record's values are then read many times)
    const int nv = std::max(a.nl, a.nr);
    const double value_cells = a.nl * (double)nLs + a.nr * (double)nRs;
    Block sval;
    if (carry) {
        // both sides' value cells are the sorted payloads themselves
        a.sval[0] = reinterpret_cast<const int32_t*>(svals);
        a.use_sval = 1;
    } else if (nv > 0 && total >= Ns) {
        sval = alloc_block(ctx, size_t(nv) * nb4);
    }
    if (sval.ok()) {
        GatherArgs g{};
        g.vals = svals;
        g.n = Ns;
        g.n_left = nL;
        g.nl = a.nl;
        g.nr = a.nr;
        for (int i = 0; i < a.nl; i++) g.lcol[i] = a.lcol[i];
        for (int i = 0; i < a.nr; i++) g.rcol[i] = a.rcol[i];
        for (int c = 0; c < nv; c++) {
            g.out[c] = reinterpret_cast<int32_t*>(ctx->arena.ptr(sval.off) + c * nb4);
            a.sval[c] = g.out[c];
        }
        a.use_sval = 1;
        ph = ctx->prof_begin(7);
        hipError_t ge = launch_gather_values(g, ctx->stream);
        // reads every payload and each value cell once, writes nv cells per record
        ctx->prof_end(ph, 4.0 * Ns + 4.0 * value_cells + 4.0 * nv * (double)Ns);
        if (ge != hipSuccess) {
            free_table(ctx, &m);
            return ctx->fail(MAPSQ_ERR_HIP, std::string("gather: ") + hipGetErrorString(ge));
        }
    }
    ph = ctx->prof_begin(3);
    hipError_t e = launch_materialize(a, ctx->stream);
    // writes 4 B per output cell; reads each segment's key and table entries
    // and each value cell once (from the gathered copy when there is one,
    // else through every record's payload)
    ctx->prof_end(ph, 4.0 * nc_mat * (double)total + 20.0 * nseg + 4.0 * value_cells + (a.use_sval ? 0.0 : 4.0 * Ns));
    ctx->acc.joins += 1;
    ctx->acc.rows_out += (int64_t)total;
    if (e != hipSuccess) {
        free_table(ctx, &m);
        return ctx->fail(MAPSQ_ERR_HIP, std::string("materialize: ") + hipGetErrorString(e));
    }
    return finish(m, total);
}

}  // namespace mq
