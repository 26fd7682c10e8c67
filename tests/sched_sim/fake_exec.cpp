// Host-only simulation of the serving scheduler (test infrastructure).
//
// The library's own scheduler (serve.cpp), planner (planner.cpp) and arena
// (arena.cpp) are compiled unchanged with the host compiler and linked with
// this file, which stands in for the device side: pattern maps, joins,
// batched joins and index range lookups.  Tables carry no data, only their
// sizes; every size is a deterministic function of the pattern or of the
// two joined tables, so a query's plan and outcome do not depend on what
// else runs.  Memory follows the library's rules: index views take none,
// scans and join outputs take arena blocks of their exact size, joins hold
// their scratch while they run, a batch places its results in one shared
// block, and a result that cannot fit fails as the device path fails.
//
// The driver runs one scenario (seeded queries, arena size, budget, arrival
// and poll schedules), first every query alone through mq::query, then all
// of them through submit / serve_step / poll_next, and prints one JSON line:
// whether the loop ended within the round limit, each query's outcome both
// ways, and the arena's free bytes before and after.
#include <algorithm>
#include <cinttypes>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

namespace mq {

namespace {

uint64_t mix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// fake device addresses of the store's index columns (never dereferenced)
int32_t* fake_ptr(uint64_t k) { return reinterpret_cast<int32_t*>(uintptr_t(0x7f0000000000ull + (k << 32))); }

// rows of an index range [lo, hi) whose sort column(s) equal v1 (and v2)
int64_t narrowed(int64_t lo, int64_t hi, bool pso, int32_t v1, int32_t v2, bool two) {
    const uint64_t h = mix(uint64_t(lo) * 1315423911ull ^ uint64_t(uint32_t(v1)) << 1 ^ (pso ? 1 : 0) ^
                           (two ? mix(uint64_t(uint32_t(v2))) : 0));
    const int64_t n = hi - lo;
    if (n <= 0 || h % 7 == 0) return 0;
    if (two) return std::min<int64_t>(n, 1 + int64_t(h >> 40) % 4);
    return std::min<int64_t>(n, int64_t(h >> 20) % (1 + n / (2 + int64_t(h % 50))));
}

// rows kept by a scan of `range` rows with equality tests
int64_t scanned(const int32_t t[3], int64_t range) {
    const uint64_t h = mix(uint64_t(uint32_t(t[0])) * 31 ^ uint64_t(uint32_t(t[1])) << 21 ^ uint64_t(uint32_t(t[2])) << 42);
    if (range <= 0 || h % 5 == 0) return 0;
    return int64_t(h >> 16) % (1 + range / (1 + int64_t(h % 200)));
}

// exact output rows of a join (before equality filters): a fixed function
// of the two sides' sizes and the key
uint64_t join_rows(int64_t nl, int64_t nr, int32_t key, int ncl, int ncr) {
    const uint64_t h = mix(uint64_t(nl) * 0x100000001B3ull ^ mix(uint64_t(nr)) ^ uint64_t(uint32_t(key)) << 7 ^
                           uint64_t(ncl * 17 + ncr));
    const uint64_t l = uint64_t(nl), r = uint64_t(nr), m = std::min(l, r);
    // the planner runs a cross product as a join on a constant key (one segment)
    if (key == INT32_MIN + 7) return std::min<uint64_t>(l * r, SAT40_HOST);
    uint64_t v;
    switch (h % 8) {
        case 0: v = 0; break;
        case 1: case 2: case 3: v = m * (1 + (h >> 8) % 4); break;
        case 4: case 5: v = (l * r) / (1 + (h >> 16) % std::max<uint64_t>(1, m)); break;
        case 6: v = (l * r) / (1 + (h >> 16) % 16); break;
        default: v = l + r; break;
    }
    return std::min<uint64_t>(v, SAT40_HOST);
}

void zero(mapsq_table* t) { std::memset(t, 0, sizeof(*t)); }

}  // namespace

mapsq_status locate_ranges(Ctx* ctx, const LocateQuery* q, size_t n, int64_t* out) {
    for (size_t i = 0; i < n; i++) {
        const bool pso = q[i].col1 == ctx->store.pso_s;
        out[2 * i] = q[i].lo;
        out[2 * i + 1] = q[i].lo + narrowed(q[i].lo, q[i].hi, pso, q[i].v1, q[i].v2, q[i].col2 != nullptr);
    }
    return MAPSQ_OK;
}

hipError_t launch_fill_u32(uint32_t*, uint64_t, uint32_t, hipStream_t) { return hipSuccess; }

mapsq_status map_pattern(Ctx* ctx, const mapsq_pattern* pat, int32_t key_var, mapsq_table* out) {
    zero(out);
    const Store& S = ctx->store;
    const int32_t term[3] = {pat->s, pat->p, pat->o};
    std::vector<int32_t> vars;
    std::vector<int> first_pos;
    bool rep = false;
    for (int pos = 0; pos < 3; pos++)
        if (term[pos] < 0) {
            const int32_t v = -term[pos] - 1;
            auto it = std::find(vars.begin(), vars.end(), v);
            if (it == vars.end()) {
                vars.push_back(v);
                first_pos.push_back(pos);
            } else {
                rep = true;
            }
        }
    if (vars.empty()) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a triple pattern without variables");
    std::vector<int> order;
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
    for (int c = 0; c < ncols; c++) out->var[c] = vars[order[c]];
    int64_t lo = 0, hi = S.n, rows;
    int sorted_pos = -1;
    bool scan = rep;
    if (term[1] >= 0) {
        auto it = std::lower_bound(S.preds.begin(), S.preds.end(), term[1]);
        if (it == S.preds.end() || *it != term[1]) return MAPSQ_OK;
        const size_t pi = size_t(it - S.preds.begin());
        lo = S.pred_off[pi];
        hi = S.pred_off[pi + 1];
        if (term[0] >= 0) {
            hi = lo + narrowed(lo, hi, true, term[0], term[2], term[2] >= 0);
            sorted_pos = 2;
        } else if (term[2] >= 0) {
            hi = lo + narrowed(lo, hi, false, term[2], 0, false);
            sorted_pos = 0;
        } else if (key_var >= 0 && term[2] == -key_var - 1 && term[0] != term[2]) {
            sorted_pos = 2;
        } else {
            sorted_pos = 0;
        }
        rows = hi - lo;
    } else {
        scan = true;
        rows = hi - lo;
    }
    if (sorted_pos >= 0 && term[sorted_pos] < 0)
        for (int c = 0; c < ncols; c++)
            if (out->var[c] == -term[sorted_pos] - 1) out->sorted_col = c + 1;
    if (!scan) {
        out->nrows = rows;
        for (int c = 0; c < ncols; c++) out->col[c] = fake_ptr(1 + first_pos[order[c]]) + lo;
        return MAPSQ_OK;
    }
    // scan: an output sized for the scanned range plus the row masks
    mapsq_table t{};
    if (alloc_table(ctx, rows, ncols, &t)) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the map output");
    Block cs = alloc_block(ctx, size_t(rows / 8 + 4096));
    if (!cs.ok()) {
        free_table(ctx, &t);
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the map's row masks");
    }
    out->owned = 1;
    out->block = t.block;
    out->nrows = scanned(term, rows);
    for (int c = 0; c < ncols; c++) out->col[c] = t.col[c];
    return MAPSQ_OK;
}

mapsq_status join_tables(Ctx* ctx, const mapsq_table* L, const mapsq_table* R, int32_t key_var, mapsq_table* out) {
    zero(out);
    const int lk = col_of(L, key_var), rk = col_of(R, key_var);
    if (lk < 0 || rk < 0) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "both tables must bind the key variable");
    if (L->nrows >= (int64_t(1) << 31) || R->nrows >= (int64_t(1) << 31))
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, "a join input of 2^31 rows or more");
    std::vector<int32_t> mv{key_var};
    int extra = 0;
    for (int c = 0; c < L->ncols; c++)
        if (c != lk) mv.push_back(L->var[c]);
    std::vector<int32_t> keep = mv;
    for (int c = 0; c < R->ncols; c++) {
        if (c == rk) continue;
        if (col_of(L, R->var[c]) >= 0)
            extra++;
        else
            keep.push_back(R->var[c]);
        mv.push_back(R->var[c]);
    }
    const int nc_mat = (int)mv.size(), nc_out = (int)keep.size();
    if (nc_mat > MAPSQ_MAX_COLS) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 16 columns in the join");
    auto meta = [&](mapsq_table* t) {
        t->ncols = nc_out;
        for (int c = 0; c < nc_out; c++) t->var[c] = keep[c];
        t->key_max = std::max(L->key_max, R->key_max);
        t->sorted_col = 1;
        t->owned = 1;
    };
    ctx->last = mapsq_join_stats{};
    const int64_t nL = L->nrows, nR = R->nrows;
    if (nL == 0 || nR == 0) {
        meta(out);
        return MAPSQ_OK;
    }
    const uint64_t total = join_rows(nL, nR, key_var, L->ncols, R->ncols);
    const uint64_t N = uint64_t(nL + nR);
    const bool merge = L->sorted_col == lk + 1 && R->sorted_col == rk + 1;
    Block scratch;
    if (merge) {
        scratch = alloc_block(ctx, size_t(std::min(nL, nR)) * 24);
        if (!scratch.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for merge segments");
    } else {
        if (N >= (uint64_t(1) << 24)) {  // exact count before the shuffle
            ctx->last.out_rows = (int64_t)total;
            if (total >= SAT40_HOST) return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds 2^40 rows");
            if ((double)align_up(size_t(total) * 4, ARENA_ALIGN) * nc_mat > (double)ctx->arena.free_bytes())
                return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds the arena's free space");
        }
        scratch = alloc_block(ctx, size_t(N) * 24);
        if (!scratch.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for join scratch");
    }
    ctx->last.out_rows = (int64_t)total;
    if (total >= SAT40_HOST) return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds 2^40 rows");
    if (total == 0) {
        meta(out);
        return MAPSQ_OK;
    }
    const size_t colb = align_up(size_t(total) * 4, ARENA_ALIGN);
    if (ctx->arena.largest() < colb * nc_mat)
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds the arena's free space");
    mapsq_table m{};
    if (alloc_table(ctx, (int64_t)total, nc_mat, &m))
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join result exceeds the arena's free space");
    if (extra == 0) {
        const uint64_t blk = m.block;
        meta(out);
        out->block = blk;
        out->nrows = (int64_t)total;
        for (int c = 0; c < nc_out; c++) out->col[c] = m.col[c];
        return MAPSQ_OK;
    }
    mapsq_table f{};
    if (alloc_table(ctx, (int64_t)total, nc_out, &f)) {
        free_table(ctx, &m);
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, "filtered join result exceeds the arena's free space");
    }
    free_table(ctx, &m);
    const uint64_t blk = f.block;
    meta(out);
    out->block = blk;
    out->nrows = (int64_t)(total / 3);
    for (int c = 0; c < nc_out; c++) out->col[c] = f.col[c];
    return MAPSQ_OK;
}

// A batch in tolerant mode: the joins' scratch together, one output region
// (the largest free block) holding every result that fits in order, shared
// by those results; the others through the plain join.
mapsq_status join_batch(Ctx* ctx, const mapsq_join_desc* d, int32_t n, mapsq_table* outs, mapsq_status* per_join,
                        int64_t* need_rows) {
    std::vector<bool> done(n, false);
    for (int i = 0; i < n; i++) {
        zero(&outs[i]);
        per_join[i] = MAPSQ_OK;
        need_rows[i] = 0;
    }
    uint64_t recs = 0;
    for (int i = 0; i < n; i++) recs += uint64_t(d[i].left->nrows + d[i].right->nrows);
    Block scratch = alloc_block(ctx, size_t(recs) * 24 + 4096);
    if (scratch.ok()) {
        const size_t cap = ctx->arena.largest() / ARENA_ALIGN * ARENA_ALIGN;
        Block region;
        if (cap >= ARENA_ALIGN) region = alloc_block(ctx, cap);
        size_t used = 0;
        uint32_t refs = 0;
        for (int i = 0; i < n && region.ok(); i++) {
            const mapsq_table* L = d[i].left;
            const mapsq_table* R = d[i].right;
            if (L->nrows == 0 || R->nrows == 0) continue;
            bool extra = false;
            int ncols = L->ncols;
            for (int c = 0; c < R->ncols; c++)
                if (R->var[c] != d[i].key_var) {
                    extra = extra || col_of(L, R->var[c]) >= 0;
                    ncols++;
                }
            if (extra || ncols > BATCH_MAXNC) continue;
            const uint64_t total = join_rows(L->nrows, R->nrows, d[i].key_var, L->ncols, R->ncols);
            if (total >= SAT40_HOST) {
                per_join[i] = MAPSQ_ERR_TOO_LARGE;
                need_rows[i] = (int64_t)total;
                done[i] = true;
                continue;
            }
            const size_t bytes = align_up(size_t(total) * 4 * ncols, ARENA_ALIGN);
            if (used + bytes > cap) continue;  // through the plain join below
            mapsq_table& t = outs[i];
            t.ncols = ncols;
            t.var[0] = d[i].key_var;
            int k = 1;
            for (int c = 0; c < L->ncols; c++)
                if (L->var[c] != d[i].key_var) t.var[k++] = L->var[c];
            for (int c = 0; c < R->ncols; c++)
                if (R->var[c] != d[i].key_var) t.var[k++] = R->var[c];
            t.owned = 1;
            t.nrows = (int64_t)total;
            t.key_max = std::max(L->key_max, R->key_max);
            t.sorted_col = 1;
            if (total > 0) {
                t.block = region.off + 1;
                for (int c = 0; c < ncols; c++) t.col[c] = reinterpret_cast<int32_t*>(ctx->arena.ptr(region.off + used));
                used += bytes;
                refs++;
            }
            done[i] = true;
        }
        if (region.ok()) {
            if (refs == 0) {
                region.reset();
            } else {
                ctx->arena.shrink(region.off, used);
                ctx->shared_refs[region.off] = refs;
                region.release();
            }
        }
    }
    scratch.reset();
    for (int i = 0; i < n; i++) {
        if (done[i]) continue;
        mapsq_status st = join_tables(ctx, d[i].left, d[i].right, d[i].key_var, &outs[i]);
        if (st) {
            per_join[i] = st;
            need_rows[i] = ctx->last.out_rows;
            zero(&outs[i]);
        }
    }
    return MAPSQ_OK;
}

}  // namespace mq

// ------------------------------------------------------------- driver ---

namespace {

struct Rng {
    uint64_t s;
    uint64_t next() { return s = mq::mix(s); }
    int64_t below(int64_t n) { return n <= 0 ? 0 : int64_t(next() % uint64_t(n)); }
    double unit() { return double(next() >> 11) / double(1ull << 53); }
};

struct Query {
    std::vector<mapsq_pattern> pats;
};

// 1-5 patterns chained through shared variables, with 0-2 constants each
Query draw_query(Rng& r, const mq::Store& S) {
    Query q;
    const int m = 1 + (int)r.below(5);
    int nvars = 1;
    for (int i = 0; i < m; i++) {
        mapsq_pattern p{};
        const int32_t link = -(1 + (int32_t)r.below(nvars));  // a variable already in the query
        const int32_t fresh = -(1 + nvars);
        const double u = r.unit();
        const int32_t pred = S.preds[size_t(r.below((int64_t)S.preds.size()))];
        const int32_t ent = (int32_t)r.below(1 << 20);
        if (u < 0.45) {  // ?link p ?fresh  or  ?fresh p ?link
            p = r.below(2) ? mapsq_pattern{link, pred, fresh} : mapsq_pattern{fresh, pred, link};
            nvars++;
        } else if (u < 0.8) {  // one constant beside the predicate
            p = r.below(2) ? mapsq_pattern{link, pred, ent} : mapsq_pattern{ent, pred, link};
        } else if (u < 0.9) {  // variable predicate
            p = mapsq_pattern{link, fresh, ent};
            nvars++;
        } else if (u < 0.95) {  // repeated variable
            p = mapsq_pattern{link, pred, link};
        } else {  // shares nothing with the others: a cross product
            p = mapsq_pattern{-(1 + nvars), pred, ent};
            nvars++;
        }
        if (i == 0 && p.s >= 0 && p.o >= 0) p.s = -1;
        q.pats.push_back(p);
    }
    return q;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 8) {
        std::fprintf(stderr, "usage: sim seed nqueries arena_mb budget_permille arrive_every poll_every max_active\n");
        return 2;
    }
    const uint64_t seed = std::strtoull(argv[1], nullptr, 10);
    const int nq = std::atoi(argv[2]);
    const uint64_t arena_bytes = std::strtoull(argv[3], nullptr, 10) << 20;
    const double budget_frac = std::atof(argv[4]) / 1000.0;
    const int arrive_every = std::atoi(argv[5]);  // rounds between arrivals (0: all at once)
    const int poll_every = std::atoi(argv[6]);    // rounds between polls (0: only once nothing is in flight)
    const int max_active = std::atoi(argv[7]);
    const long max_rounds = 200000;

    mq::Ctx ctx;
    ctx.arena.init(reinterpret_cast<char*>(uintptr_t(0x100000000000ull)), arena_bytes);
    Rng r{seed * 7919 + 1};
    mq::Store& S = ctx.store;
    S.loaded = true;
    const int npred = 16 + (int)r.below(48);
    int64_t off = 0;
    S.pred_off.push_back(0);
    for (int i = 0; i < npred; i++) {
        S.preds.push_back(1000000 + i);
        off += 1 + (int64_t)(40000000.0 / (1.0 + i) * r.unit());
        S.pred_off.push_back(off);
        const int64_t sz = S.pred_off.back() - S.pred_off[S.pred_off.size() - 2];
        S.pred_ds.push_back(1 + r.below(sz));
        S.pred_do.push_back(1 + r.below(sz));
    }
    S.n = off;
    S.max_id = (1 << 20) + npred + 1000000;
    S.pso_s = mq::fake_ptr(10);
    S.pso_o = mq::fake_ptr(11);
    S.pos_o = mq::fake_ptr(12);
    S.pos_s = mq::fake_ptr(13);
    // the store's own share of the arena
    const size_t store_off = ctx.arena.alloc(std::min<uint64_t>(arena_bytes / 8, uint64_t(S.n) * 4));
    const size_t free0 = ctx.arena.free_bytes();

    std::vector<Query> qs;
    for (int i = 0; i < nq; i++) qs.push_back(draw_query(r, S));
    // every query alone
    std::vector<int> st_alone(nq), st_served(nq, 1);
    std::vector<int64_t> rows_alone(nq, -1), rows_served(nq, -1);
    const char* trace = std::getenv("SIM_TRACE");
    for (int i = 0; i < nq; i++) {
        mapsq_table t{};
        st_alone[i] = mq::query(&ctx, qs[i].pats.data(), (int32_t)qs[i].pats.size(), nullptr, 0, &t);
        if (trace && std::atoi(trace) == i) {
            std::fprintf(stderr, "query %d alone: status %d (%s); patterns", i, st_alone[i], ctx.err.c_str());
            for (auto& p : qs[i].pats) std::fprintf(stderr, " (%d %d %d)", p.s, p.p, p.o);
            std::fprintf(stderr, "\n");
        }
        if (!st_alone[i]) {
            rows_alone[i] = t.nrows;
            mq::free_table(&ctx, &t);
        }
    }
    const size_t free_alone = ctx.arena.free_bytes();
    // all of them served
    mq::serve_config(&ctx, (uint64_t)(budget_frac * (double)free0), max_active);
    std::vector<uint64_t> ticket(nq, 0);
    int submitted = 0, ended = 0, step_errors = 0;
    long rounds = 0;
    std::vector<mapsq_table> held;
    auto poll_all = [&]() {
        for (;;) {
            uint64_t tk = 0;
            int32_t done = 0;
            mapsq_table t{};
            const mapsq_status st = mq::poll_next(&ctx, &tk, &done, &t);
            if (!tk) break;
            const int j = int(std::find(ticket.begin(), ticket.end(), tk) - ticket.begin());
            st_served[j] = st;
            if (trace && std::atoi(trace) == j)
                std::fprintf(stderr, "query %d served: status %d (%s) at round %ld\n", j, st, st ? ctx.err.c_str() : "",
                             rounds);
            if (!st) {
                rows_served[j] = t.nrows;
                mq::free_table(&ctx, &t);
            }
            ended++;
        }
    };
    while (ended < nq && rounds < max_rounds) {
        if (submitted < nq && (arrive_every == 0 || rounds % arrive_every == 0)) {
            const int k = arrive_every == 0 ? nq : 1 + (int)r.below(3);
            for (int a = 0; a < k && submitted < nq; a++, submitted++)
                if (mq::submit(&ctx, qs[submitted].pats.data(), (int32_t)qs[submitted].pats.size(), nullptr, 0,
                               &ticket[submitted])) {
                    st_served[submitted] = -100;  // refused at submission
                    ended++;
                }
        }
        int32_t active = 0, waiting = 0;
        if (mq::serve_step(&ctx, &active, &waiting)) step_errors++;
        rounds++;
        const bool idle = active == 0 && waiting == 0;
        if ((poll_every > 0 && rounds % poll_every == 0) || idle) poll_all();
    }
    poll_all();
    mq::destroy_server(&ctx);
    const size_t free_end = ctx.arena.free_bytes();
    ctx.arena.free(store_off);
    std::printf("{\"seed\": %" PRIu64 ", \"rounds\": %ld, \"terminated\": %s, \"step_errors\": %d, \"free0\": %zu, "
                "\"free_alone\": %zu, \"free_end\": %zu, \"alone\": [",
                seed, rounds, ended >= nq ? "true" : "false", step_errors, free0, free_alone, free_end);
    for (int i = 0; i < nq; i++) std::printf("%s[%d, %" PRId64 "]", i ? ", " : "", st_alone[i], rows_alone[i]);
    std::printf("], \"served\": [");
    for (int i = 0; i < nq; i++) std::printf("%s[%d, %" PRId64 "]", i ? ", " : "", st_served[i], rows_served[i]);
    std::printf("]}\n");
    return 0;
}
