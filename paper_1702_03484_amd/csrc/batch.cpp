// Host side of mapsq_join_batch: lays the joins' records out in whole record
// tiles, uploads one device header and the per-join descriptors, replays a
// cached hipGraph of the batched kernels (captured on first use per digit
// width, tile size and pass count), synchronises once, and turns the
// device-placed results into tables.  Joins outside the batched kernels'
// scope, and results that did not fit the output region, go through the
// plain path afterwards.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "runtime.h"

namespace mq {

#define HIPCHK_B(x)                                                                                   \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) return ctx->fail(MAPSQ_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

void Ctx::release_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
}

bool ensure_stage(Ctx* ctx, size_t bytes) {
    if (bytes <= ctx->stage_bytes) return true;
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    ctx->stage = nullptr;
    ctx->stage_bytes = 0;
    size_t want = std::max(bytes, size_t(1) << 20);
    if (hipHostMalloc(&ctx->stage, want, hipHostMallocDefault) != hipSuccess) return false;
    ctx->stage_bytes = want;
    return true;
}

namespace {
struct Plan {
    int idx;             // position in the caller's array
    bool batched;        // runs in the batched kernels
    bool empty;          // one side has no rows
    int lk, rk;          // key columns
    std::vector<int> lv, rv;  // value columns
};
}  // namespace

mapsq_status join_batch(Ctx* ctx, const mapsq_join_desc* d, int32_t n, mapsq_table* outs,
                        mapsq_status* per_join, int64_t* need_rows) {
    if (n < 0 || (n > 0 && (!d || !outs))) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "bad batch arguments");
    for (int i = 0; i < n; i++) std::memset(&outs[i], 0, sizeof(mapsq_table));
    if (per_join)
        for (int i = 0; i < n; i++) per_join[i] = MAPSQ_OK;
    if (need_rows)
        for (int i = 0; i < n; i++) need_rows[i] = 0;
    if (n == 0) return MAPSQ_OK;
    std::vector<Plan> plan(n);
    int32_t kmax = 0;
    bool known = true;
    std::vector<bool> invalid(n, false);
    for (int i = 0; i < n; i++) {
        mapsq_status st;
        Plan& p = plan[i];
        p.idx = i;
        p.batched = false;
        p.empty = false;
        if ((st = check_table(ctx, d[i].left, "left")) || (st = check_table(ctx, d[i].right, "right"))) {
            if (!per_join) return st;
            per_join[i] = st;  // tolerant mode: this join fails alone
            invalid[i] = true;
            continue;
        }
        const mapsq_table* L = d[i].left;
        const mapsq_table* R = d[i].right;
        p.lk = col_of(L, d[i].key_var);
        p.rk = col_of(R, d[i].key_var);
        if (p.lk < 0 || p.rk < 0) {
            if (!per_join)
                return ctx->fail(MAPSQ_ERR_INVALID_ARG, "join " + std::to_string(i) + ": key variable not bound on both sides");
            per_join[i] = MAPSQ_ERR_INVALID_ARG;
            invalid[i] = true;
            continue;
        }
        bool extra = false;
        for (int c = 0; c < L->ncols; c++)
            if (c != p.lk) p.lv.push_back(c);
        for (int c = 0; c < R->ncols; c++) {
            if (c == p.rk) continue;
            if (col_of(L, R->var[c]) >= 0) extra = true;
            p.rv.push_back(c);
        }
        p.empty = L->nrows == 0 || R->nrows == 0;
        p.batched = !extra && 1 + p.lv.size() + p.rv.size() <= (size_t)BATCH_MAXNC;
        if (p.batched && !p.empty) {
            if (L->key_max < 0 || R->key_max < 0) known = false;
            kmax = std::max(kmax, std::max(L->key_max, R->key_max));
        }
    }
    // A join with an unknown key bound may hold any int32 key: its keys are
    // sorted as k - INT32_MIN (the sign bit flipped), which keeps their
    // signed order over the full 32 bits; joins with a bound sort k itself.
    const int key_bits = known ? bitlen((uint32_t)kmax) : 32;
    uint64_t all_rec = 0;
    for (int i = 0; i < n; i++)
        if (plan[i].batched && !plan[i].empty) all_rec += (uint64_t)d[i].left->nrows + (uint64_t)d[i].right->nrows;
    int rb, kpt;
    pick_tuning(ctx, key_bits, rb, kpt, all_rec);
    // Unless set explicitly, 32 keys per thread (8,192-record tiles): every
    // batched kernel's cost grows with its tiles' look-backs more than with
    // its records, and half the tiles took the 512-join workload's two
    // launches from 67.9 to 62.1 ms.
    if (!ctx->tune_kpt) kpt = 32;
    const int passes = std::max(1, (key_bits + rb - 1) / rb);
    const uint32_t TILE = BLOCK_THREADS * (uint32_t)kpt;  // records per tile
    const size_t buckets = size_t(1) << rb;

    // record tiles of the batched, non-empty joins
    std::vector<BatchJoin> J(n);
    std::vector<uint32_t> tile_join;
    uint64_t tiles = 0;
    for (int i = 0; i < n; i++) {
        std::memset(&J[i], 0, sizeof(BatchJoin));
        const Plan& p = plan[i];
        if (!p.batched || invalid[i]) continue;
        const mapsq_table* L = d[i].left;
        const mapsq_table* R = d[i].right;
        BatchJoin& b = J[i];
        b.lkey = L->col[p.lk];
        b.rkey = R->col[p.rk];
        b.key_base = (L->key_max < 0 || R->key_max < 0) ? INT32_MIN : 0;
        b.nvl = (int)p.lv.size();
        b.nvr = (int)p.rv.size();
        for (int c = 0; c < b.nvl; c++) b.lcol[c] = L->col[p.lv[c]];
        for (int c = 0; c < b.nvr; c++) b.rcol[c] = R->col[p.rv[c]];
        if (p.empty) continue;
        b.nl = (uint32_t)L->nrows;
        b.nr = (uint32_t)R->nrows;
        b.nrec = b.nl + b.nr;  // a filtered join's kept count is set on the device
        if ((uint64_t)b.nl + b.nr >= (1ull << 32)) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a join with 2^32 records");
        b.ntiles = (uint32_t)((uint64_t(b.nl) + b.nr + TILE - 1) / TILE);
        b.tile_off = (uint32_t)tiles;
        b.rec_off = (uint32_t)(tiles * TILE);
        tiles += b.ntiles;
        if (tiles * TILE >= (1ull << 32)) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a batch of 2^32 records or more");
        tile_join.insert(tile_join.end(), b.ntiles, (uint32_t)i);
    }
    const uint64_t nrec = tiles * TILE;
    // Semi-join filters: automatic for joins whose larger side has at least
    // twice the smaller side's rows (the probed side is the larger one),
    // every join with semijoin = 2, none with semijoin = 1.  16 bits per
    // build-side row, at least 64 words.
    std::vector<uint64_t> filt_at(n, 0);
    uint64_t filt_words = 0;
    for (int i = 0; i < n; i++) {
        BatchJoin& b = J[i];
        if (!plan[i].batched || invalid[i] || plan[i].empty || ctx->semijoin == 1) continue;
        const uint32_t small = std::min(b.nl, b.nr), big = std::max(b.nl, b.nr);
        if (ctx->semijoin == 0 && (uint64_t)big < 2ull * small) continue;
        uint64_t words = 64;
        while (words < (uint64_t(small) + 3) / 4) words <<= 1;
        b.fmask = (uint32_t)(words - 1);
        b.probe_right = b.nr > b.nl ? 1u : 0u;
        b.nrec = 0;
        filt_at[i] = filt_words + 1;  // the pointer is set once the scratch exists
        filt_words += words;
    }

    std::vector<mapsq_table> res(n);
    std::vector<bool> done(invalid);
    mapsq_join_stats bst{};  // sums over the joins the batched kernels ran
    bst.path = MAPSQ_PATH_SORT;
    bool batched_any = false;
    auto fail_all = [&](mapsq_status code, const std::string& msg) {
        for (int i = 0; i < n; i++) {
            free_table(ctx, &res[i]);
            std::memset(&outs[i], 0, sizeof(mapsq_table));
        }
        return ctx->fail(code, msg);
    };
    auto meta = [&](int i, mapsq_table* t) {
        const mapsq_table* L = d[i].left;
        const mapsq_table* R = d[i].right;
        const Plan& p = plan[i];
        t->ncols = 1 + (int)p.lv.size() + (int)p.rv.size();
        t->var[0] = d[i].key_var;
        int k = 1;
        for (int c : p.lv) t->var[k++] = L->var[c];
        for (int c : p.rv) t->var[k++] = R->var[c];
        t->key_max = (L->key_max >= 0 && R->key_max >= 0) ? std::max(L->key_max, R->key_max) : -1;
        t->sorted_col = 1;  // grouped by ascending key
    };

    if (tiles > 0) {
        // scratch: sort ping-pong (16 B/record; the spare pair later holds
        // segment starts and splits) and segment offsets (8 B/record)
        const size_t nb4 = align_up(nrec * 4, ARENA_ALIGN);
        const size_t hist_bytes = align_up(size_t(n) * passes * buckets * 4, ARENA_ALIGN);
        const size_t tj_bytes = align_up(tiles * 4, ARENA_ALIGN);
        const size_t jd_bytes = align_up(sizeof(BatchJoin) * n, ARENA_ALIGN);
        const size_t filt_bytes = align_up(filt_words * 8, ARENA_ALIGN);
        Block scratch = alloc_block(ctx, nb4 * 6 + hist_bytes + tj_bytes + jd_bytes + filt_bytes);
        bool room = scratch.ok() && ctx->ensure_status(size_t(tiles) * buckets);
        if (room && ctx->bhdr_off == SIZE_MAX) {
            ctx->bhdr_off = ctx->arena.alloc(sizeof(BatchHdr));
            room = ctx->bhdr_off != SIZE_MAX;
            if (room) ctx->bhdr = reinterpret_cast<BatchHdr*>(ctx->arena.ptr(ctx->bhdr_off));
        }
        if (!room) {
            if (!per_join) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the batch scratch");
            // tolerant mode: every join goes through the plain path below
            goto plain_rest;
        }
        char* sb = ctx->arena.ptr(scratch.off);
        // value columns in sorted record order (joins with more output rows
        // than records use them); without room, materialisation gathers
        uint32_t nsval = 0;
        for (int i = 0; i < n; i++)
            if (plan[i].batched && !plan[i].empty)
                nsval = std::max(nsval, (uint32_t)std::max(J[i].nvl, J[i].nvr));
        Block svb;
        if (nsval) svb = alloc_block(ctx, nb4 * nsval);
        if (!svb.ok()) nsval = 0;
        // the output region: the largest free block that is left
        const size_t cap_bytes = ctx->arena.largest() / ARENA_ALIGN * ARENA_ALIGN;
        Block region;
        if (cap_bytes >= ARENA_ALIGN) region = alloc_block(ctx, cap_bytes);
        BatchHdr H{};
        H.joins = reinterpret_cast<BatchJoin*>(sb + nb4 * 6 + hist_bytes + tj_bytes);
        H.tile_join = reinterpret_cast<const uint32_t*>(sb + nb4 * 6 + hist_bytes);
        H.njoins = (uint32_t)n;
        H.total_tiles = (uint32_t)tiles;
        H.passes = (uint32_t)passes;
        // epochs: one per radix pass, heads, counts, the semi-join compaction
        if (ctx->epoch + passes + 3 >= (1u << 22)) {
            (void)launch_fill_u64(ctx->status, ctx->status_words, 0ull, ctx->stream);
            ctx->epoch = 0;
        }
        H.epoch0 = ctx->epoch + 1;
        ctx->epoch += passes + 3;
        for (int k = 0; k < 2; k++) {
            H.keys[k] = reinterpret_cast<uint32_t*>(sb + nb4 * k);
            H.vals[k] = reinterpret_cast<uint32_t*>(sb + nb4 * (2 + k));
        }
        H.seg_off = reinterpret_cast<uint64_t*>(sb + nb4 * 4);
        H.hist = reinterpret_cast<uint32_t*>(sb + nb4 * 6);
        H.ctr = ctx->small + SMALL_CTR;
        H.status = ctx->status;
        H.out_base = region.ok() ? region.as<int32_t>() : nullptr;
        H.nsval = nsval;
        for (uint32_t c = 0; c < nsval; c++)
            H.sval[c] = reinterpret_cast<int32_t*>(ctx->arena.ptr(svb.off) + c * nb4);
        H.out_cap_words = region.ok() ? cap_bytes / 4 : 0;
        H.filt = reinterpret_cast<uint64_t*>(sb + nb4 * 6 + hist_bytes + tj_bytes + jd_bytes);
        H.filt_words = filt_words;
        for (int i = 0; i < n; i++)
            if (filt_at[i]) J[i].filt = H.filt + (filt_at[i] - 1);
        // upload header, descriptors and the tile map through pinned staging
        const size_t up = sizeof(BatchHdr) + sizeof(BatchJoin) * n + tiles * 4;
        if (!ensure_stage(ctx, up)) return ctx->fail(MAPSQ_ERR_HIP, "pinned staging allocation failed");
        char* stg = reinterpret_cast<char*>(ctx->stage);
        std::memcpy(stg, &H, sizeof(BatchHdr));
        std::memcpy(stg + sizeof(BatchHdr), J.data(), sizeof(BatchJoin) * n);
        std::memcpy(stg + sizeof(BatchHdr) + sizeof(BatchJoin) * n, tile_join.data(), tiles * 4);
        HIPCHK_B(hipMemcpyAsync(ctx->bhdr, stg, sizeof(BatchHdr), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK_B(hipMemcpyAsync(H.joins, stg + sizeof(BatchHdr), sizeof(BatchJoin) * n, hipMemcpyHostToDevice,
                                ctx->stream));
        HIPCHK_B(hipMemcpyAsync(const_cast<uint32_t*>(H.tile_join), stg + sizeof(BatchHdr) + sizeof(BatchJoin) * n,
                                tiles * 4, hipMemcpyHostToDevice, ctx->stream));
        // launch: a cached graph when the stream can be captured
        const int ph = ctx->prof_begin(6);
        const uint64_t gkey = (uint64_t)rb | ((uint64_t)kpt << 8) | ((uint64_t)passes << 16);
        const char* env = std::getenv("MAPSQ_BATCH_GRAPH");
        const bool graph = ctx->use_graph && ctx->stream != nullptr && !(env && env[0] == '0');
        if (graph) {
            auto it = ctx->graphs.find(gkey);
            if (it == ctx->graphs.end()) {
                hipGraph_t g = nullptr;
                hipGraphExec_t ge = nullptr;
                HIPCHK_B(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
                hipError_t le = launch_batch(ctx->bhdr, rb, kpt, passes, ctx->stream);
                hipError_t ce = hipStreamEndCapture(ctx->stream, &g);
                if (le != hipSuccess || ce != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return ctx->fail(MAPSQ_ERR_HIP, std::string("batch capture: ") +
                                                        hipGetErrorString(le != hipSuccess ? le : ce));
                }
                hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) return ctx->fail(MAPSQ_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
                it = ctx->graphs.emplace(gkey, ge).first;
            }
            HIPCHK_B(hipGraphLaunch(it->second, ctx->stream));
        } else {
            HIPCHK_B(launch_batch(ctx->bhdr, rb, kpt, passes, ctx->stream));
        }
        // read back the placed results (the one synchronisation of the batch)
        const size_t down = sizeof(BatchHdr) + sizeof(BatchJoin) * n;
        HIPCHK_B(hipMemcpyAsync(stg, ctx->bhdr, sizeof(BatchHdr), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK_B(hipMemcpyAsync(stg + sizeof(BatchHdr), H.joins, sizeof(BatchJoin) * n, hipMemcpyDeviceToHost,
                                ctx->stream));
        HIPCHK_B(hipStreamSynchronize(ctx->stream));
        (void)down;
        BatchHdr Hr;
        std::memcpy(&Hr, stg, sizeof(BatchHdr));
        std::memcpy(J.data(), stg + sizeof(BatchHdr), sizeof(BatchJoin) * n);
        {
            double bytes = 0;
            for (int i = 0; i < n; i++) {
                const BatchJoin& b = J[i];
                if (!plan[i].batched || plan[i].empty) continue;
                // unfiltered: histogram and first pass read every key, the
                // first pass writes N records and later passes move them;
                // filtered: the filter's side read once to build it, every
                // key read once by the compaction, which writes the N kept
                // records; the histogram reads their keys, and every pass
                // moves them; then heads and counts over the N records
                const double all = double(b.nl) + b.nr;
                const double N = b.nrec;
                if (b.filt)
                    bytes += 4.0 * (b.probe_right ? b.nl : b.nr) + 4.0 * all + 8.0 * N + 4.0 * N + 16.0 * N * passes;
                else
                    bytes += 8.0 * all + 8.0 * N + 16.0 * N * (passes - 1);
                bytes += 8.0 * N + 28.0 * b.nseg;
                if (b.status == 0) {
                    const double cells = b.nvl * double(b.nl) + b.nvr * double(b.nr);
                    const uint32_t nv = (uint32_t)std::max(b.nvl, b.nvr);
                    bytes += 4.0 * (1 + b.nvl + b.nvr) * double(b.total) + 4.0 * N + 20.0 * b.nseg + 4.0 * cells;
                    if (nv && nv <= nsval && double(b.total) >= N)  // the sorted-order copy of the values
                        bytes += 4.0 * cells + 4.0 * nv * N;
                }
                ctx->acc.rows_out += (int64_t)b.total;
                ctx->acc.joins += 1;
                bst.left_rows += b.nl;
                bst.right_rows += b.nr;
                bst.segments += b.nseg;
                bst.out_rows += (int64_t)b.total;
                bst.sorted_records += b.nrec;
                if (b.filt) bst.path = MAPSQ_PATH_SEMIJOIN;
                batched_any = true;
            }
            ctx->prof_end(ph, bytes);
            bst.radix_bits = rb;
            bst.passes = passes;
            bst.key_bits = key_bits;
        }
        for (int i = 0; i < n; i++)
            if (plan[i].batched && !plan[i].empty && J[i].status == 2) {
                if (!per_join) return ctx->fail(MAPSQ_ERR_TOO_LARGE, "join " + std::to_string(i) + ": over 2^40 rows");
                per_join[i] = MAPSQ_ERR_TOO_LARGE;
                if (need_rows) need_rows[i] = (int64_t)J[i].total;
                done[i] = true;
            }
        // results in the output region share its block
        const size_t used = size_t(Hr.out_used_words) * 4;
        uint32_t refs = 0;
        for (int i = 0; i < n; i++) {
            const BatchJoin& b = J[i];
            if (!plan[i].batched || plan[i].empty || done[i]) continue;
            if (b.status != 0) continue;
            mapsq_table& t = res[i];
            meta(i, &t);
            t.owned = 1;
            t.nrows = (int64_t)b.total;
            if (b.total > 0) {
                t.block = region.off + 1;
                for (int c = 0; c < t.ncols; c++)
                    t.col[c] = region.as<int32_t>() + b.out_word + (uint64_t)c * b.col_words;
                refs++;
            }
            done[i] = true;
        }
        if (region.ok()) {
            if (refs == 0 || used == 0) {
                region.reset();
                for (int i = 0; i < n; i++) res[i].block = 0;
            } else {
                ctx->arena.shrink(region.off, used);
                ctx->shared_refs[region.off] = refs;
                region.release();
            }
        }
    }
plain_rest:
    // empty joins, and the joins the batched kernels did not take
    for (int i = 0; i < n; i++) {
        if (done[i]) continue;
        if (plan[i].batched && plan[i].empty) {
            meta(i, &res[i]);
            res[i].owned = 1;
            res[i].nrows = 0;
            done[i] = true;
            continue;
        }
        mapsq_status st = join_tables(ctx, d[i].left, d[i].right, d[i].key_var, &res[i]);
        if (st) {
            std::string msg = ctx->err;
            if (!per_join) return fail_all(st, "join " + std::to_string(i) + ": " + msg);
            per_join[i] = st;
            if (need_rows) need_rows[i] = ctx->last.out_rows;
            std::memset(&res[i], 0, sizeof(mapsq_table));
        }
        done[i] = true;
    }
    for (int i = 0; i < n; i++) outs[i] = res[i];
    if (batched_any) ctx->last = bst;
    return MAPSQ_OK;
}

}  // namespace mq
