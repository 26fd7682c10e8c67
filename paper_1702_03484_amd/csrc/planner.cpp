// Host planner of mapsq_query: the CPU side of the paper's CPU/GPU
// coprocessing (abstract; Section 2: partial matching per pattern, then
// pattern-by-pattern merging of the partial results on a shared variable).
// The host maps every pattern (exact partial-match sizes come back from the
// index ranges), orders the joins greedily and hands each one to the GPU.
#include <algorithm>
#include <cstring>

#include "runtime.h"

namespace mq {

// Internal variable of the constant key that turns a cross product into a
// one-segment join (user variables are >= 0).
constexpr int32_t CROSS_VAR = INT32_MIN + 7;

static bool binds(const mapsq_table& t, int32_t v) {
    for (int c = 0; c < t.ncols; c++)
        if (t.var[c] == v) return true;
    return false;
}

// Table with one extra all-zero column bound to CROSS_VAR (owned scratch).
static mapsq_status with_zero_key(Ctx* ctx, const mapsq_table& t, mapsq_table* out, Block* zeros) {
    if (t.ncols >= MAPSQ_MAX_COLS) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 16 columns");
    *zeros = alloc_block(ctx, size_t(std::max<int64_t>(t.nrows, 1)) * 4);
    if (!zeros->ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for a cross-product key");
    hipError_t e = launch_fill_u32(zeros->as<uint32_t>(), (uint64_t)t.nrows, 0u, ctx->stream);
    if (e != hipSuccess) return ctx->fail(MAPSQ_ERR_HIP, "fill failed");
    *out = t;
    out->owned = 0;
    out->block = 0;
    out->var[t.ncols] = CROSS_VAR;
    out->col[t.ncols] = zeros->as<int32_t>();
    out->ncols = t.ncols + 1;
    out->key_max = std::max(t.key_max, 0);
    if (t.key_max < 0) out->key_max = -1;
    return MAPSQ_OK;
}

mapsq_status query(Ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                   mapsq_table* out) {
    std::memset(out, 0, sizeof(*out));
    if (!pats || npats < 1 || npats > 64) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "npats must be in [1, 64]");
    if (nsel < 0 || (nsel > 0 && !sel)) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "bad select list");
    if (!ctx->store.loaded) return ctx->fail(MAPSQ_ERR_STATE, "no store loaded");
    // query variables in first-appearance order
    std::vector<int32_t> qvars;
    for (int i = 0; i < npats; i++) {
        const int32_t t[3] = {pats[i].s, pats[i].p, pats[i].o};
        bool any = false;
        for (int k = 0; k < 3; k++)
            if (t[k] < 0) {
                any = true;
                int32_t v = -t[k] - 1;
                if (std::find(qvars.begin(), qvars.end(), v) == qvars.end()) qvars.push_back(v);
            }
        if (!any) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a triple pattern without variables");
    }
    std::vector<int32_t> want;
    if (nsel == 0) {
        want = qvars;
    } else {
        for (int i = 0; i < nsel; i++) {
            if (std::find(qvars.begin(), qvars.end(), sel[i]) == qvars.end())
                return ctx->fail(MAPSQ_ERR_INVALID_ARG, "a selected variable is not in the query");
            if (std::find(want.begin(), want.end(), sel[i]) != want.end())
                return ctx->fail(MAPSQ_ERR_INVALID_ARG, "a variable is selected twice");
            want.push_back(sel[i]);
        }
    }
    if ((int)want.size() > MAPSQ_MAX_COLS) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 16 variables");

    // partial matching of every pattern
    std::vector<mapsq_table> tabs(npats);
    std::vector<bool> used(npats, false);
    auto cleanup = [&]() {
        for (int i = 0; i < npats; i++)
            if (!used[i]) free_table(ctx, &tabs[i]);
    };
    for (int i = 0; i < npats; i++) {
        mapsq_status st = map_pattern(ctx, &pats[i], -1, &tabs[i]);
        if (st) {
            for (int j = 0; j < i; j++) free_table(ctx, &tabs[j]);
            return st;
        }
    }
    // greedy order: start from the smallest table; next, the smallest table
    // connected to the bound variables (ties: lowest pattern index)
    int start = 0;
    for (int i = 1; i < npats; i++)
        if (tabs[i].nrows < tabs[start].nrows) start = i;
    mapsq_table cur = tabs[start];
    used[start] = true;
    for (int step = 1; step < npats; step++) {
        int pick = -1;
        bool connected = false;
        for (int i = 0; i < npats; i++) {
            if (used[i]) continue;
            bool con = false;
            for (int c = 0; c < tabs[i].ncols; c++) con = con || binds(cur, tabs[i].var[c]);
            if (pick < 0 || (con && !connected) || (con == connected && tabs[i].nrows < tabs[pick].nrows)) {
                pick = i;
                connected = con;
            }
        }
        mapsq_table nxt{};
        mapsq_status st;
        if (connected) {
            int32_t key = -1;
            for (int32_t v : qvars)
                if (binds(cur, v) && binds(tabs[pick], v)) {
                    key = v;
                    break;
                }
            st = join_tables(ctx, &cur, &tabs[pick], key, &nxt);
        } else {
            mapsq_table a{}, b{};
            Block za, zb;
            st = with_zero_key(ctx, cur, &a, &za);
            if (!st) st = with_zero_key(ctx, tabs[pick], &b, &zb);
            if (!st) st = join_tables(ctx, &a, &b, CROSS_VAR, &nxt);
            if (!st) {
                // drop the constant key column (column 0)
                for (int c = 1; c < nxt.ncols; c++) {
                    nxt.var[c - 1] = nxt.var[c];
                    nxt.col[c - 1] = nxt.col[c];
                }
                nxt.ncols -= 1;
                nxt.col[nxt.ncols] = nullptr;
                nxt.key_max = (cur.key_max >= 0 && tabs[pick].key_max >= 0)
                                  ? std::max(cur.key_max, tabs[pick].key_max)
                                  : -1;
            }
        }
        if (st) {
            free_table(ctx, &cur);
            cleanup();
            return st;
        }
        free_table(ctx, &cur);
        free_table(ctx, &tabs[pick]);
        used[pick] = true;
        cur = nxt;
    }
    // projection (bag): pick the selected columns in the requested order
    mapsq_table res = cur;
    for (size_t i = 0; i < want.size(); i++) {
        int c = -1;
        for (int k = 0; k < cur.ncols; k++)
            if (cur.var[k] == want[i]) c = k;
        res.var[i] = want[i];
        res.col[i] = cur.col[c];
    }
    for (size_t i = want.size(); i < MAPSQ_MAX_COLS; i++) {
        res.var[i] = 0;
        res.col[i] = nullptr;
    }
    res.ncols = (int32_t)want.size();
    *out = res;
    return MAPSQ_OK;
}

}  // namespace mq
