// Host planner of mapsq_query: the CPU side of the paper's CPU/GPU
// coprocessing (abstract; Section 2: partial matching per pattern, then
// pattern-by-pattern merging of the partial results on a shared variable).
// The host maps every pattern (exact partial-match sizes come back from the
// index ranges), orders the joins greedily -- on those pattern sizes, or on
// exact join sizes that the GPU counts for every candidate step -- and hands
// each join to the GPU.
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

// Greedy join order (the host's share of the CPU/GPU split): start from the
// smallest table, then repeatedly take the smallest table that shares a
// variable with the bound ones (ties: lowest index), joining on the first
// shared variable in the query's first-appearance order; a table sharing
// nothing joins by cross product.
void greedy_plan(const std::vector<std::vector<int32_t>>& vars, const std::vector<int64_t>& rows,
                 const std::vector<int32_t>& qvars, int* start, std::vector<PlanStep>* steps) {
    const int m = (int)vars.size();
    *start = 0;
    for (int i = 1; i < m; i++)
        if (rows[i] < rows[*start]) *start = i;
    std::vector<int32_t> bound = vars[*start];
    std::vector<bool> used(m, false);
    used[*start] = true;
    steps->clear();
    auto has = [](const std::vector<int32_t>& vs, int32_t v) { return std::find(vs.begin(), vs.end(), v) != vs.end(); };
    for (int step = 1; step < m; step++) {
        int pick = -1;
        bool connected = false;
        for (int i = 0; i < m; i++) {
            if (used[i]) continue;
            bool con = false;
            for (int32_t v : vars[i]) con = con || has(bound, v);
            if (pick < 0 || (con && !connected) || (con == connected && rows[i] < rows[pick])) {
                pick = i;
                connected = con;
            }
        }
        PlanStep ps{pick, -1, !connected};
        if (connected)
            for (int32_t v : qvars)
                if (has(bound, v) && has(vars[pick], v)) {
                    ps.key = v;
                    break;
                }
        for (int32_t v : vars[pick])
            if (!has(bound, v)) bound.push_back(v);
        used[pick] = true;
        steps->push_back(ps);
    }
}

mapsq_status cross_join(Ctx* ctx, const mapsq_table& a, const mapsq_table& b, mapsq_table* out);

// Each pattern's variables (first occurrence order) with their distinct
// counts: a subject or object variable of a constant predicate takes the
// predicate's distinct subjects or objects (at most the pattern's rows),
// anything else the rows.  A join keeps |L| |R| / max(distinct keys) rows,
// a cross product |L| |R|; after a step every distinct count is capped by
// its rows (System-R style).
std::vector<double> estimate_steps(const Ctx* ctx, const mapsq_pattern* pats, const std::vector<int64_t>& rows,
                                   int start, const std::vector<PlanStep>& steps, double* scan_bytes,
                                   std::vector<size_t>* out_cols) {
    const Store& St = ctx->store;
    const size_t m = rows.size();
    std::vector<std::vector<int32_t>> vars(m);
    std::vector<std::vector<double>> dist(m);
    double scans = 0;
    for (size_t i = 0; i < m; i++) {
        const mapsq_pattern& p = pats[i];
        const int32_t t[3] = {p.s, p.p, p.o};
        double ds = (double)rows[i], dob = (double)rows[i];
        if (p.p >= 0 && St.pred_ds.size() == St.preds.size()) {
            auto it = std::lower_bound(St.preds.begin(), St.preds.end(), p.p);
            if (it != St.preds.end() && *it == p.p) {
                const size_t pi = size_t(it - St.preds.begin());
                ds = std::min(ds, (double)St.pred_ds[pi]);
                dob = std::min(dob, (double)St.pred_do[pi]);
            }
        }
        for (int k = 0; k < 3; k++)
            if (t[k] < 0) {
                const int32_t v = -t[k] - 1;
                if (std::find(vars[i].begin(), vars[i].end(), v) != vars[i].end()) continue;
                vars[i].push_back(v);
                dist[i].push_back(k == 0 ? ds : (k == 2 ? dob : (double)rows[i]));
            }
        const bool scan = p.p < 0 || (p.s < 0 && (p.s == p.p || p.s == p.o)) || (p.p < 0 && p.p == p.o);
        if (scan) scans += 4.0 * vars[i].size() * (double)rows[i];
    }
    if (scan_bytes) *scan_bytes = scans;
    std::vector<double> est_rows;
    double cur_rows = (double)rows[start];
    std::vector<int32_t> cv = vars[start];
    std::vector<double> cd = dist[start];
    for (const PlanStep& ps : steps) {
        const double r2 = (double)rows[ps.pick];
        double est;
        if (ps.cross) {
            est = cur_rows * r2;
        } else {
            double d1 = 1, d2 = 1;
            for (size_t k = 0; k < cv.size(); k++)
                if (cv[k] == ps.key) d1 = cd[k];
            for (size_t k = 0; k < vars[ps.pick].size(); k++)
                if (vars[ps.pick][k] == ps.key) d2 = dist[ps.pick][k];
            est = cur_rows * r2 / std::max(1.0, std::max(d1, d2));
        }
        for (size_t k = 0; k < vars[ps.pick].size(); k++)
            if (std::find(cv.begin(), cv.end(), vars[ps.pick][k]) == cv.end()) {
                cv.push_back(vars[ps.pick][k]);
                cd.push_back(dist[ps.pick][k]);
            }
        for (double& d : cd) d = std::min(d, est);
        est_rows.push_back(est);
        if (out_cols) out_cols->push_back(cv.size());
        cur_rows = est;
    }
    return est_rows;
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
    out->sorted_col = t.ncols + 1;  // a constant column is in order: the join pairs the two runs directly
    return MAPSQ_OK;
}

// Cartesian product as a join on a constant key (one segment); the key
// column is dropped from the result.
mapsq_status cross_join(Ctx* ctx, const mapsq_table& cur, const mapsq_table& other, mapsq_table* nxt) {
    // the size is exact before anything runs: refuse what cannot fit
    const uint64_t total = (uint64_t)std::max<int64_t>(cur.nrows, 0) * (uint64_t)std::max<int64_t>(other.nrows, 0);
    ctx->last = mapsq_join_stats{};
    ctx->last.out_rows = (int64_t)std::min<uint64_t>(total, SAT40_HOST);
    if (total >= SAT40_HOST) return ctx->fail(MAPSQ_ERR_TOO_LARGE, "cross product exceeds 2^40 rows");
    const double need = (double)align_up(size_t(total) * 4, ARENA_ALIGN) * (1 + cur.ncols + other.ncols);
    if (need > (double)ctx->arena.free_bytes())
        return ctx->fail(MAPSQ_ERR_TOO_LARGE,
                         "cross product (" + std::to_string(total) + " rows) exceeds the arena's free space");
    mapsq_table a{}, b{};
    Block za, zb;
    mapsq_status st = with_zero_key(ctx, cur, &a, &za);
    if (!st) st = with_zero_key(ctx, other, &b, &zb);
    if (!st) st = join_tables(ctx, &a, &b, CROSS_VAR, nxt);
    if (st) return st;
    for (int c = 1; c < nxt->ncols; c++) {
        nxt->var[c - 1] = nxt->var[c];
        nxt->col[c - 1] = nxt->col[c];
    }
    nxt->ncols -= 1;
    nxt->col[nxt->ncols] = nullptr;
    nxt->key_max = (cur.key_max >= 0 && other.key_max >= 0) ? std::max(cur.key_max, other.key_max) : -1;
    nxt->sorted_col = 0;
    return MAPSQ_OK;
}

// The columns of `cur` picked in the order of `want` (a bag projection; the
// table keeps its block).
mapsq_table project_table(const mapsq_table& cur, const std::vector<int32_t>& want) {
    mapsq_table res = cur;
    res.sorted_col = 0;
    for (size_t i = 0; i < want.size(); i++) {
        int c = -1;
        for (int k = 0; k < cur.ncols; k++)
            if (cur.var[k] == want[i]) c = k;
        res.var[i] = want[i];
        res.col[i] = cur.col[c];
        if (cur.sorted_col == c + 1) res.sorted_col = (int32_t)i + 1;
    }
    for (size_t i = want.size(); i < MAPSQ_MAX_COLS; i++) {
        res.var[i] = 0;
        res.col[i] = nullptr;
    }
    res.ncols = (int32_t)want.size();
    return res;
}

// Query variables (first-appearance order) and the projection list; checks
// the patterns and the SELECT list.
mapsq_status query_vars(Ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                        std::vector<int32_t>* qvars, std::vector<int32_t>* want) {
    if (!pats || npats < 1 || npats > 64) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "npats must be in [1, 64]");
    if (nsel < 0 || (nsel > 0 && !sel)) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "bad select list");
    qvars->clear();
    want->clear();
    for (int i = 0; i < npats; i++) {
        const int32_t t[3] = {pats[i].s, pats[i].p, pats[i].o};
        bool any = false;
        for (int k = 0; k < 3; k++)
            if (t[k] < 0) {
                any = true;
                int32_t v = -t[k] - 1;
                if (std::find(qvars->begin(), qvars->end(), v) == qvars->end()) qvars->push_back(v);
            }
        if (!any) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a triple pattern without variables");
    }
    if (nsel == 0) {
        *want = *qvars;
    } else {
        for (int i = 0; i < nsel; i++) {
            if (std::find(qvars->begin(), qvars->end(), sel[i]) == qvars->end())
                return ctx->fail(MAPSQ_ERR_INVALID_ARG, "a selected variable is not in the query");
            if (std::find(want->begin(), want->end(), sel[i]) != want->end())
                return ctx->fail(MAPSQ_ERR_INVALID_ARG, "a variable is selected twice");
            want->push_back(sel[i]);
        }
    }
    if ((int)want->size() > MAPSQ_MAX_COLS) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 16 variables");
    return MAPSQ_OK;
}

// Table i re-made from the other index where that puts its rows in the
// order of `key` (so that a join on it pairs key runs without a shuffle).
// Owned tables and views already in key order are left alone.
static mapsq_status view_on_key(Ctx* ctx, const mapsq_pattern* pats, mapsq_table* tabs, int i, int32_t key) {
    const int kc = col_of(&tabs[i], key);
    if (tabs[i].owned || kc < 0 || tabs[i].sorted_col == kc + 1) return MAPSQ_OK;
    mapsq_table t{};
    if (mapsq_status st = map_pattern(ctx, &pats[i], key, &t)) return st;
    if (t.owned)
        free_table(ctx, &t);
    else if (t.sorted_col == 1)
        tabs[i] = t;
    return MAPSQ_OK;
}

// Views re-made for a whole plan: each picked table on its step's key, the
// start table on the first step's key.
mapsq_status key_sort_views(Ctx* ctx, const mapsq_pattern* pats, mapsq_table* tabs, int start,
                            const std::vector<PlanStep>& steps) {
    for (size_t k = 0; k < steps.size(); k++) {
        if (steps[k].cross) continue;
        if (mapsq_status st = view_on_key(ctx, pats, tabs, steps[k].pick, steps[k].key)) return st;
        if (k == 0)
            if (mapsq_status st = view_on_key(ctx, pats, tabs, start, steps[k].key)) return st;
    }
    return MAPSQ_OK;
}

// Exact |a JOIN b| on key (and every further shared variable, as the join
// itself groups them): the join's own path up to its count, no rows
// written.  A count that cannot run (no scratch, over 2^40 rows) reads as
// the largest size, so the candidate goes last; the join itself then
// reports what stops it.
static int64_t count_join(Ctx* ctx, const mapsq_table& a, const mapsq_table& b, int32_t key) {
    mapsq_table t{};
    ctx->count_only = true;
    const mapsq_status st = join_tables(ctx, &a, &b, key, &t);
    ctx->count_only = false;
    if (st) {
        ctx->err.clear();
        return INT64_MAX;
    }
    return t.nrows;
}

// The variable a join of tables with variables `a` and `b` uses as its key:
// the first shared one in the query's first-appearance order (-1: none).
static int32_t first_shared(const std::vector<int32_t>& qvars, const mapsq_table& a, const mapsq_table& b) {
    for (int32_t v : qvars)
        if (binds(a, v) && binds(b, v)) return v;
    return -1;
}

mapsq_status query(Ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                   mapsq_table* out) {
    std::memset(out, 0, sizeof(*out));
    if (!ctx->store.loaded) return ctx->fail(MAPSQ_ERR_STATE, "no store loaded");
    std::vector<int32_t> qvars, want;
    mapsq_status vst = query_vars(ctx, pats, npats, sel, nsel, &qvars, &want);
    if (vst) return vst;

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
    std::vector<mapsq_plan_step> plan;
    mapsq_table cur{};
    // one join step: cur JOIN tabs[pick] (a cross product when key < 0);
    // est_rows is the step's expected output (negative: none)
    auto step = [&](int pick, int32_t key, int32_t candidates, double est_rows) -> mapsq_status {
        mapsq_table nxt{};
        ctx->join_est_rows = key < 0 ? -1.0 : est_rows;
        mapsq_status st = key < 0 ? cross_join(ctx, cur, tabs[pick], &nxt)
                                  : join_tables(ctx, &cur, &tabs[pick], key, &nxt);
        ctx->join_est_rows = -1.0;
        if (st) {
            free_table(ctx, &cur);
            cleanup();
            return st;
        }
        free_table(ctx, &cur);
        free_table(ctx, &tabs[pick]);
        used[pick] = true;
        cur = nxt;
        plan.push_back(mapsq_plan_step{pick, key, cur.nrows, candidates, 0});
        return MAPSQ_OK;
    };

    if (ctx->planner == MAPSQ_PLAN_EXACT && npats > 2) {
        // first join: the connected pair with the smallest exact |RS|, the
        // smaller table (ties: lower index) on the left
        int64_t best = INT64_MAX;
        int bl = -1, br = -1, counted = 0;
        int32_t bkey = -1;
        for (int i = 0; i < npats; i++)
            for (int j = i + 1; j < npats; j++) {
                const int32_t key = first_shared(qvars, tabs[i], tabs[j]);
                if (key < 0) continue;
                const bool i_left = tabs[i].nrows <= tabs[j].nrows;
                const int l = i_left ? i : j, r = i_left ? j : i;
                if (mapsq_status st = view_on_key(ctx, pats, tabs.data(), l, key)) return cleanup(), st;
                if (mapsq_status st = view_on_key(ctx, pats, tabs.data(), r, key)) return cleanup(), st;
                const int64_t n = count_join(ctx, tabs[l], tabs[r], key);
                counted++;
                if (bl < 0 || n < best) {
                    best = n;
                    bl = l;
                    br = r;
                    bkey = key;
                }
            }
        if (bl < 0) {  // no two patterns share a variable: cross products from the smallest
            bl = 0;
            for (int i = 1; i < npats; i++)
                if (tabs[i].nrows < tabs[bl].nrows) bl = i;
        }
        if (mapsq_status st = view_on_key(ctx, pats, tabs.data(), bl, bkey)) return cleanup(), st;
        if (br >= 0)
            if (mapsq_status st = view_on_key(ctx, pats, tabs.data(), br, bkey)) return cleanup(), st;
        cur = tabs[bl];
        used[bl] = true;
        plan.push_back(mapsq_plan_step{bl, -1, cur.nrows, 0, 0});
        if (br >= 0)  // its size was counted exactly
            if (mapsq_status st = step(br, bkey, counted, (double)best)) return st;
        // then the connected table whose exact |RS| with the result is smallest
        while ((int)plan.size() < npats) {
            int pick = -1;
            int32_t pkey = -1;
            int64_t pbest = INT64_MAX;
            counted = 0;
            for (int j = 0; j < npats; j++) {
                if (used[j]) continue;
                const int32_t key = first_shared(qvars, cur, tabs[j]);
                if (key < 0) continue;
                if (mapsq_status st = view_on_key(ctx, pats, tabs.data(), j, key)) {
                    free_table(ctx, &cur);
                    cleanup();
                    return st;
                }
                const int64_t n = count_join(ctx, cur, tabs[j], key);
                counted++;
                if (pick < 0 || n < pbest) {
                    pbest = n;
                    pick = j;
                    pkey = key;
                }
            }
            if (pick < 0)  // nothing connected: the smallest remaining table by cross product
                for (int j = 0; j < npats; j++)
                    if (!used[j] && (pick < 0 || tabs[j].nrows < tabs[pick].nrows)) pick = j;
            if (mapsq_status st = step(pick, pkey, counted, (double)pbest)) return st;
        }
    } else {
        std::vector<std::vector<int32_t>> tv(npats);
        std::vector<int64_t> tr(npats);
        for (int i = 0; i < npats; i++) {
            tv[i].assign(tabs[i].var, tabs[i].var + tabs[i].ncols);
            tr[i] = tabs[i].nrows;
        }
        int start;
        std::vector<PlanStep> steps;
        greedy_plan(tv, tr, qvars, &start, &steps);
        if (mapsq_status s2 = key_sort_views(ctx, pats, tabs.data(), start, steps)) {
            cleanup();
            return s2;
        }
        const std::vector<double> est = estimate_steps(ctx, pats, tr, start, steps);
        cur = tabs[start];
        used[start] = true;
        plan.push_back(mapsq_plan_step{start, -1, cur.nrows, 0, 0});
        for (size_t k = 0; k < steps.size(); k++) {
            const PlanStep& ps = steps[k];
            if (mapsq_status st = step(ps.pick, ps.cross ? -1 : ps.key, 0, est[k])) return st;
        }
    }
    ctx->last_plan = plan;
    // projection (bag): pick the selected columns in the requested order
    mapsq_table res = project_table(cur, want);
    *out = res;
    return MAPSQ_OK;
}

}  // namespace mq
