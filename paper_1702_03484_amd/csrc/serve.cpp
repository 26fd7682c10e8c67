// Serving: continuous batching of queries over the resident store.
//
// mapsq_submit queues a query.  Each mapsq_serve_step is one scheduling
// round: the waiting queries get exact partial-match sizes from the index
// ranges (one batched range-location launch), a greedy join plan and a
// predicted intermediate-byte cost; the head of the queue is admitted while
// the predicted bytes of the admitted queries stay within the budget;
// newly admitted queries map their patterns; then the next join step of
// every active query runs in one batched launch (mapsq_join_batch's graph).
// Queries that arrive while others are in flight join at the next round, so
// their steps share launches with the others'.  A step whose output finds
// no room waits, goes behind the queue or starts over rather than fail while
// memory held by other queries could still make room, so every query ends
// as it would alone (mapsq_query).  The CPU assigns the steps and the GPU
// joins them (the paper's coprocessing split).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <unordered_map>
#include <unordered_set>

#include "runtime.h"

namespace mq {

namespace {

enum QState { Q_WAITING = 0, Q_ACTIVE = 1, Q_DONE = 2, Q_FAILED = 3 };

struct SQuery {
    uint64_t ticket = 0;
    std::vector<mapsq_pattern> pats;
    std::vector<int32_t> qvars, want;
    int state = Q_WAITING;
    mapsq_status err = MAPSQ_OK;
    std::string why;  // message of the failed step
    bool sized = false;
    std::vector<int64_t> rows;             // pattern sizes (exact, or an upper bound for scans)
    double predicted = 0;                  // predicted intermediate bytes
    std::vector<mapsq_table> tabs;         // partial-match tables
    std::vector<bool> consumed;
    int start = 0;
    std::vector<PlanStep> steps;
    std::vector<double> est;               // estimated output rows of each step
    size_t next = 0;
    mapsq_table cur{};
    mapsq_table result{};
    uint64_t admitted = 0;  // admission order (the latest is preempted first)
    double reserve = 0;     // budget bytes held while admitted
    int passed_over = 0;    // rounds in which later queries were admitted first
    int stalls = 0;         // rounds in a row its join step waited for memory
    bool restarted = false; // started over once, alone, on a less fragmented arena
    int deferrals = 0;      // times it gave its memory back and went behind the queue
    double wait_bytes = 0;  // output bytes its join step `wait_step` found no room for
    size_t wait_step = 0;
    int unpolled_waits = 0;  // rounds its join step waited, alone, for results the caller has not polled
    uint64_t poll_mark = 0;  // the server's poll count when that count last started over
    bool await_poll = false; // its admission waits for the caller to poll a result
    int adm_waits = 0;       // rounds its admission waited for a poll
    uint64_t adm_mark = 0;   // the server's poll count when that count last started over
};

// a waiting query may be passed over by later ones this many rounds, then
// admission waits for it (no starvation)
constexpr int MAX_PASSED_OVER = 8;
// a join step that waited for memory this many rounds in a row stops
// admission until it runs (no starvation of large queries)
constexpr int MAX_STALLS = 8;
// a join step that must wait for memory while other queries wait to be
// admitted gives its memory back and goes behind them, at most this often:
// the queries that need most of the arena then run together once the others
// have drained, rather than each draining the active set on its own
constexpr int MAX_DEFERRALS = 2;
// join steps of at least this many records run through the plain join path
// (merge join, semi-join reduction) rather than the batched kernels
constexpr int64_t PLAIN_STEP_RECORDS = int64_t(1) << 20;
// a query alone whose output needs memory held by finished results the
// caller has not polled waits this many rounds without a poll, then fails
constexpr int MAX_UNPOLLED_WAITS = 8;
// rounds in a row in which no join step completes and no query ends, while
// queries are in flight or waiting, before the scheduler gives up on them
// (the policy above always makes progress; this bounds the loop regardless)
constexpr int MAX_IDLE_ROUNDS = 256;

}  // namespace

struct Server {
    uint64_t next_ticket = 1;
    std::deque<SQuery*> waiting;
    std::vector<SQuery*> active;
    std::unordered_map<uint64_t, std::unique_ptr<SQuery>> all;
    double budget = 0;  // 0: set from the arena at the first round
    double reserved = 0;
    int max_active = 256;
    uint64_t admissions = 0;
    bool hold = false;  // after a preemption: admit nothing until a query ends
    std::deque<uint64_t> finished;  // tickets in the order their queries ended
    uint64_t polls = 0;             // finished queries retired by the caller
    SQuery* solo = nullptr;         // a query that started over: nothing else is admitted until it ends
    uint64_t ends = 0;              // queries that ended (done or failed)
    int idle_rounds = 0;            // rounds in a row without a completed step or an end
};

void destroy_server(Ctx* ctx) {
    if (!ctx->server) return;
    for (auto& kv : ctx->server->all) {
        SQuery* q = kv.second.get();
        for (size_t i = 0; i < q->tabs.size(); i++)
            if (!q->consumed[i]) free_table(ctx, &q->tabs[i]);
        if (q->state == Q_ACTIVE && q->cur.owned) free_table(ctx, &q->cur);
        if (q->state == Q_DONE) free_table(ctx, &q->result);
    }
    delete ctx->server;
    ctx->server = nullptr;
}

static Server* server(Ctx* ctx) {
    if (!ctx->server) ctx->server = new Server();
    return ctx->server;
}

mapsq_status serve_config(Ctx* ctx, uint64_t budget_bytes, int32_t max_active) {
    if (max_active < 0) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "max_active must be >= 0");
    Server* S = server(ctx);
    S->budget = (double)budget_bytes;
    S->max_active = max_active ? max_active : 256;
    return MAPSQ_OK;
}

mapsq_status submit(Ctx* ctx, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                    uint64_t* ticket) {
    if (!ticket) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null ticket");
    *ticket = 0;
    if (!ctx->store.loaded) return ctx->fail(MAPSQ_ERR_STATE, "no store loaded");
    std::unique_ptr<SQuery> q(new SQuery());
    mapsq_status st = query_vars(ctx, pats, npats, sel, nsel, &q->qvars, &q->want);
    if (st) return st;
    for (int i = 0; i < npats; i++) {
        const int32_t t[3] = {pats[i].s, pats[i].p, pats[i].o};
        for (int k = 0; k < 3; k++)
            if (t[k] == INT32_MAX) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "constant outside [0, 2^31 - 1)");
    }
    Server* S = server(ctx);
    q->pats.assign(pats, pats + npats);
    q->ticket = S->next_ticket++;
    *ticket = q->ticket;
    S->waiting.push_back(q.get());
    S->all.emplace(q->ticket, std::move(q));
    return MAPSQ_OK;
}

// Exact sizes of the waiting queries' patterns: predicate ranges from the
// host table, narrowed on the device by one batched range-location launch;
// patterns that need a scan (variable predicate or a repeated variable)
// get the scanned range as an upper bound.
static mapsq_status size_waiting(Ctx* ctx, Server* S) {
    const Store& St = ctx->store;
    std::vector<LocateQuery> lq;
    std::vector<std::pair<SQuery*, int>> who;
    std::vector<SQuery*> sized;
    for (SQuery* q : S->waiting) {
        if (q->sized) continue;
        q->rows.assign(q->pats.size(), 0);
        for (size_t i = 0; i < q->pats.size(); i++) {
            const mapsq_pattern& p = q->pats[i];
            const bool rep = (p.s < 0 && (p.s == p.p || p.s == p.o)) || (p.p < 0 && p.p == p.o);
            if (p.p < 0) {
                q->rows[i] = St.n;
                continue;
            }
            auto it = std::lower_bound(St.preds.begin(), St.preds.end(), p.p);
            if (it == St.preds.end() || *it != p.p) {
                q->rows[i] = 0;
                continue;
            }
            const size_t pi = size_t(it - St.preds.begin());
            LocateQuery x{};
            x.lo = St.pred_off[pi];
            x.hi = St.pred_off[pi + 1];
            if (p.s >= 0) {
                x.col1 = St.pso_s;
                x.v1 = p.s;
                if (p.o >= 0) {
                    x.col2 = St.pso_o;
                    x.v2 = p.o;
                }
            } else if (p.o >= 0) {
                x.col1 = St.pos_o;
                x.v1 = p.o;
            }
            if (!x.col1 || rep) {
                q->rows[i] = x.hi - x.lo;
                continue;
            }
            lq.push_back(x);
            who.emplace_back(q, (int)i);
        }
        sized.push_back(q);
    }
    if (!lq.empty()) {
        std::vector<int64_t> r(2 * lq.size());
        // on failure no query counts as sized: the next round sizes them again
        if (mapsq_status st = locate_ranges(ctx, lq.data(), lq.size(), r.data())) return st;
        for (size_t k = 0; k < who.size(); k++) who[k].first->rows[who[k].second] = r[2 * k + 1] - r[2 * k];
    }
    for (SQuery* q : sized) q->sized = true;
    return MAPSQ_OK;
}

// Predicted intermediate bytes of a query: the greedy plan on the exact
// pattern sizes, each join's output estimated as |L| |R| / max(distinct
// keys) from the per-predicate statistics (System-R style), plus the scan
// outputs and the join scratch (24 B per record).
static void predict(Ctx* ctx, SQuery* q) {
    const size_t m = q->pats.size();
    std::vector<std::vector<int32_t>> vars(m);
    for (size_t i = 0; i < m; i++) {
        const mapsq_pattern& p = q->pats[i];
        for (int32_t t : {p.s, p.p, p.o})
            if (t < 0 && std::find(vars[i].begin(), vars[i].end(), -t - 1) == vars[i].end()) vars[i].push_back(-t - 1);
    }
    int start;
    std::vector<PlanStep> steps;
    greedy_plan(vars, q->rows, q->qvars, &start, &steps);
    double bytes = 0;
    std::vector<size_t> cols;
    const std::vector<double> est = estimate_steps(ctx, q->pats.data(), q->rows, start, steps, &bytes, &cols);
    double rows = (double)q->rows[start];
    for (size_t k = 0; k < steps.size(); k++) {
        bytes += 24.0 * (rows + (double)q->rows[steps[k].pick]) + 4.0 * (double)cols[k] * est[k];
        rows = est[k];
    }
    q->predicted = bytes;
}

static void fail_query(Ctx* ctx, Server* S, SQuery* q, mapsq_status err) {
    for (size_t i = 0; i < q->tabs.size(); i++)
        if (!q->consumed[i]) free_table(ctx, &q->tabs[i]);
    if (q->cur.owned) free_table(ctx, &q->cur);
    std::memset(&q->cur, 0, sizeof(mapsq_table));
    if (q->state == Q_ACTIVE) S->reserved -= q->reserve;
    q->state = Q_FAILED;
    q->err = err;
    q->why = ctx->err;
    S->hold = false;
    if (S->solo == q) S->solo = nullptr;
    S->finished.push_back(q->ticket);
    S->ends++;
}

// Give back everything a stalled query holds and queue it again, at the
// head (admission then waits for a running query to end) or, deferred, at
// the tail; it restarts from its partial matches.
static void preempt_query(Ctx* ctx, Server* S, SQuery* q, bool to_tail = false) {
    for (size_t i = 0; i < q->tabs.size(); i++)
        if (!q->consumed[i]) free_table(ctx, &q->tabs[i]);
    if (q->cur.owned) free_table(ctx, &q->cur);
    std::memset(&q->cur, 0, sizeof(mapsq_table));
    q->tabs.clear();
    q->consumed.clear();
    q->steps.clear();
    q->next = 0;
    q->stalls = 0;
    q->wait_bytes = 0;
    q->unpolled_waits = 0;
    S->reserved -= q->reserve;
    q->state = Q_WAITING;
    if (to_tail) {
        S->waiting.push_back(q);
    } else {
        S->waiting.push_front(q);
        S->hold = true;
    }
}

static void finish_query(Server* S, SQuery* q) {
    q->result = project_table(q->cur, q->want);
    std::memset(&q->cur, 0, sizeof(mapsq_table));
    q->state = Q_DONE;
    S->reserved -= q->reserve;
    S->hold = false;
    if (S->solo == q) S->solo = nullptr;
    S->finished.push_back(q->ticket);
    S->ends++;
}

// Map the patterns of a newly admitted query and fix its plan on the exact
// table sizes.
static mapsq_status activate(Ctx* ctx, Server* S, SQuery* q) {
    const size_t m = q->pats.size();
    q->tabs.assign(m, mapsq_table{});
    q->consumed.assign(m, true);
    for (size_t i = 0; i < m; i++) {
        mapsq_status st = map_pattern(ctx, &q->pats[i], -1, &q->tabs[i]);
        if (st) return st;
        q->consumed[i] = false;
    }
    std::vector<std::vector<int32_t>> vars(m);
    std::vector<int64_t> rows(m);
    for (size_t i = 0; i < m; i++) {
        vars[i].assign(q->tabs[i].var, q->tabs[i].var + q->tabs[i].ncols);
        rows[i] = q->tabs[i].nrows;
    }
    greedy_plan(vars, rows, q->qvars, &q->start, &q->steps);
    q->est = estimate_steps(ctx, q->pats.data(), rows, q->start, q->steps);
    if (mapsq_status st = key_sort_views(ctx, q->pats.data(), q->tabs.data(), q->start, q->steps)) return st;
    q->cur = q->tabs[q->start];
    q->consumed[q->start] = true;
    q->next = 0;
    q->state = Q_ACTIVE;
    if (q->steps.empty()) finish_query(S, q);
    return MAPSQ_OK;
}

mapsq_status serve_step(Ctx* ctx, int32_t* n_active, int32_t* n_waiting) {
    Server* S = server(ctx);
    if (!ctx->store.loaded) return ctx->fail(MAPSQ_ERR_STATE, "no store loaded");
    if (S->budget <= 0) S->budget = 0.6 * (double)ctx->arena.free_bytes();
    // 1. sizes, plans and predictions of the waiting queries; admission in
    // arrival order while the admitted predictions fit the budget, later
    // queries that fit going first (a query passed over MAX_PASSED_OVER
    // rounds stops that).  A prediction above the whole budget reserves
    // nothing: the exact size of each of its joins decides (step 2).
    mapsq_status st = size_waiting(ctx, S);
    // no room even for the index range lookups: this round admits nothing
    // (the waiting queries are sized again in the next one)
    const bool unsized = st == MAPSQ_ERR_CAPACITY;
    if (unsized)
        st = MAPSQ_OK;
    else if (st)
        return st;
    auto live_others = [&](const SQuery* q) {
        int k = 0;
        for (const SQuery* o : S->active) k += o != q && o->state == Q_ACTIVE;
        return k;
    };
    // bytes the query could use if every other query let go of what it
    // holds: the free space plus every arena block that only other queries'
    // tables reference (a batch's shared block counts whole)
    auto tables_of = [](const SQuery* o, auto&& f) {
        if (o->state == Q_ACTIVE) {
            f(o->cur);
            for (size_t i = 0; i < o->tabs.size(); i++)
                if (!o->consumed[i]) f(o->tabs[i]);
        } else if (o->state == Q_DONE) {
            f(o->result);
        }
    };
    auto blocks_of = [&](const SQuery* q) {
        std::unordered_set<uint64_t> own;
        tables_of(q, [&](const mapsq_table& t) {
            if (t.owned && t.block) own.insert(t.block);
        });
        return own;
    };
    // free space plus the blocks the query holds itself
    auto own_room = [&](const SQuery* q) {
        double b = (double)ctx->arena.free_bytes();
        for (uint64_t blk : blocks_of(q)) b += (double)ctx->arena.block_size(size_t(blk - 1));
        return b;
    };
    // blocks held only by finished results the caller has not polled yet
    auto unpolled_room = [&](const SQuery* q) {
        const std::unordered_set<uint64_t> own = blocks_of(q);
        std::unordered_set<uint64_t> done;
        for (auto& kv : S->all)
            if (kv.second->state == Q_DONE)
                tables_of(kv.second.get(), [&](const mapsq_table& t) {
                    if (t.owned && t.block && !own.count(t.block)) done.insert(t.block);
                });
        double b = 0;
        for (uint64_t blk : done) b += (double)ctx->arena.block_size(size_t(blk - 1));
        return b;
    };
    auto room_alone = [&](const SQuery* q) {
        const std::unordered_set<uint64_t> own = blocks_of(q);
        std::unordered_set<uint64_t> others;
        for (auto& kv : S->all)
            if (kv.second.get() != q)
                tables_of(kv.second.get(), [&](const mapsq_table& t) {
                    if (t.owned && t.block && !own.count(t.block)) others.insert(t.block);
                });
        double b = (double)ctx->arena.free_bytes();
        for (uint64_t blk : others) b += (double)ctx->arena.block_size(size_t(blk - 1));
        // a batch's shared block holding one of q's tables stays while q
        // holds it; the part that is not q's comes back if q starts over
        double mine = 0;
        tables_of(q, [&](const mapsq_table& t) {
            if (t.owned && t.block && ctx->shared_refs.count(size_t(t.block - 1)))
                mine += 4.0 * (double)t.nrows * t.ncols;
        });
        for (uint64_t blk : own)
            if (ctx->shared_refs.count(size_t(blk - 1))) b += (double)ctx->arena.block_size(size_t(blk - 1));
        return b - mine;
    };
    bool starving = false;
    for (const SQuery* o : S->active) starving = starving || (o->state == Q_ACTIVE && o->stalls > MAX_STALLS);
    for (auto it = S->waiting.begin(); it != S->waiting.end() && !S->hold && !starving && !unsized;) {
        SQuery* q = *it;
        if ((int)S->active.size() >= S->max_active) break;
        if (S->solo && q != S->solo) break;
        // a query that starts over runs on an arena as clean as mapsq_query
        // would find it: first the caller polls the finished results (a
        // bounded number of rounds without a poll)
        if (S->solo == q && unpolled_room(q) > 0) {
            if (q->adm_mark != S->polls) {
                q->adm_mark = S->polls;
                q->adm_waits = 0;
            }
            if (++q->adm_waits <= MAX_UNPOLLED_WAITS) break;
        }
        // its partial matches found no room while finished results waited
        // to be polled: admission waits for a poll (a bounded number of
        // rounds), then it tries again
        if (q->await_poll) {
            if (q->adm_mark != S->polls) {
                q->await_poll = false;
                q->adm_waits = 0;
            } else if (++q->adm_waits <= MAX_UNPOLLED_WAITS) {
                break;
            }
        }
        if (q->predicted == 0) predict(ctx, q);
        const double r = q->predicted > S->budget ? 0.0 : q->predicted;
        if (S->reserved + r > S->budget) {
            if (++q->passed_over > MAX_PASSED_OVER) break;
            ++it;
            continue;
        }
        it = S->waiting.erase(it);
        q->reserve = r;
        S->reserved += r;
        S->active.push_back(q);
        q->state = Q_ACTIVE;
        q->admitted = ++S->admissions;
        st = activate(ctx, S, q);
        if (st == MAPSQ_ERR_CAPACITY && live_others(q) > 0) {
            preempt_query(ctx, S, q);  // its partial matches do not fit yet
        } else if (st == MAPSQ_ERR_CAPACITY && !q->await_poll && q->adm_waits == 0 && unpolled_room(q) > 0) {
            preempt_query(ctx, S, q);  // they may fit once finished results are polled
            S->hold = false;
            q->await_poll = true;
            q->adm_mark = S->polls;
            break;
        } else if (st) {
            fail_query(ctx, S, q, st == MAPSQ_ERR_CAPACITY ? MAPSQ_ERR_TOO_LARGE : st);
        }
        if (S->hold) break;
    }
    // 2. the next join step of every active query: small ones together in
    // one batched launch, large or key-sorted ones through the plain path
    std::vector<SQuery*> in_batch, in_plain;
    std::vector<mapsq_join_desc> descs;
    int progress = 0;
    int steps_done = 0;  // join steps completed this round
    const uint64_t ends0 = S->ends;
    // a finished step: the intermediate must stay joinable (under 2^31 rows)
    auto advance = [&](SQuery* q, const mapsq_table& nxt, int pick) {
        free_table(ctx, &q->cur);
        free_table(ctx, &q->tabs[pick]);
        q->consumed[pick] = true;
        q->cur = nxt;
        q->stalls = 0;
        q->wait_bytes = 0;
        q->unpolled_waits = 0;
        progress++;
        steps_done++;
        if (++q->next == q->steps.size())
            finish_query(S, q);
        else if (q->cur.nrows >= (int64_t(1) << 31))
            fail_query(ctx, S, q, ctx->fail(MAPSQ_ERR_TOO_LARGE, "an intermediate of 2^31 rows or more"));
    };
    std::vector<SQuery*> stalled;
    // a failed step: wait for memory while others hold some, unless the
    // exact output could not fit even then
    // A step whose output found no room.  With other queries in flight it
    // waits (or first goes behind the queue) if the output would fit once
    // they let go of everything.  Alone, it tries again next round when only
    // results not yet polled stand in the way, and starts over once, from a
    // cleaner arena, when its own tables split the free space.  Otherwise the
    // query fails as it would alone.
    auto failed = [&](SQuery* q, mapsq_status e, int64_t need_rows) {
        const bool memory = e == MAPSQ_ERR_CAPACITY || e == MAPSQ_ERR_TOO_LARGE;
        if (memory && need_rows < SAT40_HOST) {
            const PlanStep& ps = q->steps[q->next];
            const mapsq_table& R = q->tabs[ps.pick];
            const double cols = q->cur.ncols + R.ncols - 1;
            // the output, and the join's scratch held while it is written:
            // 24 B per run of the smaller side for key-sorted inputs, else
            // 24 B per record (28 B when a second shared variable makes the
            // key composite)
            int shared = 0;
            for (int c = 0; c < R.ncols; c++) shared += col_of(&q->cur, R.var[c]) >= 0 ? 1 : 0;
            const bool comp = !ps.cross && shared >= 2 && ctx->composite == 0;
            const bool sorted = !ps.cross && !comp && q->cur.sorted_col == col_of(&q->cur, ps.key) + 1 &&
                                R.sorted_col == col_of(&R, ps.key) + 1;
            const double recs = sorted ? (double)std::min(q->cur.nrows, R.nrows) : (double)(q->cur.nrows + R.nrows);
            const double need = 4.0 * (double)need_rows * cols + (comp ? 28.0 : 24.0) * recs;
            if (live_others(q) > 0) {
                q->wait_bytes = need;
                q->wait_step = q->next;
                q->unpolled_waits = 0;
                if (need <= room_alone(q) && q->deferrals < MAX_DEFERRALS && !S->waiting.empty()) {
                    q->deferrals++;
                    preempt_query(ctx, S, q, true);
                    progress++;
                    return;
                }
                if (need <= room_alone(q)) {
                    q->stalls++;
                    stalled.push_back(q);
                    return;
                }
            } else {
                const double own = own_room(q);
                // finished results hold memory until the caller polls them:
                // wait for that (without running the join again) for a
                // bounded number of rounds in which nothing is polled
                // (those blocks can also split the free space: wait for them
                // even when the free bytes alone would be enough)
                const double unpolled = unpolled_room(q);
                if (unpolled > 0 && need <= own + unpolled) {
                    // a new wait (another step, or the first) counts from zero
                    const bool again = q->wait_bytes > 0 && q->wait_step == q->next && q->unpolled_waits > 0;
                    q->wait_bytes = need;
                    q->wait_step = q->next;
                    if (!again || q->poll_mark != S->polls) {
                        q->unpolled_waits = 0;
                        q->poll_mark = S->polls;
                    }
                    if (++q->unpolled_waits <= MAX_UNPOLLED_WAITS) {
                        q->stalls++;
                        progress++;
                        return;
                    }
                    ctx->fail(MAPSQ_ERR_TOO_LARGE, "the step's output needs memory held by finished results "
                                                   "that were not polled");
                }
                if (!q->restarted && !blocks_of(q).empty() && need <= own) {
                    // it runs again alone, as mapsq_query would: nothing
                    // else is admitted until it ends
                    q->restarted = true;
                    preempt_query(ctx, S, q);
                    S->hold = false;
                    S->solo = q;
                    progress++;
                    return;
                }
            }
        }
        fail_query(ctx, S, q, memory ? MAPSQ_ERR_TOO_LARGE : e);
        progress++;
    };
    for (SQuery* q : S->active) {
        if (q->state != Q_ACTIVE || q->next >= q->steps.size()) continue;
        // a step that found no room waits, without running its join again,
        // until a free block could hold its output
        if (q->wait_bytes > 0 && q->wait_step == q->next && live_others(q) > 0 &&
            (double)ctx->arena.largest() < q->wait_bytes) {
            q->stalls++;
            stalled.push_back(q);
            continue;
        }
        // alone, waiting for finished results to be polled: the count of
        // rounds starts over whenever the caller retires a result
        if (q->wait_bytes > 0 && q->wait_step == q->next && live_others(q) == 0 && q->unpolled_waits > 0 &&
            (double)ctx->arena.largest() < q->wait_bytes && unpolled_room(q) > 0) {
            if (q->poll_mark != S->polls) {
                q->unpolled_waits = 0;
                q->poll_mark = S->polls;
            }
            if (++q->unpolled_waits > MAX_UNPOLLED_WAITS) {
                ctx->fail(MAPSQ_ERR_TOO_LARGE, "the step's output needs memory held by finished results "
                                               "that were not polled");
                fail_query(ctx, S, q, MAPSQ_ERR_TOO_LARGE);
            }
            q->stalls++;
            progress++;
            continue;
        }
        const PlanStep& ps = q->steps[q->next];
        if (ps.cross) {  // rare: run it now through the plain path
            mapsq_table nxt{};
            st = cross_join(ctx, q->cur, q->tabs[ps.pick], &nxt);
            if (st)
                failed(q, st, ctx->last.out_rows);
            else
                advance(q, nxt, ps.pick);
            continue;
        }
        const mapsq_table& R = q->tabs[ps.pick];
        const bool sorted = q->cur.sorted_col == col_of(&q->cur, ps.key) + 1 && R.sorted_col == col_of(&R, ps.key) + 1;
        // a query that started over runs alone through the plain path: its
        // intermediates then get blocks of their own
        if (sorted || q->restarted || q->cur.nrows + R.nrows >= PLAIN_STEP_RECORDS) {
            in_plain.push_back(q);
        } else {
            in_batch.push_back(q);
            descs.push_back(mapsq_join_desc{&q->cur, &q->tabs[ps.pick], ps.key, 0});
        }
    }
    if (!descs.empty()) {
        std::vector<mapsq_table> outs(descs.size());
        std::vector<mapsq_status> per(descs.size());
        std::vector<int64_t> need(descs.size());
        st = join_batch(ctx, descs.data(), (int32_t)descs.size(), outs.data(), per.data(), need.data());
        if (st) return st;
        for (size_t k = 0; k < in_batch.size(); k++) {
            SQuery* q = in_batch[k];
            if (per[k] != MAPSQ_OK) {
                ctx->fail(per[k], "batched join step (" + std::to_string(need[k]) + " output rows) failed");
                failed(q, per[k], need[k]);
            } else {
                advance(q, outs[k], q->steps[q->next].pick);
            }
        }
    }
    for (SQuery* q : in_plain) {
        const PlanStep& ps = q->steps[q->next];
        mapsq_table nxt{};
        ctx->join_est_rows = q->est[q->next];
        st = join_tables(ctx, &q->cur, &q->tabs[ps.pick], ps.key, &nxt);
        ctx->join_est_rows = -1.0;
        if (st)
            failed(q, st, ctx->last.out_rows);
        else
            advance(q, nxt, ps.pick);
    }
    // a round in which every step waited for memory: the latest admitted
    // waiting query gives its memory back and restarts later
    if (progress == 0 && !stalled.empty()) {
        SQuery* v = *std::max_element(stalled.begin(), stalled.end(),
                                      [](const SQuery* a, const SQuery* b) { return a->admitted < b->admitted; });
        preempt_query(ctx, S, v);
    }
    // 3. retire finished queries from the active set
    S->active.erase(std::remove_if(S->active.begin(), S->active.end(),
                                   [](SQuery* q) { return q->state != Q_ACTIVE; }),
                    S->active.end());
    // 4. a bound on rounds without a completed join step or an ended query
    if (steps_done == 0 && S->ends == ends0 && (!S->active.empty() || !S->waiting.empty()))
        S->idle_rounds++;
    else
        S->idle_rounds = 0;
    if (S->idle_rounds > MAX_IDLE_ROUNDS) {
        const std::string msg = "serving made no progress in " + std::to_string(MAX_IDLE_ROUNDS) + " rounds";
        for (SQuery* q : S->active) {
            ctx->fail(MAPSQ_ERR_STATE, msg);
            fail_query(ctx, S, q, MAPSQ_ERR_STATE);
        }
        for (SQuery* q : S->waiting) {
            ctx->fail(MAPSQ_ERR_STATE, msg);
            fail_query(ctx, S, q, MAPSQ_ERR_STATE);
        }
        S->active.clear();
        S->waiting.clear();
        S->reserved = 0;
        S->idle_rounds = 0;
        if (n_active) *n_active = 0;
        if (n_waiting) *n_waiting = 0;
        return ctx->fail(MAPSQ_ERR_STATE, msg + "; every query in flight failed with MAPSQ_ERR_STATE");
    }
    if (n_active) *n_active = (int32_t)S->active.size();
    if (n_waiting) *n_waiting = (int32_t)S->waiting.size();
    return MAPSQ_OK;
}

mapsq_status poll(Ctx* ctx, uint64_t ticket, int32_t* done, mapsq_table* out) {
    if (!done || !out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
    *done = 0;
    std::memset(out, 0, sizeof(mapsq_table));
    Server* S = server(ctx);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "unknown ticket");
    SQuery* q = it->second.get();
    if (q->state == Q_DONE) {
        *out = q->result;
        *done = 1;
        S->all.erase(it);
        S->polls++;
        return MAPSQ_OK;
    }
    if (q->state == Q_FAILED) {
        const mapsq_status err = q->err;
        const std::string msg = "query " + std::to_string(ticket) + " failed: " + q->why;
        *done = 1;
        S->polls++;
        S->all.erase(it);  // destroys q
        return ctx->fail(err, msg);
    }
    return MAPSQ_OK;
}

mapsq_status poll_next(Ctx* ctx, uint64_t* ticket, int32_t* done, mapsq_table* out) {
    if (!ticket || !done || !out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
    *ticket = 0;
    *done = 0;
    std::memset(out, 0, sizeof(mapsq_table));
    Server* S = server(ctx);
    while (!S->finished.empty()) {
        const uint64_t tk = S->finished.front();
        S->finished.pop_front();
        if (!S->all.count(tk)) continue;  // already retired by mapsq_poll
        *ticket = tk;
        return poll(ctx, tk, done, out);
    }
    return MAPSQ_OK;
}

}  // namespace mq
