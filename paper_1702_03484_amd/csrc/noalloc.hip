// mapsq_join_into: the join of mapsq_join written to caller-owned output
// columns, with every scratch buffer (sort buffers, segment tables, scan
// partials, look-back status words, histograms, counters and scalars) taken
// from one fixed device array of this library instead of the context's
// arena.  For callers that cannot allocate device memory at call time.
//
// The array is a file-scope __device__ variable: every device the library
// runs on holds its own copy from module load until the process ends.  Its
// device address is looked up once per device (hipGetSymbolAddress, with
// that device current) when the first context on the device is created;
// host code uses only that address, never the variable's name.  Calls on
// one device share the array, so calls that overlap on a device race; each
// call clears what must start at zero (its scalar area and status words).
#include <cstring>
#include <mutex>
#include <string>

#include "runtime.h"

namespace mq {

constexpr size_t JOIN_INTO_SCRATCH = MAPSQ_JOIN_INTO_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[JOIN_INTO_SCRATCH];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on `device` (the current device).
mapsq_status join_into_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return MAPSQ_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return MAPSQ_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MAPSQ_ERR_HIP;
    g_scratch_ptr[device] = p;
    return MAPSQ_OK;
}

static void* scratch_of(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

mapsq_status join_into(Ctx* ctx, const mapsq_table* L, const mapsq_table* R, int32_t key_var,
                       int32_t* const* out_cols, int64_t out_capacity, mapsq_table* out) {
    std::memset(out, 0, sizeof(*out));
    mapsq_status st;
    if ((st = check_table(ctx, L, "left")) || (st = check_table(ctx, R, "right"))) return st;
    if (!out_cols || out_capacity < 0) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output columns or negative capacity");
    const int lk = col_of(L, key_var), rk = col_of(R, key_var);
    if (lk < 0 || rk < 0) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "both tables must bind the key variable");
    for (int c = 0; c < R->ncols; c++)
        if (c != rk && col_of(L, R->var[c]) >= 0)
            return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "a join into caller columns shares only the key variable");
    const int nc = L->ncols + R->ncols - 1;
    if (nc > MAPSQ_MAX_COLS) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "more than 16 columns in the join");
    if (out_capacity > 0)
        for (int c = 0; c < nc; c++)
            if (!out_cols[c]) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output column");
    if ((uint64_t)L->nrows + (uint64_t)R->nrows > MAPSQ_JOIN_INTO_MAX_RECORDS)
        return ctx->fail(MAPSQ_ERR_CAPACITY, "mapsq_join_into: " + std::to_string(L->nrows + R->nrows) +
                                                 " records exceed its limit of " +
                                                 std::to_string(MAPSQ_JOIN_INTO_MAX_RECORDS));
    char* base = static_cast<char*>(scratch_of(ctx->device));
    if (!base) return ctx->fail(MAPSQ_ERR_STATE, "scratch array of the device not set up");

    // A working context over the scratch array: same stream and pinned
    // staging as the caller's, same join options, default digit widths
    // (whose look-back status words always fit; every width gives the same
    // rows in the same order).
    Ctx w;
    w.device = ctx->device;
    w.stream = ctx->stream;
    w.pinned = ctx->pinned;
    w.semijoin = ctx->semijoin;
    w.merge_mode = ctx->merge_mode;
    w.precount = ctx->precount;
    w.use_graph = false;
    w.arena.init(base, JOIN_INTO_SCRATCH);
    w.small_off = w.arena.alloc(SMALL_WORDS * 4);
    w.small = reinterpret_cast<uint32_t*>(w.arena.ptr(w.small_off));
    if (launch_fill_u32(w.small, SMALL_WORDS, 0u, w.stream) != hipSuccess)
        return ctx->fail(MAPSQ_ERR_HIP, "clearing the scratch scalars failed");
    w.out_cols = out_cols;
    w.out_cap = out_capacity;
    st = join_tables(&w, L, R, key_var, out);
    ctx->last = w.last;
    if (st) {
        std::memset(out, 0, sizeof(*out));
        return ctx->fail(st, w.err);
    }
    out->owned = 0;
    out->block = 0;
    for (int c = 0; c < out->ncols; c++) out->col[c] = out_cols[c];
    return MAPSQ_OK;
}

}  // namespace mq
