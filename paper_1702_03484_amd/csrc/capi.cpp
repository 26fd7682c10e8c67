// extern "C" boundary of libmapsq.so (declared in include/mapsq.h): checks
// arguments, selects the context's device for the duration of the call and
// keeps C++ exceptions from crossing the ABI.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>

#include "runtime.h"

using mq::Ctx;

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <typename F>
mapsq_status guarded(mapsq_ctx* c, F&& f) {
    if (!c) return MAPSQ_ERR_INVALID_ARG;
    Ctx* ctx = &c->impl;
    ctx->err.clear();
    DeviceGuard g(ctx->device);
    if (!g.ok) return ctx->fail(MAPSQ_ERR_HIP, "hipSetDevice failed");
    try {
        return f(ctx);
    } catch (const std::bad_alloc&) {
        return ctx->fail(MAPSQ_ERR_CAPACITY, "host allocation failed");
    } catch (...) {
        return ctx->fail(MAPSQ_ERR_HIP, "unexpected host exception");
    }
}

}  // namespace

extern "C" {

mapsq_status mapsq_create(int device, void* arena, size_t arena_bytes, void* hip_stream, mapsq_ctx** out) {
    if (!out) return MAPSQ_ERR_INVALID_ARG;
    *out = nullptr;
    if (!arena || arena_bytes < (size_t(64) << 20) || reinterpret_cast<uintptr_t>(arena) % mq::ARENA_ALIGN)
        return MAPSQ_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MAPSQ_ERR_HIP;
    DeviceGuard g(device);
    if (!g.ok) return MAPSQ_ERR_HIP;
    mapsq_ctx* c = new (std::nothrow) mapsq_ctx();
    if (!c) return MAPSQ_ERR_CAPACITY;
    Ctx* ctx = &c->impl;
    ctx->device = device;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx->arena.init(reinterpret_cast<char*>(arena), arena_bytes);
    ctx->small_off = ctx->arena.alloc(mq::SMALL_WORDS * 4);
    ctx->small = reinterpret_cast<uint32_t*>(ctx->arena.ptr(ctx->small_off));
    if (hipHostMalloc(&ctx->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return MAPSQ_ERR_HIP;
    }
    if (mq::launch_fill_u32(ctx->small, mq::SMALL_WORDS, 0u, ctx->stream) != hipSuccess ||
        !ctx->ensure_status(1 << 16) || mq::join_into_setup(device) != MAPSQ_OK) {
        (void)hipHostFree(ctx->pinned);
        delete c;
        return MAPSQ_ERR_HIP;
    }
    // MAPSQ_FAULT=alloc:N: the context's (N+1)-th arena allocation fails
    if (const char* f = std::getenv("MAPSQ_FAULT")) {
        if (std::strncmp(f, "alloc:", 6) == 0) {
            char* end = nullptr;
            const long long n = std::strtoll(f + 6, &end, 10);
            if (end != f + 6 && *end == '\0' && n >= 0) ctx->arena.fail_after = n;
        }
    }
    *out = c;
    return MAPSQ_OK;
}

mapsq_status mapsq_debug_fail_alloc(mapsq_ctx* c, int64_t after) {
    return guarded(c, [&](Ctx* ctx) {
        ctx->arena.fail_after = after < 0 ? -1 : after;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_destroy(mapsq_ctx* c) {
    if (!c) return MAPSQ_OK;
    {
        DeviceGuard g(c->impl.device);
        (void)hipStreamSynchronize(c->impl.stream);
        mq::destroy_server(&c->impl);
        c->impl.prof_release();
        c->impl.release_graphs();
        if (c->impl.stage) (void)hipHostFree(c->impl.stage);
        if (c->impl.pinned) (void)hipHostFree(c->impl.pinned);
    }
    delete c;
    return MAPSQ_OK;
}

const char* mapsq_last_error(const mapsq_ctx* c) {
    if (!c) return "null context";
    return c->impl.err.c_str();
}

mapsq_status mapsq_load_triples(mapsq_ctx* c, const int32_t* s, const int32_t* p, const int32_t* o, int64_t n,
                                uint32_t flags) {
    return guarded(c, [&](Ctx* ctx) { return mq::load_triples(ctx, s, p, o, n, flags); });
}

mapsq_status mapsq_store_info(mapsq_ctx* c, mapsq_store_facts* out) {
    return guarded(c, [&](Ctx* ctx) {
        if (!out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        std::memset(out, 0, sizeof(*out));
        if (!ctx->store.loaded) return ctx->fail(MAPSQ_ERR_STATE, "no store loaded");
        out->n_triples = ctx->store.n;
        out->n_predicates = (int64_t)ctx->store.preds.size();
        out->max_id = ctx->store.max_id;
        out->id_bits = ctx->store.id_bits;
        out->device_bytes = ctx->store.bytes;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_predicate_stats(mapsq_ctx* c, int32_t predicate, int64_t* triples, int64_t* distinct_s,
                                   int64_t* distinct_o) {
    return guarded(c, [&](Ctx* ctx) {
        if (!triples || !distinct_s || !distinct_o) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        *triples = *distinct_s = *distinct_o = 0;
        const mq::Store& S = ctx->store;
        if (!S.loaded) return ctx->fail(MAPSQ_ERR_STATE, "no store loaded");
        if (S.pred_ds.size() != S.preds.size()) return ctx->fail(MAPSQ_ERR_UNSUPPORTED, "no predicate statistics");
        auto it = std::lower_bound(S.preds.begin(), S.preds.end(), predicate);
        if (it == S.preds.end() || *it != predicate) return (mapsq_status)MAPSQ_OK;
        const size_t i = size_t(it - S.preds.begin());
        *triples = S.pred_off[i + 1] - S.pred_off[i];
        *distinct_s = S.pred_ds[i];
        *distinct_o = S.pred_do[i];
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_map_pattern(mapsq_ctx* c, const mapsq_pattern* pattern, int32_t key_var, mapsq_table* out) {
    return guarded(c, [&](Ctx* ctx) {
        if (!out || !pattern) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null argument");
        return mq::map_pattern(ctx, pattern, key_var, out);
    });
}

mapsq_status mapsq_join(mapsq_ctx* c, const mapsq_table* left, const mapsq_table* right, int32_t key_var,
                        mapsq_table* out) {
    return guarded(c, [&](Ctx* ctx) {
        if (!out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        return mq::join_tables(ctx, left, right, key_var, out);
    });
}

mapsq_status mapsq_join_into(mapsq_ctx* c, const mapsq_table* left, const mapsq_table* right, int32_t key_var,
                             int32_t* const* out_cols, int64_t out_capacity, mapsq_table* out) {
    return guarded(c, [&](Ctx* ctx) {
        if (!out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        return mq::join_into(ctx, left, right, key_var, out_cols, out_capacity, out);
    });
}

mapsq_status mapsq_query(mapsq_ctx* c, const mapsq_pattern* pats, int32_t npats, const int32_t* select_vars,
                         int32_t nselect, mapsq_table* out) {
    return guarded(c, [&](Ctx* ctx) {
        if (!out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        return mq::query(ctx, pats, npats, select_vars, nselect, out);
    });
}

mapsq_status mapsq_join_batch(mapsq_ctx* c, const mapsq_join_desc* joins, int32_t n, mapsq_table* outs) {
    return guarded(c, [&](Ctx* ctx) { return mq::join_batch(ctx, joins, n, outs); });
}

mapsq_status mapsq_serve_config(mapsq_ctx* c, uint64_t budget_bytes, int32_t max_active) {
    return guarded(c, [&](Ctx* ctx) { return mq::serve_config(ctx, budget_bytes, max_active); });
}

mapsq_status mapsq_submit(mapsq_ctx* c, const mapsq_pattern* pats, int32_t npats, const int32_t* sel, int32_t nsel,
                          uint64_t* ticket) {
    return guarded(c, [&](Ctx* ctx) { return mq::submit(ctx, pats, npats, sel, nsel, ticket); });
}

mapsq_status mapsq_serve_step(mapsq_ctx* c, int32_t* active, int32_t* waiting) {
    return guarded(c, [&](Ctx* ctx) { return mq::serve_step(ctx, active, waiting); });
}

mapsq_status mapsq_poll(mapsq_ctx* c, uint64_t ticket, int32_t* done, mapsq_table* out) {
    return guarded(c, [&](Ctx* ctx) { return mq::poll(ctx, ticket, done, out); });
}

mapsq_status mapsq_poll_next(mapsq_ctx* c, uint64_t* ticket, int32_t* done, mapsq_table* out) {
    return guarded(c, [&](Ctx* ctx) { return mq::poll_next(ctx, ticket, done, out); });
}

mapsq_status mapsq_table_free(mapsq_ctx* c, mapsq_table* t) {
    return guarded(c, [&](Ctx* ctx) {
        if (!t) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null table");
        return mq::free_table(ctx, t);
    });
}

mapsq_status mapsq_last_join_stats(mapsq_ctx* c, mapsq_join_stats* out) {
    return guarded(c, [&](Ctx* ctx) {
        if (!out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        *out = ctx->last;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_set_join_options(mapsq_ctx* c, int32_t semijoin, int32_t merge, int32_t precount,
                                    int32_t composite) {
    return guarded(c, [&](Ctx* ctx) {
        if (semijoin < 0 || semijoin > 2) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "semijoin must be 0, 1 or 2");
        if (merge < 0 || merge > 1) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "merge must be 0 or 1");
        if (precount < 0 || precount > 2) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "precount must be 0, 1 or 2");
        if (composite < 0 || composite > 1) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "composite must be 0 or 1");
        ctx->semijoin = semijoin;
        ctx->merge_mode = merge;
        ctx->precount = precount;
        ctx->composite = composite;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_dict_create(mapsq_ctx* c, int64_t max_terms, int64_t max_bytes) {
    return guarded(c, [&](Ctx* ctx) { return mq::dict_create(ctx, max_terms, max_bytes); });
}

mapsq_status mapsq_dict_encode(mapsq_ctx* c, const uint8_t* bytes, const int64_t* offsets, int64_t n, uint32_t flags,
                               int32_t* ids, int64_t* n_new) {
    return guarded(c, [&](Ctx* ctx) { return mq::dict_encode(ctx, bytes, offsets, n, flags, ids, n_new); });
}

mapsq_status mapsq_dict_decode(mapsq_ctx* c, const int32_t* ids, int64_t n, uint32_t flags, int64_t* offsets,
                               uint8_t* bytes, int64_t cap_bytes, int64_t* need) {
    return guarded(c, [&](Ctx* ctx) { return mq::dict_decode(ctx, ids, n, flags, offsets, bytes, cap_bytes, need); });
}

mapsq_status mapsq_dict_info(mapsq_ctx* c, int64_t* terms, int64_t* bytes) {
    return guarded(c, [&](Ctx* ctx) {
        if (!terms || !bytes) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        *terms = 0;
        *bytes = 0;
        if (!ctx->dict.made) return ctx->fail(MAPSQ_ERR_STATE, "no dictionary (mapsq_dict_create)");
        *terms = ctx->dict.nterms;
        *bytes = ctx->dict.nbytes;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_set_planner(mapsq_ctx* c, int32_t mode) {
    return guarded(c, [&](Ctx* ctx) {
        if (mode != MAPSQ_PLAN_SIZES && mode != MAPSQ_PLAN_EXACT)
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "planner mode must be MAPSQ_PLAN_SIZES or MAPSQ_PLAN_EXACT");
        ctx->planner = mode;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_last_plan(mapsq_ctx* c, mapsq_plan_step* out, int32_t cap, int32_t* n) {
    return guarded(c, [&](Ctx* ctx) {
        if (!n || cap < 0 || (cap > 0 && !out)) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "bad output arguments");
        *n = 0;
        if (ctx->last_plan.empty()) return ctx->fail(MAPSQ_ERR_STATE, "no query has completed");
        *n = (int32_t)ctx->last_plan.size();
        for (int32_t i = 0; i < std::min(cap, *n); i++) out[i] = ctx->last_plan[i];
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_set_tuning(mapsq_ctx* c, int32_t radix_bits, int32_t keys_per_thread) {
    return guarded(c, [&](Ctx* ctx) {
        if (radix_bits != 0 && (radix_bits < 4 || radix_bits > 11))
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "radix_bits must be 0 or in [4, 11]");
        if (keys_per_thread != 0 && keys_per_thread != 8 && keys_per_thread != 16)
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "keys_per_thread must be 0, 8 or 16");
        ctx->tune_rb = radix_bits;
        ctx->tune_kpt = keys_per_thread;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_profile_enable(mapsq_ctx* c, int32_t on) {
    return guarded(c, [&](Ctx* ctx) {
        (void)hipStreamSynchronize(ctx->stream);
        ctx->prof_harvest();
        ctx->acc = mapsq_profile{};
        ctx->prof = on != 0;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_profile_read(mapsq_ctx* c, mapsq_profile* out) {
    return guarded(c, [&](Ctx* ctx) {
        if (!out) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return ctx->fail(MAPSQ_ERR_HIP, hipGetErrorString(e));
        ctx->prof_harvest();
        *out = ctx->acc;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_tune_record(mapsq_ctx* c, int32_t key_bits, int32_t log2_records, int32_t radix_bits,
                               int32_t keys_per_thread) {
    return guarded(c, [&](Ctx* ctx) {
        if (key_bits < 0 || key_bits > 32 || log2_records < 0 || log2_records > 40)
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "key_bits in [0, 32], log2_records in [0, 40]");
        const uint32_t k = ((uint32_t)key_bits << 8) | (uint32_t)log2_records;
        if (radix_bits == 0) {
            ctx->tuned.erase(k);
            return (mapsq_status)MAPSQ_OK;
        }
        if (radix_bits < 4 || radix_bits > 11 || (keys_per_thread != 8 && keys_per_thread != 16))
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "radix_bits in [4, 11], keys_per_thread 8 or 16");
        ctx->tuned[k] = ((uint32_t)radix_bits << 8) | (uint32_t)keys_per_thread;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_set_mat_tuning(mapsq_ctx* c, int32_t max_blocks) {
    return guarded(c, [&](Ctx* ctx) {
        if (max_blocks != 0 && (max_blocks < 64 || max_blocks > 65536))
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "max_blocks must be 0 or in [64, 65536]");
        ctx->tune_mat_blocks = max_blocks;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_tune_record_mat(mapsq_ctx* c, int32_t log2_rows, int32_t max_blocks) {
    return guarded(c, [&](Ctx* ctx) {
        if (log2_rows < 0 || log2_rows > 41) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "log2_rows in [0, 41]");
        if (max_blocks == 0) {
            ctx->mat_tuned.erase((uint32_t)log2_rows);
            return (mapsq_status)MAPSQ_OK;
        }
        if (max_blocks < 64 || max_blocks > 65536)
            return ctx->fail(MAPSQ_ERR_INVALID_ARG, "max_blocks must be 0 or in [64, 65536]");
        ctx->mat_tuned[(uint32_t)log2_rows] = (uint32_t)max_blocks;
        return (mapsq_status)MAPSQ_OK;
    });
}

mapsq_status mapsq_arena_free_bytes(mapsq_ctx* c, uint64_t* free_bytes, uint64_t* largest_block) {
    return guarded(c, [&](Ctx* ctx) {
        if (!free_bytes || !largest_block) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output");
        *free_bytes = ctx->arena.free_bytes();
        *largest_block = ctx->arena.largest();
        return (mapsq_status)MAPSQ_OK;
    });
}

}  // extern "C"
