// Host-only part of the runtime: the first-fit sub-allocator over the
// caller's arena and small table helpers.  Nothing here touches the device,
// so the serving scheduler can be built and exercised on a host without a
// GPU against a simulated executor.
#include <algorithm>
#include <cstring>

#include "runtime.h"

namespace mq {

void Arena::init(char* base, size_t size) {
    base_ = base;
    size_ = size / ARENA_ALIGN * ARENA_ALIGN;
    free_.clear();
    used_.clear();
    if (size_) free_[0] = size_;
}

size_t Arena::alloc(size_t bytes) {
    if (fail_after >= 0 && fail_after-- == 0) return SIZE_MAX;
    bytes = align_up(std::max<size_t>(bytes, 1), ARENA_ALIGN);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
            size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > bytes) free_[off + bytes] = sz - bytes;
            used_[off] = bytes;
            return off;
        }
    }
    return SIZE_MAX;
}

void Arena::free(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t sz = u->second;
    used_.erase(u);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + sz == nx->first) {
        sz += nx->second;
        nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += sz;
            return;
        }
    }
    free_[off] = sz;
}

void Arena::shrink(size_t off, size_t bytes) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    bytes = align_up(std::max<size_t>(bytes, 1), ARENA_ALIGN);
    if (bytes >= u->second) return;
    size_t tail = off + bytes, tsz = u->second - bytes;
    u->second = bytes;
    used_[tail] = tsz;
    free(tail);
}

size_t Arena::free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
}

size_t Arena::largest() const {
    size_t s = 0;
    for (auto& kv : free_) s = std::max(s, kv.second);
    return s;
}

void Block::reset() {
    if (ctx && off != SIZE_MAX) ctx->arena.free(off);
    off = SIZE_MAX;
}

Block alloc_block(Ctx* ctx, size_t bytes) {
    Block b;
    b.ctx = ctx;
    b.off = ctx->arena.alloc(bytes);
    return b;
}

int col_of(const mapsq_table* t, int32_t v) {
    for (int c = 0; c < t->ncols; c++)
        if (t->var[c] == v) return c;
    return -1;
}

static void zero_table(mapsq_table* t) { std::memset(t, 0, sizeof(*t)); }

// Allocate an owned table of `rows` rows x `ncols` columns (one block), or
// hand out the caller's output columns when the context has them.
mapsq_status alloc_table(Ctx* ctx, int64_t rows, int ncols, mapsq_table* t) {
    if (ctx->out_cols) {
        if (rows > ctx->out_cap) return MAPSQ_ERR_CAPACITY;
        t->owned = 0;
        t->block = 0;
        t->ncols = ncols;
        t->nrows = rows;
        for (int c = 0; c < ncols; c++) t->col[c] = ctx->out_cols[c];
        return MAPSQ_OK;
    }
    const size_t colb = align_up(size_t(std::max<int64_t>(rows, 1)) * 4, ARENA_ALIGN);
    size_t off = ctx->arena.alloc(colb * std::max(ncols, 1));
    if (off == SIZE_MAX) return MAPSQ_ERR_CAPACITY;
    t->owned = 1;
    t->block = off + 1;
    t->ncols = ncols;
    t->nrows = rows;
    for (int c = 0; c < ncols; c++) t->col[c] = reinterpret_cast<int32_t*>(ctx->arena.ptr(off + c * colb));
    return MAPSQ_OK;
}

mapsq_status free_table(Ctx* ctx, mapsq_table* t) {
    if (t->owned && t->block) {
        const size_t off = size_t(t->block - 1);
        auto it = ctx->shared_refs.find(off);
        if (it != ctx->shared_refs.end() && --it->second > 0) {
            zero_table(t);
            return MAPSQ_OK;
        }
        if (it != ctx->shared_refs.end()) ctx->shared_refs.erase(it);
        ctx->arena.free(off);
    }
    zero_table(t);
    return MAPSQ_OK;
}

}  // namespace mq
