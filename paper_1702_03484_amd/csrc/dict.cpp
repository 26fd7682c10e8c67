// Host side of the term dictionary (mapsq_dict_*): capacity checks, staging
// of host buffers, the read-backs that size each step, and rollback of a
// batch that does not fit.  The hashing, numbering, appending and decoding
// run in k_dict.hip.
#include <algorithm>
#include <cstring>

#include "runtime.h"

namespace mq {

#define HIPCHK_D(x)                                                                                   \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) return ctx->fail(MAPSQ_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

void dict_release(Ctx* ctx) {
    Dict& d = ctx->dict;
    for (size_t off : {d.table_off, d.off_off, d.bytes_off})
        if (off != SIZE_MAX) ctx->arena.free(off);
    d = Dict{};
}

static DictDev dev_of(const Dict& d) {
    return DictDev{d.table, d.slots - 1, d.off, d.bytes, (uint32_t)d.nterms};
}

static mapsq_status sync_read(Ctx* ctx, const void* dev, size_t bytes, void* host) {
    HIPCHK_D(hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK_D(hipStreamSynchronize(ctx->stream));
    std::memcpy(host, ctx->pinned, bytes);
    return MAPSQ_OK;
}

mapsq_status dict_create(Ctx* ctx, int64_t max_terms, int64_t max_bytes) {
    if (max_terms < 1 || max_terms > (int64_t(1) << 30))
        return ctx->fail(MAPSQ_ERR_INVALID_ARG, "max_terms must be in [1, 2^30]");
    if (max_bytes < 0 || max_bytes > (int64_t(1) << 40))
        return ctx->fail(MAPSQ_ERR_INVALID_ARG, "max_bytes must be in [0, 2^40]");
    dict_release(ctx);
    Dict& d = ctx->dict;
    d.slots = 1;
    while (d.slots <= 2 * (uint64_t)max_terms) d.slots <<= 1;
    d.table_off = ctx->arena.alloc(d.slots * 8);
    d.off_off = ctx->arena.alloc(size_t(max_terms + 1) * 8);
    d.bytes_off = ctx->arena.alloc(size_t(std::max<int64_t>(max_bytes, 1)));
    if (d.table_off == SIZE_MAX || d.off_off == SIZE_MAX || d.bytes_off == SIZE_MAX) {
        dict_release(ctx);
        return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for the dictionary");
    }
    d.table = reinterpret_cast<uint64_t*>(ctx->arena.ptr(d.table_off));
    d.off = reinterpret_cast<int64_t*>(ctx->arena.ptr(d.off_off));
    d.bytes = reinterpret_cast<uint8_t*>(ctx->arena.ptr(d.bytes_off));
    d.cap_terms = max_terms;
    d.cap_bytes = max_bytes;
    HIPCHK_D(launch_fill_u64(d.table, d.slots, ~0ull, ctx->stream));
    HIPCHK_D(launch_fill_u64(reinterpret_cast<uint64_t*>(d.off), 1, 0ull, ctx->stream));
    d.made = true;
    return MAPSQ_OK;
}

mapsq_status dict_encode(Ctx* ctx, const uint8_t* bytes, const int64_t* offsets, int64_t n, uint32_t flags,
                         int32_t* ids, int64_t* n_new) {
    Dict& d = ctx->dict;
    if (n_new) *n_new = 0;
    if (!d.made) return ctx->fail(MAPSQ_ERR_STATE, "no dictionary (mapsq_dict_create)");
    if (flags & ~(MAPSQ_DICT_DEVICE_PTRS | MAPSQ_DICT_LOOKUP)) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "unknown flags");
    if (n < 0 || (n > 0 && (!offsets || !ids))) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "bad batch arguments");
    if (n > (int64_t)DICT_SCAN_MAX || n > d.cap_terms)
        return ctx->fail(MAPSQ_ERR_CAPACITY, "a batch holds at most min(2^26, max_terms) terms");
    if (n == 0) return MAPSQ_OK;
    const bool dev = flags & MAPSQ_DICT_DEVICE_PTRS;
    const bool insert = !(flags & MAPSQ_DICT_LOOKUP);
    const uint32_t nn = (uint32_t)n;

    // the batch on the device, its offsets checked before any byte is read
    Block sb, so;
    const uint8_t* tb = bytes;
    const int64_t* to = offsets;
    int64_t total = 0;
    Block sc = alloc_block(ctx, 64);  // scalars: err, new terms, new bytes, total
    if (!sc.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for dictionary scalars");
    uint32_t* err = sc.as<uint32_t>();
    uint32_t* new_terms = err + 2;
    uint64_t* new_bytes = reinterpret_cast<uint64_t*>(err + 4);
    HIPCHK_D(launch_fill_u32(err, 16, 0u, ctx->stream));
    if (dev) {
        HIPCHK_D(launch_dict_check_offsets(offsets, nn, err, ctx->stream));
        uint32_t e = 0;
        if (mapsq_status st = sync_read(ctx, err, 4, &e)) return st;
        if (e) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "offsets must start at 0 and not decrease");
        if (mapsq_status st = sync_read(ctx, offsets + n, 8, &total)) return st;
    } else {
        if (offsets[0] != 0) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "offsets must start at 0 and not decrease");
        for (int64_t i = 0; i < n; i++)
            if (offsets[i + 1] < offsets[i])
                return ctx->fail(MAPSQ_ERR_INVALID_ARG, "offsets must start at 0 and not decrease");
        total = offsets[n];
        if (total > 0 && !bytes) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null bytes");
        sb = alloc_block(ctx, size_t(std::max<int64_t>(total, 1)));
        so = alloc_block(ctx, size_t(n + 1) * 8);
        if (!sb.ok() || !so.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room to stage the batch");
        HIPCHK_D(hipMemcpyAsync(sb.as<void>(), bytes, size_t(total), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK_D(hipMemcpyAsync(so.as<void>(), offsets, size_t(n + 1) * 8, hipMemcpyHostToDevice, ctx->stream));
        tb = sb.as<uint8_t>();
        to = so.as<int64_t>();
    }
    if (total > 0 && !tb) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null bytes");

    const size_t a4 = align_up(size_t(n) * 4, ARENA_ALIGN), a8 = align_up(size_t(n) * 8, ARENA_ALIGN);
    Block ws = alloc_block(ctx, 4 * a4 + 2 * a8 + align_up(scan_part_bytes(nn), ARENA_ALIGN) +
                                    (dev ? 0 : a4));
    if (!ws.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for dictionary scratch");
    char* w0 = ctx->arena.ptr(ws.off);
    DictScratch w{};
    w.rep = reinterpret_cast<uint32_t*>(w0);
    w.first = reinterpret_cast<uint32_t*>(w0 + a4);
    w.flag = reinterpret_cast<uint32_t*>(w0 + 2 * a4);
    w.rank = reinterpret_cast<uint32_t*>(w0 + 3 * a4);
    w.blen = reinterpret_cast<uint64_t*>(w0 + 4 * a4);
    w.boff = reinterpret_cast<uint64_t*>(w0 + 4 * a4 + a8);
    w.part = w0 + 4 * a4 + 2 * a8;
    int32_t* ids_dev = dev ? ids : reinterpret_cast<int32_t*>(w0 + 4 * a4 + 2 * a8 +
                                                             align_up(scan_part_bytes(nn), ARENA_ALIGN));
    w.err = err;
    w.new_terms = new_terms;
    w.new_bytes = new_bytes;
    HIPCHK_D(launch_fill_u32(w.first, nn, ~0u, ctx->stream));
    const TermsDev t{tb, to, nn};
    const DictDev dd = dev_of(d);
    HIPCHK_D(launch_dict_encode_front(dd, t, insert ? 1 : 0, w, ctx->stream));
    uint32_t sv[6];  // err, pad, new terms, pad, new bytes (2 words)
    if (mapsq_status st = sync_read(ctx, err, sizeof(sv), sv)) return st;
    if (sv[0] & 2) {
        if (insert) (void)launch_dict_commit(dd, t, w, (uint32_t)d.nterms, d.nbytes, 0, ctx->stream);
        return ctx->fail(MAPSQ_ERR_HIP, "dictionary table full");
    }
    uint32_t added = insert ? sv[2] : 0;
    uint64_t added_bytes = 0;
    if (insert) std::memcpy(&added_bytes, &sv[4], 8);
    if (insert && (d.nterms + (int64_t)added > d.cap_terms || d.nbytes + (int64_t)added_bytes > d.cap_bytes)) {
        HIPCHK_D(launch_dict_commit(dd, t, w, (uint32_t)d.nterms, d.nbytes, 0, ctx->stream));
        HIPCHK_D(hipStreamSynchronize(ctx->stream));
        return ctx->fail(MAPSQ_ERR_CAPACITY, "dictionary full: " + std::to_string(d.nterms + added) + " terms, " +
                                                 std::to_string(d.nbytes + (int64_t)added_bytes) + " bytes");
    }
    HIPCHK_D(launch_dict_ids(t, w, (uint32_t)d.nterms, ids_dev, ctx->stream));
    if (insert) {
        HIPCHK_D(launch_dict_commit(dd, t, w, (uint32_t)d.nterms, d.nbytes, 1, ctx->stream));
        HIPCHK_D(launch_fill_u64(reinterpret_cast<uint64_t*>(d.off + d.nterms + added), 1,
                                 (uint64_t)(d.nbytes + (int64_t)added_bytes), ctx->stream));
        d.nterms += added;
        d.nbytes += (int64_t)added_bytes;
    }
    if (!dev) HIPCHK_D(hipMemcpyAsync(ids, ids_dev, size_t(n) * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK_D(hipStreamSynchronize(ctx->stream));
    if (n_new) *n_new = added;
    return MAPSQ_OK;
}

mapsq_status dict_decode(Ctx* ctx, const int32_t* ids, int64_t n, uint32_t flags, int64_t* offsets, uint8_t* bytes,
                         int64_t cap_bytes, int64_t* need_bytes) {
    Dict& d = ctx->dict;
    if (need_bytes) *need_bytes = 0;
    if (!d.made) return ctx->fail(MAPSQ_ERR_STATE, "no dictionary (mapsq_dict_create)");
    if (flags & ~MAPSQ_DICT_DEVICE_PTRS) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "unknown flags");
    if (n < 0 || (n > 0 && !ids) || !offsets || cap_bytes < 0)
        return ctx->fail(MAPSQ_ERR_INVALID_ARG, "bad decode arguments");
    if (n > (int64_t)DICT_SCAN_MAX) return ctx->fail(MAPSQ_ERR_CAPACITY, "a decode holds at most 2^26 identifiers");
    const bool dev = flags & MAPSQ_DICT_DEVICE_PTRS;
    if (n == 0) {
        const int64_t zero = 0;
        if (dev)
            HIPCHK_D(hipMemcpyAsync(offsets, &zero, 8, hipMemcpyHostToDevice, ctx->stream));
        else
            offsets[0] = 0;
        HIPCHK_D(hipStreamSynchronize(ctx->stream));
        return MAPSQ_OK;
    }
    const uint32_t nn = (uint32_t)n;
    const size_t a8 = align_up(size_t(n) * 8, ARENA_ALIGN), a4 = align_up(size_t(n) * 4, ARENA_ALIGN);
    Block ws = alloc_block(ctx, 2 * a8 + a4 + align_up(scan_part_bytes(nn), ARENA_ALIGN) + 64);
    if (!ws.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room for decode scratch");
    char* w0 = ctx->arena.ptr(ws.off);
    uint64_t* len = reinterpret_cast<uint64_t*>(w0);
    uint64_t* pos = reinterpret_cast<uint64_t*>(w0 + a8);
    int32_t* ids_dev = reinterpret_cast<int32_t*>(w0 + 2 * a8);
    void* part = w0 + 2 * a8 + a4;
    uint32_t* err = reinterpret_cast<uint32_t*>(w0 + 2 * a8 + a4 + align_up(scan_part_bytes(nn), ARENA_ALIGN));
    uint64_t* total = reinterpret_cast<uint64_t*>(err + 2);
    HIPCHK_D(launch_fill_u32(err, 4, 0u, ctx->stream));
    if (dev)
        ids_dev = const_cast<int32_t*>(ids);
    else
        HIPCHK_D(hipMemcpyAsync(ids_dev, ids, size_t(n) * 4, hipMemcpyHostToDevice, ctx->stream));
    const DictDev dd = dev_of(d);
    HIPCHK_D(launch_dict_decode(dd, ids_dev, nn, len, pos, total, part, err, ctx->stream));
    uint32_t sv[4];
    if (mapsq_status st = sync_read(ctx, err, sizeof(sv), sv)) return st;
    if (sv[0]) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "an identifier outside the dictionary");
    uint64_t need;
    std::memcpy(&need, &sv[2], 8);
    if (need_bytes) *need_bytes = (int64_t)need;
    if ((int64_t)need > cap_bytes)
        return ctx->fail(MAPSQ_ERR_TOO_LARGE, "decoded terms need " + std::to_string(need) + " bytes");
    if (need > 0 && !bytes) return ctx->fail(MAPSQ_ERR_INVALID_ARG, "null output bytes");
    Block ob;
    uint8_t* out = bytes;
    if (!dev) {
        ob = alloc_block(ctx, size_t(std::max<uint64_t>(need, 1)));
        if (!ob.ok()) return ctx->fail(MAPSQ_ERR_CAPACITY, "arena: no room to stage decoded terms");
        out = ob.as<uint8_t>();
    }
    HIPCHK_D(launch_dict_gather(dd, ids_dev, nn, pos, out, ctx->stream));
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK_D(hipMemcpyAsync(offsets, pos, size_t(n) * 8, k, ctx->stream));
    HIPCHK_D(hipMemcpyAsync(offsets + n, total, 8, k, ctx->stream));
    if (!dev && need > 0) HIPCHK_D(hipMemcpyAsync(bytes, out, size_t(need), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK_D(hipStreamSynchronize(ctx->stream));
    return MAPSQ_OK;
}

}  // namespace mq
