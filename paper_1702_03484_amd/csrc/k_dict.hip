// Dictionary encoding of RDF terms on gfx950: byte-string terms <-> dense
// int32 identifiers, numbered in order of first appearance (the terms of
// Table 1 become the identifiers the join works on, and results decode back
// to terms).
//
// Encoding a batch of n terms (concatenated bytes + n + 1 offsets):
//   hash     FNV-1a (Fowler-Noll-Vo, 64-bit) of every term;
//   insert   open addressing with linear probing into a table of 64-bit
//            slots [hash >> 32 | ref]: ref is a dictionary identifier, or
//            (bit 31 set) the index of the batch's term that claimed the slot
//            with a 64-bit CAS.  A slot is never emptied while terms are
//            being inserted, so equal terms meet at the first slot their
//            probe sequence finds free or holding them;
//   first    per claimed slot, the lowest batch index of its term (atomicMin);
//   number   the first occurrences of new terms, scanned in batch order,
//            become identifiers dictionary_size + rank;
//   append   their bytes go to the dictionary's byte store (offsets from a
//            scan of their lengths) and the table's slots are re-pointed from
//            batch indices to identifiers.
// Decoding gathers each identifier's bytes to offsets from a scan of lengths.
#include "device_common.h"
#include "kernels.h"

#include <algorithm>

namespace mq {

constexpr uint32_t DICT_NEW = 1u << 31;      // ref names a batch index
constexpr uint32_t DICT_NONE = 0xFFFFFFFFu;  // term absent (lookups)
constexpr uint64_t DICT_EMPTY = ~0ull;

static uint32_t grid_of(uint64_t n, uint32_t per_block = 256 * 4, uint32_t cap = 16384) {
    const uint64_t g = (n + per_block - 1) / per_block;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

// FNV-1a, 64-bit: offset basis and prime of the published definition.
__device__ __forceinline__ uint64_t fnv1a64(const uint8_t* p, int64_t len) {
    uint64_t h = 14695981039346656037ull;
    for (int64_t k = 0; k < len; k++) {
        h ^= p[k];
        h *= 1099511628211ull;
    }
    return h;
}

__device__ __forceinline__ bool same_bytes(const uint8_t* a, const uint8_t* b, int64_t len) {
    for (int64_t k = 0; k < len; k++)
        if (a[k] != b[k]) return false;
    return true;
}

// offsets non-decreasing from 0: err |= 1 otherwise
__global__ void dict_check_offsets_kernel(const int64_t* __restrict__ off, uint32_t n, uint32_t* err) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        const bool bad = i == 0 ? off[0] != 0 : off[i] < off[i - 1];
        if (bad) atomicOr(err, 1u);
    }
}

__global__ void dict_insert_kernel(DictDev d, TermsDev t, int insert, uint32_t* __restrict__ rep,
                                   uint32_t* __restrict__ err) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < t.n; i += gridDim.x * blockDim.x) {
        const uint8_t* p = t.bytes + t.off[i];
        const int64_t len = t.off[i + 1] - t.off[i];
        const uint64_t h = fnv1a64(p, len);
        const uint64_t tag = h >> 32;
        const uint64_t mine = tag << 32 | (DICT_NEW | i);
        uint64_t slot = h & d.mask;
        uint32_t r = DICT_NONE;
        bool done = false;
        for (uint64_t probe = 0; probe <= d.mask && !done; probe++, slot = (slot + 1) & d.mask) {
            uint64_t cur = __hip_atomic_load(d.table + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur == DICT_EMPTY) {
                if (!insert) {
                    done = true;  // r stays DICT_NONE
                    break;
                }
                const uint64_t prev = atomicCAS((unsigned long long*)(d.table + slot), DICT_EMPTY, mine);
                if (prev == DICT_EMPTY) {
                    r = DICT_NEW | i;
                    done = true;
                    break;
                }
                cur = prev;
            }
            if ((cur >> 32) != tag) continue;
            const uint32_t ref = (uint32_t)cur;
            const uint8_t* q;
            int64_t qlen;
            if (ref & DICT_NEW) {
                const uint32_t j = ref & ~DICT_NEW;
                q = t.bytes + t.off[j];
                qlen = t.off[j + 1] - t.off[j];
            } else {
                q = d.bytes + d.off[ref];
                qlen = d.off[ref + 1] - d.off[ref];
            }
            if (qlen == len && same_bytes(p, q, len)) {
                r = ref;
                done = true;
            }
        }
        if (!done) atomicOr(err, 2u);  // table full: cannot happen within the capacity checks
        rep[i] = r;
    }
}

// first[j] = lowest batch index whose term claimed slot-owner j (first[]
// pre-set to ~0).  A plain read skips the atomic once a lower index is in:
// a frequent term would otherwise send every occurrence's atomic to one
// address, and those serialise.
__global__ void dict_first_kernel(const uint32_t* __restrict__ rep, uint32_t n, uint32_t* __restrict__ first) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t r = rep[i];
        if (r == DICT_NONE || !(r & DICT_NEW)) continue;
        uint32_t* f = first + (r & ~DICT_NEW);
        if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > i) atomicMin(f, i);
    }
}

// flag[i] = 1 and blen[i] = its length when term i is the first occurrence
// of a term new to the dictionary
__global__ void dict_flags_kernel(TermsDev t, const uint32_t* __restrict__ rep, const uint32_t* __restrict__ first,
                                  uint32_t* __restrict__ flag, uint64_t* __restrict__ blen) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < t.n; i += gridDim.x * blockDim.x) {
        const uint32_t r = rep[i];
        const bool f = r != DICT_NONE && (r & DICT_NEW) && first[r & ~DICT_NEW] == i;
        flag[i] = f ? 1u : 0u;
        blen[i] = f ? (uint64_t)(t.off[i + 1] - t.off[i]) : 0ull;
    }
}

// identifiers: a dictionary term keeps its own, a new term takes
// base + rank of its first occurrence, an absent one (lookup) -1
__global__ void dict_ids_kernel(const uint32_t* __restrict__ rep, const uint32_t* __restrict__ first,
                                const uint32_t* __restrict__ rank, uint32_t n, uint32_t base,
                                int32_t* __restrict__ ids) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t r = rep[i];
        ids[i] = r == DICT_NONE ? -1 : (r & DICT_NEW) ? (int32_t)(base + rank[first[r & ~DICT_NEW]]) : (int32_t)r;
    }
}

// new terms into the byte store; one wave per term, lanes copy its bytes
__global__ __launch_bounds__(256) void dict_append_kernel(DictDev d, TermsDev t, const uint32_t* __restrict__ flag,
                                                          const uint32_t* __restrict__ rank,
                                                          const uint64_t* __restrict__ boff, uint32_t base,
                                                          int64_t bbase) {
    const uint32_t waves = gridDim.x * (blockDim.x / MQ_WAVE);
    for (uint32_t i = blockIdx.x * (blockDim.x / MQ_WAVE) + threadIdx.x / MQ_WAVE; i < t.n; i += waves) {
        if (!flag[i]) continue;
        const int64_t at = bbase + (int64_t)boff[i];
        const int64_t len = t.off[i + 1] - t.off[i];
        const uint8_t* src = t.bytes + t.off[i];
        for (int64_t k = lane(); k < len; k += MQ_WAVE) d.bytes[at + k] = src[k];
        if (lane() == 0) d.off[base + rank[i]] = at;
    }
}

// slots claimed by batch terms now name their identifiers (commit) or are
// emptied again (rollback: the table is back to its state before the batch)
__global__ void dict_fix_kernel(DictDev d, const uint32_t* __restrict__ first, const uint32_t* __restrict__ rank,
                                uint32_t base, int commit) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s <= d.mask;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t w = d.table[s];
        if (w == DICT_EMPTY || !((uint32_t)w & DICT_NEW)) continue;
        d.table[s] = commit ? (w & 0xFFFFFFFF00000000ull) | (uint64_t)(base + rank[first[(uint32_t)w & ~DICT_NEW]])
                            : DICT_EMPTY;
    }
}

// decoding: lengths (err |= 1 for an identifier outside [0, nterms))
__global__ void dict_lens_kernel(DictDev d, const int32_t* __restrict__ ids, uint32_t n, uint64_t* __restrict__ len,
                                 uint32_t* __restrict__ err) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t id = ids[i];
        if (id < 0 || (uint32_t)id >= d.nterms) {
            atomicOr(err, 1u);
            len[i] = 0;
        } else {
            len[i] = (uint64_t)(d.off[id + 1] - d.off[id]);
        }
    }
}

// decoding: one wave per term copies its bytes to out + pos[i]
__global__ __launch_bounds__(256) void dict_gather_kernel(DictDev d, const int32_t* __restrict__ ids, uint32_t n,
                                                          const uint64_t* __restrict__ pos, uint8_t* __restrict__ out) {
    const uint32_t waves = gridDim.x * (blockDim.x / MQ_WAVE);
    for (uint32_t i = blockIdx.x * (blockDim.x / MQ_WAVE) + threadIdx.x / MQ_WAVE; i < n; i += waves) {
        const int32_t id = ids[i];
        const int64_t a = d.off[id], len = d.off[id + 1] - a;
        for (int64_t k = lane(); k < len; k += MQ_WAVE) out[pos[i] + k] = d.bytes[a + k];
    }
}

// ---- exclusive scan of up to SCAN_MAX values (three launches) -------------
constexpr uint32_t SCAN_IPT = 8;
constexpr uint32_t SCAN_TILE = MQ_BLOCK * SCAN_IPT;

template <typename T>
__global__ __launch_bounds__(MQ_BLOCK) void scan_reduce_kernel(const T* __restrict__ in, uint32_t n,
                                                               T* __restrict__ part) {
    __shared__ T tmp[MQ_WAVES];
    const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_IPT;
    T s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_IPT; k++) s += base + k < n ? in[base + k] : T(0);
    s = wave_sum(s);
    if (lane() == 0) tmp[threadIdx.x / MQ_WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int w = 0; w < MQ_WAVES; w++) t += tmp[w];
        part[blockIdx.x] = t;
    }
}

// one block: part[0..np) -> exclusive prefixes, *total = sum
template <typename T>
__global__ __launch_bounds__(MQ_BLOCK) void scan_parts_kernel(T* __restrict__ part, uint32_t np, T* __restrict__ total) {
    __shared__ T tmp[MQ_WAVES];
    const uint32_t per = (np + MQ_BLOCK - 1) / MQ_BLOCK;
    const uint32_t b0 = threadIdx.x * per, b1 = min(b0 + per, np);
    T s = 0;
    for (uint32_t k = b0; k < b1; k++) s += part[k];
    T all;
    T run = block_excl_scan<T>(s, tmp, &all);
    for (uint32_t k = b0; k < b1; k++) {
        const T v = part[k];
        part[k] = run;
        run += v;
    }
    if (threadIdx.x == 0) *total = all;
}

template <typename T>
__global__ __launch_bounds__(MQ_BLOCK) void scan_write_kernel(const T* __restrict__ in, uint32_t n,
                                                              const T* __restrict__ part, T* __restrict__ out) {
    __shared__ T tmp[MQ_WAVES];
    const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_IPT;
    T v[SCAN_IPT];
    T s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_IPT; k++) {
        v[k] = base + k < n ? in[base + k] : T(0);
        s += v[k];
    }
    T all;
    T run = part[blockIdx.x] + block_excl_scan<T>(s, tmp, &all);
#pragma unroll
    for (uint32_t k = 0; k < SCAN_IPT; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

size_t scan_part_bytes(uint32_t n) { return 8ull * ((n + SCAN_TILE - 1) / SCAN_TILE + 1); }

template <typename T>
static hipError_t scan_excl(const T* in, uint32_t n, T* out, T* total, void* part_scratch, hipStream_t s) {
    if (n > DICT_SCAN_MAX) return hipErrorInvalidValue;
    const uint32_t np = std::max<uint32_t>(1, (n + SCAN_TILE - 1) / SCAN_TILE);
    T* part = static_cast<T*>(part_scratch);
    if (n == 0) return hipErrorInvalidValue;  // callers skip empty batches
    scan_reduce_kernel<T><<<np, MQ_BLOCK, 0, s>>>(in, n, part);
    scan_parts_kernel<T><<<1, MQ_BLOCK, 0, s>>>(part, np, total);
    scan_write_kernel<T><<<np, MQ_BLOCK, 0, s>>>(in, n, part, out);
    return hipGetLastError();
}

// ---- launchers ------------------------------------------------------------
hipError_t launch_dict_check_offsets(const int64_t* off, uint32_t n, uint32_t* err, hipStream_t s) {
    dict_check_offsets_kernel<<<grid_of(uint64_t(n) + 1), 256, 0, s>>>(off, n, err);
    return hipGetLastError();
}

hipError_t launch_dict_encode_front(const DictDev& d, const TermsDev& t, int insert, DictScratch w, hipStream_t s) {
    if (t.n == 0) return hipSuccess;
    dict_insert_kernel<<<grid_of(t.n, 256, 65536), 256, 0, s>>>(d, t, insert, w.rep, w.err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !insert) return e;
    dict_first_kernel<<<grid_of(t.n), 256, 0, s>>>(w.rep, t.n, w.first);
    dict_flags_kernel<<<grid_of(t.n), 256, 0, s>>>(t, w.rep, w.first, w.flag, w.blen);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_excl<uint32_t>(w.flag, t.n, w.rank, w.new_terms, w.part, s)) != hipSuccess) return e;
    return scan_excl<uint64_t>(w.blen, t.n, w.boff, w.new_bytes, w.part, s);
}

hipError_t launch_dict_ids(const TermsDev& t, DictScratch w, uint32_t base, int32_t* ids, hipStream_t s) {
    if (t.n == 0) return hipSuccess;
    dict_ids_kernel<<<grid_of(t.n), 256, 0, s>>>(w.rep, w.first, w.rank, t.n, base, ids);
    return hipGetLastError();
}

hipError_t launch_dict_commit(const DictDev& d, const TermsDev& t, DictScratch w, uint32_t base, int64_t bbase,
                              int commit, hipStream_t s) {
    if (t.n == 0) return hipSuccess;
    if (commit) {
        dict_append_kernel<<<grid_of(uint64_t(t.n) * MQ_WAVE, 256, 32768), 256, 0, s>>>(d, t, w.flag, w.rank, w.boff,
                                                                                         base, bbase);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dict_fix_kernel<<<grid_of(d.mask + 1), 256, 0, s>>>(d, w.first, w.rank, base, commit);
    return hipGetLastError();
}

hipError_t launch_dict_decode(const DictDev& d, const int32_t* ids, uint32_t n, uint64_t* len, uint64_t* pos,
                              uint64_t* total, void* part, uint32_t* err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dict_lens_kernel<<<grid_of(n), 256, 0, s>>>(d, ids, n, len, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_excl<uint64_t>(len, n, pos, total, part, s);
}

hipError_t launch_dict_gather(const DictDev& d, const int32_t* ids, uint32_t n, const uint64_t* pos, uint8_t* out,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    dict_gather_kernel<<<grid_of(uint64_t(n) * MQ_WAVE, 256, 32768), 256, 0, s>>>(d, ids, n, pos, out);
    return hipGetLastError();
}

}  // namespace mq
