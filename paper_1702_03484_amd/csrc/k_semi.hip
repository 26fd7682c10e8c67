// Semi-join reduction ahead of the shuffle.  A record whose key does not
// occur on the other side of the join meets no partner in Reduce and gives
// no output row, so it need not be sorted at all.  When one side is much
// larger, the smaller side's keys go into a bitmap over the key range and
// the larger side is filtered against it in one pass that also writes the
// surviving records (relative key, record id) in input order, ready for the
// first radix pass.  Because the kept records keep their order and ids,
// the sorted sequence is the unfiltered one with only unmatched keys'
// records removed, and the join's rows come out unchanged, row for row.
#include "device_common.h"
#include "kernels.h"

#include <algorithm>

namespace mq {

constexpr int SEMI_IPT = 16;

// keys outside [base, base + range) (a caller's key bound that does not
// hold) set nothing.  Of a run of equal keys in consecutive lanes (a side
// sorted on the key) only the first lane sets the bit, and a bit found set
// already is not set again, so repeated keys do not queue on one word.
__global__ __launch_bounds__(MQ_BLOCK) void bitmap_set_kernel(const int32_t* __restrict__ keys, uint32_t n,
                                                              int32_t base, uint64_t range, uint32_t* __restrict__ bm) {
    for (uint32_t i0 = blockIdx.x * MQ_BLOCK; i0 < n; i0 += gridDim.x * MQ_BLOCK) {
        const uint32_t i = i0 + threadIdx.x;
        const uint32_t k = i < n ? (uint32_t)keys[i] - (uint32_t)base : ~0u;
        const uint32_t kp = __shfl_up(k, 1, MQ_WAVE);
        const bool first = lane() == 0 || kp != k;
        if (i < n && first && k < range) {
            const uint32_t bit = 1u << (k & 31u);
            if (!(__hip_atomic_load(&bm[k >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit))
                atomicOr(&bm[k >> 5], bit);
        }
    }
}

// Persistent tiles of 256 x SEMI_IPT records: one __ballot per record slot,
// wave totals scanned in LDS, the tile's output offset from a decoupled
// look-back; kept records are written in input order.
__global__ __launch_bounds__(MQ_BLOCK) void semi_filter_kernel(SemiArgs a, uint64_t* __restrict__ status,
                                                               uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint32_t TILE = MQ_BLOCK * SEMI_IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wtot[MQ_WAVES];
    __shared__ uint64_t s_excl;
    const uint32_t ntiles = (a.n + TILE - 1) / TILE;
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    for (;;) {
        const uint32_t tile = next_tile(tile_ctr, &s_tile);
        if (tile >= ntiles) break;
        const uint32_t base = tile * TILE;
        uint32_t key[SEMI_IPT];
        uint64_t km[SEMI_IPT];
#pragma unroll
        for (int i = 0; i < SEMI_IPT; i++) {
            const uint32_t idx = base + (w * SEMI_IPT + i) * MQ_WAVE + lane();
            key[i] = idx < a.n ? (uint32_t)a.keys[idx] - (uint32_t)a.base : 0u;
        }
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < SEMI_IPT; i++) {
            const uint32_t idx = base + (w * SEMI_IPT + i) * MQ_WAVE + lane();
            const bool ok = idx < a.n && key[i] < a.range && ((a.bm[key[i] >> 5] >> (key[i] & 31u)) & 1u);
            km[i] = __ballot(ok);
            run += (uint32_t)__popcll(km[i]);
        }
        if (lane() == 0) s_wtot[w] = run;
        __syncthreads();
        uint32_t wex = 0, ttot = 0;
#pragma unroll
        for (int i = 0; i < MQ_WAVES; i++) {
            if ((uint32_t)i < w) wex += s_wtot[i];
            ttot += s_wtot[i];
        }
        if (w == 0) {
            const uint64_t ex = tile_prefix_wave0(status, tile, epoch, ttot);
            if (lane() == 0) {
                s_excl = ex;
                if (tile == ntiles - 1) *a.count = (uint32_t)(ex + ttot);
            }
        }
        __syncthreads();
        uint32_t pos = (uint32_t)s_excl + wex;
        for (int i = 0; i < SEMI_IPT; i++) {  // fully unrolled by the compiler (km stays in registers)
            if ((km[i] >> lane()) & 1ull) {
                const uint32_t idx = base + (w * SEMI_IPT + i) * MQ_WAVE + lane();
                const uint32_t at = pos + (uint32_t)__popcll(km[i] & lt);
                a.kout[at] = key[i];
                a.vout[at] = a.id_base + idx;
            }
            pos += (uint32_t)__popcll(km[i]);
        }
    }
}

// Every record of one side, written from position (*at_dev if given) + i.
__global__ __launch_bounds__(MQ_BLOCK) void side_records_kernel(const int32_t* __restrict__ keys, uint32_t n,
                                                                int32_t base, uint32_t id_base,
                                                                const uint32_t* __restrict__ at_dev,
                                                                uint32_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout) {
    const uint32_t at = at_dev ? *at_dev : 0u;
    for (uint32_t i = blockIdx.x * MQ_BLOCK + threadIdx.x; i < n; i += gridDim.x * MQ_BLOCK) {
        kout[at + i] = (uint32_t)keys[i] - (uint32_t)base;
        vout[at + i] = id_base + i;
    }
}

hipError_t launch_bitmap_set(const int32_t* keys, uint32_t n, int32_t base, uint64_t range, uint32_t* bm,
                             hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((n + MQ_BLOCK - 1) / MQ_BLOCK, 2048u);
    bitmap_set_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(keys, n, base, range, bm);
    return hipGetLastError();
}

hipError_t launch_semi_filter(const SemiArgs& a, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch,
                              hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    const uint32_t tiles = (a.n + MQ_BLOCK * SEMI_IPT - 1) / (MQ_BLOCK * SEMI_IPT);
    const uint32_t blocks = std::min<uint32_t>(tiles, 256u * 8u);
    semi_filter_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(a, status, tile_ctr, epoch);
    return hipGetLastError();
}

uint32_t semi_filter_tiles(uint32_t n) { return (n + MQ_BLOCK * SEMI_IPT - 1) / (MQ_BLOCK * SEMI_IPT); }

hipError_t launch_side_records(const int32_t* keys, uint32_t n, int32_t base, uint32_t id_base,
                               const uint32_t* at_dev, uint32_t* kout, uint32_t* vout, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((n + MQ_BLOCK - 1) / MQ_BLOCK, 2048u);
    side_records_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(keys, n, base, id_base, at_dev, kout, vout);
    return hipGetLastError();
}

}  // namespace mq

namespace mq {

// Exact |RS| before any shuffle: the smaller side's keys are counted into a
// dense array over the key range, then every record of the larger side
// adds the count of its key (sum over keys of cL * cR, Algorithm 1's
// ReduceDuplicate without grouping).  Keys outside [base, base + range)
// count nothing.
// Each thread counts 16 consecutive keys, one atomic per run of equal keys;
// when the wave's 1024 keys are all one key (a hot key of a key-sorted
// side) one atomic counts them all, so hot keys do not serialise.
constexpr int KC_IPT = 16;

__global__ __launch_bounds__(MQ_BLOCK) void key_count_kernel(const int32_t* __restrict__ keys, uint32_t n, int32_t base,
                                                             uint64_t range, uint32_t* __restrict__ cnt) {
    constexpr uint32_t TILE = MQ_BLOCK * KC_IPT;
    for (uint64_t t0 = (uint64_t)blockIdx.x * TILE; t0 < n; t0 += (uint64_t)gridDim.x * TILE) {
        const uint64_t first = t0 + (uint64_t)threadIdx.x * KC_IPT;
        uint32_t k[KC_IPT];
#pragma unroll
        for (int i = 0; i < KC_IPT; i++)
            k[i] = first + i < n ? (uint32_t)keys[first + i] - (uint32_t)base : 0xffffffffu;
        const int cnt_here = first >= n ? 0 : (int)min((uint64_t)KC_IPT, n - first);
        const bool full = __ballot(cnt_here == KC_IPT) == ~0ull;
        const uint32_t k0 = __shfl(k[0], 0, MQ_WAVE), k1 = __shfl(k[KC_IPT - 1], MQ_WAVE - 1, MQ_WAVE);
        if (full && k0 == k1) {
            // sorted input, one key over the whole wave (unsorted input with
            // this property is one key too: the test is exact either way)
            bool same = true;
#pragma unroll
            for (int i = 0; i < KC_IPT; i++) same = same && k[i] == k0;
            if (__ballot(!same) == 0ull) {
                if (lane() == 0 && k0 < range) atomicAdd(&cnt[k0], (uint32_t)(MQ_WAVE * KC_IPT));
                continue;
            }
        }
        uint32_t cur = k[0], run = 0;
#pragma unroll
        for (int i = 0; i < KC_IPT; i++) {
            if (i < cnt_here) {
                if (k[i] != cur) {
                    if (cur < range) atomicAdd(&cnt[cur], run);
                    cur = k[i];
                    run = 0;
                }
                run++;
            }
        }
        if (run && cur < range) atomicAdd(&cnt[cur], run);
    }
}

__global__ __launch_bounds__(MQ_BLOCK) void key_dot_kernel(const int32_t* __restrict__ keys, uint32_t n, int32_t base,
                                                           uint64_t range, const uint32_t* __restrict__ cnt,
                                                           unsigned long long* __restrict__ total) {
    __shared__ uint64_t s_w[MQ_WAVES];
    uint64_t acc = 0;
    for (uint32_t i = blockIdx.x * MQ_BLOCK + threadIdx.x; i < n; i += gridDim.x * MQ_BLOCK) {
        const uint32_t k = (uint32_t)keys[i] - (uint32_t)base;
        if (k < range) acc += cnt[k];
    }
    acc = wave_sum(acc);
    if (lane() == 0) s_w[threadIdx.x / MQ_WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < MQ_WAVES; w++) t += s_w[w];
        if (t) atomicAdd(total, (unsigned long long)t);
    }
}

hipError_t launch_key_count(const int32_t* keys, uint32_t n, int32_t base, uint64_t range, uint32_t* cnt,
                            hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((n + MQ_BLOCK * KC_IPT - 1) / (MQ_BLOCK * KC_IPT), 4096u);
    key_count_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(keys, n, base, range, cnt);
    return hipGetLastError();
}

hipError_t launch_key_dot(const int32_t* keys, uint32_t n, int32_t base, uint64_t range, const uint32_t* cnt,
                          uint64_t* total, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((n + MQ_BLOCK * 8 - 1) / (MQ_BLOCK * 8), 4096u);
    key_dot_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(keys, n, base, range, cnt,
                                                    reinterpret_cast<unsigned long long*>(total));
    return hipGetLastError();
}

}  // namespace mq
