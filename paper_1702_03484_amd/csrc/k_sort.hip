// Shuffle of Algorithm 1 ("sort intermediates"): stable LSD radix sort of
// (u32 key, u32 payload) pairs for gfx950.
//
// One histogram launch counts the digits of every pass at once; each pass is
// then one launch that ranks a tile in LDS and scatters it to its final
// place, the tile's global offsets coming from a decoupled look-back over
// per-digit status words.  Ranking is stable: within a wave64 the peers of a
// digit are found with one __ballot per digit bit, waves own consecutive
// slices of the tile, and tiles take dynamic ids in input order.
//
// First-pass ("gen") mode reads the keys of two input segments (the LEFT
// then the RIGHT partial-match table of a join), subtracts a base and
// generates the payload as the record's position in that concatenation, so
// the intermediate records are never written out before the first scatter.
#include "device_common.h"
#include "kernels.h"

#include <algorithm>

namespace mq {

template <int RB>
struct Radix {
    static constexpr int BUCKETS = 1 << RB;
    static constexpr uint32_t MASK = BUCKETS - 1;
    static constexpr int MAXP = (32 + RB - 1) / RB;
    static constexpr int BPT = (BUCKETS + MQ_BLOCK - 1) / MQ_BLOCK;  // buckets per thread
};

__device__ __forceinline__ uint32_t src_key(const SortSrc& s, uint32_t idx) {
    int32_t k = idx < s.n0 ? s.k0[idx] : s.k1[idx - s.n0];
    return (uint32_t)k - (uint32_t)s.base;
}

template <int RB, bool GEN>
__global__ __launch_bounds__(MQ_BLOCK) void radix_hist_kernel(SortSrc src, const uint32_t* __restrict__ keys,
                                                              uint32_t n, int passes, uint32_t* __restrict__ hist) {
    using R = Radix<RB>;
    __shared__ uint32_t sh[R::MAXP * R::BUCKETS];
    for (int i = threadIdx.x; i < R::MAXP * R::BUCKETS; i += MQ_BLOCK) sh[i] = 0;
    __syncthreads();
    const uint32_t stride = gridDim.x * MQ_BLOCK;
    for (uint32_t i = blockIdx.x * MQ_BLOCK + threadIdx.x; i < n; i += stride) {
        uint32_t k = GEN ? src_key(src, i) : keys[i];
        for (int p = 0; p < passes; p++) atomicAdd(&sh[p * R::BUCKETS + ((k >> (p * RB)) & R::MASK)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * R::BUCKETS; i += MQ_BLOCK) {
        uint32_t c = sh[i];
        if (c) atomicAdd(&hist[i], c);
    }
}

// Exclusive scan of BUCKETS values held in LDS `in`, written to LDS `out`
// (may alias).  Thread t owns the BPT consecutive buckets t*BPT...
template <int RB>
__device__ __forceinline__ void scan_buckets(const uint32_t* in, uint32_t* out, uint32_t* tmp) {
    using R = Radix<RB>;
    uint32_t loc[R::BPT];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < R::BPT; k++) {
        uint32_t d = threadIdx.x * R::BPT + k;
        loc[k] = d < (uint32_t)R::BUCKETS ? in[d] : 0u;
        sum += loc[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(sum, tmp, &tot);
#pragma unroll
    for (int k = 0; k < R::BPT; k++) {
        uint32_t d = threadIdx.x * R::BPT + k;
        if (d < (uint32_t)R::BUCKETS) out[d] = ex;
        ex += loc[k];
    }
    __syncthreads();
}

template <int RB, int KPT, bool GEN>
__global__ __launch_bounds__(MQ_BLOCK) void radix_pass_kernel(SortSrc src, const uint32_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin,
                                                              uint32_t* __restrict__ kout,
                                                              uint32_t* __restrict__ vout, uint32_t n, int shift,
                                                              const uint32_t* __restrict__ ghist,
                                                              uint64_t* __restrict__ status,
                                                              uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    using R = Radix<RB>;
    constexpr int TILE = MQ_BLOCK * KPT;
    __shared__ uint32_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_wcnt[MQ_WAVES][R::BUCKETS];
    __shared__ uint32_t s_local[R::BUCKETS];
    __shared__ uint32_t s_goff[R::BUCKETS];
    __shared__ uint32_t s_tmp[MQ_WAVES];
    __shared__ uint32_t s_tile;

    const uint32_t tile = next_tile(tile_ctr, &s_tile);
    const uint32_t base = tile * (uint32_t)TILE;
    const uint32_t valid_n = min((uint32_t)TILE, n - base);
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint32_t ln = lane();

    // global start of every digit for this pass, and cleared wave counters
    for (int d = threadIdx.x; d < R::BUCKETS; d += MQ_BLOCK) {
        s_goff[d] = ghist[d];
#pragma unroll
        for (int i = 0; i < MQ_WAVES; i++) s_wcnt[i][d] = 0;
    }
    __syncthreads();
    scan_buckets<RB>(s_goff, s_goff, s_tmp);

    // load a wave-striped slice: element i of this lane is base + (w*KPT + i)*64 + lane
    uint32_t key[KPT], val[KPT], rank[KPT];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < KPT; i++) {
        uint32_t off = (w * KPT + i) * MQ_WAVE + ln;
        uint32_t idx = base + off;
        bool ok = off < valid_n;
        if (GEN) {
            key[i] = ok ? src_key(src, idx) : 0u;
            val[i] = idx;
        } else {
            key[i] = ok ? kin[idx] : 0u;
            val[i] = ok ? vin[idx] : 0u;
        }
    }
    // stable rank within the wave, digit by digit through the wave counters
#pragma unroll
    for (int i = 0; i < KPT; i++) {
        uint32_t off = (w * KPT + i) * MQ_WAVE + ln;
        bool ok = off < valid_n;
        uint32_t dg = (key[i] >> shift) & R::MASK;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < RB; b++) {
            uint32_t bit = (dg >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t below = __popcll(peers & lt);
        uint32_t old = ok ? s_wcnt[w][dg] : 0u;
        if (ok && below == 0) s_wcnt[w][dg] = old + (uint32_t)__popcll(peers);
        rank[i] = old + below;
    }
    __syncthreads();

    // per digit: exclusive prefix over waves, tile total, local digit starts
    uint32_t tot[R::BPT];
#pragma unroll
    for (int k = 0; k < R::BPT; k++) {
        uint32_t d = threadIdx.x * R::BPT + k;
        uint32_t run = 0;
        if (d < (uint32_t)R::BUCKETS) {
#pragma unroll
            for (int i = 0; i < MQ_WAVES; i++) {
                uint32_t c = s_wcnt[i][d];
                s_wcnt[i][d] = run;
                run += c;
            }
            s_local[d] = run;
        }
        tot[k] = run;
    }
    __syncthreads();
    scan_buckets<RB>(s_local, s_local, s_tmp);

    // publish this tile's digit totals, then look back for the prefix
    uint64_t* st = status + (uint64_t)tile * R::BUCKETS;
#pragma unroll
    for (int k = 0; k < R::BPT; k++) {
        uint32_t d = threadIdx.x * R::BPT + k;
        if (d < (uint32_t)R::BUCKETS) st_store(st + d, st_pack(epoch, tile == 0 ? ST_INC : ST_AGG, tot[k]));
    }
    if (tile > 0) {
#pragma unroll
        for (int k = 0; k < R::BPT; k++) {
            uint32_t d = threadIdx.x * R::BPT + k;
            if (d < (uint32_t)R::BUCKETS) {
                uint64_t ex = lookback(status + d, tile, 0, R::BUCKETS, epoch);
                st_store(st + d, st_pack(epoch, ST_INC, ex + tot[k]));
                s_goff[d] += (uint32_t)ex;
            }
        }
    }
    // local scatter into LDS in digit order
#pragma unroll
    for (int i = 0; i < KPT; i++) {
        uint32_t off = (w * KPT + i) * MQ_WAVE + ln;
        if (off < valid_n) {
            uint32_t dg = (key[i] >> shift) & R::MASK;
            uint32_t pos = s_local[dg] + s_wcnt[w][dg] + rank[i];
            s_keys[pos] = key[i];
            s_vals[pos] = val[i];
        }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < valid_n; j += MQ_BLOCK) {
        uint32_t k = s_keys[j];
        uint32_t dg = (k >> shift) & R::MASK;
        uint32_t g = s_goff[dg] + (j - s_local[dg]);
        kout[g] = k;
        vout[g] = s_vals[j];
    }
}

#define MQ_RB_LIST(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11)

hipError_t launch_radix_hist(const SortSrc& src, const uint32_t* keys, uint32_t n, int rb, int passes,
                             uint32_t* hist, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint32_t blocks = std::min((n + MQ_BLOCK * 16 - 1) / (MQ_BLOCK * 16), 2048u);
    bool gen = keys == nullptr;
#define MQ_H(B)                                                                                         \
    case B:                                                                                             \
        if (gen)                                                                                        \
            radix_hist_kernel<B, true><<<blocks, MQ_BLOCK, 0, stream>>>(src, keys, n, passes, hist);    \
        else                                                                                            \
            radix_hist_kernel<B, false><<<blocks, MQ_BLOCK, 0, stream>>>(src, keys, n, passes, hist);   \
        break;
    switch (rb) {
        MQ_RB_LIST(MQ_H)
        default: return hipErrorInvalidValue;
    }
#undef MQ_H
    return hipGetLastError();
}

hipError_t launch_radix_pass(int rb, int kpt, const SortSrc& src, const uint32_t* kin, const uint32_t* vin,
                             uint32_t* kout, uint32_t* vout, uint32_t n, int pass, const uint32_t* hist_pass,
                             uint64_t* status, uint32_t* tile_ctr, uint32_t epoch, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    bool gen = kin == nullptr;
    int shift = pass * rb;
#define MQ_P(B, K)                                                                                          \
    {                                                                                                       \
        uint32_t tiles = (n + MQ_BLOCK * K - 1) / (MQ_BLOCK * K);                                           \
        if (gen)                                                                                            \
            radix_pass_kernel<B, K, true><<<tiles, MQ_BLOCK, 0, stream>>>(src, kin, vin, kout, vout, n, shift, \
                                                                          hist_pass, status, tile_ctr, epoch); \
        else                                                                                                \
            radix_pass_kernel<B, K, false><<<tiles, MQ_BLOCK, 0, stream>>>(src, kin, vin, kout, vout, n, shift, \
                                                                           hist_pass, status, tile_ctr, epoch); \
    }
#define MQ_PK(B)                     \
    case B:                          \
        if (kpt == 8) MQ_P(B, 8)     \
        else MQ_P(B, 16)             \
        break;
    switch (rb) {
        MQ_RB_LIST(MQ_PK)
        default: return hipErrorInvalidValue;
    }
#undef MQ_PK
#undef MQ_P
    return hipGetLastError();
}

uint32_t radix_tiles(uint32_t n, int kpt) { return (n + MQ_BLOCK * kpt - 1) / (MQ_BLOCK * kpt); }

}  // namespace mq
