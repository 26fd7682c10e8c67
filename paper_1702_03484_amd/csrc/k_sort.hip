// The Shuffle step of Algorithm 1 (both sides' records grouped by key):
// stable LSD radix sort of (u32 key, u32 payload) pairs for gfx950.
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
// generates the payload as the record's position in that concatenation, or
// reads it from the record's one value column (the side then rides in the
// key's low bit), so the intermediate records are never written out before
// the first scatter.
#include "device_common.h"
#include "kernels.h"
#include "tile_ops.h"

#include <algorithm>

namespace mq {

// Cell idx of the concatenation c0 (n0 cells) ++ c1.  Callers clamp idx
// into range and load unconditionally, then transform: a load (or its use)
// inside a divergent branch makes every load wait for the one before.
__device__ __forceinline__ int32_t src_load(const int32_t* c0, const int32_t* c1, uint32_t n0, uint32_t idx) {
    const bool right = idx >= n0;
    return (right ? c1 : c0)[right ? idx - n0 : idx];
}

__device__ __forceinline__ uint32_t src_key_of(const SortSrc& s, int32_t raw, uint32_t idx) {
    const uint32_t rel = (uint32_t)raw - (uint32_t)s.base;
    return s.carry ? rel << 1 | (idx >= s.n0 ? 1u : 0u) : rel;
}

// Digit histograms of every pass in two launches: each block counts its
// keys into LDS (all loads of a tile in flight at once, one atomic per run
// of equal digits) and stores its counts to its own row of a partial table;
// a second kernel sums the rows.
// No device-wide atomics: they serialise on the few hundred counters.
constexpr int HIST_IPT = 16;
constexpr uint32_t HIST_BLOCKS = 512;

template <int RB, bool GEN>
__global__ __launch_bounds__(MQ_BLOCK) void radix_hist_kernel(SortSrc src, const uint32_t* __restrict__ keys,
                                                              uint32_t n, int passes, uint32_t* __restrict__ part) {
    using R = Radix<RB>;
    __shared__ uint32_t sh[R::MAXP * R::BUCKETS];
    for (int i = threadIdx.x; i < R::MAXP * R::BUCKETS; i += MQ_BLOCK) sh[i] = 0;
    __syncthreads();
    constexpr uint32_t TILE = MQ_BLOCK * HIST_IPT;
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // each thread takes HIST_IPT consecutive keys: runs of one digit
        // (index-ordered keys have long ones) cost one LDS atomic per run
        // instead of one per key
        const uint32_t first = t * TILE + threadIdx.x * HIST_IPT;
        uint32_t k[HIST_IPT];
#pragma unroll
        for (int i = 0; i < HIST_IPT; i++) {
            const uint32_t idx = first + i;
            if (GEN)
                k[i] = (uint32_t)src_load(src.k0, src.k1, src.n0, min(idx, n - 1));
            else
                k[i] = idx < n ? keys[idx] : 0u;
        }
        if (GEN) {
#pragma unroll
            for (int i = 0; i < HIST_IPT; i++) k[i] = src_key_of(src, (int32_t)k[i], first + i);
        }
        const int cnt = first >= n ? 0 : (int)min((uint32_t)HIST_IPT, n - first);
        for (int p = 0; p < passes; p++) {
            const int sh_p = p * RB;
            uint32_t cur = (k[0] >> sh_p) & R::MASK, run = 0;
#pragma unroll
            for (int i = 0; i < HIST_IPT; i++) {
                if (i < cnt) {
                    const uint32_t d = (k[i] >> sh_p) & R::MASK;
                    if (d != cur) {
                        atomicAdd(&sh[p * R::BUCKETS + cur], run);
                        cur = d;
                        run = 0;
                    }
                    run++;
                }
            }
            if (run) atomicAdd(&sh[p * R::BUCKETS + cur], run);
        }
    }
    __syncthreads();
    uint32_t* row = part + (uint64_t)blockIdx.x * passes * R::BUCKETS;
    for (int i = threadIdx.x; i < passes * R::BUCKETS; i += MQ_BLOCK) row[i] = sh[i];
}

// hist[c] = sum over the partial rows.  A block of 16 waves owns 64
// counters: lane L of wave w adds rows w, w + 16, ... of counter c0 + L
// (coalesced 256-byte row slices, four loads in flight per lane), and the
// 16 partial sums meet in LDS.
constexpr int HRED_WAVES = 16;

__global__ __launch_bounds__(HRED_WAVES * MQ_WAVE) void hist_reduce_kernel(const uint32_t* __restrict__ part,
                                                                           uint32_t rows, uint32_t width,
                                                                           uint32_t* __restrict__ hist) {
    __shared__ uint32_t sh[HRED_WAVES][MQ_WAVE];
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint32_t c = blockIdx.x * MQ_WAVE + lane();
    uint32_t s = 0;
    if (c < width) {
        uint32_t r = w;
        for (; r + 3 * HRED_WAVES < rows; r += 4 * HRED_WAVES) {
            const uint32_t a0 = part[(uint64_t)r * width + c];
            const uint32_t a1 = part[(uint64_t)(r + HRED_WAVES) * width + c];
            const uint32_t a2 = part[(uint64_t)(r + 2 * HRED_WAVES) * width + c];
            const uint32_t a3 = part[(uint64_t)(r + 3 * HRED_WAVES) * width + c];
            s += (a0 + a1) + (a2 + a3);
        }
        for (; r < rows; r += HRED_WAVES) s += part[(uint64_t)r * width + c];
    }
    sh[w][lane()] = s;
    __syncthreads();
    if (w == 0 && c < width) {
        uint32_t t = 0;
#pragma unroll
        for (int k = 0; k < HRED_WAVES; k++) t += sh[k][lane()];
        hist[c] = t;
    }
}

uint32_t radix_hist_part_words(int rb, int passes) { return HIST_BLOCKS * (uint32_t)passes << rb; }

// Waves per block of a radix pass for digits of up to 8 bits at 16 keys per
// thread: 16 for a carried pass (16,384-record tiles in 140 KB of LDS, one
// block and 4 waves per SIMD on a CU) and 8 for the first pass (8,192-record
// tiles, two blocks per CU at its 128-VGPR bound), else 4.  Fewer, larger
// tiles mean fewer tile-id atomics and look-backs: on a 16M + 16M-record
// sort 4- and 8-wave blocks took 0.79 ms, 8 and 8 0.76 ms, 8 and 16 0.75 ms.
__host__ __device__ constexpr int sort_waves(int rb, int kpt, bool gen) {
    return rb <= 8 && kpt == 16 ? (gen ? 8 : 16) : 4;
}

// the first pass is held to 128 VGPRs (4 waves per SIMD instead of 3, no spills)
template <int RB, int KPT, bool GEN, int NW = sort_waves(RB, KPT, GEN)>
__global__ __launch_bounds__(NW * MQ_WAVE, GEN ? 4 : 1) void radix_pass_kernel(SortSrc src, const uint32_t* __restrict__ kin,
                                                                  const uint32_t* __restrict__ vin,
                                                                  uint32_t* __restrict__ kout,
                                                                  uint32_t* __restrict__ vout, uint32_t n, int shift,
                                                                  const uint32_t* __restrict__ ghist,
                                                                  uint64_t* __restrict__ status,
                                                                  uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr int TILE = NW * MQ_WAVE * KPT;
    __shared__ SortSmem<RB, KPT, NW> sm;
    __shared__ uint32_t s_tile;
    const uint32_t tile = next_tile(tile_ctr, &s_tile);
    const uint32_t base = tile * (uint32_t)TILE;
    const uint32_t valid_n = min((uint32_t)TILE, n - base);
    const uint32_t w = threadIdx.x / MQ_WAVE;
    // wave-striped slice: element i of this lane is base + (w*KPT + i)*64 + lane
    uint32_t key[KPT], val[KPT];
    if (GEN) {
        // every load first (clamped into range), then the keys and payloads
        int32_t rk[KPT], rv[KPT];
        if (base + (uint32_t)TILE <= src.n0 || base >= src.n0) {
            // the whole tile on one side: loads from a uniform base
            const bool right = base >= src.n0;
            const uint32_t b0 = right ? base - src.n0 : base;
            const int32_t* kt = (right ? src.k1 : src.k0) + b0;
            const int32_t* vt = (right ? src.v1 : src.v0) + b0;
#pragma unroll
            for (int i = 0; i < KPT; i++) {
                const uint32_t off = min((w * KPT + i) * MQ_WAVE + lane(), valid_n - 1);
                rk[i] = kt[off];
                rv[i] = src.carry ? vt[off] : 0;
            }
        } else {
#pragma unroll
            for (int i = 0; i < KPT; i++) {
                const uint32_t idx = min(base + (w * KPT + i) * MQ_WAVE + lane(), n - 1);
                rk[i] = src_load(src.k0, src.k1, src.n0, idx);
                rv[i] = src.carry ? src_load(src.v0, src.v1, src.n0, idx) : 0;
            }
        }
#pragma unroll
        for (int i = 0; i < KPT; i++) {
            const uint32_t off = (w * KPT + i) * MQ_WAVE + lane();
            const uint32_t idx = base + off;
            const bool ok = off < valid_n;
            key[i] = ok ? src_key_of(src, rk[i], idx) : 0u;
            val[i] = ok ? (src.carry ? (uint32_t)rv[i] : idx) : 0u;
        }
    } else {
        // from the tile's (uniform) base with 32-bit offsets: scalar-base loads
        const uint32_t* kt = kin + base;
        const uint32_t* vt = vin + base;
#pragma unroll
        for (int i = 0; i < KPT; i++) {
            const uint32_t off = (w * KPT + i) * MQ_WAVE + lane();
            const bool ok = off < valid_n;
            key[i] = ok ? kt[off] : 0u;
            val[i] = ok ? vt[off] : 0u;
        }
    }
    sort_tile<RB, KPT, NW>(sm, key, val, valid_n, shift, ghist, status, tile, 0, epoch, kout, vout, n);
}

#define MQ_RB_LIST(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11)

hipError_t launch_radix_hist(const SortSrc& src, const uint32_t* keys, uint32_t n, int rb, int passes,
                             uint32_t* part, uint32_t* hist, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min((n + MQ_BLOCK * HIST_IPT - 1) / (MQ_BLOCK * HIST_IPT), HIST_BLOCKS);
    bool gen = keys == nullptr;
#define MQ_H(B)                                                                                         \
    case B:                                                                                             \
        if (gen)                                                                                        \
            radix_hist_kernel<B, true><<<blocks, MQ_BLOCK, 0, stream>>>(src, keys, n, passes, part);    \
        else                                                                                            \
            radix_hist_kernel<B, false><<<blocks, MQ_BLOCK, 0, stream>>>(src, keys, n, passes, part);   \
        break;
    switch (rb) {
        MQ_RB_LIST(MQ_H)
        default: return hipErrorInvalidValue;
    }
#undef MQ_H
    const uint32_t width = (uint32_t)passes << rb;
    hist_reduce_kernel<<<(width + MQ_WAVE - 1) / MQ_WAVE, HRED_WAVES * MQ_WAVE, 0, stream>>>(part, blocks, width, hist);
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
        const uint32_t tiles = radix_tiles(n, K, B, gen);                                                   \
        if (gen)                                                                                            \
            radix_pass_kernel<B, K, true><<<tiles, sort_waves(B, K, true) * MQ_WAVE, 0, stream>>>(          \
                src, kin, vin, kout, vout, n, shift, hist_pass, status, tile_ctr, epoch);                   \
        else                                                                                                \
            radix_pass_kernel<B, K, false><<<tiles, sort_waves(B, K, false) * MQ_WAVE, 0, stream>>>(        \
                src, kin, vin, kout, vout, n, shift, hist_pass, status, tile_ctr, epoch);                   \
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

uint32_t radix_tiles(uint32_t n, int kpt, int rb, bool gen) {
    const uint32_t tile = (uint32_t)(sort_waves(rb, kpt, gen) * MQ_WAVE * kpt);
    return (n + tile - 1) / tile;
}

}  // namespace mq
