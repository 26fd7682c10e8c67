// Device helpers shared by the gfx950 kernels: wave64 scans, block scans and
// the status words of single-pass decoupled look-back.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MQ_WAVE 64
#define MQ_BLOCK 256
#define MQ_WAVES (MQ_BLOCK / MQ_WAVE)

namespace mq {

// Bounds-checked build (-DMQ_DEBUG; `python -m paper_1702_03484_amd.build
// --debug` writes libmapsq_debug.so, loaded when MAPSQ_LIB=debug): every
// data-dependent store index of the sort, segment, materialisation and
// compaction kernels is checked against the extent of what it writes; an
// index outside it is printed with its file and line and the store is
// skipped, so a wrong index shows up as a message instead of a memory fault.
// In the normal build the check is the constant true and costs nothing.
#ifdef MQ_DEBUG
__device__ __noinline__ inline bool dbg_in_bounds(uint64_t i, uint64_t n, const char* file, int line) {
    if (i < n) return true;
    printf("mapsq bounds check: %s:%d index %llu outside [0, %llu)\n", file, line, (unsigned long long)i,
           (unsigned long long)n);
    return false;
}
#define MQ_IN_BOUNDS(i, n) ::mq::dbg_in_bounds((uint64_t)(i), (uint64_t)(n), __FILE__, __LINE__)
#else
#define MQ_IN_BOUNDS(i, n) true
#endif

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
    for (int o = 1; o < MQ_WAVE; o <<= 1) {
        T t = __shfl_up(v, o, MQ_WAVE);
        if ((int)lane() >= o) v += t;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = MQ_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, MQ_WAVE);
    return v;
}

// Exclusive scan over the block (MQ_BLOCK threads).  `tmp` is MQ_WAVES
// entries of LDS.  Returns the exclusive prefix; *total gets the block sum.
// Contains __syncthreads(); every thread of the block must call it.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* tmp, T* total) {
    T inc = wave_incl_scan(v);
    const uint32_t w = threadIdx.x / MQ_WAVE;
    if (lane() == MQ_WAVE - 1) tmp[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < MQ_WAVES; i++) {
        T x = tmp[i];
        if ((uint32_t)i < w) before += x;
        all += x;
    }
    *total = all;
    __syncthreads();
    return before + inc - v;
}

// ---- decoupled look-back status words ------------------------------------
// 64-bit word: [63:42] epoch (22 bits), [41:40] flag, [39:0] value.  A word
// whose epoch differs from the running pass's epoch counts as "not yet
// published", so the status array is never cleared between passes.
constexpr uint32_t ST_AGG = 1;  // the tile's own aggregate
constexpr uint32_t ST_INC = 2;  // inclusive prefix up to and including the tile
constexpr uint64_t ST_VAL_MASK = (1ull << 40) - 1ull;
constexpr uint64_t SAT40 = ST_VAL_MASK;  // saturation cap of 40-bit sums

__device__ __forceinline__ uint64_t st_pack(uint32_t epoch, uint32_t flag, uint64_t v) {
    return ((uint64_t)epoch << 42) | ((uint64_t)flag << 40) | (v & ST_VAL_MASK);
}
__device__ __forceinline__ void st_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t st_load(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s > SAT40 ? SAT40 : s;
}

// Exclusive prefix of tile `tile` over tiles [first_tile, tile) for one
// status column; `stride` is the distance between consecutive tiles' words.
// Reads up to 4 predecessors per round so their load latencies overlap;
// spins until predecessors publish.  Sums saturate at 2^40 - 1.  (Windows of
// 8 and 16 were slower on a 16M + 16M-record sort, 0.81 and 1.13 against
// 0.79 ms: every poll is a device-scope load, and wider polls add traffic
// the spinning waves compete for.)
__device__ __forceinline__ uint64_t lookback(const uint64_t* status, uint32_t tile, uint32_t first_tile,
                                             uint32_t stride, uint32_t epoch) {
    constexpr int WIN = 4;
    uint64_t excl = 0;
    int64_t t = (int64_t)tile - 1;
    while (t >= (int64_t)first_tile) {
        uint64_t w[WIN];
#pragma unroll
        for (int k = 0; k < WIN; k++)
            w[k] = (t - k >= (int64_t)first_tile) ? st_load(status + (uint64_t)(t - k) * stride) : 0ull;
        int k = 0;
        bool done = false;
        for (; k < WIN && t - k >= (int64_t)first_tile; k++) {
            const uint32_t flag = (uint32_t)(w[k] >> 40) & 3u;
            if ((uint32_t)(w[k] >> 42) != epoch || flag == 0) break;  // not yet published: retry from here
            excl = sat_add(excl, w[k] & ST_VAL_MASK);
            if (flag == ST_INC) {
                done = true;
                break;
            }
        }
        if (done) break;
        if (k == 0) __builtin_amdgcn_s_sleep(1);
        t -= k;
    }
    return excl;
}

// Wave-parallel look-back over one status column (stride 1): each probe
// reads the LB_PER_LANE * 64 predecessors below `top` at once (lane L the
// LB_PER_LANE nearest after those of lanes < L) and stops at the nearest
// inclusive prefix.  One word per lane was the fastest window on the
// 512-join batched launch (67.9 ms, against 69.4 with 2 words per lane,
// 71.0 with 4 and 72.8 with 8): a wider probe shortens the walk over
// aggregates but every word is a device-scope load.  Every lane of the
// calling wave must call it; all lanes return the exclusive prefix of `tile`
// (saturating at 2^40 - 1).
constexpr int LB_PER_LANE = 1;

__device__ __forceinline__ uint64_t wave_lookback(const uint64_t* status, uint32_t tile, uint32_t first_tile,
                                                  uint32_t epoch) {
    constexpr int64_t WIN = (int64_t)LB_PER_LANE * MQ_WAVE;
    uint64_t excl = 0;
    int64_t top = (int64_t)tile - 1;
    while (top >= (int64_t)first_tile) {
        uint64_t w[LB_PER_LANE];
        bool inr[LB_PER_LANE];
#pragma unroll
        for (int j = 0; j < LB_PER_LANE; j++) {
            const int64_t t = top - (int64_t)lane() * LB_PER_LANE - j;
            inr[j] = t >= (int64_t)first_tile;
            w[j] = inr[j] ? st_load(status + t) : 0ull;
        }
        // this lane: the first of its words that is an inclusive prefix (or
        // out of range), and whether any word before it is unpublished
        int jinc = LB_PER_LANE;
        bool pending = false;
#pragma unroll
        for (int j = LB_PER_LANE - 1; j >= 0; j--) {
            const uint32_t flag = (uint32_t)(w[j] >> 40) & 3u;
            const bool valid = !inr[j] || ((uint32_t)(w[j] >> 42) == epoch && flag != 0);
            const bool inc = !inr[j] || (valid && flag == ST_INC);
            if (inc) jinc = j;
        }
#pragma unroll
        for (int j = 0; j < LB_PER_LANE; j++) {
            const uint32_t flag = (uint32_t)(w[j] >> 40) & 3u;
            const bool valid = !inr[j] || ((uint32_t)(w[j] >> 42) == epoch && flag != 0);
            if (j <= jinc && !valid) pending = true;
        }
        const uint64_t incm = __ballot(jinc < LB_PER_LANE);
        const uint32_t stop = incm ? (uint32_t)__builtin_ctzll(incm) : 64u;  // lanes 0..stop count
        const uint64_t need = stop >= 63 ? ~0ull : ((2ull << stop) - 1ull);
        if (__ballot(pending) & need) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t v = 0;
        if (lane() <= stop) {
#pragma unroll
            for (int j = 0; j < LB_PER_LANE; j++)
                if (inr[j] && (lane() < stop || j <= jinc)) v += w[j] & ST_VAL_MASK;
        }
        v = wave_sum(v);  // at most 256 * 2^40: no overflow
        excl = sat_add(excl, v > SAT40 ? SAT40 : v);
        if (stop < 64) break;
        top -= WIN;
    }
    return excl;
}

// Publish a tile aggregate and resolve its exclusive prefix over tiles
// [first_tile, tile) with one wave (all 64 lanes of that wave call it).
// Returns the exclusive prefix in every lane of the wave.
__device__ __forceinline__ uint64_t tile_prefix_wave(uint64_t* status, uint32_t tile, uint32_t first_tile,
                                                     uint32_t epoch, uint64_t agg) {
    agg = agg > SAT40 ? SAT40 : agg;
    if (tile == first_tile) {
        if (lane() == 0) st_store(status + tile, st_pack(epoch, ST_INC, agg));
        return 0;
    }
    if (lane() == 0) st_store(status + tile, st_pack(epoch, ST_AGG, agg));
    const uint64_t ex = wave_lookback(status, tile, first_tile, epoch);
    if (lane() == 0) st_store(status + tile, st_pack(epoch, ST_INC, sat_add(ex, agg)));
    return ex;
}

__device__ __forceinline__ uint64_t tile_prefix_wave0(uint64_t* status, uint32_t tile, uint32_t epoch, uint64_t agg) {
    return tile_prefix_wave(status, tile, 0, epoch, agg);
}

// Next dynamic tile id from a counter (thread 0), broadcast through LDS.
__device__ __forceinline__ uint32_t next_tile(uint32_t* counter, uint32_t* s_slot) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(counter, 1u);
    __syncthreads();
    uint32_t t = *s_slot;
    __syncthreads();
    return t;
}

}  // namespace mq
