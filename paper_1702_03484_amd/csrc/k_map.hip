// Map of Algorithm 1 on gfx950: scan a range of the store (or any SoA
// table), keep the rows that pass the pattern's equality tests, and emit
// the variable columns.  Single pass: each wave takes one __ballot per row
// slot, the block scans the wave totals, and the tile's output offset comes
// from a decoupled look-back, so kept rows stay in input order.
// The same kernel filters join results on further shared variables.
#include "device_common.h"
#include "kernels.h"

#include <algorithm>

namespace mq {

constexpr int CMP_IPT = 16;

__global__ __launch_bounds__(MQ_BLOCK) void compact_kernel(CompactArgs a, uint64_t* __restrict__ status,
                                                           uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint64_t TILE = MQ_BLOCK * CMP_IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wtot[MQ_WAVES];
    __shared__ uint64_t s_excl;
    const uint64_t ntiles = (a.n + TILE - 1) / TILE;
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    for (;;) {
        const uint32_t tile = next_tile(tile_ctr, &s_tile);
        if (tile >= ntiles) break;
        const uint64_t base = (uint64_t)tile * TILE;
        uint64_t km[CMP_IPT];
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < CMP_IPT; i++) {
            uint64_t idx = base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane());
            bool ok = idx < a.n;
            if (ok) {
                for (int t = 0; t < a.nterm; t++) {
                    int32_t va = a.in[a.term_a[t]][idx];
                    int32_t vb = a.term_b[t] >= 0 ? a.in[a.term_b[t]][idx] : a.term_c[t];
                    ok = ok && va == vb;
                }
            }
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
                if (tile == ntiles - 1) *a.count = ex + ttot;
            }
        }
        __syncthreads();
        uint64_t pos = s_excl + wex;
#pragma unroll
        for (int i = 0; i < CMP_IPT; i++) {
            if ((km[i] >> lane()) & 1ull) {
                uint64_t idx = base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane());
                uint64_t at = pos + (uint64_t)__popcll(km[i] & lt);
                for (int c = 0; c < a.nout; c++) a.out[c][at] = a.in[a.out_src[c]][idx];
            }
            pos += (uint64_t)__popcll(km[i]);
        }
    }
}

hipError_t launch_compact(const CompactArgs& a, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch,
                          hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    uint64_t tiles = (a.n + MQ_BLOCK * CMP_IPT - 1) / (MQ_BLOCK * CMP_IPT);
    uint32_t blocks = (uint32_t)std::min<uint64_t>(tiles, 256ull * 8);
    compact_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(a, status, tile_ctr, epoch);
    return hipGetLastError();
}

// First index in [lo, hi) whose value is >= v (upper = false) or > v
// (upper = true), by a 64-ary search: one coalesced probe of 64 positions and
// one __ballot per level.  Every lane of the wave calls it with the same
// arguments.
__device__ __forceinline__ int64_t wave_bound(const int32_t* __restrict__ c, int64_t lo, int64_t hi, int32_t v,
                                              bool upper) {
    while (lo < hi) {
        const int64_t step = (hi - lo + MQ_WAVE - 1) / MQ_WAVE;
        const int64_t pos = lo + (int64_t)lane() * step;
        bool below = false;
        if (pos < hi) {
            const int32_t x = c[pos];
            below = upper ? x <= v : x < v;
        }
        const uint32_t cnt = (uint32_t)__popcll(__ballot(below));  // probes before the bound (a prefix)
        if (cnt == 0) return lo;
        const int64_t nlo = lo + (int64_t)(cnt - 1) * step + 1;
        hi = std::min(hi, lo + (int64_t)cnt * step);
        lo = nlo;
    }
    return lo;
}

// one wave per query
__global__ __launch_bounds__(MQ_WAVE) void locate_kernel(const LocateQuery* __restrict__ q, int32_t nq,
                                                         int64_t* __restrict__ out) {
    const int i = blockIdx.x;
    if (i >= nq) return;
    const LocateQuery x = q[i];
    int64_t lo = x.lo, hi = x.hi;
    if (x.col1) {
        const int64_t l = wave_bound(x.col1, lo, hi, x.v1, false);
        hi = wave_bound(x.col1, l, hi, x.v1, true);
        lo = l;
    }
    if (x.col2) {
        const int64_t l = wave_bound(x.col2, lo, hi, x.v2, false);
        hi = wave_bound(x.col2, l, hi, x.v2, true);
        lo = l;
    }
    if (lane() == 0) {
        out[2 * i] = lo;
        out[2 * i + 1] = hi;
    }
}

hipError_t launch_locate(const LocateQuery* q_dev, int32_t nq, int64_t* out, hipStream_t stream) {
    if (nq <= 0) return hipSuccess;
    locate_kernel<<<nq, MQ_WAVE, 0, stream>>>(q_dev, nq, out);
    return hipGetLastError();
}

}  // namespace mq
