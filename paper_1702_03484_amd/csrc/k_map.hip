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
        if (threadIdx.x == 0) {
            uint64_t ex = 0;
            if (tile == 0) {
                st_store(status, st_pack(epoch, ST_INC, ttot));
            } else {
                st_store(status + tile, st_pack(epoch, ST_AGG, ttot));
                ex = lookback(status, tile, 0, 1, epoch);
                st_store(status + tile, st_pack(epoch, ST_INC, ex + ttot));
            }
            s_excl = ex;
            if (tile == ntiles - 1) *a.count = ex + ttot;
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

__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* c, int64_t lo, int64_t hi, int32_t v) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (c[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int64_t upper_bound_i32(const int32_t* c, int64_t lo, int64_t hi, int32_t v) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (c[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void locate_kernel(const LocateQuery* __restrict__ q, int32_t nq, int64_t* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    LocateQuery x = q[i];
    int64_t lo = x.lo, hi = x.hi;
    if (x.col1) {
        int64_t l = lower_bound_i32(x.col1, lo, hi, x.v1);
        hi = upper_bound_i32(x.col1, l, hi, x.v1);
        lo = l;
    }
    if (x.col2) {
        int64_t l = lower_bound_i32(x.col2, lo, hi, x.v2);
        hi = upper_bound_i32(x.col2, l, hi, x.v2);
        lo = l;
    }
    out[2 * i] = lo;
    out[2 * i + 1] = hi;
}

hipError_t launch_locate(const LocateQuery* q_dev, int32_t nq, int64_t* out, hipStream_t stream) {
    if (nq <= 0) return hipSuccess;
    locate_kernel<<<(nq + 63) / 64, 64, 0, stream>>>(q_dev, nq, out);
    return hipGetLastError();
}

}  // namespace mq
