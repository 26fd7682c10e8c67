// Reduce without a shuffle for two tables already in key order (a view of
// the PSO or POS index whose next sort column is the key, or the result of
// a join on the same key).  The stable sort of the two sides' records would
// be their merge, LEFT before RIGHT within a key, so the segments of
// Algorithm 1's ReduceDuplicate are the two sides' runs of each key: one
// pass over the smaller side finds, at the head of each run, the run's end
// (galloping) and the key's run in the larger side (binary search).  Keys on
// both sides become segments in ascending key order, with cL * cR output
// rows each; their count and offsets come from two decoupled look-backs.
// Materialisation then reads both tables' columns in place.
#include "device_common.h"
#include "kernels.h"

#include <algorithm>

namespace mq {

constexpr int MRG_IPT = 4;

// first index in [lo, hi) with a[i] >= v (a ascending)
__device__ __forceinline__ uint32_t lower_bound_i32(const int32_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                                    int32_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first index in [lo, hi) with a[i] > v (a ascending)
__device__ __forceinline__ uint32_t upper_bound_i32(const int32_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                                    int32_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// end of the run of v that starts at i (a[i] == v, a ascending, n < 2^31):
// gallop, then binary search; short runs cost a load or two
__device__ __forceinline__ uint32_t run_end(const int32_t* __restrict__ a, uint32_t i, uint32_t n, int32_t v) {
    uint32_t lo = i + 1, step = 1;  // a[lo - 1] == v
    for (;;) {
        const uint32_t probe = (uint32_t)min((uint64_t)n, (uint64_t)i + step);
        if (probe == n || a[probe] != v) return upper_bound_i32(a, lo, probe, v);
        lo = probe + 1;
        step <<= 1;
    }
}

__global__ __launch_bounds__(MQ_BLOCK) void merge_segments_kernel(MergeArgs a, uint64_t* __restrict__ status,
                                                                  uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint32_t TILE = MQ_BLOCK * MRG_IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wseg[MQ_WAVES];
    __shared__ uint64_t s_wrow[MQ_WAVES];
    __shared__ uint64_t s_ex[2];
    const uint32_t ntiles = (a.ns + TILE - 1) / TILE;
    uint64_t* st_seg = status;           // segment counts
    uint64_t* st_row = status + ntiles;  // output rows
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    for (;;) {
        const uint32_t tile = next_tile(tile_ctr, &s_tile);
        if (tile >= ntiles) break;
        const uint32_t base = tile * TILE;
        uint32_t bl[MRG_IPT], bc[MRG_IPT], sc[MRG_IPT];
        uint64_t km[MRG_IPT];
        uint64_t rows[MRG_IPT];
        uint32_t wseg = 0;
        uint64_t wrow = 0;
#pragma unroll
        for (int k = 0; k < MRG_IPT; k++) {
            const uint32_t idx = base + (w * MRG_IPT + k) * MQ_WAVE + lane();
            bool keep = false;
            bl[k] = bc[k] = sc[k] = 0;
            if (idx < a.ns) {
                const int32_t key = a.skey[idx];
                if (idx == 0 || a.skey[idx - 1] != key) {
                    const uint32_t lb = lower_bound_i32(a.bkey, 0, a.nb, key);
                    if (lb < a.nb && a.bkey[lb] == key) {
                        bl[k] = lb;
                        bc[k] = upper_bound_i32(a.bkey, lb + 1, a.nb, key) - lb;
                        sc[k] = run_end(a.skey, idx, a.ns, key) - idx;
                        keep = true;
                    }
                }
            }
            km[k] = __ballot(keep);
            rows[k] = keep ? (uint64_t)sc[k] * bc[k] : 0ull;
            wseg += (uint32_t)__popcll(km[k]);
            wrow += wave_sum(rows[k]);
        }
        if (lane() == 0) {
            s_wseg[w] = wseg;
            s_wrow[w] = wrow;
        }
        __syncthreads();
        uint32_t seg_before = 0, seg_tot = 0;
        uint64_t row_before = 0, row_tot = 0;
#pragma unroll
        for (int i = 0; i < MQ_WAVES; i++) {
            if ((uint32_t)i < w) {
                seg_before += s_wseg[i];
                row_before += s_wrow[i];
            }
            seg_tot += s_wseg[i];
            row_tot += s_wrow[i];
        }
        if (w == 0) {
            const uint64_t es = tile_prefix_wave0(st_seg, tile, epoch, seg_tot);
            const uint64_t er = tile_prefix_wave0(st_row, tile, epoch, row_tot);
            if (lane() == 0) {
                s_ex[0] = es;
                s_ex[1] = er;
                if (tile == ntiles - 1) {
                    *a.nseg = (uint32_t)(es + seg_tot);
                    *a.total = sat_add(er, row_tot > SAT40 ? SAT40 : row_tot);
                }
            }
        }
        __syncthreads();
        uint32_t sp = (uint32_t)s_ex[0] + seg_before;
        uint64_t rp = sat_add(s_ex[1], row_before);
#pragma unroll
        for (int k = 0; k < MRG_IPT; k++) {
            const uint64_t rincl = wave_incl_scan(rows[k]);
            if ((km[k] >> lane()) & 1ull) {
                const uint32_t idx = base + (w * MRG_IPT + k) * MQ_WAVE + lane();
                const uint32_t at = sp + (uint32_t)__popcll(km[k] & lt);
                const uint32_t ls = a.small_is_left ? idx : bl[k], lc = a.small_is_left ? sc[k] : bc[k];
                const uint32_t rs = a.small_is_left ? bl[k] : idx, rc = a.small_is_left ? bc[k] : sc[k];
                a.seg_lstart[at] = ls;
                a.seg_lcount[at] = lc;
                a.seg_rstart[at] = rs;
                a.seg_rcount[at] = rc;
                a.seg_off[at] = sat_add(rp, rincl - rows[k]);
            }
            sp += (uint32_t)__popcll(km[k]);
            rp = sat_add(rp, __shfl(rincl, MQ_WAVE - 1, MQ_WAVE));
        }
    }
}

uint32_t merge_tiles(uint32_t ns) { return (ns + MQ_BLOCK * MRG_IPT - 1) / (MQ_BLOCK * MRG_IPT); }

hipError_t launch_merge_segments(const MergeArgs& a, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch,
                                 hipStream_t stream) {
    if (a.ns == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>(merge_tiles(a.ns), 256u * 8u);
    merge_segments_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(a, status, tile_ctr, epoch);
    return hipGetLastError();
}

}  // namespace mq
