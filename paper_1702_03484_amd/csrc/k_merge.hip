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

// one smaller-side record per thread: the searches of a thread cannot
// overlap, those of different threads do
constexpr int MRG_IPT = 1;

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

// Both bounds of v in b[0, n) at once: lower (first b[i] >= v) and upper
// (first b[i] > v).  A table of MRG_SAMPLES evenly spaced keys in LDS gives
// each bound's bracket; the two global binary searches then run
// interleaved, so their loads overlap.
constexpr int MRG_SAMPLES = 2048;

__device__ __forceinline__ uint32_t sample_pos(uint32_t j, uint32_t n) {
    return (uint32_t)(((uint64_t)j * n) / MRG_SAMPLES);
}

__device__ __forceinline__ void bounds_i32(const int32_t* __restrict__ b, uint32_t n, const int32_t* samp, int32_t v,
                                           uint32_t& lower, uint32_t& upper) {
    // samples below v (jl) and at most v (ju), by binary search in LDS
    uint32_t jl = 0, jh = MRG_SAMPLES, ul = 0, uh = MRG_SAMPLES;
    while (jl < jh) {
        const uint32_t m = (jl + jh) >> 1;
        if (samp[m] < v) jl = m + 1;
        else jh = m;
    }
    while (ul < uh) {
        const uint32_t m = (ul + uh) >> 1;
        if (samp[m] <= v) ul = m + 1;
        else uh = m;
    }
    // the bound lies in (pos(j - 1), pos(j)], with pos(-1) = -1 and pos(S) = n
    uint32_t l0 = jl == 0 ? 0u : sample_pos(jl - 1, n) + 1, l1 = jl == MRG_SAMPLES ? n : sample_pos(jl, n);
    uint32_t u0 = ul == 0 ? 0u : sample_pos(ul - 1, n) + 1, u1 = ul == MRG_SAMPLES ? n : sample_pos(ul, n);
    while (l0 < l1 || u0 < u1) {
        const uint32_t lm = l0 + ((l1 - l0) >> 1), um = u0 + ((u1 - u0) >> 1);
        const bool lgo = l0 < l1, ugo = u0 < u1;
        const int32_t lv = lgo ? b[lm] : 0, uv = ugo ? b[um] : 0;
        if (lgo) {
            if (lv < v) l0 = lm + 1;
            else l1 = lm;
        }
        if (ugo) {
            if (uv <= v) u0 = um + 1;
            else u1 = um;
        }
    }
    lower = l0;
    upper = u0;
}

__global__ __launch_bounds__(MQ_BLOCK) void merge_segments_kernel(MergeArgs a, uint64_t* __restrict__ status,
                                                                  uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint32_t TILE = MQ_BLOCK * MRG_IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wseg[MQ_WAVES];
    __shared__ uint64_t s_wrow[MQ_WAVES];
    __shared__ uint64_t s_ex[2];
    __shared__ int32_t s_samp[MRG_SAMPLES];
    const uint32_t ntiles = (a.ns + TILE - 1) / TILE;
    uint64_t* st_seg = status;           // segment counts
    uint64_t* st_row = status + ntiles;  // output rows
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    // nb >= 1: the caller returns early on an empty side
    for (uint32_t j = threadIdx.x; j < MRG_SAMPLES; j += MQ_BLOCK) s_samp[j] = a.bkey[sample_pos(j, a.nb)];
    __syncthreads();
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
                    uint32_t lb, ub;
                    bounds_i32(a.bkey, a.nb, s_samp, key, lb, ub);
                    if (ub > lb) {
                        bl[k] = lb;
                        bc[k] = ub - lb;
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

