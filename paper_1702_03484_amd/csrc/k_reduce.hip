// ReduceDuplicate of Algorithm 1 on gfx950: after the shuffle, records with
// equal keys are contiguous, LEFT records (payload < n_left) ahead of RIGHT
// records within each key.  Three kernels:
//   seg_heads    compacts the first position of every distinct key,
//   seg_count    finds each key's LEFT/RIGHT split, counts cL*cR pairs and
//                scans the counts into exact output offsets,
//   materialize  writes the per-key cross products, LEFT-major, with the
//                output rows split evenly over the grid (a key with a huge
//                product is spread over many blocks).
#include "device_common.h"
#include "kernels.h"

#include <algorithm>

namespace mq {

constexpr int HEADS_IPT = 16;
constexpr int COUNT_IPT = 8;
constexpr uint32_t PERSIST_BLOCKS = 256 * 8;

__global__ __launch_bounds__(MQ_BLOCK) void seg_heads_kernel(const uint32_t* __restrict__ keys, uint32_t n,
                                                             uint32_t* __restrict__ seg_start,
                                                             uint32_t* __restrict__ nseg,
                                                             uint64_t* __restrict__ status,
                                                             uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint32_t TILE = MQ_BLOCK * HEADS_IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wtot[MQ_WAVES];
    __shared__ uint64_t s_excl;
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    for (;;) {
        const uint32_t tile = next_tile(tile_ctr, &s_tile);
        if (tile >= ntiles) break;
        const uint32_t base = tile * TILE;
        uint64_t hm[HEADS_IPT];
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < HEADS_IPT; i++) {
            uint32_t idx = base + (w * HEADS_IPT + i) * MQ_WAVE + lane();
            bool h = false;
            if (idx < n) h = idx == 0 || keys[idx] != keys[idx - 1];
            hm[i] = __ballot(h);
            run += (uint32_t)__popcll(hm[i]);
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
            if (tile == ntiles - 1) *nseg = (uint32_t)(ex + ttot);
        }
        __syncthreads();
        uint32_t pos = (uint32_t)s_excl + wex;
#pragma unroll
        for (int i = 0; i < HEADS_IPT; i++) {
            if ((hm[i] >> lane()) & 1ull) {
                uint32_t idx = base + (w * HEADS_IPT + i) * MQ_WAVE + lane();
                seg_start[pos + (uint32_t)__popcll(hm[i] & lt)] = idx;
            }
            pos += (uint32_t)__popcll(hm[i]);
        }
    }
}

hipError_t launch_seg_heads(const uint32_t* keys, uint32_t n, uint32_t* seg_start, uint32_t* nseg,
                            uint64_t* status, uint32_t* tile_ctr, uint32_t epoch, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint32_t tiles = (n + MQ_BLOCK * HEADS_IPT - 1) / (MQ_BLOCK * HEADS_IPT);
    uint32_t blocks = std::min(tiles, PERSIST_BLOCKS);
    seg_heads_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(keys, n, seg_start, nseg, status, tile_ctr, epoch);
    return hipGetLastError();
}

__global__ __launch_bounds__(MQ_BLOCK) void seg_count_kernel(const uint32_t* __restrict__ vals, uint32_t n,
                                                             uint32_t n_left,
                                                             const uint32_t* __restrict__ seg_start,
                                                             const uint32_t* __restrict__ nseg_p,
                                                             uint32_t* __restrict__ seg_split,
                                                             uint64_t* __restrict__ seg_off,
                                                             uint64_t* __restrict__ total,
                                                             uint64_t* __restrict__ status,
                                                             uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint32_t TILE = MQ_BLOCK * COUNT_IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_tmp[MQ_WAVES];
    __shared__ uint64_t s_excl;
    const uint32_t ns = n == 0 ? 0u : *nseg_p;
    const uint32_t ntiles = (ns + TILE - 1) / TILE;
    if (ns == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *total = 0;
        return;
    }
    for (;;) {
        const uint32_t tile = next_tile(tile_ctr, &s_tile);
        if (tile >= ntiles) break;
        // blocked layout: thread t owns segments base + t*IPT ... (+IPT-1)
        const uint32_t first = tile * TILE + threadIdx.x * COUNT_IPT;
        uint64_t cnt[COUNT_IPT];
        uint32_t split[COUNT_IPT];
        uint64_t sum = 0;
#pragma unroll
        for (int i = 0; i < COUNT_IPT; i++) {
            uint32_t s = first + i;
            cnt[i] = 0;
            split[i] = 0;
            if (s < ns) {
                uint32_t st = seg_start[s];
                uint32_t en = s + 1 < ns ? seg_start[s + 1] : n;
                uint32_t lo = st, hi = en;
                while (lo < hi) {
                    uint32_t mid = lo + ((hi - lo) >> 1);
                    if (vals[mid] < n_left) lo = mid + 1;
                    else hi = mid;
                }
                split[i] = lo;
                uint64_t c = (uint64_t)(lo - st) * (uint64_t)(en - lo);
                cnt[i] = c > SAT40 ? SAT40 : c;
            }
            sum += cnt[i];
        }
        uint64_t ttot;
        uint64_t ex_in = block_excl_scan<uint64_t>(sum, s_tmp, &ttot);
        if (threadIdx.x == 0) {
            uint64_t agg = ttot > SAT40 ? SAT40 : ttot;
            uint64_t ex = 0;
            if (tile == 0) {
                st_store(status, st_pack(epoch, ST_INC, agg));
            } else {
                st_store(status + tile, st_pack(epoch, ST_AGG, agg));
                ex = lookback(status, tile, 0, 1, epoch);
                st_store(status + tile, st_pack(epoch, ST_INC, sat_add(ex, agg)));
            }
            s_excl = ex;
            if (tile == ntiles - 1) *total = sat_add(ex, agg);
        }
        __syncthreads();
        uint64_t off = s_excl + ex_in;
#pragma unroll
        for (int i = 0; i < COUNT_IPT; i++) {
            uint32_t s = first + i;
            if (s < ns) {
                seg_split[s] = split[i];
                seg_off[s] = off > SAT40 ? SAT40 : off;
            }
            off += cnt[i];
        }
    }
}

hipError_t launch_seg_count(const uint32_t* vals, uint32_t n, uint32_t n_left, const uint32_t* seg_start,
                            const uint32_t* nseg, uint32_t max_seg, uint32_t* seg_split, uint64_t* seg_off,
                            uint64_t* total, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch,
                            hipStream_t stream) {
    uint32_t tiles = (max_seg + MQ_BLOCK * COUNT_IPT - 1) / (MQ_BLOCK * COUNT_IPT);
    uint32_t blocks = std::max(1u, std::min(tiles, PERSIST_BLOCKS));
    seg_count_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(vals, n, n_left, seg_start, nseg, seg_split, seg_off, total,
                                                      status, tile_ctr, epoch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Materialisation.  Output row j of segment s (offset off[s]) is the pair
// (LEFT record li, RIGHT record ri) with r = j - off[s], li = r / cR,
// ri = r % cR.  A thread owns RPT consecutive rows: one division, then
// increments, and one 16-byte store per column.
// ---------------------------------------------------------------------------
constexpr int MAT_RPT = 4;
constexpr uint32_t MAT_CHUNK = MQ_BLOCK * MAT_RPT;

// last segment s in [lo, hi] with off[s] <= j (off is non-decreasing)
__device__ __forceinline__ uint32_t seg_of(const uint64_t* off, uint32_t lo, uint32_t hi, uint64_t j) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int NC>
__global__ __launch_bounds__(MQ_BLOCK) void materialize_kernel(MatArgs a) {
    __shared__ uint32_t s_lo, s_hi;
    const uint32_t ns = *a.nseg;
    const uint64_t nchunks = (a.row_end - a.row_begin + MAT_CHUNK - 1) / MAT_CHUNK;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t j0 = a.row_begin + c * MAT_CHUNK;
        const uint64_t jend = min(j0 + MAT_CHUNK, a.row_end);
        if (threadIdx.x == 0) s_lo = seg_of(a.seg_off, 0, ns - 1, j0);
        if (threadIdx.x == 1) s_hi = seg_of(a.seg_off, 0, ns - 1, jend - 1);
        __syncthreads();
        const uint64_t j = j0 + (uint64_t)threadIdx.x * MAT_RPT;
        if (j < jend) {
            uint32_t s = seg_of(a.seg_off, s_lo, s_hi, j);
            uint32_t st = a.seg_start[s], sp = a.seg_split[s];
            uint32_t en = s + 1 < ns ? a.seg_start[s + 1] : a.n;
            uint32_t cl = sp - st, cr = en - sp;
            uint64_t r = j - a.seg_off[s];
            uint32_t li, ri;
            if (r < 0xffffffffull) {
                li = (uint32_t)r / cr;
                ri = (uint32_t)r - li * cr;
            } else {
                li = (uint32_t)(r / cr);
                ri = (uint32_t)(r - (uint64_t)li * cr);
            }
            int32_t key = (int32_t)(a.keys[st] + (uint32_t)a.key_base);
            uint32_t lrow = a.vals[st + li];
            int32_t v[NC][MAT_RPT];
            const int nk = (int)min((uint64_t)MAT_RPT, jend - j);
#pragma unroll
            for (int k = 0; k < MAT_RPT; k++) {
                if (k < nk) {
                    if (li == cl) {  // next non-empty segment
                        do {
                            s++;
                        } while (s + 1 < ns && a.seg_off[s + 1] <= j + k);
                        st = a.seg_start[s];
                        sp = a.seg_split[s];
                        en = s + 1 < ns ? a.seg_start[s + 1] : a.n;
                        cl = sp - st;
                        cr = en - sp;
                        li = 0;
                        ri = 0;
                        key = (int32_t)(a.keys[st] + (uint32_t)a.key_base);
                        lrow = a.vals[st];
                    }
                    const uint32_t rrow = a.vals[sp + ri] - a.n_left;
                    v[0][k] = key;
#pragma unroll
                    for (int col = 1; col < NC; col++)
                        v[col][k] = col <= a.nl ? a.lcol[col - 1][lrow] : a.rcol[col - 1 - a.nl][rrow];
                    if (++ri == cr) {
                        ri = 0;
                        if (++li < cl) lrow = a.vals[st + li];
                    }
                }
            }
            if (nk == MAT_RPT) {
#pragma unroll
                for (int col = 0; col < NC; col++)
                    *reinterpret_cast<int4*>(a.out[col] + j) = make_int4(v[col][0], v[col][1], v[col][2], v[col][3]);
            } else {
#pragma unroll
                for (int col = 0; col < NC; col++)
#pragma unroll
                    for (int k = 0; k < MAT_RPT; k++)
                        if (k < nk) a.out[col][j + k] = v[col][k];
            }
        }
        __syncthreads();
    }
}

hipError_t launch_materialize(const MatArgs& a, hipStream_t stream) {
    if (a.row_end <= a.row_begin) return hipSuccess;
    if (a.row_begin % MAT_RPT) return hipErrorInvalidValue;
    const int nc = 1 + a.nl + a.nr;
    uint64_t nchunks = (a.row_end - a.row_begin + MAT_CHUNK - 1) / MAT_CHUNK;
    uint32_t blocks = (uint32_t)std::min<uint64_t>(nchunks, 256ull * 16);
#define MQ_M(C) \
    case C: materialize_kernel<C><<<blocks, MQ_BLOCK, 0, stream>>>(a); break;
    switch (nc) {
        MQ_M(1) MQ_M(2) MQ_M(3) MQ_M(4) MQ_M(5) MQ_M(6) MQ_M(7) MQ_M(8)
        MQ_M(9) MQ_M(10) MQ_M(11) MQ_M(12) MQ_M(13) MQ_M(14) MQ_M(15) MQ_M(16)
        default: return hipErrorInvalidValue;
    }
#undef MQ_M
    return hipGetLastError();
}

}  // namespace mq
