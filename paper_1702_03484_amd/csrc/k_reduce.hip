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
#include "tile_ops.h"

#include <algorithm>

namespace mq {

constexpr int HEADS_IPT = 16;
constexpr int COUNT_IPT = 8;
constexpr uint32_t PERSIST_BLOCKS = 256 * 8;

__global__ __launch_bounds__(MQ_BLOCK) void seg_heads_kernel(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ vals, uint32_t n,
                                                             uint32_t n_left, uint32_t* __restrict__ seg_start,
                                                             uint32_t* __restrict__ seg_split,
                                                             uint32_t* __restrict__ nseg,
                                                             uint64_t* __restrict__ status,
                                                             uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint32_t TILE = MQ_BLOCK * HEADS_IPT;
    __shared__ HeadsSmem sm;
    __shared__ uint32_t s_tile;
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    for (;;) {
        const uint32_t tile = next_tile(tile_ctr, &s_tile);
        if (tile >= ntiles) break;
        heads_tile<HEADS_IPT>(sm, keys, vals, n, n_left, tile * TILE, tile, 0, tile == ntiles - 1, seg_start,
                              seg_split, nseg, status, epoch);
    }
}

hipError_t launch_seg_heads(const uint32_t* keys, const uint32_t* vals, uint32_t n, uint32_t n_left,
                            uint32_t* seg_start, uint32_t* seg_split, uint32_t* nseg, uint64_t* status,
                            uint32_t* tile_ctr, uint32_t epoch, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint32_t tiles = (n + MQ_BLOCK * HEADS_IPT - 1) / (MQ_BLOCK * HEADS_IPT);
    uint32_t blocks = std::min(tiles, PERSIST_BLOCKS);
    seg_heads_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(keys, vals, n, n_left, seg_start, seg_split, nseg, status,
                                                      tile_ctr, epoch);
    return hipGetLastError();
}

// cnt[s] = (split - start) * (end - split), scanned into exact output
// offsets (saturating at 2^40 - 1); *total = the sum.
__global__ __launch_bounds__(MQ_BLOCK) void seg_count_kernel(uint32_t n, const uint32_t* __restrict__ seg_start,
                                                             const uint32_t* __restrict__ nseg_p,
                                                             const uint32_t* __restrict__ seg_split,
                                                             uint64_t* __restrict__ seg_off,
                                                             uint64_t* __restrict__ total,
                                                             uint64_t* __restrict__ status,
                                                             uint32_t* __restrict__ tile_ctr, uint32_t epoch) {
    constexpr uint32_t TILE = MQ_BLOCK * COUNT_IPT;
    __shared__ CountSmem sm;
    __shared__ uint32_t s_tile;
    const uint32_t ns = n == 0 ? 0u : *nseg_p;
    const uint32_t ntiles = (ns + TILE - 1) / TILE;
    if (ns == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *total = 0;
        return;
    }
    for (;;) {
        const uint32_t tile = next_tile(tile_ctr, &s_tile);
        if (tile >= ntiles) break;
        count_tile<COUNT_IPT>(sm, n, ns, tile * TILE, tile, 0, tile == ntiles - 1, seg_start, seg_split, seg_off,
                              total, status, epoch);
    }
}

hipError_t launch_seg_count(uint32_t n, const uint32_t* seg_start, const uint32_t* nseg, uint32_t max_seg,
                            const uint32_t* seg_split, uint64_t* seg_off, uint64_t* total, uint64_t* status,
                            uint32_t* tile_ctr, uint32_t epoch, hipStream_t stream) {
    uint32_t tiles = (max_seg + MQ_BLOCK * COUNT_IPT - 1) / (MQ_BLOCK * COUNT_IPT);
    uint32_t blocks = std::max(1u, std::min(tiles, PERSIST_BLOCKS));
    seg_count_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(n, seg_start, nseg, seg_split, seg_off, total, status,
                                                      tile_ctr, epoch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Materialisation: waves own chunks of 64*RPT consecutive output rows.
// ---------------------------------------------------------------------------
template <int NC>
struct MatShape {
    static constexpr int RPT = NC <= 4 ? 16 : (NC <= 8 ? 8 : 4);  // rows per lane
    static constexpr uint32_t WROWS = MQ_WAVE * RPT;               // rows per wave chunk
};

template <int NC, int NLC>
__global__ __launch_bounds__(MQ_BLOCK) void materialize_kernel(MatArgs a) {
    constexpr uint32_t WROWS = MatShape<NC>::WROWS;
    __shared__ uint64_t s_segs[MQ_WAVES][MAT_LDS_SEGS];
    MatJoin mj;
    mj.keys = a.keys;
    mj.vals = a.vals;
    mj.seg_start = a.seg_start;
    mj.seg_split = a.seg_split;
    mj.seg_off = a.seg_off;
    mj.ns = *a.nseg;
    mj.n = a.n;
    mj.n_left = a.n_left;
    mj.key_base = a.key_base;
    mj.nl = NLC >= 0 ? NLC : a.nl;
    mj.nr = NLC >= 0 ? NC - 1 - NLC : a.nr;
    const bool merged = a.seg_cl != nullptr;
    mj.sorted_vals = merged || a.use_sval != 0;
    mj.seg_cl = a.seg_cl;
    mj.seg_cr = a.seg_cr;
#pragma unroll
    for (int c = 0; c < NC; c++) {
        mj.out[c] = a.out[c];
        if (c >= 1) {
            const bool left = c <= mj.nl;
            mj.src[c] = left ? a.lcol[c - 1] : a.rcol[c - 1 - mj.nl];
            // merge join: runs index the tables' own (key-sorted) columns
            mj.ssrc[c] = merged ? mj.src[c] : (left ? a.sval[c - 1] : a.sval[c - 1 - mj.nl]);
        }
    }
    // chunks strided over the waves (the rows being written at any moment
    // stay in one window of the output); a wave's previous segment is the
    // starting guess for its next chunk
    const int qn = a.sparse ? 1 : MatShape<NC>::RPT / 4;
    const uint32_t crows = a.sparse ? 4 * MQ_WAVE : WROWS;
    const uint64_t nchunks = (a.row_end - a.row_begin + crows - 1) / crows;
    const uint64_t gw = (uint64_t)blockIdx.x * MQ_WAVES + threadIdx.x / MQ_WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * MQ_WAVES;
    uint32_t hint = 0;
    for (uint64_t c = gw; c < nchunks; c += nw) {
        const uint64_t j0 = a.row_begin + c * crows;
        mat_wave_chunk<NC, MatShape<NC>::RPT, NLC>(mj, j0, min(j0 + crows, a.row_end), hint,
                                                   s_segs[threadIdx.x / MQ_WAVE], qn);
    }
}

// One pass over the sorted records: every record's value columns move into
// sorted order, so that materialisation reads contiguous ranges instead of
// gathering each output row's values through its record id.
__global__ __launch_bounds__(MQ_BLOCK) void gather_values_kernel(GatherArgs g) {
    const uint32_t stride = gridDim.x * MQ_BLOCK;
    for (uint32_t i = blockIdx.x * MQ_BLOCK + threadIdx.x; i < g.n; i += stride) {
        const uint32_t r = g.vals[i];
        if (r < g.n_left) {
            for (int c = 0; c < g.nl; c++) g.out[c][i] = g.lcol[c][r];
        } else {
            for (int c = 0; c < g.nr; c++) g.out[c][i] = g.rcol[c][r - g.n_left];
        }
    }
}

hipError_t launch_gather_values(const GatherArgs& g, hipStream_t stream) {
    if (g.n == 0 || (g.nl == 0 && g.nr == 0)) return hipSuccess;
    const uint32_t blocks = std::min((g.n + MQ_BLOCK * 4 - 1) / (MQ_BLOCK * 4), 8192u);
    gather_values_kernel<<<blocks, MQ_BLOCK, 0, stream>>>(g);
    return hipGetLastError();
}

hipError_t launch_materialize(const MatArgs& a, hipStream_t stream) {
    if (a.row_end <= a.row_begin) return hipSuccess;
    if (a.row_begin % 16) return hipErrorInvalidValue;
    const int nc = 1 + a.nl + a.nr;
    const uint64_t rows = a.row_end - a.row_begin;
    // narrow joins get the value-column split fixed at compile time
#define MQ_LAUNCH(C, L)                                                                             \
    {                                                                                               \
        const uint64_t crows = a.sparse ? 4 * MQ_WAVE : MatShape<C>::WROWS;                         \
        uint64_t chunks = (rows + crows - 1) / crows;                                               \
        uint32_t blocks = (uint32_t)std::min<uint64_t>((chunks + MQ_WAVES - 1) / MQ_WAVES, 256ull * 32); \
        materialize_kernel<C, L><<<blocks, MQ_BLOCK, 0, stream>>>(a);                               \
    }
    if (nc <= 4) {
        const int key = nc * 4 + a.nl;
        switch (key) {
            case 1 * 4 + 0: MQ_LAUNCH(1, 0) break;
            case 2 * 4 + 0: MQ_LAUNCH(2, 0) break;
            case 2 * 4 + 1: MQ_LAUNCH(2, 1) break;
            case 3 * 4 + 0: MQ_LAUNCH(3, 0) break;
            case 3 * 4 + 1: MQ_LAUNCH(3, 1) break;
            case 3 * 4 + 2: MQ_LAUNCH(3, 2) break;
            case 4 * 4 + 0: MQ_LAUNCH(4, 0) break;
            case 4 * 4 + 1: MQ_LAUNCH(4, 1) break;
            case 4 * 4 + 2: MQ_LAUNCH(4, 2) break;
            case 4 * 4 + 3: MQ_LAUNCH(4, 3) break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (nc) {
        case 5: MQ_LAUNCH(5, -1) break;
        case 6: MQ_LAUNCH(6, -1) break;
        case 7: MQ_LAUNCH(7, -1) break;
        case 8: MQ_LAUNCH(8, -1) break;
        case 9: MQ_LAUNCH(9, -1) break;
        case 10: MQ_LAUNCH(10, -1) break;
        case 11: MQ_LAUNCH(11, -1) break;
        case 12: MQ_LAUNCH(12, -1) break;
        case 13: MQ_LAUNCH(13, -1) break;
        case 14: MQ_LAUNCH(14, -1) break;
        case 15: MQ_LAUNCH(15, -1) break;
        case 16: MQ_LAUNCH(16, -1) break;
        default: return hipErrorInvalidValue;
    }
#undef MQ_LAUNCH
    return hipGetLastError();
}

}  // namespace mq
