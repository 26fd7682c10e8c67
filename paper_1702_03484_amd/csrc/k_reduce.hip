// ReduceDuplicate of Algorithm 1 on gfx950: after the shuffle, records with
// equal keys are contiguous, LEFT records (payload < n_left) ahead of RIGHT
// records within each key.  Three phases:
//   heads        compacts the first position of every distinct key and its
//                LEFT/RIGHT split,
//   count        counts cL*cR pairs per key and scans the counts into exact
//                output offsets,
//   materialize  writes the per-key cross products, with the output rows
//                split evenly over the grid (a key with a huge product is
//                spread over many blocks).
// Heads and count each run as two kernels with no ordering between blocks
// (no tile counter, no look-back): a sum pass in which block b owns a
// contiguous run of tiles and stores each tile's offset within the run and
// the run's total, one block that turns the run totals into prefix sums,
// then a write pass with one tile per block whose offset is its run's
// prefix plus its in-run offset.
#include "device_common.h"
#include "kernels.h"
#include "tile_ops.h"

#include <algorithm>

namespace mq {

constexpr int HEADS_IPT = 16;
constexpr uint32_t HEADS_TILE = MQ_BLOCK * HEADS_IPT;
constexpr int COUNT_IPT = 8;
constexpr uint32_t COUNT_TILE = MQ_BLOCK * COUNT_IPT;
// blocks of a sum pass: one resident round of the sum kernels (up to 64
// VGPRs, 8 blocks per CU on 256 CUs), so each block sums only a few tiles
// (1,024 blocks: count phase of the 16M + 16M join 0.279 ms; 2,048: 0.247)
constexpr uint32_t RUN_BLOCKS = 2048;

struct RunGrid {
    uint32_t ntiles, chunk, blocks;
};

__host__ __device__ inline RunGrid run_grid(uint32_t ntiles) {
    RunGrid g;
    g.ntiles = ntiles;
    const uint32_t want = ntiles < RUN_BLOCKS ? ntiles : RUN_BLOCKS;
    g.chunk = want ? (ntiles + want - 1) / want : 0;
    g.blocks = g.chunk ? (ntiles + g.chunk - 1) / g.chunk : 0;
    return g;
}

// Key and payload of record idx and of its neighbours, for every lane of a
// wave that covers 64 consecutive records (lanes past n see key ~0u).
struct RecView {
    uint32_t k, v, kprev, vprev, knext;
};

// vals may be null (the side rides in the key): payloads then read as 0.
__device__ __forceinline__ RecView rec_view(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                            uint32_t n, uint32_t idx) {
    RecView r;
    const bool in = idx < n;
    r.k = in ? keys[idx] : ~0u;
    r.v = in && vals ? vals[idx] : 0u;
    // neighbours from the adjacent lanes; the wave's edge lanes load them
    r.kprev = __shfl_up(r.k, 1, MQ_WAVE);
    r.vprev = __shfl_up(r.v, 1, MQ_WAVE);
    r.knext = __shfl_down(r.k, 1, MQ_WAVE);
    if (lane() == 0 && in && idx > 0) {
        r.kprev = keys[idx - 1];
        r.vprev = vals ? vals[idx - 1] : 0u;
    }
    if (lane() == MQ_WAVE - 1 && idx + 1 < n) r.knext = keys[idx + 1];
    return r;
}

// fs = 1 when the key's low bit is the side (segments group keys >> 1)
__device__ __forceinline__ bool rec_is_head(const RecView& r, uint32_t idx, uint32_t n, uint32_t fs) {
    return idx < n && (idx == 0 || (r.kprev >> fs) != (r.k >> fs));
}

// sum pass: heads of every tile of the block's run (BRK: a record flagged in
// brk also heads a segment: the further words of a composite key change)
template <bool BRK>
__global__ __launch_bounds__(MQ_BLOCK) void heads_sum_kernel(const uint32_t* __restrict__ keys,
                                                             const uint8_t* __restrict__ brk, uint32_t n,
                                                             uint32_t fs, uint64_t* __restrict__ run_tot,
                                                             uint32_t* __restrict__ tloc, RunGrid g) {
    __shared__ uint32_t s_wtot[MQ_WAVES];
    __shared__ uint32_t s_run;
    const uint32_t w = threadIdx.x / MQ_WAVE;
    if (threadIdx.x == 0) s_run = 0;
    const uint32_t t0 = blockIdx.x * g.chunk;
    const uint32_t t1 = min(t0 + g.chunk, g.ntiles);
    for (uint32_t tile = t0; tile < t1; tile++) {
        const uint32_t base = tile * HEADS_TILE;
        uint32_t k[HEADS_IPT];
        bool f[HEADS_IPT];
#pragma unroll
        for (int i = 0; i < HEADS_IPT; i++) {
            const uint32_t idx = base + (w * HEADS_IPT + i) * MQ_WAVE + lane();
            k[i] = idx < n ? keys[idx] : 0u;
            f[i] = BRK && idx < n && brk[idx] != 0;
        }
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < HEADS_IPT; i++) {
            const uint32_t idx = base + (w * HEADS_IPT + i) * MQ_WAVE + lane();
            uint32_t kp = __shfl_up(k[i], 1, MQ_WAVE);
            if (lane() == 0 && idx > 0 && idx < n) kp = keys[idx - 1];
            const bool head = (kp >> fs) != (k[i] >> fs) || f[i];
            run += (uint32_t)__popcll(__ballot(idx < n && (idx == 0 || head)));
        }
        if (lane() == 0) s_wtot[w] = run;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
#pragma unroll
            for (int i = 0; i < MQ_WAVES; i++) tot += s_wtot[i];
            tloc[tile] = s_run;
            s_run += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) run_tot[blockIdx.x] = s_run;
}

// write pass: one tile per block
template <bool BRK>
__global__ __launch_bounds__(MQ_BLOCK) void heads_write_kernel(const uint32_t* __restrict__ keys,
                                                               const uint8_t* __restrict__ brk,
                                                               const uint32_t* __restrict__ vals, uint32_t n,
                                                               uint32_t n_left, uint32_t fs,
                                                               const uint64_t* __restrict__ run_excl,
                                                               const uint32_t* __restrict__ tloc, RunGrid g,
                                                               uint32_t* __restrict__ seg_start,
                                                               uint32_t* __restrict__ seg_split) {
    __shared__ uint32_t s_wtot[MQ_WAVES];
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    const uint32_t tile = blockIdx.x;
    const uint32_t base = tile * HEADS_TILE;
    RecView r[HEADS_IPT];
    bool f[HEADS_IPT], fnext[HEADS_IPT];  // this record / the next one flagged in brk
#pragma unroll
    for (int i = 0; i < HEADS_IPT; i++) {
        const uint32_t idx = base + (w * HEADS_IPT + i) * MQ_WAVE + lane();
        r[i] = rec_view(keys, vals, n, idx);
        f[i] = BRK && idx < n && brk[idx] != 0;
        fnext[i] = BRK && idx + 1 < n && brk[idx + 1] != 0;
    }
    uint64_t hm[HEADS_IPT];
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < HEADS_IPT; i++) {
        const uint32_t idx = base + (w * HEADS_IPT + i) * MQ_WAVE + lane();
        hm[i] = __ballot(rec_is_head(r[i], idx, n, fs) || f[i]);
        run += (uint32_t)__popcll(hm[i]);
    }
    if (lane() == 0) s_wtot[w] = run;
    __syncthreads();
    // heads before this tile: its run's prefix, then its offset within the run
    uint32_t pos = (uint32_t)run_excl[tile / g.chunk] + tloc[tile];
#pragma unroll
    for (int i = 0; i < MQ_WAVES; i++) pos += (uint32_t)i < w ? s_wtot[i] : 0u;
#pragma unroll
    for (int i = 0; i < HEADS_IPT; i++) {
        const uint32_t idx = base + (w * HEADS_IPT + i) * MQ_WAVE + lane();
        const bool h = (hm[i] >> lane()) & 1ull;
        const uint32_t bef = pos + (uint32_t)__popcll(hm[i] & lt);  // heads before this record
        if (idx < n) {
            const bool is_r = fs ? (r[i].k & 1u) != 0 : r[i].v >= n_left;
            const bool prev_r = fs ? (r[i].kprev & 1u) != 0 : r[i].vprev >= n_left;
            const bool last = idx + 1 == n || (r[i].knext >> fs) != (r[i].k >> fs) || fnext[i];
            const bool first_r = is_r && (h || !prev_r);
            if (h && MQ_IN_BOUNDS(bef, n)) seg_start[bef] = idx;
            if (first_r || (last && !is_r)) {
                const uint32_t sid = h ? bef : bef - 1u;  // record 0 is always a head
                if (MQ_IN_BOUNDS(sid, n)) seg_split[sid] = first_r ? idx : idx + 1;
            }
        }
        pos += (uint32_t)__popcll(hm[i]);
    }
}

// Scratch of the heads and count phases (u64 words first): heads run
// totals, count run totals, count run maxima, count per-tile offsets, then
// heads per-tile offsets (u32).
struct SegScratch {
    uint64_t *h_run, *c_run, *c_max, *c_tloc;
    uint32_t* h_tloc;
};

static RunGrid heads_grid(uint32_t n) { return run_grid((n + HEADS_TILE - 1) / HEADS_TILE); }
static RunGrid count_grid(uint32_t max_seg) { return run_grid(std::max(1u, (max_seg + COUNT_TILE - 1) / COUNT_TILE)); }

static SegScratch seg_scratch(void* p, uint32_t n) {
    const RunGrid gh = heads_grid(n), gc = count_grid(n);
    SegScratch s;
    s.h_run = static_cast<uint64_t*>(p);
    s.c_run = s.h_run + gh.blocks;
    s.c_max = s.c_run + gc.blocks;
    s.c_tloc = s.c_max + gc.blocks;
    s.h_tloc = reinterpret_cast<uint32_t*>(s.c_tloc + gc.ntiles);
    return s;
}

size_t seg_scratch_bytes(uint32_t n) {
    const RunGrid gh = heads_grid(n), gc = count_grid(n);
    return 8ull * (gh.blocks + 2ull * gc.blocks + gc.ntiles) + 4ull * gh.ntiles;
}

hipError_t launch_seg_heads(const uint32_t* keys, const uint32_t* vals, uint32_t n, uint32_t n_left,
                            int side_bit, uint32_t* seg_start, uint32_t* seg_split, uint32_t* nseg, void* scratch,
                            hipStream_t stream, const uint8_t* brk) {
    const uint32_t fs = side_bit ? 1u : 0u;
    if (n == 0) return hipSuccess;
    const RunGrid g = heads_grid(n);
    const SegScratch ss = seg_scratch(scratch, n);
    if (brk)
        heads_sum_kernel<true><<<g.blocks, MQ_BLOCK, 0, stream>>>(keys, brk, n, fs, ss.h_run, ss.h_tloc, g);
    else
        heads_sum_kernel<false><<<g.blocks, MQ_BLOCK, 0, stream>>>(keys, nullptr, n, fs, ss.h_run, ss.h_tloc, g);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan_runs(ss.h_run, g.blocks, nullptr, nseg, nullptr, nullptr, stream);
    if (e != hipSuccess) return e;
    if (brk)
        heads_write_kernel<true><<<g.ntiles, MQ_BLOCK, 0, stream>>>(keys, brk, fs ? nullptr : vals, n, n_left, fs,
                                                                   ss.h_run, ss.h_tloc, g, seg_start, seg_split);
    else
        heads_write_kernel<false><<<g.ntiles, MQ_BLOCK, 0, stream>>>(keys, nullptr, fs ? nullptr : vals, n, n_left,
                                                                    fs, ss.h_run, ss.h_tloc, g, seg_start, seg_split);
    return hipGetLastError();
}

__device__ __forceinline__ uint64_t block_reduce_sum(uint64_t v, uint64_t* tmp) {
#pragma unroll
    for (int o = MQ_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane() == 0) tmp[threadIdx.x / MQ_WAVE] = v;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < MQ_WAVES; i++) t += tmp[i];
    __syncthreads();
    return t;
}

// pairs of segment s: (split - start) * (end - split), capped at 2^40 - 1
__device__ __forceinline__ uint64_t seg_pairs(const uint32_t* __restrict__ seg_start,
                                              const uint32_t* __restrict__ seg_split, uint32_t n, uint32_t ns,
                                              uint32_t s) {
    if (s >= ns) return 0;
    const uint32_t st = seg_start[s];
    const uint32_t en = s + 1 < ns ? seg_start[s + 1] : n;
    const uint32_t sp = seg_split[s];
    const uint64_t c = (uint64_t)(sp - st) * (uint64_t)(en - sp);
    return c > SAT40 ? SAT40 : c;
}

// The segment count lives on the device; both count kernels are sized for
// max_seg segments and treat tiles past the real count as empty.
__global__ __launch_bounds__(MQ_BLOCK) void count_sum_kernel(uint32_t n, const uint32_t* __restrict__ seg_start,
                                                             const uint32_t* __restrict__ nseg_p,
                                                             const uint32_t* __restrict__ seg_split,
                                                             uint64_t* __restrict__ run_tot,
                                                             uint64_t* __restrict__ run_max,
                                                             uint64_t* __restrict__ tloc, RunGrid g) {
    __shared__ uint64_t s_tmp[MQ_WAVES];
    __shared__ uint64_t s_run;
    uint64_t mx = 0;  // this thread's largest count
    const uint32_t ns = n == 0 ? 0u : *nseg_p;
    if (threadIdx.x == 0) s_run = 0;
    const uint32_t t0 = blockIdx.x * g.chunk;
    const uint32_t t1 = min(t0 + g.chunk, g.ntiles);
    for (uint32_t tile = t0; tile < t1; tile++) {
        // any order within the tile: coalesced, segment base + i * 256 + thread
        const uint32_t base = tile * COUNT_TILE;
        uint64_t sum = 0;
        if (base < ns) {
#pragma unroll
            for (int i = 0; i < COUNT_IPT; i++) {
                const uint64_t c = seg_pairs(seg_start, seg_split, n, ns, base + i * MQ_BLOCK + threadIdx.x);
                sum += c;
                mx = c > mx ? c : mx;
            }
        }
        const uint64_t tot = block_reduce_sum(sum, s_tmp);
        if (threadIdx.x == 0) {
            tloc[tile] = s_run;
            s_run = sat_add(s_run, tot > SAT40 ? SAT40 : tot);
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = MQ_WAVE / 2; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(mx, o);
        mx = y > mx ? y : mx;
    }
    if (lane() == 0) s_tmp[threadIdx.x / MQ_WAVE] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        run_tot[blockIdx.x] = s_run;
        for (int i = 0; i < MQ_WAVES; i++) mx = s_tmp[i] > mx ? s_tmp[i] : mx;
        run_max[blockIdx.x] = mx;
    }
}

__global__ __launch_bounds__(MQ_BLOCK) void count_write_kernel(uint32_t n, const uint32_t* __restrict__ seg_start,
                                                               const uint32_t* __restrict__ nseg_p,
                                                               const uint32_t* __restrict__ seg_split,
                                                               const uint64_t* __restrict__ run_excl,
                                                               const uint64_t* __restrict__ tloc, RunGrid g,
                                                               uint64_t* __restrict__ seg_off) {
    __shared__ uint64_t s_tmp[MQ_WAVES];
    const uint32_t ns = n == 0 ? 0u : *nseg_p;
    const uint32_t tile = blockIdx.x;
    const uint32_t ntiles = (ns + COUNT_TILE - 1) / COUNT_TILE;
    if (tile >= ntiles) return;
    // wave-striped: slot i of wave w holds segments base + (w * IPT + i) * 64 + lane
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint32_t base = tile * COUNT_TILE + w * COUNT_IPT * MQ_WAVE;
    uint32_t st[COUNT_IPT], sp[COUNT_IPT];
#pragma unroll
    for (int i = 0; i < COUNT_IPT; i++) {
        const uint32_t s = base + i * MQ_WAVE + lane();
        st[i] = s < ns ? seg_start[s] : n;
        sp[i] = s < ns ? seg_split[s] : n;
    }
    uint64_t cnt[COUNT_IPT];
    uint64_t wsum = 0;  // this wave's pairs before slot i
    uint64_t excl[COUNT_IPT];
#pragma unroll
    for (int i = 0; i < COUNT_IPT; i++) {
        const uint32_t s = base + i * MQ_WAVE + lane();
        uint32_t en = __shfl_down(st[i], 1, MQ_WAVE);
        if (lane() == MQ_WAVE - 1) en = s + 1 < ns ? seg_start[s + 1] : n;
        if (s + 1 >= ns) en = n;
        const uint64_t c = s < ns ? (uint64_t)(sp[i] - st[i]) * (uint64_t)(en - sp[i]) : 0ull;
        cnt[i] = c > SAT40 ? SAT40 : c;
        const uint64_t inc = wave_incl_scan<uint64_t>(cnt[i]);
        excl[i] = wsum + inc - cnt[i];
        wsum += (uint64_t)__shfl(inc, MQ_WAVE - 1, MQ_WAVE);
    }
    if (lane() == 0) s_tmp[w] = wsum;
    __syncthreads();
    // pairs before this tile: its run's prefix (capped), then its offset within the run
    uint64_t off = sat_add(run_excl[tile / g.chunk], tloc[tile]), wex = 0;
#pragma unroll
    for (int i = 0; i < MQ_WAVES; i++) wex += (uint32_t)i < w ? s_tmp[i] : 0ull;
    off = sat_add(off, wex > SAT40 ? SAT40 : wex);
#pragma unroll
    for (int i = 0; i < COUNT_IPT; i++) {
        const uint32_t s = base + i * MQ_WAVE + lane();
        if (s < ns) seg_off[s] = sat_add(off, excl[i] > SAT40 ? SAT40 : excl[i]);
    }
}

hipError_t launch_seg_count(uint32_t n, const uint32_t* seg_start, const uint32_t* nseg, uint32_t max_seg,
                            const uint32_t* seg_split, uint64_t* seg_off, uint64_t* total, uint64_t* max_pairs,
                            void* scratch, hipStream_t stream) {
    if (max_seg > n) return hipErrorInvalidValue;  // the scratch is laid out for n
    const RunGrid g = count_grid(max_seg);
    const SegScratch ss = seg_scratch(scratch, n);
    count_sum_kernel<<<g.blocks, MQ_BLOCK, 0, stream>>>(n, seg_start, nseg, seg_split, ss.c_run, ss.c_max, ss.c_tloc,
                                                       g);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan_runs(ss.c_run, g.blocks, total, nullptr, ss.c_max, max_pairs, stream);
    if (e != hipSuccess) return e;
    count_write_kernel<<<g.ntiles, MQ_BLOCK, 0, stream>>>(n, seg_start, nseg, seg_split, ss.c_run, ss.c_tloc, g,
                                                         seg_off);
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
__device__ __forceinline__ MatJoin mat_join_of(const MatArgs& a) {
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
    mj.key_shift = a.key_shift;
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
    return mj;
}

template <int NC, int NLC>
__global__ __launch_bounds__(MQ_BLOCK) void materialize_kernel(MatArgs a) {
    constexpr uint32_t WROWS = MatShape<NC>::WROWS;
    __shared__ uint64_t s_segs[MQ_WAVES][MAT_LDS_SEGS];
    const MatJoin mj = mat_join_of<NC, NLC>(a);
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

// Segment-major materialisation (mat_seg_group): one wave per group of 64
// keys, for outputs whose key products are small.
template <int NC, int NLC>
__global__ __launch_bounds__(MQ_BLOCK) void mat_seg_kernel(MatArgs a) {
    __shared__ uint64_t s_grp[MQ_WAVES][MAT_SEG_LDS_WORDS];
    const MatJoin mj = mat_join_of<NC, NLC>(a);
    const uint32_t ngroups = (mj.ns + MQ_WAVE - 1) / MQ_WAVE;
    const uint32_t nw = gridDim.x * MQ_WAVES;
    for (uint32_t grp = blockIdx.x * MQ_WAVES + threadIdx.x / MQ_WAVE; grp < ngroups; grp += nw)
        mat_seg_group<NC, NLC>(mj, grp, a.row_end, s_grp[threadIdx.x / MQ_WAVE]);
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
    if (a.seg_major && (a.row_begin != 0 || a.seg_cl != nullptr)) return hipErrorInvalidValue;
    const int nc = 1 + a.nl + a.nr;
    const uint64_t rows = a.row_end - a.row_begin;
    const uint64_t cap = a.max_blocks ? a.max_blocks : MAT_MAX_BLOCKS;
    // narrow joins get the value-column split fixed at compile time
#define MQ_LAUNCH(C, L)                                                                             \
    if (a.seg_major) {                                                                              \
        const uint64_t groups = (a.seg_count + MQ_WAVE - 1) / MQ_WAVE;                              \
        uint32_t blocks = (uint32_t)std::min<uint64_t>((groups + MQ_WAVES - 1) / MQ_WAVES, cap);       \
        mat_seg_kernel<C, L><<<std::max(blocks, 1u), MQ_BLOCK, 0, stream>>>(a);                     \
    } else {                                                                                        \
        const uint64_t crows = a.sparse ? 4 * MQ_WAVE : MatShape<C>::WROWS;                         \
        uint64_t chunks = (rows + crows - 1) / crows;                                               \
        uint32_t blocks = (uint32_t)std::min<uint64_t>((chunks + MQ_WAVES - 1) / MQ_WAVES, cap);       \
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
