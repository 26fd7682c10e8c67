// Map of Algorithm 1 on gfx950: scan a range of the store (or any SoA
// table), keep the rows that pass the pattern's equality tests, and emit
// the variable columns in input order.  Up to 2^31 rows, one launch
// (compact_fused_kernel below); beyond that, two passes with no ordering
// between blocks (no tile counter, no look-back).  In the test pass block b owns a
// contiguous run of tiles; it reads only the columns the tests use and
// stores one __ballot word per 64 rows, the kept rows of its run before
// each tile, and its run's total.  One block turns the run totals into
// their prefix sums.  The write pass takes one tile per block (so clustered
// output spreads over the whole grid): its offset is its run's prefix plus
// its in-run offset, and it copies the output columns of the rows its mask
// words mark.
// The same kernels filter join results on further shared variables.
#include "device_common.h"
#include "kernels.h"

#include <algorithm>

namespace mq {

constexpr int CMP_IPT = 16;                                // row slots per thread per tile
constexpr uint64_t CMP_TILE = (uint64_t)MQ_BLOCK * CMP_IPT;  // rows per tile
constexpr uint64_t CMP_TILE_WORDS = CMP_TILE / 64;          // mask words per tile
constexpr uint64_t CMP_MAX_BLOCKS = 1024;                   // 4 blocks per CU: one resident wave of blocks

struct CompactGrid {
    uint64_t ntiles, chunk, blocks;
};

__host__ __device__ inline CompactGrid grid_of_runs(uint64_t n, uint64_t max_blocks) {
    CompactGrid g;
    g.ntiles = (n + CMP_TILE - 1) / CMP_TILE;
    const uint64_t want = g.ntiles < max_blocks ? g.ntiles : max_blocks;
    g.chunk = want ? (g.ntiles + want - 1) / want : 0;
    g.blocks = g.chunk ? (g.ntiles + g.chunk - 1) / g.chunk : 0;
    return g;
}

__host__ __device__ inline CompactGrid compact_grid(uint64_t n) { return grid_of_runs(n, CMP_MAX_BLOCKS); }

// the single-launch kernel: one resident round of blocks (4-5 per CU); each
// block then runs about a dozen tiles back to back (more blocks, each with
// fewer tiles, measured slower: they wait for a second round)
constexpr uint64_t CMP_FUSED_BLOCKS = 1024;
__host__ __device__ inline CompactGrid compact_grid_fused(uint64_t n) { return grid_of_runs(n, CMP_FUSED_BLOCKS); }

// the kept count of the calling wave's 64-row slot i sits in lane i of `mine`
__device__ __forceinline__ uint64_t pick_slot(const uint64_t (&km)[CMP_IPT]) {
    uint64_t mine = 0;
#pragma unroll
    for (int i = 0; i < CMP_IPT; i++) mine = lane() == (uint32_t)i ? km[i] : mine;
    return mine;
}

__global__ __launch_bounds__(MQ_BLOCK) void compact_test_kernel(CompactArgs a, uint64_t* __restrict__ counts,
                                                                uint32_t* __restrict__ tloc,
                                                                uint64_t* __restrict__ mask, CompactGrid g) {
    __shared__ uint32_t s_wtot[MQ_WAVES];
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t t0 = (uint64_t)blockIdx.x * g.chunk;
    const uint64_t t1 = t0 + g.chunk < g.ntiles ? t0 + g.chunk : g.ntiles;
    __shared__ uint32_t s_run;  // kept rows of the run's tiles so far
    if (threadIdx.x == 0) s_run = 0;
    for (uint64_t tile = t0; tile < t1; tile++) {
        const uint64_t base = tile * CMP_TILE;
        // the first test's operands of every row slot are loaded before any
        // compare, so each wave keeps CMP_IPT loads in flight; further tests
        // (a repeated variable next to a constant) load per slot
        bool ok[CMP_IPT];
        {
            const int32_t* A = a.nterm > 0 ? a.in[a.term_a[0]] : nullptr;
            const int32_t* B = a.nterm > 0 && a.term_b[0] >= 0 ? a.in[a.term_b[0]] : nullptr;
            const int32_t c0 = a.nterm > 0 ? a.term_c[0] : 0;
            int32_t va[CMP_IPT], vb[CMP_IPT];
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) {
                const uint64_t idx = base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane());
                ok[i] = idx < a.n;
                va[i] = A && ok[i] ? A[idx] : 0;
                vb[i] = B && ok[i] ? B[idx] : c0;
            }
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) ok[i] = ok[i] && (!A || va[i] == vb[i]);
        }
        for (int t = 1; t < a.nterm; t++) {
            const int32_t* A = a.in[a.term_a[t]];
            const int32_t* B = a.term_b[t] >= 0 ? a.in[a.term_b[t]] : nullptr;
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) {
                const uint64_t idx = base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane());
                if (ok[i]) ok[i] = A[idx] == (B ? B[idx] : a.term_c[t]);
            }
        }
        uint64_t km[CMP_IPT];
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < CMP_IPT; i++) {
            km[i] = __ballot(ok[i]);
            run += (uint32_t)__popcll(km[i]);
        }
        // slot i of wave w covers rows base + (w * CMP_IPT + i) * 64 + [0, 64)
        const uint64_t mine = pick_slot(km);
        if (lane() < (uint32_t)CMP_IPT) mask[tile * CMP_TILE_WORDS + w * CMP_IPT + lane()] = mine;
        if (lane() == 0) s_wtot[w] = run;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
#pragma unroll
            for (int i = 0; i < MQ_WAVES; i++) tot += s_wtot[i];
            tloc[tile] = s_run;
            s_run += tot;
        }
        __syncthreads();  // s_wtot is rewritten by the next tile
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s_run;
}

__global__ __launch_bounds__(MQ_BLOCK) void compact_write_kernel(CompactArgs a, const uint64_t* __restrict__ counts,
                                                                 const uint32_t* __restrict__ tloc,
                                                                 const uint64_t* __restrict__ mask, CompactGrid g) {
    __shared__ uint32_t s_wtot[MQ_WAVES];
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    const uint64_t tile = blockIdx.x;
    const uint64_t run_of = tile / g.chunk;  // the test-pass block that owned this tile
    const uint64_t base = tile * CMP_TILE;
    const uint64_t mine = lane() < (uint32_t)CMP_IPT ? mask[tile * CMP_TILE_WORDS + w * CMP_IPT + lane()] : 0ull;
    uint32_t run = (uint32_t)__popcll(mine);
#pragma unroll
    for (int o = MQ_WAVE / 2; o > 0; o >>= 1) run += __shfl_xor(run, o);
    if (lane() == 0) s_wtot[w] = run;
    __syncthreads();
    uint32_t wex = 0, ttot = 0;
#pragma unroll
    for (int i = 0; i < MQ_WAVES; i++) {
        if ((uint32_t)i < w) wex += s_wtot[i];
        ttot += s_wtot[i];
    }
    if (ttot == 0) return;  // nothing kept here (most tiles of a selective scan)
    // rows kept before this tile: the runs before its run (counts holds their
    // exclusive prefix by now), then its offset within the run
    const uint64_t pos0 = counts[run_of] + tloc[tile];
    const uint64_t pos = pos0 + wex;
    if (run == 0) return;
    {
        // slot masks as wave-uniform values, and each lane's output row per slot
        uint64_t km[CMP_IPT];
        uint32_t rel[CMP_IPT];
        uint32_t acc = 0;
#pragma unroll
        for (int i = 0; i < CMP_IPT; i++) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine, i);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mine >> 32), i);
            km[i] = (uint64_t)hi << 32 | lo;
            rel[i] = acc + (uint32_t)__popcll(km[i] & lt);
            acc += (uint32_t)__popcll(km[i]);
        }
        // per column, every slot's gather is issued before any store, so a
        // sparse tile waits for one load latency per column, not one per slot
        for (int c = 0; c < a.nout; c++) {
            const int32_t* __restrict__ src = a.in[a.out_src[c]];
            int32_t* __restrict__ dst = a.out[c];
            int32_t v[CMP_IPT];
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) {
                const uint64_t idx = base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane());
                v[i] = (km[i] >> lane()) & 1ull ? src[idx] : 0;
            }
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++)
                if ((km[i] >> lane()) & 1ull && MQ_IN_BOUNDS(pos + rel[i], a.n)) dst[pos + rel[i]] = v[i];
        }
    }
}

// One launch for scans whose runs have at most CMP_FUSED_CHUNK tiles: block
// b (in the order blocks start, from a tile counter) tests the tiles of run
// b as the test pass does, keeping each tile's in-run offset and each wave's
// offset inside the tile in LDS; wave 0 publishes the run's kept count and
// looks back over the earlier runs for their total; then every wave writes
// the rows its own mask words mark (the words it stored itself, so no block
// barrier is needed between tiles).  A selective scan thus reads its tested
// columns once and touches only the tiles with kept rows a second time,
// from the same block, without a second launch over every tile.
constexpr uint32_t CMP_FUSED_CHUNK = 512;
// A run keeping at most this many rows lists them (record index by run
// position) in LDS during its test phase and writes them with the whole
// block after the look-back; larger runs walk their tiles' masks again.
constexpr uint32_t CMP_LIST = 2048;

// The first test's operands of one tile's row slots for the calling thread,
// from clamped indices and unconditionally (a load under a per-lane
// condition would wait for the one before it).
__device__ __forceinline__ void load_first_test(const int32_t* A, const int32_t* B, int32_t c0, uint64_t n,
                                                uint64_t base, uint32_t w, int32_t (&va)[CMP_IPT],
                                                int32_t (&vb)[CMP_IPT]) {
    // tile-relative 32-bit offsets from a wave-uniform base (base < n)
    const int32_t* Ab = A ? A + base : nullptr;
    const int32_t* Bb = B ? B + base : nullptr;
    const uint64_t left = n - 1 - base;
    const uint32_t lim = left < CMP_TILE ? (uint32_t)left : (uint32_t)(CMP_TILE - 1);
#pragma unroll
    for (int i = 0; i < CMP_IPT; i++) {
        const uint32_t off = min((w * CMP_IPT + i) * MQ_WAVE + lane(), lim);
        va[i] = Ab ? Ab[off] : 0;
        vb[i] = Bb ? Bb[off] : c0;
    }
}

// MULTI: the pattern has further equality tests after the first; PAIR: the
// first test compares two columns (else a column with a constant, or none)
template <bool MULTI, bool PAIR>
__global__ __launch_bounds__(MQ_BLOCK) void compact_fused_kernel(CompactArgs a, uint64_t* __restrict__ status,
                                                                 uint32_t* __restrict__ run_ctr,
                                                                 uint64_t* __restrict__ mask, CompactGrid g) {
    __shared__ uint32_t s_wtot[2][MQ_WAVES];
    __shared__ uint32_t s_tloc[CMP_FUSED_CHUNK];
    __shared__ uint32_t s_wofs[CMP_FUSED_CHUNK][MQ_WAVES];
    __shared__ uint32_t s_list[CMP_LIST];
    __shared__ uint32_t s_slot;
    __shared__ uint64_t s_pos;
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    const uint32_t run_id = next_tile(run_ctr, &s_slot);
    const uint64_t t0 = (uint64_t)run_id * g.chunk;
    const uint64_t t1 = t0 + g.chunk < g.ntiles ? t0 + g.chunk : g.ntiles;
    const int32_t* A0 = a.nterm > 0 ? a.in[a.term_a[0]] : nullptr;
    const int32_t* B0 = PAIR ? a.in[a.term_b[0]] : nullptr;
    const int32_t c0 = a.nterm > 0 ? a.term_c[0] : 0;
    uint32_t run_tot = 0;  // kept rows of the run's tiles so far (same in every thread)
    for (uint64_t tile = t0; tile < t1; tile++) {
        const uint64_t base = tile * CMP_TILE;
        // the kept rows of each 64-row slot as one ballot word (kept in
        // scalar registers: no per-row flags stay live)
        uint64_t km[CMP_IPT];
        if (base + CMP_TILE <= a.n) {
            // a whole tile: the wave's row slots are one base address plus
            // constant offsets, and a constant right side needs no loads
            const uint64_t wbase = base + (uint64_t)(w * CMP_IPT * MQ_WAVE) + lane();
            if (PAIR) {
                int32_t va[CMP_IPT], vb[CMP_IPT];
#pragma unroll
                for (int i = 0; i < CMP_IPT; i++) {
                    va[i] = A0[wbase + i * MQ_WAVE];
                    vb[i] = B0[wbase + i * MQ_WAVE];
                }
#pragma unroll
                for (int i = 0; i < CMP_IPT; i++) km[i] = __ballot(va[i] == vb[i]);
            } else if (A0) {
                int32_t va[CMP_IPT];
#pragma unroll
                for (int i = 0; i < CMP_IPT; i++) va[i] = A0[wbase + i * MQ_WAVE];
#pragma unroll
                for (int i = 0; i < CMP_IPT; i++) km[i] = __ballot(va[i] == c0);
            } else {
#pragma unroll
                for (int i = 0; i < CMP_IPT; i++) km[i] = ~0ull;
            }
        } else {
            int32_t va[CMP_IPT], vb[CMP_IPT];
            load_first_test(A0, B0, c0, a.n, base, w, va, vb);
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) {
                const uint64_t idx = base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane());
                km[i] = __ballot(idx < a.n && (!A0 || va[i] == vb[i]));
            }
        }
        // further tests read their columns for every row slot, like the first
        for (int t = 1; MULTI && t < a.nterm; t++) {
            int32_t va[CMP_IPT], vb[CMP_IPT];
            load_first_test(a.in[a.term_a[t]], a.term_b[t] >= 0 ? a.in[a.term_b[t]] : nullptr, a.term_c[t], a.n,
                            base, w, va, vb);
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) km[i] &= __ballot(va[i] == vb[i]);
        }
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < CMP_IPT; i++) run += (uint32_t)__popcll(km[i]);
        const uint64_t mine = pick_slot(km);
        if (lane() < (uint32_t)CMP_IPT) mask[tile * CMP_TILE_WORDS + w * CMP_IPT + lane()] = mine;
        // one barrier per tile: the wave totals alternate between two slots,
        // and no wave can be two barriers ahead of a reader
        const int sl = (int)(tile & 1);
        if (lane() == 0) s_wtot[sl][w] = run;
        __syncthreads();
        uint32_t ttot = 0, wex = 0;
#pragma unroll
        for (int i = 0; i < MQ_WAVES; i++) {
            if ((uint32_t)i < w) wex += s_wtot[sl][i];
            ttot += s_wtot[sl][i];
        }
        if (lane() == 0) s_wofs[tile - t0][w] = wex;
        if (threadIdx.x == 0) s_tloc[tile - t0] = run_tot;
        // the kept rows' record indices by their position in the run
        if (run_tot + ttot <= CMP_LIST && run != 0) {
            uint32_t at = run_tot + wex;
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) {
                if ((km[i] >> lane()) & 1ull)
                    s_list[at + (uint32_t)__popcll(km[i] & lt)] =
                        (uint32_t)(base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane()));
                at += (uint32_t)__popcll(km[i]);
            }
        }
        run_tot += ttot;
    }
    __syncthreads();  // s_wofs, s_tloc and s_list complete
    if (w == 0) {
        const uint64_t ex = tile_prefix_wave0(status, run_id, 1u, run_tot);
        if (lane() == 0) {
            s_pos = ex;
            if (run_id == g.blocks - 1) *a.count = ex + run_tot;
        }
    }
    __syncthreads();
    if (run_tot == 0) return;
    const uint64_t pos_run = s_pos;
    if (run_tot <= CMP_LIST) {
        // every kept row of the run at once: consecutive threads, consecutive outputs
        for (uint32_t j = threadIdx.x; j < run_tot; j += MQ_BLOCK) {
            const uint32_t idx = s_list[j];
            if (!MQ_IN_BOUNDS(pos_run + j, a.n)) continue;
            for (int c = 0; c < a.nout; c++) a.out[c][pos_run + j] = a.in[a.out_src[c]][idx];
        }
        return;
    }
    for (uint64_t tile = t0; tile < t1; tile++) {
        const uint64_t mine = lane() < (uint32_t)CMP_IPT ? mask[tile * CMP_TILE_WORDS + w * CMP_IPT + lane()] : 0ull;
        if (__ballot(mine != 0ull) == 0ull) continue;  // none of this wave's rows kept here
        const uint64_t base = tile * CMP_TILE;
        const uint64_t pos = pos_run + s_tloc[tile - t0] + s_wofs[tile - t0][w];
        uint64_t km[CMP_IPT];
        uint32_t rel[CMP_IPT];
        uint32_t acc = 0;
#pragma unroll
        for (int i = 0; i < CMP_IPT; i++) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine, i);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mine >> 32), i);
            km[i] = (uint64_t)hi << 32 | lo;
            rel[i] = acc + (uint32_t)__popcll(km[i] & lt);
            acc += (uint32_t)__popcll(km[i]);
        }
        for (int c = 0; c < a.nout; c++) {
            const int32_t* __restrict__ src = a.in[a.out_src[c]];
            int32_t* __restrict__ dst = a.out[c];
            int32_t v[CMP_IPT];
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++) {
                const uint64_t idx = base + (uint64_t)((w * CMP_IPT + i) * MQ_WAVE + lane());
                v[i] = (km[i] >> lane()) & 1ull ? src[idx] : 0;
            }
#pragma unroll
            for (int i = 0; i < CMP_IPT; i++)
                if ((km[i] >> lane()) & 1ull && MQ_IN_BOUNDS(pos + rel[i], a.n)) dst[pos + rel[i]] = v[i];
        }
    }
}

size_t compact_scratch_words(uint64_t n) {
    const CompactGrid g = compact_grid(n);
    // run totals (u64 per run), in-run tile offsets (u32 per tile), the mask
    // words of whole tiles, then the fused kernel's run counter (one word)
    // and its look-back status words (one per run)
    return (size_t)(g.blocks + (g.ntiles + 1) / 2 + g.ntiles * CMP_TILE_WORDS + 1 + CMP_FUSED_BLOCKS);
}

hipError_t launch_compact(const CompactArgs& a, uint64_t* scratch, hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    const CompactGrid g = compact_grid(a.n);
    if (g.ntiles * MQ_BLOCK > 0xffffffffull) return hipErrorInvalidValue;  // grid size in work-items is 32-bit
    uint64_t* counts = scratch;
    uint32_t* tloc = reinterpret_cast<uint32_t*>(scratch + g.blocks);
    uint64_t* mask = scratch + g.blocks + (g.ntiles + 1) / 2;
    const CompactGrid gf = compact_grid_fused(a.n);
    if (gf.chunk <= CMP_FUSED_CHUNK) {
        uint64_t* ctr = mask + g.ntiles * CMP_TILE_WORDS;  // word 0: run counter; then status words
        hipError_t e = launch_fill_u64(ctr, 1 + gf.blocks, 0ull, stream);
        if (e != hipSuccess) return e;
        const bool multi = a.nterm > 1, pair = a.nterm > 0 && a.term_b[0] >= 0;
        auto* k = multi ? (pair ? compact_fused_kernel<true, true> : compact_fused_kernel<true, false>)
                        : (pair ? compact_fused_kernel<false, true> : compact_fused_kernel<false, false>);
        k<<<(uint32_t)gf.blocks, MQ_BLOCK, 0, stream>>>(a, ctr + 1, reinterpret_cast<uint32_t*>(ctr), mask, gf);
        return hipGetLastError();
    }
    compact_test_kernel<<<(uint32_t)g.blocks, MQ_BLOCK, 0, stream>>>(a, counts, tloc, mask, g);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan_runs(counts, (uint32_t)g.blocks, a.count, nullptr, nullptr, nullptr, stream);
    if (e != hipSuccess) return e;
    compact_write_kernel<<<(uint32_t)g.ntiles, MQ_BLOCK, 0, stream>>>(a, counts, tloc, mask, g);
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
