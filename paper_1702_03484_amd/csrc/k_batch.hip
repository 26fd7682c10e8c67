// Batched joins on gfx950: many independent joins of uneven sizes in one
// sequence of persistent launches (captured once as a hipGraph by the host).
// Each join's records occupy whole record tiles; a tile -> join table sends
// every tile to its join, each join's look-back stops at its own first tile,
// and a placement kernel lays the results out in one output region on the
// device, so no size travels to the host between launches.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"
#include "tile_ops.h"

namespace mq {

// Persistent grids are sized to one resident round of blocks on the 256 CUs
// (a block beyond it only starts when another ends): 4 blocks per CU for
// the kernels of up to 128 VGPRs, 5 for those of up to 96, 8 for the
// histogram's 48 (measured on the 512-join batch: 6% off the launch).
constexpr uint32_t BATCH_BLOCKS = 1024;
constexpr uint32_t BATCH_BLOCKS_5 = 1280;
constexpr uint32_t BATCH_BLOCKS_8 = 2048;
constexpr uint32_t BMAT_BLOCKS = 2048;
constexpr int BMAT_RPT = 8;
constexpr uint32_t BMAT_WROWS = MQ_WAVE * BMAT_RPT;

uint32_t batch_chunk_rows() { return BMAT_WROWS; }

// Relative key of record idx (< nl + nr) of a join: the column is selected
// per lane before one load, and callers clamp idx into range instead of
// branching, so a thread's loads are all in flight together.
__device__ __forceinline__ uint32_t bsrc_key(const BatchJoin& J, uint32_t idx) {
    const bool right = idx >= J.nl;
    const int32_t k = (right ? J.rkey : J.lkey)[right ? idx - J.nl : idx];
    return (uint32_t)k - (uint32_t)J.key_base;
}

// Semi-join reduction (a record whose key the other side lacks meets no
// partner in Reduce): a blocked Bloom filter per join holds the relative
// keys of one side; a key selects one 64-bit word of it and three bits in
// that word (a multiplicative hash finished by a xor-shift-multiply round),
// so a probe is one load.  It has no false negatives: a dropped record
// never had a partner, and the kept records keep their relative order, so
// every key that has partners on both sides yields the same runs, and the
// same rows in the same order, as without the filter.
__device__ __forceinline__ uint64_t bloom_hash(uint32_t k) {
    uint64_t x = (uint64_t)k * 0x9E3779B97F4A7C15ull;
    x ^= x >> 29;
    x *= 0xBF58476D1CE4E5B9ull;
    return x ^ (x >> 32);
}
__device__ __forceinline__ uint64_t bloom_bits(uint64_t x) {
    return (1ull << (x & 63)) | (1ull << ((x >> 6) & 63)) | (1ull << ((x >> 12) & 63));
}
__device__ __forceinline__ uint32_t bloom_word(uint64_t x, uint32_t fmask) { return (uint32_t)(x >> 32) & fmask; }

// Whether record idx (relative key k) of join J goes through the sort: the
// side the filter was built from always does, the probed side only when the
// filter may hold its key.
__device__ __forceinline__ bool bkeep(const BatchJoin& J, uint32_t idx, uint32_t k) {
    if (!J.filt || (idx >= J.nl) != (J.probe_right != 0)) return true;
    const uint64_t x = bloom_hash(k);
    const uint64_t m = bloom_bits(x);
    return (J.filt[bloom_word(x, J.fmask)] & m) == m;
}

template <int RB>
__global__ void bclear_kernel(const BatchHdr* __restrict__ h) {
    const uint64_t words = (uint64_t)h->njoins * h->passes * Radix<RB>::BUCKETS;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += stride) h->hist[i] = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < h->filt_words; i += stride) h->filt[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < h->passes + 4) h->ctr[threadIdx.x] = 0;
}

// Filters of the joins that have one: every record of the build side sets
// its key's bits (a word already holding them is left alone).
template <int KPT>
__global__ __launch_bounds__(MQ_BLOCK) void bfilt_kernel(const BatchHdr* __restrict__ h) {
    constexpr uint32_t TILE = MQ_BLOCK * KPT;
    for (uint32_t t = blockIdx.x; t < h->total_tiles; t += gridDim.x) {
        const BatchJoin& J = h->joins[h->tile_join[t]];
        if (!J.filt) continue;
        const uint32_t base = (t - J.tile_off) * TILE;
        // LEFT records [0, nl) build when RIGHT is probed, else RIGHT [nl, nl + nr)
        const uint32_t b0 = J.probe_right ? 0u : J.nl;
        const uint32_t b1 = J.probe_right ? J.nl : J.nl + J.nr;
        const uint32_t i0 = max(base, b0), i1 = min(base + TILE, b1);
        for (uint32_t i = i0 + threadIdx.x; i < i1; i += MQ_BLOCK) {
            const uint64_t x = bloom_hash(bsrc_key(J, i));
            const uint64_t m = bloom_bits(x);
            unsigned long long* wp = reinterpret_cast<unsigned long long*>(J.filt + bloom_word(x, J.fmask));
            if ((__hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & m) != m)
                atomicOr(wp, (unsigned long long)m);
        }
    }
}

// Semi-join compaction of the filtered joins: tile by tile in order (a tile
// counter), the records the filter keeps go, in input order, to the front
// of the join's region of the spare sort buffers as (relative key, record
// index), where the histogram and the first radix pass read them as a later
// pass reads its input.  A decoupled look-back over the join's tiles gives
// each tile its offset; the join's last tile writes the kept count.  (Packed
// densely first, the kept records fill the first pass's tiles: scattered
// straight from sparse tiles, each tile would put only a few records in
// each digit bucket and the pass's writes would break into partial lines.)
template <int KPT>
__global__ __launch_bounds__(MQ_BLOCK) void bcompact_kernel(const BatchHdr* __restrict__ h) {
    constexpr uint32_t TILE = MQ_BLOCK * KPT;
    __shared__ uint32_t s_wtot[MQ_WAVES];
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_tile;
    const uint32_t T = h->total_tiles, passes = h->passes;
    const uint32_t epoch = h->epoch0 + passes + 2;
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    for (;;) {
        const uint32_t t = next_tile(&h->ctr[passes + 2], &s_tile);
        if (t >= T) break;
        BatchJoin& J = h->joins[h->tile_join[t]];
        if (!J.filt) continue;  // block-uniform
        const uint32_t n = J.nl + J.nr;
        const uint32_t base = (t - J.tile_off) * TILE;
        uint32_t k[KPT];
#pragma unroll
        for (int i = 0; i < KPT; i++) k[i] = bsrc_key(J, min(base + (w * KPT + i) * MQ_WAVE + lane(), n - 1));
        uint64_t km[KPT];
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < KPT; i++) {
            const uint32_t idx = base + (w * KPT + i) * MQ_WAVE + lane();
            km[i] = __ballot(idx < n && bkeep(J, idx, k[i]));
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
            const uint64_t ex = tile_prefix_wave(h->status, t, J.tile_off, epoch, ttot);
            if (lane() == 0) {
                s_excl = ex;
                if (t - J.tile_off + 1 == J.ntiles) J.nrec = (uint32_t)(ex + ttot);
            }
        }
        __syncthreads();
        uint32_t pos = (uint32_t)s_excl + wex;
        uint32_t* ko = h->keys[1] + J.rec_off;
        uint32_t* vo = h->vals[1] + J.rec_off;
#pragma unroll
        for (int i = 0; i < KPT; i++) {
            if ((km[i] >> lane()) & 1ull) {
                const uint32_t at = pos + (uint32_t)__popcll(km[i] & lt);
                if (MQ_IN_BOUNDS(at, n)) {
                    ko[at] = k[i];
                    vo[at] = base + (w * KPT + i) * MQ_WAVE + lane();
                }
            }
            pos += (uint32_t)__popcll(km[i]);
        }
    }
}

// Per-join digit histograms of all passes over the records the sort takes:
// every record of an unfiltered join (read from the tables), the compacted
// kept records of a filtered one.  Block b takes a contiguous range of
// record tiles and flushes its LDS counts whenever the join changes.
template <int RB, int KPT>
__global__ __launch_bounds__(MQ_BLOCK) void bhist_kernel(const BatchHdr* __restrict__ h) {
    using R = Radix<RB>;
    constexpr uint32_t TILE = MQ_BLOCK * KPT;
    __shared__ uint32_t sh[R::MAXP * R::BUCKETS];
    const uint32_t T = h->total_tiles, passes = h->passes;
    const uint32_t t0 = (uint32_t)((uint64_t)blockIdx.x * T / gridDim.x);
    const uint32_t t1 = (uint32_t)((uint64_t)(blockIdx.x + 1) * T / gridDim.x);
    for (int i = threadIdx.x; i < R::MAXP * R::BUCKETS; i += MQ_BLOCK) sh[i] = 0;
    __syncthreads();
    int64_t cur = -1;
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t j = h->tile_join[t];
        if ((int64_t)j != cur) {
            if (cur >= 0) {
                __syncthreads();
                for (uint32_t i = threadIdx.x; i < passes * R::BUCKETS; i += MQ_BLOCK) {
                    const uint32_t c = sh[i];
                    if (c) atomicAdd(&h->hist[(uint64_t)cur * passes * R::BUCKETS + i], c);
                    sh[i] = 0;
                }
                __syncthreads();
            }
            cur = j;
        }
        const BatchJoin& J = h->joins[j];
        const bool packed = J.filt != nullptr;
        const uint32_t n = J.nrec;
        const uint32_t base = (t - J.tile_off) * TILE;
        if (base >= n) continue;  // past the kept records (block-uniform)
        const uint32_t* kc = h->keys[1] + J.rec_off;
        uint32_t k[KPT];
#pragma unroll
        for (int i = 0; i < KPT; i++) {
            const uint32_t idx = min(base + i * MQ_BLOCK + threadIdx.x, n - 1);
            k[i] = packed ? kc[idx] : bsrc_key(J, idx);
        }
#pragma unroll
        for (int i = 0; i < KPT; i++) {
            const uint32_t idx = base + i * MQ_BLOCK + threadIdx.x;
            if (idx < n)
                for (uint32_t p = 0; p < passes; p++) atomicAdd(&sh[p * R::BUCKETS + ((k[i] >> (p * RB)) & R::MASK)], 1u);
        }
    }
    __syncthreads();
    if (cur >= 0)
        for (uint32_t i = threadIdx.x; i < passes * R::BUCKETS; i += MQ_BLOCK) {
            const uint32_t c = sh[i];
            if (c) atomicAdd(&h->hist[(uint64_t)cur * passes * R::BUCKETS + i], c);
        }
}

// 16 keys per thread: at most 168 VGPRs (3 waves per SIMD instead of 2);
// 32: the 72 KB tile in LDS allows 2 blocks per CU, so up to 256 VGPRs
template <int RB, int KPT, bool GEN>
__global__ __launch_bounds__(MQ_BLOCK, KPT > 16 ? 2 : 3) void bpass_kernel(const BatchHdr* __restrict__ h, int pass) {
    using R = Radix<RB>;
    constexpr uint32_t TILE = MQ_BLOCK * KPT;
    __shared__ SortSmem<RB, KPT> sm;
    __shared__ uint32_t s_tile;
    const uint32_t T = h->total_tiles, passes = h->passes;
    const uint32_t epoch = h->epoch0 + pass;
    const int src = (pass - 1) & 1, dst = pass & 1;  // the first pass writes buffer 0
    const uint32_t w = threadIdx.x / MQ_WAVE;
    for (;;) {
        const uint32_t t = next_tile(&h->ctr[pass], &s_tile);
        if (t >= T) break;
        const uint32_t j = h->tile_join[t];
        const BatchJoin& J = h->joins[j];
        // the first pass of an unfiltered join reads its records from the
        // tables; every other pass (and the first one of a filtered join)
        // reads the sorted records of the previous one (the compacted kept
        // records), and the join's tiles past them have nothing to do (no
        // later tile of the join waits on them)
        const bool gen = GEN && !J.filt;
        const uint32_t n = J.nrec;
        const uint32_t base = (t - J.tile_off) * TILE;
        if (base >= n) continue;
        const uint32_t valid_n = min(TILE, n - base);
        uint32_t key[KPT], val[KPT];
        const uint32_t* kin = h->keys[src] + J.rec_off;
        const uint32_t* vin = h->vals[src] + J.rec_off;
#pragma unroll
        for (int i = 0; i < KPT; i++) {
            const uint32_t off = (w * KPT + i) * MQ_WAVE + lane();
            const uint32_t idx = base + off;
            const bool ok = off < valid_n;
            if (gen) {
                const uint32_t k = bsrc_key(J, min(idx, n - 1));
                key[i] = ok ? k : 0u;
                val[i] = idx;
            } else {
                key[i] = ok ? kin[idx] : 0u;
                val[i] = ok ? vin[idx] : 0u;
            }
        }
        sort_tile<RB, KPT>(sm, key, val, valid_n, pass * RB, h->hist + ((uint64_t)j * passes + pass) * R::BUCKETS,
                           h->status, t, J.tile_off, epoch, h->keys[dst] + J.rec_off, h->vals[dst] + J.rec_off, n);
    }
}

template <int KPT>
__global__ __launch_bounds__(MQ_BLOCK) void bheads_kernel(BatchHdr* __restrict__ h) {
    constexpr uint32_t TILE = MQ_BLOCK * KPT;
    __shared__ HeadsSmem sm;
    __shared__ uint32_t s_tile;
    const uint32_t T = h->total_tiles, passes = h->passes;
    const int fin = (passes - 1) & 1;
    const uint32_t epoch = h->epoch0 + passes;
    for (;;) {
        const uint32_t t = next_tile(&h->ctr[passes], &s_tile);
        if (t >= T) break;
        const uint32_t j = h->tile_join[t];
        BatchJoin& J = h->joins[j];
        const uint32_t lt = t - J.tile_off;
        const uint32_t n = J.nrec;
        if (lt * TILE >= n) continue;  // beyond the kept records (block-uniform)
        heads_tile<KPT>(sm, h->keys[fin] + J.rec_off, h->vals[fin] + J.rec_off, n, J.nl, lt * TILE, t, J.tile_off,
                        (lt + 1) * TILE >= n, h->keys[1 - fin] + J.rec_off, h->vals[1 - fin] + J.rec_off, &J.nseg,
                        h->status, epoch);
    }
}

template <int KPT>
__global__ __launch_bounds__(MQ_BLOCK) void bcount_kernel(BatchHdr* __restrict__ h) {
    constexpr uint32_t TILE = MQ_BLOCK * KPT;
    __shared__ CountSmem sm;
    __shared__ uint32_t s_tile;
    const uint32_t T = h->total_tiles, passes = h->passes;
    const int fin = (passes - 1) & 1;
    const uint32_t epoch = h->epoch0 + passes + 1;
    for (;;) {
        const uint32_t t = next_tile(&h->ctr[passes + 1], &s_tile);
        if (t >= T) break;
        const uint32_t j = h->tile_join[t];
        BatchJoin& J = h->joins[j];
        const uint32_t lt = t - J.tile_off;
        const uint32_t ns = J.nseg;
        if (lt * TILE >= ns) continue;  // beyond the join's segments (block-uniform)
        const uint32_t last = (ns + TILE - 1) / TILE - 1;
        count_tile<KPT>(sm, J.nrec, ns, lt * TILE, t, J.tile_off, lt == last, h->keys[1 - fin] + J.rec_off,
                        h->vals[1 - fin] + J.rec_off, h->seg_off + J.rec_off, &J.total, h->status, epoch,
                        &J.max_pairs);
    }
}

// One block: lay every join's result out in the output region (columns of a
// multiple of 64 rows, 256-byte aligned), flag joins that do not fit, and
// number the materialisation chunks.
__global__ __launch_bounds__(MQ_BLOCK) void bplace_kernel(BatchHdr* __restrict__ h) {
    __shared__ uint64_t s_tmp[MQ_WAVES];
    uint64_t run_words = 0, run_chunks = 0;
    const uint32_t nj = h->njoins;
    for (uint32_t b = 0; b < nj; b += MQ_BLOCK) {
        const uint32_t j = b + threadIdx.x;
        uint64_t words = 0, cw = 0, tot = 0;
        uint32_t st = 0, ns = 0;
        bool seg = false;
        int nc = 0;
        if (j < nj) {
            const BatchJoin& J = h->joins[j];
            tot = J.total;
            ns = J.nseg;
            seg = mat_seg_use(tot, ns, J.max_pairs);
            nc = 1 + J.nvl + J.nvr;
            if (tot >= SAT40) {
                st = 2;
            } else {
                cw = (tot + 63) / 64 * 64;
                words = cw * (uint64_t)nc;
            }
        }
        uint64_t wsum;
        const uint64_t wex = block_excl_scan<uint64_t>(words, s_tmp, &wsum);
        const uint64_t at = run_words + wex;
        if (st == 0 && at + words > h->out_cap_words) st = 1;
        // work items: groups of 64 keys (segment-major) or chunks of rows
        const uint64_t chunks = st != 0 ? 0 : (seg ? (ns + MQ_WAVE - 1) / MQ_WAVE : (tot + BMAT_WROWS - 1) / BMAT_WROWS);
        uint64_t csum;
        const uint64_t cex = block_excl_scan<uint64_t>(chunks, s_tmp, &csum);
        if (j < nj) {
            BatchJoin& J = h->joins[j];
            J.status = st;
            J.seg_major = seg ? 1u : 0u;
            J.out_word = at;
            J.col_words = cw;
            J.chunk_off = run_chunks + cex;
            for (int c = 0; c < BATCH_MAXNC; c++) J.out[c] = (st == 0 && c < nc) ? h->out_base + at + c * cw : nullptr;
        }
        run_words += wsum;
        run_chunks += csum;
    }
    if (threadIdx.x == 0) {
        h->out_used_words = run_words < h->out_cap_words ? run_words : h->out_cap_words;
        h->total_chunks = run_chunks;
    }
}

// last join j with chunk_off <= c (wave-uniform; every lane calls it)
__device__ __forceinline__ uint32_t wave_join_of(const BatchJoin* __restrict__ js, uint32_t nj, uint64_t c) {
    uint32_t lo = 0, hi = nj - 1;
    while (hi > lo) {
        const uint32_t step = (hi - lo + MQ_WAVE) / MQ_WAVE;
        const uint32_t pos = lo + lane() * step;
        const bool ok = pos <= hi && js[pos].chunk_off <= c;
        const uint64_t m = __ballot(ok);
        const uint32_t top = 63u - (uint32_t)__clzll(m);
        lo = lo + top * step;
        hi = min(hi, lo + step - 1);
    }
    return lo;
}

// A join whose output has at least as many rows as records reads each
// record's values many times: they move into sorted record order first
// (one pass over the sorted payloads), and materialisation reads them in
// place of the record-id gathers.
__device__ __forceinline__ bool bjoin_uses_sval(const BatchHdr* h, const BatchJoin& J) {
    const uint32_t nv = (uint32_t)max(J.nvl, J.nvr);
    return J.status == 0 && nv > 0 && nv <= h->nsval && J.total >= (uint64_t)J.nrec;
}

template <int KPT>
__global__ __launch_bounds__(MQ_BLOCK) void bgather_kernel(const BatchHdr* __restrict__ h) {
    constexpr uint32_t TILE = MQ_BLOCK * KPT;
    // work units of at most 4,096 records whatever the tile size (with
    // 8,192-record units the launch took 6.40 instead of 5.67 ms)
    constexpr uint32_t UNIT = TILE < 4096u ? TILE : 4096u;
    constexpr uint32_t UPT = TILE / UNIT;
    const int fin = (h->passes - 1) & 1;
    const uint32_t nu = h->total_tiles * UPT;
    for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
        const uint32_t t = u / UPT;
        const BatchJoin& J = h->joins[h->tile_join[t]];
        if (!bjoin_uses_sval(h, J)) continue;
        const uint32_t n = J.nrec;
        const uint32_t i0 = (t - J.tile_off) * TILE + (u % UPT) * UNIT;
        if (i0 >= n) continue;
        const uint32_t i1 = min(i0 + UNIT, n);
        const uint32_t* vals = h->vals[fin] + J.rec_off;
        for (uint32_t i = i0 + threadIdx.x; i < i1; i += MQ_BLOCK) {
            const uint32_t r = vals[i];
            if (!MQ_IN_BOUNDS(r, J.nl + J.nr)) continue;
            if (r < J.nl) {
                for (int c = 0; c < J.nvl; c++) h->sval[c][J.rec_off + i] = J.lcol[c][r];
            } else {
                for (int c = 0; c < J.nvr; c++) h->sval[c][J.rec_off + i] = J.rcol[c][r - J.nl];
            }
        }
    }
}

// Materialisation of every join of the batch: chunks strided over the
// waves, each chunk's join found by a 64-ary search over the joins.
static_assert(MAT_SEG_LDS_WORDS <= (int)MAT_LDS_SEGS, "a wave's LDS rows hold a key group");

// at most 128 VGPRs (4 waves per SIMD): a few spill, the gathers overlap more
__global__ __launch_bounds__(MQ_BLOCK, 4) void bmat_kernel(const BatchHdr* __restrict__ h) {
    __shared__ uint64_t s_segs[MQ_WAVES][MAT_LDS_SEGS];
    const uint64_t nchunks = h->total_chunks;
    const uint32_t passes = h->passes;
    const int fin = (passes - 1) & 1;
    const uint64_t gw = (uint64_t)blockIdx.x * MQ_WAVES + threadIdx.x / MQ_WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * MQ_WAVES;
    for (uint64_t c = gw; c < nchunks; c += nw) {
        const uint32_t j = wave_join_of(h->joins, h->njoins, c);
        const BatchJoin& J = h->joins[j];
        MatJoin mj;
        mj.keys = h->keys[fin] + J.rec_off;
        mj.vals = h->vals[fin] + J.rec_off;
        mj.seg_start = h->keys[1 - fin] + J.rec_off;
        mj.seg_split = h->vals[1 - fin] + J.rec_off;
        mj.seg_off = h->seg_off + J.rec_off;
        mj.ns = J.nseg;
        mj.n = J.nrec;
        mj.n_left = J.nl;
        mj.key_base = J.key_base;
        mj.key_shift = 0;
        mj.nl = J.nvl;
        mj.nr = J.nvr;
        mj.sorted_vals = bjoin_uses_sval(h, J);
        mj.seg_cl = nullptr;
        mj.seg_cr = nullptr;
#pragma unroll
        for (int col = 0; col < BATCH_MAXNC; col++) {
            mj.out[col] = J.out[col];
            if (col >= 1) {
                mj.src[col] = col <= J.nvl ? J.lcol[col - 1] : J.rcol[col - 1 - J.nvl];
                const int sc = col <= J.nvl ? col - 1 : col - 1 - J.nvl;
                mj.ssrc[col] = mj.sorted_vals && sc < (int)h->nsval ? h->sval[sc] + J.rec_off : nullptr;
            }
        }
        if (J.seg_major) {
            mat_seg_group<BATCH_MAXNC, -1>(mj, (uint32_t)(c - J.chunk_off), J.total, s_segs[threadIdx.x / MQ_WAVE]);
            continue;
        }
        const uint64_t j0 = (c - J.chunk_off) * BMAT_WROWS;
        uint32_t hint = 0;  // chunks of a wave may belong to different joins
        mat_wave_chunk<BATCH_MAXNC, BMAT_RPT>(mj, j0, min(j0 + BMAT_WROWS, J.total), hint,
                                              s_segs[threadIdx.x / MQ_WAVE]);
    }
}

template <int RB, int KPT>
static hipError_t launch_batch_t(const BatchHdr* hdr, int passes, hipStream_t stream) {
    BatchHdr* h = const_cast<BatchHdr*>(hdr);
    bclear_kernel<RB><<<256, MQ_BLOCK, 0, stream>>>(hdr);
    bfilt_kernel<KPT><<<BATCH_BLOCKS, MQ_BLOCK, 0, stream>>>(hdr);
    bcompact_kernel<KPT><<<BATCH_BLOCKS_5, MQ_BLOCK, 0, stream>>>(hdr);
    bhist_kernel<RB, KPT><<<BATCH_BLOCKS_8, MQ_BLOCK, 0, stream>>>(hdr);
    for (int p = 0; p < passes; p++) {
        if (p == 0) bpass_kernel<RB, KPT, true><<<BATCH_BLOCKS, MQ_BLOCK, 0, stream>>>(hdr, p);
        else bpass_kernel<RB, KPT, false><<<BATCH_BLOCKS, MQ_BLOCK, 0, stream>>>(hdr, p);
    }
    bheads_kernel<KPT><<<BATCH_BLOCKS_5, MQ_BLOCK, 0, stream>>>(h);
    bcount_kernel<KPT><<<BATCH_BLOCKS, MQ_BLOCK, 0, stream>>>(h);
    bplace_kernel<<<1, MQ_BLOCK, 0, stream>>>(h);
    bgather_kernel<KPT><<<BATCH_BLOCKS, MQ_BLOCK, 0, stream>>>(hdr);
    bmat_kernel<<<BMAT_BLOCKS, MQ_BLOCK, 0, stream>>>(hdr);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchHdr* hdr, int rb, int kpt, int passes, hipStream_t stream) {
#define MQ_B(B)                                                                                 \
    case B:                                                                                     \
        return kpt == 8    ? launch_batch_t<B, 8>(hdr, passes, stream)                          \
               : kpt == 16 ? launch_batch_t<B, 16>(hdr, passes, stream)                         \
                           : launch_batch_t<B, 32>(hdr, passes, stream);
    switch (rb) {
        MQ_B(4) MQ_B(5) MQ_B(6) MQ_B(7) MQ_B(8) MQ_B(9) MQ_B(10) MQ_B(11)
        default: return hipErrorInvalidValue;
    }
#undef MQ_B
}

}  // namespace mq
