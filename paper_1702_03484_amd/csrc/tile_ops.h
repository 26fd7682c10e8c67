// Per-tile bodies of the join kernels, shared by the one-join kernels
// (k_sort.hip, k_reduce.hip) and the batched ones (k_batch.hip).  A "tile"
// is a contiguous slice of one join's records; every function works on
// join-relative indexes and takes the first tile of its join, so that the
// decoupled look-back of a batched launch never crosses into another join.
#pragma once
#include "device_common.h"

namespace mq {

// ----------------------------------------------------------------- sort ---

template <int RB>
struct Radix {
    static constexpr int BUCKETS = 1 << RB;
    static constexpr uint32_t MASK = BUCKETS - 1;
    static constexpr int MAXP = (32 + RB - 1) / RB;
    static constexpr int BPT = (BUCKETS + MQ_BLOCK - 1) / MQ_BLOCK;  // buckets per thread
};

// NW waves per block (a tile is NW * 64 * KPT records)
template <int RB, int KPT, int NW = MQ_WAVES>
struct SortSmem {
    static constexpr int TILE = NW * MQ_WAVE * KPT;
    uint32_t keys[TILE];
    uint32_t vals[TILE];
    uint32_t wcnt[NW][Radix<RB>::BUCKETS];
    uint32_t local[Radix<RB>::BUCKETS];
    uint32_t goff[Radix<RB>::BUCKETS];
    uint32_t tmp[NW];
};

// Exclusive scan of the BUCKETS values in LDS `in` into LDS `out` (may
// alias), by wave 0 alone (lane L owns buckets L*PER ... L*PER + PER - 1),
// then one barrier: the other waves only wait once.
template <int RB>
__device__ __forceinline__ void scan_buckets(const uint32_t* in, uint32_t* out, uint32_t* tmp) {
    using R = Radix<RB>;
    constexpr int PER = (R::BUCKETS + MQ_WAVE - 1) / MQ_WAVE;
    (void)tmp;
    if (threadIdx.x < MQ_WAVE) {
        uint32_t loc[PER];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const uint32_t d = lane() * PER + k;
            loc[k] = d < (uint32_t)R::BUCKETS ? in[d] : 0u;
            sum += loc[k];
        }
        uint32_t ex = wave_incl_scan(sum) - sum;
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const uint32_t d = lane() * PER + k;
            if (d < (uint32_t)R::BUCKETS) out[d] = ex;
            ex += loc[k];
        }
    }
    __syncthreads();
}

// One stable radix pass over one tile whose records are already in
// registers (wave-striped: element i of a lane is tile position
// (wave*KPT + i)*64 + lane; positions >= valid_n are padding).  Ranks the
// digits, publishes the tile's digit counts, looks back over the join's
// earlier tiles, and scatters the tile to kout/vout (join-relative).
// `ghist` is the join's digit histogram of this pass; n_out the records of
// the output (checked in the bounds-checked build only).  Every thread of
// the block calls it.
template <int RB, int KPT, int NW = MQ_WAVES>
__device__ __forceinline__ void sort_tile(SortSmem<RB, KPT, NW>& sm, const uint32_t (&key)[KPT],
                                          const uint32_t (&val)[KPT], uint32_t valid_n, int shift,
                                          const uint32_t* __restrict__ ghist, uint64_t* __restrict__ status,
                                          uint32_t tile, uint32_t first_tile, uint32_t epoch,
                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                          uint32_t n_out) {
    using R = Radix<RB>;
    constexpr int NT = NW * MQ_WAVE;                       // threads of the block
    constexpr int BPT = (R::BUCKETS + NT - 1) / NT;        // buckets per thread
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint32_t ln = lane();
    for (int d = threadIdx.x; d < R::BUCKETS; d += NT) {
        sm.goff[d] = ghist[d];
#pragma unroll
        for (int i = 0; i < NW; i++) sm.wcnt[i][d] = 0;
    }
    __syncthreads();
    scan_buckets<RB>(sm.goff, sm.goff, sm.tmp);

    // stable rank within the wave, digit by digit through the wave counters
    // (ranks are below the tile size, 2^16: two per register)
    static_assert(NT * KPT <= 65536 && KPT % 2 == 0, "16-bit ranks");
    uint32_t rank2[KPT / 2];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < KPT; i++) {
        const uint32_t off = (w * KPT + i) * MQ_WAVE + ln;
        const bool ok = off < valid_n;
        const uint32_t dg = (key[i] >> shift) & R::MASK;
        // lanes whose digit differs in some bit: per bit, the ballot of
        // that bit xor this lane's bit spread over 64 bits (0 or all ones)
        uint32_t diff_lo = 0, diff_hi = 0;
#pragma unroll
        for (int b = 0; b < RB; b++) {
            const int32_t top = (int32_t)(dg << (31 - b));  // digit bit b in the sign bit
            const uint64_t m = __ballot(top < 0);
            const uint32_t spread = (uint32_t)(top >> 31);
            diff_lo |= (uint32_t)m ^ spread;
            diff_hi |= (uint32_t)(m >> 32) ^ spread;
        }
        const uint64_t peers = __ballot(ok) & ~((uint64_t)diff_hi << 32 | diff_lo);
        const uint32_t below = __popcll(peers & lt);
        const uint32_t old = ok ? sm.wcnt[w][dg] : 0u;
        if (ok && below == 0) sm.wcnt[w][dg] = old + (uint32_t)__popcll(peers);
        if (i % 2 == 0)
            rank2[i / 2] = old + below;
        else
            rank2[i / 2] |= (old + below) << 16;
    }
    __syncthreads();

    // per digit: exclusive prefix over waves, tile total, local digit starts
    uint32_t tot[BPT];
#pragma unroll
    for (int k = 0; k < BPT; k++) {
        const uint32_t d = threadIdx.x * BPT + k;
        uint32_t run = 0;
        if (d < (uint32_t)R::BUCKETS) {
#pragma unroll
            for (int i = 0; i < NW; i++) {
                const uint32_t c = sm.wcnt[i][d];
                sm.wcnt[i][d] = run;
                run += c;
            }
            sm.local[d] = run;
        }
        tot[k] = run;
    }
    __syncthreads();
    scan_buckets<RB>(sm.local, sm.local, sm.tmp);

    // publish this tile's digit totals, then look back for the prefix
    uint64_t* st = status + (uint64_t)tile * R::BUCKETS;
#pragma unroll
    for (int k = 0; k < BPT; k++) {
        const uint32_t d = threadIdx.x * BPT + k;
        if (d < (uint32_t)R::BUCKETS) st_store(st + d, st_pack(epoch, tile == first_tile ? ST_INC : ST_AGG, tot[k]));
    }
    if (tile > first_tile) {
#pragma unroll
        for (int k = 0; k < BPT; k++) {
            const uint32_t d = threadIdx.x * BPT + k;
            if (d < (uint32_t)R::BUCKETS) {
                const uint64_t ex = lookback(status + d, tile, first_tile, R::BUCKETS, epoch);
                st_store(st + d, st_pack(epoch, ST_INC, ex + tot[k]));
                sm.goff[d] += (uint32_t)ex;
            }
        }
    }
    // local scatter into LDS in digit order
#pragma unroll
    for (int i = 0; i < KPT; i++) {
        const uint32_t off = (w * KPT + i) * MQ_WAVE + ln;
        if (off < valid_n) {
            const uint32_t dg = (key[i] >> shift) & R::MASK;
            const uint32_t pos = sm.local[dg] + sm.wcnt[w][dg] + ((rank2[i / 2] >> (16 * (i % 2))) & 0xffffu);
            sm.keys[pos] = key[i];
            sm.vals[pos] = val[i];
        }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < valid_n; j += NT) {
        const uint32_t k = sm.keys[j];
        const uint32_t dg = (k >> shift) & R::MASK;
        const uint32_t g = sm.goff[dg] + (j - sm.local[dg]);
        if (MQ_IN_BOUNDS(g, n_out)) {
            kout[g] = k;
            vout[g] = sm.vals[j];
        }
    }
}

// ------------------------------------------------- segment heads/splits ---
// Within a key every LEFT record (payload < n_left) precedes every RIGHT
// one, so exactly one record of each segment writes its split: the first
// RIGHT record (split = its position), or, in a segment without RIGHT
// records, the last record (split = its position + 1).

struct HeadsSmem {
    uint32_t wtot[MQ_WAVES];
    uint64_t excl;
};

// One tile of IPT*256 records at join-relative positions base..; returns
// (in every thread) nothing; the tile's last-segment count goes to *nseg
// when `last_tile`.
template <int IPT>
__device__ __forceinline__ void heads_tile(HeadsSmem& sm, const uint32_t* __restrict__ keys,
                                           const uint32_t* __restrict__ vals, uint32_t n, uint32_t n_left,
                                           uint32_t base, uint32_t tile, uint32_t first_tile, bool last_tile,
                                           uint32_t* __restrict__ seg_start, uint32_t* __restrict__ seg_split,
                                           uint32_t* __restrict__ nseg, uint64_t* __restrict__ status,
                                           uint32_t epoch) {
    const uint32_t w = threadIdx.x / MQ_WAVE;
    const uint64_t lt = lanemask_lt();
    uint64_t hm[IPT];
    uint32_t wbits = 0, sbits = 0;  // per item: writes a split; is a first RIGHT record
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        const uint32_t idx = base + (w * IPT + i) * MQ_WAVE + lane();
        bool h = false;
        if (idx < n) {
            const uint32_t k = keys[idx];
            const bool is_r = vals[idx] >= n_left;
            h = idx == 0 || keys[idx - 1] != k;
            const bool last = idx + 1 == n || keys[idx + 1] != k;
            const bool first_r = is_r && (h || vals[idx - 1] < n_left);
            if (first_r || (last && !is_r)) wbits |= 1u << i;
            if (first_r) sbits |= 1u << i;
        }
        hm[i] = __ballot(h);
        run += (uint32_t)__popcll(hm[i]);
    }
    if (lane() == 0) sm.wtot[w] = run;
    __syncthreads();
    uint32_t wex = 0, ttot = 0;
#pragma unroll
    for (int i = 0; i < MQ_WAVES; i++) {
        if ((uint32_t)i < w) wex += sm.wtot[i];
        ttot += sm.wtot[i];
    }
    if (w == 0) {
        const uint64_t ex = tile_prefix_wave(status, tile, first_tile, epoch, ttot);
        if (lane() == 0) {
            sm.excl = ex;
            if (last_tile) *nseg = (uint32_t)(ex + ttot);
        }
    }
    __syncthreads();
    uint32_t pos = (uint32_t)sm.excl + wex;  // heads before item i's lane 0
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        const uint32_t idx = base + (w * IPT + i) * MQ_WAVE + lane();
        const bool h = (hm[i] >> lane()) & 1ull;
        const uint32_t before = pos + (uint32_t)__popcll(hm[i] & lt);  // heads before this record
        if (h && MQ_IN_BOUNDS(before, n)) seg_start[before] = idx;
        if ((wbits >> i) & 1u) {
            const uint32_t sid = h ? before : before - 1u;  // record 0 is always a head
            if (MQ_IN_BOUNDS(sid, n)) seg_split[sid] = ((sbits >> i) & 1u) ? idx : idx + 1;
        }
        pos += (uint32_t)__popcll(hm[i]);
    }
}

// ------------------------------------------------------ count and scan ---

struct CountSmem {
    uint64_t tmp[MQ_WAVES];
    uint64_t mx[MQ_WAVES];
    uint64_t excl;
};

// Segments base + t*IPT ... (blocked) of one join: count cL*cR, scan into
// exact offsets (saturating at 2^40-1); the join's last tile writes *total.
template <int IPT>
__device__ __forceinline__ void count_tile(CountSmem& sm, uint32_t n, uint32_t ns, uint32_t base, uint32_t tile,
                                           uint32_t first_tile, bool last_tile,
                                           const uint32_t* __restrict__ seg_start,
                                           const uint32_t* __restrict__ seg_split, uint64_t* __restrict__ seg_off,
                                           uint64_t* __restrict__ total, uint64_t* __restrict__ status,
                                           uint32_t epoch, uint64_t* __restrict__ max_pairs) {
    const uint32_t first = base + threadIdx.x * IPT;
    uint64_t cnt[IPT];
    uint64_t sum = 0, mx = 0;
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        const uint32_t s = first + i;
        cnt[i] = 0;
        if (s < ns) {
            const uint32_t st = seg_start[s];
            const uint32_t en = s + 1 < ns ? seg_start[s + 1] : n;
            const uint32_t sp = seg_split[s];
            const uint64_t c = (uint64_t)(sp - st) * (uint64_t)(en - sp);
            cnt[i] = c > SAT40 ? SAT40 : c;
        }
        sum += cnt[i];
        mx = cnt[i] > mx ? cnt[i] : mx;
    }
    // the tile's largest count raises the join's maximum (one atomic per tile)
#pragma unroll
    for (int o = MQ_WAVE / 2; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(mx, o);
        mx = y > mx ? y : mx;
    }
    if (lane() == 0) sm.mx[threadIdx.x / MQ_WAVE] = mx;
    uint64_t ttot;
    const uint64_t ex_in = block_excl_scan<uint64_t>(sum, sm.tmp, &ttot);
    if (threadIdx.x < MQ_WAVE) {
        const uint64_t ex = tile_prefix_wave(status, tile, first_tile, epoch, ttot);
        if (lane() == 0) {
            sm.excl = ex;
            if (last_tile) *total = sat_add(ex, ttot > SAT40 ? SAT40 : ttot);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && max_pairs) {
        uint64_t m = 0;
#pragma unroll
        for (int w = 0; w < MQ_WAVES; w++) m = sm.mx[w] > m ? sm.mx[w] : m;
        atomicMax(reinterpret_cast<unsigned long long*>(max_pairs), (unsigned long long)m);
    }
    uint64_t off = sm.excl + ex_in;
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        const uint32_t s = first + i;
        if (s < ns) seg_off[s] = off > SAT40 ? SAT40 : off;
        off += cnt[i];
    }
}

// --------------------------------------------------------- materialise ---
// Output row j of segment s (offset off[s]) is the pair (LEFT record li,
// RIGHT record ri) with r = j - off[s], li = r / cR, ri = r % cR.  A wave
// owns a chunk of 64*RPT consecutive rows and finds the chunk's segments with
// a 64-ary search (one coalesced probe and one __ballot per level); each
// lane owns RPT consecutive rows: one division, then increments, and
// 16-byte stores.

// last s in [lo, hi] with off[s] <= j; off is non-decreasing and off[lo] <= j.
// Wave-uniform arguments; every lane of the wave must call it.  near: the
// answer is likely within 64 of lo, so the 64 offsets from lo are probed
// first (one round trip when it is) before the 64-ary search of the rest.
__device__ __forceinline__ uint32_t wave_seg_of(const uint64_t* __restrict__ off, uint32_t lo, uint32_t hi,
                                                uint64_t j, bool near = false) {
    if (near && hi > lo) {
        const uint32_t pos = lo + lane();
        const bool ok = pos <= hi && off[pos] <= j;
        const uint64_t m = __ballot(ok);  // a prefix of lanes, lane 0 always set
        const uint32_t top = 63u - (uint32_t)__clzll(m);
        if (top < MQ_WAVE - 1 || hi - lo <= MQ_WAVE - 1) return lo + top;
        lo += MQ_WAVE - 1;  // off[lo + 63] <= j: the answer is at or past it
    }
    while (hi > lo) {
        const uint32_t step = (hi - lo + MQ_WAVE) / MQ_WAVE;  // ceil(span / 64)
        const uint32_t pos = lo + lane() * step;
        const bool ok = pos <= hi && off[pos] <= j;
        const uint64_t m = __ballot(ok);  // a prefix of lanes, lane 0 always set
        const uint32_t top = 63u - (uint32_t)__clzll(m);
        lo = lo + top * step;
        hi = min(hi, lo + step - 1);
    }
    return lo;
}

// last s in [lo, hi] with off[s] <= j (per lane)
__device__ __forceinline__ uint32_t seg_of(const uint64_t* __restrict__ off, uint32_t lo, uint32_t hi, uint64_t j) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr int MAT_MAXNC = 16;

// One join as seen by materialisation.  Output column c >= 1 takes its
// values from src[c] (a LEFT value column when c <= nl, else a RIGHT one),
// indexed by record id, or, when sorted_vals is set, from ssrc[c] indexed
// by sorted record position (values gathered into sorted order beforehand,
// or carried through the sort as the payload itself).
// Held by value and indexed only with compile-time column numbers, so the
// pointers stay in registers.
struct MatJoin {
    const uint32_t* keys;  // sorted relative keys
    const uint32_t* vals;  // sorted payloads (record ids unless values were carried)
    const uint32_t* seg_start;
    const uint32_t* seg_split;
    const uint64_t* seg_off;
    uint32_t ns, n, n_left;
    int32_t key_base;
    int32_t key_shift;  // 1: the side rides in the key's low bit
    int32_t nl, nr;
    bool sorted_vals;
    // merge-join segments: LEFT run [seg_start, + seg_cl) of the LEFT
    // table and RIGHT run [seg_split, + seg_cr) of the RIGHT table (null:
    // both runs lie in one sorted record sequence, ended by the next start)
    const uint32_t* seg_cl;
    const uint32_t* seg_cr;
    const int32_t* src[MAT_MAXNC];
    const int32_t* ssrc[MAT_MAXNC];
    int32_t* out[MAT_MAXNC];
};

// Pair order inside a segment.  The segment's cL x cR rows run over one
// side in the outer loop and the other in the inner loop; the inner side is
// the one whose value cells take fewer bytes (cL * nl against cR * nr, LEFT
// inner when strictly smaller), so the block that every outer step reads
// again is the smaller one and stays cached while the output streams out.
// Row r of the segment is (outer = r / c_inner, inner = r mod c_inner).
struct SegPos {
    uint32_t st, sp, cl, cr;  // LEFT run [st, sp), RIGHT run [sp, sp + cr)
    bool left_inner;
    uint32_t outer, inner;    // position of the current row
};

__device__ __forceinline__ bool left_inner_of(uint32_t cl, uint32_t cr, int nl, int nr) {
    return (uint64_t)cl * (uint32_t)nl < (uint64_t)cr * (uint32_t)nr;
}

// sorted positions of the current row's LEFT and RIGHT records
__device__ __forceinline__ uint32_t seg_lpos(const SegPos& p) { return p.st + (p.left_inner ? p.inner : p.outer); }
__device__ __forceinline__ uint32_t seg_rpos(const SegPos& p) { return p.sp + (p.left_inner ? p.outer : p.inner); }

__device__ __forceinline__ void seg_locate(SegPos& p, uint64_t r) {
    const uint32_t ci = p.left_inner ? p.cl : p.cr;
    if (r < 0xffffffffull) {
        p.outer = (uint32_t)r / ci;
        p.inner = (uint32_t)r - p.outer * ci;
    } else {
        p.outer = (uint32_t)(r / ci);
        p.inner = (uint32_t)(r - (uint64_t)p.outer * ci);
    }
}

__device__ __forceinline__ void seg_step(SegPos& p) {
    if (++p.inner == (p.left_inner ? p.cl : p.cr)) {
        p.inner = 0;
        p.outer++;
    }
}

template <int NC>
__device__ __forceinline__ void seg_open(const MatJoin& a, uint32_t s, int nl, int nr, SegPos& p) {
    p.st = a.seg_start[s];
    p.sp = a.seg_split[s];
    if (a.seg_cl) {
        p.cl = a.seg_cl[s];
        p.cr = a.seg_cr[s];
    } else {
        const uint32_t en = s + 1 < a.ns ? a.seg_start[s + 1] : a.n;
        p.cl = p.sp - p.st;
        p.cr = en - p.sp;
    }
    p.left_inner = left_inner_of(p.cl, p.cr, nl, nr);
}

// value cells of one row
template <int NC>
__device__ __forceinline__ void row_values(const MatJoin& a, int nl, int nc, uint32_t lpos, uint32_t rpos,
                                           int32_t (&v)[NC][4], int k) {
    if (a.sorted_vals) {
#pragma unroll
        for (int col = 1; col < NC; col++)
            if (col < nc) v[col][k] = a.ssrc[col][col <= nl ? lpos : rpos];
    } else {
        const uint32_t lrow = nl > 0 ? a.vals[lpos] : 0u;
        const uint32_t rrow = nc - 1 > nl ? a.vals[rpos] - a.n_left : 0u;
#pragma unroll
        for (int col = 1; col < NC; col++)
            if (col < nc) v[col][k] = a.src[col][col <= nl ? lrow : rrow];
    }
}

// Rows [j, j + nk) of one lane when they may lie in different segments (a
// sparse stretch of the output).  s is the segment of row j; each row's
// segment is found by its own binary search in [s, s_last] (empty segments
// are skipped, never walked), so the rows' searches and loads overlap.  The
// offsets are read from off[t] = seg_off[off0 + t]: the global array
// (off0 = 0), or a copy of the sub-chunk's range in LDS.
template <int NC, int NLC>
__device__ __forceinline__ void mat_rows_slow(const MatJoin& a, const uint64_t* off, uint32_t off0, uint32_t s,
                                              uint32_t s_last, uint64_t j, int nk, int32_t (&v)[NC][4]) {
    const int nl = NLC >= 0 ? NLC : a.nl, nr = NLC >= 0 ? NC - 1 - NLC : a.nr;
    const int nc = 1 + nl + nr;
    uint32_t sk[4];
#pragma unroll
    for (int k = 0; k < 4; k++) sk[k] = k == 0 || k >= nk ? s : seg_of(off, s - off0, s_last - off0, j + k) + off0;
    SegPos p[4];
#pragma unroll
    for (int k = 0; k < 4; k++) seg_open<NC>(a, sk[k], nl, nr, p[k]);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if (k < nk) {
            seg_locate(p[k], j + k - off[sk[k] - off0]);
            v[0][k] = (int32_t)((a.keys[p[k].st] >> a.key_shift) + (uint32_t)a.key_base);
            row_values<NC>(a, nl, nc, seg_lpos(p[k]), seg_rpos(p[k]), v, k);
        }
    }
}

// Rows [j, j + nk) of one lane, the segments of its sub-chunk staged in
// LDS: m_off[t] is segment (s + t)'s output offset and m_u holds its LEFT
// start, RIGHT start, LEFT count, RIGHT count and output key (MAT_LDS_META
// words apart), so a row needs one search in LDS and then only its value
// loads.
constexpr uint32_t MAT_LDS_META = 128;  // segments staged with their runs (28 B each)

template <int NC, int NLC>
__device__ __forceinline__ void mat_rows_meta(const MatJoin& a, const uint64_t* m_off, const uint32_t* m_u, uint32_t m,
                                              uint64_t j, int nk, int32_t (&v)[NC][4]) {
    const int nl = NLC >= 0 ? NLC : a.nl, nr = NLC >= 0 ? NC - 1 - NLC : a.nr;
    const int nc = 1 + nl + nr;
    uint32_t t[4];
#pragma unroll
    for (int k = 0; k < 4; k++) t[k] = k < nk ? seg_of(m_off, 0, m - 1, j + k) : 0u;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if (k < nk) {
            SegPos p;
            p.st = m_u[t[k]];
            p.sp = m_u[MAT_LDS_META + t[k]];
            p.cl = m_u[2 * MAT_LDS_META + t[k]];
            p.cr = m_u[3 * MAT_LDS_META + t[k]];
            p.left_inner = left_inner_of(p.cl, p.cr, nl, nr);
            seg_locate(p, j + k - m_off[t[k]]);
            v[0][k] = (int32_t)m_u[4 * MAT_LDS_META + t[k]];
            row_values<NC>(a, nl, nc, seg_lpos(p), seg_rpos(p), v, k);
        }
    }
}

// The segment of row j (the last s with seg_off[s] <= j), given a guess:
// the segment of an earlier row of the same wave, or 0.  When j still lies
// in the guess's segment or the next one, three independent loads settle
// it; otherwise a 64-ary search from the guess on.  Every lane of the wave
// calls it with the same arguments.
__device__ __forceinline__ uint32_t seg_from_hint(const MatJoin& a, uint32_t hint, uint64_t j) {
    const uint64_t o0 = a.seg_off[hint];
    const uint64_t o1 = hint + 1 < a.ns ? a.seg_off[hint + 1] : ~0ull;
    const uint64_t o2 = hint + 2 < a.ns ? a.seg_off[hint + 2] : ~0ull;
    if (o0 <= j) {
        if (j < o1) return hint;
        if (j < o2) return hint + 1;
    }
    return wave_seg_of(a.seg_off, o0 <= j ? hint : 0, a.ns - 1, j);
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Materialise output rows [j0, jend) (at most 64*RPT rows, j0 a multiple of
// 4) of one join with one wave.  The chunk is cut into sub-chunks of 256
// rows; in each, lane L writes rows 4L..4L+3, so every 16-byte store
// instruction of the wave covers 1 KB of one column contiguously.
//
// A sub-chunk that lies inside one segment (the common case: the output of a
// hot key spans many sub-chunks) takes the wave-uniform path: the segment,
// its pair order and the divide of the sub-chunk's first row into (outer,
// inner) are computed once for the wave (scalar registers); each lane then
// needs only its offset 4L past that row, whose quotient by the inner run
// length is one compare when the run has at least 256 rows and a small
// exact divide otherwise.  Sub-chunks that cross segment boundaries take
// mat_rows_slow per lane.  NC is an upper bound of the column count
// 1 + nl + nr; NLC >= 0 fixes nl = NLC and nr = NC - 1 - NLC at compile
// time.  `hint` carries the wave's current segment from chunk to chunk.
// Offsets of at most this many segments spanned by one 256-row sub-chunk are
// staged in the wave's slice of LDS before the per-lane searches.
constexpr uint32_t MAT_LDS_SEGS = 512;

template <int NC, int RPT, int NLC = -1>
__device__ __forceinline__ void mat_wave_chunk(const MatJoin& a, uint64_t j0, uint64_t jend, uint32_t& hint,
                                               uint64_t* lds, int qn = RPT / 4) {
    constexpr int Q = RPT / 4;  // sub-chunks of 256 rows per chunk; qn <= Q of them are used
    const int nl = NLC >= 0 ? NLC : a.nl, nr = NLC >= 0 ? NC - 1 - NLC : a.nr;
    const int nc = 1 + nl + nr;
    uint32_t s = uni(seg_from_hint(a, uni(hint), j0));
    {
        SegPos p;
        seg_open<NC>(a, s, nl, nr, p);
        const uint32_t st = uni(p.st), sp = uni(p.sp), cl = uni(p.cl), cr = uni(p.cr);
        const uint64_t off = uni64(a.seg_off[s]);
        const uint64_t send = off + (uint64_t)cl * cr;
        if (j0 + (uint64_t)qn * (4 * MQ_WAVE) <= (send < jend ? send : jend)) {
            // the whole chunk lies in segment s: one uniform divide, then
            // every lane's rows of all sub-chunks, all loads before any store
            const bool left_in = left_inner_of(cl, cr, nl, nr);
            const uint32_t ci = left_in ? cl : cr;
            const uint64_t r0 = j0 - off;
            uint32_t o0, i0;
            if (r0 <= 0xffffffffull) {
                o0 = uni((uint32_t)r0 / ci);
                i0 = uni((uint32_t)r0 - o0 * ci);
            } else {
                o0 = uni((uint32_t)(r0 / ci));
                i0 = uni((uint32_t)(r0 - (uint64_t)o0 * ci));
            }
            const int32_t key = (int32_t)((a.keys[st] >> a.key_shift) + (uint32_t)a.key_base);
            int32_t v[Q][NC][4];
#pragma unroll
            for (int q = 0; q < Q; q++) {
                if (q >= qn) break;
                // this lane's first row of sub-chunk q: offset t past (o0, i0)
                const uint32_t t = i0 + (uint32_t)q * (4 * MQ_WAVE) + 4u * lane();  // < ci + 64 * RPT
                uint32_t dq, inner;
                if (ci >= (uint32_t)(4 * MQ_WAVE * Q)) {
                    dq = t >= ci ? 1u : 0u;
                    inner = t - (dq ? ci : 0u);
                } else {
                    dq = t / ci;
                    inner = t - dq * ci;
                }
                uint32_t outer = o0 + dq;
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    v[q][0][k] = key;
                    row_values<NC>(a, nl, nc, st + (left_in ? inner : outer), sp + (left_in ? outer : inner), v[q], k);
                    if (++inner == ci) {
                        inner = 0;
                        outer++;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < Q; q++) {
                if (q >= qn) break;
                const uint64_t jl = j0 + (uint64_t)q * (4 * MQ_WAVE) + 4ull * lane();
                if (!MQ_IN_BOUNDS(jl + 3, jend)) continue;
#pragma unroll
                for (int col = 0; col < NC; col++)
                    if (col < nc)
                        *reinterpret_cast<int4*>(a.out[col] + jl) =
                            make_int4(v[q][col][0], v[q][col][1], v[q][col][2], v[q][col][3]);
            }
            hint = s;
            return;
        }
    }
    // the chunk crosses segment boundaries: sub-chunk by sub-chunk
#pragma unroll 1
    for (int q = 0; q < qn; q++) {
        const uint64_t jq = j0 + (uint64_t)q * (4 * MQ_WAVE);
        if (jq >= jend) break;
        s = uni(seg_from_hint(a, s, jq));
        SegPos p;
        seg_open<NC>(a, s, nl, nr, p);
        const uint32_t st = uni(p.st), sp = uni(p.sp), cl = uni(p.cl), cr = uni(p.cr);
        const uint64_t off = uni64(a.seg_off[s]);
        const uint64_t send = off + (uint64_t)cl * cr;
        const uint64_t jl = jq + 4ull * lane();
        int32_t v[NC][4];
        int nk = 4;
        if (jq + 4 * MQ_WAVE <= (send < jend ? send : jend)) {
            // wave-uniform: the whole sub-chunk lies in segment s
            const bool left_in = left_inner_of(cl, cr, nl, nr);
            const uint32_t ci = left_in ? cl : cr;
            const uint64_t r0 = jq - off;
            uint32_t o0, i0;
            if (r0 <= 0xffffffffull) {
                o0 = uni((uint32_t)r0 / ci);
                i0 = uni((uint32_t)r0 - o0 * ci);
            } else {
                o0 = uni((uint32_t)(r0 / ci));
                i0 = uni((uint32_t)(r0 - (uint64_t)o0 * ci));
            }
            const uint32_t t = i0 + 4u * lane();  // < ci + 256
            uint32_t dq, inner;
            if (ci >= 4 * MQ_WAVE) {
                dq = t >= ci ? 1u : 0u;
                inner = t - (dq ? ci : 0u);
            } else {
                dq = t / ci;  // t < 512
                inner = t - dq * ci;
            }
            uint32_t outer = o0 + dq;
            const int32_t key = (int32_t)((a.keys[st] >> a.key_shift) + (uint32_t)a.key_base);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t lpos = st + (left_in ? inner : outer);
                const uint32_t rpos = sp + (left_in ? outer : inner);
                v[0][k] = key;
                row_values<NC>(a, nl, nc, lpos, rpos, v, k);
                if (++inner == ci) {
                    inner = 0;
                    outer++;
                }
            }
        } else {
            // the sub-chunk's last segment (every lane takes part in the
            // search), then each lane's own segment and rows
            const uint64_t jlast = (jend < jq + 4 * MQ_WAVE ? jend : jq + 4 * MQ_WAVE) - 1;
            const uint32_t s_last = wave_seg_of(a.seg_off, s, a.ns - 1, jlast, true);
            const uint32_t m = s_last - s + 1;
            nk = jl < jend ? (int)min((uint64_t)4, jend - jl) : 0;
            if (lds && m <= MAT_LDS_META) {
                // few segments (mid-density keys): each one's offset, runs and
                // key staged once, coalesced, in the wave's LDS rows
                uint64_t* m_off = lds;
                uint32_t* m_u = reinterpret_cast<uint32_t*>(lds + MAT_LDS_META);
                __builtin_amdgcn_wave_barrier();  // earlier reads of these rows are done
                for (uint32_t t = lane(); t < m; t += MQ_WAVE) {
                    SegPos p;
                    seg_open<NC>(a, s + t, nl, nr, p);
                    m_off[t] = a.seg_off[s + t];
                    m_u[t] = p.st;
                    m_u[MAT_LDS_META + t] = p.sp;
                    m_u[2 * MAT_LDS_META + t] = p.cl;
                    m_u[3 * MAT_LDS_META + t] = p.cr;
                    m_u[4 * MAT_LDS_META + t] = (a.keys[p.st] >> a.key_shift) + (uint32_t)a.key_base;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (nk > 0) mat_rows_meta<NC, NLC>(a, m_off, m_u, m, jl, nk, v);
                goto store;
            }
            // many segments (a sparse stretch of the output): their offsets in
            // LDS, so that each lane's searches stay on chip
            const uint64_t* off = a.seg_off;
            uint32_t off0 = 0;
            if (lds && m > 2 && m <= MAT_LDS_SEGS) {
                __builtin_amdgcn_wave_barrier();
                for (uint32_t t = lane(); t < m; t += MQ_WAVE) lds[t] = a.seg_off[s + t];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                off = lds;
                off0 = s;
            }
            if (nk > 0)
                mat_rows_slow<NC, NLC>(a, off, off0, seg_of(off, s - off0, s_last - off0, jl) + off0, s_last, jl,
                                       nk, v);
        }
    store:
        if (nk > 0 && !MQ_IN_BOUNDS(jl + nk - 1, jend)) nk = 0;
        if (nk == 4) {
#pragma unroll
            for (int col = 0; col < NC; col++)
                if (col < nc) *reinterpret_cast<int4*>(a.out[col] + jl) = make_int4(v[col][0], v[col][1], v[col][2], v[col][3]);
        } else if (nk > 0) {
#pragma unroll
            for (int col = 0; col < NC; col++)
                if (col < nc)
#pragma unroll
                    for (int k = 0; k < 4; k++)
                        if (k < nk) a.out[col][jl + k] = v[col][k];
        }
    }
    hint = s;
}

// Segment-major materialisation of one group of 64 consecutive keys
// [64 * grp, 64 * grp + 64) for outputs whose key products are small: the
// group's starts, splits, offsets and output keys are loaded once,
// coalesced, into the wave's LDS rows; its rows (at most 64 times the
// largest product) go out lane-strided, each row finding its key by a
// binary search over the group's offsets, so consecutive lanes store
// consecutive rows.  row_end = |RS|.  lds: MAT_SEG_LDS_WORDS words of this
// wave's LDS.  Every lane of the wave calls it.
constexpr int MAT_SEG_LDS_WORDS = MQ_WAVE + 1 + 2 * MQ_WAVE;  // offsets, then 4 x 64 u32

template <int NC, int NLC>
__device__ __forceinline__ void mat_seg_group(const MatJoin& mj, uint32_t grp, uint64_t row_end, uint64_t* lds) {
    const int nl = NLC >= 0 ? NLC : mj.nl, nr = NLC >= 0 ? NC - 1 - NLC : mj.nr;
    const int nc = 1 + nl + nr;
    uint64_t* s_off = lds;
    uint32_t* s_st = reinterpret_cast<uint32_t*>(lds + MQ_WAVE + 1);
    uint32_t* s_sp = s_st + MQ_WAVE;
    uint32_t* s_en = s_sp + MQ_WAVE;
    int32_t* s_key = reinterpret_cast<int32_t*>(s_en + MQ_WAVE);
    const uint32_t ns = mj.ns;
    const uint32_t s0 = grp * MQ_WAVE;
    const uint32_t s = s0 + lane();
    const bool in = s < ns;
    const uint32_t st = in ? mj.seg_start[s] : mj.n;
    const uint32_t sp = in ? mj.seg_split[s] : mj.n;
    uint32_t en = __shfl_down(st, 1, MQ_WAVE);
    if (lane() == MQ_WAVE - 1 && s + 1 < ns) en = mj.seg_start[s + 1];
    if (s + 1 >= ns) en = mj.n;
    // keys past the end sit at the end of the output: no row finds them
    const uint64_t off = in ? mj.seg_off[s] : row_end;
    const uint64_t off_end = s0 + MQ_WAVE < ns ? mj.seg_off[s0 + MQ_WAVE] : row_end;
    const int32_t key = in ? (int32_t)((mj.keys[st] >> mj.key_shift) + (uint32_t)mj.key_base) : 0;
    __builtin_amdgcn_wave_barrier();  // the previous group's reads of these LDS rows are done
    s_off[lane()] = off;
    if (lane() == 0) s_off[MQ_WAVE] = off_end;
    s_st[lane()] = st;
    s_sp[lane()] = sp;
    s_en[lane()] = en;
    s_key[lane()] = key;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t off0 = s_off[0];
    const uint32_t rows = (uint32_t)(off_end - off0);
    for (uint32_t r = lane(); r < rows; r += MQ_WAVE) {
        const uint64_t j = off0 + r;
        // the last key of the group starting at or before row j (empty keys
        // share the next one's offset and lose the tie)
        uint32_t lo = 0, hi = MQ_WAVE - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= j) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t kst = s_st[lo], ksp = s_sp[lo], ken = s_en[lo];
        const uint32_t cl = ksp - kst, cr = ken - ksp;
        const bool left_in = left_inner_of(cl, cr, nl, nr);
        const uint32_t ci = left_in ? cl : cr;
        const uint32_t rr = (uint32_t)(j - s_off[lo]);  // below the key's product
        const uint32_t outer = rr / ci, inner = rr - outer * ci;
        const uint32_t lpos = kst + (left_in ? inner : outer);
        const uint32_t rpos = ksp + (left_in ? outer : inner);
        if (!MQ_IN_BOUNDS(j, row_end)) continue;
        mj.out[0][j] = s_key[lo];
        if (mj.sorted_vals) {
#pragma unroll
            for (int col = 1; col < NC; col++)
                if (col < nc) mj.out[col][j] = mj.ssrc[col][col <= nl ? lpos : rpos];
        } else {
            const uint32_t lrow = nl > 0 ? mj.vals[lpos] : 0u;
            const uint32_t rrow = nc - 1 > nl ? mj.vals[rpos] - mj.n_left : 0u;
#pragma unroll
            for (int col = 1; col < NC; col++)
                if (col < nc) mj.out[col][j] = mj.src[col][col <= nl ? lrow : rrow];
        }
    }
}

}  // namespace mq
