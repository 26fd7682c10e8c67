// Host-side launchers of the gfx950 kernels (one translation unit per
// kernel family).  All launches are asynchronous on the given stream; a
// launcher returns the launch error, if any.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mq {

constexpr uint32_t BLOCK_THREADS = 256;  // threads per block of every tiled kernel

// ---- shuffle: LSD radix sort (k_sort.hip) --------------------------------
// Keys of a first pass come from two int32 segments (k0[0..n0) then
// k1[0..n1)), minus `base`; the payload is the position in that
// concatenation.
// First-pass source of a join's shuffle: the LEFT key column k0 (n0 rows)
// then the RIGHT one k1 (n1 rows), keys relative to base.  carry = 0: the
// payload is the record's position in that concatenation (RIGHT records
// from n0 on).  carry = 1: the payload is the record's value cell (v0 or v1;
// a side without a value column points at any column of its rows and its
// payloads go unused) and the key is (relative key << 1) | side, so LEFT
// records still sort ahead of RIGHT ones within a key.
struct SortSrc {
    const int32_t* k0;
    uint32_t n0;
    const int32_t* k1;
    uint32_t n1;
    int32_t base;
    const int32_t* v0;
    const int32_t* v1;
    int32_t carry;
};

// Merge join of two tables already sorted on the key (k_merge.hip).  One
// pass over the smaller side: at the head of each key run, the run's end is
// found by galloping and the key's run in the larger side by binary search;
// keys present on both sides become segments (ascending key), each with its
// LEFT run, RIGHT run and output offset; *nseg and *total get the counts.
struct MergeArgs {
    const int32_t* skey;   // smaller side's key column (sorted)
    uint32_t ns;
    const int32_t* bkey;   // larger side's key column (sorted)
    uint32_t nb;
    int32_t small_is_left;
    uint32_t* seg_lstart;
    uint32_t* seg_lcount;
    uint32_t* seg_rstart;
    uint32_t* seg_rcount;
    uint64_t* seg_off;
    uint32_t* nseg;
    uint64_t* total;
};
hipError_t launch_merge_segments(const MergeArgs& a, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch,
                                 hipStream_t stream);
uint32_t merge_tiles(uint32_t ns);

// Semi-join reduction (k_semi.hip).  Bits of keys - base are set in bm
// (range bits, cleared by the caller); the filter keeps the records of
// `keys` whose relative key is set, writing (relative key, id_base + index)
// in input order to kout/vout and the kept count to *count.
struct SemiArgs {
    const int32_t* keys;
    uint32_t n;
    int32_t base;
    uint64_t range;  // bits in bm
    const uint32_t* bm;
    uint32_t id_base;
    uint32_t* kout;
    uint32_t* vout;
    uint32_t* count;
};
hipError_t launch_bitmap_set(const int32_t* keys, uint32_t n, int32_t base, uint64_t range, uint32_t* bm,
                             hipStream_t stream);
hipError_t launch_semi_filter(const SemiArgs& a, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch,
                              hipStream_t stream);
uint32_t semi_filter_tiles(uint32_t n);
// Exact join size: cnt[k - base] += 1 over one side's keys (cnt cleared by
// the caller, range entries), then *total += sum of cnt[k - base] over the
// other side's keys (*total cleared by the caller).
hipError_t launch_key_count(const int32_t* keys, uint32_t n, int32_t base, uint64_t range, uint32_t* cnt,
                            hipStream_t stream);
hipError_t launch_key_dot(const int32_t* keys, uint32_t n, int32_t base, uint64_t range, const uint32_t* cnt,
                          uint64_t* total, hipStream_t stream);
// all n records of one side at kout/vout[(*at_dev or 0) + i]
hipError_t launch_side_records(const int32_t* keys, uint32_t n, int32_t base, uint32_t id_base,
                               const uint32_t* at_dev, uint32_t* kout, uint32_t* vout, hipStream_t stream);

// Digit histograms of `passes` passes into hist[passes][2^rb] (overwritten).
// keys == nullptr: read the keys from `src`.  `part` is scratch of
// radix_hist_part_words(rb, passes) words.
hipError_t launch_radix_hist(const SortSrc& src, const uint32_t* keys, uint32_t n, int rb, int passes,
                             uint32_t* part, uint32_t* hist, hipStream_t stream);
uint32_t radix_hist_part_words(int rb, int passes);
// One stable pass on digit `pass`.  kin == nullptr: first-pass mode from
// `src` (vin ignored).  hist_pass = this pass's histogram; status holds
// radix_tiles(n,kpt,rb,true) * 2^rb words; tile_ctr is zero before the launch.
hipError_t launch_radix_pass(int rb, int kpt, const SortSrc& src, const uint32_t* kin, const uint32_t* vin,
                             uint32_t* kout, uint32_t* vout, uint32_t n, int pass, const uint32_t* hist_pass,
                             uint64_t* status, uint32_t* tile_ctr, uint32_t epoch, hipStream_t stream);
// record tiles of a radix pass over n records (gen: the first pass, reading
// the input columns; its tiles are never larger than the other passes')
uint32_t radix_tiles(uint32_t n, int kpt, int rb, bool gen);

// ---- reduce (k_reduce.hip) -------------------------------------------------
// Segment heads of the sorted records: seg_start[s] = first position of the
// s-th distinct key, seg_split[s] = position of its first RIGHT record
// (payload >= n_left), or its end when it has none; *nseg = segments.
// scratch: seg_scratch_bytes(n) bytes of device memory shared by the two
// launches below (run totals and per-tile offsets; no clearing needed).
// side_bit: the side is the key's low bit (a carried shuffle) instead of
// payload >= n_left; segments then group keys >> 1.
// brk (may be null): one flag per sorted record, 1 where the further words
// of a composite key change (launch_key_breaks); segments then also start
// at every flagged record.
hipError_t launch_seg_heads(const uint32_t* keys, const uint32_t* vals, uint32_t n, uint32_t n_left,
                            int side_bit, uint32_t* seg_start, uint32_t* seg_split, uint32_t* nseg, void* scratch,
                            hipStream_t stream, const uint8_t* brk = nullptr);
// count[s] = (split - start) * (end - split); seg_off = exclusive scan of the
// counts (saturating at 2^40-1); *total = the full sum.  max_seg bounds the
// device count *nseg (sizes the grids).
// *max_pairs gets the largest single count.
hipError_t launch_seg_count(uint32_t n, const uint32_t* seg_start, const uint32_t* nseg, uint32_t max_seg,
                            const uint32_t* seg_split, uint64_t* seg_off, uint64_t* total, uint64_t* max_pairs,
                            void* scratch, hipStream_t stream);
size_t seg_scratch_bytes(uint32_t n);

// Value columns in sorted record order: for every record i, with
// r = vals[i], out[c][i] = lcol[c][r] (a LEFT record, r < n_left, c < nl) or
// rcol[c][r - n_left] (a RIGHT record, c < nr).
struct GatherArgs {
    const uint32_t* vals;
    uint32_t n, n_left;
    int32_t nl, nr;
    const int32_t* lcol[16];
    const int32_t* rcol[16];
    int32_t* out[16];
};
hipError_t launch_gather_values(const GatherArgs& g, hipStream_t stream);

struct MatArgs {
    const uint32_t* keys;      // sorted relative keys
    const uint32_t* vals;      // sorted payloads (record positions)
    const uint32_t* seg_start;
    const uint32_t* seg_split;
    const uint64_t* seg_off;
    const uint32_t* nseg;      // device count of segments
    uint32_t n;                // records
    uint32_t n_left;
    int32_t key_base;
    int32_t nl, nr;            // value columns of each side
    const int32_t* lcol[16];
    const int32_t* rcol[16];
    int32_t* out[16];          // 1 + nl + nr output columns
    uint64_t row_begin, row_end;  // materialise output rows [row_begin, row_end)
    const int32_t* sval[16];   // value columns in sorted record order (GatherArgs.out), if use_sval
    int32_t use_sval;
    // merge join (seg_cl != null): segment s pairs LEFT rows [seg_start[s],
    // + seg_cl[s]) of lcol with RIGHT rows [seg_split[s], + seg_cr[s]) of
    // rcol; keys is the LEFT key column (key_base 0); vals and sval unused
    const uint32_t* seg_cl;
    const uint32_t* seg_cr;
    // 1: one 256-row sub-chunk per wave (a sparse output: few rows per
    // segment, so the per-row searches want many waves); 0: the default
    int32_t sparse;
    // 1: keys carry the side in their low bit (output key = (key >> 1) + base)
    int32_t key_shift;
    // 1: segment-major writing (one wave per 64 keys; see mat_seg_use);
    // needs row_begin == 0, row_end == |RS| and seg_cl == null
    int32_t seg_major;
    uint32_t seg_count;  // host copy of *nseg (sizes the segment-major grid)
    uint32_t max_blocks; // grid cap of the launch (0: MAT_MAX_BLOCKS); waves stride over the work
};
constexpr uint32_t MAT_MAX_BLOCKS = 256 * 32;
// Segment-major materialisation pays for sparse outputs: fewer than
// MAT_SEG_ROWS_PER_SEG output rows per key on average and no key product
// above MAT_SEG_MAX_PAIRS, so a wave writes at most 4,096 rows.  With a few
// hundred rows per key, 64-key groups are too coarse a work item (a batch of
// such joins materialised 15% slower than with the row-chunk kernel).
constexpr uint64_t MAT_SEG_MAX_PAIRS = 64;
constexpr uint64_t MAT_SEG_ROWS_PER_SEG = 64;
__host__ __device__ inline bool mat_seg_use(uint64_t rows, uint64_t nseg, uint64_t max_pairs) {
    return rows < MAT_SEG_ROWS_PER_SEG * nseg && max_pairs <= MAT_SEG_MAX_PAIRS;
}
hipError_t launch_materialize(const MatArgs& a, hipStream_t stream);

// ---- map and filters (k_map.hip) -----------------------------------------
// Stream compaction of the rows of up to 16 int32 columns that pass every
// equality term; copies the selected columns.  A term compares column a
// with column b (b >= 0) or with constant c (b < 0).
struct CompactArgs {
    const int32_t* in[16];
    int32_t nin;
    uint64_t n;
    int32_t nterm;
    int32_t term_a[6];
    int32_t term_b[6];
    int32_t term_c[6];
    int32_t nout;
    int32_t out_src[16];
    int32_t* out[16];
    uint64_t* count;           // device: rows kept
};
// u64 words of device scratch launch_compact needs for n rows (block
// counts, then one mask word per 64 rows of whole tiles)
size_t compact_scratch_words(uint64_t n);
hipError_t launch_compact(const CompactArgs& a, uint64_t* scratch, hipStream_t stream);

// Range location in sorted columns: for query q, lo/hi start as the given
// range; level 1 narrows it to rows whose col1 value equals v1, level 2
// (if col2) narrows further to col2 == v2.  out[2q], out[2q+1] = result.
struct LocateQuery {
    const int32_t* col1;
    const int32_t* col2;
    int64_t lo, hi;
    int32_t v1, v2;
};
hipError_t launch_locate(const LocateQuery* q_dev, int32_t nq, int64_t* out, hipStream_t stream);

// ---- batched joins (k_batch.hip) -----------------------------------------
// Every size and pointer of a batch lives in device memory (BatchHdr and
// its BatchJoin array), so one captured graph serves every batch that uses
// the same digit width, tile size and pass count.
constexpr int BATCH_MAXNC = 8;  // output columns per batched join

struct BatchJoin {
    const int32_t* lkey;
    const int32_t* rkey;
    const int32_t* lcol[BATCH_MAXNC];
    const int32_t* rcol[BATCH_MAXNC];
    int32_t* out[BATCH_MAXNC];  // set on the device by the placement kernel
    uint32_t nl, nr;            // rows of each side
    uint32_t rec_off;           // first record slot (a multiple of the record tile)
    uint32_t tile_off, ntiles;  // record tiles [tile_off, tile_off + ntiles)
    int32_t key_base;
    int32_t nvl, nvr;           // value columns of each side
    // results (written on the device)
    uint32_t nseg;
    uint32_t status;            // 0 ok, 1 did not fit the output region, 2 over 2^40 rows
    uint64_t total;             // exact |RS| (saturating at 2^40 - 1)
    uint64_t out_word;          // word offset of column 0 in the output region
    uint64_t col_words;         // words per column (a multiple of 64)
    uint64_t chunk_off;         // first materialisation work item
    uint64_t max_pairs;         // largest key product (zero before the launch)
    uint32_t seg_major;         // work items are groups of 64 keys, not row chunks
    // Semi-join reduction: a blocked Bloom filter (fmask + 1 words, a power
    // of two) of the keys of one side; records of the other side (RIGHT when
    // probe_right, else LEFT) whose key it does not hold are dropped before
    // the sort.  filt = nullptr: every record is kept.
    uint64_t* filt;
    uint32_t fmask;
    uint32_t probe_right;
    uint32_t nrec;              // records sorted: nl + nr, or (filtered) the kept count, written on the device
};

struct BatchHdr {
    BatchJoin* joins;
    const uint32_t* tile_join;  // record tile -> join
    uint32_t njoins;
    uint32_t total_tiles;
    uint32_t passes;
    uint32_t epoch0;            // kernels use epoch0 .. epoch0 + passes + 1
    uint32_t* keys[2];
    uint32_t* vals[2];
    uint64_t* seg_off;
    uint32_t* hist;             // [njoins][passes][2^rb]
    uint32_t* ctr;              // tile counters: passes + 4 words, zero before the launch
    uint64_t* status;
    int32_t* out_base;          // output region
    uint64_t out_cap_words;
    uint64_t out_used_words;    // result
    uint64_t total_chunks;      // result
    // value columns in sorted record order (record slots as keys/vals), used
    // by joins with at least as many output rows as records; nsval = 0: none
    int32_t* sval[BATCH_MAXNC - 1];
    uint32_t nsval;
    uint64_t* filt;             // every join's filter words (cleared by the launch)
    uint64_t filt_words;
};

// The whole batch in kernel launches (a graph capture records them).
hipError_t launch_batch(const BatchHdr* hdr_dev, int rb, int kpt, int passes, hipStream_t stream);
// Rows per materialisation chunk of the batched kernels.
uint32_t batch_chunk_rows();

// ---- dictionary encoding of terms (k_dict.hip) ------------------------------
// The dictionary on the device: a hash table of 64-bit slots (mask + 1 of
// them, a power of two; ~0 = empty), and the terms in identifier order as
// bytes with nterms + 1 offsets.
struct DictDev {
    uint64_t* table;
    uint64_t mask;
    int64_t* off;
    uint8_t* bytes;
    uint32_t nterms;
};
// A batch of n terms: bytes[off[i] .. off[i + 1]) is term i.
struct TermsDev {
    const uint8_t* bytes;
    const int64_t* off;
    uint32_t n;
};
// Per-batch device scratch: u32 arrays of n (rep, first, flag, rank), u64
// arrays of n (blen, boff), scalars and the scan partials
// (scan_part_bytes(n)).  first must hold ~0 before the launch and err 0.
struct DictScratch {
    uint32_t *rep, *first, *flag, *rank;
    uint64_t *blen, *boff;
    uint32_t* new_terms;
    uint64_t* new_bytes;
    void* part;
    uint32_t* err;
};
constexpr uint32_t DICT_SCAN_MAX = 1u << 26;  // terms per batch
size_t scan_part_bytes(uint32_t n);
// err |= 1 unless off[0] == 0 and off is non-decreasing over n + 1 entries
hipError_t launch_dict_check_offsets(const int64_t* off, uint32_t n, uint32_t* err, hipStream_t s);
// hash and insert (insert = 0: look up only), then number the new terms:
// *new_terms, *new_bytes, rank and boff of their first occurrences
hipError_t launch_dict_encode_front(const DictDev& d, const TermsDev& t, int insert, DictScratch w, hipStream_t s);
// ids[i]: the identifier of term i (new terms: base + rank; absent: -1)
hipError_t launch_dict_ids(const TermsDev& t, DictScratch w, uint32_t base, int32_t* ids, hipStream_t s);
// commit = 1: append the new terms (identifiers from base, bytes from
// bbase) and re-point their slots; commit = 0: empty the slots the batch
// claimed, restoring the table
hipError_t launch_dict_commit(const DictDev& d, const TermsDev& t, DictScratch w, uint32_t base, int64_t bbase,
                              int commit, hipStream_t s);
// decoding: len[i] of each identifier (err |= 1 for one outside the
// dictionary), pos = their exclusive scan, *total = the sum
hipError_t launch_dict_decode(const DictDev& d, const int32_t* ids, uint32_t n, uint64_t* len, uint64_t* pos,
                              uint64_t* total, void* part, uint32_t* err, hipStream_t s);
hipError_t launch_dict_gather(const DictDev& d, const int32_t* ids, uint32_t n, const uint64_t* pos, uint8_t* out,
                              hipStream_t s);

// ---- utilities (k_util.hip) -----------------------------------------------
// Between the two passes of a two-pass scan: the run totals tot[0..nruns)
// (nruns <= 1024) become their exclusive prefix sums, in place, capped at
// 2^40 - 1; the sum goes to *total64 and/or *total32 (either may be null)
// and, when run_max is given, the largest of run_max[0..nruns) to *max_out.
hipError_t launch_scan_runs(uint64_t* tot, uint32_t nruns, uint64_t* total64, uint32_t* total32,
                            const uint64_t* run_max, uint64_t* max_out, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t stream);
// out[i] = src[idx[i]] - base
hipError_t launch_gather(const int32_t* src, const uint32_t* idx, int32_t* out, uint64_t n, int32_t base,
                         hipStream_t stream);
// Composite keys of up to MAX_KEY_WORDS variables.  Packed: out[i] = OR
// over j of (col[j][i] - base[j]) << shift[j] as u32 (the caller makes sure
// the relative ranges fit side by side; shifts in [0, 31]).
constexpr int MAX_KEY_WORDS = 3;
struct PackArgs {
    const int32_t* col[MAX_KEY_WORDS];
    int32_t base[MAX_KEY_WORDS];
    int32_t shift[MAX_KEY_WORDS];
    int32_t ncols;
};
hipError_t launch_pack_keys(const PackArgs& a, uint64_t n, uint32_t* out, hipStream_t stream);
// Not packed: brk[i] = 1 when sorted record ids[i] differs from ids[i - 1]
// in any of the nw further key words (record r < n_left reads lcol[j][r],
// else rcol[j][r - n_left]); brk[0] = 0.
struct BreakArgs {
    const int32_t* lcol[MAX_KEY_WORDS];
    const int32_t* rcol[MAX_KEY_WORDS];
    uint32_t n_left;
    int32_t nw;
};
hipError_t launch_key_breaks(const BreakArgs& a, const uint32_t* ids, uint32_t n, uint8_t* brk, hipStream_t stream);
// out[i] = cell of record ids[i] minus base, the record being LEFT row
// ids[i] of lcol (ids[i] < n_left) or RIGHT row ids[i] - n_left of rcol.
hipError_t launch_side_gather(const int32_t* lcol, const int32_t* rcol, uint32_t n_left, const uint32_t* ids,
                              uint32_t n, int32_t base, uint32_t* out, hipStream_t stream);
// minmax[0] = min, minmax[1] = max over the int32 values of two segments
// (minmax pre-set to INT32_MAX / INT32_MIN by the caller).
hipError_t launch_minmax(const int32_t* a, uint64_t na, const int32_t* b, uint64_t nb, int32_t* minmax,
                         hipStream_t stream);
// Run boundaries of a sorted column: for every i with v[i] != v[i-1] (or
// i == 0) appends (v[i], i) to out_val/out_pos at atomicAdd(count).
hipError_t launch_run_bounds(const int32_t* v, uint64_t n, int32_t* out_val, int64_t* out_pos, uint32_t* count,
                             uint32_t cap, hipStream_t stream);
// Duplicate flags of the (p,s,o)-sorted store: keep[perm[i]] = 1 if triple
// i differs from triple i-1 (or i == 0), else 0.
hipError_t launch_dup_flags(const int32_t* p, const int32_t* s, const int32_t* o, const uint32_t* perm,
                            uint64_t n, int32_t* keep, hipStream_t stream);
// Runs of equal values in the sorted range x[lo, hi), added to *out.
hipError_t launch_count_runs(const int32_t* x, uint64_t lo, uint64_t hi, unsigned long long* out,
                             hipStream_t stream);
// IDs outside [0, 2^31-1): count into *bad.
hipError_t launch_check_ids(const int32_t* a, uint64_t n, uint32_t* bad, hipStream_t stream);

}  // namespace mq
