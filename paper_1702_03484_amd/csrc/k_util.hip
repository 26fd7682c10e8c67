// Small gfx950 utility kernels: fills, gathers, min/max, run boundaries,
// duplicate flags and ID checks used when a store is loaded and indexed.
#include "device_common.h"
#include "kernels.h"

namespace mq {

static uint32_t grid_for(uint64_t n, uint32_t per_block, uint32_t cap) {
    uint64_t b = (n + per_block - 1) / per_block;
    return (uint32_t)(b < 1 ? 1 : (b > cap ? cap : b));
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, uint64_t n, T v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

constexpr uint32_t SCAN_RUNS_MAX = 8 * 256;

__global__ __launch_bounds__(256) void scan_runs_kernel(uint64_t* __restrict__ tot, uint32_t nruns,
                                                        uint64_t* __restrict__ total64,
                                                        uint32_t* __restrict__ total32,
                                                        const uint64_t* __restrict__ run_max,
                                                        uint64_t* __restrict__ max_out) {
    __shared__ uint64_t tmp[MQ_WAVES];
    __shared__ uint64_t s_mx[MQ_WAVES];
    uint64_t v[8], sum = 0, mx = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const uint32_t i = threadIdx.x * 8 + k;
        v[k] = i < nruns ? tot[i] : 0ull;
        sum += v[k];
        if (run_max && i < nruns) mx = run_max[i] > mx ? run_max[i] : mx;
    }
    uint64_t all;
    uint64_t ex = block_excl_scan<uint64_t>(sum, tmp, &all);  // each total < 2^41: no overflow
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const uint32_t i = threadIdx.x * 8 + k;
        if (i < nruns) tot[i] = ex > SAT40 ? SAT40 : ex;
        ex += v[k];
    }
#pragma unroll
    for (int o = MQ_WAVE / 2; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(mx, o);
        mx = y > mx ? y : mx;
    }
    if (lane() == 0) s_mx[threadIdx.x / MQ_WAVE] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (total64) *total64 = all > SAT40 ? SAT40 : all;
        if (total32) *total32 = (uint32_t)all;
        if (run_max) {
            for (int i = 0; i < MQ_WAVES; i++) mx = s_mx[i] > mx ? s_mx[i] : mx;
            *max_out = mx;
        }
    }
}

hipError_t launch_scan_runs(uint64_t* tot, uint32_t nruns, uint64_t* total64, uint32_t* total32,
                            const uint64_t* run_max, uint64_t* max_out, hipStream_t stream) {
    if (nruns > SCAN_RUNS_MAX) return hipErrorInvalidValue;
    scan_runs_kernel<<<1, 256, 0, stream>>>(tot, nruns, total64, total32, run_max, max_out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    fill_kernel<uint32_t><<<grid_for(n, 256 * 4, 4096), 256, 0, stream>>>(p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    fill_kernel<uint64_t><<<grid_for(n, 256 * 4, 4096), 256, 0, stream>>>(p, n, v);
    return hipGetLastError();
}

__global__ void gather_kernel(const int32_t* __restrict__ src, const uint32_t* __restrict__ idx,
                              int32_t* __restrict__ out, uint64_t n, int32_t base) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = src[idx[i]] - base;
}
hipError_t launch_gather(const int32_t* src, const uint32_t* idx, int32_t* out, uint64_t n, int32_t base,
                         hipStream_t stream) {
    if (n == 0) return hipSuccess;
    gather_kernel<<<grid_for(n, 256 * 4, 8192), 256, 0, stream>>>(src, idx, out, n, base);
    return hipGetLastError();
}

// Composite key of up to MAX_KEY_WORDS columns packed into one word:
// OR over j of (col_j - base_j) << shift_j (the caller makes sure the
// relative ranges fit side by side in 32 bits; every shift is below 32).
__global__ void pack_keys_kernel(PackArgs a, uint64_t n, uint32_t* __restrict__ out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t k = 0;
        for (int j = 0; j < a.ncols; j++) k |= ((uint32_t)a.col[j][i] - (uint32_t)a.base[j]) << a.shift[j];
        out[i] = k;
    }
}
hipError_t launch_pack_keys(const PackArgs& a, uint64_t n, uint32_t* out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    if (a.ncols < 1 || a.ncols > MAX_KEY_WORDS) return hipErrorInvalidValue;
    for (int j = 0; j < a.ncols; j++)
        if (a.shift[j] < 0 || a.shift[j] > 31) return hipErrorInvalidValue;
    pack_keys_kernel<<<grid_for(n, 256 * 4, 8192), 256, 0, stream>>>(a, n, out);
    return hipGetLastError();
}

// Breaks between consecutive sorted records in the further words of a
// composite key: brk[i] = 1 when record ids[i] differs from record
// ids[i - 1] in any of the words (LEFT cells from lcol, RIGHT cells from
// rcol), else 0; brk[0] = 0.  Each wave shares its lanes' cells through
// shuffles; lane 0 loads its predecessor's.
__global__ __launch_bounds__(256) void key_breaks_kernel(BreakArgs a, const uint32_t* __restrict__ ids, uint32_t n,
                                                         uint8_t* __restrict__ brk) {
    const uint32_t stride = gridDim.x * blockDim.x;
    // every lane of a wave iterates together (the shuffles need all 64)
    const uint32_t n_up = (n + MQ_WAVE - 1) / MQ_WAVE * MQ_WAVE;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_up; i += stride) {
        const bool in = i < n;
        const uint32_t r = in ? ids[i] : 0u;
        bool diff = false;
        for (int j = 0; j < a.nw; j++) {
            const int32_t v = in ? (r < a.n_left ? a.lcol[j][r] : a.rcol[j][r - a.n_left]) : 0;
            int32_t pv = __shfl_up(v, 1, MQ_WAVE);
            if (lane() == 0 && in && i > 0) {
                const uint32_t q = ids[i - 1];
                pv = q < a.n_left ? a.lcol[j][q] : a.rcol[j][q - a.n_left];
            }
            diff |= v != pv;
        }
        if (in) brk[i] = (i > 0 && diff) ? 1 : 0;
    }
}
hipError_t launch_key_breaks(const BreakArgs& a, const uint32_t* ids, uint32_t n, uint8_t* brk, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    if (a.nw < 1 || a.nw > MAX_KEY_WORDS) return hipErrorInvalidValue;
    key_breaks_kernel<<<grid_for(n, 256 * 4, 8192), 256, 0, stream>>>(a, ids, n, brk);
    return hipGetLastError();
}

// One column of both sides in record order: out[i] = the cell of record
// ids[i] (a LEFT row when ids[i] < n_left, else RIGHT row ids[i] - n_left),
// relative to base.
__global__ void side_gather_kernel(const int32_t* __restrict__ lcol, const int32_t* __restrict__ rcol,
                                   uint32_t n_left, const uint32_t* __restrict__ ids, uint32_t n, int32_t base,
                                   uint32_t* __restrict__ out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t r = ids[i];
        const int32_t v = r < n_left ? lcol[r] : rcol[r - n_left];
        out[i] = (uint32_t)v - (uint32_t)base;
    }
}
hipError_t launch_side_gather(const int32_t* lcol, const int32_t* rcol, uint32_t n_left, const uint32_t* ids,
                              uint32_t n, int32_t base, uint32_t* out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    side_gather_kernel<<<grid_for(n, 256 * 4, 8192), 256, 0, stream>>>(lcol, rcol, n_left, ids, n, base, out);
    return hipGetLastError();
}

// Min and max of a[0..na) and b[0..nb): 8 independent loads in flight per
// thread, a block-level reduction, then one atomic pair per block (atomics
// on one address serialise, so there are few blocks).
constexpr int MM_UNROLL = 8;
constexpr uint32_t MM_BLOCKS = 1024;

__global__ __launch_bounds__(256) void minmax_kernel(const int32_t* __restrict__ a, uint64_t na,
                                                     const int32_t* __restrict__ b, uint64_t nb,
                                                     int32_t* __restrict__ mm) {
    __shared__ int32_t s_lo[256 / MQ_WAVE], s_hi[256 / MQ_WAVE];
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    const uint64_t n = na + nb;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i0 < n; i0 += stride * MM_UNROLL) {
        int32_t v[MM_UNROLL];
        bool ok[MM_UNROLL];
#pragma unroll
        for (int u = 0; u < MM_UNROLL; u++) {
            const uint64_t i = i0 + (uint64_t)u * stride;
            ok[u] = i < n;
            v[u] = i < na ? a[i] : (ok[u] ? b[i - na] : 0);
        }
#pragma unroll
        for (int u = 0; u < MM_UNROLL; u++)
            if (ok[u]) {
                lo = min(lo, v[u]);
                hi = max(hi, v[u]);
            }
    }
#pragma unroll
    for (int o = MQ_WAVE / 2; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, MQ_WAVE));
        hi = max(hi, __shfl_xor(hi, o, MQ_WAVE));
    }
    if (mq::lane() == 0) {
        s_lo[threadIdx.x / MQ_WAVE] = lo;
        s_hi[threadIdx.x / MQ_WAVE] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / MQ_WAVE; w++) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}
hipError_t launch_minmax(const int32_t* a, uint64_t na, const int32_t* b, uint64_t nb, int32_t* minmax,
                         hipStream_t stream) {
    if (na + nb == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((na + nb + 255) / 256, MM_BLOCKS);
    minmax_kernel<<<blocks, 256, 0, stream>>>(a, na, b, nb, minmax);
    return hipGetLastError();
}

__global__ void run_bounds_kernel(const int32_t* __restrict__ v, uint64_t n, int32_t* __restrict__ out_val,
                                  int64_t* __restrict__ out_pos, uint32_t* __restrict__ count, uint32_t cap) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (i == 0 || v[i] != v[i - 1]) {
            uint32_t at = atomicAdd(count, 1u);
            if (at < cap) {
                out_val[at] = v[i];
                out_pos[at] = (int64_t)i;
            }
        }
    }
}
hipError_t launch_run_bounds(const int32_t* v, uint64_t n, int32_t* out_val, int64_t* out_pos, uint32_t* count,
                             uint32_t cap, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    run_bounds_kernel<<<grid_for(n, 256 * 8, 4096), 256, 0, stream>>>(v, n, out_val, out_pos, count, cap);
    return hipGetLastError();
}

__global__ void dup_flags_kernel(const int32_t* __restrict__ p, const int32_t* __restrict__ s,
                                 const int32_t* __restrict__ o, const uint32_t* __restrict__ perm, uint64_t n,
                                 int32_t* __restrict__ keep) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        bool first = i == 0 || p[i] != p[i - 1] || s[i] != s[i - 1] || o[i] != o[i - 1];
        keep[perm[i]] = first ? 1 : 0;
    }
}
hipError_t launch_dup_flags(const int32_t* p, const int32_t* s, const int32_t* o, const uint32_t* perm,
                            uint64_t n, int32_t* keep, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    dup_flags_kernel<<<grid_for(n, 256 * 8, 8192), 256, 0, stream>>>(p, s, o, perm, n, keep);
    return hipGetLastError();
}

__global__ void check_ids_kernel(const int32_t* __restrict__ a, uint64_t n, uint32_t* __restrict__ bad) {
    uint32_t c = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        int32_t v = a[i];
        c += (v < 0 || v == INT32_MAX) ? 1u : 0u;
    }
    c = wave_sum(c);
    if (mq::lane() == 0 && c) atomicAdd(bad, c);
}
hipError_t launch_check_ids(const int32_t* a, uint64_t n, uint32_t* bad, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    check_ids_kernel<<<grid_for(n, 256 * 16, 2048), 256, 0, stream>>>(a, n, bad);
    return hipGetLastError();
}

// Number of runs of equal values in x[lo, hi) (a sorted range): one per
// position i with i == lo or x[i] != x[i-1].  Adds the count to *out with one
// atomic per wave.
__global__ void count_runs_kernel(const int32_t* __restrict__ x, uint64_t lo, uint64_t hi,
                                  unsigned long long* __restrict__ out) {
    uint32_t c = 0;
    for (uint64_t i = lo + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < hi; i += (uint64_t)gridDim.x * blockDim.x)
        c += (i == lo || x[i] != x[i - 1]) ? 1u : 0u;
    c = wave_sum(c);
    if (mq::lane() == 0 && c) atomicAdd(out, (unsigned long long)c);
}
hipError_t launch_count_runs(const int32_t* x, uint64_t lo, uint64_t hi, unsigned long long* out,
                             hipStream_t stream) {
    if (hi <= lo) return hipSuccess;
    count_runs_kernel<<<grid_for(hi - lo, 256 * 16, 512), 256, 0, stream>>>(x, lo, hi, out);
    return hipGetLastError();
}

}  // namespace mq
