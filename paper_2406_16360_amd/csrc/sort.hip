// Stable LSD radix sort of (32-bit key, 32-bit value) pairs for gfx950: four
// passes of 8 key bits.  A pass
//   1. counts each tile's digits (k_sort_hist: tiles of kSortTile pairs),
//   2. turns the counts, digit-major over the tiles, into global offsets with
//      an exclusive scan (k_scan_tiles, k_scan_top, k_scan_out), and
//   3. ranks each tile's pairs by digit in their original order and writes
//      them out (k_sort_scatter): the tile is reordered in LDS first, so that
//      the pairs of one digit leave as one contiguous run.
// Ranks within a tile come from wavefront ballots over the digit bits (the
// lanes of a wavefront that hold the same digit) and per-wavefront counts in
// LDS, round by round in index order, so equal keys keep their order.
// Used by the field pull-back (its points in Morton order) and by the
// deterministic adjoint (its gradient pairs grouped by record).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "runtime.h"

namespace mrs {

namespace {

constexpr int kSortThreads = 256;                         // 4 wavefronts
constexpr int kSortRounds = 16;                           // pairs per thread and tile
constexpr int kSortTile = kSortThreads * kSortRounds;     // 4096 pairs
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kDigits = 256;
static_assert(kSortThreads == kDigits, "one thread per digit in the per-digit steps");

// digit counts of each tile, stored digit-major: hist[d * nb + tile]
__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const uint32_t *__restrict__ keys, uint32_t n, int shift,
                                                           uint32_t nb, uint32_t *__restrict__ hist) {
    __shared__ uint32_t cnt[kDigits];
    const uint32_t t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const uint64_t i = base + (uint64_t)r * kSortThreads + t;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kDigits - 1)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)t * nb + blockIdx.x] = cnt[t];
}

// exclusive scan of a uint32 array: tile sums, one block scanning them, the
// tile outputs (kScanItems consecutive entries per thread)
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

// in-place inclusive scan of sh[0 .. kScanThreads) by all threads of the block
__device__ __forceinline__ void block_scan(uint32_t *sh) {
    const int t = threadIdx.x;
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t u = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const uint32_t *__restrict__ a, uint64_t n,
                                                             uint32_t *__restrict__ part) {
    __shared__ uint32_t sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) v += a[base + q];
    sh[threadIdx.x] = v;
    __syncthreads();
    block_scan(sh);
    if (threadIdx.x == kScanThreads - 1) part[blockIdx.x] = sh[kScanThreads - 1];
}

__global__ void __launch_bounds__(kScanThreads) k_scan_top(uint32_t *__restrict__ part, uint32_t nparts) {
    __shared__ uint32_t sh[kScanThreads];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < nparts; c += kScanThreads) {
        const uint32_t i = c + threadIdx.x;
        const uint32_t v = i < nparts ? part[i] : 0u;
        sh[threadIdx.x] = v;
        __syncthreads();
        block_scan(sh);
        const uint32_t incl = sh[threadIdx.x], total = sh[kScanThreads - 1];
        if (i < nparts) part[i] = carry + incl - v;
        carry += total;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_out(uint32_t *__restrict__ a, uint64_t n,
                                                           const uint32_t *__restrict__ part) {
    __shared__ uint32_t sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) v += a[base + q];
    sh[threadIdx.x] = v;
    __syncthreads();
    block_scan(sh);
    uint32_t run = part[blockIdx.x] + sh[threadIdx.x] - v;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) {
            const uint32_t x = a[base + q];
            a[base + q] = run;
            run += x;
        }
}

// One tile: pairs i = base + r * kSortThreads + t for rounds r, so rounds in
// order and threads in order visit the pairs in index order.
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(const uint32_t *__restrict__ kin,
                                                              const uint32_t *__restrict__ vin,
                                                              uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                              uint32_t n, int shift, uint32_t nb,
                                                              const uint32_t *__restrict__ offs) {
    __shared__ uint32_t s_key[kSortTile], s_val[kSortTile];
    __shared__ uint32_t s_cnt[kDigits], s_start[kDigits], s_run[kDigits], s_glob[kDigits];
    __shared__ uint32_t s_wc[kSortWaves][kDigits];
    const uint32_t t = threadIdx.x, w = t / 64, lane = __lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    uint32_t key[kSortRounds], val[kSortRounds];
    s_cnt[t] = 0;
    s_run[t] = 0;
    for (int q = 0; q < kSortWaves; ++q) s_wc[q][t] = 0;
    s_glob[t] = offs[(uint64_t)t * nb + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const uint64_t i = base + (uint64_t)r * kSortThreads + t;
        key[r] = i < n ? kin[i] : 0u;
        val[r] = i < n ? vin[i] : 0u;
        if (i < n) atomicAdd(&s_cnt[(key[r] >> shift) & (kDigits - 1)], 1u);
    }
    __syncthreads();
    // the tile's digit starts: exclusive scan of s_cnt
    s_start[t] = s_cnt[t];
    __syncthreads();
    for (int off = 1; off < kDigits; off <<= 1) {
        const uint32_t u = t >= (uint32_t)off ? s_start[t - off] : 0u;
        __syncthreads();
        s_start[t] += u;
        __syncthreads();
    }
    s_start[t] -= s_cnt[t];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const bool valid = base + (uint64_t)r * kSortThreads + t < n;
        const uint32_t d = (key[r] >> shift) & (kDigits - 1);
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if (valid && rank == 0) s_wc[w][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t p = s_start[d] + s_run[d] + rank;
            for (uint32_t q = 0; q < w; ++q) p += s_wc[q][d];
            s_key[p] = key[r];
            s_val[p] = val[r];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int q = 0; q < kSortWaves; ++q) { add += s_wc[q][t]; s_wc[q][t] = 0; }
        s_run[t] += add;
        __syncthreads();
    }
    // runs of one digit leave together: LDS slot p of digit d goes to
    // offs(d, tile) + (p - start(d))
    const uint32_t cnt = n - base < (uint64_t)kSortTile ? (uint32_t)(n - base) : (uint32_t)kSortTile;
    for (uint32_t p = t; p < cnt; p += kSortThreads) {
        const uint32_t k = s_key[p], d = (k >> shift) & (kDigits - 1);
        const uint32_t o = s_glob[d] + (p - s_start[d]);
        kout[o] = k;
        vout[o] = s_val[p];
    }
}

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// scratch layout: keys and values of the odd passes, the digit counts, the
// scan's tile sums
struct SortTmp {
    size_t keys, vals, hist, part, total;
};
SortTmp sort_tmp_layout(size_t n) {
    const auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nb = std::max<size_t>(div_up(n, kSortTile), 1);
    const size_t nh = (size_t)kDigits * nb;
    SortTmp L;
    L.keys = 0;
    L.vals = al(sizeof(uint32_t) * n);
    L.hist = L.vals + al(sizeof(uint32_t) * n);
    L.part = L.hist + al(sizeof(uint32_t) * nh);
    L.total = L.part + al(sizeof(uint32_t) * std::max<size_t>(div_up(nh, kScanTile), 1));
    return L;
}

}  // namespace

size_t sort_pairs_tmp_bytes(size_t n) { return sort_tmp_layout(n).total; }

namespace {

mrs_status sort_pairs_raw(const uint32_t *keys_in, uint32_t *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                          size_t n, void *tmp, hipStream_t s) {
    const SortTmp L = sort_tmp_layout(n);
    char *base = (char *)tmp;
    uint32_t *tk = (uint32_t *)(base + L.keys), *tv = (uint32_t *)(base + L.vals);
    uint32_t *hist = (uint32_t *)(base + L.hist), *part = (uint32_t *)(base + L.part);
    const uint32_t nb = div_up(n, kSortTile);
    const uint64_t nh = (uint64_t)kDigits * nb;
    const uint32_t nparts = div_up(nh, kScanTile);
    // passes: in -> tmp -> out -> tmp -> out
    const uint32_t *src_k = keys_in, *src_v = vals_in;
    for (int pass = 0; pass < 4; ++pass) {
        uint32_t *dk = (pass % 2 == 0) ? tk : keys_out, *dv = (pass % 2 == 0) ? tv : vals_out;
        const int shift = 8 * pass;
        k_sort_hist<<<nb, kSortThreads, 0, s>>>(src_k, (uint32_t)n, shift, nb, hist);
        k_scan_tiles<<<nparts, kScanThreads, 0, s>>>(hist, nh, part);
        k_scan_top<<<1, kScanThreads, 0, s>>>(part, nparts);
        k_scan_out<<<nparts, kScanThreads, 0, s>>>(hist, nh, part);
        k_sort_scatter<<<nb, kSortThreads, 0, s>>>(src_k, src_v, dk, dv, (uint32_t)n, shift, nb, hist);
        src_k = dk;
        src_v = dv;
    }
    return hip_check(hipGetLastError(), "radix sort");
}

}  // namespace

mrs_status sort_pairs_u32(const uint32_t *keys_in, uint32_t *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                          size_t n, DevBuf &tmp, hipStream_t s) {
    if (n > 0x7FFFFFFFull) return fail(MRS_EOVERFLOW, "sort of more than 2^31 - 1 pairs");
    if (n == 0) return MRS_OK;
    mrs_status st = tmp.reserve(sort_tmp_layout(n).total);
    if (st != MRS_OK) return st;
    return sort_pairs_raw(keys_in, keys_out, vals_in, vals_out, n, tmp.p, s);
}

}  // namespace mrs

using namespace mrs;

extern "C" size_t mrs_sort_pairs_tmp_bytes(int64_t n) { return n > 0 ? sort_tmp_layout((size_t)n).total : 0; }

extern "C" mrs_status mrs_sort_pairs_u32(const uint32_t *d_keys_in, uint32_t *d_keys_out, const uint32_t *d_vals_in,
                                         uint32_t *d_vals_out, int64_t n, void *d_tmp, size_t tmp_bytes,
                                         void *stream) {
    clear_error();
    if (n < 0) return fail(MRS_EINVAL, "mrs_sort_pairs_u32: n < 0");
    if (n == 0) return MRS_OK;
    if (n > 0x7FFFFFFFll) return fail(MRS_EOVERFLOW, "mrs_sort_pairs_u32: more than 2^31 - 1 pairs");
    if (!d_keys_in || !d_keys_out || !d_vals_in || !d_vals_out || !d_tmp)
        return fail(MRS_EINVAL, "mrs_sort_pairs_u32: null buffer");
    if (d_keys_in == d_keys_out || d_vals_in == d_vals_out)
        return fail(MRS_EINVAL, "mrs_sort_pairs_u32: the outputs must not be the inputs");
    if (tmp_bytes < sort_tmp_layout((size_t)n).total)
        return fail(MRS_EINVAL, "mrs_sort_pairs_u32: %zu scratch bytes, %zu needed", tmp_bytes,
                    sort_tmp_layout((size_t)n).total);
    return sort_pairs_raw(d_keys_in, d_keys_out, d_vals_in, d_vals_out, (size_t)n, d_tmp, (hipStream_t)stream);
}
