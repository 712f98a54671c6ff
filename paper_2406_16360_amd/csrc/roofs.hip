// Measured memory ceilings of the GPU for the benchmark's roofline report:
// the streaming HBM read rate, and the rate of independent random gathers of
// fixed-size records from tables of a given size.  A table that fits the L2
// (4 MB per XCD) or the memory-side cache (256 MB) is served from there; BVH
// traversal reads its ~30 MB of nodes and triangles this way, so its gather
// rate is compared with the table-size-matched ceiling, not with HBM.
// Measurement only: nothing in the renderer calls these.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>

namespace {

__global__ void k_stream_read(const float4 *__restrict__ src, uint64_t n, float *__restrict__ sink) {
    float acc = 0.0f;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float4 v = src[i];
        acc += v.x + v.y + v.z + v.w;
    }
    if (acc == 1.2345f) sink[blockIdx.x] = acc;   // keeps the loads; never true for the zero-filled source
}

__global__ void k_stream_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Each lane reads `per_lane` records at independent pseudo-random indices
// (xorshift32 per lane), every record as rec16 consecutive 16-byte loads.
__global__ void k_gather(const float4 *__restrict__ table, uint32_t nrec, int rec16, int per_lane,
                         float *__restrict__ sink) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x = gid * 2654435761u + 12345u;
    float acc = 0.0f;
    for (int i = 0; i < per_lane; ++i) {
        x ^= x << 13; x ^= x >> 17; x ^= x << 5;
        const uint64_t r = (uint64_t)(x % nrec) * (uint64_t)rec16;
        for (int q = 0; q < rec16; ++q) {
            const float4 v = table[r + q];
            acc += v.x + v.w;
        }
    }
    if (acc == 1.2345f) sink[gid] = acc;
}

int fail(const char *what, hipError_t e) {
    std::fprintf(stderr, "mrs_roofs: %s: %s\n", what, hipGetErrorString(e));
    return -1;
}
#define CK(x, what) do { hipError_t e_ = (x); if (e_ != hipSuccess) return fail(what, e_); } while (0)

}  // namespace

// Streaming read and copy rates (GB/s) over a `bytes` buffer (a multiple of
// 16), best of `reps` passes each.  Returns 0, or -1 on a HIP error.
extern "C" int mrs_roofs_stream(uint64_t bytes, int reps, double *read_gbps, double *copy_gbps) {
    if (!read_gbps || !copy_gbps || bytes < 16 || reps < 1) return -1;
    const uint64_t n = bytes / 16;
    float4 *a = nullptr, *b = nullptr;
    float *sink = nullptr;
    hipEvent_t e0, e1;
    CK(hipMalloc(&a, n * 16), "hipMalloc");
    CK(hipMalloc(&b, n * 16), "hipMalloc");
    CK(hipMalloc(&sink, 1 << 20), "hipMalloc");
    CK(hipMemset(a, 0, n * 16), "hipMemset");
    CK(hipEventCreate(&e0), "hipEventCreate");
    CK(hipEventCreate(&e1), "hipEventCreate");
    const unsigned grid = 256 * 32, block = 256;
    double best_r = 0.0, best_c = 0.0;
    for (int r = 0; r < reps + 1; ++r) {   // the first pass warms up
        float ms = 0.0f;
        CK(hipEventRecord(e0, nullptr), "hipEventRecord");
        k_stream_read<<<grid, block>>>(a, n, sink);
        CK(hipEventRecord(e1, nullptr), "hipEventRecord");
        CK(hipEventSynchronize(e1), "hipEventSynchronize");
        CK(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (r) best_r = std::max(best_r, (double)(n * 16) / (ms * 1e-3) / 1e9);
        CK(hipEventRecord(e0, nullptr), "hipEventRecord");
        k_stream_copy<<<grid, block>>>(a, b, n);
        CK(hipEventRecord(e1, nullptr), "hipEventRecord");
        CK(hipEventSynchronize(e1), "hipEventSynchronize");
        CK(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (r) best_c = std::max(best_c, (double)(2 * n * 16) / (ms * 1e-3) / 1e9);
    }
    *read_gbps = best_r;
    *copy_gbps = best_c;
    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
    (void)hipFree(a); (void)hipFree(b); (void)hipFree(sink);
    return 0;
}

// Random gathers of `record_bytes` records (16, 32, 48 or 64) from a table of
// `table_bytes`: the best rate over `reps` passes in GB/s of record bytes and
// in G records/s.  Returns 0, or -1 on bad sizes or a HIP error.
extern "C" int mrs_roofs_gather(uint64_t table_bytes, int record_bytes, int reps, double *gbps, double *grec_per_s) {
    if (!gbps || !grec_per_s || reps < 1 || record_bytes < 16 || record_bytes > 64 || record_bytes % 16) return -1;
    const int rec16 = record_bytes / 16;
    const uint64_t nrec64 = table_bytes / (uint64_t)record_bytes;
    if (nrec64 < 1 || nrec64 > 0xFFFFFFFFull) return -1;
    const uint32_t nrec = (uint32_t)nrec64;
    float4 *t = nullptr;
    float *sink = nullptr;
    hipEvent_t e0, e1;
    const unsigned grid = 256 * 32, block = 256;
    const int per_lane = 256;
    CK(hipMalloc(&t, (uint64_t)nrec * record_bytes), "hipMalloc");
    CK(hipMemset(t, 0, (uint64_t)nrec * record_bytes), "hipMemset");
    CK(hipMalloc(&sink, sizeof(float) * grid * block), "hipMalloc");
    CK(hipEventCreate(&e0), "hipEventCreate");
    CK(hipEventCreate(&e1), "hipEventCreate");
    double best = 0.0;
    for (int r = 0; r < reps + 1; ++r) {
        float ms = 0.0f;
        CK(hipEventRecord(e0, nullptr), "hipEventRecord");
        k_gather<<<grid, block>>>(t, nrec, rec16, per_lane, sink);
        CK(hipEventRecord(e1, nullptr), "hipEventRecord");
        CK(hipEventSynchronize(e1), "hipEventSynchronize");
        CK(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        const double recs = (double)grid * block * per_lane;
        if (r) best = std::max(best, recs / (ms * 1e-3));
    }
    *grec_per_s = best / 1e9;
    *gbps = best * record_bytes / 1e9;
    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
    (void)hipFree(t); (void)hipFree(sink);
    return 0;
}
