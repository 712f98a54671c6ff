// Host-side runtime pieces shared by the translation units of libmirres:
// thread-local error state, an owning device buffer, and the opaque objects
// handed out through the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mirres.h"

namespace mrs {

void clear_error();
mrs_status fail(mrs_status code, const char *fmt, ...);
mrs_status hip_check(hipError_t e, const char *what);

// Owning device allocation (hipMalloc / hipFree).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    mrs_status alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(MRS_ENOMEM, "hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
        }
        bytes = n;
        return MRS_OK;
    }
    // grow-only reallocation (contents are not preserved)
    mrs_status reserve(size_t n) { return (p && bytes >= n) ? MRS_OK : alloc(n); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return (T *)p; }
};

// Stable radix sort of n (32-bit key, 32-bit value) pairs by key on stream s
// (sort.hip); tmp holds the scratch space, sized by sort_pairs_tmp_bytes(n)
// (so a caller that reserves it first can run this under graph capture).
size_t sort_pairs_tmp_bytes(size_t n);
mrs_status sort_pairs_u32(const uint32_t *keys_in, uint32_t *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                          size_t n, DevBuf &tmp, hipStream_t s);

}  // namespace mrs

struct mrs_bvh {
    int32_t nf = 0, nv = 0, nnodes = 0, depth = 0;
    mrs::DevBuf nodes;   // BvhNode[nnodes]
    mrs::DevBuf tris;    // TriRec[nf], leaf order
    mrs::DevBuf faces;   // int32 [nf][3], validated copy used for shading
    // parent of every node slot ((slot << 1) | side, -1 at the root), unpadded
    // node boxes; for the refit, the node slots ordered by height (leaves 0, a
    // node one above its higher inner child) and the first position of each
    // height 1..H in that order (hstart[H + 1] = nnodes)
    mrs::DevBuf npar, nlo, nhi, horder;
    std::vector<int32_t> hstart;
    // traversal nodes (WideNode[nnodes], at the binary index of the node
    // they stand for), the traversal level each binary node heads (-1: none)
    // and each traversal node's members as binary node slots (int4)
    mrs::DevBuf wnodes, wlevel, wcut;
};

struct mrs_tape {
    int device = -1;          // device the buffers live on
    uint64_t samples = 0;     // S covered
    int32_t bounces = 0;
    uint64_t seed = 0;
    uint64_t signature = 0;   // hash of the views and sampling options it was recorded for
    mrs::DevBuf hit;          // float4 [B][S]: (b1, b2, leaf index, env texel)
    mrs::DevBuf y;            // float4 [B][S]: (y, W if the shadow ray was unoccluded else 0)
    mrs::DevBuf rr;           // float  [B][S]: continuation factor 1/q_rr (1 without roulette), 0 = path ended
    mrs::DevBuf fm;           // float4 [B][S], field mode only: the field's output at the hit
};
