// BVH traversal for gfx950: closest hit and any hit over the traversal nodes
// (four 8-bit quantised child boxes per 64-byte node, a surface-area
// collapse of the binary tree), with the watertight
// ray-triangle test of Woop, Benthin and Wald (JCGT 2013): edges count as
// inside, only t > 0 hits, degenerate triangles never hit, equal t resolves
// to the lower original face id.
#pragma once
#include <climits>
#include "device.h"

namespace mrs {

struct RayPre {
    V3 o, inv;
    int kx, ky, kz;
    float Sx, Sy, Sz;
};

__device__ __forceinline__ float comp(V3 v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }

__device__ __forceinline__ RayPre ray_pre(V3 o, V3 d) {
    RayPre r;
    r.o = o;
    // zero components become tiny ones so the slab test never forms 0 * inf
    float dx = fabsf(d.x) > 1e-30f ? d.x : copysignf(1e-30f, d.x);
    float dy = fabsf(d.y) > 1e-30f ? d.y : copysignf(1e-30f, d.y);
    float dz = fabsf(d.z) > 1e-30f ? d.z : copysignf(1e-30f, d.z);
    r.inv = V3{1.0f / dx, 1.0f / dy, 1.0f / dz};
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    if (comp(d, kz) < 0.0f) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    float dkz = comp(d, kz);
    r.Sx = comp(d, kx) / dkz;
    r.Sy = comp(d, ky) / dkz;
    r.Sz = 1.0f / dkz;
    return r;
}

// slab test of one box against [0, tmax]; returns the entry distance
__device__ __forceinline__ bool slab(const RayPre &r, float lx, float hx, float ly, float hy, float lz, float hz,
                                     float tmax, float &tnear) {
    float t0x = (lx - r.o.x) * r.inv.x, t1x = (hx - r.o.x) * r.inv.x;
    float t0y = (ly - r.o.y) * r.inv.y, t1y = (hy - r.o.y) * r.inv.y;
    float t0z = (lz - r.o.z) * r.inv.z, t1z = (hz - r.o.z) * r.inv.z;
    float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    tnear = tn;
    return tn <= tf * 1.0000008f;
}

// watertight test; on a hit with 0 < t <= tmax returns t and barycentrics of v1, v2
__device__ __forceinline__ bool tri_test(const RayPre &r, V3 a, V3 b, V3 c, float tmax, float &t, float &b1, float &b2) {
    V3 A = a - r.o, B = b - r.o, C = c - r.o;
    float Az = comp(A, r.kz), Bz = comp(B, r.kz), Cz = comp(C, r.kz);
    float Ax = comp(A, r.kx) - r.Sx * Az, Ay = comp(A, r.ky) - r.Sy * Az;
    float Bx = comp(B, r.kx) - r.Sx * Bz, By = comp(B, r.ky) - r.Sy * Bz;
    float Cx = comp(C, r.kx) - r.Sx * Cz, Cy = comp(C, r.ky) - r.Sy * Cz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float T = U * (r.Sz * Az) + V * (r.Sz * Bz) + W * (r.Sz * Cz);
    float inv = 1.0f / det;
    float tt = T * inv;
    if (!(tt > 0.0f) || tt > tmax) return false;
    t = tt;
    b1 = V * inv;
    b2 = W * inv;
    return true;
}

struct Hit { float t, b1, b2; int leaf; int prim; };

// Visit counters for measurement builds (-DMRS_COUNT_VISITS): node fetches
// and triangle tests of closest-hit [0, 1] and any-hit [2, 3] traversals.
#ifdef MRS_COUNT_VISITS
__device__ unsigned long long g_visit_counts[4];
#define MRS_COUNT(k) atomicAdd(&g_visit_counts[(k)], 1ull)
#else
#define MRS_COUNT(k) ((void)0)
#endif

#ifndef MRS_LDS_STACK
#define MRS_LDS_STACK 16   // stack entries per thread kept in LDS
#endif
constexpr int kLdsStack = MRS_LDS_STACK;

// LDS bytes a traversal kernel needs per thread
constexpr int kLdsStackBytes = kLdsStack * 4;

// Traversal stack: the first kLdsStack entries live in LDS, one column per
// thread (entry i of thread t at [i * stride + t], so a wavefront touches
// consecutive words); deeper entries spill to a private array owned by the
// caller.  The array is kept out of this struct: a dynamically indexed member
// would put the whole struct, stack pointer included, in scratch memory, and
// every push and pop would then go through the memory pipeline.
constexpr int kSpillStack = kStackSize - kLdsStack;
struct TStack {
    int *ref;          // LDS column of node refs
    int *spill_ref;    // the caller's private int[kSpillStack]
    int stride;
    int sp = 0;
    // the build rejects trees deeper than the stack, so a full stack is never
    // reached; if it were, the entry is dropped rather than written out of bounds.
    // The LDS accesses are relaxed workgroup-scope atomics, which the compiler
    // cannot fold with the private spill access into one slower flat access.
    __device__ __forceinline__ void push(int x) {
        if (sp >= kStackSize) return;
        if (sp < kLdsStack) __hip_atomic_store(ref + sp * stride, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else spill_ref[sp - kLdsStack] = x;
        ++sp;
    }
    __device__ __forceinline__ int pop() {
        --sp;
        if (sp < kLdsStack) return __hip_atomic_load(ref + sp * stride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return spill_ref[sp - kLdsStack];
    }
};

// per-thread view of the kernel's dynamic LDS (kLdsStackBytes * blockDim bytes)
__device__ __forceinline__ TStack make_stack(void *lds, int *spill) {
    TStack st;
    st.stride = blockDim.x;
    st.ref = (int *)lds + threadIdx.x;
    st.spill_ref = spill;
    return st;
}

__device__ __forceinline__ Hit no_hit() {
    Hit h;
    h.t = INFINITY; h.b1 = h.b2 = 0.0f; h.leaf = -1; h.prim = 0x7FFFFFFF;
    return h;
}

// Traversal state of a lane: the next node reference to process, >= 0 an
// inner node, another negative value a leaf, kNone once the ray is finished
// (kNone never encodes a leaf: a leaf holds at most kLeafMax triangles).
constexpr int kNone = INT_MIN;
static_assert(kLeafMax <= 7, "leaf references encode count - 1 in three bits");

// Inner-node visit of a traversal node (WideNode): tests its up to four
// child boxes against [0, tmax]; the nearest hit child is next, the other hit
// children are stacked farthest first; with no hit child the next reference
// comes off the stack.  A bound on axis a is o_a + q 2^e_a, so its slab
// distance is q (2^e_a / d_a) + (o_a - origin_a) / d_a: one fma per bound.
__device__ __forceinline__ void cswap(float &ta, int &ra, float &tb, int &rb) {
    const bool sw = tb < ta;
    const float t = sw ? tb : ta;
    const int r = sw ? rb : ra;
    tb = sw ? ta : tb; rb = sw ? ra : rb;
    ta = t; ra = r;
}
__device__ __forceinline__ float qbyte(uint32_t w, int c) { return (float)((w >> (8 * c)) & 0xFFu); }
template <bool kAny>
__device__ __forceinline__ int inner_step(const WideNode *__restrict__ nodes, const RayPre &r, float tmax, TStack &st,
                                          int node, int ctr) {
    const WideNode nd = nodes[node];
    MRS_COUNT(ctr);
    const uint32_t meta = __float_as_uint(nd.a.w);
    const int nc = (int)(meta >> 24);
    const float mx = __uint_as_float((meta & 0xFFu) << 23) * r.inv.x, bx = (nd.a.x - r.o.x) * r.inv.x;
    const float my = __uint_as_float(((meta >> 8) & 0xFFu) << 23) * r.inv.y, by = (nd.a.y - r.o.y) * r.inv.y;
    const float mz = __uint_as_float(((meta >> 16) & 0xFFu) << 23) * r.inv.z, bz = (nd.a.z - r.o.z) * r.inv.z;
    float t[4];
    int ref[4] = {(int)nd.r.z, (int)nd.r.w, (int)nd.s.x, (int)nd.s.y};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float t0x = fmaf(qbyte(nd.q.x, c), mx, bx), t1x = fmaf(qbyte(nd.q.y, c), mx, bx);
        const float t0y = fmaf(qbyte(nd.q.z, c), my, by), t1y = fmaf(qbyte(nd.q.w, c), my, by);
        const float t0z = fmaf(qbyte(nd.r.x, c), mz, bz), t1z = fmaf(qbyte(nd.r.y, c), mz, bz);
        const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
        const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
        t[c] = (c < nc && tn <= tf * 1.0000008f) ? tn : INFINITY;
    }
    if (kAny) {
        // any hit ends the ray: the members are stored largest first, so the
        // first hit one is next and the others are stacked to pop in member
        // order
        int next = kNone;
#pragma unroll
        for (int c = 3; c >= 0; --c) {
            if (t[c] == INFINITY) continue;
            if (next != kNone) st.push(next);
            next = ref[c];
        }
        if (next != kNone) return next;
        return st.sp > 0 ? st.pop() : kNone;
    }
    // ascending by entry distance (misses last)
    cswap(t[0], ref[0], t[1], ref[1]);
    cswap(t[2], ref[2], t[3], ref[3]);
    cswap(t[0], ref[0], t[2], ref[2]);
    cswap(t[1], ref[1], t[3], ref[3]);
    cswap(t[1], ref[1], t[2], ref[2]);
    if (t[0] == INFINITY) return st.sp > 0 ? st.pop() : kNone;
    if (t[3] != INFINITY) st.push(ref[3]);
    if (t[2] != INFINITY) st.push(ref[2]);
    if (t[1] != INFINITY) st.push(ref[1]);
    return ref[0];
}

// Leaf visit for the closest hit: all its triangles, then the next stacked
// reference.
__device__ __forceinline__ int closest_leaf(const TriRec *__restrict__ tris, const RayPre &r, Hit &h, TStack &st,
                                            int ref) {
    const int code = ~ref, first = code >> 3, cnt = (code & 7) + 1;
    for (int q = first; q < first + cnt; ++q) {
        TriRec tr3 = tris[q];
        MRS_COUNT(1);
        float t, b1, b2;
        int prim = __float_as_int(tr3.a.w);
        if (tri_test(r, xyz(tr3.a), xyz(tr3.b), xyz(tr3.c), h.t, t, b1, b2) && (t < h.t || prim < h.prim)) {
            h.t = t; h.b1 = b1; h.b2 = b2; h.leaf = q; h.prim = prim;
        }
    }
    return st.sp > 0 ? st.pop() : kNone;
}

// Leaf visit for any hit in (0, inf): finishes the ray on the first hit.
__device__ __forceinline__ int any_leaf(const TriRec *__restrict__ tris, const RayPre &r, TStack &st, int ref,
                                        bool &occl) {
    const int code = ~ref, first = code >> 3, cnt = (code & 7) + 1;
    for (int q = first; q < first + cnt; ++q) {
        TriRec tr3 = tris[q];
        MRS_COUNT(3);
        float t, b1, b2;
        if (tri_test(r, xyz(tr3.a), xyz(tr3.b), xyz(tr3.c), INFINITY, t, b1, b2)) { occl = true; return kNone; }
    }
    return st.sp > 0 ? st.pop() : kNone;
}

// lanes waiting at a leaf that start a leaf phase, for any-hit and for
// closest-hit traversal (closest-hit leaves cost more: their hits keep the
// ray going, so batching more of them pays)
#ifndef MRS_LEAF_BATCH
#define MRS_LEAF_BATCH 2
#endif
#ifndef MRS_LEAF_BATCH_CLOSEST
#define MRS_LEAF_BATCH_CLOSEST 8
#endif

// One traversal iteration of a wavefront (while-while traversal with
// postponed leaves, after Aila and Laine, HPG 2009).  A lane whose next
// reference is a leaf waits until at least the leaf batch of lanes of the
// wavefront are at a leaf, or none is at an inner node; then those lanes
// test their leaves together.  Lanes at an inner node then visit it.  `live`
// marks lanes with a ray; the closest-hit result (smallest t, ties to the
// lower face id) does not depend on the order of the visits.  Every lane
// that is in the calling loop must call this.
template <bool kAny>
__device__ __forceinline__ void trace_iter(const WideNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                           bool live, const RayPre &r, Hit &h, bool &occl, TStack &st, int &node) {
    const bool at_leaf = live && node < 0;
    const uint64_t leaves = __ballot(at_leaf), inner = __ballot(live && node >= 0);
    if (inner == 0 || __popcll(leaves) >= (kAny ? MRS_LEAF_BATCH : MRS_LEAF_BATCH_CLOSEST)) {
        if (at_leaf) node = kAny ? any_leaf(tris, r, st, node, occl) : closest_leaf(tris, r, h, st, node);
    }
    if (live && node >= 0) node = inner_step<kAny>(nodes, r, kAny ? INFINITY : h.t, st, node, kAny ? 2 : 0);
}

// One ray per lane, all lanes of the wavefront iterating together.
template <bool kAny>
__device__ __forceinline__ void trace_wave(const WideNode *__restrict__ nodes, const TriRec *__restrict__ tris, V3 o,
                                           V3 d, void *lds, Hit &h, bool &occl) {
    RayPre r = ray_pre(o, d);
    h = no_hit();
    occl = false;
    int spill[kSpillStack];
    TStack st = make_stack(lds, spill);
    int node = 0;
    while (__ballot(node != kNone) != 0) trace_iter<kAny>(nodes, tris, node != kNone, r, h, occl, st, node);
}

// closest hit: smallest t > 0, ties to the lower original face id
__device__ __forceinline__ Hit trace_closest(const WideNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                             V3 o, V3 d, void *lds) {
    Hit h;
    bool occl;
    trace_wave<false>(nodes, tris, o, d, lds, h, occl);
    return h;
}

// any hit in (0, inf): visibility of a shadow ray
__device__ __forceinline__ bool trace_any(const WideNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                          V3 o, V3 d, void *lds) {
    Hit h;
    bool occl;
    trace_wave<true>(nodes, tris, o, d, lds, h, occl);
    return occl;
}

#ifndef MRS_REFILL
#define MRS_REFILL 48      // idle lanes that trigger a refill of a wavefront
#endif

// Work partitions of a persistent traversal queue, each with its own claim
// counter on its own 128-byte line, so that claims do not serialise on one
// address.  kClaimWords u32 words per launch.
constexpr int kWorkParts = 64;
constexpr int kClaimStride = 32;
constexpr int kClaimWords = kWorkParts * kClaimStride;
static_assert(MRS_REFILL >= 1 && MRS_REFILL <= 64, "a refill needs between 1 and 64 idle lanes");
static_assert(kWorkParts == 64, "a wavefront reads the partition counters one per lane");
#ifndef MRS_SMALL_QUEUE
#define MRS_SMALL_QUEUE (1u << 19)
#endif
constexpr uint32_t kSmallQueue = MRS_SMALL_QUEUE;

// Persistent traversal of queue entries [0, n).  Each lane traces one ray at
// a time; once at least MRS_REFILL lanes of the wavefront have finished, the
// idle lanes claim the next unclaimed entries of the wavefront's current
// partition with one atomic per wavefront, so a wavefront runs until the
// queue is drained instead of as long as its slowest ray (ray replacement,
// after Aila and Laine, HPG 2009).  When its partition runs dry the wavefront
// moves on.  On a large queue it steps to the next partition and stops after
// seeing every one of them at its end.  On a small queue (at most
// kSmallQueue entries), where those steps, one atomic round trip each, would
// be most of the launch, it reads all partition counters at once (lane p
// reads partition p) and moves to the next partition with entries left, or
// stops when none has any.  Counters only grow, and a claim that reaches a
// partition's end has seen it drained for good, so either way a wavefront
// claims from at most kWorkParts drained partitions.  claim points at
// kClaimWords zeroed words.  load(i, o, d) fetches entry i's ray;
// done(i, hit, occluded) stores its result.  Every lane of the launch must
// call this (block sizes are multiples of 64).
// The next partition after `part` (cyclically) that still has unclaimed
// entries, or -1: lane p reads partition p's counter.  Kept out of line so
// that this rare step does not take registers from the traversal loop.
__device__ __attribute__((noinline)) int next_open_part(const uint32_t *claim, uint32_t n, int part) {
    const uint32_t lane = __lane_id();
    const uint64_t plo = (uint64_t)n * lane / kWorkParts, phi = (uint64_t)n * (lane + 1) / kWorkParts;
    const uint32_t c = __hip_atomic_load(claim + lane * kClaimStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t open = __ballot((int)lane != part && plo + c < phi);
    if (open == 0) return -1;
    const uint64_t after = part == kWorkParts - 1 ? 0ull : open & (~0ull << (part + 1));
    return __ffsll((long long)(after ? after : open)) - 1;
}

template <bool kAny, class Load, class Done>
__device__ __forceinline__ void persistent_trace(const WideNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                                 uint32_t n, uint32_t *claim, void *lds, Load load, Done done) {
    int spill[kSpillStack];
    TStack st = make_stack(lds, spill);
    RayPre r;
    Hit h = no_hit();
    bool occl = false;
    int node = kNone;
    int64_t item = -1;             // queue entry of this lane, -1 when idle
    const uint32_t lane = __lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // starting partition: blocks are dealt round-robin to the 8 XCDs, so
    // partition p is first worked on by the XCD p % 8
    const uint32_t wave = blockIdx.x / 8 * (blockDim.x / 64) + threadIdx.x / 64;
    int part = (int)(blockIdx.x % 8 + 8 * (wave % (kWorkParts / 8)));
    bool claiming = true;          // some partition may hold entries (wave-uniform)
    int seen = 0;                  // partition ends seen, stepping one partition at a time
    while (true) {
        if (claiming) {
            uint64_t idle = __ballot(item < 0);
            uint32_t nidle = (uint32_t)__popcll(idle);
            if (nidle >= MRS_REFILL) {
                const uint64_t lo = (uint64_t)n * part / kWorkParts, hi = (uint64_t)n * (part + 1) / kWorkParts;
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(claim + part * kClaimStride, nidle);
                base = __builtin_amdgcn_readfirstlane(base);
                if (lo + base + nidle >= hi) {
                    if (n <= kSmallQueue) {
                        part = next_open_part(claim, n, part);
                        claiming = part >= 0;
                    } else {
                        part = part + 1 == kWorkParts ? 0 : part + 1;
                        claiming = ++seen < kWorkParts;
                    }
                }
                if (item < 0) {
                    uint64_t idx = lo + base + (uint64_t)__popcll(idle & below);
                    if (idx < hi) {
                        V3 o, d;
                        load((uint32_t)idx, o, d);
                        r = ray_pre(o, d);
                        h = no_hit();
                        occl = false;
                        st.sp = 0;
                        node = 0;
                        item = (int64_t)idx;
                    }
                }
            }
        }
        if (__ballot(item >= 0) == 0 && !claiming) break;
        trace_iter<kAny>(nodes, tris, item >= 0, r, h, occl, st, node);
        if (item >= 0 && node == kNone) {
            done((uint32_t)item, h, occl);
            item = -1;
        }
    }
}

}  // namespace mrs
