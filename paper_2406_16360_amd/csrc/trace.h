// BVH traversal for gfx950: closest hit and any hit over the LBVH node
// layout (both child boxes per 64-byte node), with the watertight
// ray-triangle test of Woop, Benthin and Wald (JCGT 2013): edges count as
// inside, only t > 0 hits, degenerate triangles never hit, equal t resolves
// to the lower original face id.
#pragma once
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
#ifndef MRS_STACK_T
// 1: also keep each entry's box-entry distance, to skip it after a closer hit
// (doubles the LDS per thread, which cost more occupancy than it saved)
#define MRS_STACK_T 0
#endif
constexpr int kLdsStack = MRS_LDS_STACK;

// LDS bytes a traversal kernel needs per thread
constexpr int kLdsStackBytes = kLdsStack * (MRS_STACK_T ? 8 : 4);

// Traversal stack: the first kLdsStack entries live in LDS, one column per
// thread (entry i of thread t at [i * stride + t], so a wavefront touches
// consecutive words); deeper entries spill to a private array.
struct TStack {
    int *ref;          // LDS column of node refs
    float *tn;         // LDS column of entry distances (MRS_STACK_T)
    int stride;
    int sp = 0;
    int spill_ref[kStackSize - kLdsStack];
#if MRS_STACK_T
    float spill_t[kStackSize - kLdsStack];
#endif
    // the build rejects trees deeper than the stack, so a full stack is never
    // reached; if it were, the entry is dropped rather than written out of bounds
    __device__ __forceinline__ void push(int x, float t) {
        if (sp >= kStackSize) return;
        if (sp < kLdsStack) {
            ref[sp * stride] = x;
#if MRS_STACK_T
            tn[sp * stride] = t;
#endif
        } else {
            spill_ref[sp - kLdsStack] = x;
#if MRS_STACK_T
            spill_t[sp - kLdsStack] = t;
#endif
        }
        ++sp;
    }
    __device__ __forceinline__ int pop(float &t) {
        --sp;
        if (sp < kLdsStack) {
#if MRS_STACK_T
            t = tn[sp * stride];
#else
            t = 0.0f;
#endif
            return ref[sp * stride];
        }
#if MRS_STACK_T
        t = spill_t[sp - kLdsStack];
#else
        t = 0.0f;
#endif
        return spill_ref[sp - kLdsStack];
    }
};

// per-thread view of the kernel's dynamic LDS (kLdsStackBytes * blockDim bytes)
__device__ __forceinline__ TStack make_stack(void *lds) {
    TStack st;
    int *base = (int *)lds;
    st.stride = blockDim.x;
    st.ref = base + threadIdx.x;
    st.tn = (float *)(base + kLdsStack * blockDim.x) + threadIdx.x;
    return st;
}

// closest hit: smallest t > 0, ties to the lower original face id
__device__ __forceinline__ Hit trace_closest(const BvhNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                             V3 o, V3 d, void *lds) {
    constexpr int kNodeCtr = 0, kTriCtr = 1;
    RayPre r = ray_pre(o, d);
    Hit h;
    h.t = INFINITY; h.b1 = h.b2 = 0.0f; h.leaf = -1; h.prim = 0x7FFFFFFF;
    TStack st = make_stack(lds);
    int node = 0;
    while (true) {
        BvhNode nd = nodes[node];
        MRS_COUNT(kNodeCtr);
        float tl, tr;
        bool hl = slab(r, nd.n0.x, nd.n0.y, nd.n0.z, nd.n0.w, nd.n2.x, nd.n2.y, h.t, tl);
        bool hr = slab(r, nd.n1.x, nd.n1.y, nd.n1.z, nd.n1.w, nd.n2.z, nd.n2.w, h.t, tr);
        int refs[2] = {nd.n3.x, nd.n3.y};
        bool hits[2] = {hl, hr};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (hits[c] && refs[c] < 0) {
                int code = ~refs[c];
                int first = code >> 3, cnt = (code & 7) + 1;
                for (int q = first; q < first + cnt; ++q) {
                    TriRec tr3 = tris[q];
                    MRS_COUNT(kTriCtr);
                    float t, b1, b2;
                    int prim = __float_as_int(tr3.a.w);
                    if (tri_test(r, xyz(tr3.a), xyz(tr3.b), xyz(tr3.c), h.t, t, b1, b2) &&
                        (t < h.t || prim < h.prim)) {
                        h.t = t; h.b1 = b1; h.b2 = b2; h.leaf = q; h.prim = prim;
                    }
                }
                hits[c] = false;
            }
        }
        hl = hits[0]; hr = hits[1];
        if (hl && hr) {
            bool lfirst = tl <= tr;
            st.push(lfirst ? refs[1] : refs[0], lfirst ? tr : tl);
            node = lfirst ? refs[0] : refs[1];
            continue;
        }
        if (hl) { node = refs[0]; continue; }
        if (hr) { node = refs[1]; continue; }
        bool found = false;
        while (st.sp > 0) {
            float t;
            int n = st.pop(t);
            if (!MRS_STACK_T || t <= h.t * 1.0000008f) { node = n; found = true; break; }
        }
        if (!found) break;
    }
    return h;
}

// any hit in (0, inf): visibility of a shadow ray
__device__ __forceinline__ bool trace_any(const BvhNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                          V3 o, V3 d, void *lds) {
    constexpr int kNodeCtr = 2, kTriCtr = 3;
    RayPre r = ray_pre(o, d);
    TStack st = make_stack(lds);
    int node = 0;
    const float tmax = INFINITY;
    while (true) {
        BvhNode nd = nodes[node];
        MRS_COUNT(kNodeCtr);
        float tl, tr;
        bool hl = slab(r, nd.n0.x, nd.n0.y, nd.n0.z, nd.n0.w, nd.n2.x, nd.n2.y, tmax, tl);
        bool hr = slab(r, nd.n1.x, nd.n1.y, nd.n1.z, nd.n1.w, nd.n2.z, nd.n2.w, tmax, tr);
        int refs[2] = {nd.n3.x, nd.n3.y};
        bool hits[2] = {hl, hr};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (hits[c] && refs[c] < 0) {
                int code = ~refs[c];
                int first = code >> 3, cnt = (code & 7) + 1;
                for (int q = first; q < first + cnt; ++q) {
                    TriRec tr3 = tris[q];
                    MRS_COUNT(kTriCtr);
                    float t, b1, b2;
                    if (tri_test(r, xyz(tr3.a), xyz(tr3.b), xyz(tr3.c), tmax, t, b1, b2)) return true;
                }
                hits[c] = false;
            }
        }
        hl = hits[0]; hr = hits[1];
        if (hl && hr) {
            bool lfirst = tl <= tr;
            st.push(lfirst ? refs[1] : refs[0], 0.0f);
            node = lfirst ? refs[0] : refs[1];
            continue;
        }
        if (hl) { node = refs[0]; continue; }
        if (hr) { node = refs[1]; continue; }
        if (st.sp == 0) break;
        float t;
        node = st.pop(t);
    }
    return false;
}

}  // namespace mrs
