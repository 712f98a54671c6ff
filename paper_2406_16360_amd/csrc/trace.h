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

// closest hit: smallest t > 0, ties to the lower original face id
__device__ __forceinline__ Hit trace_closest(const BvhNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                             V3 o, V3 d) {
    RayPre r = ray_pre(o, d);
    Hit h;
    h.t = INFINITY; h.b1 = h.b2 = 0.0f; h.leaf = -1; h.prim = 0x7FFFFFFF;
    int stack[kStackSize];
    float stackt[kStackSize];
    int sp = 0;
    int node = 0;
    while (true) {
        BvhNode nd = nodes[node];
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
            int nearn = lfirst ? refs[0] : refs[1];
            int farn = lfirst ? refs[1] : refs[0];
            if (sp < kStackSize) { stack[sp] = farn; stackt[sp] = lfirst ? tr : tl; ++sp; }
            node = nearn;
            continue;
        }
        if (hl) { node = refs[0]; continue; }
        if (hr) { node = refs[1]; continue; }
        bool found = false;
        while (sp > 0) {
            --sp;
            if (stackt[sp] <= h.t * 1.0000008f) { node = stack[sp]; found = true; break; }
        }
        if (!found) break;
    }
    return h;
}

// any hit in (0, inf): visibility of a shadow ray
__device__ __forceinline__ bool trace_any(const BvhNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                                          V3 o, V3 d) {
    RayPre r = ray_pre(o, d);
    int stack[kStackSize];
    int sp = 0;
    int node = 0;
    const float tmax = INFINITY;
    while (true) {
        BvhNode nd = nodes[node];
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
                    float t, b1, b2;
                    if (tri_test(r, xyz(tr3.a), xyz(tr3.b), xyz(tr3.c), tmax, t, b1, b2)) return true;
                }
                hits[c] = false;
            }
        }
        hl = hits[0]; hr = hits[1];
        if (hl && hr) {
            bool lfirst = tl <= tr;
            if (sp < kStackSize) { stack[sp] = lfirst ? refs[1] : refs[0]; ++sp; }
            node = lfirst ? refs[0] : refs[1];
            continue;
        }
        if (hl) { node = refs[0]; continue; }
        if (hr) { node = refs[1]; continue; }
        if (sp == 0) break;
        node = stack[--sp];
    }
    return false;
}

}  // namespace mrs
