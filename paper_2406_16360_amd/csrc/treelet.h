// Treelet restructuring of a binary BVH (Karras and Aila, "Fast parallel
// construction of high-quality bounding volume hierarchies", HPG 2013): a
// node's subtree is opened into a treelet of up to kTreeletLeaves subtrees
// (repeatedly splitting the treelet leaf of largest surface area), and the
// treelet's internal nodes are rearranged into the binary topology over those
// subtrees that minimises the surface area heuristic, found by dynamic
// programming over all subsets of them.  The subtrees themselves, their
// triangles and the treelet root's box stay as they are.
//
// Cost model (of a subtree with box area A holding c triangles):
//   c <= kLeafMax:  kSahTri * c * A   (the node layout makes such a subtree a leaf)
//   otherwise:      kSahNode * A + cost(left) + cost(right)
// Shared by the bottom-up kernel and host-side checks of the same routine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace mrs {

constexpr int kTreeletLeaves = 7;
constexpr int kTreeletSets = 1 << kTreeletLeaves;
constexpr float kSahNode = 1.2f, kSahTri = 1.0f;

// PLOC's merge arrays: ids < n are triangles (one-triangle clusters), ids in
// [n, 2n - 1) merged nodes with two children each; boxes are unpadded.
struct MergeTree {
    int2 *child;
    int32_t *parent, *cnt;
    float4 *lo, *hi;
    float *cost;   // subtree cost under the model above, filled bottom-up
    int n;
};

// tables of the subset search (one thread's, or a wavefront's shared in
// LDS), entry S at [S * stride]
struct TreeletScratch {
    float *cost;
    uint8_t *split;
    int stride;
};

__host__ __device__ inline float box_half_area(float4 l, float4 h) {
    const float dx = h.x - l.x, dy = h.y - l.y, dz = h.z - l.z;
    return dx * dy + dy * dz + dz * dx;
}

__host__ __device__ inline float subtree_cost(float area, int cnt, float cl, float cr) {
    return cnt <= kLeafMax ? kSahTri * (float)cnt * area : kSahNode * area + cl + cr;
}

__host__ __device__ inline int lowest_bit(uint32_t s) {
    int b = 0;
    while (!((s >> b) & 1u)) ++b;
    return b;
}

// union box and triangle count of the treelet leaves in set s
__host__ __device__ __forceinline__ void set_box(uint32_t s, const float4 *llo, const float4 *lhi, const int *lcnt,
                                                 float4 &lo, float4 &hi, int &cnt) {
    lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    cnt = 0;
#pragma unroll
    for (int q = 0; q < kTreeletLeaves; ++q) {
        if (!((s >> q) & 1u)) continue;
        lo.x = fminf(lo.x, llo[q].x); lo.y = fminf(lo.y, llo[q].y); lo.z = fminf(lo.z, llo[q].z);
        hi.x = fmaxf(hi.x, lhi[q].x); hi.y = fmaxf(hi.y, lhi[q].y); hi.z = fmaxf(hi.z, lhi[q].z);
        cnt += lcnt[q];
    }
}

// A treelet: its leaves (subtrees kept as they are), its internal nodes
// (root first) and the leaves' boxes and triangle counts.
struct Treelet {
    int leaf[kTreeletLeaves], inner[kTreeletLeaves - 1];
    float4 llo[kTreeletLeaves], lhi[kTreeletLeaves];
    int lcnt[kTreeletLeaves];
    int nl;
};

// open root's subtree: split the merged treelet leaf of largest area until
// there are kTreeletLeaves leaves or only triangles are left
__host__ __device__ __forceinline__ void treelet_form(const MergeTree &t, int root, Treelet &tl) {
    const int2 rc = t.child[root];
    int ni = 1;
    tl.nl = 2;
    tl.inner[0] = root;
    tl.leaf[0] = rc.x;
    tl.leaf[1] = rc.y;
    while (tl.nl < kTreeletLeaves) {
        int best = -1;
        float ba = -1.0f;
        for (int q = 0; q < tl.nl; ++q) {
            if (tl.leaf[q] < t.n) continue;
            const float a = box_half_area(t.lo[tl.leaf[q]], t.hi[tl.leaf[q]]);
            if (a > ba) { ba = a; best = q; }
        }
        if (best < 0) break;
        const int x = tl.leaf[best];
        tl.inner[ni++] = x;
        tl.leaf[best] = t.child[x].x;
        tl.leaf[tl.nl++] = t.child[x].y;
    }
#pragma unroll
    for (int q = 0; q < kTreeletLeaves; ++q) {
        const int id = q < tl.nl ? tl.leaf[q] : tl.leaf[0];
        tl.llo[q] = t.lo[id];
        tl.lhi[q] = t.hi[id];
        tl.lcnt[q] = q < tl.nl ? t.cnt[id] : 0;
    }
}

// the cost of root's subtree as it stands
__host__ __device__ inline float treelet_keep_cost(const MergeTree &t, int root) {
    const int2 rc = t.child[root];
    return subtree_cost(box_half_area(t.lo[root], t.hi[root]), t.cnt[root], t.cost[rc.x], t.cost[rc.y]);
}

// best cost and split of leaf set s (1 <= s < 2^nl), from the entries of its
// proper subsets, which must be set already; llo, lhi and lcnt are the
// treelet leaves' boxes and counts (tl's own, or a copy)
__host__ __device__ __forceinline__ void treelet_subset(const MergeTree &t, const Treelet &tl, const float4 *llo,
                                                        const float4 *lhi, const int *lcnt, uint32_t s,
                                                        const TreeletScratch &w) {
    float4 lo, hi;
    int cnt;
    set_box(s, llo, lhi, lcnt, lo, hi, cnt);
    const uint32_t low = s & (0u - s), rest = s ^ low;
    if (rest == 0u) {   // one treelet leaf: its subtree as it is
        w.cost[s * w.stride] = t.cost[tl.leaf[lowest_bit(s)]];
        return;
    }
    float best = INFINITY;
    uint32_t bp = low;
    if (cnt > kLeafMax) {
        // the two sides p and s ^ p, with p holding the lowest member
        for (uint32_t q = (rest - 1u) & rest;; q = (q - 1u) & rest) {
            const uint32_t p = low | q;
            const float v = w.cost[p * w.stride] + w.cost[(s ^ p) * w.stride];
            if (v < best) { best = v; bp = p; }
            if (q == 0u) break;
        }
    }
    w.cost[s * w.stride] = subtree_cost(box_half_area(lo, hi), cnt, best, 0.0f);
    w.split[s * w.stride] = (uint8_t)bp;
}

// Sets t.cost[root]; when the best topology beats keep (the cost as it
// stands) by more than rounding (the search sums costs in another order),
// rebuilds the treelet top-down over its own internal nodes first.
__host__ __device__ __forceinline__ void treelet_finish(const MergeTree &t, int root, const Treelet &tl, float keep,
                                               const TreeletScratch &w) {
    const uint32_t full = (1u << tl.nl) - 1u;
    if (!(w.cost[full * w.stride] < keep * 0.99999f)) {
        t.cost[root] = keep;
        return;
    }
    int st_node[kTreeletLeaves], st_set[kTreeletLeaves], sp = 0, next = 1;
    st_node[sp] = root;
    st_set[sp++] = (int)full;
    while (sp > 0) {
        --sp;
        const int x = st_node[sp];
        const uint32_t s = (uint32_t)st_set[sp];
        const uint32_t p = w.split[s * w.stride];
        const uint32_t part[2] = {p, s ^ p};
        int ch[2];
        for (int h = 0; h < 2; ++h) {
            if ((part[h] & (part[h] - 1u)) == 0u) {
                ch[h] = tl.leaf[lowest_bit(part[h])];
            } else {
                ch[h] = tl.inner[next++];
                st_node[sp] = ch[h];
                st_set[sp++] = (int)part[h];
            }
            t.parent[ch[h]] = x;
        }
        t.child[x] = make_int2(ch[0], ch[1]);
        float4 lo, hi;
        int cnt;
        set_box(s, tl.llo, tl.lhi, tl.lcnt, lo, hi, cnt);
        t.lo[x] = lo;
        t.hi[x] = hi;
        t.cnt[x] = cnt;
        t.cost[x] = w.cost[s * w.stride];
    }
}

// Sets t.cost[root] from its children's costs, first rearranging the treelet
// under root when that lowers the cost; one thread, subsets in increasing
// order (a proper subset of s is a smaller number than s).  Every node below
// root must be final (its cost set and its subtree no longer changing);
// root's parent, box and triangle count do not change.
__host__ __device__ inline void treelet_optimize(const MergeTree &t, int root, const TreeletScratch &w) {
    Treelet tl;
    treelet_form(t, root, tl);
    const float keep = treelet_keep_cost(t, root);
    const uint32_t full = (1u << tl.nl) - 1u;
    for (uint32_t s = 1; s <= full; ++s) treelet_subset(t, tl, tl.llo, tl.lhi, tl.lcnt, s, w);
    treelet_finish(t, root, tl, keep, w);
}

}  // namespace mrs
